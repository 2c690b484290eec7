"""Host-side scheduling of the serving loop (paper_2509_19821_amd/serve.py),
on the CPU: the server drives a stand-in pool whose generations advance a
simulated clock by a fixed cost, so admission order, memory-budget waits,
generation chunks against the earliest deadline, delivery and the per-request
records can be checked without a GPU. The device side of the same loop is
covered by tests/test_gpu_serve.py."""
import numpy as np
import pytest

from paper_2509_19821_amd import serve


class Clock:
    """Simulated seconds; every reading moves time on by a microsecond, so a
    loop that only waits still reaches the next arrival."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-6
        return self.t


class Inst:
    def __init__(self, n, m):
        self.n, self.m, self.gen = n, m, 0

    def front(self, with_x=True):
        f = np.full((1, self.m), float(self.gen), dtype=np.float32)
        return {"f": f, "x": np.zeros((1, 2), dtype=np.float32) if with_x else None}

    def read(self, what):
        assert what == "GEN"
        return np.array([self.gen], dtype=np.int64)

    def quality(self, ref, hv_point, hv_samples=0):
        return {"igd": 0.25, "hv": 1.5}


class Pool:
    """Footprint of a request = its n_req; one generation of the whole pool
    costs gen_cost simulated seconds."""

    def __init__(self, clock, budget, gen_cost):
        self.clock, self.budget, self.gen_cost = clock, budget, gen_cost
        self.slots, self.used, self.steps, self.admitted = {}, 0, [], []
        self.peak = 0

    def try_admit(self, problem, config, record=False):
        need = config["n_req"]
        if self.used + need > self.budget:
            return None
        slot = min(set(range(len(self.slots) + 1)) - set(self.slots))
        self.slots[slot] = Inst(need, problem["m"])
        self.used += need
        self.peak = max(self.peak, self.used)
        self.admitted.append(config["rid"])
        return slot

    def instance(self, slot):
        return self.slots[slot]

    def step(self, k):
        assert self.slots, "a step with nothing resident"
        for inst in self.slots.values():
            inst.gen += k
        self.clock.t += k * self.gen_cost
        self.steps.append(k)

    def sync(self):
        pass

    def release(self, slot):
        self.used -= self.slots.pop(slot).n

    def close(self):
        pass


def _requests(count, seed, n_lo=100, n_hi=1000, with_ref_every=3):
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(0.002, count))
    out = []
    for r in range(count):
        ref = np.zeros((4, 2), dtype=np.float32) if r % with_ref_every == 0 else None
        out.append(serve.Request(r, {"m": 2}, {"n_req": int(rng.integers(n_lo, n_hi)), "rid": r},
                                 deadline_s=float(rng.uniform(0.005, 0.05)), arrival=float(arrivals[r]),
                                 reference=ref))
    return out


def _server(budget, gen_cost, max_chunk=8):
    clock = Clock()
    pool = Pool(clock, budget, gen_cost)
    return serve.Server(budget, clock=clock, max_chunk=max_chunk, pool=pool), pool


def test_every_request_delivered_once_close_to_its_deadline():
    gen_cost = 2e-4
    srv, pool = _server(budget=10 ** 9, gen_cost=gen_cost)
    reqs = _requests(60, seed=1)
    res = srv.run(reqs)
    assert sorted(r.rid for r in res) == list(range(len(reqs)))
    by = {r.rid: r for r in res}
    for q in reqs:
        r = by[q.rid]
        assert r.arrival == q.arrival and r.deadline == pytest.approx(q.arrival + q.deadline_s)
        assert r.admitted >= r.arrival
        assert r.delivered >= r.deadline  # never cut short
        # the chunk never runs past the earliest deadline by more than one
        # generation (the estimate is the measured cost), plus the loop's own time
        assert r.lateness <= 1.5 * gen_cost + 1e-4, (r.rid, r.lateness)
        assert r.generations >= 1
        assert r.front_f.shape == (1, 2) and r.front_f[0, 0] == r.generations  # the front at delivery
        assert (r.igd is not None) == (q.reference is not None)
    assert all(1 <= k <= 8 for k in pool.steps)
    assert max(pool.steps) > 1  # chunks of several generations were used
    assert not pool.slots and pool.used == 0  # every slot released


def test_offspring_count_matches_generations_delivered():
    srv, pool = _server(budget=10 ** 9, gen_cost=1e-4)
    res = srv.run(_requests(20, seed=2))
    # each resident solve contributes 2 n offspring per generation it received
    assert srv.offspring == sum(2 * r.n * r.generations for r in res)


def test_admission_waits_for_memory_in_arrival_order():
    srv, pool = _server(budget=1500, gen_cost=3e-4)
    reqs = _requests(25, seed=3, n_lo=600, n_hi=1000)  # at most two fit at once
    res = srv.run(reqs)
    assert pool.peak <= 1500
    assert pool.admitted == [q.rid for q in sorted(reqs, key=lambda q: q.arrival)]
    by = {r.rid: r for r in res}
    adm = [by[q.rid].admitted for q in sorted(reqs, key=lambda q: q.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert len(res) == len(reqs)


def test_chunk_of_one_without_estimate_and_bounded_by_max():
    srv, pool = _server(budget=10 ** 9, gen_cost=1e-5, max_chunk=3)
    req = serve.Request(0, {"m": 2}, {"n_req": 100, "rid": 0}, deadline_s=0.01, arrival=0.0)
    res = srv.run([req])
    assert pool.steps[0] == 1  # no cost estimate before the first step
    assert max(pool.steps) == 3 and all(1 <= k <= 3 for k in pool.steps)
    assert res[0].generations == sum(pool.steps)


def test_request_that_cannot_fit_an_empty_pool_is_an_error():
    srv, _ = _server(budget=50, gen_cost=1e-4)
    req = serve.Request(0, {"m": 2}, {"n_req": 100, "rid": 0}, deadline_s=0.01, arrival=0.0)
    with pytest.raises(MemoryError):
        srv.run([req])


def test_summary_fields():
    srv, _ = _server(budget=10 ** 9, gen_cost=1e-4)
    res = srv.run(_requests(10, seed=4))
    s = serve.summarize(res, wall_s=1.0, offspring=srv.offspring, host_s=srv.host_s)
    assert s["requests"] == 10 and s["offspring_per_s"] == srv.offspring
    assert s["p50_time_to_front_s"] <= s["p99_time_to_front_s"]
    assert s["igd_at_deadline"]["count"] == sum(r.igd is not None for r in res)
    assert s["hv_at_deadline"]["median"] == 1.5
