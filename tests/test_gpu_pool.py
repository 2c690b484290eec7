"""Batched generations over a pool of resident instances (uneven N, d, m,
constraint counts): every instance must compute bit-identically to running
alone, admission must respect the device-memory budget, and releasing slots
must not disturb the others."""
import numpy as np
import pytest

import cmop_inputs as ci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


def _mix():
    out = [ci.workload_small(3)[:2], ci.workload_medium(4)[:2]]
    out.append((ci.make_problem(ci.FAMILY_SPHERE, 2, 7, 3, True, False, 7),
                ci.method_config(300, 6, 7, t1=1, t2=1)))
    out.append((ci.make_problem(ci.FAMILY_CURVE, 2, 23, 4, False, False, 8),
                ci.method_config(700, 10, 8, agg=1)))
    out.append((ci.make_problem(ci.FAMILY_SPHERE, 3, 100, 4, False, True, 9, eq_tol=1e-4),
                ci.method_config(3000, 32, 9)))
    out += ci.batch_instances(count=6, master_seed=11, n_hi=4000)
    return out


def _alone(G, prob, cfg, gens):
    gp = G.Gmpea(prob, cfg)
    try:
        gp.step(gens)
        return gp.state()
    finally:
        gp.close()


def _same(a, b):
    assert a["gen"] == b["gen"]
    assert np.array_equal(a["z"], b["z"])
    for p in range(2):
        assert np.array_equal(a["X"][p], b["X"][p])
        assert np.array_equal(a["F"][p], b["F"][p])
        assert np.array_equal(a["CV"][p], b["CV"][p])


def test_batched_equals_alone(G):
    mix = _mix()
    gens = 37  # two graph replays of 16 plus eager generations
    pool = G.Pool(8 << 30)
    try:
        slots = [pool.admit(p, c) for p, c in mix]
        pool.step(gens)
        pool.sync()
        for (p, c), s in zip(mix, slots):
            _same(pool.instance(s).state(), _alone(G, p, c, gens))
        assert pool.query()["active"] == len(mix)
    finally:
        pool.close()


def test_tuning_does_not_change_results(G):
    mix = _mix()[:6]
    pool = G.Pool(8 << 30)
    try:
        slots = [pool.admit(p, c) for p, c in mix]
        done = pool.tune(200)
        assert done == 200
        q = pool.query()
        assert q["schedule"] in (0, 1) and q["chunk"] in (0, 16, 64)
        for (p, c), s in zip(mix, slots):
            _same(pool.instance(s).state(), _alone(G, p, c, 200))
    finally:
        pool.close()


def test_steps_after_tuning_and_admission(G):
    """The tuner leaves graphs cached per (schedule, chunk); later steps replay
    them, and an admission rebuilds the work lists and drops them."""
    mix = _mix()[:5]
    pool = G.Pool(8 << 30)
    try:
        slots = [pool.admit(p, c) for p, c in mix[:4]]
        assert pool.tune(150) == 150
        pool.step(40)
        pool.release(slots[3])
        late = pool.admit(*mix[4])
        pool.step(33)
        for (p, c), s in zip(mix[:3], slots[:3]):
            _same(pool.instance(s).state(), _alone(G, p, c, 223))
        _same(pool.instance(late).state(), _alone(G, *mix[4], 33))
    finally:
        pool.close()


def test_admission_by_budget_and_release(G):
    small = ci.workload_small(0)[:2]
    medium = ci.workload_medium(0)[:2]
    probe = G.Pool(1 << 30)
    try:
        probe.admit(*small)
        one = probe.query()["used_bytes"]
        probe.admit(*medium)
        med = probe.query()["used_bytes"] - one
    finally:
        probe.close()
    assert med > 2 * one
    pool = G.Pool(int(2.5 * one))  # two small instances, never a medium one
    try:
        a = pool.admit(*small)
        used = pool.query()["used_bytes"]
        assert used == one
        assert pool.try_admit(*medium) is None          # footprint above what is left
        assert pool.query()["used_bytes"] == used        # nothing kept from the refusal
        b = pool.admit(*small)
        pool.step(5)
        pool.release(a)
        c = pool.admit(*ci.workload_small(1)[:2])        # reuses the freed slot
        assert c == a
        pool.step(5)
        pool.sync()
        # the untouched instance ran 10 generations exactly as alone
        _same(pool.instance(b).state(), _alone(G, small[0], small[1], 10))
        _same(pool.instance(c).state(), _alone(G, *ci.workload_small(1)[:2], 5))
    finally:
        pool.close()


def test_pool_front_and_empty_steps(G):
    pool = G.Pool(1 << 30)
    try:
        pool.step(3)  # no instances: nothing to do
        s = pool.admit(*ci.workload_medium(2)[:2])
        pool.step(20)
        fr = pool.instance(s).front()
        assert fr["x"].shape[0] > 0 and np.all(fr["cv"] == 0)
        assert pool.instance(s).read("GEN")[0] == 20
    finally:
        pool.close()


def test_batched_mixed_objectives_equal_alone(G):
    """A pool holding m = 2 .. 8, SBX and DE, PBI and Tchebycheff: the m > 3
    instances run in their own batched kernels (the row copies are shared by
    all), and every instance still equals its run alone, bit for bit."""
    S = ci.FAMILY_SPHERE
    mix = [ci.workload_small(13)[:2], ci.workload_many5(14)[:2], ci.workload_many8(15)[:2],
           (ci.make_problem(S, 6, 33, 2, True, False, 16),
            ci.method_config(2, 10, 16, op=1, h_outer=5, h_inner=3)),
           (ci.make_problem(S, 3, 40, 2, True, False, 17), ci.method_config(900, 12, 17)),
           (ci.make_problem(S, 4, 9, 1, False, False, 18), ci.method_config(400, 8, 18, agg=1)),
           # m <= 3 with DE, and with Tchebycheff, a high mutation rate and eta_c = 3
           (ci.make_problem(S, 3, 25, 2, True, False, 19), ci.method_config(500, 10, 19, op=1)),
           (ci.make_problem(ci.FAMILY_CURVE, 2, 11, 1, False, False, 20),
            ci.method_config(200, 10, 20, agg=1, pm=0.75, eta_c=3.0))]
    gens = 21  # one graph replay of 16 plus eager generations
    pool = G.Pool(4 << 30)
    try:
        slots = [pool.admit(p, c) for p, c in mix]
        pool.step(gens)
        pool.sync()
        for (p, c), s in zip(mix, slots):
            _same(pool.instance(s).state(), _alone(G, p, c, gens))
        # releasing the wide instances leaves a pool of m <= 3 only, and back
        pool.release(slots[1])
        pool.release(slots[2])
        pool.step(3)
        pool.sync()
        _same(pool.instance(slots[0]).state(), _alone(G, *mix[0], gens + 3))
        _same(pool.instance(slots[3]).state(), _alone(G, *mix[3], gens + 3))
    finally:
        pool.close()
