"""Continuous-batching server: results are the same alone and in the mix (at
the generation count each solve received), and requests wait for memory."""
import numpy as np
import pytest

import cmop_inputs as ci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


def _requests(n, seed, d_lo=0.02, d_hi=0.15, rate=400.0):
    from paper_2509_19821_amd.serve import Request
    arr = ci.serve_arrivals(rate=rate, window_s=n / rate * 1.5, master_seed=seed,
                            d_lo=d_lo, d_hi=d_hi)[:n]
    inst = ci.batch_instances(count=n, master_seed=seed, n_hi=3000, d_hi=40)
    return [Request(k, p, c, dl, t) for k, ((t, dl), (p, c)) in enumerate(zip(arr, inst))]


def test_served_results_equal_alone(G):
    from paper_2509_19821_amd.serve import Server, summarize
    reqs = _requests(24, seed=5)
    srv = Server(4 << 30)
    try:
        res = srv.run(reqs)
    finally:
        srv.close()
    assert sorted(r.rid for r in res) == list(range(len(reqs)))
    s = summarize(res, max(r.delivered for r in res), srv.offspring)
    assert s["p99_time_to_front_s"] is not None
    by = {r.rid: r for r in res}
    for rid in (0, 5, 11, 17, 23):
        r, q = by[rid], reqs[rid]
        assert r.generations >= 1
        gp = G.Gmpea(q.problem, q.config)
        try:
            gp.step(r.generations)
            fr = gp.front()
        finally:
            gp.close()
        assert np.array_equal(fr["f"], r.front_f), rid
        assert np.array_equal(fr["x"], r.front_x), rid


def test_requests_wait_for_memory(G):
    from paper_2509_19821_amd.serve import Request, Server
    prob, cfg, _ = ci.workload_medium(0)
    probe = G.Pool(1 << 30)
    try:
        probe.admit(prob, cfg)
        one = probe.query()["used_bytes"]
    finally:
        probe.close()
    reqs = [Request(k, prob, dict(cfg, seed=k), 0.03, 0.0) for k in range(5)]
    srv = Server(int(2.2 * one))
    peak = 0
    try:
        for r in reqs:
            srv.submit(r)
        srv.now()
        while srv.waiting or srv.active:
            srv.step()
            peak = max(peak, len(srv.active))
    finally:
        srv.close()
    assert peak == 2
    assert len(srv.results) == 5
    by = {r.rid: r for r in srv.results}
    # the first two ran from the start; the others waited for memory, and a
    # request whose deadline passed while it waited gets its initial front
    assert by[0].generations >= 1 and by[1].generations >= 1
    assert all(by[k].admitted >= min(by[0].delivered, by[1].delivered) for k in (2, 3, 4))
    assert all(r.generations >= 0 and r.front_f.shape[1] == 3 for r in srv.results)


def test_igd_at_deadline_sample(G):
    """Quality of the fronts the server delivers at their deadlines: IGD (Eq. (14))
    against each problem's reference front, for a sample of served requests
    (printed); every request that ran at least 20 generations delivers a
    non-empty front of finite IGD. The server measures IGD and the Monte Carlo
    HV on the device at the deadline; both must match the oracle's metrics on
    the delivered front (IGD within 1e-5 relative, HV within 2e-3 of the
    oracle's estimate from the same samples)."""
    from oracle import metrics
    from paper_2509_19821_amd.serve import Server
    reqs = _requests(16, seed=9, d_lo=0.05, d_hi=0.4)
    refs = {}
    for q in reqs[:8]:
        ref = metrics.reference_front(q.problem, density=60).astype(np.float32)
        refs[q.rid] = ref
        q.reference = ref
        q.hv_point = (1.1 * ref.max(0)).astype(np.float32)
    srv = Server(4 << 30, hv_samples=1 << 18)
    try:
        res = srv.run(reqs)
    finally:
        srv.close()
    rows = []
    for r in sorted(res, key=lambda x: x.rid)[:8]:
        q = reqs[r.rid]
        ref = refs[r.rid].astype(np.float64)
        F = r.front_f.astype(np.float64)
        v = metrics.igd(ref, F) if len(F) else float("inf")
        rows.append((r.rid, r.n, r.generations, v))
        print("request %d: N=%d, %d generations by its deadline, IGD %.5f (device %.5f), HV device %.5f"
              % (r.rid, r.n, r.generations, v, r.igd, r.hv), flush=True)
        if len(F):
            assert abs(r.igd - v) <= 1e-5 * v, (r.rid, r.igd, v)
            mc = metrics.hv_mc(F, q.hv_point.astype(np.float64), 1 << 18, seed=0)
            assert abs(r.hv - mc) <= 2e-3 * mc + 1e-12, (r.rid, r.hv, mc)
        else:
            assert r.igd == float("inf") and r.hv == 0.0
    assert all(np.isfinite(v) for (_, _, gens, v) in rows if gens >= 20)


def test_delivery_in_a_full_pool(G):
    """A pool whose budget is exactly two instances' footprint plus the pool's
    own tables: deliveries (front and device quality at each deadline)
    allocate nothing beyond what admission reserved, so every request is
    delivered with its IGD and HV while the pool stays full."""
    from oracle import metrics
    from paper_2509_19821_amd.serve import Request, Server
    prob, cfg, _ = ci.workload_medium(2)
    probe = G.Pool(1 << 30)
    try:  # two instances and the pool's own device tables (state array, work lists)
        probe.admit(prob, cfg)
        probe.admit(prob, dict(cfg, seed=99))
        probe.step(1)
        probe.sync()
        full = probe.query()["used_bytes"]
    finally:
        probe.close()
    ref = metrics.reference_front(prob, density=40).astype(np.float32)
    hvp = (1.1 * ref.max(0)).astype(np.float32)
    reqs = [Request(k, prob, dict(cfg, seed=k), 0.02, 0.0, reference=ref, hv_point=hvp)
            for k in range(6)]
    srv = Server(full, hv_samples=1 << 16)
    peak = 0
    try:
        for r in reqs:
            srv.submit(r)
        srv.now()
        while srv.waiting or srv.active:
            srv.step()
            peak = max(peak, len(srv.active))
            assert srv.pool.query()["used_bytes"] <= full
    finally:
        srv.close()
    assert peak == 2
    assert sorted(r.rid for r in srv.results) == list(range(6))
    assert all(r.igd is not None and r.hv is not None for r in srv.results)
