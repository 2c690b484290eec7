"""GPU parity for many objectives (4 <= m <= 8): records of two or three float4,
the layered reference set (R28), and kernels instantiated per m, against the
FP64 oracle through the C ABI.

Shapes cover every lane grouping of k_vary (d = 7, 17, 30, 100 give 1, 2, 4 and
8 lanes per offspring), one and two layers, both aggregations, DE, the equality
constraint, several 256-row tiles with ragged tails, and m = 4 .. 8. Tolerances
and the teacher-forced protocol are those of the m <= 3 parity tests.
"""
import numpy as np
import pytest

import cmop_inputs as ci
from oracle import core
from test_gpu_parity import TOL, _err, _log, _pair, _teacher_forced

pytestmark = pytest.mark.gpu

S = ci.FAMILY_SPHERE
CASES = {
    # label: (problem, config)
    "m4 d7": (ci.make_problem(S, 4, 7, 2, True, False, 21), ci.method_config(300, 10, 21)),
    "m5 layers d30": (ci.make_problem(S, 5, 30, 3, True, False, 22),
                      ci.method_config(2, 12, 22, h_outer=8, h_inner=5)),
    "m7 d100 eq": (ci.make_problem(S, 7, 100, 4, False, True, 23, eq_tol=1e-4),
                   ci.method_config(900, 16, 23)),
    "m8 layers d17 tche": (ci.make_problem(S, 8, 17, 2, True, False, 24),
                           ci.method_config(2, 10, 24, agg=1, h_outer=3, h_inner=2)),
    "m6 layers DE": (ci.make_problem(S, 6, 40, 2, True, False, 25),
                     ci.method_config(2, 10, 25, op=1, h_outer=5, h_inner=3)),
}


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


@pytest.mark.parametrize("label", list(CASES))
def test_many_structures_and_init(G, label):
    prob, cfg = CASES[label]
    _log("many structures: %s" % label)
    gp, o = _pair(prob, cfg, record=False)
    try:
        info = gp.info()
        assert info["m"] == prob["m"] and info["H"] == o.dv["H"] and info["H2"] == o.dv["H2"]
        assert np.array_equal(gp.read("W"), o.W.astype(np.float32))
        for p in range(2):
            assert np.array_equal(gp.read("B", p), o.B[p]), p
        o.set_state(o.init_x(0), o.init_x(1), None, gen=0)
        for p in range(2):
            assert np.array_equal(gp.read("X", p), o.X[p].astype(np.float32)), p
            assert _err(gp.read("F", p), o.F[p]) <= TOL
            assert _err(gp.read("CV", p), o.CV[p]) <= TOL
        assert _err(gp.read("Z"), o.z) <= TOL
    finally:
        gp.close()


@pytest.mark.parametrize("label", list(CASES))
def test_many_generation_teacher_forced(G, label):
    prob, cfg = CASES[label]
    _log("many teacher-forced: %s" % label)
    gp, o = _pair(prob, cfg)
    try:
        gp.step(3)
        frac = _teacher_forced(gp, o, 2, label)
        assert frac < 0.005
    finally:
        gp.close()


def test_many_front_and_checkpoint(G):
    """Front filter at m = 5 against the oracle's on the device's values, and a
    bit-exact resume from a checkpoint of both populations (records of two
    float4 written back through gmpea_write)."""
    prob, cfg, _ = ci.workload_many5(1)
    gp = G.Gmpea(prob, cfg)
    try:
        gp.step(40)
        fr = gp.front()
        F = gp.read("F", 0).astype(np.float64)
        CV = gp.read("CV", 0).astype(np.float64)
        keep = core.front_mask(F, CV)
        assert np.array_equal(fr["idx"], np.nonzero(keep)[0])
        assert np.array_equal(fr["f"], F[keep].astype(np.float32))
        snap = gp.state()
        gp.step(25)
        ref = gp.state()
    finally:
        gp.close()
    gp = G.Gmpea(prob, cfg)
    try:
        gp.load_state(snap)
        gp.step(25)
        got = gp.state()
    finally:
        gp.close()
    for p in range(2):
        assert np.array_equal(got["X"][p], ref["X"][p])
        assert np.array_equal(got["F"][p], ref["F"][p])
        assert np.array_equal(got["CV"][p], ref["CV"][p])
    assert np.array_equal(got["z"], ref["z"])


def test_quality_on_device(G):
    """gmpea_quality against the oracle's metrics on the device's own front:
    IGD (FP32 distances, FP64 sum) within 1e-5 relative; the Monte Carlo HV
    equal to the oracle's estimate from the same samples within 2e-3 relative
    (FP32 against FP64 sample coordinates can flip a boundary sample), and
    within five standard errors of the exact HV for m = 3."""
    from oracle import metrics
    for which, steps in (("medium", 60), ("many5", 40), ("many8", 40)):
        prob, cfg, _ = ci.WORKLOADS[which](2)
        _log("quality: %s" % which)
        gp = G.Gmpea(prob, cfg)
        try:
            gp.step(steps)
            F = gp.front()["f"].astype(np.float64)
            m = prob["m"]
            if m == 3:
                ref = metrics.reference_front(prob, density=60)
            else:
                W, _ = core.reference_set(m, 6 if m == 5 else 3, 0 if m == 5 else 2)
                ref = W / np.linalg.norm(W, axis=1, keepdims=True)
            r = (1.1 * np.max(F, axis=0)).astype(np.float32)
            S = 1 << 20
            q = gp.quality(ref, r, hv_samples=S, hv_seed=5)
            assert q["front_count"] == F.shape[0] > 0
            want = metrics.igd(ref.astype(np.float32).astype(np.float64), F)
            assert abs(q["igd"] - want) <= 1e-5 * want, (which, q["igd"], want)
            mc = metrics.hv_mc(F, r.astype(np.float64), S, seed=5)
            assert abs(q["hv"] - mc) <= 2e-3 * mc, (which, q["hv"], mc)
            if m == 3:
                exact = metrics.hv(F, r.astype(np.float64))
                vol = float(np.prod(r.astype(np.float64) - F.min(0)))
                p = exact / vol
                assert abs(q["hv"] - exact) <= 5 * vol * np.sqrt(p * (1 - p) / S)
            # reproducible: the same call gives the same numbers
            q2 = gp.quality(ref, r, hv_samples=S, hv_seed=5)
            assert q2 == q
        finally:
            gp.close()


@pytest.mark.parametrize("m,h1,h2,T", [(8, 8, 6, 20), (4, 40, 0, 32), (6, 7, 4, 128)])
def test_device_neighbourhoods_match_host(G, m, h1, h2, T):
    """The device's exact neighbour search (radix select per row) against the
    host's brute force at thousands of rows: both neighbourhoods equal, the
    smaller one the prefix of the larger (t up to 256)."""
    prob = ci.make_problem(ci.FAMILY_SPHERE, m, m + 5, 1, False, False, 41)
    cfg = ci.method_config(2, T, 41, h_outer=h1, h_inner=h2)
    gp = G.Gmpea(prob, cfg, record=False)
    try:
        t1, t2 = gp.t
        _, Bh = G.reference_set(m, h1, h2, max(t1, t2))
        assert np.array_equal(gp.read("B", 0), Bh[:, :t1])
        assert np.array_equal(gp.read("B", 1), Bh[:, :t2])
    finally:
        gp.close()
