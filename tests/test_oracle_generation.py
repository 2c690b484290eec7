"""Pins of the oracle's whole generation: a from-scratch Python composition of
the generation for tiny sizes (Alg. 1 body: mating, SBX, PM, evaluation, ideal
point, then Alg. 2 via the dense transcription) must reproduce the C oracle's
state; plus determinism across thread counts."""
import math

import numpy as np
import pytest

import cmop_inputs as ci
from oracle import core
from oracle.dense_alg2 import dense_select

TAG_INIT, TAG_MATE, TAG_VAR = 1, 2, 3


def _words(key, c0, i, k, tag, pop):
    ctr = np.array([[c0, i, k, (tag << 24) | (pop << 16)]], dtype=np.uint32)
    return [int(x) for x in core.philox(ctr, np.array(key, dtype=np.uint32))[0]]


def _objectives(prob, x):
    m, d = prob["m"], prob["d"]
    if prob["family"] == 0:
        g = 1 + 9 * sum(x[1:]) / (d - 1)
        return [x[0], g * (1 - math.sqrt(x[0] / g))]
    g = sum((v - 0.5) ** 2 for v in x[m - 1:])
    th = [math.pi / 2 * v for v in x[:m - 1]]
    f = []
    for k in range(m):
        v = 1 + g
        for j in range(m - 1 - k):
            v *= math.cos(th[j])
        if k > 0:
            v *= math.sin(th[m - 1 - k])
        f.append(v)
    return f


def _cv(prob, x, f):
    m = prob["m"]
    cv = 0.0
    for c, r in zip(np.asarray(prob["ring_center"]).reshape(-1, m), prob["ring_radius"]):
        cv += max(0.0, r * r - sum((f[k] - c[k]) ** 2 for k in range(m)))
    if prob["has_sum_lower"]:
        cv += max(0.0, prob["sum_lower"] - sum(f))
    if prob["n_eq"]:
        cv += max(0.0, abs(x[0] + x[1] - 1) - prob["eq_tol"])
    return cv


def _python_offspring(o, k):
    """Offspring of one generation written independently from the paper's steps."""
    prob, dv, N, d, m = o.prob, o.dv, o.N, o.d, o.m
    key = dv["key"]
    eta_c, eta_m, tpm = dv["eta_c"], dv["eta_m"], dv["tpm"]
    lb, ub = prob["lb"], prob["ub"]
    Xo = np.empty((2, N, d))
    Fo = np.empty((2, N, m))
    CVo = np.empty((2, N))
    for p in range(2):
        t = dv["t"][p]
        for i in range(N):
            w = _words(key, 0, i, k, TAG_MATE, p)
            r1 = (w[0] * t) >> 32
            r2 = (w[1] * (t - 1)) >> 32 if t > 1 else r1
            if t > 1 and r2 >= r1:
                r2 += 1
            a, b = o.X[p][o.B[p][i, r1]], o.X[p][o.B[p][i, r2]]
            for l in range(d):
                v = _words(key, l >> 1, i, k, TAG_VAR, p)
                wA, wB = v[2 * (l & 1)], v[2 * (l & 1) + 1]
                c = a[l]
                if wA & 1:  # crossed: beta from the SBX spread distribution
                    u = (wA >> 8) / 2.0**24
                    beta = (2 * u) ** (1 / (eta_c + 1)) if u <= 0.5 else (1 / (2 * (1 - u))) ** (1 / (eta_c + 1))
                    if wA & 2:
                        beta = -beta
                    c = (1 + beta) / 2 * a[l] + (1 - beta) / 2 * b[l]
                c = min(max(c, lb[l]), ub[l])
                if wB < tpm:
                    u = wB / tpm
                    span = ub[l] - lb[l]
                    if u < 0.5:
                        dq = (2 * u + (1 - 2 * u) * (1 - (c - lb[l]) / span) ** (eta_m + 1)) ** (1 / (eta_m + 1)) - 1
                    else:
                        dq = 1 - (2 * (1 - u) + 2 * (u - 0.5) * (1 - (ub[l] - c) / span) ** (eta_m + 1)) ** (1 / (eta_m + 1))
                    c = min(max(c + dq * span, lb[l]), ub[l])
                Xo[p, i, l] = c
            Fo[p, i] = _objectives(prob, Xo[p, i])
            CVo[p, i] = _cv(prob, Xo[p, i], Fo[p, i])
    return Xo, Fo, CVo


def _python_select(o, Xo, Fo, CVo):
    """Ideal-point update, then Alg. 2 through the dense transcription, then the
    synchronous replacement."""
    z = np.minimum(o.z, Fo.reshape(-1, o.m).min(0))
    sw, win = dense_select(o.F, o.CV, Fo, CVo, o.W, z, o.B, kind=o.dv["agg"],
                           theta=o.dv["theta"])
    X = [o.X[p].copy() for p in range(2)]
    for p in range(2):
        for j in range(o.N):
            i = win[p, j]
            if i >= 0:
                X[p][j] = Xo[p ^ sw[p, i], i]
    return z, sw, win, X


@pytest.mark.parametrize("which,seed", [("small", 0), ("small", 5), ("medium", 1)])
def test_generation_matches_python_composition(which, seed):
    if which == "small":
        prob, cfg, _ = ci.workload_small(seed)
        cfg["n_req"] = 24
    else:
        prob = ci.make_problem(ci.FAMILY_SPHERE, 3, 7, 3, True, False, seed)
        cfg = ci.method_config(28, 6, seed)
    cfg["T"] = 8
    o = core.Oracle(prob, cfg)
    o.run(3)  # start from an evolved state
    Xo, Fo, CVo = _python_offspring(o, o.gen + 1)
    # selection on the oracle's own offspring values: an offspring that copies its
    # parent must compare as an exact tie, which a re-evaluation in another
    # rounding order would break
    F_before = [f.copy() for f in o.F]
    CV_before = [c.copy() for c in o.CV]
    X_before = [x.copy() for x in o.X]
    z_before = o.z.copy()
    dbg = o.step(debug=True)
    assert np.allclose(dbg["Xo"], Xo, rtol=0, atol=1e-13)
    assert np.allclose(dbg["Fo"], Fo, rtol=1e-12, atol=1e-13)
    assert np.allclose(dbg["CVo"], CVo, rtol=1e-12, atol=1e-13)
    o_prev = type("S", (), {})()
    o_prev.F, o_prev.CV, o_prev.X, o_prev.z = F_before, CV_before, X_before, z_before
    o_prev.W, o_prev.B, o_prev.N, o_prev.m, o_prev.dv = o.W, o.B, o.N, o.m, o.dv
    z, sw, win, X = _python_select(o_prev, dbg["Xo"], dbg["Fo"], dbg["CVo"])
    assert np.allclose(o.z, z, rtol=0, atol=1e-15)
    assert np.array_equal(dbg["op1"], sw)
    assert np.array_equal(dbg["win"], win)
    for p in range(2):
        assert np.allclose(o.X[p], X[p], rtol=0, atol=1e-13)


def test_threads_do_not_change_results():
    prob, cfg, _ = ci.workload_medium(2)
    cfg["n_req"] = 300
    out = []
    for nt in (1, 4):
        core.set_threads(nt)
        o = core.Oracle(prob, cfg)
        o.run(5)
        out.append((o.X[0].copy(), o.X[1].copy(), o.z.copy()))
    core.set_threads(0)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_init_uniform_in_box():
    prob = ci.make_problem(ci.FAMILY_SPHERE, 3, 9, 1, False, False, 0,
                           lb=np.full(9, -2.0), ub=np.full(9, 3.0))
    o = core.Oracle(prob, ci.method_config(200, 10, 9))
    for p in range(2):
        assert np.all(o.X[p] >= -2.0) and np.all(o.X[p] < 3.0)
        assert abs(o.X[p].mean() - 0.5) < 0.1
    assert not np.array_equal(o.X[0], o.X[1])  # independent draws (R4)
