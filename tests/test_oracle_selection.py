"""Pins of the oracle's environmental selection (Alg. 2): the reverse-neighbour
pull against the literal dense N x N transcription, special cases that reduce
it to simpler rules, and run invariants."""
import numpy as np
import pytest

import cmop_inputs as ci
from oracle import core
from oracle.dense_alg2 import dense_select


def _tiny_oracle(m, n_req, T, kind=0, t1=0, t2=0, n_ring=2, seed=0):
    fam = ci.FAMILY_CURVE if m == 2 else ci.FAMILY_SPHERE
    prob = ci.make_problem(fam, m, 6, n_ring, m == 3, False, seed)
    cfg = ci.method_config(n_req, T, seed, agg=kind, t1=t1, t2=t2)
    return core.Oracle(prob, cfg, init=False)


def _random_state(o, rng, tie_frac=0.3, dup_frac=0.2):
    """Random parents/offspring with forced CV ties (many exact zeros and shared
    positive values) and duplicated offspring rows."""
    N, m = o.N, o.m
    F = [rng.uniform(0, 2, (N, m)) for _ in range(2)]
    Fo = rng.uniform(0, 2, (2 * N, m))
    vals = np.array([0.0, 0.0, 0.0, 0.5, 1.25])

    def cvs(n):
        cv = rng.uniform(0, 2, n)
        pick = rng.random(n) < tie_frac
        cv[pick] = rng.choice(vals, pick.sum())
        return cv

    CV = [cvs(N), cvs(N)]
    CVo = cvs(2 * N)
    dup = np.nonzero(rng.random(2 * N) < dup_frac)[0]
    for q in dup:
        src = int(rng.integers(0, 2 * N))
        Fo[q] = Fo[src]
        CVo[q] = CVo[src]
    # some offspring are exact copies of a parent
    for q in np.nonzero(rng.random(2 * N) < 0.1)[0]:
        p, j = int(rng.integers(0, 2)), int(rng.integers(0, N))
        Fo[q] = F[p][j]
        CVo[q] = CV[p][j]
    z = np.minimum(np.min(np.concatenate([F[0], F[1], Fo]), 0), 0.0) - rng.uniform(0, 0.1, m)
    CM = [np.where(c == 0, -1.0, c) for c in CV]
    CMo = np.where(CVo == 0, -1.0, CVo)
    X = [rng.uniform(0, 1, (N, o.d)) for _ in range(2)]
    Xo = rng.uniform(0, 1, (2 * N, o.d))
    return F, CV, CM, Fo, CVo, CMo, z, X, Xo


@pytest.mark.parametrize("m,n_req,T,kind", [(2, 20, 6, 0), (2, 24, 10, 1), (3, 28, 8, 0),
                                            (3, 36, 6, 1), (3, 21, 10, 0)])
def test_pull_equals_dense_alg2(m, n_req, T, kind):
    o = _tiny_oracle(m, n_req, T, kind)
    rng = np.random.default_rng(100 + m * 7 + T)
    for trial in range(12):
        F, CV, CM, Fo, CVo, CMo, z, X, Xo = _random_state(o, rng)
        sw, _, win, _ = o.select(X, F, CV, CM, Xo, Fo, CVo, CMo, z)
        Fo2 = Fo.reshape(2, o.N, m)
        CVo2 = CVo.reshape(2, o.N)
        dsw, dwin = dense_select(F, CV, Fo2, CVo2, o.W, z, o.B, kind=kind, theta=5.0)
        assert np.array_equal(sw, dsw), trial
        assert np.array_equal(win, dwin), trial


def test_pull_equals_dense_with_nan():
    o = _tiny_oracle(3, 28, 8)
    rng = np.random.default_rng(77)
    F, CV, CM, Fo, CVo, CMo, z, X, Xo = _random_state(o, rng)
    Fo[3, 0] = np.nan
    Fo[o.N + 5, 1] = np.nan
    F[0][2, 2] = np.nan
    CVo[7] = np.nan
    sw, _, win, _ = o.select(X, F, CV, CM, Xo, Fo, CVo, CMo, z)
    dsw, dwin = dense_select(F, CV, Fo.reshape(2, o.N, 3), CVo.reshape(2, o.N), o.W, z, o.B)
    assert np.array_equal(sw, dsw) and np.array_equal(win, dwin)
    # a NaN offspring never wins a slot
    for p in range(2):
        for j in range(o.N):
            i = win[p, j]
            if i >= 0:
                src = (p ^ sw[p, i]) * o.N + i
                assert np.all(np.isfinite(Fo[src])) and np.isfinite(CVo[src])


def test_neighbourhood_larger_than_population_is_rejected():
    with pytest.raises(ValueError):
        _tiny_oracle(3, 21, 20)


def test_unit_neighbourhood_is_pairwise():
    """t1 = t2 = 1: each slot only meets its own subproblem's new offspring."""
    o = _tiny_oracle(3, 28, 2, t1=1, t2=1)
    rng = np.random.default_rng(5)
    F, CV, CM, Fo, CVo, CMo, z, X, Xo = _random_state(o, rng)
    sw, _, win, _ = o.select(X, F, CV, CM, Xo, Fo, CVo, CMo, z)
    from oracle.dense_alg2 import agg_rows
    for p in range(2):
        for j in range(o.N):
            src = (p ^ sw[p, j]) * o.N + j
            g_new = agg_rows(0, 5.0, Fo[src][None], o.W[j][None], z)[0]
            g_old = agg_rows(0, 5.0, F[p][j][None], o.W[j][None], z)[0]
            if p == 0:
                better = CVo[src] < CV[0][j] or (CVo[src] == CV[0][j] and g_new < g_old)
            else:
                better = g_new < g_old
            assert win[p, j] == (j if better else -1)


def test_unconstrained_population_rules_coincide():
    """With every CV zero, equal neighbourhoods and equal parents, population 1's
    feasibility rule reduces to population 2's aggregation rule."""
    o = _tiny_oracle(3, 36, 10, t1=10, t2=10)
    rng = np.random.default_rng(6)
    F, CV, CM, Fo, CVo, CMo, z, X, Xo = _random_state(o, rng, dup_frac=0.0)
    F = [F[0], F[0].copy()]
    CV = [np.zeros(o.N), np.zeros(o.N)]
    CM = [np.full(o.N, -1.0), np.full(o.N, -1.0)]
    CVo = np.zeros(2 * o.N)
    CMo = np.full(2 * o.N, -1.0)
    sw, _, win, _ = o.select(X, F, CV, CM, Xo, Fo, CVo, CMo, z)
    # same chosen offspring content and same winners
    for i in range(o.N):
        assert (0 ^ sw[0, i]) * o.N + i == (1 ^ sw[1, i]) * o.N + i
    assert np.array_equal(win[0], win[1])


def test_generation_invariants():
    """Population 1's per-slot CV never increases; per-slot (CV, g) under the
    selection-time ideal point never increases lexicographically; population 2's
    per-slot g never increases."""
    prob, cfg, _ = ci.workload_small(3)
    o = core.Oracle(prob, cfg)
    from oracle.dense_alg2 import agg_rows
    for _ in range(25):
        F_old = [f.copy() for f in o.F]
        CV_old = [c.copy() for c in o.CV]
        z_old = o.z.copy()
        o.step()
        z = o.z
        assert np.all(z <= z_old)
        assert np.all(o.CV[0] <= CV_old[0])
        g_old = [agg_rows(0, 5.0, F_old[p], o.W, z) for p in range(2)]
        g_new = [agg_rows(0, 5.0, o.F[p], o.W, z) for p in range(2)]
        same_cv = o.CV[0] == CV_old[0]
        assert np.all(g_new[0][same_cv] <= g_old[0][same_cv] + 1e-12)
        assert np.all(g_new[1] <= g_old[1] + 1e-12)


def test_ideal_point_is_running_minimum():
    prob, cfg, _ = ci.workload_small(4)
    o = core.Oracle(prob, cfg)
    z0 = np.minimum(o.F[0].min(0), o.F[1].min(0))
    assert np.array_equal(o.z, z0)
    seen = z0.copy()
    for _ in range(10):
        d = o.step(debug=True)
        seen = np.minimum(seen, d["Fo"].reshape(-1, o.m).min(0))
        assert np.array_equal(o.z, seen)


def _op1_oracle(rule):
    fam = ci.FAMILY_CURVE
    prob = ci.make_problem(fam, 2, 6, 2, False, False, 0)
    cfg = dict(ci.method_config(20, 6, 0), op1_rule=rule)
    return core.Oracle(prob, cfg, init=False)


@pytest.mark.parametrize("rule", [0, 1])
def test_op1_rules_worked_cases(rule):
    """Population 1's OP1 switch (S1: take population 2's offspring) on cases
    that separate the pseudocode's FPR (lower CV, then lower aggregation) from
    the prose's feasibility-first rule (feasible first; otherwise the lower
    aggregation), with population 2's rule (lower aggregation) alongside."""
    o = _op1_oracle(rule)
    N, m, d = o.N, o.m, o.d
    z = np.zeros(m)
    w = o.W
    # offspring on each subproblem's own direction at distance s: g = s (PBI, d2 = 0)
    def on_ray(i, s):
        u = w[i] / np.linalg.norm(w[i])
        return s * u
    cases = {  # (cv1, g1, cv2, g2) -> (S1 under FPR, S1 under prose, S2)
        0: ((1.0, 0.2, 0.5, 0.9), (1, 0, 1)),   # both infeasible: FPR by CV, prose by g
        1: ((0.0, 0.9, 0.0, 0.2), (1, 1, 0)),   # both feasible: g decides everywhere
        2: ((0.3, 0.1, 0.0, 0.9), (1, 1, 1)),   # only off2 feasible: both rules take it
        3: ((0.0, 0.9, 0.4, 0.1), (0, 0, 0)),   # only off1 feasible: both keep it
        4: ((0.7, 0.5, 0.7, 0.5), (0, 0, 0)),   # exact copy: no switch
    }
    Fo = np.zeros((2 * N, m))
    CVo = np.full(2 * N, 2.0)
    for i, ((c1, g1, c2, g2), _) in cases.items():
        Fo[i], CVo[i] = on_ray(i + 1, g1), c1
        Fo[N + i], CVo[N + i] = on_ray(i + 1, g2), c2
    # evaluate at subproblem i + 1 by placing the cases there
    Fo2 = np.zeros_like(Fo)
    CVo2 = np.full(2 * N, 2.0)
    for i in cases:
        Fo2[i + 1], CVo2[i + 1] = Fo[i], CVo[i]
        Fo2[N + i + 1], CVo2[N + i + 1] = Fo[N + i], CVo[N + i]
    F = [np.full((N, m), 5.0), np.full((N, m), 5.0)]
    CV = [np.full(N, 9.0), np.full(N, 9.0)]
    CM = [CV[0].copy(), CV[1].copy()]
    X = [np.zeros((N, d)), np.zeros((N, d))]
    Xo = np.zeros((2 * N, d))
    sw, _, _, _ = o.select(X, F, CV, CM, Xo, Fo2, CVo2, np.where(CVo2 == 0, -1.0, CVo2), z)
    for i, (_, want) in cases.items():
        assert sw[0, i + 1] == want[rule], (i, rule)
        assert sw[1, i + 1] == want[2], i
