"""Pins of the oracle's many-objective generalisation (m > 3): the two-layer
reference set (reading R28), its neighbourhoods, the sphere family, the
aggregations and the front filter at m up to 8, and whole generations against
the from-scratch Python composition."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import cmop_inputs as ci
from oracle import core
from oracle.dense_alg2 import dense_select


# ------------------------------------------------------- reference set ----

@pytest.mark.parametrize("m,H1,H2,n", [(8, 3, 2, 156), (10, 3, 2, 275), (15, 2, 1, 135),
                                       (5, 6, 0, 210), (3, 12, 0, 91)])
def test_reference_set_sizes(m, H1, H2, n):
    """The reference-point counts commonly used for many-objective suites
    (8, 10 and 15 objectives with two layers; 5 with one)."""
    W, K = core.reference_set(m, H1, H2)
    assert W.shape == (n, m) and K.shape == (n, m)
    assert n == math.comb(H1 + m - 1, m - 1) + (math.comb(H2 + m - 1, m - 1) if H2 else 0)


def _exact_rows(m, H1, H2):
    """Independent definition in exact rationals: every composition of H1 into m
    parts over H1, then every composition of H2 over H2 moved halfway to the
    centroid, each block in lexicographic order."""
    def comps(H):
        return sorted(c for c in itertools.product(range(H + 1), repeat=m) if sum(c) == H)
    rows = [[Fraction(k, H1) for k in c] for c in comps(H1)]
    if H2:
        rows += [[(Fraction(k, H2) + Fraction(1, m)) / 2 for k in c] for c in comps(H2)]
    return rows


@pytest.mark.parametrize("m,H1,H2", [(4, 3, 2), (5, 2, 1), (6, 2, 2), (4, 5, 0), (2, 4, 2)])
def test_reference_set_exact(m, H1, H2):
    W, K = core.reference_set(m, H1, H2)
    rows = _exact_rows(m, H1, H2)
    assert len(rows) == W.shape[0]
    S = 2 * m * H1 * H2 if H2 else H1
    for r, ex in enumerate(rows):
        # FP64 values are the exact rationals rounded once, integer coordinates exact
        assert all(W[r, a] == float(ex[a]) for a in range(m)), r
        assert all(Fraction(int(K[r, a]), S) == ex[a] for a in range(m)), r
        assert sum(ex) == 1
    if H2:
        inner = W[math.comb(H1 + m - 1, m - 1):]
        assert inner.min() >= 1.0 / (2 * m)  # half-way to the centroid keeps off every facet


def _knn_exact(rows, t):
    """(exact squared distance, index) order by full sort."""
    n = len(rows)
    out = []
    for i in range(n):
        d = [sum((rows[i][a] - rows[j][a]) ** 2 for a in range(len(rows[i]))) for j in range(n)]
        out.append(sorted(range(n), key=lambda j: (d[j], j))[:t])
    return np.array(out, dtype=np.int32)


@pytest.mark.parametrize("m,H1,H2,t", [(4, 3, 1, 6), (4, 2, 2, 9), (5, 2, 1, 10), (2, 4, 2, 3),
                                       (6, 2, 0, 8)])
def test_two_layer_neighbourhoods_exact(m, H1, H2, t):
    W, K = core.reference_set(m, H1, H2)
    B = core.knn(K, t)
    assert np.array_equal(B, _knn_exact(_exact_rows(m, H1, H2), t))


def test_duplicate_vectors_order_by_index():
    """With H1 = 4 and H2 = 2 at m = 2 every inner point repeats an outer one
    ((k / 2 + 1 / 2) / 2 = (k + 1) / 4): the copies are at distance 0 from each
    other, so each row starts with the lower index of its pair, then the higher."""
    W, K = core.reference_set(2, 4, 2)
    assert np.array_equal(W[5:], W[1:4])
    B = core.knn(K, 3)
    for r in range(len(W)):
        same = [q for q in range(len(W)) if np.all(W[q] == W[r])]
        assert list(B[r][:len(same)]) == same, r


def test_derive_layers():
    prob = ci.make_problem(ci.FAMILY_SPHERE, 8, 17, 1, False, False, 0)
    dv = core.derive(prob, ci.method_config(5, 10, 0, h_outer=3, h_inner=2))
    assert (dv["H"], dv["H2"], dv["N"]) == (3, 2, 156)
    dv = core.derive(prob, ci.method_config(5, 10, 0, h_outer=3))
    assert (dv["H"], dv["H2"], dv["N"]) == (3, 0, 120)
    dv = core.derive(prob, ci.method_config(100, 10, 0))  # from n_req: smallest lattice >= 100
    assert (dv["H"], dv["H2"], dv["N"]) == (3, 0, 120)
    with pytest.raises(ValueError):
        core.derive(prob, ci.method_config(5, 10, 0, h_inner=2))


# ------------------------------------------------------- sphere family ----

@pytest.mark.parametrize("m", [4, 5, 8])
def test_sphere_radius_many(m):
    p = ci.make_problem(ci.FAMILY_SPHERE, m, 14, 0, False, False, 0)
    rng = np.random.default_rng(80 + m)
    x = rng.uniform(0, 1, size=(300, 14))
    F, CV, _ = core.evaluate(p, x)
    g = ((x[:, m - 1:] - 0.5) ** 2).sum(1)
    assert np.allclose(np.linalg.norm(F, axis=1), 1 + g, rtol=1e-13)
    assert np.all(F >= 0) and np.all(CV == 0)


@pytest.mark.parametrize("m", [4, 6, 8])
def test_sphere_corners_many(m):
    """Angles 0 .. 0, 1 (j leading zeros) put the point on axis m - 1 - j."""
    p = ci.make_problem(ci.FAMILY_SPHERE, m, m + 2, 0, False, False, 0)
    for j in range(m):
        x = np.full(m + 2, 0.5)
        x[:m - 1] = 0.37  # arbitrary angles past the first one are irrelevant
        x[:j] = 0.0
        if j < m - 1:
            x[j] = 1.0
        F, _, _ = core.evaluate(p, x[None, :])
        want = np.zeros(m)
        want[m - 1 - j if j < m - 1 else 0] = 1.0
        assert np.allclose(F[0], want, atol=1e-15), (m, j, F[0])


def test_rings_in_many_dimensions():
    m = 6
    p = ci.make_problem(ci.FAMILY_SPHERE, m, 9, 2, True, False, 3)
    x = np.random.default_rng(4).uniform(0, 1, (50, 9))
    F, _, _ = core.evaluate(p, x)
    p["ring_center"] = np.vstack([F[7], np.full(m, 9.0)])
    p["ring_radius"] = np.array([0.3, 0.1])
    p["sum_lower"] = 0.0
    _, CV, _ = core.evaluate(p, x[7:8])
    assert abs(CV[0] - 0.09) < 1e-15


# ----------------------------------------------------------- aggregation ----

def test_pbi_closed_forms_many():
    rng = np.random.default_rng(12)
    for _ in range(300):
        m = int(rng.integers(4, 9))
        w = rng.uniform(0.01, 1, m)
        u = w / np.linalg.norm(w)
        z = rng.uniform(-1, 1, m)
        s = rng.uniform(0, 3)
        e = rng.normal(size=m)
        e -= e.dot(u) * u
        theta = rng.uniform(0, 10)
        g = core.agg(0, theta, z + s * u + e, w, z)
        assert abs(g - (s + theta * np.linalg.norm(e))) < 1e-11


def test_tchebycheff_minimiser_many():
    rng = np.random.default_rng(13)
    for m in (4, 6, 8):
        w = rng.uniform(0.1, 1.0, m)
        want = (1 / w) / (1 / w).sum()
        z = np.zeros(m)
        g_star = core.agg(1, 0.0, want, w, z)
        assert abs(g_star - 1.0 / (1 / w).sum()) < 1e-14
        pts = rng.dirichlet(np.ones(m), size=5000)
        assert g_star <= min(core.agg(1, 0.0, q, w, z) for q in pts) + 1e-12


# --------------------------------------------------------------- front ----

@pytest.mark.parametrize("m,n", [(5, 400), (8, 300)])
def test_front_many_against_dominance_matrix(m, n):
    rng = np.random.default_rng(m * 31 + n)
    F = np.round(rng.uniform(0, 1, (n, m)), 1)  # coarse grid: ties and duplicates
    CV = np.where(rng.random(n) < 0.3, rng.uniform(0, 1, n), 0.0)
    feas = CV == 0
    le = np.all(F[:, None, :] <= F[None, :, :], axis=2)
    lt = np.any(F[:, None, :] < F[None, :, :], axis=2)
    want = feas & ~(le & lt & feas[:, None]).any(0)
    assert np.array_equal(core.front_mask(F, CV), want)


# ----------------------------------------------------------- selection ----

def _many_oracle(m, h1, h2, T, kind=0, seed=0):
    prob = ci.make_problem(ci.FAMILY_SPHERE, m, m + 3, 2, True, False, seed)
    cfg = ci.method_config(2, T, seed, agg=kind, h_outer=h1, h_inner=h2)
    return core.Oracle(prob, cfg, init=False)


@pytest.mark.parametrize("m,h1,h2,T,kind", [(5, 3, 0, 8, 0), (5, 2, 1, 6, 1), (8, 2, 1, 10, 0)])
def test_pull_equals_dense_alg2_many(m, h1, h2, T, kind):
    o = _many_oracle(m, h1, h2, T, kind)
    rng = np.random.default_rng(300 + m + h1)
    N = o.N
    for trial in range(6):
        F = [rng.uniform(0, 2, (N, m)) for _ in range(2)]
        Fo = rng.uniform(0, 2, (2 * N, m))
        CV = [np.where(rng.random(N) < 0.5, 0.0, rng.uniform(0, 1, N)) for _ in range(2)]
        CVo = np.where(rng.random(2 * N) < 0.5, 0.0, rng.uniform(0, 1, 2 * N))
        z = np.minimum(np.min(np.concatenate([F[0], F[1], Fo]), 0), 0.0)
        CM = [np.where(c == 0, -1.0, c) for c in CV]
        CMo = np.where(CVo == 0, -1.0, CVo)
        X = [rng.uniform(0, 1, (N, o.d)) for _ in range(2)]
        Xo = rng.uniform(0, 1, (2 * N, o.d))
        sw, _, win, _ = o.select(X, F, CV, CM, Xo, Fo, CVo, CMo, z)
        dsw, dwin = dense_select(F, CV, Fo.reshape(2, N, m), CVo.reshape(2, N), o.W, z, o.B,
                                 kind=kind, theta=5.0)
        assert np.array_equal(sw, dsw), trial
        assert np.array_equal(win, dwin), trial


@pytest.mark.parametrize("m,h1,h2,seed", [(5, 3, 0, 0), (6, 2, 1, 1)])
def test_generation_many_matches_python_composition(m, h1, h2, seed):
    from test_oracle_generation import _python_offspring, _python_select
    o = _many_oracle(m, h1, h2, 8, seed=seed)
    o.set_state(o.init_x(0), o.init_x(1), None, gen=0)
    o.run(3)
    Xo, Fo, CVo = _python_offspring(o, o.gen + 1)
    prev = type("S", (), {})()
    prev.F, prev.CV = [f.copy() for f in o.F], [c.copy() for c in o.CV]
    prev.X, prev.z = [x.copy() for x in o.X], o.z.copy()
    prev.W, prev.B, prev.N, prev.m, prev.dv = o.W, o.B, o.N, o.m, o.dv
    dbg = o.step(debug=True)
    assert np.allclose(dbg["Xo"], Xo, rtol=0, atol=1e-13)
    assert np.allclose(dbg["Fo"], Fo, rtol=1e-12, atol=1e-13)
    assert np.allclose(dbg["CVo"], CVo, rtol=1e-12, atol=1e-13)
    z, sw, win, X = _python_select(prev, dbg["Xo"], dbg["Fo"], dbg["CVo"])
    assert np.allclose(o.z, z, rtol=0, atol=1e-15)
    assert np.array_equal(dbg["op1"], sw)
    assert np.array_equal(dbg["win"], win)
    for p in range(2):
        assert np.allclose(o.X[p], X[p], rtol=0, atol=1e-13)
