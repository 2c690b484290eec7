"""Pins of the oracle's variation operators (SBX R7, PM R8), evaluation
(Eqs. (1)-(3), R9) and aggregation (Eq. (7) with R13, Tchebycheff)."""
import math

import numpy as np
import pytest
from scipy import stats

import cmop_inputs as ci


# ----------------------------------------------------------------- SBX ----

def test_sbx_pairwise_mean_invariant(oracle_core):
    rng = np.random.default_rng(2)
    for _ in range(2000):
        a, b = rng.uniform(-3, 3, size=2)
        wA = int(rng.integers(0, 2**32))
        c, s, beta = oracle_core.sbx_dim(a, b, wA, 20.0)
        assert abs((c + s) - (a + b)) <= 1e-12 * max(1.0, abs(a) + abs(b))
        if wA & 1:
            # child = mean + beta (a - b) / 2 with the drawn sign
            assert abs((c - s) - beta * (a - b)) <= 1e-12 * max(1.0, abs(a - b))
            assert (beta < 0) == bool(wA & 2) or beta == 0.0
        else:
            assert c == a and s == b and beta == 0.0


def test_sbx_spread_density(oracle_core):
    """|beta| follows the SBX spread density: 0.5 (eta+1) b^eta on [0, 1] and
    0.5 (eta+1) b^-(eta+2) above 1, i.e. CDF 0.5 b^(eta+1) then 1 - 0.5 b^-(eta+1)."""
    eta = 20.0
    rng = np.random.default_rng(3)
    w = rng.integers(0, 2**32, size=60000, dtype=np.uint64)
    w = (w | 1).astype(np.uint32)  # crossed dimensions only
    betas = np.array([abs(oracle_core.sbx_dim(1.0, 0.0, int(x), eta)[2]) for x in w])

    def cdf(b):
        b = np.asarray(b, dtype=np.float64)
        return np.where(b <= 1.0, 0.5 * b ** (eta + 1), 1.0 - 0.5 * b ** (-(eta + 1)))

    res = stats.kstest(betas, cdf)
    assert res.pvalue > 1e-3


def test_sbx_uncrossed_copy_exact(oracle_core):
    for wA in (0, 2, 0xFFFFFFFE, 0x12345670):
        c, s, beta = oracle_core.sbx_dim(0.123456789, 0.987654321, wA, 20.0)
        assert c == 0.123456789 and s == 0.987654321


# ------------------------------------------------------------------ PM ----

def test_pm_identity_when_probability_zero(oracle_core):
    rng = np.random.default_rng(4)
    for _ in range(500):
        y = rng.uniform(0, 1)
        w = int(rng.integers(0, 2**32))
        assert oracle_core.pm_dim(y, 0.0, 1.0, w, 0, 20.0) == y


def test_pm_zero_step_at_half(oracle_core):
    tpm = 2 * 214748364  # even, so wB = tpm / 2 gives u = 0.5 exactly
    wB = tpm // 2
    for y in (0.0, 0.2, 0.5, 0.999, 1.0):
        assert oracle_core.pm_dim(y, 0.0, 1.0, wB, tpm, 20.0) == y


def test_pm_bounds_and_stays_at_bound(oracle_core):
    rng = np.random.default_rng(5)
    tpm = 2**32  # always mutate
    for _ in range(3000):
        lo, hi = sorted(rng.uniform(-5, 5, size=2))
        y = rng.uniform(lo, hi)
        w = int(rng.integers(0, 2**32))
        v = oracle_core.pm_dim(y, lo, hi, w, tpm, 20.0)
        assert lo <= v <= hi
    # at the lower bound a downward draw (u < 0.5) cannot move the variable
    assert oracle_core.pm_dim(0.0, 0.0, 1.0, 1000, tpm, 20.0) == 0.0
    assert oracle_core.pm_dim(1.0, 0.0, 1.0, 0xFFFFFF00, tpm, 20.0) == 1.0


def test_pm_perturbation_density(oracle_core):
    """Away from the bounds the step delta = (y' - y)/(hi - lo) has the
    polynomial density 0.5 (eta+1) (1 - |delta|)^eta, CDF 0.5 (1 + delta)^(eta+1)
    for delta <= 0 and 1 - 0.5 (1 - delta)^(eta+1) above."""
    eta = 20.0
    lo, hi, y = -100.0, 100.0, 0.0  # (1 - delta_1)^(eta+1) = 0.5^21: negligible
    rng = np.random.default_rng(6)
    w = rng.integers(0, 2**32, size=40000)
    deltas = np.array([(oracle_core.pm_dim(y, lo, hi, int(x), 2**32, eta) - y) / (hi - lo)
                       for x in w])

    def cdf(d):
        d = np.asarray(d, dtype=np.float64)
        return np.where(d <= 0, 0.5 * (1 + d) ** (eta + 1), 1 - 0.5 * (1 - d) ** (eta + 1))

    assert stats.kstest(deltas, cdf).pvalue > 1e-3


def test_pm_rate(oracle_core):
    tpm = int(math.floor(2**32 / 10))
    rng = np.random.default_rng(7)
    w = rng.integers(0, 2**32, size=50000)
    moved = np.mean([oracle_core.pm_dim(0.5, 0, 1, int(x), tpm, 20.0) != 0.5 for x in w])
    assert abs(moved - 0.1) < 0.006


# ---------------------------------------------------------- evaluation ----

def _prob(**kw):
    p = ci.make_problem(kw.pop("family", 1), kw.pop("m", 3), kw.pop("d", 8), 0, False, False, 0)
    p.update(kw)
    return p


def test_curve_front_closed_form(oracle_core):
    p = _prob(family=0, m=2, d=10)
    x = np.zeros((50, 10))
    x[:, 0] = np.linspace(0, 1, 50)
    F, CV, _ = oracle_core.evaluate(p, x)
    assert np.allclose(F[:, 0], x[:, 0], rtol=0, atol=1e-15)
    assert np.allclose(F[:, 1], 1 - np.sqrt(x[:, 0]), rtol=0, atol=1e-14)
    assert np.all(CV == 0)
    # g = 1 + 9 mean(x2..xd): all ones gives g = 10, f2 = 10 (1 - sqrt(f1 / 10))
    x[:, 1:] = 1.0
    F, _, _ = oracle_core.evaluate(p, x)
    assert np.allclose(F[:, 1], 10 * (1 - np.sqrt(x[:, 0] / 10)), atol=1e-13)


@pytest.mark.parametrize("m", [2, 3])
def test_sphere_radius(oracle_core, m):
    p = _prob(family=1, m=m, d=12)
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 1, size=(200, 12))
    F, _, _ = oracle_core.evaluate(p, x)
    g = ((x[:, m - 1:] - 0.5) ** 2).sum(1)
    assert np.allclose(np.linalg.norm(F, axis=1), 1 + g, rtol=1e-13)
    x[:, m - 1:] = 0.5
    F, _, _ = oracle_core.evaluate(p, x)
    assert np.allclose(np.linalg.norm(F, axis=1), 1.0, rtol=1e-13)
    assert np.all(F >= 0)


def test_sphere_angle_assignment(oracle_core):
    p = _prob(family=1, m=3, d=5)
    x = np.array([[0.0, 0.0, 0.5, 0.5, 0.5], [0.0, 1.0, 0.5, 0.5, 0.5], [1.0, 0.3, 0.5, 0.5, 0.5]])
    F, _, _ = oracle_core.evaluate(p, x)
    assert np.allclose(F, [[1, 0, 0], [0, 1, 0], [0, 0, 1]], atol=1e-15)


def test_ring_and_cv(oracle_core):
    p = _prob(family=1, m=3, d=6)
    x0 = np.array([[0.3, 0.6, 0.5, 0.5, 0.5, 0.5]])
    F0, _, _ = oracle_core.evaluate(p, x0)
    # ring centred on F(x0): that ring contributes r^2
    p["ring_center"] = np.vstack([F0, [[5.0, 5.0, 5.0]]])
    p["ring_radius"] = np.array([0.25, 0.1])
    F, CV, CM = oracle_core.evaluate(p, x0)
    assert abs(CV[0] - 0.0625) < 1e-15 and abs(CM[0] - 0.0625) < 1e-15
    # far outside every ring: feasible, CV exactly 0, max constraint negative
    p["ring_center"] = np.array([[5.0, 5.0, 5.0], [-4.0, 0.0, 0.0]])
    F, CV, CM = oracle_core.evaluate(p, np.random.default_rng(9).uniform(0, 1, (100, 6)))
    assert np.all(CV == 0) and np.all(CM < 0)


def test_linear_and_equality(oracle_core):
    p = _prob(family=1, m=3, d=6)
    p["has_sum_lower"] = 1
    p["sum_lower"] = 1.5
    x = np.array([[0.3, 0.6, 0.5, 0.5, 0.5, 0.5]])
    F, CV, _ = oracle_core.evaluate(p, x)
    assert abs(CV[0] - max(0.0, 1.5 - F.sum())) < 1e-14
    p["has_sum_lower"] = 0
    p["n_eq"] = 1
    p["eq_tol"] = 1e-4
    for s, want in ((1.0, 0.0), (1.0 + 5e-5, 0.0), (1.0 + 3e-4, 2e-4), (0.5, 0.5 - 1e-4)):
        x = np.array([[s / 2, s / 2, 0.5, 0.5, 0.5, 0.5]])
        _, CV, _ = oracle_core.evaluate(p, x)
        assert abs(CV[0] - want) < 1e-12


def test_cv_sums_violations(oracle_core):
    # two rings both containing F and a violated linear bound: CV adds all three
    p = _prob(family=0, m=2, d=4)
    x = np.array([[0.25, 0.0, 0.0, 0.0]])  # F = (0.25, 0.5)
    p["ring_center"] = np.array([[0.25, 0.5], [0.35, 0.5]])
    p["ring_radius"] = np.array([0.2, 0.3])
    p["has_sum_lower"] = 1
    p["sum_lower"] = 1.0
    _, CV, CM = oracle_core.evaluate(p, x)
    want = 0.04 + (0.09 - 0.01) + 0.25
    assert abs(CV[0] - want) < 1e-14 and abs(CM[0] - 0.25) < 1e-14


# --------------------------------------------------------- aggregation ----

def test_pbi_closed_forms(oracle_core):
    rng = np.random.default_rng(10)
    for _ in range(300):
        m = int(rng.integers(2, 5))
        w = rng.uniform(0.01, 1, m)
        u = w / np.linalg.norm(w)
        z = rng.uniform(-1, 1, m)
        s = rng.uniform(0, 3)
        assert abs(oracle_core.agg(0, 5.0, z + s * u, w, z) - s) < 1e-12
        e = rng.normal(size=m)
        e -= e.dot(u) * u
        theta = rng.uniform(0, 10)
        g = oracle_core.agg(0, theta, z + s * u + e, w, z)
        assert abs(g - (s + theta * np.linalg.norm(e))) < 1e-11
        # scaling w leaves PBI unchanged
        g2 = oracle_core.agg(0, theta, z + s * u + e, 7.0 * w, z)
        assert abs(g - g2) < 1e-11


def test_tchebycheff_closed_form(oracle_core):
    # value: max_k w_k |f_k - z_k|
    assert oracle_core.agg(1, 5.0, [0.5, 2.0, 1.0], [0.2, 0.3, 0.5], [0.0, 1.0, -1.0]) == pytest.approx(1.0)
    # minimiser on the simplex sum f = 1 with z = 0 is f_k = (1/w_k) / sum_l (1/w_l)
    rng = np.random.default_rng(11)
    for m in (2, 3):
        w = rng.uniform(0.1, 1.0, m)
        want = (1 / w) / (1 / w).sum()
        pts = rng.dirichlet(np.ones(m), size=20000)
        z = np.zeros(m)
        vals = np.array([oracle_core.agg(1, 0.0, p, w, z) for p in pts])
        best = pts[np.argmin(vals)]
        assert np.allclose(best, want, atol=0.03)
        # the closed-form minimiser is at least as good as every sample; its value is 1 / sum(1/w)
        g_star = oracle_core.agg(1, 0.0, want, w, z)
        assert g_star <= vals.min() + 1e-12
        assert abs(g_star - 1.0 / (1 / w).sum()) < 1e-14


# ------------------------------------------------------------------ DE ----
# The DE operator of the LIR-CMOP experiments (CR = 1, F = 0.5), read as the
# neighbourhood form x_i + F (x_a - x_b) followed by polynomial mutation.

NO_PM = 0xFFFFFFFF  # a draw above every mutation threshold below


def test_de_special_cases(oracle_core):
    """F = 0.5 with x_i = x_b gives the midpoint of the two picks; equal picks
    leave x_i unchanged; F = 0 returns x_i; with x_i = x_a the mutant is the
    reflection of x_b through x_a scaled by one half."""
    rng = np.random.default_rng(11)
    tpm = 2**32 // 10
    for _ in range(500):
        xi, a, b = rng.uniform(0.2, 0.8, size=3)
        assert oracle_core.de_dim(b, a, b, 0.5, 0.0, 1.0, NO_PM, tpm, 20.0) == pytest.approx(0.5 * (a + b), abs=1e-15)
        assert oracle_core.de_dim(xi, a, a, 0.5, 0.0, 1.0, NO_PM, tpm, 20.0) == xi
        assert oracle_core.de_dim(xi, a, b, 0.0, 0.0, 1.0, NO_PM, tpm, 20.0) == xi
        v = oracle_core.de_dim(a, a, b, 0.5, -10.0, 10.0, NO_PM, tpm, 20.0)
        assert v - a == pytest.approx(0.5 * (a - b), abs=1e-15)


def test_de_clip_then_mutation(oracle_core):
    """The mutant is clipped to the box; a mutation draw then applies bounded PM
    to the clipped value (which stays in the box)."""
    tpm = 2**32 // 10
    assert oracle_core.de_dim(0.9, 1.0, 0.0, 0.5, 0.0, 1.0, NO_PM, tpm, 20.0) == 1.0
    assert oracle_core.de_dim(0.1, 0.0, 1.0, 0.5, 0.0, 1.0, NO_PM, tpm, 20.0) == 0.0
    rng = np.random.default_rng(12)
    for _ in range(500):
        xi, a, b = rng.uniform(0, 1, size=3)
        w = int(rng.integers(0, tpm))
        v = oracle_core.de_dim(xi, a, b, 0.5, 0.0, 1.0, w, tpm, 20.0)
        base = min(1.0, max(0.0, xi + 0.5 * (a - b)))
        assert v == oracle_core.pm_dim(base, 0.0, 1.0, w, tpm, 20.0)
        assert 0.0 <= v <= 1.0


def test_de_spread(oracle_core):
    """With x_i fixed at the centre and independent uniform picks, the mutant has
    mean x_i and variance F^2 (Var a + Var b) = 0.25 * 2 / 12 (no clipping can
    occur: |F (a - b)| <= 0.5)."""
    rng = np.random.default_rng(13)
    a, b = rng.uniform(0, 1, size=(2, 40000))
    v = np.array([oracle_core.de_dim(0.5, x, y, 0.5, 0.0, 1.0, NO_PM, 1, 20.0) for x, y in zip(a, b)])
    assert abs(v.mean() - 0.5) < 4 * math.sqrt(1 / 24 / v.size)
    assert abs(v.var() - 1 / 24) < 0.02 / 24 * 4


def test_de_generation_wiring(oracle_core):
    """In a whole generation with the DE operator, every offspring variable that
    drew no mutation equals clip(x_i + 0.5 (x_a - x_b)) for the recorded picks
    (a, b) and the subproblem's own row x_i of the same population."""
    prob, cfg, _ = ci.workload_small(3)
    cfg = dict(cfg, op=1)
    o = oracle_core.Oracle(prob, cfg)
    o.run(2)
    X = [o.X[0].copy(), o.X[1].copy()]
    dbg = o.step(debug=True)
    dv = o.dv
    N, d = o.N, o.d
    key = np.array(dv["key"], dtype=np.uint32)
    checked = 0
    for p in range(2):
        for i in range(N):
            a, b = dbg["mate"][p][i]
            for l in range(d):
                ctr = np.array([l >> 1, i, o.gen, (3 << 24) | (p << 16)], dtype=np.uint32)
                wB = int(oracle_core.philox(ctr[None, :], key)[0][2 * (l & 1) + 1])
                if wB < dv["tpm"]:
                    continue
                want = min(1.0, max(0.0, X[p][i, l] + 0.5 * (X[p][a, l] - X[p][b, l])))
                assert dbg["Xo"][p][i, l] == pytest.approx(want, abs=1e-15)
                checked += 1
    assert checked > 0.8 * 2 * N * d  # pm = 1/d mutates about one variable in d
