"""Pins of the front filter (Eqs. (4)-(5), R20) and of IGD / HV (Eqs. (14)-(15))."""
import numpy as np
import pytest

import cmop_inputs as ci
from oracle import core, metrics


def _nd_matrix(F, CV):
    """Independent definition: dominance matrix over the feasible rows."""
    feas = CV == 0
    le = np.all(F[:, None, :] <= F[None, :, :], axis=2)
    lt = np.any(F[:, None, :] < F[None, :, :], axis=2)
    dom = le & lt & feas[:, None]  # dom[j, i]: feasible j dominates i
    return feas & ~dom.any(0)


@pytest.mark.parametrize("m,n", [(2, 300), (3, 500), (3, 1500)])
def test_front_against_dominance_matrix(m, n):
    rng = np.random.default_rng(m * 1000 + n)
    F = np.round(rng.uniform(0, 1, (n, m)), 2)  # coarse grid: many ties and duplicates
    CV = np.where(rng.random(n) < 0.3, rng.uniform(0, 1, n), 0.0)
    assert np.array_equal(core.front_mask(F, CV), _nd_matrix(F, CV))


def test_front_two_objective_sweep():
    rng = np.random.default_rng(1)
    F = rng.uniform(0, 1, (2000, 2))
    keep = core.front_mask(F, np.zeros(2000))
    order = np.lexsort((F[:, 1], F[:, 0]))
    best = np.inf
    want = np.zeros(2000, dtype=bool)
    for i in order:
        if F[i, 1] < best:
            want[i] = True
            best = F[i, 1]
    assert np.array_equal(keep, want)


@pytest.mark.parametrize("grid", [True, False])
def test_two_objective_filter_against_dominance_matrix(grid):
    """The sweep filter used for two-objective reference fronts keeps exactly
    the rows no other row dominates (duplicates and equal-f1 groups included)."""
    rng = np.random.default_rng(11 if grid else 12)
    for trial in range(60):
        n = int(rng.integers(1, 400))
        F = (rng.integers(0, 9, (n, 2)) / 8.0) if grid else rng.uniform(0, 1, (n, 2))
        want = _nd_matrix(F, np.zeros(n))
        assert np.array_equal(metrics.nd_mask_2d(F), want), trial


def test_front_keeps_duplicates_and_drops_infeasible():
    F = np.array([[0.1, 0.9], [0.1, 0.9], [0.5, 0.5], [0.05, 0.05]])
    CV = np.array([0.0, 0.0, 0.0, 0.3])
    assert list(core.front_mask(F, CV)) == [True, True, True, False]


def test_igd_closed_forms():
    P = np.random.default_rng(2).uniform(0, 1, (50, 3))
    assert metrics.igd(P, P) == 0.0
    ref = np.array([[0.0, 0.0], [3.0, 4.0]])
    assert metrics.igd(ref, np.array([[0.0, 0.0]])) == pytest.approx(2.5)
    assert metrics.igd(ref, np.array([[0.0, 0.0], [3.0, 0.0]])) == pytest.approx(2.0)


def test_hv_closed_forms():
    r = np.array([1.0, 1.0, 1.0])
    assert metrics.hv(np.array([[0.5, 0.25, 0.0]]), r) == pytest.approx(0.5 * 0.75 * 1.0)
    assert metrics.hv(np.array([[0.5, 0.5]]), r[:2]) == pytest.approx(0.25)
    # points beyond the reference point contribute nothing
    assert metrics.hv(np.array([[1.5, 0.0]]), r[:2]) == 0.0


@pytest.mark.parametrize("m", [2, 3])
def test_hv_against_inclusion_exclusion(m):
    rng = np.random.default_rng(10 + m)
    r = np.full(m, 1.1)
    for _ in range(20):
        P = rng.uniform(0, 1, (int(rng.integers(1, 8)), m))
        assert metrics.hv(P, r) == pytest.approx(metrics.hv_inclusion_exclusion(P, r), rel=1e-12)


def test_reference_front_small_problem():
    prob, _, _ = ci.workload_small(0)
    ref = metrics.reference_front(prob, density=100)
    assert ref.shape[0] > 500
    # every reference point is attainable, feasible and mutually non-dominated
    assert np.all(ref[:, 1] >= 1 - np.sqrt(np.clip(ref[:, 0], 0, 1)) - 1e-9)
    for c, rr in zip(prob["ring_center"], prob["ring_radius"]):
        assert np.all(((ref - c) ** 2).sum(1) >= rr * rr - 1e-9)
    assert core.front_mask(ref, np.zeros(len(ref))).all()


def test_reference_front_sphere_problem():
    prob, _, _ = ci.workload_medium(0)
    ref = metrics.reference_front(prob, density=60)
    assert ref.shape[0] > 200
    assert np.all(np.linalg.norm(ref, axis=1) >= 1 - 1e-9)
    assert np.all(ref.sum(1) >= prob["sum_lower"] - 1e-9)


@pytest.mark.parametrize("m,n", [(2, 30), (3, 40)])
def test_hv_monte_carlo_against_exact(m, n):
    """The Monte Carlo HV (the library's sampling rule) agrees with the exact
    sweep within five standard errors."""
    rng = np.random.default_rng(40 + m)
    P = rng.dirichlet(np.ones(m), size=n)
    r = np.full(m, 1.1)
    S = 1 << 16
    est = metrics.hv_mc(P, r, S, seed=7)
    exact = metrics.hv(P, r)
    vol = float(np.prod(r - P.min(0)))
    p = exact / vol
    assert abs(est - exact) <= 5 * vol * np.sqrt(p * (1 - p) / S)


@pytest.mark.parametrize("m", [5, 8])
def test_hv_monte_carlo_many_objectives(m):
    """m > 3: against inclusion-exclusion on tiny fronts, within five standard
    errors; a single point gives exactly the box (every sample is covered)."""
    rng = np.random.default_rng(50 + m)
    r = np.full(m, 1.2)
    P = rng.uniform(0.2, 0.9, (5, m))
    S = 1 << 15
    est = metrics.hv_mc(P, r, S, seed=3)
    exact = metrics.hv_inclusion_exclusion(P, r)
    vol = float(np.prod(r - P.min(0)))
    p = exact / vol
    assert abs(est - exact) <= 5 * vol * np.sqrt(p * (1 - p) / S)
    one = P[:1]
    assert metrics.hv_mc(one, r, 1000, seed=1) == pytest.approx(float(np.prod(r - one[0])), rel=1e-12)
    assert metrics.hv_mc(np.full((1, m), 2.0), r, 100) == 0.0
