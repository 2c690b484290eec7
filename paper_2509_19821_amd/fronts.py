"""Reference fronts of the seeded synthetic CMOPs, for measuring delivered
fronts by IGD (Eq. (14)) on the device (gmpea_quality).

The paper measures on suites whose true fronts are published; the synthetic
problems here have none, so a reference front is built from what is known in
closed form. Every constraint lives in objective space (rings, the linear
bound), so the constrained front lies on the union of the attainable region's
lower boundary (g at its minimum: f2 = 1 - sqrt(f1) for the curve family, the
unit sphere octant for the sphere family) and the constraint surfaces (ring
boundaries, the plane sum F = sum_lower), restricted to the attainable region.
Points of that union are placed deterministically (lattice directions on the
sphere and the plane, even spacing on curves and circles), the infeasible ones
dropped, and the non-dominated rest kept. Problems with the decision-space
equality constraint are not covered (their front is not a union of these
surfaces).

Host-side numpy, measurement only: no part of the generation depends on it.
"""
from __future__ import annotations

import math

import numpy as np


def _simplex_lattice(m: int, n: int) -> np.ndarray:
    """Points of the unit simplex on the smallest lattice with at least n rows."""
    H = 1
    while math.comb(H + m - 1, m - 1) < n:
        H += 1
    rows = []

    def rec(prefix, left, k):
        if k == m - 1:
            rows.append(prefix + [left])
            return
        for v in range(left + 1):
            rec(prefix + [v], left - v, k + 1)

    rec([], H, 0)
    return np.asarray(rows, dtype=np.float64) / H


def _sphere_dirs(m: int, n: int) -> np.ndarray:
    """Unit vectors spread over the whole sphere (all octants), m = 2 or 3."""
    if m == 2:
        t = np.linspace(0.0, 2 * np.pi, n, endpoint=False)
        return np.stack([np.cos(t), np.sin(t)], 1)
    k = np.arange(n) + 0.5  # Fibonacci lattice
    z = 1.0 - 2.0 * k / n
    phi = k * np.pi * (3.0 - math.sqrt(5.0))
    rr = np.sqrt(1.0 - z * z)
    return np.stack([rr * np.cos(phi), rr * np.sin(phi), z], 1)


def _non_dominated(F: np.ndarray) -> np.ndarray:
    """Rows no other row dominates (<= everywhere, < somewhere); sorting by the
    objective sum first means a row can only be dominated by an earlier one."""
    F = F[np.argsort(F.sum(1), kind="stable")]
    keep = np.ones(F.shape[0], dtype=bool)
    for i in range(1, F.shape[0]):
        prev = F[:i][keep[:i]]
        le = np.all(prev <= F[i], axis=1)
        lt = np.any(prev < F[i], axis=1)
        keep[i] = not np.any(le & lt)
    return F[keep]


def reference_front(problem: dict, n: int = 2000) -> np.ndarray:
    """About n (before filtering) points of the constrained front of a seeded
    curve (m = 2) or sphere (m = 2, 3) problem without the equality constraint."""
    m = int(problem["m"])
    if problem.get("n_eq", 0):
        raise ValueError("reference_front: the equality constraint is not covered")
    if m > 3:
        raise ValueError("reference_front: written for m <= 3")
    centers = np.asarray(problem["ring_center"], dtype=np.float64).reshape(-1, m)
    radii = np.asarray(problem["ring_radius"], dtype=np.float64).reshape(-1)
    curve = int(problem["family"]) == 0
    parts = []
    if curve:
        f1 = np.linspace(0.0, 1.0, n)
        parts.append(np.stack([f1, 1.0 - np.sqrt(f1)], 1))

        def attainable(F):
            return (F[:, 0] >= 0) & (F[:, 0] <= 1) & (F[:, 1] >= 1.0 - np.sqrt(np.clip(F[:, 0], 0, 1)) - 1e-12)
    else:
        s = _simplex_lattice(m, n)
        parts.append(s / np.linalg.norm(s, axis=1, keepdims=True))

        def attainable(F):
            return np.all(F >= 0, axis=1) & (np.linalg.norm(F, axis=1) >= 1.0 - 1e-12)
    dirs = _sphere_dirs(m, n)
    for c, r in zip(centers, radii):
        ring = c + r * dirs
        parts.append(ring[attainable(ring)])
    if problem.get("has_sum_lower", 0):
        plane = _simplex_lattice(m, n) * float(problem["sum_lower"])
        parts.append(plane[attainable(plane)])
    F = np.concatenate(parts, 0)
    ok = np.ones(F.shape[0], dtype=bool)
    for c, r in zip(centers, radii):
        ok &= np.sum((F - c) ** 2, axis=1) >= r * r - 1e-12
    if problem.get("has_sum_lower", 0):
        ok &= F.sum(1) >= float(problem["sum_lower"]) - 1e-12
    return _non_dominated(F[ok])
