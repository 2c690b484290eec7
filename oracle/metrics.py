"""Quality indicators and reference fronts. TEST INFRASTRUCTURE ONLY.

IGD follows Eq. (14), HV Eq. (15). The paper fixes neither the reference fronts
of synthetic problems nor the HV reference point, so two readings apply:
  R21  the reference front of a seeded problem is built once by densely sampling
       the attainable objective region's lower boundary together with every
       constraint surface, keeping feasible samples, then the non-dominated ones;
  R22  the HV reference point is 1.1 x the per-objective maximum of that front.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import core


def igd(ref: np.ndarray, P: np.ndarray) -> float:
    """Mean over reference points v of the Euclidean distance to the nearest row of P."""
    ref = np.asarray(ref, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    if P.shape[0] == 0:
        return float("inf")
    out = np.empty(ref.shape[0])
    step = max(1, 2_000_000 // max(1, P.shape[0]))
    for s in range(0, ref.shape[0], step):
        r = ref[s:s + step]
        d2 = ((r[:, None, :] - P[None, :, :]) ** 2).sum(-1)
        out[s:s + step] = np.sqrt(d2.min(1))
    return float(out.mean())


def hv2(P: np.ndarray, r: np.ndarray) -> float:
    """Exact 2-D hypervolume by a sweep over f1."""
    P = np.asarray(P, dtype=np.float64)
    P = P[np.all(P < r, axis=1)]
    if P.shape[0] == 0:
        return 0.0
    P = P[np.lexsort((P[:, 1], P[:, 0]))]
    area, best2 = 0.0, r[1]
    for k in range(P.shape[0]):
        if P[k, 1] < best2:
            x_next = r[0]
            area += (x_next - P[k, 0]) * (best2 - P[k, 1])
            best2 = P[k, 1]
    return float(area)


def hv3(P: np.ndarray, r: np.ndarray) -> float:
    """Exact 3-D hypervolume by slicing along f3 (2-D sweep per slab)."""
    P = np.asarray(P, dtype=np.float64)
    P = P[np.all(P < r, axis=1)]
    if P.shape[0] == 0:
        return 0.0
    P = P[np.argsort(P[:, 2], kind="stable")]
    vol = 0.0
    for k in range(P.shape[0]):
        top = P[k + 1, 2] if k + 1 < P.shape[0] else r[2]
        h = top - P[k, 2]
        if h > 0:
            vol += h * hv2(P[:k + 1, :2], r[:2])
    return float(vol)


def hv(P: np.ndarray, r: np.ndarray) -> float:
    P = np.asarray(P, dtype=np.float64)
    if P.shape[1] == 2:
        return hv2(P, r)
    if P.shape[1] == 3:
        return hv3(P, r)
    raise ValueError("hv: m must be 2 or 3")


def hv_inclusion_exclusion(P: np.ndarray, r: np.ndarray) -> float:
    """Brute-force HV over all subsets (tiny sets only): the measure of a union
    of boxes [p, r] by inclusion-exclusion."""
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    tot = 0.0
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            corner = P[list(S)].max(0)
            side = np.clip(r - corner, 0.0, None)
            tot += (-1) ** (k + 1) * float(np.prod(side))
    return tot


def hv_mc(P: np.ndarray, r: np.ndarray, samples: int, seed: int = 0, chunk: int = 1 << 16) -> float:
    """Monte Carlo HV (Eq. (15)) with the library's sampling rule, in FP64:
    sample s is uniform in the box from P's per-objective minimum to r, its
    coordinates u_k = (w_k >> 8) 2^-24 from Philox4x32-10 keyed by seed with
    counters (s mod 2^32, s >> 32, b, 4 << 24), b = 0 for objectives 1..4 and
    b = 1 for 5..8; a sample counts when some row of P is <= it in every
    objective. Returns box volume x covered share."""
    P = np.asarray(P, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    if P.shape[0] == 0:
        return 0.0
    m = P.shape[1]
    lo = P.min(0)
    vol = float(np.prod(np.clip(r - lo, 0.0, None)))
    if not vol > 0:
        return 0.0
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    hits = 0
    for s0 in range(0, samples, chunk):
        s = np.arange(s0, min(samples, s0 + chunk), dtype=np.uint64)
        words = []
        for b in range(2 if m > 4 else 1):
            ctr = np.stack([s & 0xFFFFFFFF, s >> 32, np.full_like(s, b),
                            np.full_like(s, 4 << 24)], 1).astype(np.uint32)
            words.append(core.philox(ctr, key))
        w = np.concatenate(words, 1)[:, :m].astype(np.float64)
        u = np.floor(w / 256.0) * 2.0 ** -24
        X = lo + u * (r - lo)
        covered = np.zeros(X.shape[0], dtype=bool)
        for q0 in range(0, P.shape[0], 256):
            covered |= np.any(np.all(P[None, q0:q0 + 256, :] <= X[:, None, :], axis=2), axis=1)
        hits += int(covered.sum())
    return vol * hits / samples


def _feasible_objective(prob: dict, F: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """Objective-space constraints (rings, linear bound) satisfied within tol."""
    ok = np.ones(F.shape[0], dtype=bool)
    for c, r in zip(np.asarray(prob["ring_center"]).reshape(-1, prob["m"]),
                    np.asarray(prob["ring_radius"]).reshape(-1)):
        ok &= ((F - c) ** 2).sum(1) >= r * r - tol
    if prob["has_sum_lower"]:
        ok &= F.sum(1) >= prob["sum_lower"] - tol
    return ok


def nd_mask_2d(F: np.ndarray) -> np.ndarray:
    """Non-dominated rows of a two-objective set (Eq. (4): q dominates p iff
    q <= p in both objectives and q < p in one), equal rows all kept, by a
    sweep in (f1, f2) order instead of all pairs: p is dominated iff some row
    with a smaller f1 has f2 <= p's f2, or a row with the same f1 has a
    smaller f2."""
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]
    keep = np.zeros(n, dtype=bool)
    if n == 0:
        return keep
    order = np.lexsort((F[:, 1], F[:, 0]))
    f1, f2 = F[order, 0], F[order, 1]
    # groups of equal f1 (each sorted by f2, so its first row has the least f2)
    start = np.concatenate([[True], f1[1:] != f1[:-1]])
    grp = np.cumsum(start) - 1
    gmin = f2[start]
    # smallest f2 among rows with a strictly smaller f1: the running minimum
    # over the earlier groups
    before = np.concatenate([[np.inf], np.minimum.accumulate(gmin)[:-1]])
    keep[order] = ~((before[grp] <= f2) | (gmin[grp] < f2))
    return keep


def _nd(F: np.ndarray) -> np.ndarray:
    if F.shape[1] == 2:
        return F[nd_mask_2d(F)]
    keep = core.front_mask(F, np.zeros(F.shape[0]))
    return F[keep]


def reference_front(prob: dict, density: int = 400) -> np.ndarray:
    """R21 reference front of a seeded problem (see the module docstring).
    Decision-space equality constraints restrict the sampled directions."""
    m = int(prob["m"])
    d = int(prob["d"])
    fam = int(prob["family"])
    pts = []
    centers = np.asarray(prob["ring_center"]).reshape(-1, m)
    radii = np.asarray(prob["ring_radius"]).reshape(-1)
    if fam == 0:
        if prob["n_eq"]:
            raise ValueError("reference_front: equality constraints need the sphere family")
        # lower boundary of the attainable region: f2 = 1 - sqrt(f1) (g = 1)
        s = np.linspace(0.0, 1.0, 40 * density + 1)
        pts.append(np.stack([s, 1.0 - np.sqrt(s)], 1))

        def attainable(F):
            f1, f2 = F[:, 0], F[:, 1]
            ok = (f1 >= 0) & (f1 <= 1)
            f1c = np.clip(f1, 0, 1)
            return ok & (f2 >= 1.0 - np.sqrt(f1c) - 1e-12) & (f2 <= 10.0 - np.sqrt(10.0 * f1c))

        th = np.linspace(0.0, 2 * np.pi, 40 * density, endpoint=False)
        for c, r in zip(centers, radii):
            ring = np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], 1)
            pts.append(ring[attainable(ring)])
        if prob["has_sum_lower"]:
            u = np.linspace(0.0, 1.0, 40 * density + 1)
            line = np.stack([u, prob["sum_lower"] - u], 1)
            pts.append(line[attainable(line)])
    else:
        rho_max = 1.0 + 0.25 * max(0, d - (m - 1))
        hp = np.pi / 2
        if prob["n_eq"]:
            if m != 3:
                raise ValueError("reference_front: equality sampling is written for m = 3")
            # directions with x1 + x2 = 1 (the equality), radius 1 + g >= 1
            a = np.linspace(0.0, 1.0, 40 * density + 1)
            dirs = np.stack([np.cos(hp * a) * np.cos(hp * (1 - a)),
                             np.cos(hp * a) * np.sin(hp * (1 - a)), np.sin(hp * a)], 1)
            rhos = np.linspace(1.0, min(rho_max, 3.0), 200)
            sheet = (rhos[None, :, None] * dirs[:, None, :]).reshape(-1, 3)
            pts.append(sheet)
        else:
            if m == 2:
                a = np.linspace(0.0, 1.0, 40 * density + 1)
                pts.append(np.stack([np.cos(hp * a), np.sin(hp * a)], 1))
            else:
                a, b = np.meshgrid(np.linspace(0, 1, density + 1), np.linspace(0, 1, density + 1))
                a, b = a.ravel(), b.ravel()
                pts.append(np.stack([np.cos(hp * a) * np.cos(hp * b),
                                     np.cos(hp * a) * np.sin(hp * b), np.sin(hp * a)], 1))

            def attainable(F):
                n = np.linalg.norm(F, axis=1)
                return np.all(F >= -1e-12, axis=1) & (n >= 1.0 - 1e-12) & (n <= rho_max)

            rng = np.random.default_rng(12345)
            for c, r in zip(centers, radii):
                v = rng.normal(size=(8 * density * density // 10 + 1000, m))
                v /= np.linalg.norm(v, axis=1, keepdims=True)
                sph = c + r * v
                pts.append(sph[attainable(sph)])
            if prob["has_sum_lower"]:
                u = rng.dirichlet(np.ones(m), size=4 * density * density // 10 + 1000)
                plane = u * prob["sum_lower"]
                pts.append(plane[attainable(plane)])
    F = np.concatenate(pts, 0)
    F = F[_feasible_objective(prob, F)]
    return _nd(F)
