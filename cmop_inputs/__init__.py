"""Seeded synthetic CMOP inputs shared by the oracle and the HIP path.

This module only draws problem constants and lists workload sizes. It holds
none of the method's arithmetic: no evaluation, no variation, no selection,
no derived parameters (neighbourhood sizes, mutation thresholds, RNG keys are
each side's own business).

The paper's benchmark suites (C-DTLZ, DC-DTLZ, LIR-CMOP, WTA) are not
available here; these seeded problems stand in for them. Both families follow
the CMOP statement of Eq. (1): minimise F(x) subject to inequality constraints
g(x) <= 0 and equality constraints h(x) = 0, on a box.

Families
--------
``curve`` (m = 2): f1 = x1, g = 1 + 9 mean(x2..xd), f2 = g (1 - sqrt(f1 / g)).
``sphere`` (m >= 2): a sphere-octant front in objective space, radius 1 + g
    with g = sum over the non-angle variables of (x - 0.5)^2.

Constraints (all in objective space unless stated)
--------------------------------------------------
``ring``   c_j = r_j^2 - ||F - a_j||^2 <= 0 (stay outside a ball), a_j ~ U[0.2, 1]^m,
           r_j ~ U[0.1, 0.3].
``linear`` sum_lower - sum_k f_k <= 0 with sum_lower = 1 + delta, delta ~ U[0, 0.2].
``equality`` h = x1 + x2 - 1 = 0 on the decision vector, with tolerance eq_tol.
"""
from __future__ import annotations

import math

import numpy as np

FAMILY_CURVE = 0
FAMILY_SPHERE = 1

_PROBLEM_STREAM = 0x434D4F50  # distinguishes problem draws from other uses of a seed
_BATCH_STREAM = 0x42415443
_SERVE_STREAM = 0x53455256


def make_problem(family: int, m: int, d: int, n_ring: int, linear: bool, equality: bool,
                 seed: int, eq_tol: float = 1e-6, lb=None, ub=None) -> dict:
    """Draw one seeded CMOP instance. Returns plain FP64 numpy arrays and ints."""
    rng = np.random.default_rng([int(seed), _PROBLEM_STREAM])
    centers = rng.uniform(0.2, 1.0, size=(n_ring, m))
    radii = rng.uniform(0.1, 0.3, size=n_ring)
    delta = rng.uniform(0.0, 0.2)
    return {
        "family": int(family),
        "m": int(m),
        "d": int(d),
        "lb": np.zeros(d) if lb is None else np.asarray(lb, dtype=np.float64).copy(),
        "ub": np.ones(d) if ub is None else np.asarray(ub, dtype=np.float64).copy(),
        "ring_center": np.ascontiguousarray(centers, dtype=np.float64),
        "ring_radius": np.ascontiguousarray(radii, dtype=np.float64),
        "has_sum_lower": int(bool(linear)),
        "sum_lower": float(1.0 + delta) if linear else 0.0,
        "n_eq": int(bool(equality)),
        "eq_tol": float(eq_tol),
    }


def method_config(n_req: int, T: int, seed: int, agg: int = 0, theta: float = 5.0,
                  t1: int = 0, t2: int = 0, eta_c: float = 20.0, eta_m: float = 20.0,
                  pc: float = 1.0, pm: float = 0.0, op: int = 0, de_f: float = 0.5,
                  op1_rule: int = 0, h_outer: int = 0, h_inner: int = 0) -> dict:
    """Raw method parameters (the paper's settings: theta = 5, eta = 20, pc = 1,
    pm = 1/d written as 0, t1 = T/2 and t2 = 2T written as 0; op 0 = SBX, op 1 =
    DE with F = 0.5 and CR = 1). h_outer > 0 gives the reference set's layer
    divisions explicitly (h_inner > 0 adds an inner layer) instead of n_req."""
    return {"n_req": int(n_req), "T": int(T), "t1": int(t1), "t2": int(t2), "agg": int(agg),
            "theta": float(theta), "eta_c": float(eta_c), "eta_m": float(eta_m),
            "pc": float(pc), "pm": float(pm), "seed": int(seed), "op": int(op),
            "de_f": float(de_f), "op1_rule": int(op1_rule), "h_outer": int(h_outer),
            "h_inner": int(h_inner)}


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def workload_small(seed: int = 0):
    """Two objectives, d = 10, N = 100, T = 20, two rings, 100 generations."""
    prob = make_problem(FAMILY_CURVE, 2, 10, 2, False, False, seed)
    return prob, method_config(100, 20, seed), 100


def workload_medium(seed: int = 0):
    """Three objectives, d = 30, N = 1,000, T = 20, three rings + linear bound,
    500 generations."""
    prob = make_problem(FAMILY_SPHERE, 3, 30, 3, True, False, seed)
    return prob, method_config(1000, 20, seed), 500


def workload_large(seed: int = 0):
    """Three objectives, d = 100, N = 100,000, T = 32, four rings + the equality
    x1 + x2 = 1 with tolerance 1e-4, 200 generations."""
    prob = make_problem(FAMILY_SPHERE, 3, 100, 4, False, True, seed, eq_tol=1e-4)
    return prob, method_config(100000, 32, seed), 200


def workload_many5(seed: int = 0):
    """Five objectives (sphere family), d = 14, one layer of N = 210 (H = 6),
    T = 20, three rings + linear bound, 300 generations."""
    prob = make_problem(FAMILY_SPHERE, 5, 14, 3, True, False, seed)
    return prob, method_config(210, 20, seed), 300


def workload_many8(seed: int = 0):
    """Eight objectives (sphere family), d = 17, two layers (H = 3 and 2:
    120 + 36 = 156 vectors), T = 20, two rings + linear bound, 300 generations."""
    prob = make_problem(FAMILY_SPHERE, 8, 17, 2, True, False, seed)
    return prob, method_config(156, 20, seed, h_outer=3, h_inner=2), 300


def workload_many_large(seed: int = 0, m: int = 8):
    """Many-objective throughput shape: m objectives (sphere family), d = 100,
    two layers of about 1e5 vectors per population (m = 5: H = 35 and 22,
    82,251 + 14,950; m = 8: H = 13 and 10, 77,520 + 19,448), T = 32, four rings
    + linear bound, 200 generations."""
    layers = {5: (35, 22), 8: (13, 10)}[m]
    prob = make_problem(FAMILY_SPHERE, m, 100, 4, True, False, seed)
    return prob, method_config(2, 32, seed, h_outer=layers[0], h_inner=layers[1]), 200


WORKLOADS = {"small": workload_small, "medium": workload_medium, "large": workload_large,
             "many5": workload_many5, "many8": workload_many8}


def batch_instances(count: int = 256, master_seed: int = 0, n_lo: int = 100,
                    n_hi: int = 20000, d_lo: int = 10, d_hi: int = 100, T: int = 20):
    """Uneven independent instances: N ~ U{n_lo..n_hi}, d ~ U{d_lo..d_hi},
    m in {2, 3}, q ~ U{1..4} rings; m = 2 draws the curve family, m = 3 the
    sphere family with a linear bound. Instance q evolves with seed q + 1."""
    rng = np.random.default_rng([int(master_seed), _BATCH_STREAM])
    out = []
    for q in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        m = int(rng.integers(2, 4))
        nr = int(rng.integers(1, 5))
        seed = q + 1
        if m == 2:
            prob = make_problem(FAMILY_CURVE, 2, d, nr, False, False, seed)
        else:
            prob = make_problem(FAMILY_SPHERE, 3, d, nr, True, False, seed)
        out.append((prob, method_config(n, T, seed)))
    return out


def serve_arrivals(rate: float = 200.0, window_s: float = 60.0, master_seed: int = 0,
                   d_lo: float = 0.01, d_hi: float = 1.0):
    """Poisson arrivals (exponential gaps at `rate` per second) over a window,
    each with a deadline drawn log-uniformly in [d_lo, d_hi] seconds."""
    rng = np.random.default_rng([int(master_seed), _SERVE_STREAM])
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= window_s:
            break
        dl = math.exp(rng.uniform(math.log(d_lo), math.log(d_hi)))
        out.append((t, dl))
    return out
