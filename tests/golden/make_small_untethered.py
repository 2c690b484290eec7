"""Writes small_untethered_oracle.txt: the FP64 oracle's final-front quality on
the small workload (m = 2, d = 10, N = 100, T = 20, two rings, 100
generations) for seeds 0 .. 2047, one line per seed: seed, IGD (Eq. (14))
against the problem's reference front (reading R21, density 100), HV
(Eq. (15)) at 1.1 x that front's maximum (reading R22).

Calls only the oracle and the seeded input generators. Run from the
repository root:
    python tests/golden/make_small_untethered.py [--seeds 2048] [--jobs 8]
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_untethered_oracle.txt")


def oracle_quality(seed: int):
    """(IGD, HV) of the oracle's final feasible non-dominated front of population 1."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import cmop_inputs as ci
    from oracle import core, metrics
    core.set_threads(1)
    prob, cfg, K = ci.workload_small(seed)
    ref = metrics.reference_front(prob, density=100)
    o = core.Oracle(prob, cfg)
    o.run(K)
    fo = o.F[0][o.front(0)]
    return seed, metrics.igd(ref, fo), metrics.hv(fo, 1.1 * ref.max(0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=2048)
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    with mp.get_context("spawn").Pool(a.jobs) as pool:
        rows = pool.map(oracle_quality, range(a.seeds), chunksize=16)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle, small workload (m=2, d=10, N=100, T=20, 2 rings), 100 generations\n")
        fh.write("# written by tests/golden/make_small_untethered.py --seeds %d\n" % a.seeds)
        fh.write("# seed igd hv\n")
        for s, ig, hv in rows:
            fh.write("%d %.17g %.17g\n" % (s, ig, hv))


if __name__ == "__main__":
    main()
