"""The paper's neighbourhood ablation on the synthetic problems: GMPEA
(population 1 small, population 2 large: t1 = T/2, t2 = 2T) against GMPEA-S
(both small) and GMPEA-L (both large), plus the OP1 feasibility-first variant
and Tchebycheff aggregation, all on the GPU path with the same seeds. Prints
the mean IGD table (reference fronts as for the untethered runs); asserts only
that every variant ends with a non-empty feasible front of finite IGD, since the
ranking is an empirical outcome, not a property."""
import numpy as np
import pytest

import cmop_inputs as ci
from oracle import metrics

pytestmark = pytest.mark.gpu

SEEDS = range(5)


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


def _variants(cfg):
    T = cfg["T"]
    return {
        "GMPEA": dict(cfg),
        "GMPEA-S": dict(cfg, t1=max(1, T // 2), t2=max(1, T // 2)),
        "GMPEA-L": dict(cfg, t1=2 * T, t2=2 * T),
        "OP1 feasible-first": dict(cfg, op1_rule=1),
        "Tchebycheff": dict(cfg, agg=1),
    }


@pytest.mark.parametrize("which", ["small", "medium"])
def test_neighbourhood_ablation(G, which):
    rows = {}
    for s in SEEDS:
        prob, cfg, K = ci.WORKLOADS[which](s)
        ref = metrics.reference_front(prob, density=100)
        for name, c in _variants(cfg).items():
            gp = G.Gmpea(prob, c)
            try:
                gp.run(K)
                f = gp.front()["f"].astype(np.float64)
            finally:
                gp.close()
            assert f.shape[0] > 0, (which, name, s)
            v = metrics.igd(ref, f)
            assert np.isfinite(v)
            rows.setdefault(name, []).append(v)
    print("\n%s workload, mean IGD (std) over %d seeds:" % (which, len(SEEDS)))
    for name, v in rows.items():
        print("  %-20s %.6f (%.6f)" % (name, np.mean(v), np.std(v)), flush=True)
