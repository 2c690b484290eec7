"""Write-set check (GMPEA_CHECK_WRITES=1 at init): every generation's writes
are counted per target on the device and verified on the host: each
offspring row gets each chunk once and each offspring record once (variation,
OP1), and each parent slot gets at most one of a replacement (record and
location) or a move of its kept row home (location and every chunk), so the
selection's pull never writes a slot it does not own. The checked run must
also compute exactly what the unchecked run computes."""
import numpy as np
import pytest

import cmop_inputs as ci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


def _case(name):
    if name == "medium":
        prob, cfg, _ = ci.workload_medium(3)
        return prob, cfg
    if name == "small curve":
        prob, cfg, _ = ci.workload_small(4)
        return prob, cfg
    if name == "long rows (lane groups)":
        prob = ci.make_problem(ci.FAMILY_SPHERE, 3, 200, 2, True, False, 5)
        return prob, ci.method_config(1000, 20, 5)
    if name == "DE":
        prob, cfg, _ = ci.workload_medium(6)
        return prob, dict(cfg, op=1)
    if name == "m=5 two layers":
        prob = ci.make_problem(ci.FAMILY_SPHERE, 5, 14, 3, True, False, 7)
        return prob, ci.method_config(0, 20, 7, h_outer=6, h_inner=3)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["medium", "small curve", "long rows (lane groups)", "DE", "m=5 two layers"])
def test_write_sets_are_disjoint(G, name, monkeypatch):
    prob, cfg = _case(name)
    gens = 40  # past the arena's eight offspring generations, so kept rows move home
    monkeypatch.setenv("GMPEA_CHECK_WRITES", "1")
    gp = G.Gmpea(prob, cfg)
    monkeypatch.delenv("GMPEA_CHECK_WRITES")
    ref = G.Gmpea(prob, cfg)
    try:
        gp.step(gens)
        gp.sync()
        assert gp.info()["checked_generations"] == gens
        ref.step(gens)
        ref.sync()
        assert ref.info()["checked_generations"] == 0
        for p in range(2):
            for k in ("X", "F", "CV"):
                assert np.array_equal(gp.read(k, p), ref.read(k, p)), (name, k, p)
    finally:
        gp.close()
        ref.close()
