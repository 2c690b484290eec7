"""The package's reference fronts (used to measure delivered fronts by IGD on
the device) against the oracle's R21 fronts: each set lies close to the other
(both directions of the mean nearest distance are small) for seeded problems of
the batched and serving distributions."""
import numpy as np
import pytest

import cmop_inputs as ci
from oracle import metrics
from paper_2509_19821_amd import fronts


@pytest.mark.parametrize("q", range(6))
def test_reference_front_matches_oracle(q):
    prob, _ = ci.batch_instances(count=6, master_seed=3)[q]
    mine = fronts.reference_front(prob, n=1500)
    ref = metrics.reference_front(prob, density=120)
    assert mine.shape[1] == prob["m"] and mine.shape[0] > 20
    assert metrics.igd(ref, mine) < 0.02, q   # every oracle point has a close point here
    assert metrics.igd(mine, ref) < 0.02, q   # and the other way round
    # non-dominated and feasible by construction
    F = mine
    for c, r in zip(np.asarray(prob["ring_center"]).reshape(-1, prob["m"]), prob["ring_radius"]):
        assert np.all(((F - c) ** 2).sum(1) >= r * r - 1e-9)


def test_reference_front_rejects_uncovered():
    prob = ci.make_problem(ci.FAMILY_SPHERE, 3, 10, 1, False, True, 0)
    with pytest.raises(ValueError):
        fronts.reference_front(prob)
