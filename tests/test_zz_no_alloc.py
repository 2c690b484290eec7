"""gmpea_front_static (the front for callers that cannot allocate device
memory) against gmpea_front through the C ABI: the same rows, values and
errors on two calls in a row, the second on a smaller instance, for every
selector, with and without decision vectors; and its fixed-scratch limit."""
import ctypes

import numpy as np
import pytest

import cmop_inputs as ci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


def _front(fn, gp, what, cap, with_x):
    x = np.full((max(cap, 1), gp.d), np.nan, dtype=np.float32)
    f = np.full((max(cap, 1), gp.m), np.nan, dtype=np.float32)
    cv = np.full(max(cap, 1), np.nan, dtype=np.float32)
    idx = np.full(max(cap, 1), -7, dtype=np.int32)
    cnt = ctypes.c_int32(-1)
    st = fn(gp.handle, what, cap, x.ctypes.data if with_x else None, f.ctypes.data, cv.ctypes.data,
            idx.ctypes.data, ctypes.byref(cnt))
    return st, cnt.value, x, f, cv, idx


def test_front_static_equals_front(G):
    from paper_2509_19821_amd import gmpea as GM
    L = GM.lib()
    cases = [  # the second instance is the smaller input
        ("sphere m=3 d=30 N=5050", ci.make_problem(ci.FAMILY_SPHERE, 3, 30, 3, True, False, 41),
         ci.method_config(5000, 20, 41), 40),
        ("curve m=2 d=10 N=100", ci.make_problem(ci.FAMILY_CURVE, 2, 10, 2, False, False, 42),
         ci.method_config(100, 20, 42), 20),
    ]
    for label, prob, cfg, gens in cases:
        print("no-alloc front: %s" % label, flush=True)
        gp = G.Gmpea(prob, cfg)
        try:
            gp.step(gens)
            gp.sync()
            for what in (G.FRONT_FEASIBLE_ND, G.FRONT_POP1, G.FRONT_POP2):
                for with_x in (True, False):
                    a = _front(L.gmpea_front, gp, what, gp.n, with_x)
                    b = _front(L.gmpea_front_static, gp, what, gp.n, with_x)
                    assert a[0] == 0 and b[0] == 0, (label, what, a[0], b[0])
                    assert a[1] == b[1] and a[1] >= 1, (label, what, a[1], b[1])
                    for u, v in zip(a[2:], b[2:]):
                        assert np.array_equal(u, v, equal_nan=True), (label, what, with_x)
            # an undersized output: the same error and required count
            n_front = _front(L.gmpea_front, gp, G.FRONT_FEASIBLE_ND, gp.n, False)[1]
            a = _front(L.gmpea_front, gp, G.FRONT_FEASIBLE_ND, n_front - 1, True)
            b = _front(L.gmpea_front_static, gp, G.FRONT_FEASIBLE_ND, n_front - 1, True)
            assert a[0] == b[0] == -4 and a[1] == b[1] == n_front
        finally:
            gp.close()


def test_front_static_rejects_populations_beyond_its_scratch(G):
    """A population whose flags, row list and records exceed the fixed scratch
    is refused before any work (two objectives, about 1.7 million rows)."""
    from paper_2509_19821_amd import gmpea as GM
    prob = ci.make_problem(ci.FAMILY_CURVE, 2, 2, 1, False, False, 43)
    gp = G.Gmpea(prob, ci.method_config(1_700_000, 2, 43))
    try:
        st, cnt, *_ = _front(GM.lib().gmpea_front_static, gp, G.FRONT_POP1, 0, False)
        assert st == -6 and cnt == -1
        assert b"scratch" in GM.lib().gmpea_last_error()
    finally:
        gp.close()
