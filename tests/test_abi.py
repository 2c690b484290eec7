"""The C-ABI library loads, exports every function include/gmpea.h declares, and
rejects invalid input before any GPU work (no compute calls: CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import cmop_inputs as ci

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmpea.h")


@pytest.fixture(scope="module")
def glib():
    from paper_2509_19821_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    import paper_2509_19821_amd as g
    return g


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmpea_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("gmpea_init", "gmpea_step", "gmpea_run", "gmpea_front"):
        assert want in names


def test_library_exports_every_declared_symbol(glib):
    L = ctypes.CDLL(glib.lib_path())
    for name in _declared():
        assert hasattr(L, name), name


def _init(glib, prob, cfg, allocator=None):
    """Call gmpea_init directly; validation errors return before any HIP call."""
    from paper_2509_19821_amd import gmpea as G
    L = G.lib()
    m, d = prob["m"], prob["d"]
    keep = [np.ascontiguousarray(prob["lb"], dtype=np.float64),
            np.ascontiguousarray(prob["ub"], dtype=np.float64),
            np.ascontiguousarray(prob["ring_center"], dtype=np.float64).reshape(-1),
            np.ascontiguousarray(prob["ring_radius"], dtype=np.float64)]
    nr = keep[3].size
    P = G.Problem(prob["family"], m, d, keep[0].ctypes.data, keep[1].ctypes.data, nr,
                  keep[2].ctypes.data if nr else None, keep[3].ctypes.data if nr else None,
                  prob["has_sum_lower"], prob["sum_lower"], prob["n_eq"], prob["eq_tol"])
    C = G.Config(cfg["n_req"], cfg["T"], cfg["t1"], cfg["t2"], cfg["agg"], cfg["theta"],
                 cfg["eta_c"], cfg["eta_m"], cfg["pc"], cfg["pm"], cfg["seed"], 0,
                 cfg.get("op", 0), cfg.get("de_f", 0.0), cfg.get("op1_rule", 0),
                 cfg.get("h_outer", 0), cfg.get("h_inner", 0))
    h = ctypes.c_void_p()
    st = L.gmpea_init(ctypes.byref(P), ctypes.byref(C), ctypes.byref(allocator) if allocator else None,
                      None, ctypes.byref(h))
    if st == 0:
        L.gmpea_destroy(h)
    return st, L.gmpea_last_error().decode()


@pytest.mark.parametrize("mutate,code", [
    (lambda p, c: c.update(T=400), -1),                      # t2 = 800 > N = 100
    (lambda p, c: c.update(t1=101), -1),                     # t1 > N
    (lambda p, c: c.update(n_req=1), -1),                    # fewer than two subproblems
    (lambda p, c: p.update(ub=np.zeros(10)), -1),            # lb >= ub
    (lambda p, c: p.update(m=9), -6),                        # beyond the objectives supported
    (lambda p, c: p.update(m=4), -1),                        # the curve family has two
    (lambda p, c: p.update(family=1, m=8, d=6), -1),         # sphere: d below m - 1
    (lambda p, c: c.update(h_inner=2), -1),                  # inner layer without an outer one
    (lambda p, c: c.update(h_outer=-1), -1),                 # negative divisions
    (lambda p, c: p.update(family=7), -1),                   # unknown family
    (lambda p, c: c.update(agg=5), -1),                      # unknown aggregation
    (lambda p, c: c.update(pm=1.5), -1),                     # probability above 1
    (lambda p, c: c.update(op=2), -1),                       # unknown operator
    (lambda p, c: c.update(de_f=-0.5), -1),                  # negative DE scale
    (lambda p, c: c.update(op1_rule=3), -1),                 # unknown OP1 rule
    (lambda p, c: p.update(ring_center=np.zeros((9, 2)), ring_radius=np.zeros(9)), -1),
])
def test_init_rejects_invalid_input(glib, mutate, code):
    prob, cfg, _ = ci.workload_small(0)
    mutate(prob, cfg)
    st, msg = _init(glib, prob, cfg)
    assert st == code, msg
    assert msg


class _CountingHook:
    """An allocator hook that hands out nothing (NULL), counting its calls."""

    def __init__(self, G):
        self.calls = 0
        self.freed = 0
        self.fa = G.ALLOC_FN(self._alloc)
        self.ff = G.FREE_FN(self._free)
        self.al = G.Allocator(self.fa, self.ff, None)

    def _alloc(self, nbytes, ctx):
        self.calls += 1
        return None

    def _free(self, ptr, ctx):
        self.freed += 1


def test_allocator_hook_is_checked_before_use(glib):
    """An allocator without both callbacks is refused; invalid input is
    refused before the hook is called; with a hook that returns NULL, init
    fails with ENOMEM (or with EHIP where no device is visible, before any
    allocation) and frees nothing it was not given."""
    from paper_2509_19821_amd import gmpea as G
    prob, cfg, _ = ci.workload_small(0)
    hook = _CountingHook(G)
    half = G.Allocator(hook.fa, G.FREE_FN(), None)
    st, msg = _init(glib, prob, cfg, allocator=half)
    assert st == -1 and "allocator" in msg
    bad = dict(cfg, t1=101)
    st, msg = _init(glib, prob, bad, allocator=hook.al)
    assert st == -1 and hook.calls == 0 and hook.freed == 0
    st, msg = _init(glib, prob, cfg, allocator=hook.al)
    if G.device_count() == 0:
        assert st in (-2, -3), msg  # ENOMEM, or EHIP: no device for the stream or scratch
    else:
        assert st == -2 and hook.calls == 1, msg
    assert hook.freed == 0  # NULL is never handed back


def test_calls_on_dead_handles_are_rejected(glib):
    from paper_2509_19821_amd import gmpea as G
    L = G.lib()
    bogus = ctypes.c_void_p(0x1234)
    assert L.gmpea_step(bogus, 1) == -5
    assert L.gmpea_step(None, 1) == -5
    cnt = ctypes.c_int32(0)
    assert L.gmpea_front(bogus, 0, 0, None, None, None, None, ctypes.byref(cnt)) == -5
    L.gmpea_destroy(bogus)  # no-op
    L.gmpea_destroy(None)


def test_refuses_older_framework_runtime_in_process(glib):
    """A process that imported a PyTorch bundling an older HIP runtime than the
    library's toolchain is refused before the library is loaded."""
    import json
    import subprocess
    import sys
    info = json.load(open(os.path.join(os.path.dirname(glib.lib_path()), "build_info.json")))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import torch\n"
            "from paper_2509_19821_amd import gmpea as G\n"
            "have = G._version_tuple(torch.version.hip or '')\n"
            "built = G._version_tuple(%r)\n"
            "try:\n"
            "    G.lib(); print('loaded', have, built)\n"
            "except ImportError as e:\n"
            "    print('refused', have, built)\n") % (ROOT, info["hip_version"])
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    words = out.stdout.split()
    have = tuple(int(x) for x in "".join(words[1:3]).strip("()").split(","))
    built = tuple(int(x) for x in "".join(words[3:5]).strip("()").split(","))
    assert words[0] == ("refused" if have < built else "loaded")


@pytest.mark.parametrize("m,n_req,t", [(2, 100, 10), (2, 100, 40), (2, 700, 700), (2, 5, 1),
                                       (3, 1000, 10), (3, 1000, 40), (3, 300, 64), (3, 3000, 64),
                                       (3, 50, 55), (2, 20000, 40)])
def test_host_lattice_matches_bruteforce(glib, m, n_req, t):
    """The library's host lattice and neighbourhoods (the sorted-offset walk with
    its box-walk fallback) equal the oracle's brute-force search (Alg. 1
    initialisation: Das-Dennis rows, t nearest by squared lattice distance with
    ties by index)."""
    from oracle import core
    H, K, B = glib.lattice(m, n_req, t)
    assert H == core.dd_H(m, n_req)
    Ko = core.dd_lattice(m, H)
    assert np.array_equal(K, Ko)
    assert np.array_equal(B, core.knn(Ko, t))
    assert np.all(B[:, 0] == np.arange(K.shape[0]))


def test_host_lattice_rejects_invalid(glib):
    from paper_2509_19821_amd import gmpea as G
    with pytest.raises(G.GmpeaError):
        glib.lattice(9, 100, 10)
    with pytest.raises(G.GmpeaError):
        glib.lattice(2, 100, 101)
    H, n = ctypes.c_int32(0), ctypes.c_int32(0)
    K = np.empty((2, 2), dtype=np.int32)
    st = G.lib().gmpea_lattice(2, 100, 3, 2, K.ctypes.data, None, ctypes.byref(H), ctypes.byref(n))
    assert st == -4 and n.value == 100 and H.value == 99


@pytest.mark.parametrize("m,n_req,t", [(4, 200, 20), (5, 210, 20), (8, 120, 40), (6, 500, 10)])
def test_host_lattice_many_objectives(glib, m, n_req, t):
    """Single-layer lattices for m > 3 (the offset walk in m - 1 leading
    coordinates) against the oracle's brute force."""
    from oracle import core
    H, K, B = glib.lattice(m, n_req, t)
    Ko = core.dd_lattice(m, H)
    assert np.array_equal(K, Ko)
    assert np.array_equal(B, core.knn(Ko, t))


@pytest.mark.parametrize("m,h1,h2,t", [(8, 3, 2, 20), (5, 4, 2, 16), (4, 6, 3, 30), (2, 4, 2, 3),
                                       (6, 3, 0, 12), (3, 12, 6, 40)])
def test_host_reference_set_matches_oracle(glib, m, h1, h2, t):
    """The library's layered reference set (R28) and its brute-force neighbourhoods
    equal the oracle's, integer coordinates included."""
    from oracle import core
    K, B = glib.reference_set(m, h1, h2, t)
    _, Ko = core.reference_set(m, h1, h2)
    assert np.array_equal(K, Ko)
    assert np.array_equal(B, core.knn(Ko, t))


def test_host_reference_set_rejects_invalid(glib):
    from paper_2509_19821_amd import gmpea as G
    for args in ((9, 3, 2, 5), (4, 0, 2, 5), (4, 3, -1, 5), (4, 3, 2, 1000)):
        with pytest.raises(G.GmpeaError):
            glib.reference_set(*args)
    n = ctypes.c_int32(0)
    K = np.empty((2, 8), dtype=np.int32)
    st = G.lib().gmpea_reference_set(8, 3, 2, 5, 2, K.ctypes.data, None, ctypes.byref(n))
    assert st == -4 and n.value == 156
