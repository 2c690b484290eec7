"""A caller's allocator hook and a caller's stream through gmpea_init: the
instance computes what it computes with its own memory and stream, the hook
sees every allocation and gets each one back once, a NULL from the hook is
ENOMEM with nothing kept, and the caller's stream outlives the instance."""
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


@pytest.fixture(scope="module")
def hip():
    L = ctypes.CDLL("libamdhip64.so.7")
    L.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    L.hipFree.argtypes = [ctypes.c_void_p]
    L.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    L.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    L.hipStreamQuery.argtypes = [ctypes.c_void_p]
    L.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    return L


class Hook:
    """Device memory from hipMalloc, every pointer tracked; `fail_at` makes
    that call (0-based) return NULL."""

    def __init__(self, G, hip, fail_at=None):
        self.hip, self.fail_at = hip, fail_at
        self.calls, self.live, self.freed, self.bad_frees = 0, {}, 0, 0
        from paper_2509_19821_amd import gmpea as binding
        self.fa, self.ff = binding.ALLOC_FN(self._alloc), binding.FREE_FN(self._free)
        self.al = binding.Allocator(self.fa, self.ff, None)

    def _alloc(self, nbytes, ctx):
        k = self.calls
        self.calls += 1
        if self.fail_at is not None and k == self.fail_at:
            return None
        p = ctypes.c_void_p()
        if self.hip.hipMalloc(ctypes.byref(p), nbytes) != 0:
            return None
        self.live[p.value] = nbytes
        return p.value

    def _free(self, ptr, ctx):
        if ptr not in self.live:
            self.bad_frees += 1
            return
        del self.live[ptr]
        self.freed += 1
        self.hip.hipFree(ptr)


def _final(gp):
    gp.sync()
    return {k: gp.read(k, p) for k in ("X", "F", "CV") for p in (0, 1)}


def _equal(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


def test_allocator_hook_and_caller_stream(G, hip):
    prob, cfg, _ = ci.workload_medium(1)
    ref = G.Gmpea(prob, cfg)
    try:
        ref.step(7)
        want = _final(ref)
    finally:
        ref.close()
    hook = Hook(G, hip)
    s = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(s)) == 0
    try:
        gp = G.Gmpea(prob, cfg, stream=s.value, allocator=hook.al)
        try:
            assert hook.calls >= 1 and hook.live
            assert gp.info()["device_bytes"] == sum(hook.live.values())
            gp.step(3)      # eager
            gp.step(0)      # capture the graph on the caller's stream
            gp.step(4)
            assert hip.hipStreamSynchronize(s) == 0
            got = _final(gp)
            fr = gp.front()
        finally:
            gp.close()
        assert _equal(got, want)
        assert len(fr["f"]) >= 1
        # every allocation came back once, and the caller's stream is still usable
        assert not hook.live and hook.freed == hook.calls and hook.bad_frees == 0
        assert hip.hipStreamQuery(s) == 0
    finally:
        hip.hipStreamDestroy(s)


@pytest.mark.parametrize("case", ["sphere m=3", "sphere m=5 two layers"])
def test_allocator_returning_null_is_enomem(G, hip, case):
    """NULL at each of the hook's calls in turn: ENOMEM, every block the hook
    handed out is returned, and a later init with a working hook succeeds."""
    if case == "sphere m=3":
        prob, cfg, _ = ci.workload_medium(0)
    else:
        prob = ci.make_problem(ci.FAMILY_SPHERE, 5, 12, 2, True, False, 3)
        cfg = ci.method_config(0, 10, 3, h_outer=4, h_inner=2)
    counting = Hook(G, hip)
    gp = G.Gmpea(prob, cfg, allocator=counting.al)
    gp.close()
    n_calls = counting.calls
    assert n_calls >= 1 and not counting.live
    for k in range(n_calls):
        hook = Hook(G, hip, fail_at=k)
        with pytest.raises(G.GmpeaError) as ei:
            G.Gmpea(prob, cfg, allocator=hook.al)
        assert ei.value.status == -2, (k, str(ei.value))
        assert not hook.live and hook.bad_frees == 0, k
    ok = Hook(G, hip)
    gp = G.Gmpea(prob, cfg, allocator=ok.al)
    try:
        gp.step(2)
        gp.sync()
    finally:
        gp.close()
    assert not ok.live
