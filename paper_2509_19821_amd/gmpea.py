"""ctypes binding of libgmpea.so (include/gmpea.h). Argument marshalling only.

By default the library allocates its device memory with hipMalloc and enqueues
on a stream it owns, so nothing beyond the HIP runtime it was built against is
loaded. A caller may instead hand in a PyTorch stream and PyTorch's caching
allocator (device memory and streams only) when that PyTorch build's HIP
runtime is at least as new as the library's toolchain; the binding refuses a
process whose already-loaded PyTorch carries an older HIP runtime, because
both runtimes share one soname and the older one would serve the library.
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# GMPEA_LIBRARY names another build of the library (a debug or host-sanitizer
# build); by default the in-tree one
_LIB_PATH = os.environ.get("GMPEA_LIBRARY") or os.path.join(_PKG, "_build", "libgmpea.so")
_BUILD_INFO = os.path.join(os.path.dirname(_LIB_PATH), "build_info.json")

FAMILY_CURVE, FAMILY_SPHERE = 0, 1
OP_SBX, OP_DE = 0, 1
OP1_FPR, OP1_FEASIBLE_FIRST = 0, 1
AGG_PBI, AGG_TCHE = 0, 1
FRONT_FEASIBLE_ND, FRONT_POP1, FRONT_POP2 = 0, 1, 2
BUF = {"X": 0, "F": 1, "CV": 2, "XOFF": 3, "FOFF": 4, "CVOFF": 5, "Z": 6, "GEN": 7, "W": 8,
       "B": 9, "MATE": 10, "OP1": 11, "WIN": 12}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ECAPACITY", -5: "ESTATE",
          -6: "EUNSUPPORTED"}
EXPORTS = ["gmpea_init", "gmpea_step", "gmpea_run", "gmpea_front", "gmpea_get_info", "gmpea_read",
           "gmpea_write", "gmpea_destroy", "gmpea_last_error", "gmpea_sync", "gmpea_profile",
           "gmpea_philox", "gmpea_copy", "gmpea_pool_create", "gmpea_pool_admit",
           "gmpea_pool_step", "gmpea_pool_tune", "gmpea_pool_handle", "gmpea_pool_release",
           "gmpea_pool_query", "gmpea_pool_sync", "gmpea_pool_destroy", "gmpea_lattice",
           "gmpea_reference_set", "gmpea_quality", "gmpea_shape", "gmpea_copy_probe",
           "gmpea_front_static"]
COPY_STRIDED, COPY_WIDE, COPY_WIDE_NT, COPY_RUNTIME = 0, 1, 2, 3
PHASES = ("vary", "op1", "select")


class GmpeaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, message))
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("m", ctypes.c_int32), ("d", ctypes.c_int32),
                ("lb", ctypes.c_void_p), ("ub", ctypes.c_void_p), ("n_ring", ctypes.c_int32),
                ("ring_center", ctypes.c_void_p), ("ring_radius", ctypes.c_void_p),
                ("has_sum_lower", ctypes.c_int32), ("sum_lower", ctypes.c_double),
                ("n_eq", ctypes.c_int32), ("eq_tol", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("n_req", ctypes.c_int32), ("T", ctypes.c_int32), ("t1", ctypes.c_int32),
                ("t2", ctypes.c_int32), ("agg", ctypes.c_int32), ("theta", ctypes.c_double),
                ("eta_c", ctypes.c_double), ("eta_m", ctypes.c_double), ("pc", ctypes.c_double),
                ("pm", ctypes.c_double), ("seed", ctypes.c_uint64), ("record", ctypes.c_int32),
                ("op", ctypes.c_int32), ("de_f", ctypes.c_double), ("op1_rule", ctypes.c_int32),
                ("h_outer", ctypes.c_int32), ("h_inner", ctypes.c_int32)]


MAX_M = 8  # GMPEA_MAX_M

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("d", ctypes.c_int32),
                ("t1", ctypes.c_int32), ("t2", ctypes.c_int32), ("H", ctypes.c_int32),
                ("H2", ctypes.c_int32), ("generation", ctypes.c_int64), ("z", ctypes.c_float * MAX_M),
                ("replaced", ctypes.c_int64 * 2), ("feasible_frac", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("task_dealt", ctypes.c_int32),
                ("checked_generations", ctypes.c_int64)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def _version_tuple(text):
    parts = [int(p) for p in str(text).split(".")[:2] if p.isdigit()]
    return tuple(parts) if len(parts) == 2 else None


def _check_process_runtime():
    """Refuse to load next to an already-imported PyTorch whose bundled HIP
    runtime is older than the library's toolchain (same soname: that runtime
    would serve the library)."""
    torch = sys.modules.get("torch")
    if torch is None:
        return
    have = _version_tuple(getattr(getattr(torch, "version", None), "hip", None) or "")
    try:
        with open(_BUILD_INFO) as fh:
            built = _version_tuple(json.load(fh)["hip_version"])
    except (OSError, ValueError, KeyError):
        built = None
    if have is not None and built is not None and have < built:
        raise ImportError(
            "libgmpea.so was built with HIP %d.%d but this process already imported a PyTorch "
            "that bundles HIP %d.%d; load the library in a process without that PyTorch "
            "(or rebuild it with a matching toolchain)" % (built + have))


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libgmpea.so is not built (expected at %s); run "
                              "`python -m paper_2509_19821_amd.build`" % _LIB_PATH)
        _check_process_runtime()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.gmpea_init.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Config),
                                 ctypes.POINTER(Allocator), vp, ctypes.POINTER(vp)]
        L.gmpea_step.argtypes = [vp, i32]
        L.gmpea_run.argtypes = [vp, i32, ctypes.c_double, ctypes.POINTER(i32)]
        L.gmpea_front.argtypes = [vp, i32, i32, vp, vp, vp, vp, ctypes.POINTER(i32)]
        L.gmpea_front_static.argtypes = [vp, i32, i32, vp, vp, vp, vp, ctypes.POINTER(i32)]
        L.gmpea_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.gmpea_read.argtypes = [vp, i32, i32, vp, i64]
        L.gmpea_write.argtypes = [vp, i32, i32, vp, i64]
        L.gmpea_destroy.argtypes = [vp]
        L.gmpea_destroy.restype = None
        L.gmpea_last_error.restype = ctypes.c_char_p
        L.gmpea_philox.argtypes = [vp, i64, ctypes.c_uint64, vp, vp]
        L.gmpea_profile.argtypes = [vp, i32, vp]
        L.gmpea_sync.argtypes = [vp]
        L.gmpea_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.gmpea_copy_probe.argtypes = [vp, vp, ctypes.c_size_t, i32, i32, vp,
                                       ctypes.POINTER(ctypes.c_float)]
        L.gmpea_pool_create.argtypes = [ctypes.c_size_t, ctypes.POINTER(Allocator), vp,
                                        ctypes.POINTER(vp)]
        L.gmpea_pool_admit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(Config),
                                       ctypes.POINTER(i32)]
        L.gmpea_pool_step.argtypes = [vp, i32]
        L.gmpea_pool_tune.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.gmpea_pool_handle.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.gmpea_pool_release.argtypes = [vp, i32]
        L.gmpea_pool_query.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]
        L.gmpea_pool_sync.argtypes = [vp]
        L.gmpea_pool_destroy.argtypes = [vp]
        L.gmpea_pool_destroy.restype = None
        L.gmpea_lattice.argtypes = [i32, i32, i32, i32, vp, vp, ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]
        L.gmpea_reference_set.argtypes = [i32, i32, i32, i32, i32, vp, vp, ctypes.POINTER(i32)]
        L.gmpea_quality.argtypes = [vp, vp, i32, vp, i64, ctypes.c_uint64, vp, vp, vp]
        L.gmpea_shape.argtypes = [vp] + [ctypes.POINTER(i32)] * 5
        for name in EXPORTS:
            if name not in ("gmpea_destroy", "gmpea_last_error", "gmpea_pool_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise GmpeaError(status, lib().gmpea_last_error().decode(errors="replace"))


def _torch_allocator():
    """Allocator hook over torch's caching allocator (device memory only)."""
    import torch

    def _alloc(nbytes, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
        except Exception:  # out of memory -> NULL -> GMPEA_ENOMEM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    return Allocator(fa, ff, None), (fa, ff)


def _f64(a, n=None):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if n is not None and arr.size != n:
        raise ValueError("expected %d values, got %d" % (n, arr.size))
    return arr


class Gmpea:
    """One GMPEA instance resident on the GPU.

    problem: dict with family, m, d, lb, ub, ring_center (n_ring x m),
             ring_radius, has_sum_lower, sum_lower, n_eq, eq_tol.
    config:  dict with n_req, T, t1, t2, agg, theta, eta_c, eta_m, pc, pm, seed
             (and optionally record).
    stream:  None (a stream owned by the instance), a raw hipStream_t integer,
             or a torch.cuda.Stream.
    use_torch_allocator: take device memory from PyTorch's caching allocator
             instead of hipMalloc.
    allocator: an Allocator (device memory hook) instead of hipMalloc; its
             callbacks must stay alive until the instance is closed.
    """

    def __init__(self, problem: dict, config: dict, stream=None, use_torch_allocator=False,
                 record: bool = False, allocator=None):
        L = lib()
        self._h = None
        self._owned = True
        self._prob, self._cfg, self._keep = _structs(problem, config, record)
        self._alloc = None
        if allocator is not None and use_torch_allocator:
            raise ValueError("give allocator or use_torch_allocator, not both")
        if allocator is not None:
            self._alloc = allocator
        elif use_torch_allocator:
            self._alloc, self._cb = _torch_allocator()
        self.stream = self._stream_handle(stream)
        h = ctypes.c_void_p()
        _check(L.gmpea_init(ctypes.byref(self._prob), ctypes.byref(self._cfg),
                            ctypes.byref(self._alloc) if self._alloc else None,
                            ctypes.c_void_p(self.stream) if self.stream else None, ctypes.byref(h)))
        self._h = h
        self._describe()

    def _describe(self):
        v = [ctypes.c_int32(0) for _ in range(5)]
        _check(lib().gmpea_shape(self._h, *[ctypes.byref(x) for x in v]))  # no device access
        self.n, self.m, self.d = v[0].value, v[1].value, v[2].value
        self.t = (v[3].value, v[4].value)

    @classmethod
    def _borrow(cls, handle, keep):
        """View of a handle owned elsewhere (a pool slot); never destroyed here."""
        obj = cls.__new__(cls)
        obj._h = handle
        obj._owned = False
        obj._keep = keep
        obj._describe()
        return obj

    @staticmethod
    def _stream_handle(stream):
        if stream is None:
            return 0
        if isinstance(stream, int):
            return stream
        return int(stream.cuda_stream)

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if self._h is not None:
            if getattr(self, "_owned", True):
                lib().gmpea_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- calls ----------------------------------------------------------------
    def step(self, n_gen: int = 1):
        _check(lib().gmpea_step(self._h, int(n_gen)))

    def sync(self):
        _check(lib().gmpea_sync(self._h))

    def run(self, max_gen: int, time_limit_s: float = 0.0) -> int:
        done = ctypes.c_int32(0)
        _check(lib().gmpea_run(self._h, int(max_gen), float(time_limit_s), ctypes.byref(done)))
        return int(done.value)

    def front(self, what: int = FRONT_FEASIBLE_ND, with_x: bool = True) -> dict:
        """Rows of a front selector; with_x=False leaves the decision vectors
        on the device (the returned "x" is empty)."""
        # one call with room for the whole population (the front is a subset)
        cnt = ctypes.c_int32(0)
        n = self.n
        x = np.empty((n if with_x else 0, self.d), dtype=np.float32)
        f = np.empty((n, self.m), dtype=np.float32)
        cv = np.empty(n, dtype=np.float32)
        idx = np.empty(n, dtype=np.int32)
        _check(lib().gmpea_front(self._h, int(what), n, x.ctypes.data if with_x else None,
                                 f.ctypes.data, cv.ctypes.data, idx.ctypes.data, ctypes.byref(cnt)))
        k = int(cnt.value)
        return {"x": x[:k].copy(), "f": f[:k].copy(), "cv": cv[:k].copy(), "idx": idx[:k].copy()}

    def quality(self, ref=None, hv_point=None, hv_samples: int = 1 << 20, hv_seed: int = 0) -> dict:
        """gmpea_quality: IGD against the reference points `ref` (n x m) and the
        Monte Carlo HV below `hv_point`, both computed on the device from the
        feasible non-dominated rows of population 1 (either may be None)."""
        igd, hv, cnt = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_int32(0)
        r = None if ref is None else np.ascontiguousarray(ref, dtype=np.float32).reshape(-1, self.m)
        hp = None if hv_point is None else np.ascontiguousarray(hv_point, dtype=np.float32).reshape(self.m)
        _check(lib().gmpea_quality(self._h, None if r is None else r.ctypes.data,
                                   0 if r is None else r.shape[0],
                                   None if hp is None else hp.ctypes.data, int(hv_samples),
                                   int(hv_seed) & 0xFFFFFFFFFFFFFFFF,
                                   None if r is None else ctypes.byref(igd),
                                   None if hp is None else ctypes.byref(hv), ctypes.byref(cnt)))
        return {"igd": None if r is None else float(igd.value),
                "hv": None if hp is None else float(hv.value), "front_count": int(cnt.value)}

    def profile(self, n_gen: int) -> dict:
        """Mean per-kernel durations (ms) over n_gen generations, HIP events on
        the handle's stream, and the variation kernel's mean over n_gen
        launches back to back ("vary_back_to_back")."""
        ms = np.zeros(len(PHASES) + 1, dtype=np.float32)  # one mean per phase, then vary back to back
        _check(lib().gmpea_profile(self._h, int(n_gen), ms.ctypes.data))
        out = dict(zip(PHASES, (float(v) for v in ms)))
        out["vary_back_to_back"] = float(ms[len(PHASES)])
        return out

    def info(self) -> dict:
        inf = Info()
        _check(lib().gmpea_get_info(self._h, ctypes.byref(inf)))
        return {"n": inf.n, "m": inf.m, "d": inf.d, "t1": inf.t1, "t2": inf.t2, "H": inf.H, "H2": inf.H2,
                "generation": int(inf.generation), "z": np.array(inf.z[:inf.m], dtype=np.float32),
                "replaced": (int(inf.replaced[0]), int(inf.replaced[1])),
                "feasible_frac": float(inf.feasible_frac), "device_bytes": int(inf.device_bytes),
                "task_dealt": bool(inf.task_dealt), "checked_generations": int(inf.checked_generations)}

    def _shape(self, name: str, pop: int):
        n, m, d = self.n, self.m, self.d
        return {"X": ((n, d), np.float32), "XOFF": ((n, d), np.float32), "F": ((n, m), np.float32),
                "FOFF": ((n, m), np.float32), "CV": ((n,), np.float32), "CVOFF": ((n,), np.float32),
                "Z": ((m,), np.float32), "GEN": ((1,), np.int64), "W": ((n, m), np.float32),
                "B": ((n, self.t[pop]), np.int32), "MATE": ((n, 2), np.int32),
                "OP1": ((n,), np.uint8), "WIN": ((n,), np.int32)}[name]

    def read(self, name: str, pop: int = 0) -> np.ndarray:
        shape, dt = self._shape(name, pop)
        out = np.empty(shape, dtype=dt)
        _check(lib().gmpea_read(self._h, BUF[name], int(pop), out.ctypes.data, int(out.size)))
        return out

    def write(self, name: str, arr, pop: int = 0):
        shape, dt = self._shape(name, pop)
        a = np.ascontiguousarray(np.asarray(arr, dtype=dt).reshape(shape))
        _check(lib().gmpea_write(self._h, BUF[name], int(pop), a.ctypes.data, int(a.size)))

    def state(self) -> dict:
        """Snapshot of both populations, the ideal point and the generation count."""
        return {"X": [self.read("X", p) for p in range(2)], "F": [self.read("F", p) for p in range(2)],
                "CV": [self.read("CV", p) for p in range(2)], "z": self.read("Z"),
                "gen": int(self.read("GEN")[0])}

    def load_state(self, s: dict):
        for p in range(2):
            self.write("X", s["X"][p], p)
            self.write("F", s["F"][p], p)
            self.write("CV", s["CV"][p], p)
        self.write("Z", s["z"])
        self.write("GEN", np.array([s["gen"]], dtype=np.int64))


def copy(src_dev_ptr: int, dst_dev_ptr: int, nbytes: int, stream: int = 0):
    """The library's streaming copy kernel (bandwidth reference)."""
    _check(lib().gmpea_copy(ctypes.c_void_p(src_dev_ptr), ctypes.c_void_p(dst_dev_ptr), int(nbytes),
                            ctypes.c_void_p(stream) if stream else None))


def copy_probe(src_dev_ptr: int, dst_dev_ptr: int, nbytes: int, mode: int, reps: int = 5,
               stream: int = 0) -> float:
    """Fastest of `reps` timed copies (milliseconds) in one of the COPY_* forms."""
    ms = ctypes.c_float(0.0)
    _check(lib().gmpea_copy_probe(ctypes.c_void_p(src_dev_ptr), ctypes.c_void_p(dst_dev_ptr),
                                  int(nbytes), int(mode), int(reps),
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(ms)))
    return float(ms.value)


def philox(ctr_dev_ptr: int, n: int, seed: int, out_dev_ptr: int, stream: int = 0):
    """Philox4x32-10 blocks on the device (pointers to n x 4 uint32 each)."""
    _check(lib().gmpea_philox(ctypes.c_void_p(ctr_dev_ptr), int(n), int(seed) & 0xFFFFFFFFFFFFFFFF,
                              ctypes.c_void_p(out_dev_ptr), ctypes.c_void_p(stream) if stream else None))


def lattice(m: int, n_req: int, t: int):
    """(H, K, B) of gmpea_lattice: Das-Dennis lattice rows (N x m) and the t
    nearest rows of each (N x t), computed on the host."""
    H, n = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().gmpea_lattice(int(m), int(n_req), int(t), 0, None, None, ctypes.byref(H),
                               ctypes.byref(n)))
    K = np.empty((n.value, int(m)), dtype=np.int32)
    B = np.empty((n.value, int(t)), dtype=np.int32)
    _check(lib().gmpea_lattice(int(m), int(n_req), int(t), n.value, K.ctypes.data, B.ctypes.data,
                               ctypes.byref(H), ctypes.byref(n)))
    return int(H.value), K, B


def reference_set(m: int, h_outer: int, h_inner: int, t: int):
    """(K, B) of gmpea_reference_set: the layered reference set as integers over
    2 m h_outer h_inner (N x m) and the t nearest rows of each (N x t), on the host."""
    n = ctypes.c_int32(0)
    _check(lib().gmpea_reference_set(int(m), int(h_outer), int(h_inner), int(t), 0, None, None,
                                     ctypes.byref(n)))
    K = np.empty((n.value, int(m)), dtype=np.int32)
    B = np.empty((n.value, int(t)), dtype=np.int32)
    _check(lib().gmpea_reference_set(int(m), int(h_outer), int(h_inner), int(t), n.value,
                                     K.ctypes.data, B.ctypes.data, ctypes.byref(n)))
    return K, B


def _structs(problem: dict, config: dict, record: bool = False):
    m, d = int(problem["m"]), int(problem["d"])
    nr = int(np.asarray(problem["ring_radius"]).size)
    keep = [_f64(problem["lb"], d), _f64(problem["ub"], d),
            _f64(problem["ring_center"], nr * m), _f64(problem["ring_radius"], nr)]
    lb, ub, rc, rr = keep
    P = Problem(int(problem["family"]), m, d, lb.ctypes.data, ub.ctypes.data, nr,
                rc.ctypes.data if nr else None, rr.ctypes.data if nr else None,
                int(problem["has_sum_lower"]), float(problem["sum_lower"]), int(problem["n_eq"]),
                float(problem["eq_tol"]))
    c = config
    C = Config(int(c["n_req"]), int(c["T"]), int(c.get("t1", 0)), int(c.get("t2", 0)),
               int(c.get("agg", 0)), float(c.get("theta", 0.0)), float(c.get("eta_c", 0.0)),
               float(c.get("eta_m", 0.0)), float(c.get("pc", 0.0)), float(c.get("pm", 0.0)),
               int(c["seed"]) & 0xFFFFFFFFFFFFFFFF, 1 if (record or c.get("record", 0)) else 0,
               int(c.get("op", 0)), float(c.get("de_f", 0.0)), int(c.get("op1_rule", 0)),
               int(c.get("h_outer", 0)), int(c.get("h_inner", 0)))
    return P, C, keep


class Pool:
    """Resident instances advanced together by batched generations.
    Results per instance are bit-identical to running that instance alone."""

    def __init__(self, budget_bytes: int, stream=None):
        L = lib()
        self._q = None
        h = ctypes.c_void_p()
        _check(L.gmpea_pool_create(int(budget_bytes), None,
                                   ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
        self._q = h
        self._views = {}

    def admit(self, problem: dict, config: dict, record: bool = False) -> int:
        P, C, keep = _structs(problem, config, record)
        slot = ctypes.c_int32(-1)
        _check(lib().gmpea_pool_admit(self._q, ctypes.byref(P), ctypes.byref(C), ctypes.byref(slot)))
        return int(slot.value)

    def try_admit(self, problem: dict, config: dict, record: bool = False):
        """Slot index, or None when the instance does not fit the budget."""
        try:
            return self.admit(problem, config, record)
        except GmpeaError as e:
            if e.status == -2:
                return None
            raise

    def step(self, n_gen: int = 1):
        _check(lib().gmpea_pool_step(self._q, int(n_gen)))

    def tune(self, n_gen: int) -> int:
        done = ctypes.c_int32(0)
        _check(lib().gmpea_pool_tune(self._q, int(n_gen), ctypes.byref(done)))
        return int(done.value)

    def sync(self):
        _check(lib().gmpea_pool_sync(self._q))

    def instance(self, slot: int) -> "Gmpea":
        """Borrowed view of one slot (front, read, write, info, step)."""
        v = self._views.get(slot)
        if v is None:
            h = ctypes.c_void_p()
            _check(lib().gmpea_pool_handle(self._q, int(slot), ctypes.byref(h)))
            v = Gmpea._borrow(h, self)
            self._views[slot] = v
        return v

    def release(self, slot: int):
        v = self._views.pop(slot, None)
        if v is not None:
            v._h = None
        _check(lib().gmpea_pool_release(self._q, int(slot)))

    def query(self) -> dict:
        a, s, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        u, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(lib().gmpea_pool_query(self._q, ctypes.byref(a), ctypes.byref(u), ctypes.byref(b),
                                      ctypes.byref(s), ctypes.byref(c)))
        return {"active": a.value, "used_bytes": u.value, "budget_bytes": b.value,
                "schedule": s.value, "chunk": c.value}

    def close(self):
        if self._q is not None:
            for v in self._views.values():
                v._h = None
            self._views.clear()
            lib().gmpea_pool_destroy(self._q)
            self._q = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class DeviceBuffer:
    """Raw device memory from the HIP runtime that serves the library (for
    handing device pointers to gmpea_philox without another framework)."""

    def __init__(self, nbytes: int):
        lib()
        self._hip = ctypes.CDLL("libamdhip64.so.7")
        self._hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self._hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int]
        self._hip.hipFree.argtypes = [ctypes.c_void_p]
        self.ptr = ctypes.c_void_p()
        self.nbytes = int(nbytes)
        if self._hip.hipMalloc(ctypes.byref(self.ptr), self.nbytes) != 0:
            raise MemoryError("hipMalloc(%d) failed" % self.nbytes)

    def upload(self, arr: np.ndarray):
        a = np.ascontiguousarray(arr)
        assert a.nbytes <= self.nbytes
        if self._hip.hipMemcpy(self.ptr, a.ctypes.data, a.nbytes, 1) != 0:  # host to device
            raise RuntimeError("hipMemcpy to device failed")

    def download(self, out: np.ndarray):
        assert out.flags["C_CONTIGUOUS"] and out.nbytes <= self.nbytes
        if self._hip.hipMemcpy(out.ctypes.data, self.ptr, out.nbytes, 2) != 0:  # device to host
            raise RuntimeError("hipMemcpy to host failed")
        return out

    def free(self):
        if self.ptr:
            self._hip.hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def device_count() -> int:
    """GPUs visible to the HIP runtime that serves the library."""
    lib()
    hip = ctypes.CDLL("libamdhip64.so.7")
    n = ctypes.c_int(0)
    if hip.hipGetDeviceCount(ctypes.byref(n)) != 0:
        return 0
    return int(n.value)
