"""ctypes front end of the FP64 C oracle (gmpea_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU legs
of the benchmark (its baseline and the CPU columns of its sweeps); never by
the product path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmpea_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
# GMPEA_ORACLE_LIBRARY names another build of the oracle (a sanitizer build),
# used as it is
_SO_ENV = os.environ.get("GMPEA_ORACLE_LIBRARY")
_DEFAULT_SO = os.path.join(_OUT_DIR, "libgmpea_oracle.so")
_SO = _SO_ENV or _DEFAULT_SO
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Always rebuilds when force."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_DEFAULT_SO):
        tmp = _DEFAULT_SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp,
               _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _DEFAULT_SO)
    return _DEFAULT_SO


class Problem(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("m", ctypes.c_int32), ("d", ctypes.c_int32),
                ("lb", ctypes.c_void_p), ("ub", ctypes.c_void_p),
                ("n_ring", ctypes.c_int32), ("ring_center", ctypes.c_void_p),
                ("ring_radius", ctypes.c_void_p), ("has_sum_lower", ctypes.c_int32),
                ("sum_lower", ctypes.c_double), ("n_eq", ctypes.c_int32),
                ("eq_tol", ctypes.c_double)]


class Cfg(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("d", ctypes.c_int32), ("N", ctypes.c_int32),
                ("t", ctypes.c_int32 * 2), ("B", ctypes.c_void_p * 2), ("W", ctypes.c_void_p),
                ("agg", ctypes.c_int32), ("theta", ctypes.c_double),
                ("eta_c", ctypes.c_double), ("eta_m", ctypes.c_double),
                ("tpm", ctypes.c_uint64), ("tpc", ctypes.c_uint64),
                ("key", ctypes.c_uint32 * 2), ("n_eq", ctypes.c_int32), ("eq_tol", ctypes.c_double),
                ("f32", ctypes.c_int32), ("op", ctypes.c_int32), ("de_f", ctypes.c_double),
                ("op1_rule", ctypes.c_int32)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not _SO_ENV and (not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC)):
                build(force=True)
            L = ctypes.CDLL(_SO)
            vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
            L.orc_philox_many.argtypes = [i64, vp, vp, vp]
            L.orc_dd_count.argtypes = [i32, i32]
            L.orc_dd_count.restype = i64
            L.orc_dd_H.argtypes = [i32, i64]
            L.orc_dd_H.restype = i32
            L.orc_dd_lattice.argtypes = [i32, i32, vp]
            L.orc_dd_lattice.restype = i64
            L.orc_knn.argtypes = [vp, i64, i32, i32, vp]
            L.orc_knn.restype = i32
            L.orc_eval.argtypes = [vp, i64, vp, vp, vp, vp]
            L.orc_agg.argtypes = [i32, ctypes.c_double, i32, vp, vp, vp]
            L.orc_agg.restype = ctypes.c_double
            L.orc_sbx_dim.argtypes = [ctypes.c_double, ctypes.c_double, u32, ctypes.c_double,
                                      vp, vp]
            L.orc_sbx_dim.restype = ctypes.c_double
            L.orc_pm_dim.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, u32,
                                     ctypes.c_uint64, ctypes.c_double]
            L.orc_pm_dim.restype = ctypes.c_double
            L.orc_mate.argtypes = [u32, u32, i32, vp, vp]
            L.orc_de_dim.argtypes = [ctypes.c_double] * 6 + [u32, ctypes.c_uint64, ctypes.c_double]
            L.orc_de_dim.restype = ctypes.c_double
            L.orc_select.argtypes = [vp] * 18
            L.orc_reproduce.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp, vp, vp]
            L.orc_ideal.argtypes = [i64, i32, vp, vp]
            L.orc_generation.argtypes = [vp, vp, u32] + [vp] * 17
            L.orc_generation.restype = i64
            L.orc_init_x.argtypes = [vp, i32, vp, i32, vp]
            L.orc_front.argtypes = [i64, i32, vp, vp, vp]
            L.orc_front.restype = i64
            L.orc_set_threads.argtypes = [i32]
            L.orc_set_threads.restype = i32
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def set_threads(n: int) -> int:
    """Set the OpenMP thread count (n <= 0 keeps it); returns the count in use."""
    return int(lib().orc_set_threads(int(n)))


# --------------------------------------------------------------------------
# Elementary pieces
# --------------------------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 blocks for an (n, 4) uint32 counter array and a 2-word key."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty_like(ctr)
    lib().orc_philox_many(ctr.shape[0], _p(ctr), _p(key), _p(out))
    return out


def dd_count(m: int, H: int) -> int:
    return int(lib().orc_dd_count(m, H))


def dd_H(m: int, n_req: int) -> int:
    return int(lib().orc_dd_H(m, n_req))


def dd_lattice(m: int, H: int) -> np.ndarray:
    n = dd_count(m, H)
    K = np.empty((n, m), dtype=np.int32)
    got = lib().orc_dd_lattice(m, H, _p(K))
    assert got == n
    return K


def reference_set(m: int, H1: int, H2: int = 0):
    """Reference vectors W (FP64, N x m) and the same vectors as integer
    coordinates on a common denominator (exact neighbour distances).
    One layer (H2 = 0): the Das-Dennis lattice k / H1 of Alg. 1's input, with
    integer coordinates k. Two layers (reading R28, for many objectives): the
    boundary lattice k / H1 followed by the lattice k / H2 moved halfway to the
    centroid, (k / H2 + 1 / m) / 2, each in lexicographic order; on the
    denominator 2 m H1 H2 these are 2 m H2 k and m H1 k + H1 H2."""
    K1 = dd_lattice(m, H1).astype(np.int64)
    if H2 <= 0:
        return K1.astype(np.float64) / float(H1), K1.astype(np.int32)
    K2 = dd_lattice(m, H2).astype(np.int64)
    W = np.vstack([K1.astype(np.float64) / float(H1),
                   (K2.astype(np.float64) / float(H2) + 1.0 / m) * 0.5])
    Ks = np.vstack([K1 * (2 * m * H2), K2 * (m * H1) + H1 * H2])
    return W, Ks.astype(np.int32)


def knn(K: np.ndarray, t: int) -> np.ndarray:
    K = np.ascontiguousarray(K, dtype=np.int32)
    B = np.empty((K.shape[0], t), dtype=np.int32)
    if lib().orc_knn(_p(K), K.shape[0], K.shape[1], t, _p(B)) != 0:
        raise ValueError("knn: need 1 <= t <= N (t=%d, N=%d)" % (t, K.shape[0]))
    return B


class _ProblemHolder:
    """Keeps the FP64 arrays referenced by a ctypes Problem alive."""

    def __init__(self, prob: dict):
        self.d = int(prob["d"])
        self.m = int(prob["m"])
        self.lb = np.ascontiguousarray(prob["lb"], dtype=np.float64)
        self.ub = np.ascontiguousarray(prob["ub"], dtype=np.float64)
        self.rc = np.ascontiguousarray(prob["ring_center"], dtype=np.float64).reshape(-1)
        self.rr = np.ascontiguousarray(prob["ring_radius"], dtype=np.float64).reshape(-1)
        self.s = Problem(int(prob["family"]), self.m, self.d, _p(self.lb), _p(self.ub),
                         int(self.rr.shape[0]), _p(self.rc) if self.rc.size else None,
                         _p(self.rr) if self.rr.size else None, int(prob["has_sum_lower"]),
                         float(prob["sum_lower"]), int(prob["n_eq"]), float(prob["eq_tol"]))

    def ref(self):
        return ctypes.byref(self.s)


def evaluate(prob: dict, X: np.ndarray):
    """F, CV and the largest objective-space constraint value of the rows of X
    (Eqs. (1)-(3))."""
    ph = _ProblemHolder(prob)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, ph.d)
    n = X.shape[0]
    F = np.empty((n, ph.m))
    CV = np.empty(n)
    CM = np.empty(n)
    lib().orc_eval(ph.ref(), n, _p(X), _p(F), _p(CV), _p(CM))
    return F, CV, CM


def agg(kind: int, theta: float, f, w, z) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    return float(lib().orc_agg(int(kind), float(theta), f.shape[0], _p(f), _p(w), _p(z)))


def sbx_dim(a: float, b: float, wA: int, eta_c: float):
    """(child, sibling, beta) of the SBX reading R7 before clipping."""
    c = np.zeros(1)
    s = np.zeros(1)
    beta = lib().orc_sbx_dim(float(a), float(b), int(wA) & 0xFFFFFFFF, float(eta_c), _p(c), _p(s))
    return float(c[0]), float(s[0]), float(beta)


def pm_dim(y: float, lo: float, hi: float, wB: int, tpm: int, eta_m: float) -> float:
    return float(lib().orc_pm_dim(float(y), float(lo), float(hi), int(wB) & 0xFFFFFFFF,
                                  int(tpm), float(eta_m)))


def de_dim(xi: float, a: float, b: float, F: float, lo: float, hi: float, wB: int, tpm: int,
           eta_m: float) -> float:
    """One variable of the DE operator (R26): x_i + F (a - b), clipped, then PM."""
    return float(lib().orc_de_dim(float(xi), float(a), float(b), float(F), float(lo), float(hi),
                                  int(wB) & 0xFFFFFFFF, int(tpm), float(eta_m)))


def mate(w0: int, w1: int, t: int):
    r1 = np.zeros(1, dtype=np.int32)
    r2 = np.zeros(1, dtype=np.int32)
    lib().orc_mate(int(w0) & 0xFFFFFFFF, int(w1) & 0xFFFFFFFF, int(t), _p(r1), _p(r2))
    return int(r1[0]), int(r2[0])


def front_mask(F: np.ndarray, CV: np.ndarray) -> np.ndarray:
    """Feasible non-dominated filter (Eqs. (4)-(5), R20) as a boolean mask."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    CV = np.ascontiguousarray(CV, dtype=np.float64)
    keep = np.zeros(F.shape[0], dtype=np.uint8)
    lib().orc_front(F.shape[0], F.shape[1], _p(F), _p(CV), _p(keep))
    return keep.astype(bool)


# --------------------------------------------------------------------------
# Derived method parameters (the oracle's own derivation)
# --------------------------------------------------------------------------

def derive(prob: dict, cfg: dict) -> dict:
    """N_eff, H, t1, t2, thresholds and key from the raw parameters.
    t1 = T/2 and t2 = 2T follow the parameter settings unless overridden;
    pm = 0 means 1/d; thresholds are floor(p 2^32) (R8); key = seed words (R5)."""
    m, d = int(prob["m"]), int(prob["d"])
    H1, H2 = int(cfg.get("h_outer", 0)), int(cfg.get("h_inner", 0))
    if H2 > 0 and H1 <= 0:
        raise ValueError("an inner layer needs an outer one")
    if H1 > 0:  # the layers are given (R28)
        H = H1
        N = dd_count(m, H1) + (dd_count(m, H2) if H2 > 0 else 0)
    else:
        H, H2 = dd_H(m, int(cfg["n_req"])), 0
        N = dd_count(m, H)
    T = int(cfg["T"])
    t1 = int(cfg["t1"]) if cfg["t1"] > 0 else T // 2
    t2 = int(cfg["t2"]) if cfg["t2"] > 0 else 2 * T
    if not (1 <= t1 <= N and 1 <= t2 <= N):
        raise ValueError("neighbourhood sizes must satisfy 1 <= t <= N_eff")
    pm = float(cfg["pm"]) if cfg["pm"] > 0 else 1.0 / d
    seed = int(cfg["seed"]) & 0xFFFFFFFFFFFFFFFF
    return {"m": m, "d": d, "H": H, "H2": H2, "N": N, "t": (t1, t2),
            "tpm": int(np.floor(pm * 4294967296.0)), "tpc": int(np.floor(float(cfg["pc"]) * 4294967296.0)),
            "key": (seed & 0xFFFFFFFF, seed >> 32), "agg": int(cfg["agg"]),
            "theta": float(cfg["theta"]), "eta_c": float(cfg["eta_c"]),
            "eta_m": float(cfg["eta_m"]), "op": int(cfg.get("op", 0)),
            "de_f": float(cfg.get("de_f", 0.0)) or 0.5, "op1_rule": int(cfg.get("op1_rule", 0))}


class Oracle:
    """One GMPEA instance on the CPU in FP64 (Alg. 1): weights, neighbourhoods,
    initial populations, ideal point, then generations on demand."""

    def __init__(self, prob: dict, cfg: dict, init: bool = True):
        self.prob = prob
        self.ph = _ProblemHolder(prob)
        dv = derive(prob, cfg)
        self.dv = dv
        self.m, self.d, self.N = dv["m"], dv["d"], dv["N"]
        self.W, self.K = reference_set(self.m, dv["H"], dv["H2"])
        self.B = [knn(self.K, dv["t"][0]), knn(self.K, dv["t"][1])]
        self.key = np.array(dv["key"], dtype=np.uint32)
        self._cfg = Cfg(self.m, self.d, self.N, (ctypes.c_int32 * 2)(*dv["t"]),
                        (ctypes.c_void_p * 2)(_p(self.B[0]), _p(self.B[1])), _p(self.W),
                        dv["agg"], dv["theta"], dv["eta_c"], dv["eta_m"], dv["tpm"], dv["tpc"],
                        (ctypes.c_uint32 * 2)(*dv["key"]), int(prob["n_eq"]),
                        float(prob["eq_tol"]), 0, dv["op"], dv["de_f"], dv["op1_rule"])
        self.gen = 0
        if init:
            X = [self.init_x(0), self.init_x(1)]
            self.set_state(X[0], X[1], None)

    def init_x(self, pop: int) -> np.ndarray:
        X = np.empty((self.N, self.d))
        lib().orc_init_x(self.ph.ref(), self.N, _p(self.key), int(pop), _p(X))
        return X

    def set_state(self, X1, X2, z, gen: int | None = None):
        """Load both populations' decision vectors; F, CV are re-evaluated in FP64.
        z = None recomputes the ideal point as the minimum over both populations."""
        self.X = [np.ascontiguousarray(X1, dtype=np.float64).reshape(self.N, self.d).copy(),
                  np.ascontiguousarray(X2, dtype=np.float64).reshape(self.N, self.d).copy()]
        self.F, self.CV, self.CM = [], [], []
        for p in range(2):
            F, CV, CM = evaluate(self.prob, self.X[p])
            self.F.append(F)
            self.CV.append(CV)
            self.CM.append(CM)
        if z is None:
            z = np.full(self.m, np.inf)
            for p in range(2):
                lib().orc_ideal(self.N, self.m, _p(self.F[p]), _p(z))
        self.z = np.ascontiguousarray(z, dtype=np.float64).copy()
        if gen is not None:
            self.gen = int(gen)

    def step(self, debug: bool = False):
        """Run generation gen + 1 in place. With debug, returns every intermediate."""
        k = self.gen + 1
        N, d, m = self.N, self.d, self.m
        dbg = None
        if debug:
            dbg = {"mate": np.empty((2, N, 2), dtype=np.int32), "Xo": np.empty((2, N, d)),
                   "Fo": np.empty((2, N, m)), "CVo": np.empty((2, N)),
                   "op1": np.empty((2, N), dtype=np.uint8),
                   "op1_rob": np.empty((2, N), dtype=np.uint8),
                   "win": np.empty((2, N), dtype=np.int32),
                   "win_rob": np.empty((2, N), dtype=np.uint8)}
        g = (lambda k_: _p(dbg[k_])) if debug else (lambda k_: None)
        rep = lib().orc_generation(self.ph.ref(), ctypes.byref(self._cfg), k,
                                   _p(self.X[0]), _p(self.X[1]), _p(self.F[0]), _p(self.F[1]),
                                   _p(self.CV[0]), _p(self.CV[1]), _p(self.CM[0]),
                                   _p(self.CM[1]), _p(self.z), g("mate"), g("Xo"), g("Fo"),
                                   g("CVo"), g("op1"), g("op1_rob"), g("win"), g("win_rob"))
        self.gen = k
        if debug:
            dbg["replaced"] = int(rep)
            return dbg
        return int(rep)

    def run(self, K: int):
        for _ in range(K):
            self.step()

    def select(self, X, F, CV, CM, Xo, Fo, CVo, CMo, z, f32: bool = False):
        """Selection alone (Alg. 2) on explicit parents/offspring (population-major).
        X / Xo and CM / CMo only inform the robustness flags. With f32 the
        aggregation (and so every decision) is taken in FP32 arithmetic on
        FP32-rounded inputs, the device's precision; violations are compared as
        given."""
        N, m, d = self.N, self.m, self.d
        Xp = [np.ascontiguousarray(X[p], dtype=np.float64).reshape(N, d) for p in range(2)]
        Xo = np.ascontiguousarray(Xo, dtype=np.float64).reshape(2 * N, d)
        Fp = [np.ascontiguousarray(F[p], dtype=np.float64) for p in range(2)]
        CVp = [np.ascontiguousarray(CV[p], dtype=np.float64) for p in range(2)]
        CMp = [np.ascontiguousarray(CM[p], dtype=np.float64) for p in range(2)]
        Fo = np.ascontiguousarray(Fo, dtype=np.float64).reshape(2 * N, m)
        CVo = np.ascontiguousarray(CVo, dtype=np.float64).reshape(2 * N)
        CMo = np.ascontiguousarray(CMo, dtype=np.float64).reshape(2 * N)
        z = np.ascontiguousarray(z, dtype=np.float64)
        sw = np.empty(2 * N, dtype=np.uint8)
        swr = np.empty(2 * N, dtype=np.uint8)
        win = np.empty(2 * N, dtype=np.int32)
        winr = np.empty(2 * N, dtype=np.uint8)
        self._cfg.f32 = 1 if f32 else 0
        try:
            lib().orc_select(ctypes.byref(self._cfg), _p(Xp[0]), _p(Xp[1]), _p(Fp[0]), _p(Fp[1]),
                             _p(CVp[0]), _p(CVp[1]), _p(CMp[0]), _p(CMp[1]), _p(Xo), _p(Fo),
                             _p(CVo), _p(CMo), _p(z), _p(sw), _p(swr), _p(win), _p(winr))
        finally:
            self._cfg.f32 = 0
        return (sw.reshape(2, N), swr.reshape(2, N), win.reshape(2, N), winr.reshape(2, N))

    def front(self, pop: int = 0):
        """Indices (ascending) of the feasible non-dominated rows of a population."""
        keep = front_mask(self.F[pop], self.CV[pop])
        return np.nonzero(keep)[0]
