"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Per generation the comparison is teacher-forced: the oracle runs generation k
from the GPU's own pre-state (FP32 values, exact in FP64) and both sides'
results are compared.
  - RNG words, initial decision vectors (unit box) and mating picks: bit-exact.
  - Offspring X, F, CV and the ideal point: |gpu - ref| <= 1e-5 max(1, |ref|).
  - OP1 switches and the winner of each parent slot: identical wherever the
    oracle marks the decision robust (FP64 margin above 1e-4 relative, exact
    CV zeros with slack); every other decision must still be a valid one.
  - The population after replacement: within tolerance on robust slots.
Sizes span several 256-row tiles with ragged tails (N = 100, 1035, ...), d not
a multiple of 4, both aggregations, the equality constraint, unit
neighbourhoods, and the full large workload once.
"""
import os
import sys

import numpy as np
import pytest

import cmop_inputs as ci
from oracle import core

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if gpu.size == 0:
        return 0.0
    return float(np.max(np.abs(gpu - ref) / np.maximum(1.0, np.abs(ref))))


@pytest.fixture(scope="module")
def G():
    import paper_2509_19821_amd as g
    assert g.device_count() >= 1, "GPU tests need a visible MI355X"
    return g


def _pair(prob, cfg, record=True):
    import paper_2509_19821_amd as g
    gp = g.Gmpea(prob, cfg, record=record)
    o = core.Oracle(prob, cfg, init=False)
    assert gp.n == o.N
    return gp, o


def _diag(label, S, Xo, Fo, CVo, dbg, ok):
    """On a tolerance failure, keep the worst rows (inputs and outputs) for a
    replay on the CPU (only when GMPEA_DIAG_DIR names a directory)."""
    out = os.environ.get("GMPEA_DIAG_DIR")
    if ok or not out:
        return
    os.makedirs(out, exist_ok=True)
    keep = {"gen": np.array([S["gen"]]), "z_pre": S["z"]}
    for p in range(2):
        ex = np.abs(Xo[p].astype(np.float64) - dbg["Xo"][p]).max(1)
        ef = np.abs(Fo[p].astype(np.float64) - dbg["Fo"][p]).max(1)
        rows = np.unique(np.concatenate([np.argsort(ex)[-16:], np.argsort(ef)[-16:]]))
        mate = dbg["mate"][p][rows]
        keep.update({"rows_%d" % p: rows, "mate_%d" % p: mate,
                     "pa_%d" % p: S["X"][p][mate[:, 0]], "pb_%d" % p: S["X"][p][mate[:, 1]],
                     "gpu_x_%d" % p: Xo[p][rows], "ref_x_%d" % p: dbg["Xo"][p][rows],
                     "gpu_f_%d" % p: Fo[p][rows], "ref_f_%d" % p: dbg["Fo"][p][rows],
                     "gpu_cv_%d" % p: CVo[p][rows], "ref_cv_%d" % p: dbg["CVo"][p][rows]})
    name = "".join(ch if ch.isalnum() else "_" for ch in label)
    np.savez(os.path.join(out, "diag_%s.npz" % name), **keep)


def _diag_decision(label, p, slots, S, Xo, Fo, CVo, z, g_win, g_sw, dbg):
    """On a robust-decision mismatch, print the competing keys and keep the
    generation's inputs for a replay on the CPU (GMPEA_DIAG_DIR)."""
    for j in slots[:5]:
        gi, oi = int(g_win[j]), int(dbg["win"][p][j])
        _log("%s p=%d slot %d: gpu winner %d, oracle winner %d" % (label, p, j, gi, oi))
        for who, i in (("gpu", gi), ("oracle", oi)):
            if i < 0:
                continue
            sp = p ^ int(g_sw[i])
            _log("  %s cand %d src %d: gpu F %s CV %.9g | ref F %s CV %.9g | op1 gpu %d ref %d" % (
                who, i, sp, Fo[sp][i], CVo[sp][i], dbg["Fo"][sp][i], dbg["CVo"][sp][i],
                int(g_sw[i]), int(dbg["op1"][p][i])))
        _log("  parent F %s CV %.9g" % (S["F"][p][j], S["CV"][p][j]))
    out = os.environ.get("GMPEA_DIAG_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        name = "".join(ch if ch.isalnum() else "_" for ch in label)
        np.savez(os.path.join(out, "decision_%s_p%d.npz" % (name, p)), slots=slots,
                 X0=S["X"][0], X1=S["X"][1], z_pre=S["z"], gen=np.array([S["gen"]]),
                 Xo0=Xo[0], Xo1=Xo[1], Fo0=Fo[0], Fo1=Fo[1], CVo0=CVo[0], CVo1=CVo[1], z=z,
                 g_win=g_win, g_sw=g_sw, o_win=dbg["win"][p], o_op1=dbg["op1"],
                 o_Xo=dbg["Xo"], o_Fo=dbg["Fo"], o_CVo=dbg["CVo"])


def _rev_lists(B):
    """Reverse neighbourhoods rev(j) = {i : j in B(i)}, ascending: CSR (off, idx)."""
    N, t = B.shape
    j = B.reshape(-1).astype(np.int64)
    i = np.repeat(np.arange(N, dtype=np.int64), t)
    order = np.lexsort((i, j))
    off = np.zeros(N + 1, dtype=np.int64)
    np.add.at(off, j + 1, 1)
    return np.cumsum(off), i[order]


def _unchecked_valid(p, slots, S, Fo, CVo, z, g_win, g_sw, o, agg, theta):
    """Slots the FP32 comparison leaves unchecked still hold a valid outcome
    within the FP32 bound of reading R24 (margins 2e-6 (max(|a|, |b|) +
    max(1, |F|, |z|)) on g, 1e-6 max(1, |a|, |b|) on CV), keys from the
    device's own FP32 values: a kept parent has no candidate clearly better than
    it, and a chosen winner is neither clearly worse than the parent nor than
    any other candidate of the slot (Alg. 2 OP2/OP3, Eq. (8))."""
    from oracle.dense_alg2 import agg_rows
    off, idx = _rev_lists(o.B[p])
    W = o.W
    zz = z.astype(np.float64)
    for j in slots:
        cand = idx[off[j]:off[j + 1]]
        src = p ^ g_sw[cand].astype(np.int64)
        Fc = np.stack([Fo[s_][i] for s_, i in zip(src, cand)]).astype(np.float64)
        Cc = np.array([CVo[s_][i] for s_, i in zip(src, cand)], dtype=np.float64)
        Fpj = S["F"][p][j].astype(np.float64)[None, :]
        allF = np.vstack([Fpj, Fc])
        g = agg_rows(agg, theta, allF, np.repeat(W[j:j + 1], len(allF), 0), zz)
        c = np.concatenate([[float(S["CV"][p][j])], Cc]) if p == 0 else np.zeros(len(allF))
        fs = max(1.0, float(np.max(np.abs(allF))), float(np.max(np.abs(zz))))

        def clearly_less(a, b):
            bc = 1e-6 * max(1.0, abs(c[a]), abs(c[b]))
            bg = 2e-6 * (max(abs(g[a]), abs(g[b])) + fs)
            if c[a] < c[b] - bc:
                return True
            return abs(c[a] - c[b]) <= bc and g[a] < g[b] - bg

        w = int(g_win[j])
        if w < 0:
            assert not any(clearly_less(q, 0) for q in range(1, len(allF))), ("kept parent", p, j)
        else:
            q = 1 + int(np.nonzero(cand == w)[0][0])
            assert not clearly_less(0, q), ("winner worse than parent", p, j, w)
            assert not any(clearly_less(r, q) for r in range(1, len(allF)) if r != q), (
                "winner not minimal", p, j, w)


def _tf_check(gp, o, S, dbg, label, stats):
    """Checks of one teacher-forced generation (see _teacher_forced)."""
    N = o.N
    Xo = [gp.read("XOFF", p) for p in range(2)]
    Fo = [gp.read("FOFF", p) for p in range(2)]
    CVo = [gp.read("CVOFF", p) for p in range(2)]
    _diag(label, S=S, Xo=Xo, Fo=Fo, CVo=CVo, dbg=dbg, ok=all(
        _err(a[p], dbg[k][p]) <= TOL for a, k in ((Xo, "Xo"), (Fo, "Fo"), (CVo, "CVo"))
        for p in range(2)))
    for p in range(2):
        assert np.array_equal(gp.read("MATE", p), dbg["mate"][p]), (label, "mate", p)
        assert _err(Xo[p], dbg["Xo"][p]) <= TOL, (label, "Xo", p)
        assert _err(Fo[p], dbg["Fo"][p]) <= TOL, (label, "Fo", p)
        assert _err(CVo[p], dbg["CVo"][p]) <= TOL, (label, "CVo", p)
    z = gp.read("Z")
    assert _err(z, o.z) <= TOL, (label, "z")
    allF = np.concatenate([S["z"][None, :], Fo[0], Fo[1]])
    assert np.array_equal(z, np.nanmin(allF, axis=0)), (label, "z is the FP32 minimum")
    # stage 2: selection on the GPU's inputs, decisions in FP32
    zeros = [np.zeros(N), np.zeros(N)]
    sw, swr, win, winr = o.select(S["X"], S["F"], S["CV"], zeros, np.concatenate(Xo),
                                  np.concatenate(Fo), np.concatenate(CVo), np.zeros(2 * N),
                                  z.astype(np.float64), f32=True)
    for p in range(2):
        g_sw = gp.read("OP1", p)
        g_win = gp.read("WIN", p)
        r = swr[p].astype(bool)
        assert np.array_equal(g_sw[r], sw[p][r]), (label, "op1 fp32", p)
        wr = winr[p].astype(bool)
        bad = np.nonzero(g_win[wr] != win[p][wr])[0]
        assert bad.size == 0, (label, "win fp32", p, np.nonzero(wr)[0][bad[:5]])
        # FP64 decisions marked robust agree as well
        wr64 = dbg["win_rob"][p].astype(bool)
        bad64 = np.nonzero(wr64 & (g_win != dbg["win"][p]))[0]
        if bad64.size:
            _diag_decision(label, p, bad64, S, Xo, Fo, CVo, z, g_win, g_sw, dbg)
        assert bad64.size == 0, (label, "win fp64", p, bad64[:5], g_win[bad64[:5]],
                                 dbg["win"][p][bad64[:5]])
        # every decision is a valid one, and replaced rows are exact copies
        X, F, CV = gp.read("X", p), gp.read("F", p), gp.read("CV", p)
        B = o.B[p]
        for j in range(N):
            i = g_win[j]
            if i < 0:
                assert np.array_equal(X[j], S["X"][p][j]), (label, "kept row", p, j)
                continue
            assert j in B[i], (label, "invalid winner", p, j, i)
            sp = p ^ int(g_sw[i])
            assert np.array_equal(X[j], Xo[sp][i]), (label, "copied row", p, j)
            assert np.array_equal(F[j], Fo[sp][i]) and CV[j] == CVo[sp][i], (label, "copied F/CV")
        # the slots the FP32 comparison cannot check still hold a valid outcome
        _unchecked_valid(p, np.nonzero(~wr)[0], S, Fo, CVo, z, g_win, g_sw, o,
                         o.dv["agg"], o.dv["theta"])
        # F and CV are functions of x alone: bitwise-equal rows evaluate equal
        allx = np.concatenate([X, Xo[0], Xo[1]])
        allfc = np.concatenate([np.column_stack([F, CV]), np.column_stack([Fo[0], CVo[0]]),
                                np.column_stack([Fo[1], CVo[1]])])
        _, inv = np.unique(allx.view(np.dtype((np.void, allx.dtype.itemsize * allx.shape[1]))),
                           return_inverse=True)
        first = {}
        for r_, key_ in enumerate(inv.ravel()):
            if key_ in first:
                assert np.array_equal(allfc[r_], allfc[first[key_]]), (label, "F of equal x", p)
            else:
                first[key_] = r_
        stats["amb32"] += int((~wr).sum())
        stats["amb64"] += int((~wr64).sum())
        stats["slots"] += N


def _tf_summary(label, stats):
    frac = stats["amb32"] / max(1, stats["slots"])
    rob64 = 1.0 - stats["amb64"] / max(1, stats["slots"])
    _log("%s: unchecked slots %d of %d in FP32 (%.4f%%); FP64-robust share %.2f%%"
         % (label, stats["amb32"], stats["slots"], 100 * frac, 100 * rob64))
    return frac, rob64


def _teacher_forced(gp, o, gens, label, rob64_floor=0.5):
    """Run `gens` teacher-forced generations, each checked in two stages.

    Stage 1 (reproduction + evaluation): the FP64 oracle recomputes generation
    k from the GPU's pre-state; mating picks must match bit for bit, offspring
    X, F, CV and the ideal point within TOL, and every decision the oracle
    marks robust in FP64 must match.
    Stage 2 (selection, Alg. 2): the oracle's selection runs on the GPU's own
    FP32 parents, offspring and ideal point with its aggregation evaluated in
    FP32, the kernel's precision (the paper fixes none); OP1 switches and
    winners must be identical except where the two FP32 evaluations could
    round a near-tie differently, each replaced row must be a bitwise copy of
    the winning offspring row, and every slot left unchecked must still hold
    a valid outcome within the FP32 bound. Asserts that the share of slots
    whose FP64 decision is robust (and so compared with the FP64 oracle's own
    decision) is at least rob64_floor, and returns the share of stage-2 slots
    that were not checkable."""
    stats = {"amb32": 0, "amb64": 0, "slots": 0}
    for _ in range(gens):
        S = gp.state()
        o.set_state(S["X"][0], S["X"][1], S["z"].astype(np.float64), gen=S["gen"])
        gp.step(1)
        dbg = o.step(debug=True)
        _tf_check(gp, o, S, dbg, label, stats)
    frac, rob64 = _tf_summary(label, stats)
    assert rob64 >= rob64_floor, (label, "FP64-robust share", rob64, rob64_floor)
    return frac


def test_philox_device_bit_exact(G):
    n = 1 << 20
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    want = core.philox(ctr, np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32))
    dctr, dout = G.DeviceBuffer(ctr.nbytes), G.DeviceBuffer(ctr.nbytes)
    try:
        dctr.upload(ctr)
        G.philox(dctr.ptr.value, n, seed, dout.ptr.value, 0)
        got = dout.download(np.empty_like(ctr))
    finally:
        dctr.free()
        dout.free()
    assert np.array_equal(got, want)


def test_copy_probe(G):
    n = (3 << 20) + 16 * 7  # ragged against the block size
    data = np.random.default_rng(3).integers(0, 2**32, size=n // 4, dtype=np.uint64).astype(np.uint32)
    src, dst = G.DeviceBuffer(n), G.DeviceBuffer(n)
    try:
        src.upload(data)
        G.copy(src.ptr.value, dst.ptr.value, n)
        got = dst.download(np.empty_like(data))
    finally:
        src.free()
        dst.free()
    assert np.array_equal(got, data)
    with pytest.raises(G.GmpeaError):
        G.copy(0, 0, 17)


@pytest.mark.parametrize("which", ["small", "medium"])
def test_structures_and_init(G, which):
    prob, cfg, _ = ci.WORKLOADS[which](0)
    gp, o = _pair(prob, cfg, record=False)
    try:
        assert np.array_equal(gp.read("W"), o.W.astype(np.float32))
        for p in range(2):
            assert np.array_equal(gp.read("B", p), o.B[p]), p
        o.set_state(o.init_x(0), o.init_x(1), None, gen=0)
        for p in range(2):
            # the unit box makes X = U exactly in both precisions
            assert np.array_equal(gp.read("X", p), o.X[p].astype(np.float32)), p
            assert _err(gp.read("F", p), o.F[p]) <= TOL
            assert _err(gp.read("CV", p), o.CV[p]) <= TOL
        assert _err(gp.read("Z"), o.z) <= TOL
        assert gp.read("GEN")[0] == 0
    finally:
        gp.close()


def test_neighbourhoods_full_size_sampled(G):
    prob, cfg, _ = ci.workload_large(0)
    import paper_2509_19821_amd as g
    gp = g.Gmpea(prob, cfg, record=False)
    try:
        assert gp.n == 100128 and gp.t == (16, 64)
        H = core.dd_H(3, cfg["n_req"])
        K = core.dd_lattice(3, H).astype(np.int64)
        rng = np.random.default_rng(1)
        rows = np.concatenate([[0, 1, 445, 446, gp.n - 1], rng.integers(0, gp.n, 60)])
        for p, t in ((0, 16), (1, 64)):
            B = gp.read("B", p)
            for i in rows:
                dist = ((K - K[i]) ** 2).sum(1)
                order = np.lexsort((np.arange(len(K)), dist))[:t]
                assert np.array_equal(B[i], order), (p, i)
    finally:
        gp.close()


@pytest.mark.parametrize("which,agg,seed", [("small", 0, 0), ("small", 1, 1), ("medium", 0, 0),
                                            ("medium", 1, 2)])
def test_generation_teacher_forced(G, which, agg, seed):
    prob, cfg, _ = ci.WORKLOADS[which](seed)
    cfg["agg"] = agg
    gp, o = _pair(prob, cfg)
    try:
        gp.step(4)
        frac = _teacher_forced(gp, o, 3, "%s agg=%d seed=%d" % (which, agg, seed))
        assert frac < 0.005
    finally:
        gp.close()


@pytest.mark.parametrize("which,op,seed", [("small", 0, 3), ("medium", 0, 4), ("medium", 1, 5)])
def test_generation_lane_group_variation(G, which, op, seed, monkeypatch):
    """The lane-group variation kernel (taken by rows longer than 128
    variables) at the widths where the task-dealt kernel is the default
    (GMPEA_TASKED=0 at init selects it): teacher-forced generations, SBX and
    DE, and an initial evaluation that matches its summation order (copied
    rows evaluate equal to their sources)."""
    prob, cfg, _ = ci.WORKLOADS[which](seed)
    cfg = dict(cfg, op=op)
    monkeypatch.setenv("GMPEA_TASKED", "0")
    gp, o = _pair(prob, cfg)
    monkeypatch.delenv("GMPEA_TASKED")
    try:
        gp.step(3)
        frac = _teacher_forced(gp, o, 2, "%s lane groups op=%d seed=%d" % (which, op, seed))
        assert frac < 0.005
    finally:
        gp.close()


@pytest.mark.parametrize("which,seed,rule", [("small", 4, 0), ("medium", 5, 0), ("medium", 6, 1)])
def test_generation_teacher_forced_de(G, which, seed, rule):
    """The DE operator (CR = 1, F = 0.5, then PM) in place of SBX; also with
    OP1's feasibility-first variant for population 1."""
    prob, cfg, _ = ci.WORKLOADS[which](seed)
    cfg = dict(cfg, op=1, op1_rule=rule)
    gp, o = _pair(prob, cfg)
    try:
        gp.step(3)
        frac = _teacher_forced(gp, o, 2, "%s DE seed=%d op1_rule=%d" % (which, seed, rule))
        assert frac < 0.005
    finally:
        gp.close()


def test_generation_equality_and_wide_rows(G):
    """Large-workload shape (m = 3, d = 100, T = 32, four rings, x1 + x2 = 1 with
    tolerance 1e-4) at a population the oracle steps quickly."""
    prob = ci.make_problem(ci.FAMILY_SPHERE, 3, 100, 4, False, True, 5, eq_tol=1e-4)
    for op in (0, 1):
        cfg = ci.method_config(3000, 32, 5, op=op)
        gp, o = _pair(prob, cfg)
        try:
            gp.step(3)
            frac = _teacher_forced(gp, o, 2, "d100 equality op=%d" % op)
            assert frac < 0.005
        finally:
            gp.close()


@pytest.mark.parametrize("d,op", [(200, 0), (1100, 0), (1100, 1)])
def test_generation_long_rows(G, d, op):
    """Rows longer than four chunks per lane (d > 128) take the kernel's
    long-row path; d = 1100 also crosses its 32-chunk mutation flush."""
    prob = ci.make_problem(ci.FAMILY_SPHERE, 3, d, 2, True, False, 8)
    cfg = ci.method_config(120, 10, 8, op=op)
    gp, o = _pair(prob, cfg)
    try:
        gp.step(2)
        frac = _teacher_forced(gp, o, 2, "long rows d=%d op=%d" % (d, op))
        assert frac < 0.005
    finally:
        gp.close()


def test_generation_odd_shapes(G):
    """Unit neighbourhoods, d = 7 (ragged rows), m = 2 sphere family, pc < 1."""
    prob = ci.make_problem(ci.FAMILY_SPHERE, 2, 7, 3, True, False, 3)
    cfg = ci.method_config(300, 2, 3, t1=1, t2=1, pc=0.7)
    gp, o = _pair(prob, cfg)
    try:
        gp.step(2)
        assert _teacher_forced(gp, o, 2, "unit neighbourhoods") < 0.005
    finally:
        gp.close()
    prob = ci.make_problem(ci.FAMILY_CURVE, 2, 7, 1, False, False, 4)
    cfg = ci.method_config(700, 10, 4, t2=700)  # population 2 sees everyone
    gp, o = _pair(prob, cfg)
    try:
        gp.step(2)
        assert _teacher_forced(gp, o, 1, "full neighbourhood") < 0.005
    finally:
        gp.close()


@pytest.mark.parametrize("family,m,d,n_req,t1,t2", [
    (ci.FAMILY_CURVE, 2, 2, 2, 1, 2),    # the smallest lattice (H = 1), one chunk per row
    (ci.FAMILY_SPHERE, 2, 1, 2, 2, 2),   # one variable: no distance term g
    (ci.FAMILY_SPHERE, 3, 2, 3, 1, 3),   # m = 3 with only the angles, every slot sees all
])
def test_generation_smallest_shapes(G, family, m, d, n_req, t1, t2):
    """The smallest instances the boundary accepts, unconstrained (CV = 0
    throughout, so population 1's rule reduces to population 2's): a single
    partly used tile and chunk, neighbourhoods up to the whole population."""
    prob = ci.make_problem(family, m, d, 0, False, False, 7)
    cfg = ci.method_config(n_req, 2, 7, t1=t1, t2=t2)
    gp, o = _pair(prob, cfg)
    try:
        assert gp.n == n_req
        gp.step(3)
        assert _teacher_forced(gp, o, 3, "smallest m=%d d=%d" % (m, d)) < 0.005
        assert np.all(gp.read("CV", 0) == 0) and np.all(gp.read("CV", 1) == 0)
    finally:
        gp.close()


@pytest.mark.parametrize("pm", [0.75, 0.05])
def test_generation_operator_parameters(G, pm):
    """Non-default operators and box: bounds other than [0, 1] per variable
    (the clip and the mutation's span), eta_c = 2, eta_m = 5, pc = 0.6,
    theta = 2, and a mutation rate above 1/2, whose threshold floor(pm 2^32)
    needs the 64-bit numerators of the mutation step, beside one below it."""
    d = 20
    lb = np.linspace(-1.0, -0.2, d)
    ub = np.linspace(0.5, 3.0, d)
    prob = ci.make_problem(ci.FAMILY_SPHERE, 3, d, 2, True, False, 11, lb=lb, ub=ub)
    cfg = ci.method_config(300, 10, 11, theta=2.0, eta_c=2.0, eta_m=5.0, pc=0.6, pm=pm)
    gp, o = _pair(prob, cfg)
    try:
        gp.step(2)
        assert _teacher_forced(gp, o, 2, "operators pm=%g" % pm) < 0.005
        X = gp.read("X", 0)
        assert np.all(X >= lb.astype(np.float32)) and np.all(X <= ub.astype(np.float32))
    finally:
        gp.close()


def test_generation_full_size_large(G):
    """One teacher-forced generation of the large workload at full size
    (N = 100,128 per population, d = 100, t1 = 16, t2 = 64) in the launch
    configuration the benchmark times."""
    prob, cfg, _ = ci.workload_large(0)
    _log("full size: building oracle neighbourhoods")
    gp, o = _pair(prob, cfg)
    try:
        gp.step(2)
        frac = _teacher_forced(gp, o, 1, "large full size")
        assert frac < 0.005
    finally:
        gp.close()


def test_generation_large_population_short_rows(G):
    """A plain population of 65,536 or more with rows of at most 56 variables:
    the task-dealt variation builds 64 offspring per wave (the most its LDS
    holds), which changes the dealing and not the results; one teacher-forced
    generation at N = 65,703, d = 40, DE for population rows read in the task."""
    prob = ci.make_problem(ci.FAMILY_SPHERE, 3, 40, 3, True, False, 21)
    cfg = ci.method_config(65536, 20, 21, op=1)
    gp, o = _pair(prob, cfg)
    try:
        assert gp.n >= 65536
        gp.step(2)
        frac = _teacher_forced(gp, o, 1, "N=%d d=40 DE" % gp.n)
        assert frac < 0.005
    finally:
        gp.close()


def test_front_matches_bruteforce(G):
    prob, cfg, K = ci.workload_medium(1)
    import paper_2509_19821_amd as g
    gp = g.Gmpea(prob, cfg)
    try:
        gp.step(60)
        fr = gp.front()
        F = gp.read("F", 0).astype(np.float64)
        CV = gp.read("CV", 0).astype(np.float64)
        keep = core.front_mask(F, CV)
        assert np.array_equal(fr["idx"], np.nonzero(keep)[0])
        assert np.array_equal(fr["f"], F[keep].astype(np.float32))
        assert np.array_equal(fr["x"], gp.read("X", 0)[keep])
        assert np.all(fr["cv"] == 0)
        allp = gp.front(g.FRONT_POP2)
        assert np.array_equal(allp["x"], gp.read("X", 1))
    finally:
        gp.close()


@pytest.mark.parametrize("m,n_req,d", [(3, 5100, 12), (2, 20000, 8)])
def test_front_chunked_grid(G, m, n_req, d):
    """The front kernel's (row tile, column chunk) grid at sizes with many
    chunks and a ragged last tile, against the oracle's filter on the device's
    values."""
    import paper_2509_19821_amd as g
    fam = ci.FAMILY_SPHERE if m == 3 else ci.FAMILY_CURVE
    prob = ci.make_problem(fam, m, d, 3, m == 3, False, 31)
    gp = g.Gmpea(prob, ci.method_config(n_req, 10, 31))
    try:
        gp.step(30)
        fr = gp.front(with_x=False)
        F = gp.read("F", 0).astype(np.float64)
        CV = gp.read("CV", 0).astype(np.float64)
        keep = core.front_mask(F, CV)
        assert gp.n % 256 != 0
        assert np.array_equal(fr["idx"], np.nonzero(keep)[0])
        assert fr["x"].shape == (0, d)
    finally:
        gp.close()


def test_graph_replay_equals_eager(G):
    import paper_2509_19821_amd as g
    prob, cfg, _ = ci.workload_medium(3)
    out = []
    for chunk in ("0", "16", None):  # eager, 16-generation replays, the default 64
        if chunk is None:
            os.environ.pop("GMPEA_GRAPH_CHUNK", None)
        else:
            os.environ["GMPEA_GRAPH_CHUNK"] = chunk
        gp = g.Gmpea(prob, cfg)
        try:
            gp.step(0)   # captures the graph only
            gp.step(70)
            gp.step(7)
            out.append(gp.state())
        finally:
            gp.close()
    os.environ.pop("GMPEA_GRAPH_CHUNK", None)
    a = out[0]
    for b in out[1:]:
        assert a["gen"] == b["gen"] == 77
        for p in range(2):
            assert np.array_equal(a["X"][p], b["X"][p])
            assert np.array_equal(a["F"][p], b["F"][p])
        assert np.array_equal(a["z"], b["z"])


def test_checkpoint_resume_bit_exact(G):
    import paper_2509_19821_amd as g
    prob, cfg, _ = ci.workload_small(5)
    gp = g.Gmpea(prob, cfg)
    try:
        gp.step(10)
        snap = gp.state()
        gp.step(15)
        ref = gp.state()
    finally:
        gp.close()
    gp = g.Gmpea(prob, cfg)
    try:
        gp.load_state(snap)
        gp.step(15)
        got = gp.state()
    finally:
        gp.close()
    assert got["gen"] == ref["gen"] == 25
    for p in range(2):
        assert np.array_equal(got["X"][p], ref["X"][p])
        assert np.array_equal(got["CV"][p], ref["CV"][p])


def test_run_time_limit(G):
    import paper_2509_19821_amd as g
    prob, cfg, _ = ci.workload_medium(0)
    gp = g.Gmpea(prob, cfg)
    try:
        assert gp.run(50) == 50
        assert gp.read("GEN")[0] == 50
        assert gp.run(10**6, time_limit_s=1e-9) == 0   # deadline already passed
        assert gp.read("GEN")[0] == 50
        n = gp.run(10**6, time_limit_s=0.05)
        assert 1 <= n < 10**6
        assert gp.read("GEN")[0] == 50 + n
    finally:
        gp.close()


def test_record_disabled_rejects_decision_reads(G):
    import paper_2509_19821_amd as g
    prob, cfg, _ = ci.workload_small(0)
    gp = g.Gmpea(prob, cfg, record=False)
    try:
        with pytest.raises(g.GmpeaError):
            gp.read("WIN", 0)
        cnt = gp.front()
        assert cnt["x"].shape[1] == 10
    finally:
        gp.close()


def test_front_capacity_reports_required_count(G):
    """An undersized output reports GMPEA_ECAPACITY and the required row count."""
    import ctypes
    import paper_2509_19821_amd as g
    from paper_2509_19821_amd import gmpea as GM
    prob, cfg, _ = ci.workload_small(2)
    gp = g.Gmpea(prob, cfg)
    try:
        gp.step(20)
        n = gp.front()["x"].shape[0]
        assert n >= 2
        cap = n - 1
        x = np.empty((cap, gp.d), dtype=np.float32)
        f = np.empty((cap, gp.m), dtype=np.float32)
        cv = np.empty(cap, dtype=np.float32)
        idx = np.empty(cap, dtype=np.int32)
        cnt = ctypes.c_int32(-7)
        st = GM.lib().gmpea_front(gp.handle, g.FRONT_FEASIBLE_ND, cap, x.ctypes.data,
                                  f.ctypes.data, cv.ctypes.data, idx.ctypes.data, ctypes.byref(cnt))
        assert st == -4 and cnt.value == n
        assert GM.lib().gmpea_last_error()
    finally:
        gp.close()


def test_generation_nan_constraint_constant(G):
    """A NaN ring radius makes that constraint's value NaN; the clamp max(0, .)
    of Eq. (2) reads it as satisfied on both sides (comparisons with NaN are
    false), and the generation matches the oracle as usual."""
    prob, cfg, _ = ci.workload_small(6)
    prob["ring_radius"] = np.array(prob["ring_radius"], dtype=np.float64)
    prob["ring_radius"][0] = np.nan
    gp, o = _pair(prob, cfg)
    try:
        gp.step(2)
        frac = _teacher_forced(gp, o, 2, "nan ring radius")
        assert frac < 0.005
        assert np.all(np.isfinite(gp.read("CV", 0)))
    finally:
        gp.close()


def test_pool_teacher_forced(G):
    """Instances advanced by batched pool generations (one launch per phase for
    all of them) checked against the FP64 oracle exactly as plain instances
    are: the oracle runs each instance's generation from the pool's pre-state.
    The mix covers both record widths' batched kernels (m = 2, 3 and a
    five-objective layered set), both aggregations, DE, the equality, ragged
    rows and tiles."""
    import paper_2509_19821_amd as g
    mix = [("pool small", ci.workload_small(8)[:2]),
           ("pool sphere DE", (ci.make_problem(ci.FAMILY_SPHERE, 3, 30, 3, True, False, 12),
                               ci.method_config(400, 10, 12, op=1))),
           ("pool curve tche d23", (ci.make_problem(ci.FAMILY_CURVE, 2, 23, 4, False, False, 13),
                                    ci.method_config(700, 10, 13, agg=1))),
           ("pool d100 equality", (ci.make_problem(ci.FAMILY_SPHERE, 3, 100, 4, False, True, 14,
                                                   eq_tol=1e-4), ci.method_config(1500, 32, 14))),
           ("pool m5 layers", (ci.make_problem(ci.FAMILY_SPHERE, 5, 30, 3, True, False, 15),
                               ci.method_config(2, 12, 15, h_outer=8, h_inner=5)))]
    pool = g.Pool(8 << 30)
    try:
        pairs = []
        for label, (prob, cfg) in mix:
            s = pool.admit(prob, cfg, record=True)
            o = core.Oracle(prob, cfg, init=False)
            pairs.append((label, pool.instance(s), o, {"amb32": 0, "amb64": 0, "slots": 0}))
            assert pairs[-1][1].n == o.N
        pool.step(3)
        pool.sync()
        for _ in range(2):
            pre = []
            for label, gp, o, _ in pairs:
                S = gp.state()
                o.set_state(S["X"][0], S["X"][1], S["z"].astype(np.float64), gen=S["gen"])
                pre.append(S)
            pool.step(1)
            pool.sync()
            for (label, gp, o, stats), S in zip(pairs, pre):
                dbg = o.step(debug=True)
                _tf_check(gp, o, S, dbg, label, stats)
        for label, gp, o, stats in pairs:
            frac, rob64 = _tf_summary(label, stats)
            assert frac < 0.005, (label, frac)
            assert rob64 >= 0.5, (label, rob64)
    finally:
        pool.close()
