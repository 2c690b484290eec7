"""Throughput of full GMPEA generations on one MI355X.

A step is one generation of the whole hot path over both populations of the
large synthetic workload: m = 3, d = 100, N = 100,128 reference vectors per
population (Das-Dennis, H = 446), T = 32 (t1 = 16, t2 = 64), four ring
constraints plus the equality x1 + x2 = 1 (tolerance 1e-4), FP32 on device.
Inputs are resident in HBM before timing starts; the timed region is K
generations enqueued back to back (hipGraph replay of generation chunks)
between two device synchronisations.

Prints one JSON line with the value (offspring evaluated + selected per
second = 2 N K / t), the roofline of the dominant kernel (per-kernel HIP-event
timing on the stream the kernels run on, algorithmic bytes from the bytes
model), and the CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "offspring evaluated+selected/sec (FP32) and % HBM roofline; batched vs plain speedup at equal IGD"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = [os.path.join(ROOT, "paper_2509_19821_amd", "csrc", f)
              for f in ("gmpea_device.hpp", "gmpea_kernels.hip", "gmpea_kernels_wide.hip",
                        "gmpea_internal.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_large.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_large.json")
# Vector-ALU issue ceiling: 256 CUs x 4 SIMDs, each SIMD issuing one wave64
# VALU instruction every 4 cycles (16 lanes per cycle) at 2.4 GHz, i.e.
# 39.3e12 lane-operations per second for single-issue 32-bit operations. (The
# chip's 157.3 TFLOP/s FP32 figure counts an FMA as two operations and packed
# dual FP32 issue, which this build keeps off.)
SIMDS, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4
ALU_PEAK_LANE_OPS = SIMDS * 16 * CLOCK_HZ


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bytes_model(n, m, d, t, rho):
    """Algorithmic bytes per launch of each kernel (FP32 / int32 words; each item
    counted once at the level the method must move it).
      vary:   parent row (d, each row read once per generation), offspring row
              write (d), offspring F/CV write (m + 1), two mating picks
      op1:    both offspring F/CV read (2 (m + 1)), weight (m), both new
              offspring F/CV written (2 (m + 1)) -- per subproblem
      select: parent F/CV (m + 1), weight (m), reverse list (t_p entries),
              candidate F/CV once per offspring (m + 1); a replaced slot
              (rho_p) writes the winner's F/CV (m + 1) and its new location
              (1), a kept slot reads its location (1). The kernel's copies of
              kept rows out of the next generation's offspring region are not
              the method's bytes: they show in the measured traffic only."""
    vary = sum(n * 4 * (2 * d + (m + 1) + 2) for _ in range(2))
    op1 = n * 4 * (4 * (m + 1) + m)
    select = sum(n * 4 * ((m + 1) + m + t[p] + (m + 1)) + rho[p] * n * 4 * (m + 2) + (1 - rho[p]) * n * 4
                 for p in range(2))
    return {"vary": vary, "op1": op1, "select": select}


def _code_only(text):
    """C++ source without comments and with runs of whitespace collapsed, so
    that a change to comments alone keeps the hash (the sources hold no string
    literal with comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash():
    """sha256[:16] over the code of the kernel sources (device code, both
    instantiation units, the shared declarations, in that order), comments
    left out."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
    only if they were taken on the kernel source as it is now."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256_16") != kernel_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def measured_valu(kernel):
    """SQ_INSTS_VALU (wave-level VALU instructions) per launch from a committed
    rocprofv3 --pmc run, only if taken on the kernel source as it is now."""
    try:
        with open(VALU_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256_16") != kernel_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("valu_insts_per_launch")


def cpu_baseline(target_s=12.0, single_s=10.0):
    """The oracle as it stands, on the large workload's shape at a bounded
    population (N = 50,086 per population), timed over whole generations: once
    with OpenMP over subproblems on every host core, once on one thread."""
    import cmop_inputs as ci
    from oracle import core
    prob, cfg, _ = ci.workload_large(0)
    cfg = dict(cfg, n_req=50000)

    def timed(threads, budget_s, max_gens):
        cores = core.set_threads(threads)
        o = core.Oracle(prob, cfg)
        o.step()  # first generation off the clock
        gens, t0 = 0, time.perf_counter()
        while True:
            o.step()
            gens += 1
            el = time.perf_counter() - t0
            if el >= budget_s or gens >= max_gens:
                break
        return 2.0 * o.N * gens / el, int(cores), o.N, gens

    all_cores = core.set_threads(0)
    v, cores, n, gens = timed(all_cores, target_s, 200)
    v1, _, _, gens1 = timed(1, single_s, 50)
    core.set_threads(all_cores)
    shape = "large-workload shape (m=3, d=100, T=32, 4 rings + equality) at N=%d per population" % n
    return {"value": v, "unit": "offspring/s", "cores": cores, "kind": "oracle",
            "sample": "%s, %d generations after one warm-up, FP64, OpenMP over subproblems on %s"
                      % (shape, gens, _cpu_model()),
            "single_thread": {"value": v1, "cores": 1,
                              "sample": "%s, %d generations after one warm-up, FP64, one thread"
                                        % (shape, gens1)}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "an unidentified CPU"


def copy_probe(g, nbytes=512 << 20, reps=5):
    """Attainable copy bandwidth (read + write bytes per second, fastest of
    `reps`, HIP events) of four copy forms: the library's strided copy kernel
    (also the counter calibration launch), a one-pass copy with four 16-byte
    words per thread, the same with non-temporal accesses, and the runtime's
    hipMemcpyAsync."""
    src, dst = g.DeviceBuffer(nbytes), g.DeviceBuffer(nbytes)
    out = {}
    try:
        g.copy(src.ptr.value, dst.ptr.value, nbytes)
        for name, mode in (("strided_kernel", g.COPY_STRIDED), ("wide_kernel", g.COPY_WIDE),
                           ("wide_nontemporal", g.COPY_WIDE_NT), ("hipMemcpyAsync", g.COPY_RUNTIME)):
            ms = g.copy_probe(src.ptr.value, dst.ptr.value, nbytes, mode, reps)
            out[name] = round(2.0 * nbytes / (ms * 1e-3) / 1e9, 1)
    finally:
        src.free()
        dst.free()
    return out


def batched_vs_plain(g, ci, count=256, gens=300):
    """Instance throughput of one pool (batched generations) against the same
    instances solved one after another with plain launches, plus a bitwise
    comparison of every instance's final population 1 (equal fronts, so equal
    IGD, by construction)."""
    insts = ci.batch_instances(count=count, master_seed=0)
    plain_s, plain_f = 0.0, []
    t_init = time.perf_counter()
    for p, c in insts:
        gp = g.Gmpea(p, c)
        gp.sync()
        t0 = time.perf_counter()
        gp.step(gens)
        gp.sync()
        plain_s += time.perf_counter() - t0
        plain_f.append((gp.read("F", 0), gp.read("CV", 0)))
        gp.close()
    log("bench: plain %d instances x %d generations: %.3f s solving (%.1f s total)"
        % (count, gens, plain_s, time.perf_counter() - t_init))
    pool = g.Pool(200 << 30)
    try:
        slots = [pool.admit(p, c) for p, c in insts]
        pool.sync()
        t0 = time.perf_counter()
        pool.tune(gens)
        pool.sync()
        batched_s = time.perf_counter() - t0
        q = pool.query()
        same = all(np.array_equal(pool.instance(s).read("F", 0), f) and
                   np.array_equal(pool.instance(s).read("CV", 0), cv)
                   for s, (f, cv) in zip(slots, plain_f))
        offspring = sum(2 * pool.instance(s).n for s in slots) * gens
    finally:
        pool.close()
    log("bench: batched: %.3f s (schedule %d, chunk %d), identical=%s"
        % (batched_s, q["schedule"], q["chunk"], same))
    return {"instances": count, "generations": gens,
            "plain_instances_per_s": round(count / plain_s, 2),
            "batched_instances_per_s": round(count / batched_s, 2),
            "speedup": round(plain_s / batched_s, 2),
            "batched_offspring_per_s": round(offspring / batched_s, 1),
            "final_fronts_identical": bool(same), "device_bytes": int(q["used_bytes"]),
            "schedule": "xcd-grouped op1/select" if q["schedule"] == 0 else "linear",
            "graph_chunk": q["chunk"]}


def pool_only(g, ci, count=256, gens=300):
    """The batched leg's pool alone (no plain solves beside it): 256 uneven
    instances, 300 batched generations after tuning; for profiling the
    batched kernels. Prints one JSON object."""
    insts = ci.batch_instances(count=count, master_seed=0)
    pool = g.Pool(200 << 30)
    try:
        for p, c in insts:
            pool.admit(p, c)
        pool.sync()
        t0 = time.perf_counter()
        pool.tune(gens)
        pool.sync()
        el = time.perf_counter() - t0
        q = pool.query()
    finally:
        pool.close()
    print(json.dumps({"instances": count, "generations": gens, "batched_s": round(el, 4),
                      "ms_per_generation": round(1e3 * el / gens, 4), "schedule": q["schedule"],
                      "graph_chunk": q["chunk"]}), flush=True)


def serving(g, ci, window_s=5.0, rate=200.0, quality_every=16):
    """Poisson arrivals at `rate` per second over `window_s`, deadlines
    log-uniform in [10 ms, 1 s], problems from the batched-instance
    distribution; continuous batching over one pool. Every `quality_every`-th
    request carries a reference front (built before the window opens), so its
    IGD and HV at the deadline are measured on the device before delivery."""
    from paper_2509_19821_amd import fronts
    from paper_2509_19821_amd.serve import Request, Server, summarize
    arr = ci.serve_arrivals(rate=rate, window_s=window_s, master_seed=0)
    inst = ci.batch_instances(count=len(arr), master_seed=1)
    reqs = []
    for k, ((t, dl), (p, c)) in enumerate(zip(arr, inst)):
        ref = hvp = None
        if quality_every and k % quality_every == 0:
            ref = fronts.reference_front(p, n=800)
            hvp = 1.1 * ref.max(0)  # the HV reference point 1.1 x the front's maximum
        reqs.append(Request(k, p, c, dl, t, reference=ref, hv_point=hvp))
    srv = Server(200 << 30, keep_fronts=False)
    try:
        t0 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t0
        out = summarize(res, wall, srv.offspring, srv.host_s)
        out["host_s"] = {k: round(v, 3) for k, v in out["host_s"].items()}
        out.update({"window_s": window_s, "rate_per_s": rate, "batched_generations": srv.steps})
    finally:
        srv.close()
    return {k: (round(v, 5) if isinstance(v, float) else v) for k, v in out.items()}


def sweep(g, ci, sizes=(100, 1000, 5000, 10000, 100000, 1000000), gens=50, cpu_gens=3):
    """Generation time against population size on the large workload's shape
    (m = 3, d = 100, T = 32, four rings and the equality): the GPU (graph
    replay, inputs resident) and, up to N = 1e5, the CPU oracle on this host's
    cores. One JSON object per size on stdout."""
    from oracle import core
    cores = core.set_threads(0)
    for n_req in sizes:
        prob, cfg, _ = ci.workload_large(0)
        cfg = dict(cfg, n_req=n_req)
        gp = g.Gmpea(prob, cfg)
        gp.step(5)
        gp.step(0)
        gp.sync()
        t0 = time.perf_counter()
        gp.step(gens)
        gp.sync()
        gpu_us = (time.perf_counter() - t0) / gens * 1e6
        n = gp.n
        gp.close()
        row = {"n_requested": n_req, "n": n, "gpu_us_per_gen": round(gpu_us, 2),
               "gpu_offspring_per_s": round(2 * n / (gpu_us * 1e-6), 1)}
        if n_req <= 100000:
            o = core.Oracle(prob, cfg)
            o.step()
            t0 = time.perf_counter()
            for _ in range(cpu_gens):
                o.step()
            cpu_us = (time.perf_counter() - t0) / cpu_gens * 1e6
            row.update({"cpu_us_per_gen": round(cpu_us, 1), "cpu_cores": int(cores),
                        "gpu_over_cpu": round(cpu_us / gpu_us, 1)})
        print(json.dumps(row), flush=True)


def shapes(g, ci, seconds=4.0):
    """GPU against the CPU oracle at the three plain workload shapes: small
    (m = 2, d = 10, N = 100), medium (m = 3, d = 30, N = 1,035) and large
    (m = 3, d = 100, N = 100,128). GPU: generations in graph replay, inputs
    resident. CPU: the oracle on one thread and with OpenMP on every host core,
    whole generations for about `seconds` each (at least two). One JSON object
    per shape on stdout."""
    from oracle import core
    all_cores = core.set_threads(0)
    for name in ("small", "medium", "large"):
        prob, cfg, _ = ci.WORKLOADS[name](0)
        gp = g.Gmpea(prob, cfg)
        gens = 1000 if name != "large" else 200
        gp.step(5)
        gp.step(0)
        gp.sync()
        t0 = time.perf_counter()
        gp.step(gens)
        gp.sync()
        gpu_us = (time.perf_counter() - t0) / gens * 1e6
        n = gp.n
        gp.close()
        row = {"workload": name, "m": prob["m"], "d": prob["d"], "n": n,
               "gpu_us_per_gen": round(gpu_us, 2),
               "gpu_offspring_per_s": round(2 * n / (gpu_us * 1e-6), 1)}
        for label, threads in (("cpu_1thread", 1), ("cpu_all_cores", all_cores)):
            core.set_threads(threads)
            o = core.Oracle(prob, cfg)
            o.step()
            k, t0 = 0, time.perf_counter()
            while k < 2 or time.perf_counter() - t0 < seconds:
                o.step()
                k += 1
            us = (time.perf_counter() - t0) / k * 1e6
            row[label] = {"us_per_gen": round(us, 1), "threads": int(threads), "generations": k,
                          "gpu_speedup": round(us / gpu_us, 1)}
        core.set_threads(all_cores)
        row["cpu_model"] = _cpu_model()
        print(json.dumps(row), flush=True)


def many(g, ci, gens=50, cpu_gens=3):
    """Many objectives (m = 5 and 8) on the many-objective throughput shape
    (d = 100, two layers of about 1e5 reference vectors, T = 32): GPU time per
    generation (graph replay, inputs resident), per-kernel times and k_vary's
    algorithmic bandwidth; then the GPU and the CPU oracle on a layered set of
    about 2,000 vectors (the oracle's brute-force tables make 1e5 too slow
    for a bounded run). One JSON object per row on stdout."""
    from oracle import core
    cores = core.set_threads(0)
    for m in (5, 8):
        prob, cfg, _ = ci.workload_many_large(0, m)
        t0 = time.perf_counter()
        gp = g.Gmpea(prob, cfg)
        init_s = time.perf_counter() - t0
        gp.step(5)
        gp.step(0)
        gp.sync()
        t0 = time.perf_counter()
        gp.step(gens)
        gp.sync()
        us = (time.perf_counter() - t0) / gens * 1e6
        prof = gp.profile(10)
        n, d, rq = gp.n, prob["d"], (m + 4) // 4
        vary_bytes = 2 * n * (4 * 2 * d + 16 * rq + 8)
        print(json.dumps({"m": m, "n": n, "d": d, "layers": [cfg["h_outer"], cfg["h_inner"]],
                          "init_s": round(init_s, 2), "gpu_us_per_gen": round(us, 2),
                          "gpu_offspring_per_s": round(2 * n / (us * 1e-6), 1),
                          "per_kernel_ms": {k: round(v, 5) for k, v in prof.items()},
                          "vary_gbs": round(vary_bytes / (prof["vary"] * 1e-3) / 1e9, 1)}), flush=True)
        gp.close()
        small = dict(cfg, h_outer={5: 10, 8: 6}[m], h_inner={5: 6, 8: 4}[m])
        gp = g.Gmpea(prob, small)
        gp.step(5)
        gp.step(0)
        gp.sync()
        t0 = time.perf_counter()
        gp.step(gens)
        gp.sync()
        us = (time.perf_counter() - t0) / gens * 1e6
        n = gp.n
        gp.close()
        o = core.Oracle(prob, small)
        o.step()
        t0 = time.perf_counter()
        for _ in range(cpu_gens):
            o.step()
        cpu_us = (time.perf_counter() - t0) / cpu_gens * 1e6
        print(json.dumps({"m": m, "n": n, "d": d, "layers": [small["h_outer"], small["h_inner"]],
                          "gpu_us_per_gen": round(us, 2), "cpu_us_per_gen": round(cpu_us, 1),
                          "cpu_cores": int(cores), "gpu_over_cpu": round(cpu_us / us, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--profile-gens", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-window", type=float, default=60.0)
    ap.add_argument("--n-req", type=int, default=0,
                    help="reference vectors requested per population for the main line "
                         "(default: the large workload's 100,000)")
    ap.add_argument("--sweep", action="store_true",
                    help="print generation time against population size (GPU and CPU oracle) "
                         "instead of the benchmark line")
    ap.add_argument("--shapes", action="store_true",
                    help="print GPU against CPU oracle (one thread and all cores) at the small, "
                         "medium and large workload shapes instead of the benchmark line")
    ap.add_argument("--pool-only", action="store_true",
                    help="run only the batched leg's pool (256 instances, 300 generations) and "
                         "print its time instead of the benchmark line")
    ap.add_argument("--many", action="store_true",
                    help="print many-objective (m = 5, 8) generation times (GPU and CPU oracle) "
                         "instead of the benchmark line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: each instance runs on a single "
              "MI355X (instances shard across GPUs without communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import cmop_inputs as ci
    import paper_2509_19821_amd as g

    if args.sweep:
        sweep(g, ci)
        return
    if args.many:
        many(g, ci)
        return
    if args.shapes:
        shapes(g, ci)
        return
    if args.pool_only:
        pool_only(g, ci)
        return

    prob, cfg, K_total = ci.workload_large(0)
    if args.n_req > 0:
        cfg = dict(cfg, n_req=args.n_req)
    log("bench: init large workload")
    t0 = time.perf_counter()
    gp = g.Gmpea(prob, cfg)
    gp.sync()
    log("bench: init %.2f s, N=%d t=%s" % (time.perf_counter() - t0, gp.n, gp.t))
    n, m, d = gp.n, gp.m, gp.d

    gp.step(args.warmup)
    gp.step(0)  # capture the replay graph outside the timed region (no generations)
    gp.sync()
    log("bench: warmup done")
    r0 = gp.info()["replaced"]
    gp.sync()  # one process, one GPU: the barrier is this device synchronisation
    t0 = time.perf_counter()
    gp.step(args.steps)
    gp.sync()
    el = time.perf_counter() - t0
    r1 = gp.info()["replaced"]
    value = 2.0 * n * args.steps / el
    rho = [(r1[p] - r0[p]) / (n * args.steps) for p in range(2)]
    log("bench: %d generations in %.3f s (%.1f us/gen), rho=%s" % (args.steps, el,
                                                                   1e6 * el / args.steps, rho))

    ms = gp.profile(args.profile_gens)
    b2b = ms.pop("vary_back_to_back")
    model = bytes_model(n, m, d, gp.t, rho)
    dom = max(ms, key=ms.get)
    # the variation phase's kernel: k_tvary (task-dealt) or k_vary (lane groups)
    kname = ("tvary" if gp.info()["task_dealt"] else "vary") if dom == "vary" else dom
    # the dominant kernel's launch duration: the variation kernel launched back
    # to back between two events (it rewrites the same offspring when
    # repeated), the others one launch at a time between events
    t_dom = b2b if dom == "vary" else ms[dom]
    achieved = model[dom] / (t_dom * 1e-3) / 1e9
    traffic = measured_traffic(kname)
    log("bench: per-kernel ms %s; model bytes %s" % (ms, model))
    gen_bytes = sum(model.values())
    copies = copy_probe(g)
    log("bench: copy bandwidth %s GB/s" % copies)
    hbm = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    valu = measured_valu(kname)
    alu = None
    if valu is not None:
        # lane-operations per second: wave64 instructions x 64 lanes over the launch
        lane_ops = valu * 64 / (t_dom * 1e-3)
        alu = {"achieved": round(lane_ops / 1e12, 2), "peak": round(ALU_PEAK_LANE_OPS / 1e12, 2),
               "unit": "T VALU lane-ops/s", "frac": round(lane_ops / ALU_PEAK_LANE_OPS, 4),
               "valu_insts_per_launch": int(valu)}
    bind = alu if (alu is not None and alu["frac"] > hbm["frac"]) else hbm
    roof = {"bound": "alu" if bind is alu else "hbm", "kernel": "k_" + kname,
            "achieved": bind["achieved"], "peak": bind["peak"], "unit": bind["unit"],
            "frac": bind["frac"], "traffic": traffic,
            "algorithmic_bytes_per_launch": int(model[dom]), "avg_launch_ms": round(t_dom, 5),
            "launch_timing": ("%d launches back to back between two HIP events on the instance's stream"
                              % args.profile_gens if dom == "vary" else
                              "one launch between two HIP events on the instance's stream"),
            "hbm": hbm, "alu": alu,
            "per_kernel_ms": {k: round(v, 5) for k, v in ms.items()},
            "generation_gbs": round(gen_bytes / (sum(ms.values()) * 1e-3) / 1e9, 1),
            "copy_probe_gbs": copies,
            "rho": [round(r, 4) for r in rho]}
    gp.close()

    # the whole solve (200 generations from a fresh instance, initialisation
    # excluded): replacements thin out as the populations converge, and the
    # generation's cost follows
    gs = g.Gmpea(prob, cfg)
    gs.step(0)
    gs.sync()
    t0 = time.perf_counter()
    gs.step(K_total)
    gs.sync()
    el_s = time.perf_counter() - t0
    rep = gs.info()["replaced"]
    gs.close()
    solve = {"generations": K_total, "ms_per_generation": round(1e3 * el_s / K_total, 5),
             "offspring_per_s": round(2.0 * n * K_total / el_s, 1),
             "rho_mean": [round(rep[p] / (n * K_total), 4) for p in range(2)]}
    log("bench: full solve %d generations %.1f us/gen, rho %s" % (K_total, 1e6 * el_s / K_total,
                                                                 solve["rho_mean"]))

    out = {"metric": METRIC, "value": round(value, 1), "unit": "offspring/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * el / args.steps, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "large: m=3, d=100, N=%d per population (2 populations), "
                                  "T=32 (t1=16, t2=64), 4 rings + equality x1+x2=1 (tol 1e-4), "
                                  "%d generations in the full solve" % (n, K_total),
                      "global_batch": 2 * n, "parallelism": "single GPU"},
           "roofline": roof, "full_solve": solve}
    if not args.no_batched:
        log("bench: batched instances")
        out["batched"] = batched_vs_plain(g, ci)
    if not args.no_serving:
        log("bench: serving")
        out["serving"] = serving(g, ci, window_s=args.serve_window)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
