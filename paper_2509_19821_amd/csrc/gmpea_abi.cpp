// Host runtime of the GMPEA library: handle, device memory through the caller's
// allocator hook, stream, hipGraph replay of generation chunks, and the C ABI
// declared in include/gmpea.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <hip/hip_version.h>

#include "gmpea.h"
#include "gmpea_internal.hpp"

using namespace gmpea;

namespace {

// A roctx range over one call of the ABI, shown by rocprofv3 --marker-trace
// (a no-op when no tool listens).
struct Trace {
  explicit Trace(const char *name) { roctxRangePushA(name); }
  ~Trace() { roctxRangePop(); }
  Trace(const Trace &) = delete;
  Trace &operator=(const Trace &) = delete;
};

thread_local std::string g_err;

gmpea_status fail(gmpea_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

gmpea_status hip_fail(hipError_t e, const char *what) {
  return fail(GMPEA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct gmpea_s {
  gmpea_allocator al{};
  bool hook = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevState st{};
  int32_t H = 0, H2 = 0;  // reference-set divisions (outer, inner; H2 = 0: one layer)
  bool record = false;
  std::vector<std::pair<void *, size_t>> allocs;
  size_t bytes = 0;
  int device = 0;  // the device current at gmpea_init (the handle's memory and stream)
  // gmpea_front / gmpea_quality scratch, part of the allocation made at
  // gmpea_init so that delivering a front never allocates: flags and row list
  // (n each), gathered F/CV records (n), gathered decision vectors (kFrontRows
  // rows at a time), reference points (kQualityRefs at a time) and their IGD
  // partial sums, the HV box and hit counter
  uint8_t *f_keep = nullptr;
  int32_t *f_idx = nullptr;
  float *f_x = nullptr;
  float4 *f_fc = nullptr;
  float *q_ref = nullptr;
  double *q_part = nullptr;
  float *q_box = nullptr;                // lo[kMaxM], hi[kMaxM]
  unsigned long long *q_hits = nullptr;
  // write-set check (GMPEA_CHECK_WRITES=1 at init): generations verified so far
  int64_t checked = 0;
  // graph replay of `gchunk` generations
  hipGraphExec_t gexec = nullptr;
  int32_t gchunk = 0;
  int32_t graph_chunk_cfg = 64;
};

namespace {

// Decision vectors gathered per pass of gmpea_front, and reference points per
// IGD launch of gmpea_quality (a multiple of kBlock, so the per-block partial
// sums come out in the same order as one launch over every point).
constexpr int32_t kFrontRows = 4096;
constexpr int32_t kQualityRefs = 16 * kBlock;

void *dev_alloc(gmpea_s *h, size_t bytes) {
  void *p = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  if (h->hook) {
    p = h->al.alloc(bytes, h->al.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    h->allocs.emplace_back(p, bytes);
    h->bytes += bytes;
  }
  return p;
}

void dev_free(gmpea_s *h, void *p) {
  for (size_t q = 0; q < h->allocs.size(); ++q) {
    if (h->allocs[q].first == p) {
      h->bytes -= h->allocs[q].second;
      h->allocs.erase(h->allocs.begin() + static_cast<long>(q));
      break;
    }
  }
  if (h->hook)
    h->al.free(p, h->al.ctx);
  else
    (void)hipFree(p);
}

void release_all(gmpea_s *h) {
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  while (!h->allocs.empty()) dev_free(h, h->allocs.back().first);
  if (h->own_stream && h->stream) {
    (void)hipStreamDestroy(h->stream);
    h->stream = nullptr;
  }
}

// Live handles: a destroyed (or never created) handle is rejected with ESTATE
// without touching freed memory.
std::mutex g_live_mu;
std::unordered_set<const gmpea_s *> g_live;

bool valid(gmpea_t h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return h != nullptr && g_live.count(h) != 0;
}

void register_live(gmpea_s *h, bool on) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  if (on)
    g_live.insert(h);
  else
    g_live.erase(h);
}

// Several device arrays carved out of one allocation (256-byte aligned pieces):
// a first pass with no base sizes the block, a second hands out the pointers.
struct Carve {
  char *base = nullptr;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = (off + 255) & ~static_cast<size_t>(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(n * sizeof(T), 1);
    return p;
  }
};

gmpea_status sync_stream(hipStream_t s, const char *what) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, what);
  return GMPEA_OK;
}

gmpea_status sync(gmpea_s *h, const char *what) { return sync_stream(h->stream, what); }

gmpea_status validate(const gmpea_problem *P, const gmpea_config *C) {
  if (!P || !C) return fail(GMPEA_EINVAL, "gmpea_init: problem and config are required");
  if (P->m < 2) return fail(GMPEA_EINVAL, "gmpea_init: m must be at least 2");
  if (P->m > GMPEA_MAX_M) return fail(GMPEA_EUNSUPPORTED, "gmpea_init: m above GMPEA_MAX_M");
  if (P->family != GMPEA_FAMILY_CURVE && P->family != GMPEA_FAMILY_SPHERE)
    return fail(GMPEA_EINVAL, "gmpea_init: unknown problem family");
  if (P->family == GMPEA_FAMILY_CURVE && (P->m != 2 || P->d < 2))
    return fail(GMPEA_EINVAL, "gmpea_init: the curve family needs m = 2 and d >= 2");
  if (P->family == GMPEA_FAMILY_SPHERE && P->d < P->m - 1)
    return fail(GMPEA_EINVAL, "gmpea_init: the sphere family needs d >= m - 1");
  if (P->d < 1 || P->d > (1 << 20)) return fail(GMPEA_EINVAL, "gmpea_init: d out of range");
  if (P->n_eq && P->d < 2) return fail(GMPEA_EINVAL, "gmpea_init: the equality needs d >= 2");
  if (P->n_ring < 0 || P->n_ring > GMPEA_MAX_RING)
    return fail(GMPEA_EINVAL, "gmpea_init: n_ring out of range");
  if (P->n_ring > 0 && (!P->ring_center || !P->ring_radius))
    return fail(GMPEA_EINVAL, "gmpea_init: ring constants missing");
  if (P->n_eq != 0 && P->n_eq != 1) return fail(GMPEA_EINVAL, "gmpea_init: n_eq must be 0 or 1");
  if (P->n_eq && !(P->eq_tol >= 0.0)) return fail(GMPEA_EINVAL, "gmpea_init: eq_tol must be >= 0");
  if ((P->lb == nullptr) != (P->ub == nullptr))
    return fail(GMPEA_EINVAL, "gmpea_init: give both lb and ub or neither");
  if (P->lb)
    for (int32_t l = 0; l < P->d; ++l)
      if (!(P->lb[l] < P->ub[l]) || !std::isfinite(P->lb[l]) || !std::isfinite(P->ub[l]))
        return fail(GMPEA_EINVAL, "gmpea_init: need finite lb < ub in every variable");
  if (C->h_outer < 0 || C->h_inner < 0) return fail(GMPEA_EINVAL, "gmpea_init: negative layer divisions");
  if (C->h_inner > 0 && C->h_outer == 0)
    return fail(GMPEA_EINVAL, "gmpea_init: an inner layer (h_inner) needs an outer one (h_outer)");
  if (C->h_outer == 0 && C->n_req < 2) return fail(GMPEA_EINVAL, "gmpea_init: n_req must be at least 2");
  if (C->h_outer == 0 && C->n_req > (1 << 26))
    return fail(GMPEA_EUNSUPPORTED, "gmpea_init: n_req too large");
  if (C->h_outer > 4096 || C->h_inner > 4096)
    return fail(GMPEA_EUNSUPPORTED, "gmpea_init: layer divisions too large");
  if (C->agg != GMPEA_AGG_PBI && C->agg != GMPEA_AGG_TCHE)
    return fail(GMPEA_EINVAL, "gmpea_init: unknown aggregation");
  if (C->T < 0 || C->t1 < 0 || C->t2 < 0) return fail(GMPEA_EINVAL, "gmpea_init: negative size");
  if (C->pc < 0 || C->pc > 1 || C->pm < 0 || C->pm > 1)
    return fail(GMPEA_EINVAL, "gmpea_init: probabilities must lie in [0, 1]");
  if (C->eta_c < 0 || C->eta_m < 0 || C->theta < 0)
    return fail(GMPEA_EINVAL, "gmpea_init: negative distribution index or penalty");
  if (C->op != GMPEA_OP_SBX && C->op != GMPEA_OP_DE)
    return fail(GMPEA_EINVAL, "gmpea_init: unknown reproduction operator");
  if (!(C->de_f >= 0.0) || !std::isfinite(C->de_f))
    return fail(GMPEA_EINVAL, "gmpea_init: de_f must be finite and >= 0");
  if (C->op1_rule != GMPEA_OP1_FPR && C->op1_rule != GMPEA_OP1_FEASIBLE_FIRST)
    return fail(GMPEA_EINVAL, "gmpea_init: unknown OP1 rule");
  return GMPEA_OK;
}

gmpea_status build_graph(gmpea_s *h, int32_t chunk) {
  if (h->gexec && h->gchunk == chunk) return GMPEA_OK;
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  hipStream_t cap;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "graph stream");
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int32_t g = 0; g < chunk && e == hipSuccess; ++g) e = launch_generation(h->st, cap);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
  }
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    h->gexec = nullptr;
    return hip_fail(e, "graph capture");
  }
  h->gchunk = chunk;
  return GMPEA_OK;
}

// The write-set check of one generation: each offspring row got every chunk
// written once and each offspring record once; each parent slot got at most one
// of a replacement (its record and location) or a move of its kept row home
// (location and every chunk), and nothing else was written.
gmpea_status check_write_sets(gmpea_s *h) {
  const DevState &st = h->st;
  const int64_t n = st.n;
  std::vector<int32_t> c(static_cast<size_t>(8 * n));
  hipError_t e = hipMemcpyAsync(c.data(), st.wcheck, c.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(st.wcheck, 0, c.size() * sizeof(int32_t), h->stream);
  if (e != hipSuccess) return hip_fail(e, "write-set check");
  auto at = [&](int kind, int p, int64_t j) { return c[static_cast<size_t>((2 * kind + p) * n + j)]; };
  for (int p = 0; p < 2; ++p)
    for (int64_t j = 0; j < n; ++j) {
      const int32_t vr = at(0, p, j), op = at(1, p, j), rp = at(2, p, j), mv = at(3, p, j);
      const char *what = nullptr;
      if (vr != st.nq) what = "offspring row chunks";
      else if (op != 1) what = "offspring record";
      else if (rp > 1) what = "slot replacement";
      else if (mv != 0 && mv != 1 + st.nq) what = "kept row moved home";
      else if (rp == 1 && mv != 0) what = "slot both replaced and moved";
      if (what)
        return fail(GMPEA_ESTATE, "write-set check failed after generation " + std::to_string(h->checked + 1) +
                                      ": " + what + ", population " + std::to_string(p) + ", index " +
                                      std::to_string(j) + " (counts " + std::to_string(vr) + " " +
                                      std::to_string(op) + " " + std::to_string(rp) + " " + std::to_string(mv) + ")");
    }
  ++h->checked;
  return GMPEA_OK;
}

gmpea_status enqueue(gmpea_s *h, int32_t n) {
  if (h->st.wcheck) {  // one generation at a time, each verified
    for (int32_t g = 0; g < n; ++g) {
      hipError_t e = launch_generation(h->st, h->stream);
      if (e != hipSuccess) return hip_fail(e, "generation launch");
      gmpea_status s = check_write_sets(h);
      if (s != GMPEA_OK) return s;
    }
    return GMPEA_OK;
  }
  const int32_t G = h->graph_chunk_cfg;
  if (n == 0 && G >= 2) return build_graph(h, G);  // prepare the replay, launch nothing
  if (G >= 2 && n >= G) {
    gmpea_status s = build_graph(h, G);
    if (s != GMPEA_OK) return s;
    while (n >= G) {
      hipError_t e = hipGraphLaunch(h->gexec, h->stream);
      if (e != hipSuccess) return hip_fail(e, "graph launch");
      n -= G;
    }
  }
  for (int32_t g = 0; g < n; ++g) {
    hipError_t e = launch_generation(h->st, h->stream);
    if (e != hipSuccess) return hip_fail(e, "generation launch");
  }
  return GMPEA_OK;
}

template <class T>
gmpea_status d2h(gmpea_s *h, T *dst, const void *src, size_t n, const char *what) {
  hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(e, what);
  return sync(h, what);
}

template <class T>
gmpea_status h2d(gmpea_s *h, void *dst, const T *src, size_t n, const char *what) {
  hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, what);
  return sync(h, what);
}

// The library must run on a HIP runtime at least as new as the toolchain it was
// built with (HIP keeps old binaries working on newer runtimes, not the reverse).
// A process that already loaded an older runtime under the same soname (for
// example one bundled with a framework) is refused instead of crashing later.
gmpea_status check_runtime(const char *who) {
  int rt = 0;
  hipError_t e = hipRuntimeGetVersion(&rt);
  if (e != hipSuccess) return hip_fail(e, who);
  const int built = HIP_VERSION_MAJOR * 100 + HIP_VERSION_MINOR;
  const int have = (rt / 10000000) * 100 + (rt / 100000) % 100;
  if (have < built)
    return fail(GMPEA_EUNSUPPORTED,
                std::string(who) + ": HIP runtime " + std::to_string(have / 100) + "." +
                    std::to_string(have % 100) + " is older than the HIP " +
                    std::to_string(HIP_VERSION_MAJOR) + "." + std::to_string(HIP_VERSION_MINOR) +
                    " toolchain this library was built with; load it in a process whose HIP "
                    "runtime is the toolchain's (or newer)");
  return GMPEA_OK;
}

// Fixed device scratch of gmpea_front_static, for callers that cannot allocate:
// one copy per GPU, held until the process ends. In host code `scratch` names a
// host-side stand-in, never the device array: its device address on each GPU
// comes from hipGetSymbolAddress (static_scratch below).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;  // device -> that device's copy of scratch

// Device address of `device`'s copy of the scratch, looked up once per device
// with that device current.
gmpea_status static_scratch(int device, unsigned char **out, const char *who) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return GMPEA_OK;
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != device) e = hipSetDevice(device);
  void *p = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hip_fail(e, who);
  g_scratch_addr[device] = static_cast<unsigned char *>(p);
  *out = static_cast<unsigned char *>(p);
  return GMPEA_OK;
}

// Device buffers one front extraction works in: the handle's own (carved at
// gmpea_init) or the library's fixed scratch (gmpea_front_static).
struct FrontBufs {
  uint8_t *keep;   // n flags
  int32_t *idx;    // n row indices
  float4 *fc;      // n F/CV records
  float *x;        // x_rows decision vectors
  int32_t x_rows;
};

FrontBufs handle_bufs(gmpea_s *h) {
  return FrontBufs{h->f_keep, h->f_idx, h->f_fc, h->f_x, std::min(kFrontRows, h->st.n)};
}

// Row indices (ascending) of a front selector: the feasible non-dominated rows
// of population 1 (flags on the device), or every row of a population.
gmpea_status front_rows(gmpea_s *h, const FrontBufs &b, int32_t what, std::vector<int32_t> &rows,
                        const char *who) {
  const DevState &st = h->st;
  rows.clear();
  gmpea_status s = GMPEA_OK;
  if (what == GMPEA_FRONT_FEASIBLE_ND) {
    hipError_t e = st.m > 3 ? launch_front_flags_wide(st, 0, b.keep, h->stream)
                            : launch_front_flags(st, 0, b.keep, h->stream);
    std::vector<uint8_t> hk(st.n);
    s = e == hipSuccess ? d2h(h, hk.data(), b.keep, st.n, who) : hip_fail(e, who);
    if (s != GMPEA_OK) return s;
    for (int32_t i = 0; i < st.n; ++i)
      if (hk[i]) rows.push_back(i);
  } else {
    s = sync(h, who);
    if (s != GMPEA_OK) return s;
    rows.resize(st.n);
    for (int32_t i = 0; i < st.n; ++i) rows[i] = i;
  }
  return GMPEA_OK;
}

// The F/CV records of `rows` (non-empty) of population `pop` gathered into
// b.fc, in row order; the row list stays in b.idx.
gmpea_status front_gather_fc(gmpea_s *h, const FrontBufs &b, int pop, const std::vector<int32_t> &rows,
                             const char *who) {
  const int32_t cnt = static_cast<int32_t>(rows.size());
  gmpea_status s = h2d(h, b.idx, rows.data(), cnt, who);
  if (s != GMPEA_OK) return s;
  hipError_t e = launch_gather(h->st, pop, b.idx, cnt, nullptr, b.fc, h->stream);
  if (e != hipSuccess) return hip_fail(e, who);
  return GMPEA_OK;
}

// Front extraction shared by gmpea_front and gmpea_front_static.
gmpea_status front_impl(gmpea_s *h, const FrontBufs &b, int32_t what, int32_t capacity, float *x,
                        float *f, float *cv, int32_t *idx, int32_t *count, const char *who) {
  const DevState &st = h->st;
  const int pop = what == GMPEA_FRONT_POP2 ? 1 : 0;
  std::vector<int32_t> rows;
  gmpea_status s = front_rows(h, b, what, rows, who);
  if (s != GMPEA_OK) return s;
  const int32_t cnt = static_cast<int32_t>(rows.size());
  *count = cnt;
  if (cnt > capacity) return fail(GMPEA_ECAPACITY, std::string(who) + ": capacity below the row count");
  if (cnt == 0) return GMPEA_OK;
  if (idx) std::copy(rows.begin(), rows.end(), idx);
  s = front_gather_fc(h, b, pop, rows, who);
  // decision vectors in passes of b.x_rows rows
  for (int32_t r0 = 0; x && s == GMPEA_OK && r0 < cnt; r0 += b.x_rows) {
    const int32_t c = std::min(b.x_rows, cnt - r0);
    hipError_t e = launch_gather(st, pop, b.idx + r0, c, b.x, nullptr, h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    s = d2h(h, x + static_cast<size_t>(r0) * st.d, b.x, static_cast<size_t>(c) * st.d, who);
  }
  std::vector<float4> hfc;
  if (s == GMPEA_OK) {
    hfc.resize(static_cast<size_t>(cnt) * st.rq);
    s = d2h(h, hfc.data(), b.fc, hfc.size(), who);
  }
  if (s == GMPEA_OK) {
    const float *v = reinterpret_cast<const float *>(hfc.data());
    const size_t rw = static_cast<size_t>(st.rq) * 4;
    for (int32_t r = 0; r < cnt; ++r) {
      if (f)
        for (int32_t a = 0; a < st.m; ++a) f[static_cast<size_t>(r) * st.m + a] = v[r * rw + a];
      if (cv) cv[r] = v[r * rw + rw - 1];
    }
  }
  return s;
}

}  // namespace

extern "C" {

const char *gmpea_last_error(void) { return g_err.c_str(); }

gmpea_status gmpea_sync(gmpea_t h) {
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_sync: invalid handle");
  return sync(h, "gmpea_sync");
}

gmpea_status gmpea_init(const gmpea_problem *P, const gmpea_config *C, const gmpea_allocator *A,
                        void *hip_stream, gmpea_t *out) {
  Trace trace("gmpea_init");
  if (!out) return fail(GMPEA_EINVAL, "gmpea_init: out is NULL");
  gmpea_status s = validate(P, C);
  if (s != GMPEA_OK) return s;
  if (A && (!A->alloc || !A->free)) return fail(GMPEA_EINVAL, "gmpea_init: incomplete allocator");

  const int32_t m = P->m, d = P->d;
  const bool layered = C->h_outer > 0;
  const int32_t H = layered ? C->h_outer : dd_divisions(m, C->n_req);
  const int32_t H2 = layered ? C->h_inner : 0;
  // counts grow fast with m: compare in floating point before any exact count
  const double approx = std::exp(std::lgamma(H + m) - std::lgamma(m) - std::lgamma(H + 1.0)) +
                        (H2 > 0 ? std::exp(std::lgamma(H2 + m) - std::lgamma(m) - std::lgamma(H2 + 1.0)) : 0.0);
  if (approx > double(1 << 27)) return fail(GMPEA_EUNSUPPORTED, "gmpea_init: population too large");
  const int64_t n64 = refset_count(m, H, H2);
  if (n64 > (1 << 27)) return fail(GMPEA_EUNSUPPORTED, "gmpea_init: population too large");
  if (H2 > 0 && int64_t(2) * m * H * H2 * std::max(H, H2) >= (int64_t(1) << 31))
    return fail(GMPEA_EUNSUPPORTED, "gmpea_init: layer divisions too large for exact distances");
  const int32_t N = static_cast<int32_t>(n64);
  const int32_t T = C->T;
  const int32_t t1 = C->t1 > 0 ? C->t1 : T / 2;
  const int32_t t2 = C->t2 > 0 ? C->t2 : 2 * T;
  if (t1 < 1 || t2 < 1 || t1 > N || t2 > N)
    return fail(GMPEA_EINVAL, "gmpea_init: need 1 <= t1, t2 <= N (population " + std::to_string(N) +
                                  ", t1 " + std::to_string(t1) + ", t2 " + std::to_string(t2) + ")");
  if (static_cast<int64_t>(N) * std::max(t1, t2) >= (int64_t(1) << 31))
    return fail(GMPEA_EUNSUPPORTED, "gmpea_init: N * t above the 32-bit index range");
  s = check_runtime("gmpea_init");
  if (s != GMPEA_OK) return s;

  gmpea_s *h = new gmpea_s();
  if (A) {
    h->al = *A;
    h->hook = true;
  }
  if (const char *g = std::getenv("GMPEA_GRAPH_CHUNK")) h->graph_chunk_cfg = std::atoi(g);
  if (hip_stream) {
    h->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete h;
      return hip_fail(e, "gmpea_init: stream");
    }
    h->own_stream = true;
  }
  h->H = H;
  h->H2 = H2;
  h->record = C->record != 0;
  (void)hipGetDevice(&h->device);
  {
    unsigned char *sc = nullptr;  // gmpea_front_static's scratch address on this device
    s = static_scratch(h->device, &sc, "gmpea_init");
    if (s != GMPEA_OK) {
      if (h->own_stream) (void)hipStreamDestroy(h->stream);
      delete h;
      return s;
    }
  }

  // ---- neighbourhood offsets (host, a few KB) when the device builds the tables:
  // one Das-Dennis layer with m <= 3; otherwise the host builds them ----
  const int32_t ts[2] = {t1, t2};
  const bool dev_tables = m <= 3 && H2 == 0;
  std::vector<int32_t> offs;
  if (dev_tables) neighbour_offsets(m, H, std::max(t1, t2), offs);
  const int32_t noffs = static_cast<int32_t>(offs.size() / 2);

  // ---- device state ----
  DevState &st = h->st;
  st.n = N;
  st.m = m;
  st.d = d;
  st.nq = (d + 3) >> 2;
  {
    // row pitch: the variables rounded up to whole float4 chunks, or to a
    // multiple of GMPEA_ROW_ALIGN floats when set (a layout experiment knob)
    int32_t align = 4;
    if (const char *a = std::getenv("GMPEA_ROW_ALIGN")) align = std::max(4, (std::atoi(a) + 3) & ~3);
    st.stride = (4 * st.nq + align - 1) / align * align;
    // the variation kernel: task-dealt for rows of at most kTaskChunks chunks
    // (d <= 128), lane groups for longer rows; GMPEA_TASKED=0 takes lane groups
    // for every width (a comparison knob: the kernel fixes the evaluation's
    // rounding order, so runs to be compared bitwise must agree on it)
    const char *tk = std::getenv("GMPEA_TASKED");
    st.tasked = (st.nq <= kTaskChunks && !(tk && std::atoi(tk) == 0)) ? 1 : 0;
    st.task_off = task_off_for(N, st.nq, m > 3, false);
    // offspring generations kept in the arena (GMPEA_OFFSPRING_GENERATIONS, 2 to
    // 16, is a layout experiment knob; results do not depend on it)
    st.npar = kOffspringGenerations;
    if (const char *a = std::getenv("GMPEA_OFFSPRING_GENERATIONS"))
      st.npar = std::min(16, std::max(2, std::atoi(a)));
    // arena rows are 31-bit indices (the variation keeps a flag in bit 31):
    // fewer generations for the largest populations
    const int64_t rows_pad = int64_t((N + kBlock - 1) / kBlock) * kBlock;
    st.npar = static_cast<int32_t>(std::max<int64_t>(2, std::min<int64_t>(st.npar, ((int64_t(1) << 31) / rows_pad - 2) / 2)));
  }
  // the write-set check: every write of a generation counted per target and
  // verified on the host after the generation (one generation per launch set)
  const char *cw = std::getenv("GMPEA_CHECK_WRITES");
  const bool check_writes = cw && std::atoi(cw) == 1;
  st.rq = rec_quads(m);
  st.nblk = (N + kBlock - 1) / kBlock;
  st.t[0] = t1;
  st.t[1] = t2;
  for (int p = 0; p < 2; ++p) {
    // lanes per slot in k_select: sel_per_lane reverse-list entries per lane
    int l = 1;
    while (sel_per_lane(st.rq) * l < st.t[p] && l < 64) l <<= 1;
    st.lps[p] = l;
  }
  st.sel_blocks0 = (N + kBlock / st.lps[0] - 1) / (kBlock / st.lps[0]);
  st.sel_blocks1 = (N + kBlock / st.lps[1] - 1) / (kBlock / st.lps[1]);
  st.agg = C->agg;
  st.theta = static_cast<float>(C->theta > 0 ? C->theta : 5.0);
  const double eta_c = C->eta_c > 0 ? C->eta_c : 20.0, eta_m = C->eta_m > 0 ? C->eta_m : 20.0;
  const double pc = C->pc > 0 ? C->pc : 1.0, pm = C->pm > 0 ? C->pm : 1.0 / d;
  st.sbx_e = static_cast<float>(1.0 / (eta_c + 1.0));
  st.pm_p = static_cast<float>(eta_m + 1.0);
  st.pm_e = static_cast<float>(1.0 / (eta_m + 1.0));
  st.tpm = static_cast<uint64_t>(std::floor(pm * 4294967296.0));
  st.tpc = static_cast<uint64_t>(std::floor(pc * 4294967296.0));
  st.inv_tpm = st.tpm > 0 ? static_cast<float>(1.0 / static_cast<double>(st.tpm)) : 0.0f;
  st.op = C->op;
  st.op1_rule = C->op1_rule;
  st.de_f = static_cast<float>(C->de_f > 0 ? C->de_f : 0.5);
  st.key0 = static_cast<uint32_t>(C->seed & 0xFFFFFFFFull);
  st.key1 = static_cast<uint32_t>(C->seed >> 32);
  DevProblem &dp = st.prob;
  dp.family = P->family;
  dp.m = m;
  dp.d = d;
  dp.n_ring = P->n_ring;
  dp.has_sum_lower = P->has_sum_lower ? 1 : 0;
  dp.n_eq = P->n_eq;
  for (int32_t j = 0; j < P->n_ring; ++j) {
    for (int32_t a = 0; a < m; ++a)
      dp.ring_c[j * m + a] = static_cast<float>(P->ring_center[static_cast<size_t>(j) * m + a]);
    dp.ring_r2[j] = static_cast<float>(P->ring_radius[j] * P->ring_radius[j]);
  }
  dp.sum_lower = static_cast<float>(P->sum_lower);
  dp.eq_tol = static_cast<float>(P->eq_tol);
  dp.g_scale = d > 1 ? static_cast<float>(9.0 / (d - 1)) : 0.0f;

  const size_t rows = static_cast<size_t>(st.nblk) * kBlock;
  const int32_t tail_cap[2] = {static_cast<int32_t>(static_cast<int64_t>(N) * t1 / 8 + 256),
                               static_cast<int32_t>(static_cast<int64_t>(N) * t2 / 8 + 256)};
  float *lb = nullptr, *ub = nullptr, *inv_span = nullptr;
  int2 *d_offs = nullptr;
  uint32_t *d_flag = nullptr;
  auto layout = [&](Carve &c) {
    lb = c.take<float>(st.stride);
    ub = c.take<float>(st.stride);
    inv_span = c.take<float>(st.stride);
    st.rows = c.take<float>((2 + 2 * static_cast<size_t>(st.npar)) * rows * st.stride);
    for (int p = 0; p < 2; ++p) {
      st.X[p] = st.rows ? st.rows + p * rows * st.stride : nullptr;
      st.loc[p] = c.take<uint32_t>(rows);
      st.FC[p] = c.take<float4>(rows * st.rq);
      st.FCO[p] = c.take<float4>(rows * st.rq);
      st.FCN[p] = c.take<float4>(rows * st.rq);
      st.B[p] = c.take<int32_t>(static_cast<size_t>(N) * ts[p]);
      st.rhead[p] = c.take<int32_t>(static_cast<size_t>(N) * ts[p]);
      st.rtoff[p] = c.take<int32_t>(static_cast<size_t>(N) + 1);
      st.mate[p] = h->record ? c.take<int32_t>(rows * 2) : nullptr;
      st.win[p] = h->record ? c.take<int32_t>(rows) : nullptr;
    }
    st.W = c.take<float4>(rows * st.rq);
    st.src = c.take<uint8_t>(rows);
    st.zkey = c.take<uint32_t>(kMaxM);
    st.gen = c.take<uint32_t>(4);
    st.repl = c.take<unsigned long long>(2 * kReplLanes);
    d_offs = c.take<int2>(noffs);
    d_flag = c.take<uint32_t>(4);
    // reverse-list tails with room for an eighth of the entries (lattice
    // neighbourhoods put well under 1 % there); a larger tail is rebuilt exactly
    for (int p = 0; p < 2; ++p) st.rtail[p] = c.take<int32_t>(tail_cap[p]);
    st.wcheck = check_writes ? c.take<int32_t>(8 * static_cast<size_t>(N)) : nullptr;
    // delivery scratch (gmpea_front, gmpea_quality)
    h->f_keep = c.take<uint8_t>(static_cast<size_t>(N));
    h->f_idx = c.take<int32_t>(static_cast<size_t>(N));
    h->f_fc = c.take<float4>(static_cast<size_t>(N) * st.rq);
    h->f_x = c.take<float>(static_cast<size_t>(std::min(kFrontRows, N)) * d);
    h->q_ref = c.take<float>(static_cast<size_t>(kQualityRefs) * m);
    h->q_part = c.take<double>(kQualityRefs / kBlock);
    h->q_box = c.take<float>(2 * kMaxM);
    h->q_hits = c.take<unsigned long long>(1);
  };
  Carve sizing;
  layout(sizing);
  Carve carve;
  carve.base = static_cast<char *>(dev_alloc(h, sizing.off));
  if (!carve.base) {
    release_all(h);
    delete h;
    return fail(GMPEA_ENOMEM, "gmpea_init: device allocation failed");
  }
  layout(carve);
  dp.lb = lb;
  dp.ub = ub;
  dp.inv_span = inv_span;

  // bounds padded to the row stride; padding lanes get [0, 1]
  std::vector<float> lbf(st.stride, 0.0f), ubf(st.stride, 1.0f), isf(st.stride, 1.0f);
  for (int32_t l = 0; l < d; ++l) {
    const double lo = P->lb ? P->lb[l] : 0.0, hi = P->ub ? P->ub[l] : 1.0;
    lbf[l] = static_cast<float>(lo);
    ubf[l] = static_cast<float>(hi);
    isf[l] = static_cast<float>(1.0 / (static_cast<double>(ubf[l]) - static_cast<double>(lbf[l])));
  }
  hipError_t e = hipSuccess;
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream);
  };
  // buffers to clear are collected and cleared by one launch (flush); a byte
  // other than 0 or 0xFF, an unaligned span or a full list takes hipMemsetAsync
  FillSpans fl{};
  auto zero = [&](void *dst, int v, size_t bytes) {
    if (e != hipSuccess || bytes == 0) return;
    if ((v == 0 || v == 0xFF) && (reinterpret_cast<uintptr_t>(dst) & 3u) == 0 && bytes % 4 == 0 &&
        fl.count < kMaxFillSpans) {
      fl.p[fl.count] = static_cast<uint32_t *>(dst);
      fl.words[fl.count] = bytes / 4;
      fl.value[fl.count] = v ? 0xFFFFFFFFu : 0u;
      ++fl.count;
    } else {
      e = hipMemsetAsync(dst, v, bytes, h->stream);
    }
  };
  auto flush = [&]() {
    if (e == hipSuccess) e = launch_fill(fl, h->stream);
    fl.count = 0;
  };
  cp(lb, lbf.data(), st.stride * sizeof(float));
  cp(ub, ubf.data(), st.stride * sizeof(float));
  cp(inv_span, isf.data(), st.stride * sizeof(float));
  if (noffs > 0) cp(d_offs, offs.data(), offs.size() * sizeof(int32_t));
  zero(d_flag, 0, 4 * sizeof(uint32_t));
  st.region = static_cast<int64_t>(rows);
  // the home rows and the first generation slot's offspring rows (what a read
  // of X or of the offspring returns before any generation); every other
  // offspring row is written whole (padding included) before it is read
  zero(st.rows, 0, 4 * rows * st.stride * sizeof(float));
  for (int p = 0; p < 2; ++p) {
    zero(st.FC[p], 0, rows * st.rq * sizeof(float4));
    zero(st.FCO[p], 0, rows * st.rq * sizeof(float4));
    zero(st.FCN[p], 0, rows * st.rq * sizeof(float4));
    zero(const_cast<int32_t *>(st.rtoff[p]), 0, (static_cast<size_t>(N) + 1) * sizeof(int32_t));
    zero(const_cast<int32_t *>(st.rhead[p]), 0xFF, static_cast<size_t>(N) * ts[p] * sizeof(int32_t));
    if (h->record) {
      zero(st.mate[p], 0xFF, rows * 2 * sizeof(int32_t));
      zero(st.win[p], 0xFF, rows * sizeof(int32_t));
    }
  }
  zero(st.src, 0, rows);
  zero(st.zkey, 0xFF, kMaxM * sizeof(uint32_t));
  zero(st.gen, 0, 4 * sizeof(uint32_t));
  zero(st.repl, 0, 2 * kReplLanes * sizeof(unsigned long long));
  if (st.wcheck) zero(st.wcheck, 0, 8 * static_cast<size_t>(N) * sizeof(int32_t));
  flush();
  // reference vectors and neighbourhoods: on the device for one Das-Dennis layer
  // with m <= 3, else on the host (W rounded once from FP64, rq float4 per row)
  if (dev_tables) {
    // the flag that some row's offset walk came up short is read at the end
    if (e == hipSuccess)
      e = launch_tables(m, N, H, d_offs, noffs, t1, t2, C->agg, st.W, const_cast<int32_t *>(st.B[0]),
                        const_cast<int32_t *>(st.B[1]), d_flag, h->stream);
  } else if (e == hipSuccess) {
    std::vector<int32_t> K, Bh;
    std::vector<double> Wd;
    refset(m, H, H2, K, &Wd);
    std::vector<float> Wf(static_cast<size_t>(N) * st.rq * 4, 0.0f);
    for (int32_t i = 0; i < N; ++i) {
      double nrm = 0.0;
      for (int32_t a = 0; a < m; ++a) nrm += Wd[static_cast<size_t>(i) * m + a] * Wd[static_cast<size_t>(i) * m + a];
      nrm = std::sqrt(nrm);
      for (int32_t a = 0; a < m; ++a) {
        const double w = Wd[static_cast<size_t>(i) * m + a];
        Wf[static_cast<size_t>(i) * st.rq * 4 + a] = static_cast<float>(C->agg == GMPEA_AGG_PBI ? w / nrm : w);
      }
    }
    e = hipMemcpyAsync(st.W, Wf.data(), Wf.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
    const int32_t tmax = std::max(t1, t2);
    if (tmax <= kKnnMaxTHost && e == hipSuccess) {
      // exact search on the device (one block per row); every coordinate lies
      // in [0, S] with S = 2 m H1 H2 (H1 for one layer) and the rows sum to S,
      // so no squared distance exceeds 2 S^2
      const uint64_t S = H2 > 0 ? uint64_t(2) * m * H * H2 : uint64_t(H);
      int32_t *dK = static_cast<int32_t *>(dev_alloc(h, K.size() * sizeof(int32_t)));
      if (!dK) {
        release_all(h);
        delete h;
        return fail(GMPEA_ENOMEM, "gmpea_init: device allocation failed");
      }
      e = hipMemcpyAsync(dK, K.data(), K.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess)
        e = launch_knn(dK, N, m, 2 * S * S, t1, t2, const_cast<int32_t *>(st.B[0]),
                       const_cast<int32_t *>(st.B[1]), h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      dev_free(h, dK);
    } else {
      // one host search for the larger neighbourhood: the smaller one is its
      // prefix, since both lists are in (distance, index) order
      refset_neighbours(K, m, H, H2, tmax, Bh);
      std::vector<int32_t> Bp;
      for (int p = 0; p < 2 && e == hipSuccess; ++p) {
        Bp.resize(static_cast<size_t>(N) * ts[p]);
        for (int32_t i = 0; i < N; ++i)
          std::copy_n(&Bh[static_cast<size_t>(i) * tmax], ts[p], &Bp[static_cast<size_t>(i) * ts[p]]);
        e = hipMemcpyAsync(const_cast<int32_t *>(st.B[p]), Bp.data(), Bp.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // Wf is read before it goes
  }
  // reverse lists into the tails carved above. The four offspring record
  // buffers serve as the zeroed cursor arrays (one per count and fill of each
  // population, each holding at least 4N words), so the lists need no clearing
  // between their launches; clear_cursors zeroes the four again afterwards, and
  // clear_lists empties the offsets and heads (with the flags) for a rebuild.
  int32_t *const cursor[4] = {reinterpret_cast<int32_t *>(st.FCO[0]), reinterpret_cast<int32_t *>(st.FCO[1]),
                              reinterpret_cast<int32_t *>(st.FCN[0]), reinterpret_cast<int32_t *>(st.FCN[1])};
  auto reverse_lists = [&](const int32_t *cap) {
    for (int p = 0; p < 2; ++p) {
      if (e == hipSuccess)
        e = launch_reverse_count(N, ts[p], st.B[p], cursor[2 * p], const_cast<int32_t *>(st.rtoff[p]), h->stream);
      if (e == hipSuccess)
        e = launch_reverse_fill(N, ts[p], st.B[p], st.rtoff[p], cursor[2 * p + 1],
                                const_cast<int32_t *>(st.rhead[p]), const_cast<int32_t *>(st.rtail[p]), cap[p],
                                d_flag + 1 + p, h->stream);
    }
  };
  auto clear_cursors = [&]() {
    for (int c = 0; c < 4; ++c) zero(cursor[c], 0, rows * st.rq * sizeof(float4));
    flush();
  };
  auto clear_lists = [&]() {
    zero(d_flag, 0, 4 * sizeof(uint32_t));
    for (int p = 0; p < 2; ++p) {
      zero(const_cast<int32_t *>(st.rtoff[p]), 0, (static_cast<size_t>(N) + 1) * sizeof(int32_t));
      zero(const_cast<int32_t *>(st.rhead[p]), 0xFF, static_cast<size_t>(N) * ts[p] * sizeof(int32_t));
    }
    flush();
  };
  reverse_lists(tail_cap);
  clear_cursors();
  if (e == hipSuccess) e = launch_init(st, h->stream);
  // one wait for everything above: the tables' and the tails' flags
  uint32_t flags[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(flags, d_flag, sizeof(flags), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && flags[0]) {
    // some row (near a lattice corner) needs neighbours beyond the offset list:
    // the host's exact search provides both tables, then the lists again
    std::vector<int32_t> K, Bh;
    dd_lattice(m, H, K);
    for (int p = 0; p < 2 && e == hipSuccess; ++p) {
      lattice_knn(K, m, H, ts[p], Bh);
      e = hipMemcpyAsync(const_cast<int32_t *>(st.B[p]), Bh.data(), Bh.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    clear_lists();
    reverse_lists(tail_cap);
    clear_cursors();
    if (e == hipSuccess) e = hipMemcpyAsync(flags, d_flag, sizeof(flags), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  }
  if (e == hipSuccess && (flags[1] || flags[2])) {
    // a tail beyond its room: tails of the exact sizes (toff[N] after the count)
    int32_t tail_n[2] = {0, 0};
    for (int p = 0; p < 2 && e == hipSuccess; ++p)
      e = hipMemcpyAsync(&tail_n[p], st.rtoff[p] + N, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) {
      Carve sizing;
      sizing.take<int32_t>(static_cast<size_t>(tail_n[0]));
      sizing.take<int32_t>(static_cast<size_t>(tail_n[1]));
      Carve carve;
      carve.base = static_cast<char *>(dev_alloc(h, sizing.off));
      if (!carve.base) {
        release_all(h);
        delete h;
        return fail(GMPEA_ENOMEM, "gmpea_init: device allocation failed");
      }
      st.rtail[0] = carve.take<int32_t>(static_cast<size_t>(tail_n[0]));
      st.rtail[1] = carve.take<int32_t>(static_cast<size_t>(tail_n[1]));
      clear_lists();
      reverse_lists(tail_n);
      clear_cursors();
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
  }
  if (e != hipSuccess) {
    gmpea_status r = hip_fail(e, "gmpea_init");
    release_all(h);
    delete h;
    return r;
  }
  register_live(h, true);
  *out = h;
  return GMPEA_OK;
}

gmpea_status gmpea_step(gmpea_t h, int32_t n_gen) {
  Trace trace("gmpea_step");
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_step: invalid handle");
  if (n_gen < 0) return fail(GMPEA_EINVAL, "gmpea_step: n_gen < 0");
  return enqueue(h, n_gen);
}

gmpea_status gmpea_run(gmpea_t h, int32_t max_gen, double time_limit_s, int32_t *gens_done) {
  Trace trace("gmpea_run");
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_run: invalid handle");
  if (max_gen < 0) return fail(GMPEA_EINVAL, "gmpea_run: max_gen < 0");
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto elapsed = [&] { return std::chrono::duration<double>(clk::now() - t0).count(); };
  int32_t done = 0;
  gmpea_status s = GMPEA_OK;
  if (!(time_limit_s > 0.0)) {
    s = enqueue(h, max_gen);
    if (s == GMPEA_OK) s = sync(h, "gmpea_run");
    if (s == GMPEA_OK) done = max_gen;
  } else {
    // chunks sized from the measured time per generation so that each chunk is
    // expected to end before half of the remaining time has passed
    int32_t chunk = 1;
    while (done < max_gen && s == GMPEA_OK) {
      const double now = elapsed();
      if (now >= time_limit_s) break;
      const int32_t c = std::min(chunk, max_gen - done);
      const double c0 = elapsed();
      s = enqueue(h, c);
      if (s == GMPEA_OK) s = sync(h, "gmpea_run");
      if (s != GMPEA_OK) break;
      done += c;
      const double per = std::max(1e-7, (elapsed() - c0) / c);
      const double left = time_limit_s - elapsed();
      chunk = static_cast<int32_t>(std::clamp(left / per * 0.5, 1.0, 4096.0));
    }
  }
  if (gens_done) *gens_done = done;
  return s;
}

gmpea_status gmpea_front(gmpea_t h, int32_t what, int32_t capacity, float *x, float *f, float *cv,
                         int32_t *idx, int32_t *count) {
  Trace trace("gmpea_front");
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_front: invalid handle");
  if (!count) return fail(GMPEA_EINVAL, "gmpea_front: count is NULL");
  if (what != GMPEA_FRONT_FEASIBLE_ND && what != GMPEA_FRONT_POP1 && what != GMPEA_FRONT_POP2)
    return fail(GMPEA_EINVAL, "gmpea_front: unknown selector");
  if (capacity < 0) return fail(GMPEA_EINVAL, "gmpea_front: negative capacity");
  return front_impl(h, handle_bufs(h), what, capacity, x, f, cv, idx, count, "gmpea_front");
}

gmpea_status gmpea_front_static(gmpea_t h, int32_t what, int32_t capacity, float *x, float *f,
                                float *cv, int32_t *idx, int32_t *count) {
  Trace trace("gmpea_front_static");
  const char *who = "gmpea_front_static";
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_front_static: invalid handle");
  if (!count) return fail(GMPEA_EINVAL, "gmpea_front_static: count is NULL");
  if (what != GMPEA_FRONT_FEASIBLE_ND && what != GMPEA_FRONT_POP1 && what != GMPEA_FRONT_POP2)
    return fail(GMPEA_EINVAL, "gmpea_front_static: unknown selector");
  if (capacity < 0) return fail(GMPEA_EINVAL, "gmpea_front_static: negative capacity");
  const DevState &st = h->st;
  // flags, row list and records for every row, then decision vectors in passes
  // of as many rows as the rest of the scratch holds
  Carve fixed;
  fixed.take<uint8_t>(static_cast<size_t>(st.n));
  fixed.take<int32_t>(static_cast<size_t>(st.n));
  fixed.take<float4>(static_cast<size_t>(st.n) * st.rq);
  const size_t xoff = (fixed.off + 255) & ~static_cast<size_t>(255);
  const size_t row_bytes = static_cast<size_t>(st.d) * sizeof(float);
  if (xoff + row_bytes > kStaticScratchBytes)
    return fail(GMPEA_EUNSUPPORTED,
                "gmpea_front_static: population of " + std::to_string(st.n) + " rows needs " +
                    std::to_string(xoff + row_bytes) + " bytes of scratch, above the fixed " +
                    std::to_string(kStaticScratchBytes) + " (n (5 + 16 rq) + 4 d bytes, 256-aligned parts)");
  unsigned char *base = nullptr;
  gmpea_status s = static_scratch(h->device, &base, who);
  if (s != GMPEA_OK) return s;
  Carve c;
  c.base = reinterpret_cast<char *>(base);
  FrontBufs b{};
  b.keep = c.take<uint8_t>(static_cast<size_t>(st.n));
  b.idx = c.take<int32_t>(static_cast<size_t>(st.n));
  b.fc = c.take<float4>(static_cast<size_t>(st.n) * st.rq);
  b.x = reinterpret_cast<float *>(base + xoff);
  b.x_rows = static_cast<int32_t>(
      std::min<size_t>(static_cast<size_t>(st.n), (kStaticScratchBytes - xoff) / row_bytes));
  return front_impl(h, b, what, capacity, x, f, cv, idx, count, who);
}

gmpea_status gmpea_get_info(gmpea_t h, gmpea_info *info) {
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_get_info: invalid handle");
  if (!info) return fail(GMPEA_EINVAL, "gmpea_get_info: info is NULL");
  const DevState &st = h->st;
  uint32_t gen = 0, zk[kMaxM];
  unsigned long long rep[2 * kReplLanes];
  std::vector<float4> fc(static_cast<size_t>(st.n) * st.rq);
  gmpea_status s = d2h(h, &gen, st.gen, 1, "gmpea_get_info");
  if (s == GMPEA_OK) s = d2h(h, zk, st.zkey, kMaxM, "gmpea_get_info");
  if (s == GMPEA_OK) s = d2h(h, rep, st.repl, 2 * kReplLanes, "gmpea_get_info");
  if (s == GMPEA_OK) s = d2h(h, fc.data(), st.FC[0], fc.size(), "gmpea_get_info");
  if (s != GMPEA_OK) return s;
  info->n = st.n;
  info->m = st.m;
  info->d = st.d;
  info->t1 = st.t[0];
  info->t2 = st.t[1];
  info->H = h->H;
  info->H2 = h->H2;
  info->generation = gen;
  for (int a = 0; a < GMPEA_MAX_M; ++a) info->z[a] = a < st.m ? key_float(zk[a]) : 0.0f;
  for (int p = 0; p < 2; ++p) {
    unsigned long long tot = 0;
    for (int q = 0; q < kReplLanes; ++q) tot += rep[p * kReplLanes + q];
    info->replaced[p] = static_cast<int64_t>(tot);
  }
  int64_t feas = 0;
  for (int32_t i = 0; i < st.n; ++i) feas += fc[static_cast<size_t>(i) * st.rq + st.rq - 1].w == 0.0f;
  info->feasible_frac = static_cast<double>(feas) / st.n;
  info->device_bytes = h->bytes;
  info->task_dealt = h->st.tasked;
  info->checked_generations = h->checked;
  return GMPEA_OK;
}

gmpea_status gmpea_quality(gmpea_t h, const float *ref, int32_t n_ref, const float *hv_point,
                           int64_t hv_samples, uint64_t hv_seed, double *igd, double *hv,
                           int32_t *front_count) {
  Trace trace("gmpea_quality");
  const char *who = "gmpea_quality";
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_quality: invalid handle");
  if (igd && (!ref || n_ref < 1)) return fail(GMPEA_EINVAL, "gmpea_quality: IGD needs ref and n_ref >= 1");
  if (hv && (!hv_point || hv_samples < 1 || hv_samples > (int64_t(1) << 34)))
    return fail(GMPEA_EINVAL, "gmpea_quality: HV needs hv_point and 1 <= hv_samples <= 2^34");
  const DevState &st = h->st;
  const int32_t m = st.m;
  if (hv)
    for (int32_t k = 0; k < m; ++k)
      if (!std::isfinite(hv_point[k])) return fail(GMPEA_EINVAL, "gmpea_quality: hv_point must be finite");
  const FrontBufs b = handle_bufs(h);
  std::vector<int32_t> rows;
  gmpea_status s = front_rows(h, b, GMPEA_FRONT_FEASIBLE_ND, rows, who);
  if (s != GMPEA_OK) return s;
  const int32_t cnt = static_cast<int32_t>(rows.size());
  if (front_count) *front_count = cnt;
  if (cnt == 0) {  // no feasible row: no point is covered
    if (igd) *igd = std::numeric_limits<double>::infinity();
    if (hv) *hv = 0.0;
    return GMPEA_OK;
  }
  s = front_gather_fc(h, b, 0, rows, who);
  if (s != GMPEA_OK) return s;
  if (igd) {
    // reference points kQualityRefs at a time; the per-block sums are added in
    // block order, the order one launch over every point would give
    double sum = 0.0;
    std::vector<double> part(kQualityRefs / kBlock);
    for (int32_t r0 = 0; r0 < n_ref && s == GMPEA_OK; r0 += kQualityRefs) {
      const int32_t c = std::min(kQualityRefs, n_ref - r0);
      s = h2d(h, h->q_ref, ref + static_cast<size_t>(r0) * m, static_cast<size_t>(c) * m, who);
      if (s != GMPEA_OK) return s;
      int32_t blocks = 0;
      hipError_t e = launch_igd(h->q_ref, c, m, h->f_fc, cnt, st.rq, h->q_part, &blocks, h->stream);
      if (e != hipSuccess) return hip_fail(e, who);
      s = d2h(h, part.data(), h->q_part, static_cast<size_t>(blocks), who);
      for (int32_t q = 0; q < blocks && s == GMPEA_OK; ++q) sum += part[q];
    }
    if (s != GMPEA_OK) return s;
    *igd = sum / n_ref;
  }
  if (hv) {
    // the box from the front's per-objective minimum to the reference point
    // holds every dominated point below the reference point
    std::vector<float> recs(static_cast<size_t>(cnt) * st.rq * 4);
    s = d2h(h, recs.data(), h->f_fc, recs.size(), who);
    if (s != GMPEA_OK) return s;
    float box[2 * kMaxM];
    double vol = 1.0;
    for (int32_t k = 0; k < m; ++k) {
      float lo = recs[k];
      for (int32_t r = 1; r < cnt; ++r) lo = std::min(lo, recs[static_cast<size_t>(r) * st.rq * 4 + k]);
      box[k] = lo;
      box[kMaxM + k] = hv_point[k];
      vol *= std::max(0.0, static_cast<double>(hv_point[k]) - static_cast<double>(lo));
    }
    if (!(vol > 0.0)) {
      *hv = 0.0;
      return GMPEA_OK;
    }
    const unsigned long long zero = 0;
    s = h2d(h, h->q_box, box, 2 * kMaxM, who);
    if (s == GMPEA_OK) s = h2d(h, h->q_hits, &zero, 1, who);
    if (s != GMPEA_OK) return s;
    hipError_t e = launch_hv(hv_samples, m, h->q_box, h->q_box + kMaxM,
                             static_cast<uint32_t>(hv_seed & 0xFFFFFFFFull),
                             static_cast<uint32_t>(hv_seed >> 32), h->f_fc, cnt, st.rq, h->q_hits,
                             h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    unsigned long long hits = 0;
    s = d2h(h, &hits, h->q_hits, 1, who);
    if (s != GMPEA_OK) return s;
    *hv = vol * static_cast<double>(hits) / static_cast<double>(hv_samples);
  }
  return GMPEA_OK;
}

gmpea_status gmpea_shape(gmpea_t h, int32_t *n, int32_t *m, int32_t *d, int32_t *t1, int32_t *t2) {
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_shape: invalid handle");
  const DevState &st = h->st;
  if (n) *n = st.n;
  if (m) *m = st.m;
  if (d) *d = st.d;
  if (t1) *t1 = st.t[0];
  if (t2) *t2 = st.t[1];
  return GMPEA_OK;
}

gmpea_status gmpea_read(gmpea_t h, int32_t buffer, int32_t pop, void *host, int64_t count) {
  Trace trace("gmpea_read");
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_read: invalid handle");
  if (!host) return fail(GMPEA_EINVAL, "gmpea_read: host is NULL");
  if (pop != 0 && pop != 1) return fail(GMPEA_EINVAL, "gmpea_read: pop must be 0 or 1");
  const DevState &st = h->st;
  const int64_t n = st.n, m = st.m, d = st.d;
  auto need = [&](int64_t want) { return count == want; };
  switch (buffer) {
    case GMPEA_BUF_X:
    case GMPEA_BUF_XOFF: {
      if (!need(n * d)) return fail(GMPEA_EINVAL, "gmpea_read: count must be N * d");
      const float *src = st.X[pop];
      hipError_t e = hipSuccess;
      if (buffer == GMPEA_BUF_X) {
        // current rows gathered home first (the values do not change)
        e = launch_materialize(st, h->stream);
      } else {
        // the offspring of the last generation, in the regions of its slot
        uint32_t g = 0;
        gmpea_status s = d2h(h, &g, st.gen, 1, "gmpea_read");
        if (s != GMPEA_OK) return s;
        src = st.rows + static_cast<size_t>(offspring_row(st, gen_slot(st, g), pop, 0)) * st.stride;
      }
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(host, d * sizeof(float), src, st.stride * sizeof(float), d * sizeof(float), n,
                             hipMemcpyDeviceToHost, h->stream);
      if (e != hipSuccess) return hip_fail(e, "gmpea_read");
      return sync(h, "gmpea_read");
    }
    case GMPEA_BUF_F:
    case GMPEA_BUF_CV:
    case GMPEA_BUF_FOFF:
    case GMPEA_BUF_CVOFF: {
      const bool isf = buffer == GMPEA_BUF_F || buffer == GMPEA_BUF_FOFF;
      if (!need(isf ? n * m : n)) return fail(GMPEA_EINVAL, "gmpea_read: wrong count");
      const int64_t rw = int64_t(st.rq) * 4;
      std::vector<float> fc(static_cast<size_t>(n * rw));
      const float4 *src = (buffer == GMPEA_BUF_F || buffer == GMPEA_BUF_CV) ? st.FC[pop] : st.FCO[pop];
      gmpea_status s = d2h(h, fc.data(), src, fc.size(), "gmpea_read");
      if (s != GMPEA_OK) return s;
      float *o = static_cast<float *>(host);
      for (int64_t i = 0; i < n; ++i) {
        if (isf)
          for (int64_t a = 0; a < m; ++a) o[i * m + a] = fc[i * rw + a];
        else
          o[i] = fc[i * rw + rw - 1];
      }
      return GMPEA_OK;
    }
    case GMPEA_BUF_Z: {
      if (!need(m)) return fail(GMPEA_EINVAL, "gmpea_read: count must be m");
      uint32_t zk[kMaxM];
      gmpea_status s = d2h(h, zk, st.zkey, kMaxM, "gmpea_read");
      if (s != GMPEA_OK) return s;
      for (int64_t a = 0; a < m; ++a) static_cast<float *>(host)[a] = key_float(zk[a]);
      return GMPEA_OK;
    }
    case GMPEA_BUF_GEN: {
      if (!need(1)) return fail(GMPEA_EINVAL, "gmpea_read: count must be 1");
      uint32_t g = 0;
      gmpea_status s = d2h(h, &g, st.gen, 1, "gmpea_read");
      if (s == GMPEA_OK) *static_cast<int64_t *>(host) = g;
      return s;
    }
    case GMPEA_BUF_W: {
      if (!need(n * m)) return fail(GMPEA_EINVAL, "gmpea_read: count must be N * m");
      std::vector<int32_t> K;
      std::vector<double> Wd;
      refset(static_cast<int32_t>(m), h->H, h->H2, K, &Wd);
      for (size_t q = 0; q < Wd.size(); ++q) static_cast<float *>(host)[q] = static_cast<float>(Wd[q]);
      return GMPEA_OK;
    }
    case GMPEA_BUF_B: {
      if (!need(n * st.t[pop])) return fail(GMPEA_EINVAL, "gmpea_read: count must be N * t");
      return d2h(h, static_cast<int32_t *>(host), st.B[pop], n * st.t[pop], "gmpea_read");
    }
    case GMPEA_BUF_MATE:
      if (!h->record) return fail(GMPEA_EINVAL, "gmpea_read: MATE needs config.record");
      if (!need(n * 2)) return fail(GMPEA_EINVAL, "gmpea_read: count must be N * 2");
      return d2h(h, static_cast<int32_t *>(host), st.mate[pop], n * 2, "gmpea_read");
    case GMPEA_BUF_WIN:
      if (!h->record) return fail(GMPEA_EINVAL, "gmpea_read: WIN needs config.record");
      if (!need(n)) return fail(GMPEA_EINVAL, "gmpea_read: count must be N");
      return d2h(h, static_cast<int32_t *>(host), st.win[pop], n, "gmpea_read");
    case GMPEA_BUF_OP1: {
      if (!need(n)) return fail(GMPEA_EINVAL, "gmpea_read: count must be N");
      std::vector<uint8_t> sw(n);
      gmpea_status s = d2h(h, sw.data(), st.src, n, "gmpea_read");
      if (s != GMPEA_OK) return s;
      for (int64_t i = 0; i < n; ++i) static_cast<uint8_t *>(host)[i] = (sw[i] >> pop) & 1u;
      return GMPEA_OK;
    }
    default:
      return fail(GMPEA_EINVAL, "gmpea_read: unknown buffer");
  }
}

gmpea_status gmpea_write(gmpea_t h, int32_t buffer, int32_t pop, const void *host, int64_t count) {
  Trace trace("gmpea_write");
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_write: invalid handle");
  if (!host) return fail(GMPEA_EINVAL, "gmpea_write: host is NULL");
  if (pop != 0 && pop != 1) return fail(GMPEA_EINVAL, "gmpea_write: pop must be 0 or 1");
  DevState &st = h->st;
  const int64_t n = st.n, m = st.m, d = st.d;
  switch (buffer) {
    case GMPEA_BUF_X: {
      if (count != n * d) return fail(GMPEA_EINVAL, "gmpea_write: count must be N * d");
      hipError_t e = hipMemcpy2DAsync(st.X[pop], st.stride * sizeof(float), host, d * sizeof(float),
                                      d * sizeof(float), n, hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess) e = launch_loc_home(st, pop, h->stream);
      if (e != hipSuccess) return hip_fail(e, "gmpea_write");
      return sync(h, "gmpea_write");
    }
    case GMPEA_BUF_F:
    case GMPEA_BUF_CV: {
      const bool isf = buffer == GMPEA_BUF_F;
      if (count != (isf ? n * m : n)) return fail(GMPEA_EINVAL, "gmpea_write: wrong count");
      const int64_t rw = int64_t(st.rq) * 4;
      std::vector<float> fc(static_cast<size_t>(n * rw));
      gmpea_status s = d2h(h, fc.data(), st.FC[pop], fc.size(), "gmpea_write");
      if (s != GMPEA_OK) return s;
      const float *in = static_cast<const float *>(host);
      for (int64_t i = 0; i < n; ++i) {
        if (isf)
          for (int64_t a = 0; a < m; ++a) fc[i * rw + a] = in[i * m + a];
        else
          fc[i * rw + rw - 1] = in[i];
      }
      return h2d(h, st.FC[pop], fc.data(), fc.size(), "gmpea_write");
    }
    case GMPEA_BUF_Z: {
      if (count != m) return fail(GMPEA_EINVAL, "gmpea_write: count must be m");
      uint32_t zk[kMaxM];
      for (int a = 0; a < kMaxM; ++a) zk[a] = 0xFFFFFFFFu;
      for (int64_t a = 0; a < m; ++a) zk[a] = float_key(static_cast<const float *>(host)[a]);
      return h2d(h, st.zkey, zk, kMaxM, "gmpea_write");
    }
    case GMPEA_BUF_GEN: {
      if (count != 1) return fail(GMPEA_EINVAL, "gmpea_write: count must be 1");
      const int64_t g = *static_cast<const int64_t *>(host);
      if (g < 0 || g > 0xFFFFFFFFll) return fail(GMPEA_EINVAL, "gmpea_write: generation out of range");
      const uint32_t g32 = static_cast<uint32_t>(g);
      return h2d(h, st.gen, &g32, 1, "gmpea_write");
    }
    default:
      return fail(GMPEA_EINVAL, "gmpea_write: buffer is not writable");
  }
}

void gmpea_destroy(gmpea_t h) {
  if (!valid(h)) return;
  register_live(h, false);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  release_all(h);
  delete h;
}

gmpea_status gmpea_profile(gmpea_t h, int32_t n_gen, float *ms) {
  if (!valid(h)) return fail(GMPEA_ESTATE, "gmpea_profile: invalid handle");
  if (n_gen < 1 || !ms) return fail(GMPEA_EINVAL, "gmpea_profile: need n_gen >= 1 and ms");
  hipEvent_t ev[kPhases + 1];
  int made = 0;
  hipError_t e = hipSuccess;
  for (; made <= kPhases && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
  if (e != hipSuccess) --made;
  double acc[kPhases] = {};
  for (int32_t g = 0; g < n_gen && e == hipSuccess; ++g) {
    e = hipEventRecord(ev[0], h->stream);
    for (int ph = 0; ph < kPhases && e == hipSuccess; ++ph) {
      e = launch_phase(h->st, ph, h->stream);
      if (e == hipSuccess) e = hipEventRecord(ev[ph + 1], h->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[kPhases]);
    for (int ph = 0; ph < kPhases && e == hipSuccess; ++ph) {
      float t = 0.0f;
      e = hipEventElapsedTime(&t, ev[ph], ev[ph + 1]);
      acc[ph] += t;
    }
  }
  // the variation phase again, n_gen launches back to back between two events:
  // repeated, it rewrites the same offspring of the same generation (the
  // generation counter advances only in the next phase), so this times the
  // kernel without one event pair per launch
  float rep = 0.0f;
  if (e == hipSuccess) e = hipEventRecord(ev[0], h->stream);
  for (int32_t g = 0; g < n_gen && e == hipSuccess; ++g) e = launch_phase(h->st, 0, h->stream);
  if (e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&rep, ev[0], ev[1]);
  for (int q = 0; q < made; ++q) (void)hipEventDestroy(ev[q]);
  if (e != hipSuccess) return hip_fail(e, "gmpea_profile");
  // profiled generations (and the repeated variation) are not verified: the
  // write-set counts start again from zero
  if (h->st.wcheck) {
    e = hipMemsetAsync(h->st.wcheck, 0, 8 * static_cast<size_t>(h->st.n) * sizeof(int32_t), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "gmpea_profile");
  }
  for (int ph = 0; ph < kPhases; ++ph) ms[ph] = static_cast<float>(acc[ph] / n_gen);
  ms[kPhases] = rep / static_cast<float>(n_gen);
  return GMPEA_OK;
}

gmpea_status gmpea_copy(const void *src, void *dst, size_t bytes, void *hip_stream) {
  if (bytes % 16 != 0 || (bytes > 0 && (!src || !dst)) ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(GMPEA_EINVAL, "gmpea_copy: need 16-byte aligned pointers and size");
  gmpea_status st = check_runtime("gmpea_copy");
  if (st != GMPEA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = launch_copy(src, dst, static_cast<int64_t>(bytes / 16), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmpea_copy");
  return GMPEA_OK;
}

gmpea_status gmpea_copy_probe(const void *src, void *dst, size_t bytes, int32_t mode,
                              int32_t reps, void *hip_stream, float *ms) {
  if (bytes % 16 != 0 || bytes == 0 || !src || !dst || !ms || reps < 1 ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(GMPEA_EINVAL, "gmpea_copy_probe: need 16-byte aligned pointers and size, reps >= 1");
  if (mode < GMPEA_COPY_STRIDED || mode > GMPEA_COPY_RUNTIME)
    return fail(GMPEA_EINVAL, "gmpea_copy_probe: unknown mode");
  gmpea_status st = check_runtime("gmpea_copy_probe");
  if (st != GMPEA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t n16 = static_cast<int64_t>(bytes / 16);
  auto one = [&]() -> hipError_t {
    switch (mode) {
      case GMPEA_COPY_STRIDED: return launch_copy(src, dst, n16, s);
      case GMPEA_COPY_WIDE: return launch_copy4(src, dst, n16, false, s);
      case GMPEA_COPY_WIDE_NT: return launch_copy4(src, dst, n16, true, s);
      default: return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
    }
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = one();  // warm-up
  float best = 0.0f;
  for (int32_t r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = one();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess && (r == 0 || t < best)) best = t;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "gmpea_copy_probe");
  *ms = best;
  return GMPEA_OK;
}

gmpea_status gmpea_philox(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out,
                          void *hip_stream) {
  if (n < 0 || (n > 0 && (!ctr || !out))) return fail(GMPEA_EINVAL, "gmpea_philox: bad arguments");
  gmpea_status st = check_runtime("gmpea_philox");
  if (st != GMPEA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = launch_philox(ctr, n, static_cast<uint32_t>(seed & 0xFFFFFFFFull),
                               static_cast<uint32_t>(seed >> 32), out, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmpea_philox");
  return GMPEA_OK;
}

}  // extern "C"

// ============================================================================
// Pools: many resident instances advanced together (batched generations).
// ============================================================================
#include <unordered_map>

// Device memory of a pool: chunks reserved from hipMalloc (or the caller's
// allocator) and carved first-fit into 256-byte aligned blocks, with freed
// blocks merged with free neighbours. Chunks stay reserved until the pool is
// destroyed, so admitting and releasing instances costs no runtime allocation
// once the pool has grown. The budget bounds the bytes reserved.
struct PoolArena {
  struct Chunk {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;  // offset -> length, non-adjacent
  };
  std::vector<Chunk> chunks;
  std::unordered_map<void *, std::pair<size_t, size_t>> live;  // ptr -> (chunk, length)
  size_t reserved = 0, used = 0;
  static constexpr size_t kChunk = size_t(256) << 20;
};

constexpr int kWorkClasses = 4;
constexpr int kSchedules = 2;

struct gmpea_pool_s {
  gmpea_allocator user{};
  bool user_hook = false;
  gmpea_allocator hook{};  // arena-backed hook handed to every instance
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t init_stream = nullptr;  // admissions initialise here, beside generations in flight
  size_t budget = 0;
  PoolArena arena;
  std::vector<gmpea_t> slots;  // nullptr = free
  // device tables
  DevState *d_states = nullptr;
  int32_t state_cap = 0;
  // work lists per schedule, class (see in_class) and phase; both schedules'
  // lists are on the device, so the tuner switches schedule without a wait
  int2 *d_work[kSchedules][kWorkClasses][kPhases] = {};
  int32_t work_cap[kSchedules][kWorkClasses][kPhases] = {};
  int32_t nwork[kSchedules][kWorkClasses][kPhases] = {};
  bool dirty = true;
  // launch policy (the autotuner may change both; results do not depend on them)
  int32_t schedule = 0;  // 0: instance blocks grouped per XCD, 1: linear
  int32_t chunk = 16;    // generations per graph replay
  // graphs of `chunk` generations per (schedule, chunk), until the next rebuild
  struct Graph {
    int32_t schedule, chunk;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  // pinned staging of the state array and work lists: their uploads are then
  // asynchronous, and the stream is idle whenever a rebuild refills it
  char *stage = nullptr;
  size_t stage_cap = 0;
};

namespace {

std::mutex g_pool_mu;
std::unordered_set<const gmpea_pool_s *> g_pools;

bool pool_valid(gmpea_pool_t q) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  return q != nullptr && g_pools.count(q) != 0;
}

void *pool_chunk_alloc(gmpea_pool_s *q, size_t bytes) {
  void *p = nullptr;
  if (q->user_hook) {
    p = q->user.alloc(bytes, q->user.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  return p;
}

void pool_chunk_free(gmpea_pool_s *q, void *p) {
  if (q->user_hook)
    q->user.free(p, q->user.ctx);
  else
    (void)hipFree(p);
}

void *arena_take(gmpea_pool_s *q, size_t c, size_t bytes) {
  PoolArena::Chunk &ch = q->arena.chunks[c];
  for (auto it = ch.free.begin(); it != ch.free.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, len = it->second;
    ch.free.erase(it);
    if (len > bytes) ch.free.emplace(off + bytes, len - bytes);
    void *p = ch.base + off;
    q->arena.live.emplace(p, std::make_pair(c, bytes));
    q->arena.used += bytes;
    return p;
  }
  return nullptr;
}

void *pool_raw_alloc(gmpea_pool_s *q, size_t bytes) {
  PoolArena &A = q->arena;
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~static_cast<size_t>(255);
  for (size_t c = 0; c < A.chunks.size(); ++c)
    if (void *p = arena_take(q, c, bytes)) return p;
  if (A.reserved + bytes > q->budget) return nullptr;
  const size_t size = std::max(bytes, std::min(PoolArena::kChunk, q->budget - A.reserved));
  void *base = pool_chunk_alloc(q, size);
  if (!base) return nullptr;
  PoolArena::Chunk ch;
  ch.base = static_cast<char *>(base);
  ch.size = size;
  ch.free.emplace(0, size);
  A.chunks.push_back(std::move(ch));
  A.reserved += size;
  return arena_take(q, A.chunks.size() - 1, bytes);
}

void pool_raw_free(gmpea_pool_s *q, void *p) {
  PoolArena &A = q->arena;
  auto it = A.live.find(p);
  if (it == A.live.end()) return;
  const size_t c = it->second.first, len = it->second.second;
  A.live.erase(it);
  A.used -= len;
  PoolArena::Chunk &ch = A.chunks[c];
  size_t off = static_cast<size_t>(static_cast<char *>(p) - ch.base), n = len;
  auto next = ch.free.lower_bound(off);
  if (next != ch.free.end() && off + n == next->first) {  // merge with the following block
    n += next->second;
    next = ch.free.erase(next);
  }
  if (next != ch.free.begin()) {  // merge with the preceding block
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      off = prev->first;
      n += prev->second;
      ch.free.erase(prev);
    }
  }
  ch.free.emplace(off, n);
}

void pool_arena_destroy(gmpea_pool_s *q) {
  for (auto &ch : q->arena.chunks) pool_chunk_free(q, ch.base);
  q->arena = PoolArena();
}

// Allocator hook of the pool's instances: blocks of the pool's arena (NULL when
// the budget cannot hold the request).
void *pool_hook_alloc(size_t bytes, void *ctx) {
  return pool_raw_alloc(static_cast<gmpea_pool_s *>(ctx), bytes);
}

void pool_hook_free(void *p, void *ctx) { pool_raw_free(static_cast<gmpea_pool_s *>(ctx), p); }

template <class T>
gmpea_status pool_table(gmpea_pool_s *q, T **ptr, int32_t *cap, int32_t need) {
  if (need <= *cap) return GMPEA_OK;
  int32_t ncap = std::max(need, 2 * *cap);
  void *p = pool_raw_alloc(q, sizeof(T) * static_cast<size_t>(ncap));
  if (!p) return fail(GMPEA_ENOMEM, "pool: table allocation failed");
  if (*ptr) pool_raw_free(q, *ptr);
  *ptr = static_cast<T *>(p);
  *cap = ncap;
  return GMPEA_OK;
}

int32_t phase_blocks(const DevState &st, int phase) {
  if (phase == 0) return vary_grid(st);
  if (phase == 1) return st.nblk;
  return st.sel_blocks0 + st.sel_blocks1;
}

// Work list of one phase. Schedule 0 keeps each instance's consecutive OP1 and
// selection blocks on one XCD (instances placed largest first on the
// least-loaded XCD, large ones split into contiguous runs) so neighbouring
// subproblems share an L2; the hardware deals block b to XCD b mod 8, hence
// the interleaving at the end. Its variation blocks go in plain order (the
// variation is bound by VALU issue, and measured about 1 % faster so), as do
// every phase's blocks under schedule 1.
// Work-list classes of a pool: bit 0 records of m > 3 (kernels of their own);
// bit 1 the task-dealt variation in phase 0, and m = 2 in the selection phase
// (a selection kernel per m for m <= 3). OP1 splits at m > 3 only.
bool in_class(const DevState &st, int phase, int cls) {
  const int wide = st.m > 3 ? 1 : 0, tasked = st.tasked ? 1 : 0;
  if (phase == 0) return cls == (wide | (tasked << 1));
  if (phase == 2) return cls == (wide | (!wide && st.m == 2 ? 2 : 0));
  return cls == wide;
}

void build_work(const gmpea_pool_s *q, int phase, int schedule, int cls, std::vector<int2> &out) {
  out.clear();
  std::vector<std::pair<int32_t, int32_t>> inst;  // (blocks, slot)
  int64_t total = 0;
  for (int32_t s = 0; s < static_cast<int32_t>(q->slots.size()); ++s)
    if (q->slots[s] && in_class(q->slots[s]->st, phase, cls)) {
      inst.emplace_back(phase_blocks(q->slots[s]->st, phase), s);
      total += inst.back().first;
    }
  if (schedule == 1 || phase == 0) {
    for (auto &e : inst)
      for (int32_t b = 0; b < e.first; ++b) out.push_back(make_int2(e.second, b));
    return;
  }
  constexpr int kX = 8;
  std::vector<std::vector<int2>> lane(kX);
  std::vector<int64_t> load(kX, 0);
  const int64_t share = (total + kX - 1) / kX;
  std::sort(inst.begin(), inst.end(), [](const std::pair<int32_t, int32_t> &a,
                                         const std::pair<int32_t, int32_t> &b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  });
  for (auto &e : inst) {
    int32_t b = 0;
    while (b < e.first) {
      const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      const int64_t room = std::max<int64_t>(share - load[x], 1);
      const int32_t take = static_cast<int32_t>(std::min<int64_t>(e.first - b, room));
      for (int32_t k = 0; k < take; ++k) lane[x].push_back(make_int2(e.second, b + k));
      load[x] += take;
      b += take;
    }
  }
  size_t len = 0;
  for (auto &l : lane) len = std::max(len, l.size());
  for (size_t j = 0; j < len; ++j)
    for (int x = 0; x < kX; ++x) out.push_back(j < lane[x].size() ? lane[x][j] : make_int2(-1, -1));
}

void pool_drop_graphs(gmpea_pool_s *q) {
  for (auto &g : q->graphs) (void)hipGraphExecDestroy(g.exec);
  q->graphs.clear();
}

gmpea_status pool_rebuild(gmpea_pool_s *q) {
  if (!q->dirty) return GMPEA_OK;
  Trace trace("pool_rebuild");
  pool_drop_graphs(q);
  gmpea_status s = sync_stream(q->stream, "pool");
  if (s != GMPEA_OK) return s;
  const int32_t ns = static_cast<int32_t>(q->slots.size());
  s = pool_table(q, &q->d_states, &q->state_cap, std::max(ns, 1));
  if (s != GMPEA_OK) return s;
  const size_t nst = static_cast<size_t>(std::max(ns, 1));
  std::vector<int2> w[kSchedules][kWorkClasses][kPhases];
  size_t bytes = sizeof(DevState) * nst;
  for (int sc = 0; sc < kSchedules; ++sc)
    for (int c = 0; c < kWorkClasses; ++c)
      for (int ph = 0; ph < kPhases; ++ph) {
        std::vector<int2> &l = w[sc][c][ph];
        build_work(q, ph, sc, c, l);
        s = pool_table(q, &q->d_work[sc][c][ph], &q->work_cap[sc][c][ph],
                       std::max<int32_t>(1, static_cast<int32_t>(l.size())));
        if (s != GMPEA_OK) return s;
        q->nwork[sc][c][ph] = static_cast<int32_t>(l.size());
        bytes += sizeof(int2) * l.size();
      }
  if (bytes > q->stage_cap) {  // the stream is idle (synchronised above)
    const size_t cap = std::max(bytes, 2 * q->stage_cap) + (size_t(1) << 16);
    if (q->stage) (void)hipHostFree(q->stage);
    q->stage = nullptr;
    q->stage_cap = 0;
    if (hipHostMalloc(reinterpret_cast<void **>(&q->stage), cap, hipHostMallocDefault) != hipSuccess) {
      q->stage = nullptr;
      return fail(GMPEA_ENOMEM, "pool rebuild: pinned staging");
    }
    q->stage_cap = cap;
  }
  // stage everything, then upload in stream order ahead of the next generations
  size_t off = sizeof(DevState) * nst;
  DevState *hs = reinterpret_cast<DevState *>(q->stage);
  for (size_t k = 0; k < nst; ++k) hs[k] = (static_cast<int32_t>(k) < ns && q->slots[k]) ? q->slots[k]->st : DevState{};
  hipError_t e = hipMemcpyAsync(q->d_states, hs, sizeof(DevState) * nst, hipMemcpyHostToDevice, q->stream);
  for (int sc = 0; sc < kSchedules; ++sc)
    for (int c = 0; c < kWorkClasses; ++c)
      for (int ph = 0; ph < kPhases && e == hipSuccess; ++ph) {
        const std::vector<int2> &l = w[sc][c][ph];
        if (l.empty()) continue;
        std::memcpy(q->stage + off, l.data(), sizeof(int2) * l.size());
        e = hipMemcpyAsync(q->d_work[sc][c][ph], q->stage + off, sizeof(int2) * l.size(), hipMemcpyHostToDevice,
                           q->stream);
        off += sizeof(int2) * l.size();
      }
  if (e != hipSuccess) return hip_fail(e, "pool rebuild");
  q->dirty = false;
  return GMPEA_OK;
}

hipError_t pool_generation(const gmpea_pool_s *q, hipStream_t s) {
  const int sc = q->schedule;
  for (int ph = 0; ph < kPhases; ++ph) {
    for (int c = 0; c < kWorkClasses; ++c) {
      hipError_t e = launch_batch_phase(q->d_states, q->d_work[sc][c][ph], q->nwork[sc][c][ph], ph,
                                        (c & 1) != 0, (c & 2) != 0, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

gmpea_status pool_enqueue(gmpea_pool_s *q, int32_t n) {
  gmpea_status s = pool_rebuild(q);
  if (s != GMPEA_OK) return s;
  if (q->nwork[q->schedule][0][1] + q->nwork[q->schedule][1][1] == 0)
    return GMPEA_OK;  // no instance (OP1 lists hold them all)
  const int32_t G = q->chunk;
  if (G >= 2 && n >= G) {
    hipGraphExec_t exec = nullptr;
    for (const auto &g : q->graphs)
      if (g.schedule == q->schedule && g.chunk == G) exec = g.exec;
    if (!exec) {
      Trace trace("pool_graph_capture");
      hipStream_t cap;
      hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "pool graph stream");
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        for (int32_t g = 0; g < G && e == hipSuccess; ++g) e = pool_generation(q, cap);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
      }
      (void)hipStreamDestroy(cap);
      if (e != hipSuccess) return hip_fail(e, "pool graph capture");
      q->graphs.push_back({q->schedule, G, exec});
    }
    while (n >= G) {
      hipError_t e = hipGraphLaunch(exec, q->stream);
      if (e != hipSuccess) return hip_fail(e, "pool graph launch");
      n -= G;
    }
  }
  for (int32_t g = 0; g < n; ++g) {
    hipError_t e = pool_generation(q, q->stream);
    if (e != hipSuccess) return hip_fail(e, "pool generation launch");
  }
  return GMPEA_OK;
}

}  // namespace

extern "C" {

gmpea_status gmpea_lattice(int32_t m, int32_t n_req, int32_t t, int32_t cap_rows, int32_t *K,
                           int32_t *B, int32_t *H_out, int32_t *n_out) {
  if (m < 2 || m > GMPEA_MAX_M) return fail(GMPEA_EINVAL, "gmpea_lattice: m out of range");
  if (n_req < 2 || n_req > (1 << 26)) return fail(GMPEA_EINVAL, "gmpea_lattice: n_req out of range");
  const int32_t H = dd_divisions(m, n_req);
  const int64_t n = dd_count(m, H);
  if (n > (int64_t(1) << 27)) return fail(GMPEA_EUNSUPPORTED, "gmpea_lattice: lattice too large");
  if (t < 1 || t > n) return fail(GMPEA_EINVAL, "gmpea_lattice: t must lie in [1, N]");
  if (H_out) *H_out = H;
  if (n_out) *n_out = static_cast<int32_t>(n);
  if (!K && !B) return GMPEA_OK;
  if (cap_rows < n) return fail(GMPEA_ECAPACITY, "gmpea_lattice: cap_rows below N");
  try {
    std::vector<int32_t> KK, BB;
    dd_lattice(m, H, KK);
    if (K) std::memcpy(K, KK.data(), KK.size() * sizeof(int32_t));
    if (B) {
      refset_neighbours(KK, m, H, 0, t, BB);
      std::memcpy(B, BB.data(), BB.size() * sizeof(int32_t));
    }
  } catch (const std::bad_alloc &) {
    return fail(GMPEA_ENOMEM, "gmpea_lattice: host memory");
  }
  return GMPEA_OK;
}

gmpea_status gmpea_reference_set(int32_t m, int32_t h_outer, int32_t h_inner, int32_t t,
                                 int32_t cap_rows, int32_t *K, int32_t *B, int32_t *n_out) {
  if (m < 2 || m > GMPEA_MAX_M) return fail(GMPEA_EINVAL, "gmpea_reference_set: m out of range");
  if (h_outer < 1 || h_inner < 0 || h_outer > 4096 || h_inner > 4096)
    return fail(GMPEA_EINVAL, "gmpea_reference_set: layer divisions out of range");
  const int64_t n = refset_count(m, h_outer, h_inner);
  if (n > (int64_t(1) << 27)) return fail(GMPEA_EUNSUPPORTED, "gmpea_reference_set: set too large");
  if (t < 1 || t > n) return fail(GMPEA_EINVAL, "gmpea_reference_set: t must lie in [1, N]");
  if (n_out) *n_out = static_cast<int32_t>(n);
  if (!K && !B) return GMPEA_OK;
  if (cap_rows < n) return fail(GMPEA_ECAPACITY, "gmpea_reference_set: cap_rows below N");
  try {
    std::vector<int32_t> KK, BB;
    refset(m, h_outer, h_inner, KK, nullptr);
    if (K) std::memcpy(K, KK.data(), KK.size() * sizeof(int32_t));
    if (B) {
      refset_neighbours(KK, m, h_outer, h_inner, t, BB);
      std::memcpy(B, BB.data(), BB.size() * sizeof(int32_t));
    }
  } catch (const std::bad_alloc &) {
    return fail(GMPEA_ENOMEM, "gmpea_reference_set: host memory");
  }
  return GMPEA_OK;
}

gmpea_status gmpea_pool_create(size_t budget_bytes, const gmpea_allocator *A, void *hip_stream,
                               gmpea_pool_t *out) {
  if (!out) return fail(GMPEA_EINVAL, "gmpea_pool_create: out is NULL");
  if (A && (!A->alloc || !A->free)) return fail(GMPEA_EINVAL, "gmpea_pool_create: incomplete allocator");
  gmpea_status s = check_runtime("gmpea_pool_create");
  if (s != GMPEA_OK) return s;
  gmpea_pool_s *q = new gmpea_pool_s();
  if (A) {
    q->user = *A;
    q->user_hook = true;
  }
  q->hook.alloc = pool_hook_alloc;
  q->hook.free = pool_hook_free;
  q->hook.ctx = q;
  q->budget = budget_bytes;
  if (const char *g = std::getenv("GMPEA_GRAPH_CHUNK")) q->chunk = std::atoi(g);
  if (hip_stream) {
    q->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete q;
      return hip_fail(e, "gmpea_pool_create: stream");
    }
    q->own_stream = true;
  }
  {
    hipError_t e = hipStreamCreateWithFlags(&q->init_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      if (q->own_stream) (void)hipStreamDestroy(q->stream);
      delete q;
      return hip_fail(e, "gmpea_pool_create: stream");
    }
  }
  // Pinned staging for the work-list uploads, and one upload from it now: the
  // first large host-to-device copy in a process took about 7 ms of set-up
  // (measured; copies after it took microseconds), which belongs to the
  // pool's creation rather than to its first batched generations. A failure
  // here only leaves the staging to the first rebuild.
  {
    constexpr size_t kStage = size_t(4) << 20;
    if (hipHostMalloc(reinterpret_cast<void **>(&q->stage), kStage, hipHostMallocDefault) == hipSuccess) {
      q->stage_cap = kStage;
      std::memset(q->stage, 0, kStage);
      if (void *d = pool_chunk_alloc(q, kStage)) {
        if (hipMemcpyAsync(d, q->stage, kStage, hipMemcpyHostToDevice, q->stream) == hipSuccess)
          (void)hipStreamSynchronize(q->stream);
        pool_chunk_free(q, d);
      }
    } else {
      q->stage = nullptr;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pools.insert(q);
  }
  *out = q;
  return GMPEA_OK;
}

gmpea_status gmpea_pool_admit(gmpea_pool_t q, const gmpea_problem *P, const gmpea_config *C,
                              int32_t *slot) {
  Trace trace("gmpea_pool_admit");
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_admit: invalid pool");
  if (!slot) return fail(GMPEA_EINVAL, "gmpea_pool_admit: slot is NULL");
  gmpea_t h = nullptr;
  // initialise on the pool's side stream: the generations enqueued on the pool
  // stream keep running meanwhile (the new instance's memory is fresh: freed
  // blocks are recycled only after the pool's work on them has finished), and
  // gmpea_init returns once its own work is done
  gmpea_status s = gmpea_init(P, C, &q->hook, q->init_stream, &h);
  if (s == GMPEA_ENOMEM)
    return fail(GMPEA_ENOMEM, "gmpea_pool_admit: the instance does not fit the pool's budget");
  if (s != GMPEA_OK) return s;
  h->stream = q->stream;  // every later operation runs in order with the pool's generations
  h->st.task_off = task_off_for(h->st.n, h->st.nq, h->st.m > 3, true);  // same results, see task_off_for
  h->st.wcheck = nullptr;     // the write-set check verifies plain generations only
  int32_t k = 0;
  while (k < static_cast<int32_t>(q->slots.size()) && q->slots[k]) ++k;
  if (k == static_cast<int32_t>(q->slots.size())) q->slots.push_back(nullptr);
  q->slots[k] = h;
  q->dirty = true;
  *slot = k;
  return GMPEA_OK;
}

gmpea_status gmpea_pool_step(gmpea_pool_t q, int32_t n_gen) {
  Trace trace("gmpea_pool_step");
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_step: invalid pool");
  if (n_gen < 0) return fail(GMPEA_EINVAL, "gmpea_pool_step: n_gen < 0");
  return pool_enqueue(q, n_gen);
}

gmpea_status gmpea_pool_tune(gmpea_pool_t q, int32_t n_gen, int32_t *gens_done) {
  Trace trace("gmpea_pool_tune");
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_tune: invalid pool");
  if (n_gen < 0) return fail(GMPEA_EINVAL, "gmpea_pool_tune: n_gen < 0");
  // Each candidate (schedule, chunk) runs real generations, timed with events;
  // the fastest per generation is kept. The state advances by the generations
  // run, whatever the choice, and results do not depend on it. The candidates
  // are enqueued back to back and waited for once: both schedules' work lists
  // are on the device and graphs stay cached per (schedule, chunk), so the host
  // builds the next candidate's graph while the device runs the previous ones.
  // (schedule, chunk, generations timed): chunk 0 launches every generation
  // eagerly, without a graph; those come first, so the device starts at once
  constexpr int kCand = 6;
  const int32_t cand[kCand][3] = {{0, 0, 16}, {1, 0, 16}, {0, 16, 16}, {1, 16, 16}, {0, 64, 64}, {1, 64, 64}};
  hipEvent_t ev[2 * kCand] = {};
  gmpea_status s = pool_rebuild(q);
  for (int k = 0; k < 2 * kCand && s == GMPEA_OK; ++k)
    if (hipEventCreate(&ev[k]) != hipSuccess) s = fail(GMPEA_EHIP, "gmpea_pool_tune: event");
  int32_t done = 0, ran = 0;
  const int32_t s0 = q->schedule, c0 = q->chunk;
  for (int c = 0; c < kCand && s == GMPEA_OK; ++c) {
    const int32_t gens = cand[c][2];
    if (done + 2 * gens > n_gen) break;
    q->schedule = cand[c][0];
    q->chunk = cand[c][1];
    s = pool_enqueue(q, gens);  // the first half also builds the graph; time the second half
    if (s != GMPEA_OK) break;
    (void)hipEventRecord(ev[2 * c], q->stream);
    s = pool_enqueue(q, gens);
    (void)hipEventRecord(ev[2 * c + 1], q->stream);
    if (s != GMPEA_OK) break;
    done += 2 * gens;
    ran = c + 1;
  }
  int32_t bs = s0, bc = c0;
  if (s == GMPEA_OK && ran > 0) {
    if (hipEventSynchronize(ev[2 * ran - 1]) != hipSuccess) s = fail(GMPEA_EHIP, "gmpea_pool_tune: wait");
    float best = 1e30f;
    for (int c = 0; c < ran && s == GMPEA_OK; ++c) {
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]);
      if (ms / cand[c][2] < best) {
        best = ms / cand[c][2];
        bs = cand[c][0];
        bc = cand[c][1];
      }
    }
  }
  for (int k = 0; k < 2 * kCand; ++k)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  q->schedule = bs;
  q->chunk = bc;
  if (s == GMPEA_OK && done < n_gen) {
    s = pool_enqueue(q, n_gen - done);
    if (s == GMPEA_OK) done = n_gen;
  }
  if (gens_done) *gens_done = done;
  return s;
}

gmpea_status gmpea_pool_handle(gmpea_pool_t q, int32_t slot, gmpea_t *h) {
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_handle: invalid pool");
  if (!h || slot < 0 || slot >= static_cast<int32_t>(q->slots.size()) || !q->slots[slot])
    return fail(GMPEA_EINVAL, "gmpea_pool_handle: no such slot");
  *h = q->slots[slot];
  return GMPEA_OK;
}

gmpea_status gmpea_pool_release(gmpea_pool_t q, int32_t slot) {
  Trace trace("gmpea_pool_release");
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_release: invalid pool");
  if (slot < 0 || slot >= static_cast<int32_t>(q->slots.size()) || !q->slots[slot])
    return fail(GMPEA_EINVAL, "gmpea_pool_release: no such slot");
  gmpea_destroy(q->slots[slot]);
  q->slots[slot] = nullptr;
  q->dirty = true;
  return GMPEA_OK;
}

gmpea_status gmpea_pool_query(gmpea_pool_t q, int32_t *active, size_t *used_bytes,
                              size_t *budget_bytes, int32_t *schedule, int32_t *chunk) {
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_query: invalid pool");
  int32_t n = 0;
  for (auto *h : q->slots) n += h != nullptr;
  if (active) *active = n;
  if (used_bytes) *used_bytes = q->arena.used;
  if (budget_bytes) *budget_bytes = q->budget;
  if (schedule) *schedule = q->schedule;
  if (chunk) *chunk = q->chunk;
  return GMPEA_OK;
}

gmpea_status gmpea_pool_sync(gmpea_pool_t q) {
  if (!pool_valid(q)) return fail(GMPEA_ESTATE, "gmpea_pool_sync: invalid pool");
  return sync_stream(q->stream, "gmpea_pool_sync");
}

void gmpea_pool_destroy(gmpea_pool_t q) {
  if (!pool_valid(q)) return;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pools.erase(q);
  }
  (void)hipStreamSynchronize(q->stream);
  for (auto &h : q->slots)
    if (h) gmpea_destroy(h);
  pool_drop_graphs(q);
  if (q->stage) (void)hipHostFree(q->stage);
  if (q->d_states) pool_raw_free(q, q->d_states);
  for (int sc = 0; sc < kSchedules; ++sc)
    for (int ph = 0; ph < kPhases; ++ph)
      for (int c = 0; c < kWorkClasses; ++c)
        if (q->d_work[sc][c][ph]) pool_raw_free(q, q->d_work[sc][c][ph]);
  pool_arena_destroy(q);
  if (q->init_stream) (void)hipStreamDestroy(q->init_stream);
  if (q->own_stream) (void)hipStreamDestroy(q->stream);
  delete q;
}

}  // extern "C"
