// GMPEA generation kernels for gfx950 (CDNA4, wave64).
//
// One generation (Alg. 1 loop body + Alg. 2) is three launches:
//   k_vary    one lane per offspring (p, i): Philox draws, neighbourhood mating,
//             SBX + polynomial mutation, evaluation of F and CV, and the block's
//             share of the ideal-point minimum (one atomic per block and
//             objective, skipped when it cannot lower z).
//   k_op1     one lane per subproblem i: OP1 offspring cooperation at w_i with
//             the updated ideal point; writes the new offspring's F/CV and the
//             source switch (X is not copied).
//   k_select  a lane group per parent slot (p, j): OP2 + OP3 as a pull over the
//             reverse neighbour list of j (every offspring i with j in B_p(i)),
//             lexicographic minimum of the qualifiers; winners' rows are then
//             copied by the whole block with 16-byte accesses.
// The ideal point is a grid-wide dependency between k_vary and k_op1, and OP1
// must finish for every i before any slot can be decided; kernel boundaries
// provide both.
//
// Layout: X rows are `stride` floats (16-byte aligned), so a row copy is a run
// of float4 moves; F and CV share one float4 per individual.
// Blocks are remapped so that consecutive row tiles run on the same XCD (the
// hardware deals blocks to the 8 XCDs round-robin): neighbouring subproblems
// share parents and candidates, and then share that XCD's L2.
#include <algorithm>

#include "gmpea_internal.hpp"

// Floating-point contraction is off for this file (build flag -ffp-contract=off)
// and every fused multiply-add is written out as fmaf: the compiler may not
// fuse an expression in one kernel and leave it unfused in another, so a device
// function gives bitwise-equal results in the plain and the batched kernels.

namespace gmpea {

// ----------------------------------------------------------------------------
// Counter RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ----------------------------------------------------------------------------
// Each round's two 32 x 32 -> 64-bit products are written as 64-bit multiplies
// so that each becomes one v_mad_u64_u32 (high and low words together).
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    c = make_uint4(static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0, static_cast<uint32_t>(p1),
                   static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1, static_cast<uint32_t>(p0));
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ float u24(uint32_t w) {
  return static_cast<float>(w >> 8) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float keyf(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ float nan_inf(float v) { return (v != v) ? __builtin_huge_valf() : v; }

// Block index -> tile such that each XCD receives a contiguous run of tiles.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  const int x = b & 7, q = G >> 3, r = G & 7;
  return x * q + min(x, r) + (b >> 3);
}

// x^e for x >= 0 with the hardware log2/exp2 (about 1 ulp each). Every base
// used here is either exactly 0 (giving 0 for e > 0) or a normal number; a
// result below the normal range flushes to 0, which no caller can tell apart.
__device__ __forceinline__ float powpos(float x, float e) {
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x));
}

// ----------------------------------------------------------------------------
// Variation of one variable. Bounded polynomial mutation of c in [lo, hi] when
// wB < tpm, then SBX (one child kept; per-variable crossing bit, sign bit,
// 24-bit uniform) or DE (x + F (a - b), every variable) in front of it.
// ----------------------------------------------------------------------------
__device__ __forceinline__ float pm1(float c, uint32_t w, uint64_t T, float invT, float lo, float hi,
                                     float inv_span, const DevState &st) {
  // Called with w < T: u = w / T. Every coefficient of the mutation step (2u,
  // 1 - 2u, 2(1 - u), 2(u - 1/2)) comes from an exact integer numerator over T,
  // and 1 - delta from the distance to the far bound: in FP32, 1 - u itself
  // cancels catastrophically as u -> 1 and val^(1/(eta+1)) magnifies that
  // error. Both halves of the mutation share one pair of powers (selects, no
  // branch).
  float a, b;
  bool low;
  if (T <= 0x80000000ull) {  // every numerator fits 32 bits
    const uint32_t T32 = static_cast<uint32_t>(T);
    low = 2u * w < T32;  // u < 1/2
    a = static_cast<float>(low ? 2u * w : 2u * (T32 - w)) * invT;
    b = static_cast<float>(low ? T32 - 2u * w : 2u * w - T32) * invT;
  } else {
    const uint64_t w64 = w;
    low = 2u * w64 < T;
    a = static_cast<float>(low ? 2u * w64 : 2u * (T - w64)) * invT;
    b = static_cast<float>(low ? T - 2u * w64 : 2u * w64 - T) * invT;
  }
  const float xy = (low ? (hi - c) : (c - lo)) * inv_span;
  const float t = powpos(fmaf(b, powpos(xy, st.pm_p), a), st.pm_e);
  const float dq = low ? t - 1.0f : 1.0f - t;
  return __builtin_amdgcn_fmed3f(fmaf(dq, hi - lo, c), lo, hi);
}

// SBX of one variable (one child kept; crossing bit 0, sign bit 1, 24-bit
// uniform in bits 8..31), clipped to the box.
__device__ __forceinline__ float sbx1(float a, float b, uint32_t wA, float lo, float hi, bool cross,
                                      const DevState &st) {
  float c = a;
  if (cross && (wA & 1u)) {
    const float u = u24(wA);
    const bool low = u <= 0.5f;  // one power for both halves of the spread
    const float beta0 = powpos(low ? 2.0f * u : 2.0f * (1.0f - u), low ? st.sbx_e : -st.sbx_e);
    const float beta = (wA & 2u) ? -beta0 : beta0;
    c = 0.5f * fmaf(beta, a - b, a + b);
  }
  return __builtin_amdgcn_fmed3f(c, lo, hi);
}

// DE mutant of one variable (crossover rate 1), clipped to the box.
__device__ __forceinline__ float de1(float x, float a, float b, float lo, float hi,
                                     const DevState &st) {
  return __builtin_amdgcn_fmed3f(fmaf(st.de_f, a - b, x), lo, hi);
}

// Running sums of the evaluation, filled variable by variable.
struct EvalAcc {
  float s;       // curve: sum x_2..x_d; sphere: sum over non-angle variables of (x - 0.5)^2
  float x0, x1;  // first two variables (angles, f1, equality)
};

template <int M, int FAM>
__device__ __forceinline__ void eval_add(EvalAcc &e, int l, float x) {
  if (l == 0) e.x0 = x;
  if (l == 1) e.x1 = x;
  if (FAM == 0) {
    if (l >= 1) e.s += x;
  } else {
    if (l >= M - 1) e.s = fmaf(x - 0.5f, x - 0.5f, e.s);
  }
}

// F and CV from the sums (Eqs. (1)-(3)); returns (f0, f1, f2, cv).
template <int M, int FAM>
__device__ __forceinline__ float4 eval_finish(const EvalAcc &e, const DevProblem &P) {
  float f[3] = {0.0f, 0.0f, 0.0f};
  if (FAM == 0) {
    const float g = fmaf(P.g_scale, e.s, 1.0f);
    f[0] = e.x0;
    f[1] = g * (1.0f - sqrtf(e.x0 / g));
  } else {
    const float r = 1.0f + e.s;
    float s0, c0;
    sincospif(0.5f * e.x0, &s0, &c0);
    if (M == 2) {
      f[0] = r * c0;
      f[1] = r * s0;
    } else {
      float s1, c1;
      sincospif(0.5f * e.x1, &s1, &c1);
      f[0] = r * c0 * c1;
      f[1] = r * c0 * s1;
      f[2] = r * s0;
    }
  }
  float cv = 0.0f;
  for (int j = 0; j < P.n_ring; ++j) {
    float q = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const float df = f[k] - P.ring_c[j * M + k];
      q = fmaf(df, df, q);
    }
    const float c = P.ring_r2[j] - q;
    cv += (c > 0.0f) ? c : 0.0f;
  }
  if (P.has_sum_lower) {
    float sum = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) sum += f[k];
    const float c = P.sum_lower - sum;
    cv += (c > 0.0f) ? c : 0.0f;
  }
  if (P.n_eq) {
    const float c = fabsf(e.x0 + e.x1 - 1.0f) - P.eq_tol;
    cv += (c > 0.0f) ? c : 0.0f;
  }
  return make_float4(f[0], f[1], f[2], cv);
}

// Block-wide minimum of each objective, then one atomic per objective when the
// block's value can lower the ideal point. NaN never lowers it.
template <int M>
__device__ __forceinline__ void block_zmin(float (&v)[M], uint32_t *zkey) {
  __shared__ float red[M][kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    float x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    if (lane == 0) red[k][wv] = x;
  }
  __syncthreads();
  if (threadIdx.x < M) {
    const int k = threadIdx.x;
    float x = red[k][0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) x = fminf(x, red[k][w]);
    if (x == x) {
      const uint32_t kk = fkey(x);
      if (kk < __atomic_load_n(&zkey[k], __ATOMIC_RELAXED)) atomicMin(&zkey[k], kk);
    }
  }
}

// ----------------------------------------------------------------------------
// Initialisation (Alg. 1): X uniform in the box from the INIT stream,
// evaluation, ideal point.
// ----------------------------------------------------------------------------
template <int M, int FAM>
__global__ __launch_bounds__(kBlock) void k_init(DevState st) {
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int p = L >= st.nblk ? 1 : 0;
  const int i = (L - p * st.nblk) * kBlock + threadIdx.x;
  if (i >= st.n) return;
  float *row = st.X[p] + static_cast<size_t>(i) * st.stride;
  uint4 w = make_uint4(0, 0, 0, 0);
  for (int l = 0; l < st.stride; ++l) {
    float x = 0.0f;
    if (l < st.d) {
      if ((l & 3) == 0)
        w = philox10(make_uint4(l >> 2, i, 0u, (kTagInit << 24) | (p << 16)), st.key0, st.key1);
      const uint32_t word = (l & 3) == 0 ? w.x : (l & 3) == 1 ? w.y : (l & 3) == 2 ? w.z : w.w;
      const float lo = st.prob.lb[l], hi = st.prob.ub[l];
      x = fmaf(hi - lo, u24(word), lo);
    }
    row[l] = x;
  }
}

// Evaluation of a population row by a group of LPO lanes: lane g adds chunks
// g, g + LPO, ... in order, then a butterfly combines the lanes. k_vary adds
// its offspring in exactly this order, so F and CV are a function of x alone:
// an offspring that copies an individual evaluates bitwise equal to it.
template <int M, int FAM, int LPO>
__device__ __forceinline__ EvalAcc eval_row(const DevState &st, const float4 *row, int g, bool live) {
  EvalAcc e{0.0f, 0.0f, 0.0f};
  if (live) {
    const int nq = st.stride >> 2;
    for (int q = g; q < nq; q += LPO) {
      const int l0 = q << 2;
      const float4 o = row[q];
      eval_add<M, FAM>(e, l0, o.x);
      if (l0 + 1 < st.d) eval_add<M, FAM>(e, l0 + 1, o.y);
      if (l0 + 2 < st.d) eval_add<M, FAM>(e, l0 + 2, o.z);
      if (l0 + 3 < st.d) eval_add<M, FAM>(e, l0 + 3, o.w);
    }
  }
  return e;
}

// Group reduction of the sums (every lane of the wave takes part), then F/CV
// and the ideal point's block minimum.
template <int M, int FAM, int LPO>
__device__ __forceinline__ void eval_group(const DevState &st, EvalAcc e, int g, bool live,
                                           float4 *out) {
  float zv[M];
#pragma unroll
  for (int q = 0; q < M; ++q) zv[q] = __builtin_huge_valf();
#pragma unroll
  for (int o = 1; o < LPO; o <<= 1) e.s += __shfl_xor(e.s, o);
  const int base = (threadIdx.x & 63) & ~(LPO - 1);
  e.x0 = __shfl(e.x0, base);
  e.x1 = __shfl(e.x1, base);
  if (live && g == 0) {
    const float4 fc = eval_finish<M, FAM>(e, st.prob);
    *out = fc;
    zv[0] = fc.x;
    if (M > 1) zv[1] = fc.y;
    if (M > 2) zv[M - 1] = fc.z;
  }
  block_zmin<M>(zv, st.zkey);
}

// Initial evaluation (Alg. 1): F, CV and the ideal point of both populations.
template <int M, int FAM, int LPO>
__global__ __launch_bounds__(kBlock) void k_eval(DevState st) {
  constexpr int kPer = kBlock / LPO;
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int half = gridDim.x >> 1;
  const int p = L >= half ? 1 : 0;
  const int g = threadIdx.x & (LPO - 1);
  const int i = (L - p * half) * kPer + threadIdx.x / LPO;
  const bool live = i < st.n;
  const float4 *row = reinterpret_cast<const float4 *>(st.X[p] + static_cast<size_t>(live ? i : 0) * st.stride);
  const EvalAcc e = eval_row<M, FAM, LPO>(st, row, g, live);
  eval_group<M, FAM, LPO>(st, e, g, live, &st.FC[p][live ? i : 0]);
}

// ----------------------------------------------------------------------------
// Initialisation tables (Alg. 1 inputs): reference vectors and neighbourhoods.
// Row i of the Das-Dennis lattice is unranked from its index (lexicographic
// order of the leading coordinates); its neighbours are the first valid points
// k_i + delta along one offset list sorted by (distance, lexicographic order of
// delta), which is the (distance, index) order for every row because the rank
// is increasing in the lexicographic order. The first t1 and the first t2 of
// them are the two neighbourhoods.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int64_t dd_base3(int64_t H, int64_t a) {
  // rank of the first row with k_1 = a when m = 3: C(H + 2, 2) - C(H - a + 2, 2)
  return ((H + 2) * (H + 1) - (H - a + 2) * (H - a + 1)) / 2;
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_tables(int32_t n, int32_t H, const int2 *__restrict__ offs,
                                                  int32_t noffs, int32_t t1, int32_t t2, int32_t agg,
                                                  float4 *__restrict__ W, int32_t *__restrict__ B1,
                                                  int32_t *__restrict__ B2,
                                                  uint32_t *__restrict__ incomplete) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int32_t k[3] = {0, 0, 0};
  if (M == 2) {
    k[0] = i;
    k[1] = H - i;
  } else {
    int32_t lo = 0, hi = H;  // largest a with dd_base3(H, a) <= i
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (dd_base3(H, mid) <= i) lo = mid;
      else hi = mid - 1;
    }
    k[0] = lo;
    k[1] = i - static_cast<int32_t>(dd_base3(H, lo));
    k[2] = H - k[0] - k[1];
  }
  // weights in FP64, rounded once: the unit direction for PBI, the raw weight otherwise
  double w[3] = {0.0, 0.0, 0.0}, nrm = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    w[a] = static_cast<double>(k[a]) / static_cast<double>(H);
    nrm += w[a] * w[a];
  }
  nrm = sqrt(nrm);
  float v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = static_cast<float>(agg == 0 ? w[a] / nrm : w[a]);
  W[i] = make_float4(v[0], v[1], v[2], 0.0f);
  const int32_t tmax = max(t1, t2);
  int32_t c = 0;
  for (int32_t q = 0; q < noffs && c < tmax; ++q) {
    const int2 dl = offs[q];
    const int32_t a0 = k[0] + dl.x;
    int32_t rank;
    if (M == 2) {
      if (a0 < 0 || a0 > H) continue;
      rank = a0;
    } else {
      const int32_t a1 = k[1] + dl.y, a2 = H - a0 - a1;
      if (a0 < 0 || a1 < 0 || a2 < 0 || a0 > H || a1 > H || a2 > H) continue;
      rank = static_cast<int32_t>(dd_base3(H, a0)) + a1;
    }
    if (c < t1) B1[static_cast<size_t>(i) * t1 + c] = rank;
    if (c < t2) B2[static_cast<size_t>(i) * t2 + c] = rank;
    ++c;
  }
  if (c < tmax) atomicOr(incomplete, 1u);
}

// Reverse lists: lengths, the scan of their excess over t, a scatter into the
// padded head and the tail, and a per-list insertion sort (lists hold about t
// entries) so that every list is ascending.
__global__ __launch_bounds__(kBlock) void k_rev_count(int64_t nt, const int32_t *__restrict__ B,
                                                     int32_t *__restrict__ cnt) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q < nt) atomicAdd(&cnt[B[q]], 1);
}

__global__ __launch_bounds__(kBlock) void k_rev_excess(int32_t n, int32_t t, const int32_t *__restrict__ cnt,
                                                      int32_t *__restrict__ toff) {
  const int32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < n) toff[j + 1] = max(cnt[j] - t, 0);
}

constexpr int kScanThreads = 1024;

// In-place inclusive scan of off[0 .. len) by one block.
__global__ __launch_bounds__(kScanThreads) void k_scan(int32_t *off, int32_t len) {
  __shared__ int32_t part[kScanThreads];
  const int tid = threadIdx.x;
  const int per = (len + kScanThreads - 1) / kScanThreads;
  const int lo = min(len, tid * per), hi = min(len, lo + per);
  int32_t sum = 0;
  for (int q = lo; q < hi; ++q) sum += off[q];
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid > 0 ? part[tid - 1] : 0;
  for (int q = lo; q < hi; ++q) {
    run += off[q];
    off[q] = run;
  }
}

__global__ __launch_bounds__(kBlock) void k_rev_fill(int64_t nt, int32_t t, const int32_t *__restrict__ B,
                                                    const int32_t *__restrict__ toff,
                                                    int32_t *__restrict__ cursor,
                                                    int32_t *__restrict__ head,
                                                    int32_t *__restrict__ tail) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= nt) return;
  const int32_t j = B[q];
  const int32_t pos = atomicAdd(&cursor[j], 1);
  const int32_t i = static_cast<int32_t>(q / t);
  if (pos < t)
    head[static_cast<size_t>(j) * t + pos] = i;
  else
    tail[toff[j] + pos - t] = i;
}

__global__ __launch_bounds__(kBlock) void k_rev_sort(int32_t n, int32_t t, const int32_t *__restrict__ toff,
                                                    int32_t *__restrict__ head,
                                                    int32_t *__restrict__ tail) {
  const int32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  int32_t *h = head + static_cast<size_t>(j) * t;
  int32_t *tl = tail + toff[j];
  const int32_t ext = toff[j + 1] - toff[j];
  int32_t len = 0;
  while (len < t && h[len] >= 0) ++len;
  len += ext;
  // element k of the list: head for k < t, tail beyond
  auto at = [&](int32_t k) -> int32_t & { return k < t ? h[k] : tl[k - t]; };
  for (int32_t q = 1; q < len; ++q) {
    const int32_t v = at(q);
    int32_t r = q - 1;
    while (r >= 0 && at(r) > v) {
      at(r + 1) = at(r);
      --r;
    }
    at(r + 1) = v;
  }
}

// ----------------------------------------------------------------------------
// k_vary: reproduction (SBX or DE, then PM) + evaluation + ideal-point update.
// Draws (the paper fixes no RNG; this counter layout is the library's): Philox
// counter (c0, i, k, tag << 24 | p << 16) for offspring i of population p in
// generation k. The MATE block (c0 = 0) gives the two neighbourhood positions
// and the per-offspring crossing draw; VAR block c0 = l >> 1 gives (wA, wB) for
// variables l and l + 1: SBX's bits in wA, the mutation test and uniform in wB.
// A group of LPO consecutive lanes builds one offspring: lane g of the group
// takes the float4 chunks g, g + LPO, ... of the row, so with LPO = 8 the group
// reads each parent row and writes the offspring row as whole 128-byte lines.
// The group shares the mating draw (each lane computes it; the cost is one
// Philox block either way) and reduces the evaluation sums with butterflies.
// ----------------------------------------------------------------------------
template <int M, int FAM, int LPO>
__device__ __forceinline__ void vary_body(const DevState &st, int L, int G) {
  constexpr int kPer = kBlock / LPO;  // offspring per block
  const int half = G >> 1;            // blocks per population
  const int p = L >= half ? 1 : 0;
  const int g = threadIdx.x & (LPO - 1);
  const int i = (L - p * half) * kPer + threadIdx.x / LPO;
  const uint32_t k = *st.gen + 1u;
  const uint32_t tagp = (p << 16);
  const float *Xc = st.X[p];
  const bool live = i < st.n;
  EvalAcc e{0.0f, 0.0f, 0.0f};
  if (live) {
    const int t = st.t[p];
    const uint4 w = philox10(make_uint4(0u, i, k, (kTagMate << 24) | tagp), st.key0, st.key1);
    const uint32_t r1 = __umulhi(w.x, static_cast<uint32_t>(t));
    uint32_t r2 = r1;
    if (t > 1) {
      r2 = __umulhi(w.y, static_cast<uint32_t>(t - 1));
      r2 += (r2 >= r1) ? 1u : 0u;
    }
    const int32_t *Bi = st.B[p] + static_cast<size_t>(i) * t;
    const int pa = Bi[r1], pb = Bi[r2];
    if (st.mate[p] && g == 0) {
      st.mate[p][2 * i] = pa;
      st.mate[p][2 * i + 1] = pb;
    }
    const bool cross = static_cast<uint64_t>(w.z) < st.tpc;
    const float4 *ra = reinterpret_cast<const float4 *>(Xc + static_cast<size_t>(pa) * st.stride);
    const float4 *rb = reinterpret_cast<const float4 *>(Xc + static_cast<size_t>(pb) * st.stride);
    float4 *ro = reinterpret_cast<float4 *>(st.XO[p] + static_cast<size_t>(i) * st.stride);
    const float4 *lb4 = reinterpret_cast<const float4 *>(st.prob.lb);
    const float4 *ub4 = reinterpret_cast<const float4 *>(st.prob.ub);
    const float4 *is4 = reinterpret_cast<const float4 *>(st.prob.inv_span);
    const uint32_t tagv = (kTagVar << 24) | tagp;
    const int nq = st.stride >> 2;
    const bool de = st.op == 1;
    const float4 *rx = reinterpret_cast<const float4 *>(Xc + static_cast<size_t>(i) * st.stride);
    const uint64_t T = st.tpm;
    for (int q = g; q < nq; q += LPO) {
      const int l0 = q << 2;
      const float4 va = ra[q], vb = rb[q], lo = lb4[q], hi = ub4[q], is = is4[q];
      const uint4 r0 = philox10(make_uint4(2 * q, i, k, tagv), st.key0, st.key1);
      uint4 r1w = make_uint4(0, 0, 0, 0);
      if (l0 + 2 < st.d) r1w = philox10(make_uint4(2 * q + 1, i, k, tagv), st.key0, st.key1);
      float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (de) {
        const float4 vx = rx[q];
        o.x = de1(vx.x, va.x, vb.x, lo.x, hi.x, st);
        o.y = de1(vx.y, va.y, vb.y, lo.y, hi.y, st);
        o.z = de1(vx.z, va.z, vb.z, lo.z, hi.z, st);
        o.w = de1(vx.w, va.w, vb.w, lo.w, hi.w, st);
      } else {
        o.x = sbx1(va.x, vb.x, r0.x, lo.x, hi.x, cross, st);
        o.y = sbx1(va.y, vb.y, r0.z, lo.y, hi.y, cross, st);
        o.z = sbx1(va.z, vb.z, r1w.x, lo.z, hi.z, cross, st);
        o.w = sbx1(va.w, vb.w, r1w.z, lo.w, hi.w, cross, st);
      }
      // polynomial mutation of each variable whose word wB falls below tpm
      if (r0.y < T) o.x = pm1(o.x, r0.y, T, st.inv_tpm, lo.x, hi.x, is.x, st);
      if (l0 + 1 < st.d && r0.w < T) o.y = pm1(o.y, r0.w, T, st.inv_tpm, lo.y, hi.y, is.y, st);
      if (l0 + 2 < st.d && r1w.y < T) o.z = pm1(o.z, r1w.y, T, st.inv_tpm, lo.z, hi.z, is.z, st);
      if (l0 + 3 < st.d && r1w.w < T) o.w = pm1(o.w, r1w.w, T, st.inv_tpm, lo.w, hi.w, is.w, st);
      // padding variables (beyond d) stay 0
      if (l0 + 1 >= st.d) o.y = 0.0f;
      if (l0 + 2 >= st.d) o.z = 0.0f;
      if (l0 + 3 >= st.d) o.w = 0.0f;
      eval_add<M, FAM>(e, l0, o.x);
      if (l0 + 1 < st.d) eval_add<M, FAM>(e, l0 + 1, o.y);
      if (l0 + 2 < st.d) eval_add<M, FAM>(e, l0 + 2, o.z);
      if (l0 + 3 < st.d) eval_add<M, FAM>(e, l0 + 3, o.w);
      ro[q] = o;
    }
  }
  // the sums over the group's chunks (and x1, x2 from chunk 0) -> F, CV, z
  eval_group<M, FAM, LPO>(st, e, g, live, &st.FCO[p][live ? i : 0]);
}

template <int M, int FAM, int LPO>
__global__ __launch_bounds__(kBlock) void k_vary(DevState st) {
  vary_body<M, FAM, LPO>(st, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

// ----------------------------------------------------------------------------
// Aggregation. PBI (Eq. (7)) with the unit direction u = w / ||w|| stored in W:
// d1 = |(F - z) . u|, d2 = ||F - z - d1 u||, g = d1 + theta d2. Tchebycheff:
// max_k w_k |f_k - z_k| with the raw weight stored in W. NaN reads as +inf.
// ----------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ float aggregate(float4 f, float4 w, const float (&z)[M], int agg,
                                           float theta) {
  const float df[3] = {f.x - z[0], f.y - (M > 1 ? z[1] : 0.0f), f.z - (M > 2 ? z[M - 1] : 0.0f)};
  const float ww[3] = {w.x, w.y, w.z};
  float g;
  if (agg == 1) {
    // fmaxf drops NaN operands, so a NaN term is tracked on the side
    g = -__builtin_huge_valf();
    bool nan = false;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const float v = ww[k] * fabsf(df[k]);
      nan = nan || (v != v);
      g = fmaxf(g, v);
    }
    if (nan) g = __builtin_huge_valf();
  } else {
    float dot = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) dot = fmaf(df[k], ww[k], dot);
    const float d1 = fabsf(dot);
    float d2 = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const float e = df[k] - d1 * ww[k];
      d2 = fmaf(e, e, d2);
    }
    g = d1 + theta * sqrtf(d2);
  }
  return nan_inf(g);
}

template <int M>
__device__ __forceinline__ void load_z(const uint32_t *zkey, float (&z)[M]) {
#pragma unroll
  for (int k = 0; k < M; ++k) z[k] = keyf(zkey[k]);
}

// ----------------------------------------------------------------------------
// k_op1: offspring cooperation (Alg. 2 OP1, Eq. (11)) at w_i.
// Population 1 takes off2_i if it is better by the feasibility priority rule
// (Eq. (8)), or, as a variant, by the prose's feasibility-first rule (a feasible
// offspring wins; otherwise the lower aggregation); population 2 takes off1_i
// if its aggregation is lower.
// ----------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void op1_body(const DevState &st, int b) {
  const int i = b * kBlock + threadIdx.x;
  // the generation counter advances here, once k_vary of this generation has read it
  if (b == 0 && threadIdx.x == 0) st.gen[0] = st.gen[0] + 1u;
  if (i >= st.n) return;
  float z[M];
  load_z<M>(st.zkey, z);
  const float4 o1 = st.FCO[0][i], o2 = st.FCO[1][i], w = st.W[i];
  const float g1 = aggregate<M>(o1, w, z, st.agg, st.theta);
  const float g2 = aggregate<M>(o2, w, z, st.agg, st.theta);
  const float c1 = nan_inf(o1.w), c2 = nan_inf(o2.w);
  const bool s1 = st.op1_rule == 0 ? ((c2 < c1) || (c2 == c1 && g2 < g1))
                                    : ((c2 == 0.0f) != (c1 == 0.0f) ? c2 == 0.0f : g2 < g1);
  const bool s2 = g1 < g2;
  // the CV lane's sign bit tells k_select which population's offspring row this is
  float4 n1 = s1 ? o2 : o1, n2 = s2 ? o1 : o2;
  n1.w = s1 ? -fabsf(n1.w) : fabsf(n1.w);
  n2.w = s2 ? -fabsf(n2.w) : fabsf(n2.w);
  st.FCN[0][i] = n1;
  st.FCN[1][i] = n2;
  st.src[i] = static_cast<uint8_t>((s1 ? 1u : 0u) | (s2 ? 2u : 0u));
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_op1(DevState st) {
  op1_body<M>(st, blockIdx.x);
}

// ----------------------------------------------------------------------------
// k_select: OP2 + OP3 (Eqs. (12)-(13)) as a pull over parent slot j of
// population p. Offspring i qualifies iff j is in B_p(i) and its new offspring
// is strictly better than parent j at w_j (population 1: lower CV, or equal CV
// and lower aggregation; population 2: lower aggregation). The winner is the
// lexicographic minimum over the qualifiers with the first index on ties; every
// decision uses generation-k parents, and replacements land after all reads of
// the slot they overwrite.
// A group of lps lanes decides one slot (lps = t_p / 4 rounded up to a power of
// two, at most 64: about four reverse-list entries per lane). Lane g takes
// entries g, g + lps, ... of the slot's padded list head, four at a time with
// independent loads (index, then candidate F/CV), then its share of the tail
// (lists longer than t_p), and keeps its lexicographic minimum of (CV, g,
// index). No load waits on another beyond index -> candidate: the head needs no
// offset, and OP1's choice of population rides in the sign of the candidate's
// CV. The group minimum follows from DPP moves inside 16-lane rows (quad swaps,
// half-row mirror, row mirror) and lane permutes beyond, and the lane that
// holds the winner writes its F/CV from registers. That minimum qualifies
// exactly when some candidate qualifies, since qualifying means being below the
// parent in the same order; a minimum over a total order does not depend on how
// the candidates were split among lanes.
// ----------------------------------------------------------------------------
struct SelKey {
  float c, g;
  int i;
};

__device__ __forceinline__ bool sel_less(const SelKey &a, const SelKey &b) {
  return a.c < b.c || (a.c == b.c && (a.g < b.g || (a.g == b.g && a.i < b.i)));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ void sel_step_dpp(SelKey &best) {
  const SelKey o{__int_as_float(dpp_i<CTRL>(__float_as_int(best.c))),
                 __int_as_float(dpp_i<CTRL>(__float_as_int(best.g))), dpp_i<CTRL>(best.i)};
  if (sel_less(o, best)) best = o;
}

__device__ __forceinline__ void sel_step_xor(SelKey &best, int o) {
  const SelKey k{__shfl_xor(best.c, o), __shfl_xor(best.g, o), __shfl_xor(best.i, o)};
  if (sel_less(k, best)) best = k;
}

// Minimum over each aligned group of lps lanes, left in every lane of the group.
// Every lane of the wave must be active.
__device__ __forceinline__ void sel_group_min(SelKey &best, int lps) {
  if (lps > 1) sel_step_dpp<0xB1>(best);   // quad_perm [1, 0, 3, 2]
  if (lps > 2) sel_step_dpp<0x4E>(best);   // quad_perm [2, 3, 0, 1]
  if (lps > 4) sel_step_dpp<0x141>(best);  // row_half_mirror: quad q <-> the other quad of its 8
  if (lps > 8) sel_step_dpp<0x140>(best);  // row_mirror: half-row <-> the other half of its 16
  if (lps > 16) sel_step_xor(best, 16);
  if (lps > 32) sel_step_xor(best, 32);
}

template <int M>
__device__ __forceinline__ void select_body(const DevState &st, int L) {
  __shared__ int s_cnt;
  const int p = L >= st.sel_blocks0 ? 1 : 0;
  const int lps = st.lps[p];
  const int g = threadIdx.x & (lps - 1);
  const int j = (L - p * st.sel_blocks0) * (kBlock / lps) + threadIdx.x / lps;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const bool live = j < st.n;
  // keys carry i2 = 2 i + (OP1 source bit of i): the same order as i, and the
  // winner's row follows without another load
  SelKey best{__builtin_huge_valf(), __builtin_huge_valf(), 0x7FFFFFFF};
  float4 bestf = make_float4(0, 0, 0, 0);  // F/CV of this lane's best candidate
  float4 w = make_float4(0, 0, 0, 0), par = make_float4(0, 0, 0, 0);
  float z[M];
  load_z<M>(st.zkey, z);
  auto consider = [&](int32_t i, float4 c) {
    const uint32_t bit = __float_as_uint(c.w) >> 31;  // set: the other population's offspring
    c.w = fabsf(c.w);
    const SelKey k{(p == 0) ? nan_inf(c.w) : 0.0f, aggregate<M>(c, w, z, st.agg, st.theta),
                   static_cast<int>((static_cast<uint32_t>(i) << 1) | bit)};
    if (sel_less(k, best)) {
      best = k;
      bestf = c;
    }
  };
  if (live) {
    const int t = st.t[p];
    w = st.W[j];
    par = st.FC[p][j];
    const int32_t *head = st.rhead[p] + static_cast<size_t>(j) * t;
    const int32_t ta = st.rtoff[p][j], tb = st.rtoff[p][j + 1];
    const float4 *cand = st.FCN[p];
    for (int q0 = g; q0 < t; q0 += 4 * lps) {  // one pass unless t > 4 lps = 256
      int ii[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * lps;
        ii[u] = q < t ? head[q] : -1;
      }
      float4 cc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cc[u] = ii[u] >= 0 ? cand[ii[u]] : make_float4(0, 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (ii[u] >= 0) consider(ii[u], cc[u]);
    }
    for (int q = ta + g; q < tb; q += lps) {
      const int32_t i = st.rtail[p][q];
      consider(i, cand[i]);
    }
  }
  const SelKey mine = best;
  sel_group_min(best, lps);
  if (live) {
    const float pc = (p == 0) ? nan_inf(par.w) : 0.0f;
    const float pg = aggregate<M>(par, w, z, st.agg, st.theta);
    const bool win = best.i != 0x7FFFFFFF && (best.c < pc || (best.c == pc && best.g < pg));
    const int bi = best.i >> 1;
    if (!win && g == 0) {  // the parent stays
      if (st.win[p]) st.win[p][j] = -1;
      st.rsrc[p][j] = -1;
    }
    if (win && mine.i == best.i) {  // the one lane that holds the winner
      if (st.win[p]) st.win[p][j] = bi;
      st.FC[p][j] = bestf;
      st.rsrc[p][j] = ((p ^ (best.i & 1)) << 30) | bi;
      atomicAdd(&s_cnt, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt > 0)
    atomicAdd(&st.repl[p * kReplLanes + (L & (kReplLanes - 1))], static_cast<unsigned long long>(s_cnt));
}

// ----------------------------------------------------------------------------
// k_rows: the row copies of the replacement, one float4 of a population row per
// thread, streaming over both populations in place: a replaced slot takes its
// winning offspring row. All reads of X for the generation happened in earlier
// launches. (Rows are not aligned to 128-byte lines; writing the kept bytes of
// shared lines back as well, so that no line is left partially written, was
// measured slower: partial lines cost nothing extra here.)
// ----------------------------------------------------------------------------
__device__ __forceinline__ void rows_body(const DevState &st, int64_t e) {
  const int nq = st.stride >> 2;
  const int64_t per_pop = static_cast<int64_t>(st.n) * nq;
  if (e >= 2 * per_pop) return;
  const int p = e >= per_pop ? 1 : 0;
  const int64_t el = e - p * per_pop;
  const int r = static_cast<int>(el / nq);
  const int c = static_cast<int>(el - static_cast<int64_t>(r) * nq);
  const int32_t ds = st.rsrc[p][r];
  if (ds < 0) return;
  const float *src = st.XO[ds >> 30] + static_cast<size_t>(ds & 0x3FFFFFFF) * st.stride;
  reinterpret_cast<float4 *>(st.X[p] + static_cast<size_t>(r) * st.stride)[c] =
      reinterpret_cast<const float4 *>(src)[c];
}

__global__ __launch_bounds__(kBlock) void k_rows(DevState st) {
  rows_body(st, static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x);
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_select(DevState st) {
  select_body<M>(st, xcd_tile(blockIdx.x, gridDim.x));
}

// ----------------------------------------------------------------------------
// Batched generations: one launch per phase covers every instance of a pool.
// Block b runs work item work[b] = (instance, block of that instance's plain
// launch), on the instance's state in S; padding items (instance -1) idle.
// Each item runs the very device function, template and lane grouping of the
// plain launch, so every instance computes bit-identically to running alone.
// ----------------------------------------------------------------------------
template <int M, int FAM>
__device__ __forceinline__ void vary_any_lanes(const DevState &st, int L) {
  switch (vary_lanes_of(st.stride)) {
    case 8: vary_body<M, FAM, 8>(st, L, vary_blocks_of(st.n, 8)); break;
    case 4: vary_body<M, FAM, 4>(st, L, vary_blocks_of(st.n, 4)); break;
    case 2: vary_body<M, FAM, 2>(st, L, vary_blocks_of(st.n, 2)); break;
    default: vary_body<M, FAM, 1>(st, L, vary_blocks_of(st.n, 1)); break;
  }
}

__global__ __launch_bounds__(kBlock) void k_vary_batch(const DevState *__restrict__ S,
                                                      const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  if (st.m == 2 && st.prob.family == 0)
    vary_any_lanes<2, 0>(st, wi.y);
  else if (st.m == 2)
    vary_any_lanes<2, 1>(st, wi.y);
  else
    vary_any_lanes<3, 1>(st, wi.y);
}

__global__ __launch_bounds__(kBlock) void k_op1_batch(const DevState *__restrict__ S,
                                                     const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  if (st.m == 2)
    op1_body<2>(st, wi.y);
  else
    op1_body<3>(st, wi.y);
}

__global__ __launch_bounds__(kBlock) void k_select_batch(const DevState *__restrict__ S,
                                                        const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  if (st.m == 2)
    select_body<2>(st, wi.y);
  else
    select_body<3>(st, wi.y);
}

__global__ __launch_bounds__(kBlock) void k_rows_batch(const DevState *__restrict__ S,
                                                      const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  rows_body(S[wi.x], static_cast<int64_t>(wi.y) * kBlock + threadIdx.x);
}

// ----------------------------------------------------------------------------
// Front: feasible rows of population `pop` that no feasible row dominates
// (Eq. (5)); candidates staged through LDS tiles.
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_front(DevState st, int pop, uint8_t *keep) {
  __shared__ float4 tile[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  float4 me = make_float4(0, 0, 0, 1);
  bool alive = false;
  if (i < st.n) {
    me = st.FC[pop][i];
    alive = (me.w == 0.0f);
  }
  for (int t0 = 0; t0 < st.n; t0 += kBlock) {
    if (!__syncthreads_or(alive)) break;
    const int jj = t0 + threadIdx.x;
    tile[threadIdx.x] = jj < st.n ? st.FC[pop][jj] : make_float4(0, 0, 0, 1);
    __syncthreads();
    const int lim = min(kBlock, st.n - t0);
    if (alive) {
      for (int q = 0; q < lim; ++q) {
        const float4 o = tile[q];
        if (o.w != 0.0f) continue;
        bool le = o.x <= me.x, lt = o.x < me.x;
        if (M > 1) { le = le && o.y <= me.y; lt = lt || o.y < me.y; }
        if (M > 2) { le = le && o.z <= me.z; lt = lt || o.z < me.z; }
        if (le && lt) {
          alive = false;
          break;
        }
      }
    }
    __syncthreads();
  }
  if (i < st.n) keep[i] = alive ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_gather(DevState st, int pop, const int32_t *idx,
                                                   int32_t count, float *x, float4 *fc) {
  const int r = blockIdx.x;
  if (r >= count) return;
  const int row = idx[r];
  const float *srcx = st.X[pop] + static_cast<size_t>(row) * st.stride;
  for (int l = threadIdx.x; l < st.d; l += blockDim.x) x[static_cast<size_t>(r) * st.d + l] = srcx[l];
  if (threadIdx.x == 0) fc[r] = st.FC[pop][row];
}

__global__ __launch_bounds__(kBlock) void k_philox(const uint4 *ctr, int64_t n, uint32_t k0,
                                                   uint32_t k1, uint4 *out) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q < n) out[q] = philox10(ctr[q], k0, k1);
}

// Streaming copy of n16 16-byte words: the reference kernel for bandwidth and
// for calibrating hardware byte counters (each word read once, written once).
__global__ __launch_bounds__(kBlock) void k_copy(const uint4 *__restrict__ src,
                                                 uint4 *__restrict__ dst, int64_t n16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < n16; q += stride)
    dst[q] = src[q];
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
#define GMPEA_DISPATCH_MF(KER, GRID, ST, S)                                          \
  do {                                                                               \
    if ((ST).m == 2 && (ST).prob.family == 0)                                        \
      hipLaunchKernelGGL((KER<2, 0>), dim3(GRID), dim3(kBlock), 0, (S), (ST));       \
    else if ((ST).m == 2)                                                            \
      hipLaunchKernelGGL((KER<2, 1>), dim3(GRID), dim3(kBlock), 0, (S), (ST));       \
    else                                                                             \
      hipLaunchKernelGGL((KER<3, 1>), dim3(GRID), dim3(kBlock), 0, (S), (ST));       \
  } while (0)

#define GMPEA_DISPATCH_M(KER, GRID, S, ...)                                          \
  do {                                                                               \
    if (st.m == 2)                                                                   \
      hipLaunchKernelGGL((KER<2>), dim3(GRID), dim3(kBlock), 0, (S), __VA_ARGS__);   \
    else                                                                             \
      hipLaunchKernelGGL((KER<3>), dim3(GRID), dim3(kBlock), 0, (S), __VA_ARGS__);   \
  } while (0)

hipError_t launch_tables(int32_t m, int32_t n, int32_t H, const int2 *offs, int32_t noffs,
                         int32_t t1, int32_t t2, int32_t agg, float4 *W, int32_t *B1, int32_t *B2,
                         uint32_t *incomplete, hipStream_t s) {
  const int grid = (n + kBlock - 1) / kBlock;
  if (m == 2)
    hipLaunchKernelGGL(k_tables<2>, dim3(grid), dim3(kBlock), 0, s, n, H, offs, noffs, t1, t2, agg,
                       W, B1, B2, incomplete);
  else
    hipLaunchKernelGGL(k_tables<3>, dim3(grid), dim3(kBlock), 0, s, n, H, offs, noffs, t1, t2, agg,
                       W, B1, B2, incomplete);
  return hipGetLastError();
}

hipError_t launch_reverse_count(int32_t n, int32_t t, const int32_t *B, int32_t *cursor,
                                int32_t *toff, hipStream_t s) {
  const int64_t nt = static_cast<int64_t>(n) * t;
  const unsigned grid = static_cast<unsigned>((nt + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_rev_count, dim3(grid), dim3(kBlock), 0, s, nt, B, cursor);
  hipLaunchKernelGGL(k_rev_excess, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, t,
                     static_cast<const int32_t *>(cursor), toff);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, toff, n + 1);
  return hipGetLastError();
}

hipError_t launch_reverse_fill(int32_t n, int32_t t, const int32_t *B, const int32_t *toff,
                               int32_t *cursor, int32_t *head, int32_t *tail, hipStream_t s) {
  const int64_t nt = static_cast<int64_t>(n) * t;
  const unsigned grid = static_cast<unsigned>((nt + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_rev_fill, dim3(grid), dim3(kBlock), 0, s, nt, t, B, toff, cursor, head, tail);
  hipLaunchKernelGGL(k_rev_sort, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, t, toff,
                     head, tail);
  return hipGetLastError();
}

template <int LPO>
static void launch_eval_lpo(const DevState &st, hipStream_t s) {
  const int grid = vary_blocks_of(st.n, LPO);
  if (st.m == 2 && st.prob.family == 0)
    hipLaunchKernelGGL((k_eval<2, 0, LPO>), dim3(grid), dim3(kBlock), 0, s, st);
  else if (st.m == 2)
    hipLaunchKernelGGL((k_eval<2, 1, LPO>), dim3(grid), dim3(kBlock), 0, s, st);
  else
    hipLaunchKernelGGL((k_eval<3, 1, LPO>), dim3(grid), dim3(kBlock), 0, s, st);
}

hipError_t launch_init(const DevState &st, hipStream_t s) {
  GMPEA_DISPATCH_MF(k_init, 2 * st.nblk, st, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (vary_lanes_of(st.stride)) {
    case 8: launch_eval_lpo<8>(st, s); break;
    case 4: launch_eval_lpo<4>(st, s); break;
    case 2: launch_eval_lpo<2>(st, s); break;
    default: launch_eval_lpo<1>(st, s); break;
  }
  return hipGetLastError();
}

template <int LPO>
static void launch_vary_lpo(const DevState &st, hipStream_t s) {
  const int grid = vary_blocks_of(st.n, LPO);
  if (st.m == 2 && st.prob.family == 0)
    hipLaunchKernelGGL((k_vary<2, 0, LPO>), dim3(grid), dim3(kBlock), 0, s, st);
  else if (st.m == 2)
    hipLaunchKernelGGL((k_vary<2, 1, LPO>), dim3(grid), dim3(kBlock), 0, s, st);
  else
    hipLaunchKernelGGL((k_vary<3, 1, LPO>), dim3(grid), dim3(kBlock), 0, s, st);
}

hipError_t launch_phase(const DevState &st, int phase, hipStream_t s) {
  if (phase == 0) {
    switch (vary_lanes_of(st.stride)) {
      case 8: launch_vary_lpo<8>(st, s); break;
      case 4: launch_vary_lpo<4>(st, s); break;
      case 2: launch_vary_lpo<2>(st, s); break;
      default: launch_vary_lpo<1>(st, s); break;
    }
  } else if (phase == 1) {
    GMPEA_DISPATCH_M(k_op1, st.nblk, s, st);
  } else if (phase == 2) {
    GMPEA_DISPATCH_M(k_select, st.sel_blocks0 + st.sel_blocks1, s, st);
  } else {
    hipLaunchKernelGGL(k_rows, dim3(rows_blocks_of(st.n, st.stride)), dim3(kBlock), 0, s, st);
  }
  return hipGetLastError();
}

hipError_t launch_batch_phase(const DevState *states, const int2 *work, int nwork, int phase,
                              hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (phase == 0)
    hipLaunchKernelGGL(k_vary_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (phase == 1)
    hipLaunchKernelGGL(k_op1_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (phase == 2)
    hipLaunchKernelGGL(k_select_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else
    hipLaunchKernelGGL(k_rows_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  return hipGetLastError();
}

hipError_t launch_generation(const DevState &st, hipStream_t s) {
  for (int phase = 0; phase < kPhases; ++phase) {
    hipError_t e = launch_phase(st, phase, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_front_flags(const DevState &st, int pop, uint8_t *keep, hipStream_t s) {
  GMPEA_DISPATCH_M(k_front, st.nblk, s, st, pop, keep);
  return hipGetLastError();
}

hipError_t launch_gather(const DevState &st, int pop, const int32_t *idx, int32_t count, float *x,
                         float4 *fc, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(count), dim3(64), 0, s, st, pop, idx, count, x, fc);
  return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, int64_t n16, hipStream_t s) {
  if (n16 <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n16 + kBlock - 1) / kBlock, 256 * 16);
  hipLaunchKernelGGL(k_copy, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s,
                     static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_philox, dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, s,
                     reinterpret_cast<const uint4 *>(ctr), n, k0, k1, reinterpret_cast<uint4 *>(out));
  return hipGetLastError();
}

}  // namespace gmpea
