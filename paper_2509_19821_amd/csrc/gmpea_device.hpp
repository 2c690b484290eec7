// Device code of the GMPEA generation shared by the kernel translation units:
// gmpea_kernels.hip instantiates it for m <= 3 (one float4 per F/CV record),
// gmpea_kernels_wide.hip for 4 <= m <= 8. Every function is templated on the
// objective count M, so each instantiation holds only the registers its m needs.
#pragma once

#include <type_traits>

#include "gmpea_internal.hpp"

namespace gmpea {

// ----------------------------------------------------------------------------
// Counter RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ----------------------------------------------------------------------------
// Each round's two 32 x 32 -> 64-bit products are written as 64-bit multiplies
// so that each becomes one v_mad_u64_u32 (high and low words together), and
// each three-way XOR with the round key is one gfx950 v_bitop3_b32 (truth
// table 0x96) instead of two v_xor_b32.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    c = make_uint4(xor3(static_cast<uint32_t>(p1 >> 32), c.y, k0), static_cast<uint32_t>(p1),
                   xor3(static_cast<uint32_t>(p0 >> 32), c.w, k1), static_cast<uint32_t>(p0));
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

// The decision vector in arena row r (float4 view).
__device__ __forceinline__ const float4 *arena_row(const DevState &st, uint32_t r) {
  return reinterpret_cast<const float4 *>(st.rows + static_cast<size_t>(r) * st.stride);
}

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

// F/CV record of one individual in registers: objectives f_0 .. f_{M-1} from
// the first lane, CV in the last lane (kCv), unused lanes 0; rec_quads(M) float4.
template <int M>
struct Rec {
  static constexpr int Q = rec_quads(M);
  static constexpr int kCv = 4 * Q - 1;
  float v[4 * Q];
};

template <int M>
__device__ __forceinline__ Rec<M> rec_load(const float4 *base, int j) {
  Rec<M> r;
  const float4 *p = base + static_cast<size_t>(j) * Rec<M>::Q;
#pragma unroll
  for (int a = 0; a < Rec<M>::Q; ++a) {
    const float4 t = p[a];
    r.v[4 * a] = t.x;
    r.v[4 * a + 1] = t.y;
    r.v[4 * a + 2] = t.z;
    r.v[4 * a + 3] = t.w;
  }
  return r;
}

template <int M>
__device__ __forceinline__ void rec_store(float4 *base, int j, const Rec<M> &r) {
  float4 *p = base + static_cast<size_t>(j) * Rec<M>::Q;
#pragma unroll
  for (int a = 0; a < Rec<M>::Q; ++a)
    p[a] = make_float4(r.v[4 * a], r.v[4 * a + 1], r.v[4 * a + 2], r.v[4 * a + 3]);
}

template <int M>
__device__ __forceinline__ Rec<M> rec_zero() {
  Rec<M> r;
#pragma unroll
  for (int k = 0; k < 4 * Rec<M>::Q; ++k) r.v[k] = 0.0f;
  return r;
}

// Running sums of the evaluation, filled chunk by chunk, and the leading
// variables the objectives and the equality read: x1, x2 in lead for m <= 3.
// For m > 3 the first kLeadChunks float4 chunks (through the last angle
// variable x_{m-1}) go to the group's LDS slot instead (lead_slots): held in
// registers, a chunk chosen by a run-time index sends the accumulator to
// scratch memory.
template <int M>
struct EvalAcc {
  static constexpr int kLeadChunks = M <= 3 ? 0 : (M + 2) / 4;
  float s;  // curve: sum x_2..x_d; sphere: sum over non-angle variables of (x - 0.5)^2
  float lead[2];
};

// LDS slots of the leading chunks for m > 3: two float4 per lane group (at
// most kBlock groups per block).
template <int M>
__device__ __forceinline__ float4 *lead_slots(int group) {
  __shared__ float4 slots[kBlock * 2];
  return slots + 2 * group;
}

// Component k (0..3) of a float4; k is a constant wherever this is called.
__device__ __forceinline__ float f4_at(const float4 &v, int k) {
  return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

template <int M, int FAM>
__device__ __forceinline__ void eval_add(EvalAcc<M> &e, int l, float x) {
  if (l == 0) e.lead[0] = x;
  if (l == 1) e.lead[1] = x;
  if (FAM == 0) {
    if (l >= 1) e.s += x;
  } else {
    if (l >= M - 1) e.s = fmaf(x - 0.5f, x - 0.5f, e.s);
  }
}

// Adds chunk q (variables 4q .. 4q + 3, those below d) in variable order; for
// m > 3 a leading chunk is also stored to the group's slot.
template <int M, int FAM>
__device__ __forceinline__ void eval_chunk(EvalAcc<M> &e, int q, float4 o, int d, float4 *slot) {
  const int l0 = q << 2;
  if constexpr (M <= 3) {
    eval_add<M, FAM>(e, l0, o.x);
    if (l0 + 1 < d) eval_add<M, FAM>(e, l0 + 1, o.y);
    if (l0 + 2 < d) eval_add<M, FAM>(e, l0 + 2, o.z);
    if (l0 + 3 < d) eval_add<M, FAM>(e, l0 + 3, o.w);
  } else {  // the sphere family: keep the leading chunks, sum the rest
    if (q < EvalAcc<M>::kLeadChunks) slot[q] = o;
    const float xs[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (l0 + k >= M - 1 && l0 + k < d) e.s = fmaf(xs[k] - 0.5f, xs[k] - 0.5f, e.s);
  }
}

// F and CV from the sums (Eqs. (1)-(3)); c0, c1: the leading chunks for m > 3.
template <int M, int FAM>
__device__ __forceinline__ Rec<M> eval_finish(const EvalAcc<M> &e, float4 c0, float4 c1,
                                              const DevProblem &P) {
  float f[M > 3 ? M : 3];
#pragma unroll
  for (int k = 0; k < (M > 3 ? M : 3); ++k) f[k] = 0.0f;
  if (FAM == 0) {
    const float g = fmaf(P.g_scale, e.s, 1.0f);
    f[0] = e.lead[0];
    f[1] = g * (1.0f - sqrtf(e.lead[0] / g));
  } else if constexpr (M <= 3) {
    const float r = 1.0f + e.s;
    float s0, c0;
    sincospif(0.5f * e.lead[0], &s0, &c0);
    if (M == 2) {
      f[0] = r * c0;
      f[1] = r * s0;
    } else {
      float s1, c1;
      sincospif(0.5f * e.lead[1], &s1, &c1);
      f[0] = r * c0 * c1;
      f[1] = r * c0 * s1;
      f[2] = r * s0;
    }
  } else {
    // f_k = (1 + g) prod_{j < M-1-k} cos(theta_j), times sin(theta_{M-1-k}) for
    // k > 0: with the running product P_j = (1 + g) cos(theta_0) .. cos(theta_{j-1})
    // (multiplied left to right), f_{M-1-j} = P_j sin(theta_j) and f_0 = P_{M-1}
    float P = 1.0f + e.s;
#pragma unroll
    for (int j = 0; j < M - 1; ++j) {
      float sj, cj;
      sincospif(0.5f * (j < 4 ? f4_at(c0, j) : f4_at(c1, j - 4)), &sj, &cj);
      f[M - 1 - j] = P * sj;
      P = P * cj;
    }
    f[0] = P;
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
    const float x0 = M <= 3 ? e.lead[0] : c0.x, x1 = M <= 3 ? e.lead[1] : c0.y;
    const float c = fabsf(x0 + x1 - 1.0f) - P.eq_tol;
    cv += (c > 0.0f) ? c : 0.0f;
  }
  Rec<M> out = rec_zero<M>();
#pragma unroll
  for (int k = 0; k < (M > 3 ? M : 3); ++k) out.v[k] = f[k];
  out.v[Rec<M>::kCv] = cv;
  return out;
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

// Evaluation of a population row by a group of LPO lanes: lane g adds chunks
// g, g + LPO, ... in order, then a butterfly combines the lanes. k_vary adds
// its offspring in exactly this order, so F and CV are a function of x alone:
// an offspring that copies an individual evaluates bitwise equal to it.
template <int M, int FAM, int LPO>
__device__ __forceinline__ EvalAcc<M> eval_row(const DevState &st, const float4 *row, int g,
                                               bool live, float4 *slot) {
  EvalAcc<M> e{};
  if (live) {
    const int nq = st.nq;
    for (int q = g; q < nq; q += LPO) eval_chunk<M, FAM>(e, q, row[q], st.d, slot);
  }
  return e;
}

// Group reduction of the sums (every thread of the block takes part), then
// F/CV and the ideal point's block minimum. The leading variables come from the
// lanes that added their chunks (m <= 3: lane 0's registers; m > 3: the
// group's LDS slot).
template <int M, int FAM, int LPO>
__device__ __forceinline__ void eval_group(const DevState &st, EvalAcc<M> e, int g, bool live,
                                           float4 *out, int j, const float4 *slot) {
  float zv[M];
#pragma unroll
  for (int q = 0; q < M; ++q) zv[q] = __builtin_huge_valf();
#pragma unroll
  for (int o = 1; o < LPO; o <<= 1) e.s += __shfl_xor(e.s, o);
  const int base = (threadIdx.x & 63) & ~(LPO - 1);
  if constexpr (M <= 3) {
    e.lead[0] = __shfl(e.lead[0], base);
    e.lead[1] = __shfl(e.lead[1], base);
  } else {
    __syncthreads();  // the slots' stores are visible to the finishing lane
  }
  if (live && g == 0) {
    float4 c0 = make_float4(0, 0, 0, 0), c1 = c0;
    if constexpr (M > 3) {
      c0 = slot[0];
      if (EvalAcc<M>::kLeadChunks > 1) c1 = slot[1];
    }
    const Rec<M> fc = eval_finish<M, FAM>(e, c0, c1, st.prob);
    rec_store<M>(out, j, fc);
#pragma unroll
    for (int k = 0; k < M; ++k) zv[k] = fc.v[k];
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
  float4 *slot = M > 3 ? lead_slots<M>(threadIdx.x / LPO) : nullptr;
  const EvalAcc<M> e = eval_row<M, FAM, LPO>(st, row, g, live, slot);
  eval_group<M, FAM, LPO>(st, e, g, live, st.FC[p], live ? i : 0, slot);
}

// ----------------------------------------------------------------------------
// k_vary: reproduction (SBX or DE, then PM) + evaluation + ideal-point update.
// Draws (the paper fixes no RNG; this counter layout is the library's): Philox
// counter (c0, i, k, tag << 24 | p << 16) for offspring i of population p in
// generation k. The MATE block (c0 = 0) gives the two neighbourhood positions
// and the per-offspring crossing draw; VAR block c0 = l >> 1 gives (wA, wB) for
// variables l and l + 1: SBX's bits in wA, the mutation test and uniform in wB.
// A group of LPO consecutive lanes builds one offspring: lane g of the group
// takes the float4 chunks g, g + LPO, ... of the row, so each group step reads
// and writes LPO * 16 contiguous bytes of a row (whole 128-byte lines at
// LPO = 8); LPO comes from vary_lanes_of.
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
  const bool live = i < st.n;
  EvalAcc<M> e{};
  float4 *slot = M > 3 ? lead_slots<M>(threadIdx.x / LPO) : nullptr;
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
    // the parents' current decision vectors, wherever the replacement left them
    const float4 *ra = arena_row(st, st.loc[p][pa]);
    const float4 *rb = arena_row(st, st.loc[p][pb]);
    float4 *ro = reinterpret_cast<float4 *>(st.rows + static_cast<size_t>(offspring_row(st, gen_slot(st, k), p, i)) *
                                                          st.stride);
    const float4 *lb4 = reinterpret_cast<const float4 *>(st.prob.lb);
    const float4 *ub4 = reinterpret_cast<const float4 *>(st.prob.ub);
    const float4 *is4 = reinterpret_cast<const float4 *>(st.prob.inv_span);
    const uint32_t tagv = (kTagVar << 24) | tagp;
    const int nq = st.nq;
    const bool de = st.op == 1;
    const float4 *rx = de ? arena_row(st, st.loc[p][i]) : ra;
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
      eval_chunk<M, FAM>(e, q, o, st.d, slot);
      ro[q] = o;
      note_write(st, 0, p, i);
    }
  }
  // the sums over the group's chunks (and the leading variables) -> F, CV, z
  eval_group<M, FAM, LPO>(st, e, g, live, st.FCO[p], live ? i : 0, slot);
}

template <int M, int FAM, int LPO>
__global__ __launch_bounds__(kBlock) void k_vary(DevState st) {
  vary_body<M, FAM, LPO>(st, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

// ----------------------------------------------------------------------------
// Task-dealt variation for rows of at most kTaskChunks float4 chunks (d <= 128).
// A wave builds `off` = st.task_off offspring: lane o < off first draws
// offspring o's mating picks and finds its parents' rows; then the wave's
// off nq tasks (offspring o, chunk q), numbered o nq + q, are dealt to the
// lanes in order, task lane + 64 s in step s, so one wave instruction reads and
// writes 64 consecutive chunks (about 1 KB of offspring rows, the matching
// spans of the parent rows) and no lane idles before the last step. Each task
// leaves its chunk's evaluation partial in LDS; lane o then adds its
// offspring's partials in chunk order and finishes F, CV and the ideal point,
// so the results do not depend on off. The draws and the variation of every
// variable are those of vary_body. A wave's LDS (its offspring's sources, then
// kTaskPart floats of partials and leading variables) is about 5 KB, so LDS
// allows eight waves per SIMD.
// ----------------------------------------------------------------------------
// Evaluation partial of chunk q (variables 4q .. 4q + 3 below d, in order).
template <int M, int FAM>
__device__ __forceinline__ float chunk_partial(int q, float4 o, int d) {
  const float xs[4] = {o.x, o.y, o.z, o.w};
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int l = 4 * q + k;
    if (l < d) {
      if (FAM == 0) {
        if (l >= 1) s += xs[k];
      } else if (l >= M - 1) {
        s = fmaf(xs[k] - 0.5f, xs[k] - 0.5f, s);
      }
    }
  }
  return s;
}

// F/CV record of a row from its chunk partials (added in chunk order) and its
// leading chunks c0, c1 (the variables the objectives and the equality read).
template <int M, int FAM>
__device__ __forceinline__ Rec<M> eval_partials(const float *part, int nq, float4 c0, float4 c1,
                                                const DevProblem &P) {
  EvalAcc<M> e{};
  e.s = 0.0f;
  for (int q = 0; q < nq; ++q) e.s += part[q];
  e.lead[0] = c0.x;
  e.lead[1] = c0.y;
  return eval_finish<M, FAM>(e, c0, c1, P);
}

// LDS of tvary_body, one buffer per kernel whatever the template instances a
// batched kernel holds (a non-template function's shared array; m <= 3 and
// m > 3 never share a kernel): per wave, the offspring's sources (parent rows
// a and b, the crossing draw in a's bit 31, b < 0 for no offspring), then the
// chunk partials (offspring-major, off nq floats) followed, for m <= 3, by each
// offspring's x1 and x2; for m > 3 the first two chunks of each offspring.
template <bool W>
struct TvaryLds {
  static constexpr int kOff = W ? kTaskOffWide : kTaskOffNarrow;
  int2 src[kBlock / 64][kOff];
  float part[kBlock / 64][kTaskPart];
  typename std::conditional<W, float4[kBlock / 64][kOff][2], char[1]>::type lead;
};
__device__ __forceinline__ TvaryLds<false> &tvary_lds_narrow() {
  __shared__ TvaryLds<false> lds;
  return lds;
}
__device__ __forceinline__ TvaryLds<true> &tvary_lds_wide() {
  __shared__ TvaryLds<true> lds;
  return lds;
}

template <int M, int FAM>
__device__ __forceinline__ void tvary_body(const DevState &st, int L, int G) {
  constexpr bool kWide = M > 3;
  constexpr int kLead = kWide ? EvalAcc<M>::kLeadChunks : 1;
  static_assert(kLead <= 2, "at most two leading chunks");
  auto &lds = [] () -> auto & {
    if constexpr (kWide) return tvary_lds_wide();
    else return tvary_lds_narrow();
  }();
  auto &s_src = lds.src;
  auto &s_part = lds.part;
  const int half = G >> 1;  // blocks per population
  const int p = L >= half ? 1 : 0;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int off = st.task_off;
  const int base = (L - p * half) * (kBlock / 64 * off) + wv * off;  // the wave's first offspring
  const uint32_t k = *st.gen + 1u;
  const uint32_t tagp = (p << 16);
  const int n = st.n, nq = st.nq;
  // ---- lane o: offspring base + o -- mating picks and parent rows ----
  if (lane < off) {
    const int i = base + lane;
    int2 src = make_int2(0, -1);
    if (i < n) {
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
      if (st.mate[p]) {
        st.mate[p][2 * i] = pa;
        st.mate[p][2 * i + 1] = pb;
      }
      const bool cross = static_cast<uint64_t>(w.z) < st.tpc;
      src = make_int2(static_cast<int>(st.loc[p][pa] | (cross ? 0x80000000u : 0u)), static_cast<int>(st.loc[p][pb]));
    }
    s_src[wv][lane] = src;
  }
  __syncthreads();
  // ---- the wave's off nq tasks, task lane + 64 s in step s ----
  const float4 *lb4 = reinterpret_cast<const float4 *>(st.prob.lb);
  const float4 *ub4 = reinterpret_cast<const float4 *>(st.prob.ub);
  const float4 *is4 = reinterpret_cast<const float4 *>(st.prob.inv_span);
  const uint32_t tagv = (kTagVar << 24) | tagp;
  const bool de = st.op == 1;
  const uint64_t T = st.tpm;
  const int tasks = off * nq, steps = (tasks + 63) >> 6;
  const int dq = 64 % nq, dof = 64 / nq;
  int o = lane / nq, q = lane - (lane / nq) * nq;
  for (int step = 0; step < steps; ++step) {
    const int2 src = o < off ? s_src[wv][o] : make_int2(0, -1);
    if (src.y >= 0) {
      const int i = base + o;
      const bool cross = src.x < 0;
      const int l0 = q << 2;
      const float4 va = arena_row(st, static_cast<uint32_t>(src.x) & 0x7FFFFFFFu)[q];
      const float4 vb = arena_row(st, static_cast<uint32_t>(src.y))[q];
      const float4 lo = lb4[q], hi = ub4[q], is = is4[q];
      const uint4 r0 = philox10(make_uint4(2 * q, i, k, tagv), st.key0, st.key1);
      uint4 r1w = make_uint4(0, 0, 0, 0);
      if (l0 + 2 < st.d) r1w = philox10(make_uint4(2 * q + 1, i, k, tagv), st.key0, st.key1);
      float4 ov = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (de) {
        const float4 vx = arena_row(st, st.loc[p][i])[q];
        ov.x = de1(vx.x, va.x, vb.x, lo.x, hi.x, st);
        ov.y = de1(vx.y, va.y, vb.y, lo.y, hi.y, st);
        ov.z = de1(vx.z, va.z, vb.z, lo.z, hi.z, st);
        ov.w = de1(vx.w, va.w, vb.w, lo.w, hi.w, st);
      } else {
        ov.x = sbx1(va.x, vb.x, r0.x, lo.x, hi.x, cross, st);
        ov.y = sbx1(va.y, vb.y, r0.z, lo.y, hi.y, cross, st);
        ov.z = sbx1(va.z, vb.z, r1w.x, lo.z, hi.z, cross, st);
        ov.w = sbx1(va.w, vb.w, r1w.z, lo.w, hi.w, cross, st);
      }
      if (r0.y < T) ov.x = pm1(ov.x, r0.y, T, st.inv_tpm, lo.x, hi.x, is.x, st);
      if (l0 + 1 < st.d && r0.w < T) ov.y = pm1(ov.y, r0.w, T, st.inv_tpm, lo.y, hi.y, is.y, st);
      if (l0 + 2 < st.d && r1w.y < T) ov.z = pm1(ov.z, r1w.y, T, st.inv_tpm, lo.z, hi.z, is.z, st);
      if (l0 + 3 < st.d && r1w.w < T) ov.w = pm1(ov.w, r1w.w, T, st.inv_tpm, lo.w, hi.w, is.w, st);
      if (l0 + 1 >= st.d) ov.y = 0.0f;
      if (l0 + 2 >= st.d) ov.z = 0.0f;
      if (l0 + 3 >= st.d) ov.w = 0.0f;
      reinterpret_cast<float4 *>(st.rows + static_cast<size_t>(offspring_row(st, gen_slot(st, k), p, i)) *
                                               st.stride)[q] = ov;
      note_write(st, 0, p, i);
      s_part[wv][o * nq + q] = chunk_partial<M, FAM>(q, ov, st.d);
      if constexpr (kWide) {
        if (q < kLead) lds.lead[wv][o][q] = ov;
      } else if (q == 0) {
        s_part[wv][off * nq + 2 * o] = ov.x;
        s_part[wv][off * nq + 2 * o + 1] = ov.y;
      }
    }
    q += dq;
    o += dof;
    if (q >= nq) {
      q -= nq;
      ++o;
    }
  }
  __syncthreads();
  // ---- lane o: F, CV and the ideal point of offspring base + o ----
  float zv[M];
#pragma unroll
  for (int a = 0; a < M; ++a) zv[a] = __builtin_huge_valf();
  const int i = base + lane;
  if (lane < off && i < n) {
    float4 c0, c1 = make_float4(0, 0, 0, 0);
    if constexpr (kWide) {
      c0 = lds.lead[wv][lane][0];
      if (kLead > 1) c1 = lds.lead[wv][lane][kLead > 1 ? 1 : 0];
    } else {
      c0 = make_float4(s_part[wv][off * nq + 2 * lane], s_part[wv][off * nq + 2 * lane + 1], 0.0f, 0.0f);
    }
    const Rec<M> fc = eval_partials<M, FAM>(&s_part[wv][lane * nq], nq, c0, c1, st.prob);
    rec_store<M>(st.FCO[p], i, fc);
#pragma unroll
    for (int a = 0; a < M; ++a) zv[a] = fc.v[a];
  }
  block_zmin<M>(zv, st.zkey);
}

template <int M, int FAM>
__global__ __launch_bounds__(kBlock) void k_tvary(DevState st) {
  tvary_body<M, FAM>(st, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

// Initial evaluation matching tvary_body's order (rows of at most kTaskChunks
// chunks): one thread per row, chunk partials added in chunk order.
template <int M, int FAM>
__global__ __launch_bounds__(kBlock) void k_teval(DevState st) {
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int half = gridDim.x >> 1;
  const int p = L >= half ? 1 : 0;
  const int i = (L - p * half) * kBlock + threadIdx.x;
  float zv[M];
#pragma unroll
  for (int a = 0; a < M; ++a) zv[a] = __builtin_huge_valf();
  if (i < st.n) {
    const float4 *row = reinterpret_cast<const float4 *>(st.X[p] + static_cast<size_t>(i) * st.stride);
    float part[kTaskChunks];
    for (int q = 0; q < st.nq; ++q) part[q] = chunk_partial<M, FAM>(q, row[q], st.d);
    const float4 c1 = st.nq > 1 ? row[1] : make_float4(0, 0, 0, 0);
    const Rec<M> fc = eval_partials<M, FAM>(part, st.nq, row[0], c1, st.prob);
    rec_store<M>(st.FC[p], i, fc);
#pragma unroll
    for (int a = 0; a < M; ++a) zv[a] = fc.v[a];
  }
  block_zmin<M>(zv, st.zkey);
}

// ----------------------------------------------------------------------------
// Aggregation. PBI (Eq. (7)) with the unit direction u = w / ||w|| stored in W:
// d1 = |(F - z) . u|, d2 = ||F - z - d1 u||, g = d1 + theta d2. Tchebycheff:
// max_k w_k |f_k - z_k| with the raw weight stored in W. NaN reads as +inf.
// ----------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ float aggregate(const Rec<M> &f, const Rec<M> &w, const float (&z)[M],
                                           int agg, float theta) {
  float df[M], ww[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    df[k] = f.v[k] - z[k];
    ww[k] = w.v[k];
  }
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
    // the hardware square root (within one ulp; a correctly rounded sqrtf
    // costs about fifteen more instructions per candidate)
    g = d1 + theta * __builtin_amdgcn_sqrtf(d2);
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
  constexpr int kCv = Rec<M>::kCv;
  const Rec<M> o1 = rec_load<M>(st.FCO[0], i), o2 = rec_load<M>(st.FCO[1], i);
  const Rec<M> w = rec_load<M>(st.W, i);
  const float g1 = aggregate<M>(o1, w, z, st.agg, st.theta);
  const float g2 = aggregate<M>(o2, w, z, st.agg, st.theta);
  const float c1 = nan_inf(o1.v[kCv]), c2 = nan_inf(o2.v[kCv]);
  const bool s1 = st.op1_rule == 0 ? ((c2 < c1) || (c2 == c1 && g2 < g1))
                                    : ((c2 == 0.0f) != (c1 == 0.0f) ? c2 == 0.0f : g2 < g1);
  const bool s2 = g1 < g2;
  // the CV lane's sign bit tells k_select which population's offspring row this is
  Rec<M> n1 = s1 ? o2 : o1, n2 = s2 ? o1 : o2;
  n1.v[kCv] = s1 ? -fabsf(n1.v[kCv]) : fabsf(n1.v[kCv]);
  n2.v[kCv] = s2 ? -fabsf(n2.v[kCv]) : fabsf(n2.v[kCv]);
  rec_store<M>(st.FCN[0], i, n1);
  rec_store<M>(st.FCN[1], i, n2);
  note_write(st, 1, 0, i);
  note_write(st, 1, 1, i);
  st.src[i] = static_cast<uint8_t>((s1 ? 1u : 0u) | (s2 ? 2u : 0u));
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_op1(DevState st) {
  op1_body<M>(st, blockIdx.x);
}

// ----------------------------------------------------------------------------
// Kept rows moved home. A kept slot keeps its row, but a row in the offspring
// regions the next generation writes (its generation slot, gen_slot) would be
// overwritten: such a row is copied to the slot's home row (`from` -> `home`,
// arena rows) by all lanes of the wave together. The wave's pending rows are
// ranked, their (from, home) pairs staged in LDS, and the (row, chunk) copies
// dealt to the lanes in order, four per lane at a time with the four loads
// issued before the stores. No slot points at another slot's home row, so the
// copies never overwrite a row that some location still names. Every lane of
// the wave must call it. A wave reads back only what its own lanes staged, and
// one wave's LDS accesses complete in order, so a wave-level fence stands in
// for a block barrier and the block's other waves run on.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void wave_copy_home(const DevState &st, bool copy, uint32_t from, uint32_t home) {
  __shared__ uint2 s_cp[kBlock / 64][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t pending = __ballot(copy);
  if (copy) s_cp[wv][__popcll(pending & ((1ull << lane) - 1ull))] = make_uint2(from, home);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (pending == 0) return;  // uniform over the wave
  const int np = __popcll(pending);
  const int nq = st.nq, tasks = np * nq;
  const int dq = 64 % nq, dr = 64 / nq;
  int r = lane / nq, c = lane - (lane / nq) * nq;
  // one task: load its chunk (held in v, its destination in o; o < 0: none)
  auto fetch = [&](int t, float4 &v, int64_t &o) {
    o = -1;
    if (t < tasks) {
      const uint2 fh = s_cp[wv][r];
      v = arena_row(st, fh.x)[c];
      o = static_cast<int64_t>(fh.y) * st.stride + 4 * c;
    }
    c += dq;
    r += dr;
    if (c >= nq) {
      c -= nq;
      ++r;
    }
  };
  auto put = [&](const float4 &v, int64_t o) {
    if (o >= 0) {
      *reinterpret_cast<float4 *>(st.rows + o) = v;
      if (st.wcheck) {  // the home row's slot: row / stride = p region + j
        const int64_t h = o / st.stride;
        const int hp = h >= st.region ? 1 : 0;
        note_write(st, 3, hp, static_cast<int>(h - hp * st.region));
      }
    }
  };
  for (int t0 = lane; t0 < tasks; t0 += 4 * 64) {
    float4 v0, v1, v2, v3;
    int64_t o0, o1, o2, o3;
    fetch(t0, v0, o0);
    fetch(t0 + 64, v1, o1);
    fetch(t0 + 128, v2, o2);
    fetch(t0 + 192, v3, o3);
    put(v0, o0);
    put(v1, o1);
    put(v2, o2);
    put(v3, o3);
  }
}

// ----------------------------------------------------------------------------
// k_select: OP2 + OP3 (Eqs. (12)-(13)) as a pull over parent slot j of
// population p. Offspring i qualifies iff j is in B_p(i) and its new offspring
// is strictly better than parent j at w_j (population 1: lower CV, or equal CV
// and lower aggregation; population 2: lower aggregation). The winner is the
// lexicographic minimum over the qualifiers with the first index on ties; every
// decision uses generation-k parents, and replacements land after all reads of
// the slot they overwrite.
// A group of lps lanes decides one slot (lps = t_p / sel_per_lane rounded up to
// a power of two, at most 64). When t_p = K lps (K = sel_per_lane), lane g
// takes entries K g .. K g + K - 1 of the slot's padded list head (16-byte
// index loads), else entries g, g + lps, ... (every lane busy), up to K at a
// time, with independent loads (index, then candidate F/CV), then its share of the tail
// (lists longer than t_p), and keeps its lexicographic minimum of (CV, g,
// index). No load waits on another beyond index -> candidate: the head needs no
// offset, and OP1's choice of population rides in the sign of the candidate's
// CV. The group minimum follows from DPP moves inside 16-lane rows (quad swaps,
// half-row mirror, row mirror) and lane permutes beyond, and the lane that
// holds the winner writes its F/CV from registers. That minimum qualifies
// exactly when some candidate qualifies, since qualifying means being below the
// parent in the same order; a minimum over a total order does not depend on how
// the candidates were split among lanes.
// The slot's location follows the decision in the same launch: a replaced slot
// points at the winner's offspring row (written by this generation's
// variation, slot gen_slot(k)); a kept slot whose row lies in the offspring
// regions of the next generation's slot has it moved home (wave_copy_home). Neither touches a row
// or a record that another slot's decision reads.
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
  __shared__ int s_cnt[kBlock / 64];
  const int p = L >= st.sel_blocks0 ? 1 : 0;
  const int lps = st.lps[p];
  const int g = threadIdx.x & (lps - 1);
  const int j = (L - p * st.sel_blocks0) * (kBlock / lps) + threadIdx.x / lps;
  const bool live = j < st.n;
  bool copy = false;  // a kept row this lane moves home (see wave_copy_home)
  bool wrote = false;  // this lane replaced its group's slot
  uint32_t from = 0, home = 0;
  // keys carry i2 = 2 i + (OP1 source bit of i): the same order as i, and the
  // winner's row follows without another load
  constexpr int kCv = Rec<M>::kCv;
  SelKey best{__builtin_huge_valf(), __builtin_huge_valf(), 0x7FFFFFFF};
  Rec<M> w = rec_zero<M>(), par = rec_zero<M>();
  uint32_t loc0 = 0;
  float z[M];
  load_z<M>(st.zkey, z);
  // Each lane keeps only its best key; the winner's record is read again after
  // the group minimum. A candidate is taken without branches: an index < 0 (the
  // padding after a list's end, its record read from row 0) keys as
  // (+inf, +inf, INT_MAX) and never wins, and the lexicographic compare and
  // the update are compares and selects.
  auto consider = [&](int32_t i, Rec<M> c) {
    const bool ok = i >= 0;
    const uint32_t bit = __float_as_uint(c.v[kCv]) >> 31;  // set: the other population's offspring
    const float kc = ok ? ((p == 0) ? nan_inf(fabsf(c.v[kCv])) : 0.0f) : __builtin_huge_valf();
    const float kg = ok ? aggregate<M>(c, w, z, st.agg, st.theta) : __builtin_huge_valf();
    const int ki = ok ? static_cast<int>((static_cast<uint32_t>(i) << 1) | bit) : 0x7FFFFFFF;
    const bool lt = (kc < best.c) | ((kc == best.c) & ((kg < best.g) | ((kg == best.g) & (ki < best.i))));
    best.c = lt ? kc : best.c;
    best.g = lt ? kg : best.g;
    best.i = lt ? ki : best.i;
  };
  if (live) {
    const int t = st.t[p];
    w = rec_load<M>(st.W, j);
    par = rec_load<M>(st.FC[p], j);
    loc0 = st.loc[p][j];
    const int32_t *head = st.rhead[p] + static_cast<size_t>(j) * t;
    const int32_t ta = st.rtoff[p][j], tb = st.rtoff[p][j + 1];
    const float4 *cand = st.FCN[p];
    constexpr int K = sel_per_lane(Rec<M>::Q);
    if (t == K * lps) {
      // lane g takes entries K g .. K g + K - 1 (16-byte loads; head rows are
      // 16-byte aligned when t is a multiple of 4), all K candidate loads in
      // flight together; the minimum does not depend on how the entries are
      // dealt to lanes
      for (int q0 = K * g; q0 < t; q0 += K * lps) {
        int ii[K];
#pragma unroll
        for (int h4 = 0; h4 < K / 4; ++h4) {
          const int4 v = *reinterpret_cast<const int4 *>(head + q0 + 4 * h4);
          ii[4 * h4] = v.x;
          ii[4 * h4 + 1] = v.y;
          ii[4 * h4 + 2] = v.z;
          ii[4 * h4 + 3] = v.w;
        }
        Rec<M> cc[K];
#pragma unroll
        for (int u = 0; u < K; ++u) cc[u] = rec_load<M>(cand, max(ii[u], 0));
#pragma unroll
        for (int u = 0; u < K; ++u) consider(ii[u], cc[u]);
      }
    } else {
      // entries g, g + lps, ...: every lane of the group busy whatever t is
      // (one pass unless t > K lps), up to K candidate loads in flight
      for (int q0 = g; q0 < t; q0 += K * lps) {
        int ii[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
          const int q = q0 + u * lps;
          const int v = head[min(q, t - 1)];
          ii[u] = q < t ? v : -1;
        }
        Rec<M> cc[K];
#pragma unroll
        for (int u = 0; u < K; ++u) cc[u] = rec_load<M>(cand, max(ii[u], 0));
#pragma unroll
        for (int u = 0; u < K; ++u) consider(ii[u], cc[u]);
      }
    }
    for (int q = ta + g; q < tb; q += lps) {
      const int32_t i = st.rtail[p][q];
      consider(i, rec_load<M>(cand, i));
    }
  }
  sel_group_min(best, lps);
  if (live) {
    const float pc = (p == 0) ? nan_inf(par.v[kCv]) : 0.0f;
    const float pg = aggregate<M>(par, w, z, st.agg, st.theta);
    const bool win = best.i != 0x7FFFFFFF && (best.c < pc || (best.c == pc && best.g < pg));
    const int bi = best.i >> 1;
    const uint32_t k = *st.gen;  // this generation (OP1 advanced the counter)
    if (!win && g == 0) {  // the parent stays, and its row too unless the next offspring overwrite it
      if (st.win[p]) st.win[p][j] = -1;
      const uint32_t l = loc0;
      const uint32_t lo = offspring_row(st, gen_slot(st, k + 1u), 0, 0);
      if (l >= lo && l < lo + 2 * static_cast<uint32_t>(st.region)) {
        copy = true;
        from = l;
        home = static_cast<uint32_t>(p * st.region + j);
        st.loc[p][j] = home;
        note_write(st, 3, p, j);
      }
    }
    // the group's first lane: the slot takes the winner's F/CV and points at
    // its offspring row
    if (win && g == 0) {
      if (st.win[p]) st.win[p][j] = bi;
      Rec<M> bestf = rec_load<M>(st.FCN[p], bi);
      bestf.v[kCv] = fabsf(bestf.v[kCv]);
      rec_store<M>(st.FC[p], j, bestf);
      st.loc[p][j] = offspring_row(st, gen_slot(st, k), p ^ (best.i & 1), bi);
      note_write(st, 2, p, j);
      wrote = true;
    }
  }
  wave_copy_home(st, copy, from, home);
  // the block's replacements: one count per wave, one barrier, one atomic
  const uint64_t wb = __ballot(wrote);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = __popcll(wb);
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) c += s_cnt[q];
    if (c > 0) atomicAdd(&st.repl[p * kReplLanes + (L & (kReplLanes - 1))], static_cast<unsigned long long>(c));
  }
}


// m <= 3: eight waves per SIMD (at most 64 VGPRs; one float4, stored before
// the candidate loop and read after it, goes to scratch): 168-180 against
// 180-192 us at N = 1e6, 24-26
// against 25-27 us at N = 1e5. The batched kernel, which holds both m, lost
// with the same bound (1.36 against 1.28 ms per pool generation).
template <int M>
__global__ __launch_bounds__(kBlock, (M <= 3 ? 8 : 1)) void k_select(DevState st) {
  select_body<M>(st, xcd_tile(blockIdx.x, gridDim.x));
}

// ----------------------------------------------------------------------------
// Batched generations: one launch per phase covers every instance of a pool.
// Block b runs work item work[b] = (instance, block of that instance's plain
// launch), on the instance's state in S; padding items (instance -1) idle.
// Each item runs the very device function, template and lane grouping of the
// plain launch, so every instance computes bit-identically to running alone.
// ----------------------------------------------------------------------------
// Lane-group variation of one work item with the instance's lane count (the
// task-dealt kernel has batched kernels of its own, so that these keep no LDS
// for it).
template <int M, int FAM>
__device__ __forceinline__ void vary_any_lanes(const DevState &st, int L) {
  const int G = vary_grid(st);
  switch (vary_lanes_of(st)) {
    case 8: vary_body<M, FAM, 8>(st, L, G); break;
    case 4: vary_body<M, FAM, 4>(st, L, G); break;
    case 2: vary_body<M, FAM, 2>(st, L, G); break;
    default: vary_body<M, FAM, 1>(st, L, G); break;
  }
}

// ----------------------------------------------------------------------------
// Front: feasible rows of population `pop` that no feasible row dominates
// (Eq. (5)). k_front_init sets keep[i] = (row i is feasible); k_front then
// clears keep[i] when some feasible row dominates row i. Its grid is (row tile,
// column chunk): each block checks its kBlock rows against one chunk of
// candidate rows staged through LDS tiles, so a population of a few thousand
// rows still spreads over the whole chip; several blocks may clear the same
// flag, all with the same value.
// ----------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_front_init(DevState st, int pop, uint8_t *keep) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < st.n) keep[i] = rec_load<M>(st.FC[pop], i).v[Rec<M>::kCv] == 0.0f ? 1 : 0;
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_front(DevState st, int pop, uint8_t *keep, int chunk) {
  constexpr int kCv = Rec<M>::kCv;
  __shared__ float4 tile[kBlock * Rec<M>::Q];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  Rec<M> me = rec_zero<M>();
  bool alive = false;
  if (i < st.n) {
    me = rec_load<M>(st.FC[pop], i);
    alive = (me.v[kCv] == 0.0f);
  }
  const int c0 = blockIdx.y * chunk, c1 = min(st.n, c0 + chunk);
  for (int t0 = c0; t0 < c1; t0 += kBlock) {
    if (!__syncthreads_or(alive)) break;
    const int jj = t0 + threadIdx.x;
    Rec<M> r = rec_zero<M>();
    if (jj < c1) r = rec_load<M>(st.FC[pop], jj);
    else r.v[kCv] = 1.0f;  // never dominates
    rec_store<M>(tile, threadIdx.x, r);
    __syncthreads();
    const int lim = min(kBlock, c1 - t0);
    if (alive) {
      for (int q = 0; q < lim; ++q) {
        const Rec<M> o = rec_load<M>(tile, q);
        if (o.v[kCv] != 0.0f) continue;
        bool le = true, lt = false;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          le = le && o.v[k] <= me.v[k];
          lt = lt || o.v[k] < me.v[k];
        }
        if (le && lt) {
          alive = false;
          keep[i] = 0;
          break;
        }
      }
    }
    __syncthreads();
  }
}

// Column chunks of k_front: enough blocks to fill the chip, chunks of whole tiles.
__host__ __device__ inline int front_chunk(int n) {
  const int tiles = (n + kBlock - 1) / kBlock;
  const int want = (2048 + tiles - 1) / tiles;  // about 2048 blocks in all
  const int chunks = want < tiles ? want : tiles;
  const int per = (tiles + chunks - 1) / chunks;
  return per * kBlock;
}

}  // namespace gmpea
