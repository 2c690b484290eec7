// GMPEA generation kernels for gfx950 (CDNA4, wave64): the instantiations for
// m <= 3 objectives, the initialisation tables, and the kernels that do not
// depend on m. (gmpea_kernels_wide.hip instantiates the same device code for
// 4 <= m <= 8.)
//
// One generation (Alg. 1 loop body + Alg. 2) is four launches:
//   k_vary    a lane group per offspring (p, i): Philox draws, neighbourhood
//             mating, SBX or DE + polynomial mutation, evaluation of F and CV,
//             and the block's share of the ideal-point minimum (one atomic per
//             block and objective, skipped when it cannot lower z).
//   k_op1     one lane per subproblem i: OP1 offspring cooperation at w_i with
//             the updated ideal point; writes the new offspring's F/CV and the
//             source switch (X is not copied).
//   k_select  a lane group per parent slot (p, j): OP2 + OP3 as a pull over the
//             reverse neighbour list of j (every offspring i with j in B_p(i)),
//             lexicographic minimum of the qualifiers; writes the winner's F/CV
//             and the slot's new location (the winning offspring row), or, for
//             a kept slot whose row lies where the next generation writes its
//             offspring, copies that row to the slot's home row.
// The ideal point is a grid-wide dependency between k_vary and k_op1, and OP1
// must finish for every i before any slot can be decided; kernel boundaries
// provide both. The decisions read only F/CV records, so a slot's new location
// and its row copy, made in the same launch, touch nothing another decision
// reads.
//
// Layout: decision vectors are rows of `stride` floats (16-byte aligned) in one
// arena: home rows of both populations, then offspring rows of each population
// for even and odd generations. A slot reads its current row through its
// location, so the replacement moves no rows. F and CV share one float4 per
// individual for m <= 3.
// Blocks are remapped so that consecutive row tiles run on the same XCD (the
// hardware deals blocks to the 8 XCDs round-robin): neighbouring subproblems
// share parents and candidates, and then share that XCD's L2.
#include <algorithm>

#include "gmpea_device.hpp"

// Floating-point contraction is off for this file (build flag -ffp-contract=off)
// and every fused multiply-add is written out as fmaf: the compiler may not
// fuse an expression in one kernel and leave it unfused in another, so a device
// function gives bitwise-equal results in the plain and the batched kernels.

namespace gmpea {

// ----------------------------------------------------------------------------
// Initialisation (Alg. 1): X uniform in the box from the INIT stream,
// evaluation, ideal point.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init(DevState st) {
  // one thread per float4 chunk (row, q) of both populations, consecutive
  // threads on consecutive chunks of a row: chunk q takes the four words of the
  // INIT block q (variable l = 4 q + w), padding variables are 0; chunk 0 also
  // points the slot at its home row
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t per = static_cast<int64_t>(st.n) * st.nq;
  if (e >= 2 * per) return;
  const int p = e >= per ? 1 : 0;
  const int64_t r = e - p * per;
  const int i = static_cast<int>(r / st.nq);
  const int q = static_cast<int>(r - static_cast<int64_t>(i) * st.nq);
  const uint4 w = philox10(make_uint4(q, i, 0u, (kTagInit << 24) | (p << 16)), st.key0, st.key1);
  const uint32_t words[4] = {w.x, w.y, w.z, w.w};
  float x[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int l = 4 * q + u;
    x[u] = 0.0f;
    if (l < st.d) {
      const float lo = st.prob.lb[l], hi = st.prob.ub[l];
      x[u] = fmaf(hi - lo, u24(words[u]), lo);
    }
  }
  reinterpret_cast<float4 *>(st.X[p] + static_cast<size_t>(i) * st.stride)[q] =
      make_float4(x[0], x[1], x[2], x[3]);
  if (q == 0) st.loc[p][i] = static_cast<uint32_t>(p * st.region + i);
}

// Every slot of population `pop` points at its home row.
__global__ __launch_bounds__(kBlock) void k_loc_home(DevState st, int pop) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < st.n) st.loc[pop][j] = static_cast<uint32_t>(pop * st.region + j);
}

// Copy of every slot's current decision vector to its home row, one thread per
// float4 chunk (sources are offspring rows or the home row itself, never
// another slot's home row); k_loc_home then points the slots there.
__global__ __launch_bounds__(kBlock) void k_materialize(DevState st) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t per = static_cast<int64_t>(st.n) * st.nq;
  if (e >= 2 * per) return;
  const int p = e >= per ? 1 : 0;
  const int64_t r = e - p * per;
  const int j = static_cast<int>(r / st.nq);
  const int q = static_cast<int>(r - static_cast<int64_t>(j) * st.nq);
  const uint32_t l = st.loc[p][j], home = static_cast<uint32_t>(p * st.region + j);
  if (l != home)
    reinterpret_cast<float4 *>(st.rows + static_cast<size_t>(home) * st.stride)[q] = arena_row(st, l)[q];
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
  if (c < tmax) {
    // a walk that came up short: the row's remaining entries name the row
    // itself, so that every entry is a valid index until the host's exact
    // search replaces both tables
    atomicOr(incomplete, 1u);
    for (; c < tmax; ++c) {
      if (c < t1) B1[static_cast<size_t>(i) * t1 + c] = i;
      if (c < t2) B2[static_cast<size_t>(i) * t2 + c] = i;
    }
  }
}

// Reverse lists: lengths, the scan of their excess over t, a scatter into the
// padded head and the tail, and a per-list insertion sort (lists hold about t
// entries) so that every list is ascending.
// (an entry outside [0, n) is skipped by the count and the scatter alike)
__global__ __launch_bounds__(kBlock) void k_rev_count(int64_t nt, int32_t n, const int32_t *__restrict__ B,
                                                     int32_t *__restrict__ cnt) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= nt) return;
  const int32_t j = B[q];
  if (j >= 0 && j < n) atomicAdd(&cnt[j], 1);
}

__global__ __launch_bounds__(kBlock) void k_rev_excess(int32_t n, int32_t t, const int32_t *__restrict__ cnt,
                                                      int32_t *__restrict__ toff) {
  const int32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < n) toff[j + 1] = max(cnt[j] - t, 0);
}

// Inclusive scan of off[0 .. len) in three launches: per-tile sums (tiles of
// kScanTile entries), one block scanning the tile sums, then every tile adding
// its prefix (kScanTile threads per tile, one entry each).
constexpr int kScanTile = 1024;

__global__ __launch_bounds__(kScanTile) void k_scan_tiles(const int32_t *__restrict__ off, int32_t len,
                                                          int32_t *__restrict__ sums) {
  __shared__ int32_t red[kScanTile / 64];
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x;
  int32_t v = q < len ? off[q] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < kScanTile / 64; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

// Exclusive scan of the tile sums in place, by one block (each thread a
// contiguous run of them).
__global__ __launch_bounds__(kScanTile) void k_scan_sums(int32_t *sums, int32_t tiles) {
  __shared__ int32_t part[kScanTile];
  const int tid = threadIdx.x;
  const int per = (tiles + kScanTile - 1) / kScanTile;
  const int lo = min(tiles, tid * per), hi = min(tiles, lo + per);
  int32_t sum = 0;
  for (int q = lo; q < hi; ++q) sum += sums[q];
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < kScanTile; o <<= 1) {
    const int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid > 0 ? part[tid - 1] : 0;
  for (int q = lo; q < hi; ++q) {
    const int32_t v = sums[q];
    sums[q] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kScanTile) void k_scan_add(int32_t *__restrict__ off, int32_t len,
                                                        const int32_t *__restrict__ sums) {
  __shared__ int32_t part[kScanTile];
  const int tid = threadIdx.x;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kScanTile + tid;
  part[tid] = q < len ? off[q] : 0;
  __syncthreads();
  for (int o = 1; o < kScanTile; o <<= 1) {
    const int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  if (q < len) off[q] = part[tid] + sums[blockIdx.x];
}

// Scatter of the reverse lists: entries past a list's first t go to the tail,
// which holds `cap` entries; an entry beyond it is dropped and *overflow set
// (the caller then rebuilds with an exact tail).
__global__ __launch_bounds__(kBlock) void k_rev_fill(int64_t nt, int32_t t, const int32_t *__restrict__ B,
                                                    const int32_t *__restrict__ toff,
                                                    int32_t *__restrict__ cursor,
                                                    int32_t *__restrict__ head,
                                                    int32_t *__restrict__ tail, int32_t cap,
                                                    uint32_t *__restrict__ overflow) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= nt) return;
  const int32_t j = B[q];
  if (j < 0 || j >= static_cast<int32_t>(nt / t)) return;
  const int32_t pos = atomicAdd(&cursor[j], 1);
  const int32_t i = static_cast<int32_t>(q / t);
  if (pos < t) {
    head[static_cast<size_t>(j) * t + pos] = i;
  } else {
    const int32_t at = toff[j] + pos - t;
    if (at < cap)
      tail[at] = i;
    else
      atomicOr(overflow, 1u);
  }
}

// Each list sorted ascending by one wave: the wave stages the list (head
// entries, then its tail) in LDS, each lane ranks its entries by counting the
// smaller ones (the entries of a list are distinct) and writes every entry at
// its rank. A list longer than kRevSortMax (not met by lattice neighbourhoods,
// whose lists hold about t entries) is sorted by one lane in place.
constexpr int kRevSortMax = 512;

__global__ __launch_bounds__(kBlock) void k_rev_sort(int32_t n, int32_t t, const int32_t *__restrict__ toff,
                                                    int32_t *__restrict__ head,
                                                    int32_t *__restrict__ tail, int32_t cap) {
  __shared__ int32_t buf[kBlock / 64][kRevSortMax];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int32_t j = blockIdx.x * (kBlock / 64) + wv;
  // a list whose tail lies beyond the tail's room was not filled completely
  // (the caller rebuilds): left as it is
  if (j < n && toff[j + 1] > cap) j = n;
  int32_t len = 0, ext = 0;
  int32_t *h = nullptr, *tl = nullptr;
  if (j < n) {  // uniform per wave
    h = head + static_cast<size_t>(j) * t;
    tl = tail + toff[j];
    ext = toff[j + 1] - toff[j];
    // the head holds the first min(length, t) entries, then -1
    int32_t hl = 0;
    for (int32_t k0 = 0; k0 < t; k0 += 64) {
      const int32_t k = k0 + lane;
      hl += __popcll(__ballot(k < t && h[k] >= 0));
    }
    len = hl + ext;
  }
  auto at = [&](int32_t k) -> int32_t & { return k < t ? h[k] : tl[k - t]; };
  const bool staged = j < n && len <= kRevSortMax;
  if (staged)
    for (int32_t k = lane; k < len; k += 64) buf[wv][k] = at(k);
  __syncthreads();
  if (staged) {
    for (int32_t k = lane; k < len; k += 64) {
      const int32_t v = buf[wv][k];
      int32_t rank = 0;
      for (int32_t u = 0; u < len; ++u) rank += buf[wv][u] < v ? 1 : 0;
      at(rank) = v;
    }
  } else if (j < n && lane == 0) {
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

__global__ __launch_bounds__(kBlock) void k_tvary_batch(const DevState *__restrict__ S,
                                                       const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  if (st.m == 2 && st.prob.family == 0)
    tvary_body<2, 0>(st, wi.y, vary_grid(st));
  else if (st.m == 2)
    tvary_body<2, 1>(st, wi.y, vary_grid(st));
  else
    tvary_body<3, 1>(st, wi.y, vary_grid(st));
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

// One kernel per m: each holds only its own registers (m = 2 fits eight waves
// per SIMD, a kernel holding both m kept seven), at one more launch per
// generation when a pool mixes m = 2 and m = 3.
template <int M>
__global__ __launch_bounds__(kBlock) void k_select_batch(const DevState *__restrict__ S,
                                                        const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  select_body<M>(S[wi.x], wi.y);
}

// Rows idx[0 .. count) of population `pop`: decision vectors to x (count x d)
// and F/CV records to fc (count x rq); either output may be null.
__global__ __launch_bounds__(kBlock) void k_gather(DevState st, int pop, const int32_t *idx,
                                                   int32_t count, float *x, float4 *fc) {
  const int r = blockIdx.x;
  if (r >= count) return;
  const int row = idx[r];
  if (x) {
    const float *srcx = reinterpret_cast<const float *>(arena_row(st, st.loc[pop][row]));
    for (int l = threadIdx.x; l < st.d; l += blockDim.x) x[static_cast<size_t>(r) * st.d + l] = srcx[l];
  }
  if (fc && threadIdx.x < st.rq)
    fc[static_cast<size_t>(r) * st.rq + threadIdx.x] = st.FC[pop][static_cast<size_t>(row) * st.rq + threadIdx.x];
}

// ----------------------------------------------------------------------------
// Neighbourhoods of an arbitrary reference set given as integer coordinates
// (layered sets, m > 3): row i's t nearest rows by exact squared distance, ties
// by index, one block per row. A radix select over the distance's digits (8
// bits at a time from the top, each pass a 256-bin LDS histogram of the
// distances that share the digits found so far) finds the t-th smallest
// distance D and how many rows at distance D are needed; the rows below D are
// gathered, the needed rows at D are taken in index order (contiguous index
// ranges per thread and a scan of their counts), and the t rows are placed by
// their rank in (distance, index) order. B1 receives the first t1 of them and
// B2 the first t2 (t = max(t1, t2) <= kKnnMaxT).
// ----------------------------------------------------------------------------
constexpr int kKnnMaxT = 256;

__global__ __launch_bounds__(kBlock) void k_knn(const int32_t *__restrict__ K, int32_t n, int32_t m,
                                               int32_t bits, int32_t t1, int32_t t2,
                                               int32_t *__restrict__ B1, int32_t *__restrict__ B2) {
  __shared__ int32_t ki[kMaxM];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int32_t s_need, s_nsel;
  __shared__ uint64_t sel_d[kKnnMaxT];
  __shared__ int32_t sel_j[kKnnMaxT];
  __shared__ int32_t scan[kBlock];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int t = max(t1, t2);
  if (tid < m) ki[tid] = K[static_cast<size_t>(i) * m + tid];
  if (tid == 0) {
    s_prefix = 0;
    s_need = t;
    s_nsel = 0;
  }
  __syncthreads();
  auto dist = [&](int j) -> uint64_t {
    const int32_t *kj = K + static_cast<size_t>(j) * m;
    int64_t d = 0;
    for (int a = 0; a < m; ++a) {
      const int64_t df = static_cast<int64_t>(kj[a]) - ki[a];
      d += df * df;
    }
    return static_cast<uint64_t>(d);
  };
  // digits [lo, hi) from the top bit of the largest distance down: the first
  // pass already spreads the distances over the 256 bins
  for (int hi = bits; hi > 0; hi -= 8) {
    const int lo = hi > 8 ? hi - 8 : 0;
    hist[tid] = 0;
    __syncthreads();
    const uint64_t above = hi >= 64 ? 0ull : (~0ull << hi);
    const uint64_t pre = s_prefix;
    const uint64_t dmask = (1ull << (hi - lo)) - 1ull;
    for (int j = tid; j < n; j += kBlock) {
      const uint64_t d = dist(j);
      if ((d & above) == pre) atomicAdd(&hist[(d >> lo) & dmask], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      int32_t cum = 0;
      for (int b = 0; b < 256; ++b) {
        const int32_t h = static_cast<int32_t>(hist[b]);
        if (cum + h >= s_need) {
          s_prefix = pre | (static_cast<uint64_t>(b) << lo);
          s_need -= cum;
          break;
        }
        cum += h;
      }
    }
    __syncthreads();
  }
  const uint64_t D = s_prefix;
  const int32_t need = s_need;  // rows at distance D to take; t - need lie below D
  for (int j = tid; j < n; j += kBlock) {
    const uint64_t d = dist(j);
    if (d < D) {
      const int k = atomicAdd(&s_nsel, 1);
      sel_d[k] = d;
      sel_j[k] = j;
    }
  }
  const int per = (n + kBlock - 1) / kBlock;
  const int lo = min(n, tid * per), hi = min(n, lo + per);
  int32_t cnt = 0;
  for (int j = lo; j < hi; ++j) cnt += dist(j) == D;
  scan[tid] = cnt;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {  // inclusive scan of the tie counts
    const int32_t v = tid >= o ? scan[tid - o] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int32_t rank = scan[tid] - cnt;
  for (int j = lo; j < hi && rank < need; ++j)
    if (dist(j) == D) {
      sel_d[t - need + rank] = D;
      sel_j[t - need + rank] = j;
      ++rank;
    }
  __syncthreads();
  if (tid < t) {  // place entry tid by its rank in (distance, index) order
    const uint64_t d = sel_d[tid];
    const int32_t j = sel_j[tid];
    int r = 0;
    for (int q = 0; q < t; ++q) r += (sel_d[q] < d) || (sel_d[q] == d && sel_j[q] < j);
    if (r < t1) B1[static_cast<size_t>(i) * t1 + r] = j;
    if (r < t2) B2[static_cast<size_t>(i) * t2 + r] = j;
  }
}

// ----------------------------------------------------------------------------
// Front quality (Eqs. (14)-(15)), for results delivered at a deadline.
// The front's objectives are staged through LDS tiles of kBlock points; m and
// the record width are run-time values (one kernel serves every m).
// ----------------------------------------------------------------------------
__device__ __forceinline__ void stage_front(float *tile, const float4 *front, int count, int rq,
                                            int m, int t0) {
  const int jj = t0 + threadIdx.x;
  if (jj < count) {
    const float *rec = reinterpret_cast<const float *>(front + static_cast<size_t>(jj) * rq);
    for (int k = 0; k < m; ++k) tile[threadIdx.x * kMaxM + k] = rec[k];
  }
}

// IGD: one thread per reference point; the block's sum of nearest distances
// (FP64) goes to partial[blockIdx.x].
__global__ __launch_bounds__(kBlock) void k_igd(const float *__restrict__ ref, int32_t n_ref,
                                                int32_t m, const float4 *__restrict__ front,
                                                int32_t count, int32_t rq, double *partial) {
  __shared__ float tile[kBlock * kMaxM];
  __shared__ double red[kBlock / 64];
  const int r = blockIdx.x * kBlock + threadIdx.x;
  float v[kMaxM];
#pragma unroll
  for (int k = 0; k < kMaxM; ++k) v[k] = (r < n_ref && k < m) ? ref[static_cast<size_t>(r) * m + k] : 0.0f;
  float best = __builtin_huge_valf();
  for (int t0 = 0; t0 < count; t0 += kBlock) {
    stage_front(tile, front, count, rq, m, t0);
    __syncthreads();
    const int lim = min(kBlock, count - t0);
    for (int q = 0; q < lim; ++q) {
      float d2 = 0.0f;
#pragma unroll
      for (int k = 0; k < kMaxM; ++k)
        if (k < m) {
          const float df = v[k] - tile[q * kMaxM + k];
          d2 = fmaf(df, df, d2);
        }
      best = fminf(best, d2);
    }
    __syncthreads();
  }
  double x = (r < n_ref) ? static_cast<double>(sqrtf(best)) : 0.0;
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) sum += red[w];
    partial[blockIdx.x] = sum;
  }
}

// HV by Monte Carlo: one thread per sample, drawn from the counter RNG (tag
// kTagHv, counter (sample low word, sample high word, block, tag << 24)) in the
// box [lo, hi]; a sample counts when some front point is <= it in every
// objective. Tiles stop once every sample of the block is dominated.
__global__ __launch_bounds__(kBlock) void k_hv(int64_t n, int32_t m, const float *__restrict__ lo,
                                               const float *__restrict__ hi, uint32_t k0, uint32_t k1,
                                               const float4 *__restrict__ front, int32_t count,
                                               int32_t rq, unsigned long long *hits) {
  __shared__ float tile[kBlock * kMaxM];
  const int64_t sidx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  float x[kMaxM];
  const uint32_t c0 = static_cast<uint32_t>(sidx), c1 = static_cast<uint32_t>(sidx >> 32);
  const uint4 wa = philox10(make_uint4(c0, c1, 0u, kTagHv << 24), k0, k1);
  const uint4 wb = m > 4 ? philox10(make_uint4(c0, c1, 1u, kTagHv << 24), k0, k1) : make_uint4(0, 0, 0, 0);
  const uint32_t w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
#pragma unroll
  for (int k = 0; k < kMaxM; ++k) x[k] = k < m ? fmaf(hi[k] - lo[k], u24(w[k]), lo[k]) : 0.0f;
  bool dom = sidx >= n;  // samples past the end count as done (and are not counted)
  for (int t0 = 0; t0 < count; t0 += kBlock) {
    if (__syncthreads_and(dom)) break;
    stage_front(tile, front, count, rq, m, t0);
    __syncthreads();
    const int lim = min(kBlock, count - t0);
    for (int q = 0; q < lim && !dom; ++q) {
      bool le = true;
#pragma unroll
      for (int k = 0; k < kMaxM; ++k)
        if (k < m) le = le && tile[q * kMaxM + k] <= x[k];
      dom = le;
    }
    __syncthreads();
  }
  const int c = __syncthreads_count(dom && sidx < n);
  if (threadIdx.x == 0 && c > 0) atomicAdd(hits, static_cast<unsigned long long>(c));
}

// Spans set to 32-bit patterns: a few words up to 16-byte alignment, then
// 16-byte stores over the body, then the remaining words; every thread of the
// grid strides over each span in turn.
__global__ __launch_bounds__(kBlock) void k_fill(FillSpans f) {
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const uint64_t nt = static_cast<uint64_t>(gridDim.x) * kBlock;
  for (int k = 0; k < f.count; ++k) {
    uint32_t *p = f.p[k];
    const uint64_t n = f.words[k];
    const uint32_t v = f.value[k];
    const uint64_t lead = ((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 4u;
    const uint64_t h = lead < n ? lead : n;
    if (tid < h) p[tid] = v;
    uint4 *p4 = reinterpret_cast<uint4 *>(p + h);
    const uint64_t n4 = (n - h) / 4;
    const uint4 v4 = make_uint4(v, v, v, v);
    for (uint64_t i = tid; i < n4; i += nt) p4[i] = v4;
    for (uint64_t i = h + 4 * n4 + tid; i < n; i += nt) p[i] = v;
  }
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

// The same copy with four independent 16-byte words per thread in flight (all
// four loads issued before the stores) and one pass over the buffer: a second
// reading of the attainable copy bandwidth. kNt selects non-temporal loads and
// stores (streamed past the caches).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <bool kNt>
__global__ __launch_bounds__(kBlock) void k_copy4(const u32x4 *__restrict__ src,
                                                  u32x4 *__restrict__ dst, int64_t n16) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * (4 * kBlock) + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t q = base + u * kBlock;
    if (q < n16) v[u] = kNt ? __builtin_nontemporal_load(src + q) : src[q];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t q = base + u * kBlock;
    if (q < n16) {
      if (kNt)
        __builtin_nontemporal_store(v[u], dst + q);
      else
        dst[q] = v[u];
    }
  }
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
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

// Inclusive scan of off[0 .. len) with tile sums in `sums` (room for
// ceil(len / kScanTile) entries).
static hipError_t launch_scan(int32_t *off, int32_t len, int32_t *sums, hipStream_t s) {
  const int32_t tiles = (len + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanTile), 0, s, off, len, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanTile), 0, s, sums, tiles);
  hipLaunchKernelGGL(k_scan_add, dim3(tiles), dim3(kScanTile), 0, s, off, len, static_cast<const int32_t *>(sums));
  return hipGetLastError();
}

hipError_t launch_reverse_count(int32_t n, int32_t t, const int32_t *B, int32_t *cursor,
                                int32_t *toff, hipStream_t s) {
  const int64_t nt = static_cast<int64_t>(n) * t;
  const unsigned grid = static_cast<unsigned>((nt + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_rev_count, dim3(grid), dim3(kBlock), 0, s, nt, n, B, cursor);
  hipLaunchKernelGGL(k_rev_excess, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, t,
                     static_cast<const int32_t *>(cursor), toff);
  return launch_scan(toff, n + 1, cursor + n, s);
}

hipError_t launch_reverse_fill(int32_t n, int32_t t, const int32_t *B, const int32_t *toff,
                               int32_t *cursor, int32_t *head, int32_t *tail, int32_t cap,
                               uint32_t *overflow, hipStream_t s) {
  const int64_t nt = static_cast<int64_t>(n) * t;
  const unsigned grid = static_cast<unsigned>((nt + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_rev_fill, dim3(grid), dim3(kBlock), 0, s, nt, t, B, toff, cursor, head, tail, cap,
                     overflow);
  hipLaunchKernelGGL(k_rev_sort, dim3((n + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, s, n, t,
                     toff, head, tail, cap);
  return hipGetLastError();
}

// Initial evaluation in the order the variation kernel for this row width
// evaluates its offspring (so a copy of an individual evaluates bitwise equal).
template <int M, int FAM, int LPO>
static void launch_eval_lpo(const DevState &st, hipStream_t s) {
  hipLaunchKernelGGL((k_eval<M, FAM, LPO>), dim3(vary_blocks_of(st.n, LPO)), dim3(kBlock), 0, s, st);
}

template <int M, int FAM>
static void launch_eval_mf(const DevState &st, hipStream_t s) {
  if (vary_tasked(st)) {
    hipLaunchKernelGGL((k_teval<M, FAM>), dim3(2 * st.nblk), dim3(kBlock), 0, s, st);
    return;
  }
  switch (vary_lanes_of(st)) {
    case 8: launch_eval_lpo<M, FAM, 8>(st, s); break;
    case 4: launch_eval_lpo<M, FAM, 4>(st, s); break;
    case 2: launch_eval_lpo<M, FAM, 2>(st, s); break;
    default: launch_eval_lpo<M, FAM, 1>(st, s); break;
  }
}

hipError_t launch_fill(const FillSpans &f, hipStream_t s) {
  if (f.count <= 0) return hipSuccess;
  if (f.count > kMaxFillSpans) return hipErrorInvalidValue;
  uint64_t words = 0;
  for (int k = 0; k < f.count; ++k) {
    if (f.words[k] > 0 && (reinterpret_cast<uintptr_t>(f.p[k]) & 3u) != 0) return hipErrorInvalidValue;
    words += f.words[k];
  }
  if (words == 0) return hipSuccess;
  const uint64_t want = (words / 4 + kBlock - 1) / kBlock;
  const unsigned grid = static_cast<unsigned>(want < 1 ? 1 : (want > 4096 ? 4096 : want));
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, s, f);
  return hipGetLastError();
}

hipError_t launch_init(const DevState &st, hipStream_t s) {
  const int64_t chunks = 2LL * st.n * st.nq;
  hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>((chunks + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (st.m > 3) return launch_init_eval_wide(st, s);
  if (st.m == 2 && st.prob.family == 0)
    launch_eval_mf<2, 0>(st, s);
  else if (st.m == 2)
    launch_eval_mf<2, 1>(st, s);
  else
    launch_eval_mf<3, 1>(st, s);
  return hipGetLastError();
}

template <int M, int FAM>
static void launch_vary_mf(const DevState &st, hipStream_t s) {
  const int grid = vary_grid(st);
  if (vary_tasked(st)) {
    hipLaunchKernelGGL((k_tvary<M, FAM>), dim3(grid), dim3(kBlock), 0, s, st);
    return;
  }
  switch (vary_lanes_of(st)) {
    case 8: hipLaunchKernelGGL((k_vary<M, FAM, 8>), dim3(grid), dim3(kBlock), 0, s, st); break;
    case 4: hipLaunchKernelGGL((k_vary<M, FAM, 4>), dim3(grid), dim3(kBlock), 0, s, st); break;
    case 2: hipLaunchKernelGGL((k_vary<M, FAM, 2>), dim3(grid), dim3(kBlock), 0, s, st); break;
    default: hipLaunchKernelGGL((k_vary<M, FAM, 1>), dim3(grid), dim3(kBlock), 0, s, st); break;
  }
}

hipError_t launch_phase(const DevState &st, int phase, hipStream_t s) {
  if (st.m > 3) return launch_phase_wide(st, phase, s);
  if (phase == 0) {
    if (st.m == 2 && st.prob.family == 0)
      launch_vary_mf<2, 0>(st, s);
    else if (st.m == 2)
      launch_vary_mf<2, 1>(st, s);
    else
      launch_vary_mf<3, 1>(st, s);
  } else if (phase == 1) {
    GMPEA_DISPATCH_M(k_op1, st.nblk, s, st);
  } else {
    GMPEA_DISPATCH_M(k_select, st.sel_blocks0 + st.sel_blocks1, s, st);
  }
  return hipGetLastError();
}

hipError_t launch_batch_phase(const DevState *states, const int2 *work, int nwork, int phase,
                              bool wide, bool sub, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (wide) return launch_batch_phase_wide(states, work, nwork, phase, sub, s);
  if (phase == 0 && sub)
    hipLaunchKernelGGL(k_tvary_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (phase == 0)
    hipLaunchKernelGGL(k_vary_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (phase == 1)
    hipLaunchKernelGGL(k_op1_batch, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (sub)
    hipLaunchKernelGGL(k_select_batch<2>, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else
    hipLaunchKernelGGL(k_select_batch<3>, dim3(nwork), dim3(kBlock), 0, s, states, work);
  return hipGetLastError();
}

hipError_t launch_loc_home(const DevState &st, int pop, hipStream_t s) {
  hipLaunchKernelGGL(k_loc_home, dim3(st.nblk), dim3(kBlock), 0, s, st, pop);
  return hipGetLastError();
}

hipError_t launch_materialize(const DevState &st, hipStream_t s) {
  const int64_t chunks = 2LL * st.n * st.nq;
  hipLaunchKernelGGL(k_materialize, dim3(static_cast<unsigned>((chunks + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, st);
  hipError_t e = hipGetLastError();
  for (int p = 0; p < 2 && e == hipSuccess; ++p) e = launch_loc_home(st, p, s);
  return e;
}

hipError_t launch_generation(const DevState &st, hipStream_t s) {
  for (int phase = 0; phase < kPhases; ++phase) {
    hipError_t e = launch_phase(st, phase, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_front_flags(const DevState &st, int pop, uint8_t *keep, hipStream_t s) {
  if (st.m > 3) return launch_front_flags_wide(st, pop, keep, s);
  const int chunk = front_chunk(st.n);
  const dim3 grid(st.nblk, (st.n + chunk - 1) / chunk);
  GMPEA_DISPATCH_M(k_front_init, st.nblk, s, st, pop, keep);
  if (st.m == 2)
    hipLaunchKernelGGL((k_front<2>), grid, dim3(kBlock), 0, s, st, pop, keep, chunk);
  else
    hipLaunchKernelGGL((k_front<3>), grid, dim3(kBlock), 0, s, st, pop, keep, chunk);
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

hipError_t launch_copy4(const void *src, void *dst, int64_t n16, bool nontemporal, hipStream_t s) {
  if (n16 <= 0) return hipSuccess;
  const int64_t blocks = (n16 + 4 * kBlock - 1) / (4 * kBlock);
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (nontemporal)
    hipLaunchKernelGGL(k_copy4<true>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n16);
  else
    hipLaunchKernelGGL(k_copy4<false>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_knn(const int32_t *K, int32_t n, int32_t m, uint64_t max_dist, int32_t t1, int32_t t2,
                      int32_t *B1, int32_t *B2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (std::max(t1, t2) > kKnnMaxT) return hipErrorInvalidValue;
  int32_t bits = 1;  // every distance is below 2^bits
  while (bits < 63 && (max_dist >> bits) != 0) ++bits;
  hipLaunchKernelGGL(k_knn, dim3(n), dim3(kBlock), 0, s, K, n, m, bits, t1, t2, B1, B2);
  return hipGetLastError();
}

hipError_t launch_igd(const float *ref, int32_t n_ref, int32_t m, const float4 *front, int32_t count,
                      int32_t rq, double *partial, int32_t *blocks, hipStream_t s) {
  const int grid = (n_ref + kBlock - 1) / kBlock;
  *blocks = grid;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_igd, dim3(grid), dim3(kBlock), 0, s, ref, n_ref, m, front, count, rq, partial);
  return hipGetLastError();
}

hipError_t launch_hv(int64_t n, int32_t m, const float *lo, const float *hi, uint32_t k0, uint32_t k1,
                     const float4 *front, int32_t count, int32_t rq, unsigned long long *hits,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_hv, dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, s, n, m, lo, hi, k0, k1,
                     front, count, rq, hits);
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
