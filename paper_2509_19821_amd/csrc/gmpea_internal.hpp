// Internal declarations of the GMPEA HIP library: kernel argument blocks and
// launchers shared by the kernels (gmpea_kernels.hip for m <= 3,
// gmpea_kernels_wide.hip for m > 3) and the host runtime (gmpea_abi.cpp,
// lattice.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

namespace gmpea {

constexpr int kMaxM = 8;
constexpr int kMaxRing = 8;
constexpr int kBlock = 256;  // threads per block of the per-subproblem kernels
// Reverse-list entries a k_select lane takes at a time, by the float4 count of
// an F/CV record: eight one-float4 records, four wider ones (their loads in
// flight take the registers). A slot's lanes are t_p / that count rounded up to
// a power of two, at most 64.
__host__ __device__ constexpr int sel_per_lane(int rq) { return rq == 1 ? 8 : 4; }
// Replacement counters are spread over this many words per population: one
// word updated by every block serialises those atomics at one L2 channel.
constexpr int kReplLanes = 64;

// Stream tags of the counter RNG (top byte of counter word 3).
constexpr uint32_t kTagInit = 1u;
constexpr uint32_t kTagMate = 2u;
constexpr uint32_t kTagVar = 3u;
constexpr uint32_t kTagHv = 4u;  // Monte Carlo samples of the hypervolume (not the method's)

// Problem constants in the device precision, passed by value to every kernel
// that evaluates F and CV.
struct DevProblem {
  int32_t family, m, d, n_ring, has_sum_lower, n_eq;
  float ring_c[kMaxRing * kMaxM];  // centres, row-major
  float ring_r2[kMaxRing];         // squared radii
  float sum_lower, eq_tol;
  float g_scale;                   // 9 / (d - 1) for the curve family
  const float *lb, *ub;            // device, stride each (padding: 0 and 1)
  const float *inv_span;           // device, 1 / (ub - lb), stride each
};

// float4 words per F/CV record and per reference-vector row: one (f0, f1, f2,
// cv) up to three objectives, else enough for m objectives and the CV.
__host__ __device__ constexpr int rec_quads(int m) { return m <= 3 ? 1 : (m + 4) / 4; }

// Device state of one instance. Decision vectors live in one row arena of
// `stride` floats per row (a multiple of 4, at least 4 nq, so that every row
// starts 16-byte aligned), in 2 + 2 npar regions of `region` rows: regions 0
// and 1 are the home rows of populations 1 and 2 (slot j at row j), region
// 2 + 2 s + q holds the offspring of population q written by a generation in
// slot s = gen_slot(k).
// A slot's current decision vector is the arena row loc[p][j]: a replaced slot
// points at its winning offspring row, so the replacement moves a 4-byte
// location instead of a row. F and CV of one individual share a record of
// rq = rec_quads(m) float4: objectives from the first lane, CV in the last
// lane, unused lanes 0. W rows have the same width.
struct DevState {
  int32_t n, m, d, stride, nblk;  // nblk: blocks of kBlock rows per population
  int32_t nq;                      // float4 chunks holding the d variables
  int32_t tasked;                  // variation kernel: 1 task-dealt, 0 lane groups
  int32_t task_off;                // task-dealt kernel: offspring per wave (8 to 64)
  int32_t rq;                      // float4 per F/CV record and per W row
  int32_t t[2];
  int32_t lps[2];                  // lanes per slot in k_select (power of two <= 64)
  int32_t sel_blocks0, sel_blocks1;  // k_select blocks of each population
  int32_t agg;
  float theta;
  float *rows;               // the row arena (2 + 2 npar regions)
  int64_t region;            // rows per region (nblk kBlock)
  int32_t npar;              // generations whose offspring rows stay in the arena
  // Write-set check (GMPEA_CHECK_WRITES=1 at init; null otherwise): per
  // generation, counts of the writes each target received, 4 arrays of 2 n
  // (population-major): offspring-row chunk writes (variation), offspring
  // record writes (OP1), slot records and locations written for a replacement,
  // and chunk copies of a kept row home plus its location (selection).
  int32_t *wcheck;
  float *X[2];               // home rows: regions 0 and 1
  uint32_t *loc[2];          // arena row of slot j's current decision vector
  float4 *FC[2], *FCO[2], *FCN[2];
  float4 *W;                 // unit direction (PBI) or raw weight (Tchebycheff)
  const int32_t *B[2];       // n x t_p
  // Reverse lists rev_p(j) = {i : j in B_p(i)}, ascending: the first t_p entries
  // of each list in a padded head (n x t_p, -1 after the list's end), the rest
  // (lists longer than t_p, a few percent of slots) in a CSR tail.
  const int32_t *rhead[2];   // n x t_p
  const int32_t *rtoff[2];   // tail offsets, n + 1
  const int32_t *rtail[2];   // tail entries
  uint8_t *src;              // OP1 switches: bit p set = population p took the other's offspring
                             // (also carried in the sign of FCN's CV, for k_select)
  uint32_t *zkey;            // ideal point as order-preserving keys (atomic min)
  uint32_t *gen;             // generations completed (k_op1 advances it once k_vary has read it)
  unsigned long long *repl;  // replaced-slot counters: kReplLanes per population, summed on read
  int32_t *mate[2];          // optional record of parent rows (n x 2)
  int32_t *win[2];           // optional record of winners (n)
  uint32_t key0, key1;       // RNG key
  uint64_t tpm, tpc;         // mutation / crossover thresholds floor(p 2^32)
  float inv_tpm;             // 1 / tpm
  float sbx_e;               // 1 / (eta_c + 1)
  float pm_p, pm_e;          // eta_m + 1, 1 / (eta_m + 1)
  int32_t op;                // 0: SBX then PM, 1: DE then PM
  float de_f;                // DE scale factor
  int32_t op1_rule;          // OP1 for population 1: 0 FPR, 1 feasibility first
  DevProblem prob;
};

// Launch geometry shared by host and device (plain and batched launches must
// agree on it, since it fixes the lane grouping and so the rounding order).
// Variation kernels, fixed per instance (plain and batched launches must agree,
// since the kernel fixes the evaluation's rounding order). Rows of at most
// kTaskChunks chunks (d <= 128) take the task-dealt kernel (a wave builds
// task_off offspring, its lanes dealt consecutive (offspring, chunk) tasks):
// every wave instruction moves about 1 KB of consecutive chunks, which keeps
// the variation at the same cost whether the parents' rows are shared by many
// slots (early generations, most slots replaced) or all distinct (later, most
// slots kept): 60-64 us against 55-77 us for lane groups at N = 100,128, and
// 445-454 against 536-804 us at N = 1,000,405. Longer rows take the lane-group
// kernel, vary_lanes_of_chunks(nq) lanes per offspring: enough that each lane
// keeps two to four float4 chunks, except the widest rows (d > 92), where four
// lanes of six or seven chunks each measured faster than eight.
// Offspring per wave of the task-dealt kernel. A wave's LDS holds kTaskPart
// floats: the off nq chunk partials and, for m <= 3, the two leading variables
// of each offspring, so off (nq + 2) <= kTaskPart (m > 3 keeps its two leading
// chunks apart, at most kTaskOffWide offspring). The count changes only how
// the tasks are dealt, never the results (each offspring's partials are added
// in chunk order whatever the dealing), so it follows the launch: the most that
// fit (full lanes in the per-offspring parts and in every step when nq <= 14)
// for a pool's batched launches and large plain populations, fewer for small
// plain populations (shorter dependency chains per wave when the chip has few
// waves).
constexpr int kTaskChunks = 32;
constexpr int kTaskPart = 1024;
constexpr int kTaskOffNarrow = 64, kTaskOffWide = 32;
__host__ __device__ inline int task_off_fit(int nq, bool wide) {
  int off = wide ? kTaskOffWide : kTaskOffNarrow;
  while (off > 8 && off * (nq + (wide ? 0 : 2)) > kTaskPart) off >>= 1;
  return off;
}
__host__ __device__ inline int task_off_for(int n, int nq, bool wide, bool pooled) {
  const int fit = task_off_fit(nq, wide);
  if (pooled) return fit;
  const int cap = n >= 65536 ? 64 : n >= 32768 ? 16 : 8;
  return fit < cap ? fit : cap;
}
__host__ __device__ inline int vary_lanes_of_chunks(int nq) {
  return nq >= 24 ? 4 : nq >= 16 ? 8 : nq >= 6 ? 4 : nq >= 3 ? 2 : 1;
}
__host__ __device__ inline bool vary_tasked(const DevState &st) { return st.tasked != 0; }
__host__ __device__ inline int vary_lanes_of(const DevState &st) {
  return vary_tasked(st) ? 1 : vary_lanes_of_chunks(st.nq);
}
// The arena holds the home rows of both populations, then the offspring rows
// of the last npar generations: generation k writes its offspring into the
// regions of slot k mod npar (one per population), so an offspring row stays
// valid for npar generations. A kept slot whose row would be overwritten by the
// next generation's offspring moves it home then; with npar slots that is a
// slot replaced npar - 1 generations ago and kept since.
constexpr int kOffspringGenerations = 8;
// One write recorded by the write-set check (a no-op unless it is on).
__device__ __forceinline__ void note_write(const DevState &st, int kind, int p, int j) {
  if (st.wcheck) atomicAdd(&st.wcheck[(2 * static_cast<int64_t>(kind) + p) * st.n + j], 1);
}
__host__ __device__ inline uint32_t gen_slot(const DevState &st, uint32_t k) {
  return k % static_cast<uint32_t>(st.npar);
}
// Arena row of offspring i of population q written by a generation in slot par.
__host__ __device__ inline uint32_t offspring_row(const DevState &st, uint32_t par, int q, int i) {
  return static_cast<uint32_t>((2 + 2 * static_cast<int64_t>(par) + q) * st.region + i);
}
// k_vary blocks of one instance (both populations).
__host__ __device__ inline int vary_blocks_of(int n, int lanes) {
  const int per = kBlock / lanes;
  return 2 * ((n + per - 1) / per);
}
// (the task-dealt kernel builds kBlock / 64 * task_off offspring per block)
__host__ __device__ inline int vary_grid(const DevState &st) {
  return vary_tasked(st) ? vary_blocks_of(st.n, 64 / st.task_off) : vary_blocks_of(st.n, vary_lanes_of(st));
}

// Launchers (gmpea_kernels.hip). Each enqueues on `s` and returns the launch status.
hipError_t launch_init(const DevState &st, hipStream_t s);
// A generation is kPhases launches: 0 variation + evaluation + ideal point,
// 1 offspring cooperation, 2 neighbour replacement decisions and the slots'
// locations (a replaced slot points at its winner's offspring row; a kept slot
// whose row the next generation's offspring would overwrite moves it home).
constexpr int kPhases = 3;
hipError_t launch_phase(const DevState &st, int phase, hipStream_t s);
// Point every slot of population `pop` at its home row (after the home rows were written).
hipError_t launch_loc_home(const DevState &st, int pop, hipStream_t s);
// Copy every slot's current decision vector to its home row and point it there.
hipError_t launch_materialize(const DevState &st, hipStream_t s);
hipError_t launch_generation(const DevState &st, hipStream_t s);
// One phase of a batched generation over a pool: work[b] = (instance, block).
// wide: the work list holds instances with m > 3 (their kernels are separate so
// that the m <= 3 kernels keep their register budget). sub: in phase 0, the
// work list holds instances of the task-dealt variation; in phase 2 with m <= 3,
// instances with m = 2 (the selection has a kernel per m); unused otherwise. A
// pool keeps one work list per kernel.
hipError_t launch_batch_phase(const DevState *states, const int2 *work, int nwork, int phase,
                              bool wide, bool sub, hipStream_t s);
// The m > 3 launchers (gmpea_kernels_wide.hip).
hipError_t launch_init_eval_wide(const DevState &st, hipStream_t s);
hipError_t launch_phase_wide(const DevState &st, int phase, hipStream_t s);
hipError_t launch_batch_phase_wide(const DevState *states, const int2 *work, int nwork, int phase,
                                   bool tasked, hipStream_t s);
hipError_t launch_front_flags_wide(const DevState &st, int pop, uint8_t *keep, hipStream_t s);
hipError_t launch_front_flags(const DevState &st, int pop, uint8_t *keep, hipStream_t s);
hipError_t launch_gather(const DevState &st, int pop, const int32_t *idx, int32_t count,
                         float *x, float4 *fc, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, int64_t n16, hipStream_t s);
// One-pass copy, four 16-byte words per thread (optionally non-temporal).
hipError_t launch_copy4(const void *src, void *dst, int64_t n16, bool nontemporal, hipStream_t s);
// Neighbourhoods of n rows of integer coordinates K (n x m, device): B1 (n x t1)
// and B2 (n x t2) receive each row's nearest rows by exact squared distance,
// ties by index. max_dist bounds every squared distance (it sets the digits of
// the radix select). max(t1, t2) must not exceed kKnnMaxTHost.
constexpr int kKnnMaxTHost = 256;
hipError_t launch_knn(const int32_t *K, int32_t n, int32_t m, uint64_t max_dist, int32_t t1, int32_t t2,
                      int32_t *B1, int32_t *B2, hipStream_t s);
// Front quality (Eqs. (14)-(15)) of `count` front records (rq float4 each).
// IGD: partial[b] receives the sum over block b's reference points of the
// distance to the nearest front point (n_ref x m reference rows, row-major).
// HV: *hits (zero on entry) receives how many of samples [0, n) drawn uniformly
// in the box [lo, hi] are weakly dominated by some front point.
hipError_t launch_igd(const float *ref, int32_t n_ref, int32_t m, const float4 *front, int32_t count,
                      int32_t rq, double *partial, int32_t *blocks, hipStream_t s);
hipError_t launch_hv(int64_t n, int32_t m, const float *lo, const float *hi, uint32_t k0, uint32_t k1,
                     const float4 *front, int32_t count, int32_t rq, unsigned long long *hits,
                     hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s);

// Order-preserving map between floats and unsigned keys (host copies of the
// device helpers, used to read and write the ideal point).
inline uint32_t float_key(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
inline float key_float(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

// Reference vectors and neighbourhoods (lattice.cpp).
int32_t dd_divisions(int32_t m, int64_t n_req);            // smallest H with count >= n_req
int64_t dd_count(int32_t m, int32_t H);                     // C(H + m - 1, m - 1)
void dd_lattice(int32_t m, int32_t H, std::vector<int32_t> &K);
void lattice_knn(const std::vector<int32_t> &K, int32_t m, int32_t H, int32_t t,
                 std::vector<int32_t> &B);
void reverse_lists(const std::vector<int32_t> &B, int32_t n, int32_t t, std::vector<int32_t> &off,
                   std::vector<int32_t> &idx);
// Leading-coordinate offsets (pairs; second component 0 for m = 2) sorted by
// (squared lattice distance, lexicographic order), enough for t neighbours of
// interior points; the device builds neighbourhoods by walking this list.
void neighbour_offsets(int32_t m, int32_t H, int32_t t, std::vector<int32_t> &d);
// Two-layer reference set (H2 > 0): the lattice k / H1, then the lattice k / H2
// moved halfway to the centroid, (k / H2 + 1 / m) / 2. K receives the rows as
// integers on the denominator 2 m H1 H2 (H1 for one layer) and W, if given, the
// FP64 vectors. refset_knn: the t nearest rows of each row by exact squared
// distance of those integers, ties by index (brute force, threaded).
int64_t refset_count(int32_t m, int32_t H1, int32_t H2);
void refset(int32_t m, int32_t H1, int32_t H2, std::vector<int32_t> &K, std::vector<double> *W);
void refset_knn(const std::vector<int32_t> &K, int32_t m, int32_t t, std::vector<int32_t> &B);
// Neighbourhoods of the reference set refset(m, H1, H2) built: the offset walk
// for one layer with m <= 3, else the brute force.
void refset_neighbours(const std::vector<int32_t> &K, int32_t m, int32_t H1, int32_t H2, int32_t t,
                       std::vector<int32_t> &B);

// Device construction of the initialisation tables (gmpea_kernels.hip).
// W and both neighbourhoods from the offset list; *incomplete becomes nonzero
// when some row found fewer than max(t1, t2) lattice neighbours in the list.
hipError_t launch_tables(int32_t m, int32_t n, int32_t H, const int2 *offs, int32_t noffs,
                         int32_t t1, int32_t t2, int32_t agg, float4 *W, int32_t *B1, int32_t *B2,
                         uint32_t *incomplete, hipStream_t s);
// Reverse lists of B (n x t). launch_reverse_count: cursor (n + ceil((n + 1) /
// 1024) entries, the first n zero on entry; the rest is scratch of the scan)
// receives each list's length and toff (n + 1, zero on entry) the exclusive
// scan of the lengths in excess of t, so toff[n] is the tail size.
// launch_reverse_fill: head (n x t) and tail (cap entries) receive the lists,
// each ascending (cursor must be zero again); when the tail needs more than cap
// entries, *overflow becomes nonzero and the lists are incomplete.
hipError_t launch_reverse_count(int32_t n, int32_t t, const int32_t *B, int32_t *cursor,
                                int32_t *toff, hipStream_t s);
hipError_t launch_reverse_fill(int32_t n, int32_t t, const int32_t *B, const int32_t *toff,
                               int32_t *cursor, int32_t *head, int32_t *tail, int32_t cap,
                               uint32_t *overflow, hipStream_t s);

// Several device spans set to a 32-bit pattern by one launch (initialisation
// clears about twenty buffers; one hipMemsetAsync each took a launch and an
// API call apiece). Each span is p[k] .. p[k] + words[k] (32-bit words, p[k]
// 4-byte aligned); spans must not overlap.
constexpr int kMaxFillSpans = 24;
struct FillSpans {
  uint32_t *p[kMaxFillSpans];
  uint64_t words[kMaxFillSpans];
  uint32_t value[kMaxFillSpans];
  int32_t count;
};
hipError_t launch_fill(const FillSpans &f, hipStream_t s);

}  // namespace gmpea
