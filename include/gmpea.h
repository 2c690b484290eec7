/*
 * gmpea.h — C ABI of the MI355X (gfx950) GMPEA library.
 *
 * GMPEA is the decomposition-based, two-population constrained multiobjective
 * evolutionary algorithm of Huang et al., arXiv 2509.19821. One generation
 * (Alg. 1 loop body and Alg. 2) runs on the GPU for every subproblem of both
 * populations: neighbourhood mating, SBX + polynomial mutation, evaluation of
 * F and CV, the ideal-point update, OP1 offspring cooperation and the OP2/OP3
 * constraint-aware neighbour replacement.
 *
 * Conventions shared by every call:
 *  - Every call returns gmpea_status; no exception crosses the ABI. On an
 *    error, outputs are left unchanged and gmpea_last_error() explains.
 *  - Host pointers are plain C arrays owned by the caller. Device memory is
 *    owned by the handle and obtained through the caller's allocator hook
 *    (hipMalloc when none is given).
 *  - The device computes in FP32; FP64 problem constants are rounded once.
 *  - Population rows are in ascending subproblem order. Subproblem i is the
 *    i-th reference vector: the Das-Dennis lattice in lexicographic order, or
 *    for a two-layer set (gmpea_config.h_outer / h_inner) the outer layer's
 *    lattice followed by the inner layer's.
 *  - A handle is used by one host thread at a time; separate handles are
 *    independent and may share a stream.
 */
#ifndef GMPEA_H
#define GMPEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmpea_s *gmpea_t; /* opaque; owns the device memory of one instance */
typedef struct gmpea_pool_s *gmpea_pool_t; /* opaque; a set of resident instances */

typedef enum {
  GMPEA_OK = 0,
  GMPEA_EINVAL = -1,      /* invalid argument (sizes, bounds, NULL where required) */
  GMPEA_ENOMEM = -2,      /* the allocator hook (or hipMalloc) returned no memory */
  GMPEA_EHIP = -3,        /* a HIP runtime call failed */
  GMPEA_ECAPACITY = -4,   /* an output buffer is too small; *count holds the need */
  GMPEA_ESTATE = -5,      /* handle destroyed or not in a usable state */
  GMPEA_EUNSUPPORTED = -6 /* valid request outside what the library implements */
} gmpea_status;

/* Reproduction operators (the experimental settings name both). GMPEA_OP_DE
 * reads the DE operator (CR = 1, F = 0.5) in its neighbourhood form: for
 * subproblem i of population p, v = x_i + F (x_a - x_b) with x_i the current
 * solution and (a, b) the two mating picks from B_p(i), every variable taken
 * from the mutant (CR = 1), clipped to the box, then polynomial mutation as
 * after SBX. */
enum { GMPEA_OP_SBX = 0, GMPEA_OP_DE = 1 };

/* Problem families (objective functions of the synthetic CMOPs). */
enum {
  GMPEA_FAMILY_CURVE = 0, /* m = 2: f1 = x1, g = 1 + 9 mean(x2..xd), f2 = g (1 - sqrt(f1/g)) */
  GMPEA_FAMILY_SPHERE = 1 /* 2 <= m <= GMPEA_MAX_M, d >= m - 1: with angles
                             th_l = pi x_l / 2 (l < m - 1) and g = sum_{l >= m-1}
                             (x_l - 0.5)^2 (0-based l), f_k = (1 + g) prod_{j <
                             m-1-k} cos th_j, times sin th_{m-1-k} for k > 0 */
};

/* Aggregation (Eq. (7) and its Tchebycheff alternative named beside it). */
enum {
  GMPEA_AGG_PBI = 0, /* d1 + theta d2 with a unit reference direction; theta = 5 by default */
  GMPEA_AGG_TCHE = 1 /* max_k w_k |f_k - z_k| */
};

/* What gmpea_front returns. */
enum {
  GMPEA_FRONT_FEASIBLE_ND = 0, /* feasible (CV = 0) non-dominated rows of population 1 (Eq. (5)) */
  GMPEA_FRONT_POP1 = 1,        /* every row of population 1 (the output of Alg. 1) */
  GMPEA_FRONT_POP2 = 2         /* every row of population 2 */
};

/* Buffers reachable through gmpea_read / gmpea_write. Host layouts:
 *   X      N x d  float   decision vectors of population `pop`
 *   F      N x m  float   objectives
 *   CV     N      float   total constraint violation (Eq. (3))
 *   XOFF, FOFF, CVOFF     the last generation's offspring of population `pop`
 *                         (before OP1), same layouts; read only. Defined once
 *                         this handle has run a generation (zeros before the
 *                         first; after a write of GEN, until the next one, the
 *                         offspring rows are unspecified)
 *   Z      m      float   ideal point (shared by both populations); pop ignored
 *   GEN    1      int64   generations completed; pop ignored
 *   W      N x m  float   reference vectors, the raw weights (read only; pop ignored)
 *   B      N x t  int32   neighbourhood of population `pop` (read only)
 *   MATE   N x 2  int32   last generation's parent rows of population `pop`
 *   OP1    N      uint8   1 if population `pop`'s new offspring i came from the
 *                         other population in OP1 (Eq. (11))
 *   WIN    N      int32   last generation's winner per parent slot (offspring
 *                         index, -1 = parent kept)
 *   MATE and WIN exist only when gmpea_config.record is nonzero. */
enum {
  GMPEA_BUF_X = 0,
  GMPEA_BUF_F = 1,
  GMPEA_BUF_CV = 2,
  GMPEA_BUF_XOFF = 3,
  GMPEA_BUF_FOFF = 4,
  GMPEA_BUF_CVOFF = 5,
  GMPEA_BUF_Z = 6,
  GMPEA_BUF_GEN = 7,
  GMPEA_BUF_W = 8,
  GMPEA_BUF_B = 9,
  GMPEA_BUF_MATE = 10,
  GMPEA_BUF_OP1 = 11,
  GMPEA_BUF_WIN = 12
};

#define GMPEA_MAX_M 8     /* objectives the library supports */
#define GMPEA_MAX_RING 8  /* ring constraints the library supports */

/* A CMOP instance (Eq. (1)): minimise F(x) over the box [lb, ub]^d subject to
 *   ring:     r_j^2 - ||F(x) - a_j||^2 <= 0          (j < n_ring)
 *   linear:   sum_lower - sum_k f_k(x) <= 0         (if has_sum_lower)
 *   equality: x1 + x2 - 1 = 0, violation max(0, |h| - eq_tol)  (if n_eq = 1; Eq. (2))
 * CV is the sum of the violations (Eq. (3)). All pointers are host memory,
 * read during gmpea_init only. */
typedef struct {
  int32_t family, m, d;
  const double *lb, *ub;      /* d each; NULL means [0, 1]^d; need lb < ub */
  int32_t n_ring;             /* 0 .. GMPEA_MAX_RING */
  const double *ring_center;  /* n_ring x m, row-major */
  const double *ring_radius;  /* n_ring */
  int32_t has_sum_lower;
  double sum_lower;
  int32_t n_eq;               /* 0 or 1 */
  double eq_tol;              /* delta of Eq. (2); the paper's typical value is 1e-6 */
} gmpea_problem;

/* Method parameters (Alg. 1 inputs and the experimental settings). Zero means
 * the paper's default where one exists. */
typedef struct {
  int32_t n_req;   /* requested reference vectors per population; the library uses
                      the smallest Das-Dennis count N >= n_req (needs n_req >= 2
                      unless h_outer is set) */
  int32_t T;       /* base neighbourhood size: t1 = T/2, t2 = 2T unless set below */
  int32_t t1, t2;  /* population 1 (small) and population 2 (large) neighbourhoods */
  int32_t agg;     /* GMPEA_AGG_PBI (default) or GMPEA_AGG_TCHE */
  double theta;    /* PBI penalty; 0 means 5 */
  double eta_c;    /* SBX distribution index; 0 means 20 */
  double eta_m;    /* PM distribution index; 0 means 20 */
  double pc;       /* SBX probability per offspring; 0 means 1 */
  double pm;       /* PM probability per variable; 0 means 1/d */
  uint64_t seed;   /* key of the counter RNG: every random draw is a function of
                      (seed, generation, population, subproblem, variable) */
  int32_t record;  /* nonzero: keep MATE and WIN of the last generation */
  int32_t op;      /* reproduction: GMPEA_OP_SBX (SBX then PM, the C-DTLZ / DC-DTLZ
                      setting) or GMPEA_OP_DE (DE then PM, the LIR-CMOP setting) */
  double de_f;     /* DE scale factor F; 0 means 0.5 (the crossover rate is 1) */
  int32_t op1_rule; /* population 1's test in offspring cooperation (OP1):
                       GMPEA_OP1_FPR (Alg. 2: lower CV, then lower aggregation) or
                       GMPEA_OP1_FEASIBLE_FIRST (its prose: a feasible offspring
                       wins, otherwise the lower aggregation) */
  int32_t h_outer;  /* > 0: the reference set is given by layers instead of n_req
                       (the paper names many objectives as future work and fixes
                       no set for them): the Das-Dennis lattice k / h_outer ... */
  int32_t h_inner;  /* ... followed, when > 0, by the lattice k / h_inner moved
                       halfway to the centroid, (k / h_inner + 1 / m) / 2. Then
                       N = C(h_outer + m - 1, m - 1) + C(h_inner + m - 1, m - 1)
                       and neighbourhoods use exact distances of the vectors as
                       integers over 2 m h_outer h_inner. They are searched
                       exactly on the device (about 0.2 s at N = 1e5; a host
                       search when max(t1, t2) > 256). */
} gmpea_config;

enum { GMPEA_OP1_FPR = 0, GMPEA_OP1_FEASIBLE_FIRST = 1 };

/* Device allocator hook. alloc returns device memory (or NULL), free releases
 * it; ctx is passed through. A handle frees everything it allocated with the
 * same hook. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} gmpea_allocator;

typedef struct {
  int32_t n;          /* N, rows per population */
  int32_t m, d;
  int32_t t1, t2;
  int32_t H;          /* Das-Dennis divisions (of the outer layer) */
  int32_t H2;         /* inner layer's divisions, 0 for one layer */
  int64_t generation; /* generations completed */
  float z[GMPEA_MAX_M];
  int64_t replaced[2];   /* parent slots replaced, summed over all generations */
  double feasible_frac;  /* share of population 1 with CV = 0 */
  size_t device_bytes;   /* device memory held by the handle */
  int32_t task_dealt;    /* variation kernel: 1 task-dealt (rows of d <= 128), 0 lane groups */
  int64_t checked_generations; /* generations whose write sets were verified (GMPEA_CHECK_WRITES=1) */
} gmpea_info;

/* Create an instance: build the reference vectors W (Das-Dennis lattice), the
 * neighbourhoods B1/B2 (t nearest reference vectors, self first, ties by index)
 * and their reverse lists, draw the two initial populations uniformly in the box,
 * evaluate them and set the ideal point to their minimum (Alg. 1 initialisation).
 * hip_stream: a hipStream_t, or NULL for a stream owned by the handle. Work is
 * enqueued on that stream; the call returns once the handle is ready.
 * The HIP runtime in the process must be at least as new as the HIP toolchain
 * the library was built with; otherwise EUNSUPPORTED (nothing is launched).
 * With m > 3 the F/CV records and W rows take two or three float4 instead of
 * one, and the generation runs kernels instantiated for that m.
 * Every device buffer the handle will use is allocated here, including the
 * scratch of gmpea_front and gmpea_quality, so no later call on the handle
 * allocates device memory (a pool's admission reserves the whole footprint).
 * Errors: EINVAL (bad sizes: m, d < 2 for the curve family, lb >= ub, t > N,
 * n_ring out of range, h_inner without h_outer, ...), EUNSUPPORTED
 * (m > GMPEA_MAX_M), ENOMEM, EHIP. */
gmpea_status gmpea_init(const gmpea_problem *problem, const gmpea_config *config,
                        const gmpea_allocator *allocator, void *hip_stream, gmpea_t *out);

/* Enqueue n_gen generations (Alg. 1 loop body) on the handle's stream and
 * return without waiting. Runs of 64 generations replay one captured hipGraph
 * (the environment variable GMPEA_GRAPH_CHUNK sets another length, below 2 none);
 * n_gen = 0 launches nothing but captures that graph ahead of time, so a timed
 * region need not include the capture. Errors: EINVAL (n_gen < 0), EHIP. */
gmpea_status gmpea_step(gmpea_t h, int32_t n_gen);

/* Run up to max_gen generations, stopping at the first generation boundary at
 * or after time_limit_s seconds of wall time (the fixed-time comparison of the
 * experimental setup, Sec. IV-C, used for the runtime analysis of Sec. V-B;
 * <= 0 means no limit), then synchronise. *gens_done (may be NULL) receives the
 * generations run by this call. A limit already reached runs none. */
gmpea_status gmpea_run(gmpea_t h, int32_t max_gen, double time_limit_s, int32_t *gens_done);

/* Copy rows of the current populations to the host (synchronises). For
 * GMPEA_FRONT_FEASIBLE_ND: the feasible rows of population 1 that no other
 * feasible row dominates (Eq. (5)); identical objective vectors are all kept.
 * x: capacity x d, f: capacity x m, cv: capacity, idx: capacity (subproblem
 * indices, ascending); any of them may be NULL. *count receives the row count;
 * if it exceeds capacity nothing is copied and ECAPACITY is returned. */
gmpea_status gmpea_front(gmpea_t h, int32_t what, int32_t capacity, float *x, float *f,
                         float *cv, int32_t *idx, int32_t *count);

/* gmpea_front for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid it):
 * the same rows, values and errors, computed by the same kernels, with every
 * device buffer the extraction needs (flags, row list, gathered F/CV records
 * and decision vectors) in one fixed 32 MiB scratch array of the library,
 * which each GPU it runs on holds until the process ends. Calls nothing that
 * allocates device memory. The scratch must hold n (5 + 16 rq) + 4 d bytes
 * (256-byte aligned parts; rq = 1 for m <= 3, (m + 4) / 4 above), about 1.5
 * million rows for m <= 3; a larger population returns EUNSUPPORTED before any
 * work. Decision vectors are copied out in passes of as many rows as the rest
 * of the scratch holds. Every call on one GPU shares that GPU's scratch: calls
 * that overlap in time on one GPU (from several host threads) race and must
 * not be made; consecutive calls are safe, since each call synchronises. */
gmpea_status gmpea_front_static(gmpea_t h, int32_t what, int32_t capacity, float *x, float *f,
                                float *cv, int32_t *idx, int32_t *count);

/* Quality of the current front on the device: the feasible non-dominated rows
 * of population 1 (as GMPEA_FRONT_FEASIBLE_ND), measured by IGD (Eq. (14)) and
 * HV (Eq. (15)) without copying the front to the host. Synchronises.
 *  igd (may be NULL): mean over the n_ref reference points ref (n_ref x m,
 *    host, row-major) of the Euclidean distance to the nearest front point;
 *    distances in FP32, their sum in FP64 in a fixed order (reproducible).
 *  hv (may be NULL): Monte Carlo estimate of the volume weakly dominated by the
 *    front and bounded by hv_point (m host floats): hv_samples points uniform
 *    in the box from the front's per-objective minimum to hv_point, drawn from
 *    the library's Philox4x32-10 keyed by hv_seed (sample s takes blocks
 *    (s mod 2^32, s >> 32, 0 and 1, 4 << 24), words in objective order, u as
 *    in the method's draws); hv = box volume x covered share. Its standard
 *    error is box volume x sqrt(p (1 - p) / hv_samples).
 *  front_count (may be NULL): the front's row count. An empty front gives
 *    igd = +inf and hv = 0.
 * Errors: ESTATE, EINVAL (igd without ref or n_ref < 1; hv without hv_point,
 * a non-finite hv_point or hv_samples outside [1, 2^34]), ENOMEM, EHIP. */
gmpea_status gmpea_quality(gmpea_t h, const float *ref, int32_t n_ref, const float *hv_point,
                           int64_t hv_samples, uint64_t hv_seed, double *igd, double *hv,
                           int32_t *front_count);

/* Wait until every generation enqueued on the handle's stream has finished. */
gmpea_status gmpea_sync(gmpea_t h);

/* Sizes, generation count, ideal point and counters (synchronises). */
gmpea_status gmpea_get_info(gmpea_t h, gmpea_info *info);

/* Sizes of an instance (any output may be NULL): N per population, m, d and
 * the two neighbourhood sizes. Host-side only: no device access and no wait,
 * so it may be called while generations are in flight. */
gmpea_status gmpea_shape(gmpea_t h, int32_t *n, int32_t *m, int32_t *d, int32_t *t1, int32_t *t2);

/* Copy a buffer (see GMPEA_BUF_*) to host memory of `count` elements of its
 * host type; count must equal the buffer's element count. Synchronises. */
gmpea_status gmpea_read(gmpea_t h, int32_t buffer, int32_t pop, void *host, int64_t count);

/* Overwrite X, F, CV (of population `pop`), Z or GEN from host memory, e.g. to
 * resume from a checkpoint taken with gmpea_read: since every random draw is a
 * function of (seed, generation, ...), restoring X, F, CV of both populations,
 * Z and GEN resumes the run bit-exactly. Synchronises. Other buffers: EINVAL. */
gmpea_status gmpea_write(gmpea_t h, int32_t buffer, int32_t pop, const void *host,
                         int64_t count);

/* Release the handle and its device memory (waits for its work). NULL is a no-op. */
void gmpea_destroy(gmpea_t h);

/* Message of the last error on this host thread (library-owned string). */
const char *gmpea_last_error(void);

/* Run n_gen generations one launch at a time with HIP events recorded on the
 * handle's stream around every kernel, and return each kernel's mean duration in
 * milliseconds: ms[0] variation + evaluation + ideal point, ms[1] offspring
 * cooperation (OP1), ms[2] neighbour replacement decisions (OP2 + OP3) with the
 * slots' new locations; then ms[3]: the variation kernel timed over n_gen
 * launches back to back between two events (repeated, it rewrites the same
 * offspring of the same generation), which leaves out the per-launch event
 * overhead (ms holds 4 floats). The generations are real (the state advances
 * by n_gen). Synchronises. */
gmpea_status gmpea_profile(gmpea_t h, int32_t n_gen, float *ms);

/* The counter RNG every draw of the method uses (the paper names none):
 * Philox4x32-10 of Salmon et al. (SC'11). n blocks: out[4i..4i+3] =
 * Philox(ctr[4i..4i+3], key = (seed low word, seed high word)). ctr and out are
 * device pointers; the call enqueues on hip_stream (NULL: legacy default) and
 * synchronises. */
gmpea_status gmpea_philox(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out,
                          void *hip_stream);

/* Reference vectors and neighbourhoods of Alg. 1 ("uniform reference vectors"
 * and "neighbours initialization"), computed on the host with no GPU work, as
 * gmpea_init builds them. H is the smallest number of divisions whose
 * Das-Dennis count C(H + m - 1, m - 1) reaches n_req, and N is that count.
 * K (N x m, row-major, caller-owned; may be NULL): the lattice rows k with
 * k_1 + ... + k_m = H in ascending lexicographic order of (k_1 .. k_{m-1});
 * the reference vectors are W = K / H. B (N x t, caller-owned; may be NULL):
 * for each row i the t rows nearest by squared lattice distance, ties by
 * ascending index, so row i itself comes first. *H_out and *n_out (may be
 * NULL) receive H and N. EINVAL for m outside [2, GMPEA_MAX_M], n_req < 2 or
 * t outside [1, N]; ECAPACITY (with *n_out set) when cap_rows < N and K or B
 * is given. */
gmpea_status gmpea_lattice(int32_t m, int32_t n_req, int32_t t, int32_t cap_rows, int32_t *K,
                           int32_t *B, int32_t *H_out, int32_t *n_out);

/* The layered reference set of gmpea_config.h_outer / h_inner (many
 * objectives) and its neighbourhoods, on the host with no GPU work, as
 * gmpea_init builds them. K (N x m, caller-owned; may be NULL): the vectors as
 * integers over the denominator 2 m h_outer h_inner (h_outer for one layer),
 * the outer layer's rows first, each layer in ascending lexicographic order.
 * B (N x t; may be NULL): for each row the t rows nearest by exact squared
 * distance, ties by ascending index (a row is first in its own list unless an
 * earlier row holds the same vector). *n_out (may be NULL) receives N. EINVAL
 * for m outside [2, GMPEA_MAX_M], h_outer < 1, h_inner < 0 or t outside
 * [1, N]; ECAPACITY (with *n_out set) when cap_rows < N and K or B is given. */
gmpea_status gmpea_reference_set(int32_t m, int32_t h_outer, int32_t h_inner, int32_t t,
                                 int32_t cap_rows, int32_t *K, int32_t *B, int32_t *n_out);

/* ---------------------------------------------------------------------------
 * Pools: many independent instances (uneven N, d, m, constraint counts) stay
 * resident on the device and advance together. A batched generation is one
 * launch per phase over every active instance; each instance computes exactly
 * what it computes alone (same kernels, lane grouping and random streams), so
 * results are bit-identical to gmpea_step on that instance by itself.
 * ------------------------------------------------------------------------- */

/* Create a pool that may reserve at most budget_bytes of device memory in
 * total, for its instances and its own tables. Memory is reserved in chunks of
 * up to 256 MiB from the allocator hook (or hipMalloc) as instances are
 * admitted, carved into blocks, and recycled when instances are released; the
 * chunks are returned only by gmpea_pool_destroy. hip_stream: the stream every
 * instance of the pool uses, or NULL for one the pool owns. The pool also holds
 * a pinned host buffer (4 MiB, more for very large pools) that stages its work
 * lists, and at creation copies it once into a transient 4 MiB device block
 * (from the hook, if one is given) so that the copy path is set up before the
 * first generation. */
gmpea_status gmpea_pool_create(size_t budget_bytes, const gmpea_allocator *allocator,
                               void *hip_stream, gmpea_pool_t *out);

/* Initialise an instance inside the pool (as gmpea_init) and return its slot.
 * The initialisation runs on a stream of the pool's own, so generations already
 * enqueued keep running; the instance then uses the pool's stream. ENOMEM when
 * its footprint does not fit the remaining budget (nothing is kept). */
gmpea_status gmpea_pool_admit(gmpea_pool_t pool, const gmpea_problem *problem,
                              const gmpea_config *config, int32_t *slot);

/* Enqueue n_gen batched generations of every active instance; asynchronous. */
gmpea_status gmpea_pool_step(gmpea_pool_t pool, int32_t n_gen);

/* Run n_gen batched generations while choosing the launch schedule (instance
 * blocks grouped per XCD or in order) and the launch form (hipGraph replays of
 * 16 or 64 generations, or one launch per phase without a graph) by timing the
 * first generations; the choice stays for later steps. Results do not depend
 * on it. The candidates run back to back and are waited for once; the
 * generations after them are enqueued asynchronously. *gens_done (may be NULL)
 * receives the generations run or enqueued. */
gmpea_status gmpea_pool_tune(gmpea_pool_t pool, int32_t n_gen, int32_t *gens_done);

/* The handle of a slot, for gmpea_front, gmpea_read, gmpea_write,
 * gmpea_get_info and gmpea_step on that instance alone. The pool owns it: do
 * not pass it to gmpea_destroy (use gmpea_pool_release). */
gmpea_status gmpea_pool_handle(gmpea_pool_t pool, int32_t slot, gmpea_t *handle);

/* Free a slot and its device memory (waits for the pool's work). */
gmpea_status gmpea_pool_release(gmpea_pool_t pool, int32_t slot);

/* Active instances, device bytes in use and the budget, and the launch policy
 * (schedule 0: OP1 and selection blocks grouped per XCD, variation blocks
 * in order; 1: every phase in order; graph chunk length). Any output
 * may be NULL. */
gmpea_status gmpea_pool_query(gmpea_pool_t pool, int32_t *active, size_t *used_bytes,
                              size_t *budget_bytes, int32_t *schedule, int32_t *chunk);

/* Wait for all work enqueued on the pool's stream. */
gmpea_status gmpea_pool_sync(gmpea_pool_t pool);

/* Release every instance and the pool. NULL is a no-op. */
void gmpea_pool_destroy(gmpea_pool_t pool);

/* Streaming device-to-device copy of `bytes` (a multiple of 16; both pointers
 * 16-byte aligned device memory) with the library's own kernel: every byte read
 * once and written once. It serves as the reference for measured bandwidth and
 * for calibrating hardware byte counters against a known transfer. Enqueues on
 * hip_stream (NULL: legacy default) and synchronises. */
gmpea_status gmpea_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* Copy forms timed by gmpea_copy_probe. */
enum {
  GMPEA_COPY_STRIDED = 0, /* gmpea_copy's kernel: at most 4,096 blocks striding, 16 B per step */
  GMPEA_COPY_WIDE = 1,    /* one pass, four 16-byte words per thread, loads before stores */
  GMPEA_COPY_WIDE_NT = 2, /* the same with non-temporal loads and stores */
  GMPEA_COPY_RUNTIME = 3  /* the HIP runtime's hipMemcpyAsync device to device */
};

/* Attainable device-memory bandwidth, for the roofline's measured ceiling:
 * times `reps` copies (after one untimed) of `bytes` (a multiple of 16, > 0;
 * both pointers 16-byte aligned device memory, not overlapping) in one of the
 * forms above with HIP events on hip_stream (NULL: legacy default); *ms
 * receives the fastest copy's time in milliseconds (bandwidth = 2 bytes / time).
 * EINVAL for bad arguments or mode; EHIP for a runtime failure. Synchronises. */
gmpea_status gmpea_copy_probe(const void *src, void *dst, size_t bytes, int32_t mode,
                              int32_t reps, void *hip_stream, float *ms);

#ifdef __cplusplus
}
#endif

#endif /* GMPEA_H */
