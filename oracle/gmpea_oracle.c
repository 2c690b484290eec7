/*
 * GMPEA CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of one GMPEA generation (Huang et al.,
 * "Fully Tensorized GPU-accelerated Multi-population Evolutionary Algorithm for
 * Constrained Multiobjective Optimization Problems", arXiv 2509.19821).
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library. The product path (the HIP library) never links it, and
 * this file shares no code, header or table with the product path.
 *
 * Every function cites the passage of the paper it follows. Where the paper is
 * silent, the reading taken is stated where it applies and tagged R<n>; the same
 * tag marks the same reading in the kernels and the tests.
 *
 * Plain loops throughout; OpenMP only spreads independent subproblems over
 * threads (results are identical for any thread count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel Random Numbers: */
/* As Easy as 1, 2, 3"). The paper under test names no generator; R5 fixes it. */
/* ------------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

/* Stream tags (top byte of counter word 3) — R5. */
#define ORC_TAG_INIT 1u
#define ORC_TAG_MATE 2u
#define ORC_TAG_VAR 3u

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += ORC_PHILOX_W0;
    k1 += ORC_PHILOX_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out) {
  for (int64_t i = 0; i < n; ++i) orc_philox(ctr + 4 * i, key, out + 4 * i);
}

/* Counter layout (R5): (c0, c1 = subproblem i, c2 = generation k, c3 = tag<<24 | pop<<16). */
static void orc_draw(uint32_t c0, uint32_t i, uint32_t k, uint32_t tag, uint32_t pop,
                     const uint32_t key[2], uint32_t out[4]) {
  uint32_t ctr[4] = {c0, i, k, (tag << 24) | (pop << 16)};
  orc_philox(ctr, key, out);
}

/* U = (w >> 8) * 2^-24: exact in FP32 and FP64 (R5). */
static double orc_u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------------- */
/* Uniform reference vectors W (Alg. 1 input "uniform reference vectors"):     */
/* Das-Dennis simplex lattice, R1: H is the smallest value with                */
/* C(H+m-1, m-1) >= requested N; rows enumerate k in N^m with sum H in          */
/* ascending lexicographic order of (k_1..k_{m-1}).                             */
/* ------------------------------------------------------------------------- */
int64_t orc_dd_count(int32_t m, int32_t H) {
  /* C(H+m-1, m-1) by the multiplicative formula; exact for the sizes used. */
  long double c = 1.0L;
  for (int32_t j = 1; j <= m - 1; ++j) c = c * (long double)(H + j) / (long double)j;
  return (int64_t)(c + 0.5L);
}

int32_t orc_dd_H(int32_t m, int64_t n_req) {
  int32_t H = 1;
  while (orc_dd_count(m, H) < n_req) ++H;
  return H;
}

static int64_t orc_dd_fill(int32_t m, int32_t pos, int32_t left, int32_t *cur, int32_t *K,
                           int64_t row) {
  if (pos == m - 1) {
    cur[pos] = left;
    for (int32_t a = 0; a < m; ++a) K[row * m + a] = cur[a];
    return row + 1;
  }
  for (int32_t v = 0; v <= left; ++v) {
    cur[pos] = v;
    row = orc_dd_fill(m, pos + 1, left - v, cur, K, row);
  }
  return row;
}

/* K: count x m integer lattice (rows of W are K/H). Returns the row count. */
int64_t orc_dd_lattice(int32_t m, int32_t H, int32_t *K) {
  int32_t cur[64];
  if (m < 1 || m > 64) return -1;
  return orc_dd_fill(m, 0, H, cur, K, 0);
}

/* ------------------------------------------------------------------------- */
/* Neighbourhoods B_p (Alg. 1 "Neighbours initialization"; sizes t1 = T/2 and  */
/* t2 = 2T from the parameter settings). R2: B(i) holds the t indices j with   */
/* the smallest (sum_a (k_i,a - k_j,a)^2, j) — exact integer lattice distance, */
/* ties by ascending index; self (distance 0) comes first. Brute force O(N^2). */
/* ------------------------------------------------------------------------- */
int32_t orc_knn(const int32_t *K, int64_t N, int32_t m, int32_t t, int32_t *B) {
  if (t < 1 || t > N) return -1; /* a neighbourhood cannot exceed the population */
#pragma omp parallel
  {
    int64_t *bd = (int64_t *)malloc(sizeof(int64_t) * (size_t)t);
    int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)t);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
      int32_t cnt = 0;
      for (int64_t j = 0; j < N; ++j) {
        int64_t dist = 0;
        for (int32_t a = 0; a < m; ++a) {
          int64_t df = (int64_t)K[i * m + a] - (int64_t)K[j * m + a];
          dist += df * df;
        }
        /* keep the t smallest (dist, j); j ascends so an equal dist never displaces */
        if (cnt == t && dist >= bd[t - 1]) continue;
        int32_t pos = (cnt < t) ? cnt : t - 1;
        while (pos > 0 && bd[pos - 1] > dist) {
          bd[pos] = bd[pos - 1];
          bj[pos] = bj[pos - 1];
          --pos;
        }
        bd[pos] = dist;
        bj[pos] = (int32_t)j;
        if (cnt < t) ++cnt;
      }
      for (int32_t r = 0; r < t; ++r) B[i * t + r] = bj[r];
    }
    free(bd);
    free(bj);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Problems. The CMOP statement (Eq. (1)): minimise F subject to g <= 0 and    */
/* h = 0. Violations follow Eq. (2), the total CV Eq. (3).                     */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t family; /* 0: curve (m = 2), 1: sphere (m >= 2) */
  int32_t m, d;
  const double *lb, *ub;
  int32_t n_ring;
  const double *ring_center; /* n_ring x m */
  const double *ring_radius; /* n_ring */
  int32_t has_sum_lower;
  double sum_lower;
  int32_t n_eq;
  double eq_tol;
} orc_problem;

/* Objectives of one decision vector.
 * family 0 (two objectives): f1 = x1, g = 1 + 9 mean(x2..xd), f2 = g (1 - sqrt(f1 / g)).
 * family 1 (R9, sphere): g = sum_{l >= m} (x_l - 0.5)^2, angles pi x_l / 2 for l < m,
 *   f_1 = (1+g) prod cos, f_k = (1+g) prod_{j < m-k} cos(th_j) sin(th_{m-k}). */
static void orc_objectives(const orc_problem *P, const double *x, double *f) {
  const int32_t m = P->m, d = P->d;
  if (P->family == 0) {
    double s = 0.0;
    for (int32_t l = 1; l < d; ++l) s += x[l];
    double g = 1.0 + 9.0 * s / (double)(d - 1);
    f[0] = x[0];
    f[1] = g * (1.0 - sqrt(x[0] / g));
    return;
  }
  double g = 0.0;
  for (int32_t l = m - 1; l < d; ++l) g += (x[l] - 0.5) * (x[l] - 0.5);
  const double hp = 1.5707963267948966; /* pi / 2 */
  for (int32_t k = 0; k < m; ++k) {
    double v = 1.0 + g;
    for (int32_t j = 0; j < m - 1 - k; ++j) v *= cos(hp * x[j]);
    if (k > 0) v *= sin(hp * x[m - 1 - k]);
    f[k] = v;
  }
}

/* Constraint values c (<= 0 means satisfied) for one individual, in order:
 * rings r_j^2 - ||F - a_j||^2, then the linear bound sum_lower - sum F, then the
 * equality |x1 + x2 - 1| - tol (Eq. (2) turns h = 0 into |h| - delta <= 0).
 * Returns CV = sum max(0, c) (Eq. (3)); *cmax gets the largest objective-space
 * constraint value (rings, linear bound; -inf when there are none). */
static double orc_constraints(const orc_problem *P, const double *x, const double *f,
                              double *cmax) {
  const int32_t m = P->m;
  double cv = 0.0, mx = -INFINITY;
  for (int32_t j = 0; j < P->n_ring; ++j) {
    double s = 0.0;
    for (int32_t k = 0; k < m; ++k) {
      double df = f[k] - P->ring_center[j * m + k];
      s += df * df;
    }
    double c = P->ring_radius[j] * P->ring_radius[j] - s;
    cv += (c > 0.0) ? c : 0.0;
    if (c > mx) mx = c;
  }
  if (P->has_sum_lower) {
    double s = 0.0;
    for (int32_t k = 0; k < m; ++k) s += f[k];
    double c = P->sum_lower - s;
    cv += (c > 0.0) ? c : 0.0;
    if (c > mx) mx = c;
  }
  if (P->n_eq) {
    double c = fabs(x[0] + x[1] - 1.0) - P->eq_tol;
    cv += (c > 0.0) ? c : 0.0;
  }
  if (cmax) *cmax = mx;
  return cv;
}

/* Evaluation of n individuals (Alg. 1 "evaluate objectives and constraints"). */
void orc_eval(const orc_problem *P, int64_t n, const double *X, double *F, double *CV,
              double *CMAX) {
  for (int64_t i = 0; i < n; ++i) {
    orc_objectives(P, X + i * P->d, F + i * P->m);
    double cm;
    CV[i] = orc_constraints(P, X + i * P->d, F + i * P->m, &cm);
    if (CMAX) CMAX[i] = cm;
  }
}

/* ------------------------------------------------------------------------- */
/* Aggregation. PBI (Eq. (7)): d1 = |(F - z) . w| / ||w||,                      */
/* d2 = ||F - (z + d1 w/||w||)|| (R13: unit direction), g = d1 + theta d2.      */
/* Tchebycheff: g = max_k w_k |f_k - z_k|.                                     */
/* ------------------------------------------------------------------------- */
double orc_agg(int32_t agg, double theta, int32_t m, const double *f, const double *w,
               const double *z) {
  if (agg == 1) {
    double g = -INFINITY;
    for (int32_t k = 0; k < m; ++k) {
      double v = w[k] * fabs(f[k] - z[k]);
      if (v > g || isnan(v)) g = v;
      if (isnan(v)) break;
    }
    return g;
  }
  double wn = 0.0;
  for (int32_t k = 0; k < m; ++k) wn += w[k] * w[k];
  wn = sqrt(wn);
  double dot = 0.0;
  for (int32_t k = 0; k < m; ++k) dot += (f[k] - z[k]) * (w[k] / wn);
  double d1 = fabs(dot);
  double d2 = 0.0;
  for (int32_t k = 0; k < m; ++k) {
    double e = (f[k] - z[k]) - d1 * (w[k] / wn);
    d2 += e * e;
  }
  d2 = sqrt(d2);
  return d1 + theta * d2;
}

/* ------------------------------------------------------------------------- */
/* Variation: SBX (pc, eta_c) then polynomial mutation (pm, eta_m), as set in  */
/* the parameter settings of the experimental setup. R7 / R8 fix the forms.    */
/* ------------------------------------------------------------------------- */

/* R7: simple symmetric SBX on one dimension. wA bit0 = cross this dimension,
 * bit1 = negate beta, bits 8..31 = u. Writes the kept child and its sibling
 * (both before clipping). Returns beta (0 when not crossed). */
double orc_sbx_dim(double a, double b, uint32_t wA, double eta_c, double *child,
                   double *sibling) {
  if ((wA & 1u) == 0u) {
    *child = a;
    *sibling = b;
    return 0.0;
  }
  double u = orc_u24(wA);
  double beta = (u <= 0.5) ? pow(2.0 * u, 1.0 / (eta_c + 1.0))
                           : pow(2.0 * (1.0 - u), -1.0 / (eta_c + 1.0));
  if (wA & 2u) beta = -beta;
  *child = 0.5 * ((a + b) + beta * (a - b));
  *sibling = 0.5 * ((a + b) - beta * (a - b));
  return beta;
}

static double orc_clip(double v, double lo, double hi) {
  if (v < lo) v = lo;
  if (v > hi) v = hi;
  return v;
}

/* R8: bounded polynomial mutation of y in [lo, hi] when wB < tpm (integer test,
 * bit-exact on both sides); given that, wB is uniform on [0, tpm) and the
 * conditional uniform is u = wB / tpm in the working precision. */
double orc_pm_dim(double y, double lo, double hi, uint32_t wB, uint64_t tpm, double eta_m) {
  if ((uint64_t)wB >= tpm) return y;
  double u = (double)wB / (double)tpm;
  double span = hi - lo;
  double mpow = 1.0 / (eta_m + 1.0);
  double dq;
  if (u < 0.5) {
    double xy = 1.0 - (y - lo) / span;
    double val = 2.0 * u + (1.0 - 2.0 * u) * pow(xy, eta_m + 1.0);
    dq = pow(val, mpow) - 1.0;
  } else {
    double xy = 1.0 - (hi - y) / span;
    double val = 2.0 * (1.0 - u) + 2.0 * (u - 0.5) * pow(xy, eta_m + 1.0);
    dq = 1.0 - pow(val, mpow);
  }
  return orc_clip(y + dq * span, lo, hi);
}

/* R26: the DE operator of the LIR-CMOP experiments (CR = 1, F = 0.5) in its
 * neighbourhood form: the base is the subproblem's own current solution x_i, the
 * difference is taken between the two mating picks, and CR = 1 makes every
 * variable take the mutant: v = x_i + F (x_a - x_b), clipped to the box, then
 * the polynomial mutation above with the same per-variable draw wB as after
 * SBX. */
double orc_de_dim(double xi, double a, double b, double F, double lo, double hi, uint32_t wB,
                  uint64_t tpm, double eta_m) {
  double v = orc_clip(xi + F * (a - b), lo, hi);
  return orc_pm_dim(v, lo, hi, wB, tpm, eta_m);
}

/* R6: mating picks two distinct positions of B(i) from the MATE block:
 * r1 = hi32(w0 t), r2' = hi32(w1 (t-1)), r2 = r2' + [r2' >= r1]; t = 1 gives r2 = r1. */
void orc_mate(uint32_t w0, uint32_t w1, int32_t t, int32_t *r1, int32_t *r2) {
  uint32_t a = (uint32_t)(((uint64_t)w0 * (uint64_t)(uint32_t)t) >> 32);
  uint32_t b = a;
  if (t >= 2) {
    b = (uint32_t)(((uint64_t)w1 * (uint64_t)(uint32_t)(t - 1)) >> 32);
    b += (b >= a) ? 1u : 0u;
  }
  *r1 = (int32_t)a;
  *r2 = (int32_t)b;
}

/* ------------------------------------------------------------------------- */
/* One generation (Alg. 1 loop body, Alg. 2 environmental selection).          */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t m, d, N;
  int32_t t[2];
  const int32_t *B[2]; /* N x t_p */
  const double *W;     /* N x m */
  int32_t agg;
  double theta, eta_c, eta_m;
  uint64_t tpm; /* floor(pm 2^32) */
  uint64_t tpc; /* floor(pc 2^32) */
  uint32_t key[2];
  int32_t n_eq;  /* the equality x1 + x2 = 1 is active (robustness bookkeeping only) */
  double eq_tol;
  int32_t f32;   /* selection only: take the decisions in FP32 on FP32 inputs (below) */
  int32_t op;    /* reproduction operator: ORC_OP_SBX (SBX then PM) or ORC_OP_DE (DE then PM) */
  double de_f;   /* DE scale factor F */
  int32_t op1_rule; /* population 1's OP1 test: 0 the pseudocode's FPR, 1 the prose's
                       feasibility-first rule (R27) */
} orc_cfg;

#define ORC_OP_SBX 0
#define ORC_OP_DE 1

/* Robustness threshold for parity (R24). */
#define ORC_REL 1e-4

static double orc_nan_inf(double v) { return isnan(v) ? INFINITY : v; }

/* Absolute rounding bound of a total violation computed in FP32: constraints
 * only count while violated, which for the ring and linear constraints happens
 * at objective values of order one, and the equality reads two variables. */
#define ORC_CV_ABS 2e-5

/* Three-way comparison of two total violations a <=> b (-1, 0, +1). *rob = 0
 * when FP32 rounding on the device side could flip the outcome: the FP64
 * margin is at most 1e-4 max(|a|, |b|) + ORC_CV_ABS, or both are infinite and
 * equal (R24). */
static int orc_cmp(double a, double b, int *rob) {
  int c = (a < b) ? -1 : ((a > b) ? 1 : 0);
  if (isinf(a) || isinf(b)) {
    *rob = (a != b);
    return c;
  }
  *rob = fabs(a - b) > ORC_REL * fmax(fabs(a), fabs(b)) + ORC_CV_ABS;
  return c;
}

/* What the selection compares for one individual at one weight. f points at
 * the objective vector the key was computed from (used only to recognise exact
 * copies when judging robustness). */
typedef struct {
  int f32;            /* key evaluated in FP32 (orc_cfg.f32); 2 = bitwise reproducible */
  double cv, cmax, g; /* cmax: largest objective-space constraint value */
  const double *f;
  const double *x;
  double ceq; /* equality slack |x1 + x2 - 1| - tol (-inf without the equality) */
  int tk;     /* Tchebycheff: index of the term that sets g with a clear margin, else -1 */
  double fs;  /* max(1, |f|_inf, |z|_inf): the scale of g's absolute rounding error */
  int copy_ties; /* bitwise-equal keys here are bitwise equal on the device too */
} orc_key;

/* Aggregation values: FP32 rounding moves g by a few units of 1e-7 relative to
 * g and to the objective scale, so a decision on g is robust when the FP64
 * margin exceeds 1e-4 max(|a|, |b|) + 1e-5 max(fs_a, fs_b) (R24). */
static int orc_cmp_g(double a, double b, double fs, int f32, int *rob) {
  int c = (a < b) ? -1 : ((a > b) ? 1 : 0);
  if (isinf(a) || isinf(b)) {
    *rob = (a != b);
    return c;
  }
  if (f32 == 2) /* every operation is one correctly rounded FP32 step on both sides */
    *rob = 1;
  else if (f32) /* FP32 on the same inputs: only contraction and order of sums differ */
    *rob = fabs(a - b) > 2e-6 * (fmax(fabs(a), fabs(b)) + fs);
  else
    *rob = fabs(a - b) > ORC_REL * fmax(fabs(a), fabs(b)) + 1e-5 * fs;
  return c;
}

/* Index of the Tchebycheff term that attains the maximum with a margin above
 * 1e-4 max(1, term) over every other term (-1 when no term is that clear). */
static int orc_tche_arg(int32_t m, const double *f, const double *w, const double *z) {
  int best = -1;
  double v1 = -INFINITY, v2 = -INFINITY;
  for (int32_t k = 0; k < m; ++k) {
    double v = w[k] * fabs(f[k] - z[k]);
    if (isnan(v)) return -1;
    if (v > v1) {
      v2 = v1;
      v1 = v;
      best = k;
    } else if (v > v2) {
      v2 = v;
    }
  }
  if (m > 1 && !(v1 - v2 > ORC_REL * fmax(1.0, v1))) return -1;
  return best;
}

/* The equality reads x1 and x2 only: bitwise-equal pairs give bitwise-equal
 * violations in any precision (the sum commutes). */
static int orc_same_eq(orc_key a, orc_key b) {
  if (!a.x || !b.x || isinf(a.ceq) || isinf(b.ceq)) return 0;
  return (memcmp(&a.x[0], &b.x[0], sizeof(double)) == 0 &&
          memcmp(&a.x[1], &b.x[1], sizeof(double)) == 0) ||
         (memcmp(&a.x[0], &b.x[1], sizeof(double)) == 0 &&
          memcmp(&a.x[1], &b.x[0], sizeof(double)) == 0);
}

/* "a is strictly better than b". pop 0 (population 1) uses the feasibility
 * priority rule of Eq. (8): lower CV wins, equal CV falls back to the lower
 * aggregation. pop 1 (population 2) ignores constraints and compares the
 * aggregation alone. NaN is read as +inf, so it never wins. *rob receives the
 * robustness of the decision (R24). */
static int orc_better(int pop, orc_key a, orc_key b, int *rob) {
  double ga = orc_nan_inf(a.g), gb = orc_nan_inf(b.g);
  double fs = fmax(a.fs, b.fs);
  if (pop == 1) {
    return orc_cmp_g(ga, gb, fs, a.f32, rob) < 0;
  }
  double ca = orc_nan_inf(a.cv), cb = orc_nan_inf(b.cv);
  int rcv;
  int c = orc_cmp(ca, cb, &rcv);
  if (a.f32) rcv = 1; /* the same FP32 violations are compared on both sides */
  if (c != 0) {
    *rob = rcv;
    return c < 0;
  }
  /* equal CVs tie on both sides when nothing near a constraint boundary can
   * move: every objective-space constraint holds with slack, and either both
   * are feasible with slack on the equality too, or both violate only the
   * equality, read from bitwise-equal variables */
  int obj_free = a.cmax < -ORC_CV_ABS && b.cmax < -ORC_CV_ABS;
  int eq_rob = obj_free && ((ca == 0.0 && cb == 0.0 && a.ceq < -ORC_CV_ABS && b.ceq < -ORC_CV_ABS) ||
                            (ca > 0.0 && orc_same_eq(a, b)));
  if (a.f32) eq_rob = 1;
  int rg;
  int cg = orc_cmp_g(ga, gb, fs, a.f32, &rg);
  *rob = eq_rob && rg;
  return cg < 0;
}

/* Robust feasibility status for parity: clearly violated (CV above the FP32
 * rounding bound) or feasible with slack on every constraint; always robust
 * when the decision is taken on given FP32 values. */
static int orc_feas_rob(orc_key a) {
  if (a.f32) return 1;
  double ca = orc_nan_inf(a.cv);
  if (ca > ORC_CV_ABS) return 1;
  return ca == 0.0 && a.cmax < -ORC_CV_ABS && a.ceq < -ORC_CV_ABS;
}

/* R27: OP1 for population 1 as its prose describes it (a reading kept as a
 * variant; the pseudocode's FPR is the default): a feasible offspring beats an
 * infeasible one; when both are feasible or both infeasible the aggregation
 * decides. True iff a is strictly better than b. */
static int orc_better_feasfirst(orc_key a, orc_key b, int *rob) {
  double ca = orc_nan_inf(a.cv), cb = orc_nan_inf(b.cv);
  int fa = ca == 0.0, fb = cb == 0.0;
  int rs = orc_feas_rob(a) && orc_feas_rob(b);
  if (fa != fb) {
    *rob = rs;
    return fa;
  }
  int rg;
  int cg = orc_cmp_g(orc_nan_inf(a.g), orc_nan_inf(b.g), fmax(a.fs, b.fs), a.f32, &rg);
  *rob = rs && rg;
  return cg < 0;
}

/* Keys that tie exactly on both sides of a parity check, whatever the
 * precision: exact copies (bitwise-equal objectives, and CV for population 1),
 * or, for Tchebycheff, the same clearly dominant term evaluated on a bitwise-
 * equal objective (e.g. a variable copied unchanged by SBX). */
static int orc_same(int pop, int m, orc_key a, orc_key b) {
  if (!a.copy_ties || !b.copy_ties) return 0;
  if (pop == 0 && memcmp(&a.cv, &b.cv, sizeof(double)) != 0) return 0;
  if (memcmp(a.f, b.f, sizeof(double) * (size_t)m) == 0) return 1;
  return a.tk >= 0 && a.tk == b.tk && memcmp(&a.f[a.tk], &b.f[b.tk], sizeof(double)) == 0;
}

/* The aggregation in FP32 arithmetic on FP32-rounded operands: the same
 * formulas as orc_agg, for decisions taken in the device's precision. */
static double orc_agg_f32(int32_t agg, double theta, int32_t m, const double *f, const double *w,
                          const double *z) {
  float ff[64], zz[64], ww[64];
  for (int32_t k = 0; k < m; ++k) {
    ff[k] = (float)f[k];
    zz[k] = (float)z[k];
  }
  if (agg == 1) {
    for (int32_t k = 0; k < m; ++k) ww[k] = (float)w[k];
    float g = -INFINITY;
    int nan = 0;
    for (int32_t k = 0; k < m; ++k) {
      float v = ww[k] * fabsf(ff[k] - zz[k]);
      if (isnan(v)) nan = 1;
      if (v > g) g = v;
    }
    return nan ? NAN : (double)g;
  }
  double wn = 0.0; /* unit direction computed in FP64, then rounded once */
  for (int32_t k = 0; k < m; ++k) wn += w[k] * w[k];
  wn = sqrt(wn);
  for (int32_t k = 0; k < m; ++k) ww[k] = (float)(w[k] / wn);
  float dot = 0.0f;
  for (int32_t k = 0; k < m; ++k) dot += (ff[k] - zz[k]) * ww[k];
  float d1 = fabsf(dot), d2 = 0.0f;
  for (int32_t k = 0; k < m; ++k) {
    float e = (ff[k] - zz[k]) - d1 * ww[k];
    d2 += e * e;
  }
  return (double)(d1 + (float)theta * sqrtf(d2));
}

/* Keys that compare equal and are computed bitwise-reproducibly on both sides
 * (the exact FP32 mode): the tie itself is reproduced, and the index decides. */
static int orc_exact_tie(int pop, orc_key a, orc_key b) {
  if (a.f32 != 2 || b.f32 != 2) return 0;
  if (pop == 0 && !(orc_nan_inf(a.cv) == orc_nan_inf(b.cv))) return 0;
  return orc_nan_inf(a.g) == orc_nan_inf(b.g);
}

/* Key of an individual (decision vector x, objectives f, CV and the largest
 * objective-space constraint value given) at weight w. */
static orc_key orc_mk(const orc_cfg *C, double cv, double cmax, const double *x, const double *f,
                      const double *w, const double *z) {
  double g = C->f32 ? orc_agg_f32(C->agg, C->theta, C->m, f, w, z)
                    : orc_agg(C->agg, C->theta, C->m, f, w, z);
  /* In FP32, Tchebycheff is max_k w_k |f_k - z_k|: a subtraction, an absolute
   * value and a product per term, none of which a compiler can fuse, so equal
   * FP32 inputs give the bitwise-equal value on every IEEE device. */
  int mode = C->f32 ? (C->agg == 1 ? 2 : 1) : 0;
  /* FP64-equal offspring are device-equal when they are copies of equal values
   * (SBX leaves variables uncrossed; decisions on given FP32 values). DE
   * offspring are recomputed in every variable, and different triples can meet
   * exactly in FP64 (x_b + F (x_a - x_b) and x_a + F (x_b - x_a) at F = 1/2)
   * while their FP32 roundings differ: such ties are not robust (R24, R26). */
  orc_key k = {mode, cv, cmax, g, f, x, -INFINITY, -1, 1.0, C->f32 || C->op != ORC_OP_DE};
  if (C->n_eq) k.ceq = fabs(x[0] + x[1] - 1.0) - C->eq_tol;
  if (C->agg == 1) k.tk = orc_tche_arg(C->m, f, w, z);
  for (int32_t a = 0; a < C->m; ++a) {
    if (fabs(f[a]) > k.fs) k.fs = fabs(f[a]);
    if (fabs(z[a]) > k.fs) k.fs = fabs(z[a]);
  }
  return k;
}

/* Environmental selection of one generation (Alg. 2) on given parents and
 * offspring, with z already updated.
 *   X[p], F[p], CV[p], CM[p]   parents of population p (N x d, N x m, N, N)
 *   Xo, Fo, CVo, CMo           offspring, population-major (2N x d, 2N x m, 2N, 2N)
 * (X and CM serve only the robustness flags.)
 * Outputs (all 2N, population-major):
 *   sw[p N + i]   OP1: 1 if population p's new offspring at i is the other
 *                 population's offspring; swr = robustness of that switch
 *   win[p N + j]  winner offspring index for parent slot j (-1: parent kept);
 *                 winr = robustness of the slot's outcome (R24): the winner is
 *                 robustly better than the parent and than every other
 *                 candidate, or, when the parent stays, no candidate can be
 *                 better than it; a candidate whose OP1 switch is not robust is
 *                 judged under both of its possible offspring.
 * OP1 (Eq. (11)): at w_i, population 1 takes off2 if it is FPR-better than
 * off1; population 2 takes off1 if its aggregation is lower (R14, R15).
 * OP2 + OP3 (Eqs. (12)-(13)), as a pull over parent slot j: offspring i with
 * j in B_p(i) qualifies iff its new offspring is strictly better than parent j
 * at w_j; the winner is the lexicographic minimum over the qualifiers, first
 * index on ties (R17-R19). Decisions all use generation-k parents. */
void orc_select(const orc_cfg *C, const double *X0, const double *X1, const double *F0,
                const double *F1, const double *CV0, const double *CV1, const double *CM0,
                const double *CM1, const double *Xo, const double *Fo, const double *CVo,
                const double *CMo, const double *z, uint8_t *sw, uint8_t *swr, int32_t *win,
                uint8_t *winr) {
  const int32_t m = C->m, N = C->N, d = C->d;
  const double *X[2] = {X0, X1}, *F[2] = {F0, F1}, *CV[2] = {CV0, CV1}, *CM[2] = {CM0, CM1};

#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < N; ++i) {
    const double *w = C->W + (size_t)i * m;
    orc_key k1 = orc_mk(C, CVo[i], CMo[i], Xo + (size_t)i * d, Fo + (size_t)i * m, w, z);
    orc_key k2 = orc_mk(C, CVo[N + i], CMo[N + i], Xo + ((size_t)N + i) * d,
                        Fo + ((size_t)N + i) * m, w, z);
    int r1, r2;
    if (C->op1_rule == 1)
      sw[i] = (uint8_t)orc_better_feasfirst(k2, k1, &r1); /* S1 under the prose rule */
    else
      sw[i] = (uint8_t)orc_better(0, k2, k1, &r1);     /* S1: population 1 takes off2 */
    sw[N + i] = (uint8_t)orc_better(1, k1, k2, &r2); /* S2: population 2 takes off1 */
    swr[i] = (uint8_t)(r1 || orc_same(0, m, k1, k2));
    swr[N + i] = (uint8_t)(r2 || orc_same(1, m, k1, k2));
  }

  for (int p = 0; p < 2; ++p) {
    /* reverse neighbour lists rev_p(j) = {i : j in B_p(i)}, ascending in i */
    const int32_t t = C->t[p];
    int32_t *roff = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    int32_t *ridx = (int32_t *)malloc(sizeof(int32_t) * (size_t)N * t);
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (size_t q = 0; q < (size_t)N * t; ++q) roff[C->B[p][q] + 1]++;
    for (int32_t j = 0; j < N; ++j) roff[j + 1] += roff[j];
    memcpy(fill, roff, sizeof(int32_t) * (size_t)N);
    for (int32_t i = 0; i < N; ++i)
      for (int32_t r = 0; r < t; ++r) {
        int32_t j = C->B[p][(size_t)i * t + r];
        ridx[fill[j]++] = i;
      }

#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < N; ++j) {
      const double *w = C->W + (size_t)j * m;
      orc_key par = orc_mk(C, CV[p][j], CM[p][j], X[p] + (size_t)j * d, F[p] + (size_t)j * m, w, z);
      /* the decision: lexicographic minimum over qualifiers, first index on ties */
      orc_key best = par;
      int32_t bi = -1;
      for (int32_t q = roff[j]; q < roff[j + 1]; ++q) {
        int32_t i = ridx[q];
        size_t src = (size_t)(p ^ sw[(size_t)p * N + i]) * N + i;
        orc_key ck = orc_mk(C, CVo[src], CMo[src], Xo + src * d, Fo + src * m, w, z);
        int r;
        if (orc_better(p, ck, par, &r) && orc_better(p, ck, best, &r)) {
          best = ck;
          bi = i;
        }
      }
      win[(size_t)p * N + j] = bi;

      /* robustness of that outcome */
      int robust = 1;
      if (bi >= 0) {
        int r;
        if (!swr[(size_t)p * N + bi]) robust = 0;
        if (!orc_better(p, best, par, &r) || !r) robust = 0;
      }
      for (int32_t q = roff[j]; q < roff[j + 1] && robust; ++q) {
        int32_t i = ridx[q];
        if (i == bi) continue;
        int nalt = swr[(size_t)p * N + i] ? 1 : 2;
        for (int a = 0; a < nalt && robust; ++a) {
          int other = sw[(size_t)p * N + i] ^ a;
          size_t src = (size_t)(p ^ other) * N + i;
          orc_key ck = orc_mk(C, CVo[src], CMo[src], Xo + src * d, Fo + src * m, w, z);
          int r;
          if (bi >= 0) {
            /* the winner must stay ahead of this candidate */
            if (orc_same(p, m, ck, best) || orc_exact_tie(p, ck, best)) {
              if (i < bi) robust = 0;
            } else if (!orc_better(p, best, ck, &r) || !r) {
              robust = 0;
            }
          } else {
            /* no candidate may overtake the parent */
            if (!orc_same(p, m, ck, par) && !orc_exact_tie(p, ck, par) &&
                (orc_better(p, ck, par, &r) || !r))
              robust = 0;
          }
        }
      }
      winr[(size_t)p * N + j] = (uint8_t)robust;
    }
    free(roff);
    free(ridx);
    free(fill);
  }
}

/* Offspring of one generation (Alg. 1 reproduction + evaluation): each
 * population mates inside its own neighbourhood (R6), SBX then PM (R7, R8) or
 * DE then PM (R26), then objectives and constraints. Outputs population-major; mate may be NULL. */
void orc_reproduce(const orc_problem *P, const orc_cfg *C, uint32_t k, const double *X0,
                   const double *X1, double *Xo, double *Fo, double *CVo, double *CMo,
                   int32_t *mate) {
  const int32_t m = C->m, d = C->d, N = C->N;
  const double *X[2] = {X0, X1};
  const size_t nd = (size_t)N * (size_t)d;
  for (int p = 0; p < 2; ++p) {
    const int32_t t = C->t[p];
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
      uint32_t w[4], v[4] = {0, 0, 0, 0};
      orc_draw(0u, (uint32_t)i, k, ORC_TAG_MATE, (uint32_t)p, C->key, w);
      int32_t r1, r2;
      orc_mate(w[0], w[1], t, &r1, &r2);
      int32_t pa = C->B[p][(size_t)i * t + r1], pb = C->B[p][(size_t)i * t + r2];
      if (mate) {
        mate[((size_t)p * N + i) * 2 + 0] = pa;
        mate[((size_t)p * N + i) * 2 + 1] = pb;
      }
      int cross = (uint64_t)w[2] < C->tpc; /* SBX probability pc per individual */
      const double *a = X[p] + (size_t)pa * d, *b = X[p] + (size_t)pb * d;
      const double *xi = X[p] + (size_t)i * d;
      double *c = Xo + (size_t)p * nd + (size_t)i * d;
      for (int32_t l = 0; l < d; ++l) {
        if ((l & 1) == 0)
          orc_draw((uint32_t)(l >> 1), (uint32_t)i, k, ORC_TAG_VAR, (uint32_t)p, C->key, v);
        uint32_t wA = v[2 * (l & 1)], wB = v[2 * (l & 1) + 1];
        if (C->op == ORC_OP_DE) {
          c[l] = orc_de_dim(xi[l], a[l], b[l], C->de_f, P->lb[l], P->ub[l], wB, C->tpm, C->eta_m);
          continue;
        }
        double ch = a[l], sib;
        if (cross) orc_sbx_dim(a[l], b[l], wA, C->eta_c, &ch, &sib);
        ch = orc_clip(ch, P->lb[l], P->ub[l]);
        c[l] = orc_pm_dim(ch, P->lb[l], P->ub[l], wB, C->tpm, C->eta_m);
      }
      double *f = Fo + ((size_t)p * N + i) * m;
      orc_objectives(P, c, f);
      double cm;
      CVo[(size_t)p * N + i] = orc_constraints(P, c, f, &cm);
      CMo[(size_t)p * N + i] = cm;
    }
  }
}

/* Ideal point (Alg. 1 initialisation and update): z_a = min(z_a, min F_a)
 * over n rows; NaN never lowers z (R12: infeasible rows count). */
void orc_ideal(int64_t n, int32_t m, const double *F, double *z) {
  for (int64_t q = 0; q < n; ++q)
    for (int32_t a = 0; a < m; ++a) {
      double v = F[q * m + a];
      if (v < z[a]) z[a] = v;
    }
}

/* Generation k (Alg. 1 loop body) on the state of both populations, in place:
 * reproduce, evaluate, update z, select (Alg. 2), then replace synchronously.
 * Debug outputs may be NULL (shapes as in orc_reproduce / orc_select).
 * Returns the number of replaced slots over both populations. */
int64_t orc_generation(const orc_problem *P, const orc_cfg *C, uint32_t k, double *X0,
                       double *X1, double *F0, double *F1, double *CV0, double *CV1,
                       double *CM0, double *CM1, double *z, int32_t *mate, double *Xo,
                       double *Fo, double *CVo, uint8_t *op1, uint8_t *op1_rob, int32_t *win,
                       uint8_t *win_rob) {
  const int32_t m = C->m, d = C->d, N = C->N;
  double *X[2] = {X0, X1}, *F[2] = {F0, F1}, *CV[2] = {CV0, CV1}, *CM[2] = {CM0, CM1};
  const size_t nd = (size_t)N * (size_t)d;
  double *xo = (double *)malloc(sizeof(double) * 2 * nd);
  double *fo = (double *)malloc(sizeof(double) * 2 * (size_t)N * (size_t)m);
  double *cvo = (double *)malloc(sizeof(double) * 2 * (size_t)N);
  double *cmo = (double *)malloc(sizeof(double) * 2 * (size_t)N);
  uint8_t *sw = (uint8_t *)malloc(2 * (size_t)N);
  uint8_t *swr = (uint8_t *)malloc(2 * (size_t)N);
  int32_t *wn = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)N);
  uint8_t *wr = (uint8_t *)malloc(2 * (size_t)N);

  orc_reproduce(P, C, k, X0, X1, xo, fo, cvo, cmo, mate);
  orc_ideal(2 * (int64_t)N, m, fo, z);
  orc_select(C, X0, X1, F0, F1, CV0, CV1, CM0, CM1, xo, fo, cvo, cmo, z, sw, swr, wn, wr);

  int64_t replaced = 0;
  for (int p = 0; p < 2; ++p) {
    for (int32_t j = 0; j < N; ++j) {
      int32_t i = wn[(size_t)p * N + j];
      if (i < 0) continue;
      ++replaced;
      int sp = p ^ sw[(size_t)p * N + i];
      size_t src = (size_t)sp * N + i;
      memcpy(X[p] + (size_t)j * d, xo + (size_t)sp * nd + (size_t)i * d, sizeof(double) * d);
      memcpy(F[p] + (size_t)j * m, fo + src * m, sizeof(double) * m);
      CV[p][j] = cvo[src];
      CM[p][j] = cmo[src];
    }
  }

  if (Xo) memcpy(Xo, xo, sizeof(double) * 2 * nd);
  if (Fo) memcpy(Fo, fo, sizeof(double) * 2 * (size_t)N * m);
  if (CVo) memcpy(CVo, cvo, sizeof(double) * 2 * (size_t)N);
  if (op1) memcpy(op1, sw, 2 * (size_t)N);
  if (op1_rob) memcpy(op1_rob, swr, 2 * (size_t)N);
  if (win) memcpy(win, wn, sizeof(int32_t) * 2 * (size_t)N);
  if (win_rob) memcpy(win_rob, wr, 2 * (size_t)N);
  free(xo); free(fo); free(cvo); free(cmo); free(sw); free(swr); free(wn); free(wr);
  return replaced;
}

/* Initial population (Alg. 1 "Tensorized initialization", R4): X_p[i][l] =
 * lb + (ub - lb) U with U from the INIT block (l >> 2, i, 0, INIT|p), word l & 3. */
void orc_init_x(const orc_problem *P, int32_t N, const uint32_t key[2], int32_t pop, double *X) {
  const int32_t d = P->d;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < N; ++i) {
    uint32_t w[4] = {0, 0, 0, 0};
    for (int32_t l = 0; l < d; ++l) {
      if ((l & 3) == 0) orc_draw((uint32_t)(l >> 2), (uint32_t)i, 0u, ORC_TAG_INIT, (uint32_t)pop,
                                 key, w);
      X[(size_t)i * d + l] = P->lb[l] + (P->ub[l] - P->lb[l]) * orc_u24(w[l & 3]);
    }
  }
}

/* Feasible non-dominated filter of a population (Eq. (4) feasible set, Eq. (5)
 * dominance; R20): keep[i] = 1 iff CV_i = 0 and no feasible j dominates i. */
int64_t orc_front(int64_t n, int32_t m, const double *F, const double *CV, uint8_t *keep) {
  int64_t cnt = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : cnt)
  for (int64_t i = 0; i < n; ++i) {
    keep[i] = 0;
    if (!(CV[i] == 0.0)) continue;
    int dom = 0;
    for (int64_t j = 0; j < n && !dom; ++j) {
      if (j == i || !(CV[j] == 0.0)) continue;
      int le = 1, lt = 0;
      for (int32_t a = 0; a < m; ++a) {
        if (F[j * m + a] > F[i * m + a]) le = 0;
        if (F[j * m + a] < F[i * m + a]) lt = 1;
      }
      dom = le && lt;
    }
    if (!dom) {
      keep[i] = 1;
      ++cnt;
    }
  }
  return cnt;
}

int32_t orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
