// Reference vectors, neighbourhoods and reverse neighbourhood lists (host side).
//
// W: the Das-Dennis simplex lattice (the "uniform reference vectors" input of
// Alg. 1). Rows are k / H for every k in N^m with sum H, enumerated in ascending
// lexicographic order of (k_1 .. k_{m-1}); H is the smallest value whose count
// C(H + m - 1, m - 1) reaches the requested population size.
//
// B: the t nearest reference vectors of each subproblem (Alg. 1 "neighbours
// initialization"; t1 = T/2 and t2 = 2T in the parameter settings), ordered by
// exact integer lattice distance sum_a (k_i,a - k_j,a)^2 with ties broken by
// ascending index, so subproblem i itself comes first.
//
// Rank order among lattice points equals the lexicographic order of their leading
// m - 1 coordinates, so for any point i the candidates j = i + delta sort by
// (distance of delta, lexicographic order of delta), the same for every i. The
// search therefore walks one offset list, sorted once, holding every offset
// within distance R, and keeps the first t offsets that land inside the lattice.
// A point with fewer than t lattice neighbours in that list (only possible near
// corners) falls back to a box walk: it enumerates the points whose leading
// coordinates lie within a box of half-width R around k_i, ranks them directly,
// and grows R until the t-th nearest found lies within distance R. Every lattice
// point within distance R lies inside the box, so neither method can miss a
// closer point (or an equal-distance point with a smaller index).
//
// Two-layer sets (many objectives): the lattice above with H1 divisions, then a
// lattice with H2 divisions moved halfway to the centroid. Both layers become
// integer points on the common denominator 2 m H1 H2, and the neighbourhoods
// come from a brute-force search over exact squared distances (O(N^2 m) over
// host threads; such sets hold a few thousand to about 1e5 vectors).
#include <algorithm>
#include <cmath>
#include <thread>

#include "gmpea_internal.hpp"

namespace gmpea {

int64_t dd_count(int32_t m, int32_t H) {
  // C(H + m - 1, m - 1), exact in 64-bit for the supported sizes
  int64_t c = 1;
  for (int32_t j = 1; j <= m - 1; ++j) c = c * (H + j) / j;
  return c;
}

int32_t dd_divisions(int32_t m, int64_t n_req) {
  int32_t H = 1;
  while (dd_count(m, H) < n_req) ++H;
  return H;
}

void dd_lattice(int32_t m, int32_t H, std::vector<int32_t> &K) {
  const int64_t n = dd_count(m, H);
  K.assign(static_cast<size_t>(n) * m, 0);
  std::vector<int32_t> cur(m, 0);
  // odometer over (k_1 .. k_{m-1}) in lexicographic order; k_m takes the rest
  cur[m - 1] = H;
  for (int64_t row = 0; row < n; ++row) {
    for (int32_t a = 0; a < m; ++a) K[row * m + a] = cur[a];
    // advance: increase the last leading coordinate that still has room
    int32_t a = m - 2;
    while (a >= 0) {
      int32_t used = 0;
      for (int32_t b = 0; b <= a; ++b) used += cur[b];
      if (used < H) break;
      --a;
    }
    if (a < 0) break;
    cur[a] += 1;
    for (int32_t b = a + 1; b < m - 1; ++b) cur[b] = 0;
    int32_t used = 0;
    for (int32_t b = 0; b < m - 1; ++b) used += cur[b];
    cur[m - 1] = H - used;
  }
}

// Position of composition k in the enumeration above. The compositions placed
// before k at coordinate a are those with a smaller value there:
// sum_{v < k_a} C(left - v + r - 1, r - 1) with r = m - a - 1 parts left, which
// the hockey-stick identity turns into C(left + r, r) - C(left - k_a + r, r).
static int64_t dd_rank(const int32_t *k, int32_t m, int32_t H) {
  // m = 2: the rank is k_1. m = 3: C(H + 2, 2) - C(H - k_1 + 2, 2) + k_2, where
  // C(x + 2, 2) = (x + 2)(x + 1) / 2 is exact (a product of consecutive integers).
  if (m == 2) return k[0];
  if (m == 3) {
    const int64_t a = H, b = H - k[0];
    return ((a + 2) * (a + 1) - (b + 2) * (b + 1)) / 2 + k[1];
  }
  int64_t r = 0;
  int32_t left = H;
  for (int32_t a = 0; a < m - 1; ++a) {
    r += dd_count(m - a, left) - dd_count(m - a, left - k[a]);
    left -= k[a];
  }
  return r;
}

namespace {
struct Cand {
  int64_t dist;
  int32_t idx;
  bool operator<(const Cand &o) const { return dist < o.dist || (dist == o.dist && idx < o.idx); }
};
}  // namespace

// Box walk for row i (exact; used where the offset list runs out).
static void knn_row_box(const std::vector<int32_t> &K, int32_t m, int32_t H, int32_t t, int64_t i,
                        int32_t *out) {
  std::vector<Cand> cand;
  std::vector<int32_t> kk(m), off(m > 1 ? m - 1 : 1);
  const int32_t lead = m - 1;
  const int32_t *ki = &K[i * m];
  int32_t R = 1;
  while (R * R < t) ++R;
  for (;;) {
    cand.clear();
    // enumerate offsets in [-R, R]^(m-1)
    for (int32_t a = 0; a < lead; ++a) off[a] = -R;
    for (;;) {
      int32_t sum = 0;
      bool ok = true;
      for (int32_t a = 0; a < lead; ++a) {
        kk[a] = ki[a] + off[a];
        if (kk[a] < 0 || kk[a] > H) ok = false;
        sum += kk[a];
      }
      kk[m - 1] = H - sum;
      if (ok && kk[m - 1] >= 0 && kk[m - 1] <= H) {
        int64_t dist = 0;
        for (int32_t a = 0; a < m; ++a) {
          int64_t df = int64_t(kk[a]) - ki[a];
          dist += df * df;
        }
        cand.push_back({dist, static_cast<int32_t>(dd_rank(kk.data(), m, H))});
      }
      int32_t a = lead - 1;
      while (a >= 0 && off[a] == R) off[a--] = -R;
      if (a < 0) break;
      ++off[a];
    }
    if (static_cast<int32_t>(cand.size()) >= t) {
      std::partial_sort(cand.begin(), cand.begin() + t, cand.end());
      if (cand[t - 1].dist <= int64_t(R) * R) {
        for (int32_t r = 0; r < t; ++r) out[r] = cand[r].idx;
        return;
      }
    }
    R += std::max(1, R / 2);  // any R that passes the test above is exact
  }
}

namespace {
struct Offset {
  int64_t dist;
  int32_t d[kMaxM];  // leading m - 1 components
};
}  // namespace

// Every offset of the leading coordinates within distance R (last coordinate
// -sum of the others), sorted by (distance, lexicographic order).
static std::vector<Offset> sorted_offsets(int32_t m, int32_t R) {
  std::vector<Offset> out;
  const int32_t lead = m - 1;
  int32_t off[kMaxM] = {0, 0, 0};
  for (int32_t a = 0; a < lead; ++a) off[a] = -R;
  for (;;) {
    int64_t dist = 0, sum = 0;
    for (int32_t a = 0; a < lead; ++a) {
      dist += int64_t(off[a]) * off[a];
      sum += off[a];
    }
    dist += sum * sum;
    if (dist <= int64_t(R) * R) {
      Offset o{dist, {0, 0, 0}};
      for (int32_t a = 0; a < lead; ++a) o.d[a] = off[a];
      out.push_back(o);
    }
    int32_t a = lead - 1;
    while (a >= 0 && off[a] == R) off[a--] = -R;
    if (a < 0) break;
    ++off[a];
  }
  std::sort(out.begin(), out.end(), [lead](const Offset &x, const Offset &y) {
    if (x.dist != y.dist) return x.dist < y.dist;
    for (int32_t a = 0; a < lead; ++a)
      if (x.d[a] != y.d[a]) return x.d[a] < y.d[a];
    return false;
  });
  return out;
}

static void knn_rows(const std::vector<int32_t> &K, int32_t m, int32_t H, int32_t t,
                     const std::vector<Offset> &offs, int64_t lo, int64_t hi,
                     std::vector<int32_t> &B) {
  const int32_t lead = m - 1;
  int32_t kk[kMaxM];
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t *ki = &K[i * m];
    int32_t *out = &B[i * t];
    int32_t cnt = 0;
    for (const Offset &o : offs) {
      int32_t sum = 0;
      bool ok = true;
      for (int32_t a = 0; a < lead; ++a) {
        kk[a] = ki[a] + o.d[a];
        ok = ok && kk[a] >= 0 && kk[a] <= H;
        sum += kk[a];
      }
      kk[lead] = H - sum;
      if (!ok || kk[lead] < 0 || kk[lead] > H) continue;
      out[cnt++] = static_cast<int32_t>(dd_rank(kk, m, H));
      if (cnt == t) break;
    }
    if (cnt < t) knn_row_box(K, m, H, t, i, out);
  }
}

// Offsets within the smallest radius (grown geometrically, at most H) whose list
// holds about 8 t entries: interior points need t of them, points near a corner
// of the lattice a few times more.
static std::vector<Offset> offsets_for(int32_t m, int32_t H, int32_t t) {
  int32_t R = 1;
  while (R < H && static_cast<int64_t>(sorted_offsets(m, R).size()) < 8 * int64_t(t)) R += 1 + R / 4;
  return sorted_offsets(m, R);
}

void neighbour_offsets(int32_t m, int32_t H, int32_t t, std::vector<int32_t> &d) {
  const std::vector<Offset> offs = offsets_for(m, H, t);
  d.assign(offs.size() * 2, 0);
  for (size_t q = 0; q < offs.size(); ++q) {
    d[2 * q] = offs[q].d[0];
    d[2 * q + 1] = m > 2 ? offs[q].d[1] : 0;
  }
}

void lattice_knn(const std::vector<int32_t> &K, int32_t m, int32_t H, int32_t t,
                 std::vector<int32_t> &B) {
  const int64_t n = static_cast<int64_t>(K.size()) / m;
  B.assign(static_cast<size_t>(n) * t, 0);
  const std::vector<Offset> offs = offsets_for(m, H, t);
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n * t < (1 << 18)) nt = 1;
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < nt; ++w) {
    int64_t lo = n * w / nt, hi = n * (w + 1) / nt;
    pool.emplace_back([&, lo, hi] { knn_rows(K, m, H, t, offs, lo, hi, B); });
  }
  for (auto &th : pool) th.join();
}

int64_t refset_count(int32_t m, int32_t H1, int32_t H2) {
  return dd_count(m, H1) + (H2 > 0 ? dd_count(m, H2) : 0);
}

void refset(int32_t m, int32_t H1, int32_t H2, std::vector<int32_t> &K, std::vector<double> *W) {
  std::vector<int32_t> K1, K2;
  dd_lattice(m, H1, K1);
  if (H2 > 0) dd_lattice(m, H2, K2);
  const size_t n1 = K1.size() / m, n2 = K2.size() / m;
  K.assign((n1 + n2) * m, 0);
  if (W) W->assign((n1 + n2) * m, 0.0);
  // outer layer: k / H1, on the denominator 2 m H1 H2 (H1 alone for one layer)
  const int32_t so = H2 > 0 ? 2 * m * H2 : 1;
  for (size_t q = 0; q < n1 * m; ++q) {
    K[q] = K1[q] * so;
    if (W) (*W)[q] = static_cast<double>(K1[q]) / H1;
  }
  // inner layer: (k / H2 + 1 / m) / 2 = (m H1 k + H1 H2) / (2 m H1 H2)
  for (size_t q = 0; q < n2 * m; ++q) {
    K[n1 * m + q] = m * H1 * K2[q] + H1 * H2;
    if (W) (*W)[n1 * m + q] = (static_cast<double>(K2[q]) / H2 + 1.0 / m) * 0.5;
  }
}

void refset_knn(const std::vector<int32_t> &K, int32_t m, int32_t t, std::vector<int32_t> &B) {
  const int64_t n = static_cast<int64_t>(K.size()) / m;
  B.assign(static_cast<size_t>(n) * t, 0);
  auto rows = [&](int64_t lo, int64_t hi) {
    std::vector<Cand> best;  // the t smallest (distance, index) so far, sorted
    for (int64_t i = lo; i < hi; ++i) {
      best.clear();
      const int32_t *ki = &K[i * m];
      for (int64_t j = 0; j < n; ++j) {
        const int32_t *kj = &K[j * m];
        int64_t dist = 0;
        for (int32_t a = 0; a < m; ++a) {
          const int64_t df = int64_t(ki[a]) - kj[a];
          dist += df * df;
        }
        const Cand c{dist, static_cast<int32_t>(j)};
        if (static_cast<int32_t>(best.size()) == t) {
          if (!(c < best.back())) continue;
          best.pop_back();
        }
        best.insert(std::upper_bound(best.begin(), best.end(), c), c);
      }
      for (int32_t r = 0; r < t; ++r) B[i * t + r] = best[r].idx;
    }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n * n < (1 << 22)) nt = 1;
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < nt; ++w)
    pool.emplace_back(rows, n * w / nt, n * (w + 1) / nt);
  for (auto &th : pool) th.join();
}

void refset_neighbours(const std::vector<int32_t> &K, int32_t m, int32_t H1, int32_t H2, int32_t t,
                       std::vector<int32_t> &B) {
  // the offset walk enumerates boxes in m - 1 dimensions: cheap for m <= 3 only
  if (H2 == 0 && m <= 3)
    lattice_knn(K, m, H1, t, B);
  else
    refset_knn(K, m, t, B);
}

void reverse_lists(const std::vector<int32_t> &B, int32_t n, int32_t t, std::vector<int32_t> &off,
                   std::vector<int32_t> &idx) {
  off.assign(static_cast<size_t>(n) + 1, 0);
  for (size_t q = 0; q < static_cast<size_t>(n) * t; ++q) off[B[q] + 1]++;
  for (int32_t j = 0; j < n; ++j) off[j + 1] += off[j];
  idx.assign(static_cast<size_t>(n) * t, 0);
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (int32_t i = 0; i < n; ++i)  // ascending i keeps every list sorted
    for (int32_t r = 0; r < t; ++r) idx[fill[B[static_cast<size_t>(i) * t + r]]++] = i;
}

}  // namespace gmpea
