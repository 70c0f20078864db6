// Host-only check of the set-up tables (csrc/host_tables.hpp), built with
// g++ and the address and undefined-behaviour sanitizers by
// test_host_tables_sanitized.py: geometry arithmetic, the Gauss-Jordan
// inverse, the 64 Vanka local inverses, the dense coarsest inverse and the
// V1 colour lists on several box shapes.  Prints "ok" and exits 0 when every
// check holds; a sanitizer report or a failed check exits non-zero.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2312_10615_amd/csrc/host_tables.hpp"

using namespace sg;

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      std::fprintf(stderr, "FAIL %s: ", #cond); \
      std::fprintf(stderr, __VA_ARGS__);      \
      std::fprintf(stderr, "\n");             \
      ++failures;                             \
    }                                         \
  } while (0)

// L~ applied to one unit vector of slot code e = f * F + slot, written from the
// stencil of Eq. 2 / Section 4 on the padded grid (independently of
// coarse_inverse's assembly): returns (row code, value) pairs.
static void column(const Geom& g, int f, int I, int J, int K, std::vector<std::pair<long, double>>& out) {
  out.clear();
  const int F = g.field;
  auto act = [&](int ff, int i, int j, int k) {
    return ff == 0 ? g.ux_active(i, j, k) : ff == 1 ? g.uy_active(i, j, k) : ff == 2 ? g.uz_active(i, j, k)
                                                                                    : g.p_active(i, j, k);
  };
  const int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  if (f < 3) {
    out.push_back({(long)f * F + g.idx(I, J, K), 6.0 * g.c});
    for (int a = 0; a < 3; ++a)
      for (int s = -1; s <= 1; s += 2) {
        const int i = I + s * d[a][0], j = J + s * d[a][1], k = K + s * d[a][2];
        if (act(f, i, j, k)) out.push_back({(long)f * F + g.idx(i, j, k), -g.c});
      }
    // the face is the minus face of cell (I,J,K) and the plus face of the cell before it
    if (g.p_active(I, J, K)) out.push_back({3L * F + g.idx(I, J, K), g.inv_h});
    const int i = I - d[f][0], j = J - d[f][1], k = K - d[f][2];
    if (g.p_active(i, j, k)) out.push_back({3L * F + g.idx(i, j, k), -g.inv_h});
  } else {
    out.push_back({3L * F + g.idx(I, J, K), -g.gamma});
    for (int a = 0; a < 3; ++a) {
      if (act(a, I, J, K)) out.push_back({(long)a * F + g.idx(I, J, K), g.inv_h});
      const int i = I + d[a][0], j = J + d[a][1], k = K + d[a][2];
      if (act(a, i, j, k)) out.push_back({(long)a * F + g.idx(i, j, k), -g.inv_h});
    }
  }
}

static void check_geometry(int nx, int ny, int nz) {
  const int L = count_levels(nx, ny, nz, 2);
  for (int l = 0; l < L; ++l) {
    const Geom g = make_geom(nx, ny, nz, 1.0 / nx, 1.0, 1e-3, l);
    const long slots = (long)g.sz * (g.nz + 2);
    CHECK(g.sy % 2 == 1 && g.sz % 2 == 1, "odd pitches %d %d", g.sy, g.sz);
    CHECK(g.field % 8 == 0 && g.field >= slots + 8 && 2 * g.half == g.field, "field %d slots %ld", g.field, slots);
    // every slot maps to its own element inside the field
    std::vector<char> seen(g.field, 0);
    for (long s = 0; s < slots; ++s) {
      const int e = g.at((int)s);
      CHECK(e >= 0 && e < g.field && !seen[e], "slot %ld -> element %d", s, e);
      if (e >= 0 && e < g.field) seen[e] = 1;
    }
  }
}

static void check_invert() {
  std::mt19937 rng(7);
  std::normal_distribution<double> nd;
  for (int n : {1, 2, 5, 17, 40}) {
    std::vector<double> a((size_t)n * n), b;
    for (auto& v : a) v = nd(rng);
    b = a;
    CHECK(invert(b, n), "invert n=%d", n);
    double err = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += a[(size_t)i * n + k] * b[(size_t)k * n + j];
        err = std::fmax(err, std::fabs(s - (i == j)));
      }
    CHECK(err < 1e-9, "A A^-1 - I = %g (n=%d)", err, n);
  }
  std::vector<double> z(9, 0.0);
  z[0] = 1.0;
  CHECK(!invert(z, 3), "a singular matrix is reported");
}

static void check_vanka(const Geom& g) {
  std::vector<double> inv;
  CHECK(vanka_inverses(g, inv), "vanka_inverses");
  CHECK(inv.size() == 64 * 64, "size %zu", inv.size());
  for (int type = 0; type < 64; ++type) {
    auto entry = [&](int a, int b) -> double {   // C L~ C^T of the local unknowns, from the stencil
      if (a == 6 && b == 6) return -g.gamma;
      if (a == 6 || b == 6) return ((a == 6 ? b : a) & 1) ? -g.inv_h : g.inv_h;
      if (a == b) return 6.0 * g.c;
      return a / 2 == b / 2 ? -g.c : 0.0;
    };
    auto live = [&](int s) { return s == 6 || (type >> s & 1); };
    double err = 0.0;
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j < 7; ++j) {
        if (!live(i) || !live(j)) {
          CHECK(inv[type * 64 + i * 8 + j] == 0.0, "inactive entry type %d (%d,%d)", type, i, j);
          continue;
        }
        double s = 0.0;
        for (int k = 0; k < 7; ++k)
          if (live(k)) s += entry(i, k) * inv[type * 64 + k * 8 + j];
        err = std::fmax(err, std::fabs(s - (i == j)));
      }
    CHECK(err < 1e-9, "K K^-1 - I = %g for type %d", err, type);
  }
}

static void check_coarse(const Geom& g) {
  std::vector<int> dof;
  std::vector<double> inv;
  CHECK(coarse_inverse(g, dof, inv), "coarse_inverse %dx%dx%d", g.nx, g.ny, g.nz);
  const long n = (long)dof.size();
  const long want = (long)(g.nx - 1) * g.ny * g.nz + (long)g.nx * (g.ny - 1) * g.nz + (long)g.nx * g.ny * (g.nz - 1) +
                    (long)g.nx * g.ny * g.nz;
  CHECK(n == want, "unknowns %ld vs %ld", n, want);
  CHECK((long)inv.size() == n * n, "inverse size");
  // row of each unknown in dof order: element offset -> row
  const int F = g.field;
  std::vector<int> row((size_t)4 * F, -1);
  for (long r = 0; r < n; ++r) row[dof[r]] = (int)r;
  // inv * (L~ e_j) = e_j for every unknown j, L~ e_j from the stencil
  std::vector<std::pair<long, double>> col;
  double err = 0.0, asym = 0.0;
  long j = 0;
  for (int f = 0; f < 4; ++f)
    for (int K = 0; K < g.nz + 2; ++K)
      for (int J = 0; J < g.ny + 2; ++J)
        for (int I = 0; I < g.nx + 2; ++I) {
          const bool act = f == 0 ? g.ux_active(I, J, K) : f == 1 ? g.uy_active(I, J, K)
                           : f == 2 ? g.uz_active(I, J, K) : g.p_active(I, J, K);
          if (!act) continue;
          column(g, f, I, J, K, col);
          const int rj = row[(size_t)f * F + g.at(g.idx(I, J, K))];
          for (long r = 0; r < n; ++r) {
            double s = 0.0;
            for (auto& [code, v] : col) {
              const int ff = (int)(code / F), slot = (int)(code % F);
              const int c = row[(size_t)ff * F + g.at(slot)];
              CHECK(c >= 0, "stencil reaches a non-unknown");
              if (c >= 0) s += inv[(size_t)r * n + c] * v;
            }
            err = std::fmax(err, std::fabs(s - (r == rj)));
          }
          ++j;
        }
  for (long r = 0; r < n; ++r)
    for (long c = 0; c < r; ++c) asym = std::fmax(asym, std::fabs(inv[(size_t)r * n + c] - inv[(size_t)c * n + r]));
  double scale = 0.0;
  for (double v : inv) scale = std::fmax(scale, std::fabs(v));
  CHECK(j == n, "columns %ld", j);
  CHECK(err < 1e-8, "inv L~ - I = %g on %dx%dx%d", err, g.nx, g.ny, g.nz);
  CHECK(asym <= 1e-10 * scale, "inverse asymmetry %g (scale %g)", asym, scale);
}

static void check_cells(const Geom& g) {
  for (int period : {2, 3}) {
    const int nc = period * period * period;
    std::vector<int> cells[27];
    vanka_cells(g, cells, period);
    long total = 0;
    for (int c = 0; c < nc; ++c) {
      for (int s : cells[c]) {
        const int K = s / g.sz, J = (s % g.sz) / g.sy, I = (s % g.sz) % g.sy;
        const int colour = ((I - 1) % period) + period * ((J - 1) % period) + period * period * ((K - 1) % period);
        CHECK(colour == c, "slot %d in class %d, colour %d", s, c, colour);
        CHECK(I == 1 || I == g.nx || J == 1 || J == g.ny || K == 1 || K == g.nz, "slot %d not on the ring", s);
      }
      total += (long)cells[c].size();
    }
    const long ring = (long)g.nx * g.ny * g.nz - (long)std::max(g.nx - 2, 0) * std::max(g.ny - 2, 0) *
                                                     std::max(g.nz - 2, 0);
    CHECK(total == ring, "ring cells %ld vs %ld", total, ring);
  }
}

int main() {
  const int dims[][3] = {{2, 2, 2}, {4, 4, 4}, {8, 8, 8}, {4, 6, 8}, {3, 5, 2}, {6, 10, 8}, {32, 48, 16}};
  for (auto& d : dims) check_geometry(d[0], d[1], d[2]);
  check_invert();
  for (auto& d : dims) {
    const Geom g = make_geom(d[0], d[1], d[2], 1.0 / d[0], 0.7, 2e-3, 0);
    check_vanka(g);
    check_cells(g);
    if ((long)d[0] * d[1] * d[2] <= 512) check_coarse(g);
  }
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
