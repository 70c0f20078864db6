// Host-side set-up tables: level geometry, Vanka local inverses and the dense
// inverse of the coarsest-level operator.  Plain C++ (no HIP calls).
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

#include "geom.hpp"

namespace sg {

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Geometry of level l of a box with nx*ny*nz finest cells (Section 5: a
// coarse cell covers 2x2x2 fine cells; the spacing doubles).
inline Geom make_geom(int nx, int ny, int nz, double h, double eta, double gamma, int level) {
  Geom g{};
  g.nx = nx >> level;
  g.ny = ny >> level;
  g.nz = nz >> level;
  g.sy = (g.nx + 2) | 1;            // odd pitches: slot parity = colour
  g.sz = (g.sy * (g.ny + 2)) | 1;
  g.rows = (g.ny + 2) * (g.nz + 2);
  const long slots = (long)g.sz * (g.nz + 2);
  // at least 8 spare slots past the last plane (packs of the DGS kernels may
  // read up to 6 slots past a ghost plane), and a multiple of 8 (halves of 4)
  g.field = (int)((slots + 8 + 7) / 8 * 8);
  g.half = g.field / 2;
  g.h = h * std::ldexp(1.0, level);
  g.inv_h = 1.0 / g.h;
  g.c = eta / (g.h * g.h);
  g.eta = eta;
  g.gamma = gamma;
  return g;
}

// Levels allowed for a box: halving needs even axes; the automatic choice
// keeps >= 4 cells per axis, an explicit one >= 2.
inline int count_levels(int nx, int ny, int nz, int min_cells) {
  int L = 1;
  while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx / 2 >= min_cells && ny / 2 >= min_cells &&
         nz / 2 >= min_cells) {
    nx /= 2;
    ny /= 2;
    nz /= 2;
    ++L;
  }
  return L;
}

// In-place Gauss-Jordan inversion with partial pivoting of a row-major n x n
// matrix (n^3 multiply-adds: the inverse overwrites A column by column, no
// augmented identity).  Returns false if a pivot is exactly zero.
inline bool invert(std::vector<double>& a, int n) {
  std::vector<int> swapped(n);
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::fabs(a[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      const double v = std::fabs(a[(size_t)r * n + k]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0) return false;
    swapped[k] = piv;
    if (piv != k)
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)piv * n + j], a[(size_t)k * n + j]);
    double* rk = &a[(size_t)k * n];
    const double d = 1.0 / rk[k];
    rk[k] = 1.0;
    for (int j = 0; j < n; ++j) rk[j] *= d;
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      double* rr = &a[(size_t)r * n];
      const double f = rr[k];
      if (f == 0.0) continue;
      rr[k] = 0.0;
      for (int j = 0; j < n; ++j) rr[j] -= f * rk[j];
    }
  }
  // the row swaps of A become column swaps of the inverse, in reverse order
  for (int k = n - 1; k >= 0; --k)
    if (swapped[k] != k)
      for (int r = 0; r < n; ++r) std::swap(a[(size_t)r * n + k], a[(size_t)r * n + swapped[k]]);
  return true;
}

// Inverse of the local saddle matrix C_i L~ C_i^T of a one-cell Vanka
// subdomain (Eq. mv) for each of the 64 face-activity types.  Local order:
// u_x(minus), u_x(plus), u_y(minus), u_y(plus), u_z(minus), u_z(plus), p.
// Entries of L~ between these unknowns: 6 eta/h^2 on velocity diagonals,
// -eta/h^2 between the two faces of an axis (lattice neighbours), +1/h / -1/h
// between the minus / plus face and p (B^T and B), -gamma for p.  Inactive
// slots are removed; their rows and columns of the inverse are zero.
// Output: 64 blocks of 8x8 doubles (row-major, 7x7 used).
inline bool vanka_inverses(const Geom& g, std::vector<double>& out) {
  out.assign(64 * 64, 0.0);
  for (int type = 0; type < 64; ++type) {
    int map[7], n = 0;
    for (int s = 0; s < 6; ++s)
      if (type & (1 << s)) map[n++] = s;
    map[n++] = 6;
    std::vector<double> k((size_t)n * n, 0.0);
    auto entry = [&](int a, int b) -> double {
      if (a == 6 && b == 6) return -g.gamma;
      if (a == 6 || b == 6) {
        const int f = a == 6 ? b : a;
        return (f & 1) ? -g.inv_h : g.inv_h;
      }
      if (a == b) return 6.0 * g.c;
      if (a / 2 == b / 2) return -g.c;
      return 0.0;
    };
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) k[(size_t)i * n + j] = entry(map[i], map[j]);
    if (!invert(k, n)) return false;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) out[type * 64 + map[i] * 8 + map[j]] = k[(size_t)i * n + j];
  }
  return true;
}

// Dense L~ at a (small) level, in the order of `dof` (element offsets inside a
// state vector: all u_x, then u_y, u_z, p, each x-fastest), then inverted.
// The matrix is assembled on slot codes f * F + s (slot arithmetic for the
// neighbours); `dof` holds the matching element offsets f * F + at(s).
inline bool coarse_inverse(const Geom& g, std::vector<int>& dof, std::vector<double>& inv) {
  dof.clear();
  const int F = g.field;
  std::vector<int> pos((size_t)4 * F, -1);   // slot code -> row
  std::vector<int> code;                     // row -> slot code
  for (int f = 0; f < 4; ++f)
    for (int K = 0; K < g.nz + 2; ++K)
      for (int J = 0; J < g.ny + 2; ++J)
        for (int I = 0; I < g.nx + 2; ++I) {
          const bool act = f == 0 ? g.ux_active(I, J, K)
                           : f == 1 ? g.uy_active(I, J, K)
                           : f == 2 ? g.uz_active(I, J, K)
                                    : g.p_active(I, J, K);
          if (act) {
            const int slot = g.idx(I, J, K);
            pos[(size_t)f * F + slot] = (int)code.size();
            code.push_back(f * F + slot);
            dof.push_back(f * F + g.at(slot));
          }
        }
  const int n = (int)code.size();
  std::vector<double> a((size_t)n * n, 0.0);
  auto add = [&](int row, long col_code, double v) {
    const int c = pos[(size_t)col_code];
    if (c >= 0) a[(size_t)row * n + c] += v;
  };
  const int strides[3] = {1, g.sy, g.sz};
  for (int r = 0; r < n; ++r) {
    const int e = code[r];
    const int f = e / F, s = e % F;
    if (f < 3) {
      add(r, e, 6.0 * g.c);
      for (int a2 = 0; a2 < 3; ++a2) {
        add(r, e - strides[a2], -g.c);
        add(r, e + strides[a2], -g.c);
      }
      add(r, 3L * F + s, g.inv_h);                 // p of the cell on the plus side
      add(r, 3L * F + s - strides[f], -g.inv_h);   // p of the cell on the minus side
    } else {
      for (int a2 = 0; a2 < 3; ++a2) {
        add(r, (long)a2 * F + s + strides[a2], -g.inv_h);
        add(r, (long)a2 * F + s, g.inv_h);
      }
      add(r, e, -g.gamma);
    }
  }
  if (!invert(a, n)) return false;
  inv.swap(a);
  return true;
}

// Slots of the V1 cells (cells with a face on the Dirichlet layer), split by
// colour class (i mod q) + q (j mod q) + q^2 (k mod q), 0-based i, j, k;
// q = 2 gives the 8 classes of Section 6, q = 3 27 classes.  `cells` has q^3
// entries.
inline void vanka_cells(const Geom& g, std::vector<int>* cells, int period = 2) {
  const int nc = period * period * period;
  for (int c = 0; c < nc; ++c) cells[c].clear();
  for (int K = 1; K <= g.nz; ++K)
    for (int J = 1; J <= g.ny; ++J)
      for (int I = 1; I <= g.nx; ++I) {
        const bool ring = I == 1 || I == g.nx || J == 1 || J == g.ny || K == 1 || K == g.nz;
        if (!ring) continue;
        const int colour = period == 2 ? Geom::vanka_colour(I, J, K)
                                       : ((I - 1) % period) + period * ((J - 1) % period) +
                                             period * period * ((K - 1) % period);
        cells[colour].push_back(g.idx(I, J, K));
      }
}

}  // namespace sg
