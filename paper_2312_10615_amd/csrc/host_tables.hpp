// Host-side set-up tables: level geometry, Vanka local inverses and the dense
// inverse of the coarsest-level operator.  Plain C++ (no HIP calls).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <unordered_map>
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
// subdomain (Eq. mv).  Local order: u_x(minus), u_x(plus), u_y(minus),
// u_y(plus), u_z(minus), u_z(plus), p.  Entries of L~ between these unknowns:
// nd[r] eta/h^2 on velocity diagonals (6 unless exterior cells are near),
// -eta/h^2 between the two faces of an axis (lattice neighbours), +1/h / -1/h
// between the minus / plus face and p (B^T and B), -gamma for p.  Slots whose
// bit in `bits` is clear are not unknowns; their rows and columns of the
// inverse are zero.  Output: one 8x8 block (row-major, 7x7 used).
inline bool local_inverse(const Geom& g, int bits, const int* nd, double* out) {
  int map[7], n = 0;
  for (int s = 0; s < 6; ++s)
    if (bits & (1 << s)) map[n++] = s;
  map[n++] = 6;
  std::vector<double> k((size_t)n * n, 0.0);
  auto entry = [&](int a, int b) -> double {
    if (a == 6 && b == 6) return -g.gamma;
    if (a == 6 || b == 6) {
      const int f = a == 6 ? b : a;
      return (f & 1) ? -g.inv_h : g.inv_h;
    }
    if (a == b) return nd[a] * g.c;
    if (a / 2 == b / 2) return -g.c;
    return 0.0;
  };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) k[(size_t)i * n + j] = entry(map[i], map[j]);
  if (!invert(k, n)) return false;
  for (int i = 0; i < 64; ++i) out[i] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[map[i] * 8 + map[j]] = k[(size_t)i * n + j];
  return true;
}

// The 64 face-activity types of a box level (every diagonal 6 eta/h^2).
// Output: 64 blocks of 8x8 doubles.
inline bool vanka_inverses(const Geom& g, std::vector<double>& out) {
  out.assign(64 * 64, 0.0);
  const int six[6] = {6, 6, 6, 6, 6, 6};
  for (int type = 0; type < 64; ++type)
    if (!local_inverse(g, type, six, &out[(size_t)type * 64])) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Labelled domains (Section 5).  Cell labels of the padded box, one byte per
// cell, x fastest: (nx+2)(ny+2)(nz+2).  Beyond the array the outer layer
// repeats (so an exterior outflow layer stays exterior under coarsening).
// ---------------------------------------------------------------------------
enum : uint8_t { CELL_INTERIOR = 0, CELL_DIRICHLET = 1, CELL_EXTERIOR = 2 };

struct Labels {
  int nx = 0, ny = 0, nz = 0;
  std::vector<uint8_t> v;
  long idx(int i, int j, int k) const { return i + (long)(nx + 2) * (j + (long)(ny + 2) * k); }
  uint8_t at(int i, int j, int k) const {
    i = std::min(std::max(i, 0), nx + 1);
    j = std::min(std::max(j, 0), ny + 1);
    k = std::min(std::max(k, 0), nz + 1);
    return v[idx(i, j, k)];
  }
};

// Section 5: a coarse cell is Dirichlet if it covers a Dirichlet cell, else
// interior if it covers an interior cell, else exterior.  Coarse padded cell
// C covers fine padded cells 2C-1 and 2C per axis.
inline Labels coarsen(const Labels& f) {
  Labels c;
  c.nx = f.nx / 2;
  c.ny = f.ny / 2;
  c.nz = f.nz / 2;
  c.v.assign((size_t)(c.nx + 2) * (c.ny + 2) * (c.nz + 2), CELL_EXTERIOR);
  for (int K = 0; K < c.nz + 2; ++K)
    for (int J = 0; J < c.ny + 2; ++J)
      for (int I = 0; I < c.nx + 2; ++I) {
        bool dir = false, inte = false;
        for (int d = 0; d < 8; ++d) {
          const uint8_t l = f.at(2 * I - 1 + (d & 1), 2 * J - 1 + ((d >> 1) & 1), 2 * K - 1 + (d >> 2));
          dir = dir || l == CELL_DIRICHLET;
          inte = inte || l == CELL_INTERIOR;
        }
        c.v[c.idx(I, J, K)] = dir ? CELL_DIRICHLET : inte ? CELL_INTERIOR : CELL_EXTERIOR;
      }
  return c;
}

// Cells within `reach` steps (faces, edges and corners) of a marked cell;
// nothing lies beyond the array.  Separable: a 1D window per axis.
inline void dilate(std::vector<uint8_t>& m, int nx, int ny, int nz, int reach) {
  const int n[3] = {nx, ny, nz};
  const long st[3] = {1, nx, (long)nx * ny};
  std::vector<uint8_t> t(m.size());
  for (int a = 0; a < 3; ++a) {
    for (long e = 0; e < (long)m.size(); ++e) {
      const int c = (int)((e / st[a]) % n[a]);
      uint8_t v = 0;
      for (int o = -reach; o <= reach && !v; ++o)
        if (c + o >= 0 && c + o < n[a]) v = m[e + o * st[a]];
      t[e] = v;
    }
    m.swap(t);
  }
}

// Flag words of a labelled level (layout in geom.hpp) and its Vanka
// local-matrix types (at most 1024).  Faces: an unknown when one of the two
// cells beside it is interior and neither is Dirichlet (a face between an
// interior and an exterior cell carries the Neumann condition and is
// solved); V1 cells: interior cells within one cell of a Dirichlet cell or
// two of an exterior cell; n_f: the lattice neighbours of the face that are
// unknowns or Dirichlet values (a neighbour with no interior and no
// Dirichlet cell beside it lies on the exterior side: zero normal derivative).
struct LevelLabels {
  std::vector<uint32_t> flags;   // g.field words, element at(s)
  std::vector<double> kinv;      // ntypes blocks of 8x8
  int ntypes = 0;
  long n_dofs = 0;               // unknowns of the level
  long n_cells = 0;              // interior cells
  bool neumann = false;          // some unknown face borders an exterior cell
};

inline bool label_tables(const Geom& g, const Labels& lab, LevelLabels& out) {
  const int NX = g.nx + 2, NY = g.ny + 2, NZ = g.nz + 2;
  std::vector<uint8_t> nearD((size_t)NX * NY * NZ), nearE((size_t)NX * NY * NZ);
  for (long e = 0; e < (long)nearD.size(); ++e) {
    nearD[e] = lab.v[e] == CELL_DIRICHLET;
    nearE[e] = lab.v[e] == CELL_EXTERIOR;
  }
  dilate(nearD, NX, NY, NZ, 1);
  dilate(nearE, NX, NY, NZ, 2);
  auto v1 = [&](int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= NX || j >= NY || k >= NZ) return false;
    const long e = lab.idx(i, j, k);
    return lab.v[e] == CELL_INTERIOR && (nearD[e] || nearE[e]);
  };
  // kind of the face between cells c0 and c1: 0 outside (exterior side), 1 Dirichlet value, 2 unknown
  auto kind = [&](uint8_t a, uint8_t b) {
    if (a == CELL_DIRICHLET || b == CELL_DIRICHLET) return 1;
    return (a == CELL_INTERIOR || b == CELL_INTERIOR) ? 2 : 0;
  };
  const int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  auto face_kind = [&](int f, int I, int J, int K) {   // face f of padded cell (I,J,K): its minus face
    return kind(lab.at(I - d[f][0], J - d[f][1], K - d[f][2]), lab.at(I, J, K));
  };
  out.flags.assign(g.field, 0u);
  out.n_dofs = out.n_cells = 0;
  out.neumann = false;
  for (int K = 0; K < NZ; ++K)
    for (int J = 0; J < NY; ++J)
      for (int I = 0; I < NX; ++I) {
        uint32_t w = 0;
        for (int f = 0; f < 3; ++f) {
          if (face_kind(f, I, J, K) != 2) continue;
          w |= 1u << f;
          const int Im = I - d[f][0], Jm = J - d[f][1], Km = K - d[f][2];
          if (!v1(Im, Jm, Km) && !v1(I, J, K)) w |= 16u << f;
          int nd = 0;
          for (int a = 0; a < 3; ++a)
            for (int sg = -1; sg <= 1; sg += 2)
              nd += face_kind(f, I + sg * d[a][0], J + sg * d[a][1], K + sg * d[a][2]) != 0;
          w |= (uint32_t)nd << (8 + 3 * f);
          const uint8_t lm = lab.at(Im, Jm, Km), lp = lab.at(I, J, K);
          if (lm == CELL_EXTERIOR || lp == CELL_EXTERIOR) out.neumann = true;
          ++out.n_dofs;
        }
        if (lab.at(I, J, K) == CELL_INTERIOR) {
          w |= 8u;
          if (!v1(I, J, K)) w |= 128u;
          ++out.n_dofs;
          ++out.n_cells;
        }
        out.flags[g.at(g.idx(I, J, K))] = w;
      }
  // Vanka types of the V1 cells, keyed on their face bits and diagonals
  std::unordered_map<uint64_t, int> types;
  out.kinv.clear();
  Geom gh = g;
  gh.flags = out.flags.data();
  for (int K = 1; K <= g.nz; ++K)
    for (int J = 1; J <= g.ny; ++J)
      for (int I = 1; I <= g.nx; ++I) {
        if (!v1(I, J, K)) continue;
        const int bits = gh.vface_bits(I, J, K);
        int nd[6];
        const int slot[6] = {g.idx(I, J, K), g.idx(I + 1, J, K), g.idx(I, J, K), g.idx(I, J + 1, K),
                             g.idx(I, J, K), g.idx(I, J, K + 1)};
        uint64_t key = (uint64_t)bits;
        for (int r = 0; r < 6; ++r) {
          nd[r] = (bits >> r & 1) ? gh.nd(r / 2, slot[r]) : 6;
          key |= (uint64_t)nd[r] << (6 + 3 * r);
        }
        auto it = types.find(key);
        int t;
        if (it == types.end()) {
          t = (int)types.size();
          if (t >= 1024) return false;
          types.emplace(key, t);
          out.kinv.resize((size_t)(t + 1) * 64);
          if (!local_inverse(g, bits, nd, &out.kinv[(size_t)t * 64])) return false;
        } else {
          t = it->second;
        }
        out.flags[g.at(g.idx(I, J, K))] |= (uint32_t)t << 17;
      }
  out.ntypes = (int)types.size();
  return true;
}

// Dense L~ at a (small) level, in the order of `dof` (element offsets inside a
// state vector: all u_x, then u_y, u_z, p, each x-fastest), then inverted.
// A labelled level's Geom must point at its host flag words.
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
      add(r, e, g.nd(f, s) * g.c);
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

// Slots of the V1 cells (a box: cells with a face on the Dirichlet layer), split by
// colour class (i mod q) + q (j mod q) + q^2 (k mod q), 0-based i, j, k;
// q = 2 gives the 8 classes of Section 6, q = 3 27 classes.  `cells` has q^3
// entries.
inline void vanka_cells(const Geom& g, std::vector<int>* cells, int period = 2) {
  const int nc = period * period * period;
  for (int c = 0; c < nc; ++c) cells[c].clear();
  for (int K = 1; K <= g.nz; ++K)
    for (int J = 1; J <= g.ny; ++J)
      for (int I = 1; I <= g.nx; ++I) {
        // a labelled level's Geom points at its host flag words: V1 = cells with p not in V2
        const bool ring = g.flags ? g.p_active(I, J, K) && !g.p_v2(I, J, K)
                                  : I == 1 || I == g.nx || J == 1 || J == g.ny || K == 1 || K == g.nz;
        if (!ring) continue;
        const int colour = period == 2 ? Geom::vanka_colour(I, J, K)
                                       : ((I - 1) % period) + period * ((J - 1) % period) +
                                             period * period * ((K - 1) % period);
        cells[colour].push_back(g.idx(I, J, K));
      }
}

}  // namespace sg
