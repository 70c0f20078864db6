// The hot stencil passes with V cells per thread, for the single box and the
// batch: the distributive Gauss-Seidel steps (Alg. 2, Eq. dist, Eq. ldist)
// and the operator passes (Eq. 2).  The operator passes compute what the
// one-cell apply_item in kernels.hpp computes, cell by cell and in the same
// order of operations; only the memory access is different.
//
// With the red/black split every stencil neighbour of a slot of parity par
// sits in the other half, at an element shifted by a constant: slot s + o of
// the cell whose own element is e is element
//     ((par + o) & 1) * half + e + ((par + o) >> 1).
// So the V consecutive own elements of a thread have V consecutive
// neighbours for every offset o, and each operand of the stencil is one wide
// load (16 bytes: two doubles or four floats) instead of V narrow ones.  The
// stencil kernels are bound by the rate at which the texture-address units
// take load instructions, which this divides by V.
//
// A thread takes V consecutive cells of one colour inside one row; the last
// pack of a row may be short (n < V cells).  Loads may run past the row into
// the next row's elements (always inside the field, whose ghost planes and
// rows are wider than a pack); stores of a short pack go cell by cell, so no
// element another thread owns is written.  Every element a full pack stores
// belongs to its cells alone (own element, or a plus face whose minus-side
// cell is in the pack), so unchanged values written back race with nothing.
#pragma once

#include "kernels.hpp"

namespace sg {

typedef double wd2 __attribute__((ext_vector_type(2), aligned(8)));
typedef float wf2 __attribute__((ext_vector_type(2), aligned(4)));
typedef float wf4 __attribute__((ext_vector_type(4), aligned(4)));

template <typename T, int V>
struct Pack {
  T v[V];
};

// V consecutive elements in one load (the hardware accepts dword alignment).
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> ldp(const T* p) {
  Pack<T, V> r;
  if constexpr (V == 1) {
    r.v[0] = p[0];
  } else if constexpr (sizeof(T) == 8 && V == 2) {
    const wd2 w = *(const wd2*)p;
    r.v[0] = w.x;
    r.v[1] = w.y;
  } else if constexpr (sizeof(T) == 4 && V == 2) {
    const wf2 w = *(const wf2*)p;
    r.v[0] = w.x;
    r.v[1] = w.y;
  } else {
    static_assert(sizeof(T) == 4 && V == 4, "pack of 16 bytes at most");
    const wf4 w = *(const wf4*)p;
    r.v[0] = w.x;
    r.v[1] = w.y;
    r.v[2] = w.z;
    r.v[3] = w.w;
  }
  return r;
}

template <typename T, int V>
__device__ __forceinline__ void stp(T* p, const Pack<T, V>& r) {
  if constexpr (V == 1) {
    p[0] = r.v[0];
  } else if constexpr (sizeof(T) == 8 && V == 2) {
    wd2 w;
    w.x = r.v[0];
    w.y = r.v[1];
    *(wd2*)p = w;
  } else if constexpr (sizeof(T) == 4 && V == 2) {
    wf2 w;
    w.x = r.v[0];
    w.y = r.v[1];
    *(wf2*)p = w;
  } else {
    wf4 w;
    w.x = r.v[0];
    w.y = r.v[1];
    w.z = r.v[2];
    w.w = r.v[3];
    *(wf4*)p = w;
  }
}

// Store the cells of a pack that are flagged; a full pack in one store.
template <typename T, int V>
__device__ __forceinline__ void stp_cells(T* p, const Pack<T, V>& r, int n, const bool* act) {
  if (n == V) {
    stp<T, V>(p, r);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (i < n && act[i]) p[i] = r.v[i];
  }
}

// The pack of this thread: cells I0, I0+2, ... of row (J, K), colour parity par.
template <int V>
struct RowPack {
  int e0;   // element (inside the half) of the first cell
  int n;    // cells of the row in the pack, 1..V
  int I0, J, K;
  int par;
  int half;
  // element of slot s_i + o (cell i of the pack is element el(o) + i)
  __device__ __forceinline__ int el(int o) const {
    const int q = par + o;
    return (q & 1) * half + e0 + (q >> 1);
  }
};

// Packs of a row of one parity; only interior rows hold cells that change.
template <int V>
__host__ __device__ inline int pack_per_row(const Geom& g) {
  return (((g.sy + 1) >> 1) + V - 1) / V;
}

// Pack m of row (J, K); false when the row or the pack holds no cell.
template <int V>
__device__ __forceinline__ bool row_pack_at(const Geom& g, int par, int m, int J, int K, RowPack<V>& rp) {
  rp.J = J;
  rp.K = K;
  if (J < 1 || J > g.ny || K < 1 || K > g.nz) return false;
  const int q = (par + rp.J + rp.K) & 1;  // I parity of the row's slots of parity par
  const int nrow = (g.sy - q + 1) >> 1;
  const int first = m * V;
  if (first >= nrow) return false;
  rp.n = nrow - first < V ? nrow - first : V;
  rp.I0 = q + 2 * first;
  rp.e0 = ((g.sy * rp.J + g.sz * rp.K + q) >> 1) + first;
  rp.par = par;
  rp.half = g.half;
  return true;
}

// The pack of this thread in the slab mapping of the single-box kernels.
template <int V>
__device__ __forceinline__ bool row_pack(const Geom& g, int par, RowPack<V>& rp) {
  int m, J, K;
  if (!slab_item(g, pack_per_row<V>(g), m, J, K)) return false;
  return row_pack_at<V>(g, par, m, J, K, rp);
}

// Velocity Gauss-Seidel step on the V2 faces of one colour: u += r / (6 eta/h^2).
// Same-colour faces are not lattice neighbours and p is fixed, so the class
// updates at once.  Every lattice neighbour of a V2 face is an unknown (V2
// faces lie two cells or more from Dirichlet and three or more from exterior
// cells), so its diagonal is 6 eta/h^2 in a labelled domain as in a box.
template <typename T, typename TB, int V>
__device__ __forceinline__ void dgs_u_pack(const Geom& g, T* __restrict__ x, const TB* __restrict__ b, const RowPack<V>& rp) {
  const int F = g.field;
  const T* p = x + 3 * F;
  const T dinv = (T)(1.0 / (6.0 * g.c));
  const int eo = rp.el(0);
  const Pack<T, V> P = ldp<T, V>(p + eo);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    bool act[V];
    bool any = false;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int I = rp.I0 + 2 * i;
      act[i] = i < rp.n && (f == 0 ? g.ux_v2(I, rp.J, rp.K) : f == 1 ? g.uy_v2(I, rp.J, rp.K) : g.uz_v2(I, rp.J, rp.K));
      any = any || act[i];
    }
    if (!any) continue;
    T* u = x + f * F;
    const int ps = f == 0 ? 1 : f == 1 ? g.sy : g.sz;
    Pack<T, V> U = ldp<T, V>(u + eo);
    const Pack<TB, V> Bv = ldp<TB, V>(b + f * F + eo);
    const Pack<T, V> xm = ldp<T, V>(u + rp.el(-1)), xp = ldp<T, V>(u + rp.el(1));
    const Pack<T, V> ym = ldp<T, V>(u + rp.el(-g.sy)), yp = ldp<T, V>(u + rp.el(g.sy));
    const Pack<T, V> zm = ldp<T, V>(u + rp.el(-g.sz)), zp = ldp<T, V>(u + rp.el(g.sz));
    const Pack<T, V> Pm = ldp<T, V>(p + rp.el(-ps));
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (!act[i]) continue;
      const T lap = T(6) * U.v[i] - xm.v[i] - xp.v[i] - ym.v[i] - yp.v[i] - zm.v[i] - zp.v[i];
      const T row = (T)g.c * lap + (P.v[i] - Pm.v[i]) * (T)g.inv_h;
      U.v[i] = U.v[i] + ((T)Bv.v[i] - row) * dinv;
    }
    stp_cells<T, V>(u + eo, U, rp.n, act);
  }
}

template <typename T, typename TB, int V>
__global__ __launch_bounds__(BS) void k_dgs_u_v(Geom g, T* __restrict__ x, const TB* __restrict__ b, int colour) {
  RowPack<V> rp;
  if (row_pack<V>(g, colour ^ 1, rp)) dgs_u_pack<T, TB, V>(g, x, b, rp);
}

// ---------------------------------------------------------------------------
// DGS pressure steps.  The pressures go by the eight colour classes
// (i&1) + 2(j&1) + 4(k&1) (0-based cell indices), taken 0..7 in the forward
// sweep and 7..0 in the reverse one.  Two cells are face neighbours only when
// their classes differ in one bit, and then the class with that bit clear
// comes first; so the classes of equal bit count are mutually independent and
// may run together, and the sweep runs as four stages (bit count 0, 1, 2, 3)
// with the same results.  Inside a row of one parity every cell has the same
// i parity, so the whole row belongs to one class and one stage.
// ---------------------------------------------------------------------------
struct RowBits {
  int bx, by, bz, stage;
};

template <int V>
__device__ __forceinline__ RowBits row_bits(const RowPack<V>& rp) {
  RowBits r;
  r.bx = (rp.I0 - 1) & 1;
  r.by = (rp.J - 1) & 1;
  r.bz = (rp.K - 1) & 1;
  r.stage = r.bx + r.by + r.bz;
  return r;
}

// Forward-sweep pressure step on the V2 cells of a pack (Eq. dist): delta =
// r_j / d_j with d_j = (L~ M)_jj = -6 (1 + gamma eta) / h^2, then x moves along
// the column m_j of M = [[I, -B^T], [0, eta B B^T]]: the cell's six faces get
// -+delta/h and p_j gets 6 eta delta / h^2 here; the -eta delta / h^2 of each
// neighbour pressure is gathered by the neighbour in the next launch.  A V2
// cell's six faces and six neighbours are all unknowns, so m_j is the full
// interior column.  P holds p_j on entry (after any gather) and on exit.
template <typename T, typename TB, int V>
__device__ __forceinline__ void dgs_pf_own_step(const Geom& g, T* __restrict__ x, const TB* __restrict__ b,
                                                T* __restrict__ dscr, const RowPack<V>& rp, const bool* acto,
                                                Pack<T, V>& P) {
  const int F = g.field;
  T* ux = x;
  T* uy = x + F;
  T* uz = x + 2 * F;
  const double ih2 = g.inv_h * g.inv_h;
  const int eo = rp.el(0), ex = rp.el(1), ey = rp.el(g.sy), ez = rp.el(g.sz);
  Pack<T, V> X0 = ldp<T, V>(ux + eo), X1 = ldp<T, V>(ux + ex);
  Pack<T, V> Y0 = ldp<T, V>(uy + eo), Y1 = ldp<T, V>(uy + ey);
  Pack<T, V> Z0 = ldp<T, V>(uz + eo), Z1 = ldp<T, V>(uz + ez);
  const Pack<TB, V> Bp = ldp<TB, V>(b + 3 * F + eo);
  Pack<T, V> D;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    D.v[i] = T(0);
    if (!acto[i]) continue;
    const T div = (X1.v[i] - X0.v[i]) + (Y1.v[i] - Y0.v[i]) + (Z1.v[i] - Z0.v[i]);
    const T r = (T)Bp.v[i] - (-div * (T)g.inv_h - (T)g.gamma * P.v[i]);
    const T delta = r / (T)(-6.0 * (1.0 + g.gamma * g.eta) * ih2);
    D.v[i] = delta;
    const T dh = delta * (T)g.inv_h;
    X0.v[i] = X0.v[i] - dh;
    X1.v[i] = X1.v[i] + dh;
    Y0.v[i] = Y0.v[i] - dh;
    Y1.v[i] = Y1.v[i] + dh;
    Z0.v[i] = Z0.v[i] - dh;
    Z1.v[i] = Z1.v[i] + dh;
    P.v[i] = P.v[i] + (T)(6.0 * g.eta * ih2) * delta;
  }
  stp_cells<T, V>(dscr + eo, D, rp.n, acto);
  stp_cells<T, V>(ux + eo, X0, rp.n, acto);
  stp_cells<T, V>(ux + ex, X1, rp.n, acto);
  stp_cells<T, V>(uy + eo, Y0, rp.n, acto);
  stp_cells<T, V>(uy + ey, Y1, rp.n, acto);
  stp_cells<T, V>(uz + eo, Z0, rp.n, acto);
  stp_cells<T, V>(uz + ez, Z1, rp.n, acto);
}

// Launch t (0..4) of the forward pressure sweep, over the rows of stage t
// and stage t - 2 (both of colour t & 1).  First every active cell takes the
// -(eta/h^2) delta of its V2 neighbours in stage t - 1 (along an axis the two
// neighbours lie one stage down when the cell's bit for that axis is set, one
// stage up otherwise); then a stage-t V2 cell makes its own step from that
// pressure.  Every launch reads deltas written by the previous one only, and
// its own steps touch faces of stage-t cells, which share none.
template <typename T, typename TB, int V>
__device__ __forceinline__ void dgs_pf_stage_pack(const Geom& g, T* __restrict__ x, const TB* __restrict__ b,
                                                  T* __restrict__ dscr, const RowPack<V>& rp, int t) {
  const RowBits rb = row_bits<V>(rp);
  if (rb.stage != t && rb.stage != t - 2) return;
  const bool own = rb.stage == t;
  const bool gx = t > 0 && (own ? rb.bx : !rb.bx), gy = t > 0 && (own ? rb.by : !rb.by),
             gz = t > 0 && (own ? rb.bz : !rb.bz);
  bool actn[V], acto[V];
  bool any = false, anyo = false;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    actn[i] = i < rp.n && g.p_active(rp.I0 + 2 * i, rp.J, rp.K);
    acto[i] = own && i < rp.n && g.p_v2(rp.I0 + 2 * i, rp.J, rp.K);
    any = any || actn[i];
    anyo = anyo || acto[i];
  }
  if (!any || (!anyo && !gx && !gy && !gz)) return;
  T* p = x + 3 * g.field;
  const int eo = rp.el(0);
  Pack<T, V> P = ldp<T, V>(p + eo);
  const int J = rp.J, K = rp.K;
  Pack<T, V> sum;
#pragma unroll
  for (int i = 0; i < V; ++i) sum.v[i] = T(0);
  if (gx) {
    const Pack<T, V> dm = ldp<T, V>(dscr + rp.el(-1)), dp = ldp<T, V>(dscr + rp.el(1));
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int I = rp.I0 + 2 * i;
      if (g.p_v2(I - 1, J, K)) sum.v[i] += dm.v[i];
      if (g.p_v2(I + 1, J, K)) sum.v[i] += dp.v[i];
    }
  }
  if (gy) {
    const Pack<T, V> dm = ldp<T, V>(dscr + rp.el(-g.sy)), dp = ldp<T, V>(dscr + rp.el(g.sy));
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int I = rp.I0 + 2 * i;
      if (g.p_v2(I, J - 1, K)) sum.v[i] += dm.v[i];
      if (g.p_v2(I, J + 1, K)) sum.v[i] += dp.v[i];
    }
  }
  if (gz) {
    const Pack<T, V> dm = ldp<T, V>(dscr + rp.el(-g.sz)), dp = ldp<T, V>(dscr + rp.el(g.sz));
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int I = rp.I0 + 2 * i;
      if (g.p_v2(I, J, K - 1)) sum.v[i] += dm.v[i];
      if (g.p_v2(I, J, K + 1)) sum.v[i] += dp.v[i];
    }
  }
  if (gx || gy || gz) {
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (actn[i] && sum.v[i] != T(0)) P.v[i] = P.v[i] - (T)(g.eta * g.inv_h * g.inv_h) * sum.v[i];
  }
  if (anyo) dgs_pf_own_step<T, TB, V>(g, x, b, dscr, rp, acto, P);
  stp_cells<T, V>(p + eo, P, rp.n, (gx || gy || gz) ? actn : acto);
}

template <typename T, typename TB, int V>
__global__ __launch_bounds__(BS) void k_dgs_pf_v(Geom g, T* __restrict__ x, const TB* __restrict__ b,
                                                 T* __restrict__ dscr, int t) {
  RowPack<V> rp;
  if (row_pack<V>(g, (t & 1) ^ 1, rp)) dgs_pf_stage_pack<T, TB, V>(g, x, b, dscr, rp, t);
}

// Reverse-sweep pressure step (Gauss-Seidel on M^T L~, Eq. ldist) on the V2
// cells of a pack: p_j += (m_j . r) / d_j, r = b - L~ x, where m_j =
// (-B^T e_j, eta B B^T e_j) is column j of M.  The row m_j^T L~ is column j
// of L~ M: velocity part (-A B^T + eta B^T B B^T) e_j, pressure part
// -(1 + gamma eta) B B^T e_j.  When the six faces and six neighbours of j are
// unknowns (every V2 cell), B B^T e_j is the lattice stencil
// (6 e_j - neighbours)/h^2 and A acts on the faces of j as the lattice
// Laplacian; the lattice gradient commutes with the lattice Laplacian, so the
// velocity part vanishes (A = -eta Lap_u, B B^T = -Lap_p there).  Hence
//   m_j . r = m_j . b + (1 + gamma eta)(6 p_j - sum_k p_k)/h^2,
//   m_j . b = (1/h) sum_a (b(plus face) - b(minus face)) + (eta/h^2)(6 b_j - sum_k b_k):
// 13 wide loads of b and 7 of p per pack, where the thirteen local residuals
// of m_j . r read ~56 operands.  Same update up to rounding (and without the
// residual form's cancellation of the velocity terms).  Only p_j changes, and
// no value read here is a pressure of the same stage.
template <typename T, typename TB, int V>
__device__ __forceinline__ void dgs_pr_pack(const Geom& g, T* __restrict__ x, const TB* __restrict__ b, const RowPack<V>& rp) {
  bool act[V];
  bool any = false;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    act[i] = i < rp.n && g.p_v2(rp.I0 + 2 * i, rp.J, rp.K);
    any = any || act[i];
  }
  if (!any) return;
  const int F = g.field;
  T* p = x + 3 * F;
  const TB* bp = b + 3 * F;
  const int eo = rp.el(0), exm = rp.el(-1), exp_ = rp.el(1), eym = rp.el(-g.sy), eyp = rp.el(g.sy),
            ezm = rp.el(-g.sz), ezp = rp.el(g.sz);
  const Pack<TB, V> bx0 = ldp<TB, V>(b + eo), bx1 = ldp<TB, V>(b + exp_);
  const Pack<TB, V> by0 = ldp<TB, V>(b + F + eo), by1 = ldp<TB, V>(b + F + eyp);
  const Pack<TB, V> bz0 = ldp<TB, V>(b + 2 * F + eo), bz1 = ldp<TB, V>(b + 2 * F + ezp);
  const Pack<TB, V> bj = ldp<TB, V>(bp + eo);
  const Pack<TB, V> bxm = ldp<TB, V>(bp + exm), bxp = ldp<TB, V>(bp + exp_), bym = ldp<TB, V>(bp + eym),
                    byp = ldp<TB, V>(bp + eyp), bzm = ldp<TB, V>(bp + ezm), bzp = ldp<TB, V>(bp + ezp);
  const Pack<T, V> pxm = ldp<T, V>(p + exm), pxp = ldp<T, V>(p + exp_), pym = ldp<T, V>(p + eym),
                   pyp = ldp<T, V>(p + eyp), pzm = ldp<T, V>(p + ezm), pzp = ldp<T, V>(p + ezp);
  Pack<T, V> P = ldp<T, V>(p + eo);
  const double ih2 = g.inv_h * g.inv_h;
  const double kap = 1.0 + g.gamma * g.eta;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    if (!act[i]) continue;
    const T fsum = ((T)bx1.v[i] - (T)bx0.v[i]) + ((T)by1.v[i] - (T)by0.v[i]) + ((T)bz1.v[i] - (T)bz0.v[i]);
    const T bsum = (T)bxm.v[i] + (T)bxp.v[i] + (T)bym.v[i] + (T)byp.v[i] + (T)bzm.v[i] + (T)bzp.v[i];
    const T psum = pxm.v[i] + pxp.v[i] + pym.v[i] + pyp.v[i] + pzm.v[i] + pzp.v[i];
    const T rt = (fsum * (T)g.inv_h + (T)(g.eta * ih2) * (T(6) * (T)bj.v[i] - bsum)) +
                 (T)(kap * ih2) * (T(6) * P.v[i] - psum);
    P.v[i] = P.v[i] + rt / (T)(-6.0 * kap * ih2);
  }
  stp_cells<T, V>(p + eo, P, rp.n, act);
}

// The rows of stage `stage` (colour stage & 1) of the reverse pressure sweep.
template <typename T, typename TB, int V>
__device__ __forceinline__ void dgs_pr_stage_pack(const Geom& g, T* __restrict__ x, const TB* __restrict__ b,
                                                  const RowPack<V>& rp, int stage) {
  if (row_bits<V>(rp).stage == stage) dgs_pr_pack<T, TB, V>(g, x, b, rp);
}

template <typename T, typename TB, int V>
__global__ __launch_bounds__(BS) void k_dgs_pr_v(Geom g, T* __restrict__ x, const TB* __restrict__ b, int stage) {
  RowPack<V> rp;
  if (row_pack<V>(g, (stage & 1) ^ 1, rp)) dgs_pr_stage_pack<T, TB, V>(g, x, b, rp, stage);
}

// ---------------------------------------------------------------------------
// A DGS sweep of a small level in one workgroup: each launch of the sweep
// (a velocity colour, a pressure launch or stage) becomes one pass over the
// level's packs, with a workgroup barrier in place of the launch boundary.
// The packs and their arithmetic are the launches', so the values are the
// same bit for bit.  On a level of a few thousand packs a pass costs the
// workgroup a memory round trip or two, where a graph-replayed launch costs
// several microseconds.
// ---------------------------------------------------------------------------
constexpr int DSWEEP_BS = 1024;
constexpr int DSWEEP_MAX_PACKS = 4096;  // packs of one pass a level may have to run this way

template <int V>
__host__ __device__ inline int dgs_small_packs(const Geom& g) {
  return pack_per_row<V>(g) * (g.ny + 2) * (g.nz + 2);
}

// dir 0: the forward sweep (velocities red, black; pressure launches t = 0..4
// as k_dgs_pf_v); dir 1: the reverse sweep (pressure stages 3..0; velocities
// black, red).
template <typename T, typename TB, int V>
__global__ __launch_bounds__(DSWEEP_BS) void k_dgs_small(Geom g, T* __restrict__ x, const TB* __restrict__ b,
                                                         T* __restrict__ dscr, int dir) {
  const int ppr = pack_per_row<V>(g), ry = g.ny + 2;
  const int n = dgs_small_packs<V>(g);
  auto pass = [&](int par, auto&& body) {
    for (int l = threadIdx.x; l < n; l += DSWEEP_BS) {
      const int r = l / ppr;
      RowPack<V> rp;
      if (row_pack_at<V>(g, par, l - r * ppr, r % ry, r / ry, rp)) body(rp);
    }
    __syncthreads();
  };
  if (dir == 0) {
    for (int col = 0; col < 2; ++col)
      pass(col ^ 1, [&](const RowPack<V>& rp) { dgs_u_pack<T, TB, V>(g, x, b, rp); });
    for (int t = 0; t <= 4; ++t)
      pass((t & 1) ^ 1, [&](const RowPack<V>& rp) { dgs_pf_stage_pack<T, TB, V>(g, x, b, dscr, rp, t); });
  } else {
    for (int st = 3; st >= 0; --st)
      pass((st & 1) ^ 1, [&](const RowPack<V>& rp) { dgs_pr_stage_pack<T, TB, V>(g, x, b, rp, st); });
    for (int col = 1; col >= 0; --col)
      pass(col ^ 1, [&](const RowPack<V>& rp) { dgs_u_pack<T, TB, V>(g, x, b, rp); });
  }
}

// ---------------------------------------------------------------------------
// The operator passes (the ApplyMode modes) with V slots per thread.  A thread
// takes V consecutive slots of one parity in one row, every row and both
// parities (ghost slots included: y gets 0 there).  The four rows are four
// stages: at the end of a stage the base element (and the uniform sizes) pass
// through an empty asm statement that also takes the stage's results, so the
// next stage's loads can neither be merged with earlier ones nor issued
// before the stage's arithmetic, and each stage holds only its own operands
// in registers (operands shared by two rows are loaded again, from the cache).
// ---------------------------------------------------------------------------
template <int V>
__host__ __device__ inline int slot_packs_per_row(const Geom& g) {
  return 2 * ((((g.sy + 1) >> 1) + V - 1) / V);
}

// Pack X (0 <= X < slot_packs_per_row) of row (J, K).
template <int V>
__device__ __forceinline__ bool slot_pack_at(const Geom& g, int X, int J, int K, RowPack<V>& rp) {
  const int ppr = slot_packs_per_row<V>(g) >> 1;
  rp.J = J;
  rp.K = K;
  const int q = X >= ppr;  // I parity of the pack's slots
  const int m = X - q * ppr;
  const int nrow = (g.sy - q + 1) >> 1;
  const int first = m * V;
  if (first >= nrow) return false;
  rp.n = nrow - first < V ? nrow - first : V;
  rp.I0 = q + 2 * first;
  rp.e0 = ((g.sy * rp.J + g.sz * rp.K + q) >> 1) + first;
  rp.par = (q + rp.J + rp.K) & 1;
  rp.half = g.half;
  return true;
}

template <int V>
__device__ __forceinline__ bool slot_pack(const Geom& g, RowPack<V>& rp) {
  int X, J, K;
  if (!slab_item(g, slot_packs_per_row<V>(g), X, J, K)) return false;
  return slot_pack_at<V>(g, X, J, K, rp);
}

// One pack of an operator pass; returns the pack's share of the reduction.
// The p row's operands are the centres and plus neighbours of the three
// velocity rows and the centre pressure, which the velocity stages load
// anyway: the pressure centre and the divergence, summed in the order of
// row_p, are carried from stage to stage (25 wide loads of x per pack
// instead of 34).
// The values of a pack go to sink(f, v) (field f, V values; ghost and
// non-unknown slots 0) in the modes that produce y.
// STAGED = false drops the stage fences, so that every load of the pack may
// issue at once (for kernels that run few waves per SIMD).
template <int MODE, typename T, typename TB, int V, bool STAGED = true, typename Sink>
__device__ __forceinline__ double apply_pack_to(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                                double gamma, const RowPack<V>& rp, Sink&& sink) {
  double acc = 0.0;
  int F = g.field;
  int sy = g.sy, sz = g.sz, hf = g.half;
  int eb = rp.e0;
  auto stage = [&](const T* dep) {
    if constexpr (!STAGED) return;
#pragma unroll
    for (int i = 0; i < V; ++i) asm volatile("" : "+v"(eb) : "v"(dep[i]));
    asm volatile("" : "+v"(eb), "+s"(F), "+s"(sy), "+s"(sz), "+s"(hf));
  };
  auto L = [&](int f, int o) {
    const int q = rp.par + o;
    return ldp<T, V>(x + (f * F + (q & 1) * hf + eb + (q >> 1)));
  };
  const int J = rp.J, K = rp.K;
  bool actp[V];
  bool anyp = false;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    actp[i] = i < rp.n && g.p_active(rp.I0 + 2 * i, J, K);
    anyp = anyp || actp[i];
  }
  T pcv[V], dv[V];  // carried: centre pressure, divergence so far
#pragma unroll
  for (int i = 0; i < V; ++i) pcv[i] = dv[i] = T(0);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    bool act[V];
    bool any = false;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int I = rp.I0 + 2 * i;
      act[i] = f == 3 ? actp[i]
                      : i < rp.n && (f == 0 ? g.ux_active(I, J, K) : f == 1 ? g.uy_active(I, J, K) : g.uz_active(I, J, K));
      any = any || act[i];
    }
    T o[V];
    T own[V];
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = own[i] = T(0);
    if (MODE != AP_BNORM) {
      if (f == 0 && (any || anyp)) {
        const Pack<T, V> pc = L(3, 0);
#pragma unroll
        for (int i = 0; i < V; ++i) pcv[i] = pc.v[i];
      }
      if (f < 3) {
        const int ps = f == 0 ? 1 : f == 1 ? sy : sz;
        if (any || anyp) {
          const Pack<T, V> c0 = L(f, 0), up = L(f, ps);
#pragma unroll
          for (int i = 0; i < V; ++i) {
            dv[i] = f == 0 ? up.v[i] - c0.v[i] : dv[i] + (up.v[i] - c0.v[i]);
            own[i] = c0.v[i];
          }
          if (any) {
            // the minus and the two transverse pairs of neighbours; the plus neighbour is `up`
            const int oa = f == 0 ? sy : 1, ob = f == 2 ? sy : sz;
            const Pack<T, V> um = L(f, -ps), am = L(f, -oa), ap = L(f, oa), bm = L(f, -ob), bp = L(f, ob),
                             pm = L(3, -ps);
#pragma unroll
            for (int i = 0; i < V; ++i) {
              // row_u's order: n_f c - x- - x+ - y- - y+ - z- - z+
              T xm, xp, ym, yp, zm, zp;
              if (f == 0) {
                xm = um.v[i]; xp = up.v[i]; ym = am.v[i]; yp = ap.v[i]; zm = bm.v[i]; zp = bp.v[i];
              } else if (f == 1) {
                xm = am.v[i]; xp = ap.v[i]; ym = um.v[i]; yp = up.v[i]; zm = bm.v[i]; zp = bp.v[i];
              } else {
                xm = am.v[i]; xp = ap.v[i]; ym = bm.v[i]; yp = bp.v[i]; zm = um.v[i]; zp = up.v[i];
              }
              const T nd = g.flags ? T(g.nd(f, g.idx(rp.I0 + 2 * i, J, K))) : T(6);
              const T lap = nd * c0.v[i] - xm - xp - ym - yp - zm - zp;
              o[i] = (T)g.c * lap + (pcv[i] - pm.v[i]) * (T)g.inv_h;
            }
          }
        }
      } else if (any) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          o[i] = -dv[i] * (T)g.inv_h - (T)gamma * pcv[i];
          own[i] = pcv[i];
        }
      }
    }
    T v[V];
    if (MODE == AP_RESID || MODE == AP_RESNORM || MODE == AP_BNORM) {
      Pack<TB, V> bb;
#pragma unroll
      for (int i = 0; i < V; ++i) bb.v[i] = TB(0);
      if (any) bb = ldp<TB, V>(b + (f * F + (rp.par & 1) * hf + eb));
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = act[i] ? (T)bb.v[i] - o[i] : T(0);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = act[i] ? o[i] : T(0);
    }
    if (MODE == AP_APPLY || MODE == AP_RESID || MODE == AP_APPLY_DOT) sink(f, v);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (i >= rp.n) continue;
      if (MODE == AP_APPLY_DOT) acc += (double)own[i] * (double)v[i];
      if (MODE == AP_RESNORM || MODE == AP_BNORM) acc += (double)v[i] * (double)v[i];
    }
    stage(v);
  }
  return acc;
}

template <int MODE, typename T, typename TB, int V>
__device__ __forceinline__ double apply_pack(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                             T* __restrict__ y, double gamma, const RowPack<V>& rp) {
  const int F = g.field;
  return apply_pack_to<MODE, T, TB, V>(g, x, b, gamma, rp, [&](int f, const T* v) {
    T* yo = y + f * F + rp.el(0);
    if (rp.n == V) {
      Pack<T, V> w;
#pragma unroll
      for (int i = 0; i < V; ++i) w.v[i] = v[i];
      stp<T, V>(yo, w);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (i < rp.n) yo[i] = v[i];
    }
  });
}

template <int MODE, typename T, typename TB, int V>
__global__ __launch_bounds__(BS) void k_apply_v(Geom g, const T* __restrict__ x, const TB* __restrict__ b,
                                                T* __restrict__ y, double gamma, double* __restrict__ partial) {
  double acc = 0.0;
  RowPack<V> rp;
  if (slot_pack<V>(g, rp)) acc = apply_pack<MODE, T, TB, V>(g, x, b, y, gamma, rp);
  if (MODE == AP_APPLY_DOT || MODE == AP_RESNORM || MODE == AP_BNORM) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Residual and restriction without the fine residual in memory (Alg. 1:
// r = b - L~ x on level l, then the coarse right-hand side R r).  The
// restriction (the transposed prolongation over 8, Section 3.2) is a tensor
// product of 1D weights: (1/2, 1, 1/2) along a velocity component's own axis,
// (1/4, 3/4, 3/4, 1/4) along the other two, 1 over the 2x2 fine cells of a
// pressure in each direction.  Two passes:
//   k_resid_restrict_xy: a workgroup takes one fine plane under a tile of
//     RR_TX x RR_TY coarse columns; the residual over the tile's fine window
//     (its fine columns and one more on each side) goes to LDS, computed pack
//     by pack as the operator pass computes it, and each thread restricts its
//     coarse column in x and y: S[f][Kf][J][I], one value per component, fine
//     plane and coarse column (a quarter of a fine field per component);
//   k_restrict_z: the coarse unknown sums its fine planes' S with the z weights
//     (in increasing Kf) and the 1/8.
// Fine slots outside the lattice hold 0 in the window, which drops the terms
// the two-pass restriction drops at the last face planes.  The sums run in a
// different order from k_restrict, so the two differ by rounding.
// ---------------------------------------------------------------------------
constexpr int RR_TX = 16, RR_TY = 16;  // coarse columns of a workgroup: one per thread
constexpr int RR_WX = 2 * RR_TX + 2, RR_WY = 2 * RR_TY + 2;
static_assert(RR_TX * RR_TY == BS, "one coarse column per thread");

// Elements of S: 4 components x (fine planes) x (coarse rows) x (coarse row pitch).
__host__ __device__ inline long rr_plane(const Geom& f, const Geom& c) { return (long)(c.ny + 2) * c.sy; }
__host__ __device__ inline long rr_elems(const Geom& f, const Geom& c) { return 4L * (f.nz + 2) * rr_plane(f, c); }

// Tiles cover the coarse columns I = 1..nx+e, J = 1..ny+e, e = 1 on a
// labelled domain (whose faces with an exterior ghost cell, at I = nx+1 and so
// on, are unknowns) and 0 on a box (the other ghost columns have no unknown,
// and k_restrict_z writes 0 there without reading S), so a tile's fine window
// starts at the lattice's first slot: for box sides that are multiples of 32
// no window is clipped.
// Workgroups: XCD x (blockIdx % NXCD) takes a run of consecutive fine planes
// and goes through it strip by strip (a row of tiles), plane by plane, tile by
// tile, so that the lines two neighbouring tiles share and the planes below
// and above a stencil are read by the same XCD close in time (one L2).
__host__ __device__ inline int rr_ext(const Geom& c) { return c.flags ? 1 : 0; }
__host__ __device__ inline int rr_cols_x(const Geom& c) { return (c.nx + rr_ext(c) + RR_TX - 1) / RR_TX; }
__host__ __device__ inline int rr_cols_y(const Geom& c) { return (c.ny + rr_ext(c) + RR_TY - 1) / RR_TY; }
__host__ __device__ inline int rr_run(const Geom& f) { return (f.nz + 2 + NXCD - 1) / NXCD; }
__host__ __device__ inline long rr_blocks(const Geom& f, const Geom& c) {
  return (long)NXCD * rr_cols_x(c) * rr_cols_y(c) * rr_run(f);
}

template <typename T, int V>
__global__ __launch_bounds__(BS) void k_resid_restrict_xy(Geom f, Geom c, const T* __restrict__ x,
                                                          const T* __restrict__ b, T* __restrict__ S) {
  __shared__ T sr[4][RR_WY][RR_WX];
  const int cx = rr_cols_x(c), run = rr_run(f);
  const int l = blockIdx.x / NXCD;
  const int xt = l % cx, rest = l / cx;
  const int Kf = (blockIdx.x % NXCD) * run + rest % run, yt = rest / run;
  if (Kf > f.nz + 1 || yt >= rr_cols_y(c)) return;
  const int I0 = 1 + xt * RR_TX, J0 = 1 + yt * RR_TY;
  const int fi0 = 2 * I0 - 2, fj0 = 2 * J0 - 2;
  // the fine window clipped to the lattice; the rest of it holds 0
  const int ilo = max(fi0, 0), ihi = min(fi0 + RR_WX, f.nx + 2);
  const int jlo = max(fj0, 0), jhi = min(fj0 + RR_WY, f.ny + 2);
  if (ilo > fi0 || ihi < fi0 + RR_WX || jlo > fj0 || jhi < fj0 + RR_WY) {
    for (int t = threadIdx.x; t < 4 * RR_WY * RR_WX; t += BS) (&sr[0][0][0])[t] = T(0);
    __syncthreads();
  }
  constexpr int PPQ = (RR_TX + 1 + V - 1) / V;  // packs per parity of a window row
  const int npk = (jhi - jlo) * 2 * PPQ;
  for (int P = threadIdx.x; P < npk; P += BS) {
    const int row = P / (2 * PPQ), rem = P - row * (2 * PPQ);
    const int q = rem / PPQ, m = rem - q * PPQ;
    const int Jf = jlo + row;
    const int first = ilo + ((q - ilo) & 1) + 2 * V * m;  // slots of I-parity q from ilo
    if (first >= ihi) continue;
    RowPack<V> rp;
    rp.n = min(V, (ihi - first + 1) >> 1);
    rp.I0 = first;
    rp.J = Jf;
    rp.K = Kf;
    const int s0 = first + f.sy * Jf + f.sz * Kf;
    rp.e0 = s0 >> 1;
    rp.par = s0 & 1;
    rp.half = f.half;
    T* dst = &sr[0][Jf - fj0][first - fi0];
    apply_pack_to<AP_RESID, T, T, V, false>(f, x, b, f.gamma, rp, [&](int fld, const T* v) {
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (i < rp.n) dst[fld * (RR_WY * RR_WX) + 2 * i] = v[i];
    });
  }
  __syncthreads();
  const int tI = threadIdx.x % RR_TX, tJ = threadIdx.x / RR_TX;
  const int I = I0 + tI, J = J0 + tJ;
  if (I > c.nx + rr_ext(c) || J > c.ny + rr_ext(c)) return;
  const T wc[4] = {T(0.25), T(0.75), T(0.75), T(0.25)};
  const T wf[3] = {T(0.5), T(1), T(0.5)};
  const int li = 2 * tI, lj = 2 * tJ;  // window position of fine 2I-2, 2J-2
  T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const T* rx = &sr[0][lj + jj][li];
    const T* rz = &sr[2][lj + jj][li];
    s0 += wc[jj] * (wf[0] * rx[0] + wf[1] * rx[1] + wf[2] * rx[2]);
    s2 += wc[jj] * (wc[0] * rz[0] + wc[1] * rz[1] + wc[2] * rz[2] + wc[3] * rz[3]);
  }
#pragma unroll
  for (int jj = 0; jj < 3; ++jj) {
    const T* ry = &sr[1][lj + jj][li];
    s1 += wf[jj] * (wc[0] * ry[0] + wc[1] * ry[1] + wc[2] * ry[2] + wc[3] * ry[3]);
  }
  const T s3 = sr[3][lj + 1][li + 1] + sr[3][lj + 1][li + 2] + sr[3][lj + 2][li + 1] + sr[3][lj + 2][li + 2];
  const long pl = rr_plane(f, c), comp = (long)(f.nz + 2) * pl;
  const long o = Kf * pl + (long)J * c.sy + I;
  S[o] = s0;
  S[comp + o] = s1;
  S[2 * comp + o] = s2;
  S[3 * comp + o] = s3;
}

// One thread per coarse slot (slab mapping).  Coarse plane K takes fine planes
// 2K-2 .. 2K+1 (u_x, u_y: 1/4, 3/4, 3/4, 1/4), 2K-2 .. 2K (u_z: 1/2, 1, 1/2),
// 2K-1 .. 2K (p: 1, 1); planes outside the lattice add nothing.  Slots
// outside the columns and planes k_resid_restrict_xy covers (no unknown; S
// holds nothing for their columns) get 0.
template <typename T>
__global__ __launch_bounds__(BS) void k_restrict_z(Geom f, Geom c, const T* __restrict__ S, T* __restrict__ bc) {
  int I, J, K;
  if (!slab_item(c, c.sy, I, J, K)) return;
  const int s = c.at(c.idx(I, J, K)), Fc = c.field;
  const int e = rr_ext(c);
  if (I < 1 || I > c.nx + e || J < 1 || J > c.ny + e || K < 1 || K > c.nz + e) {
    bc[s] = bc[Fc + s] = bc[2 * Fc + s] = bc[3 * Fc + s] = T(0);
    return;
  }
  const T wc[4] = {T(0.25), T(0.75), T(0.75), T(0.25)};
  const T wf[3] = {T(0.5), T(1), T(0.5)};
  const long pl = rr_plane(f, c), comp = (long)(f.nz + 2) * pl;
  const long o = (long)J * c.sy + I;
  T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int Kf = 2 * K - 2 + kk;
    if (Kf < 0 || Kf > f.nz + 1) continue;
    const long e = Kf * pl + o;
    a0 += wc[kk] * S[e];
    a1 += wc[kk] * S[comp + e];
    if (kk < 3) a2 += wf[kk] * S[2 * comp + e];
    if (kk == 1 || kk == 2) a3 += S[3 * comp + e];
  }
  bc[s] = c.ux_active(I, J, K) ? a0 * T(0.125) : T(0);
  bc[Fc + s] = c.uy_active(I, J, K) ? a1 * T(0.125) : T(0);
  bc[2 * Fc + s] = c.uz_active(I, J, K) ? a2 * T(0.125) : T(0);
  bc[3 * Fc + s] = c.p_active(I, J, K) ? a3 * T(0.125) : T(0);
}

}  // namespace sg
