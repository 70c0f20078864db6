// gfx950 kernels of the MG-SQMR hot path.  Bandwidth- and latency-bound
// stencil work: no matrix cores, wave64 shuffles for reductions and the Vanka
// products, the padded red/black layout of geom.hpp, and block indices
// remapped so that each of the 8 XCDs walks a contiguous slab of the grid
// (its L2 then serves the y- and z-neighbour rows of its own rows).  The
// distributive Gauss-Seidel steps and the packed operator passes are in
// packed_kernels.hpp (V cells per thread).
#pragma once

#include <hip/hip_runtime.h>

#include "geom.hpp"

namespace sg {

constexpr int BS = 256;        // threads per block (4 waves)
constexpr int NXCD = 8;        // XCDs on MI355X; workgroups are dealt round-robin over them
constexpr int RED_BLOCKS = 2048;  // fixed grid of the BLAS-1 reductions (deterministic order)

// Logical block index: physical block b runs on XCD b % 8; give XCD x the
// contiguous range [x*per, (x+1)*per).  Grids are padded to a multiple of 8.
__device__ __forceinline__ int logical_block() {
  const int per = gridDim.x / NXCD;
  const int b = blockIdx.x;
  return (b % NXCD) * per + b / NXCD;
}

// Slab mapping of the slot kernels: XCD x (physical block b runs on XCD
// b % 8) owns the rows J in [x*R, (x+1)*R), R = ceil((ny+2)/8), for every
// plane, and walks them plane by plane.  The planes K-1, K, K+1 of a slab
// are a few hundred kB per field, so the z-neighbours a stencil reads are
// still in that XCD's L2 when it reaches them.
__device__ __forceinline__ int slab_rows(const Geom& g) { return (g.ny + 2 + NXCD - 1) / NXCD; }

// Blocks for `per_row` items per row (slots, or pairs of slots) in slab mapping.
__host__ __device__ inline int slab_blocks(const Geom& g, int per_row) {
  const int R = (g.ny + 2 + NXCD - 1) / NXCD;
  const long per_xcd = ((long)per_row * R * (g.nz + 2) + BS - 1) / BS;
  return (int)(per_xcd * NXCD);
}

// Item (column index X within the row, row J, plane K) of this thread; false
// when the thread is past the end of its slab.
__device__ __forceinline__ bool slab_item(const Geom& g, int per_row, int& X, int& J, int& K) {
  const int R = slab_rows(g);
  const int xcd = blockIdx.x % NXCD;
  const long l = (long)(blockIdx.x / NXCD) * BS + threadIdx.x;
  X = (int)(l % per_row);
  const long t = l / per_row;
  const int jl = (int)(t % R);
  K = (int)(t / R);
  J = xcd * R + jl;
  return K < g.nz + 2 && J < g.ny + 2;
}

__device__ __forceinline__ void slot_ijk(const Geom& g, int s, int& I, int& J, int& K) {
  K = s / g.sz;
  const int rem = s - K * g.sz;
  J = rem / g.sy;
  I = rem - J * g.sy;
}

// Sum over the block, result valid in thread 0.  Fixed order: deterministic.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sm[BS / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < BS / 64; ++i) t += sm[i];
  }
  return t;
}

// ---------------------------------------------------------------------------
// Rows of the operator (Eq. 2 / Section 4).  s = slot of the row; T is both
// the storage and the arithmetic type (FP64, or FP32 inside an FP32 V-cycle).
//   u_x row: (eta/h^2)(n_f u - 6 lattice neighbours) + (p(I,J,K) - p(I-1,J,K))/h
//            (n_f = 6 in a box; g.nd beside exterior cells)
//   p row  : -(1/h) sum_a (u_a(plus face) - u_a(minus face)) - gamma p
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T row_u(const Geom& g, const T* __restrict__ u, const T* __restrict__ p, int s,
                                        int pstride, int f) {
  const T lap = T(g.nd(f, s)) * u[g.at(s)] - u[g.at(s - 1)] - u[g.at(s + 1)] - u[g.at(s - g.sy)] - u[g.at(s + g.sy)] -
                u[g.at(s - g.sz)] - u[g.at(s + g.sz)];
  return (T)g.c * lap + (p[g.at(s)] - p[g.at(s - pstride)]) * (T)g.inv_h;
}

template <typename T>
__device__ __forceinline__ T row_p(const Geom& g, const T* __restrict__ ux, const T* __restrict__ uy,
                                        const T* __restrict__ uz, const T* __restrict__ p, int s, double gamma) {
  const T div = (ux[g.at(s + 1)] - ux[g.at(s)]) + (uy[g.at(s + g.sy)] - uy[g.at(s)]) +
                (uz[g.at(s + g.sz)] - uz[g.at(s)]);
  return -div * (T)g.inv_h - (T)gamma * p[g.at(s)];
}

enum ApplyMode { AP_APPLY = 0, AP_RESID = 1, AP_APPLY_DOT = 2, AP_RESNORM = 3, AP_BNORM = 4 };

// AP_APPLY:     y = L~ x                  (gamma = penalty, or 0 for L)
// AP_RESID:     y = b - L~ x
// AP_APPLY_DOT: y = L~ x, partial[blk] = sum x.y
// AP_RESNORM:   partial[blk] = sum (b - L~ x)^2 over unknowns (no y)
// AP_BNORM:     partial[blk] = sum b^2 over unknowns (x unused)
// Every slot of y is written; slots that are not unknowns get 0.
// One slot (I, J, K) of an apply pass; returns this slot's share of the reduction.
template <int MODE, typename T, typename TB>
__device__ __forceinline__ double apply_item(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                             T* __restrict__ y, double gamma, int I, int J, int K) {
  double acc = 0.0;
  {
    const int s = g.idx(I, J, K);
    const int F = g.field;
    const T* ux = x;
    const T* uy = x + F;
    const T* uz = x + 2 * F;
    const T* p = x + 3 * F;
    T o[4] = {T(0), T(0), T(0), T(0)};
    bool act[4];
    act[0] = g.ux_active(I, J, K);
    act[1] = g.uy_active(I, J, K);
    act[2] = g.uz_active(I, J, K);
    act[3] = g.p_active(I, J, K);
    if (MODE != AP_BNORM) {
      if (act[0]) o[0] = row_u(g, ux, p, s, 1, 0);
      if (act[1]) o[1] = row_u(g, uy, p, s, g.sy, 1);
      if (act[2]) o[2] = row_u(g, uz, p, s, g.sz, 2);
      if (act[3]) o[3] = row_p(g, ux, uy, uz, p, s, gamma);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      T v = o[f];
      const int e = f * F + g.at(s);
      if (MODE == AP_RESID || MODE == AP_RESNORM || MODE == AP_BNORM) v = act[f] ? (T)b[e] - v : T(0);
      if (MODE == AP_APPLY || MODE == AP_RESID || MODE == AP_APPLY_DOT) y[e] = v;
      if (MODE == AP_APPLY_DOT) acc += (double)x[e] * (double)v;
      if (MODE == AP_RESNORM || MODE == AP_BNORM) acc += v * v;
    }
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Multiplicative Vanka on V1 (Eq. mv), one colour class.  Each subdomain is
// one V1 cell with its pressure and active faces; the class takes all its
// local residuals from the state at the start of the class (part 1), then
// applies the corrections (part 2).  K^-1 of the local saddle problem comes
// from a per-level table indexed by the 6-bit face-activity type (a box), or
// by the type the flag word of a labelled domain holds.
// ---------------------------------------------------------------------------
// One thread per subdomain: thread c evaluates the cell's seven local
// residual rows (0: u_x minus face, 1: u_x plus face, 2/3: u_y, 4/5: u_z,
// 6: p) and forms delta_r = sum_j (K^-1)_rj r_j.  delta is stored by row:
// delta[r * ncells + c].  The class lists hold cells in slot order, and with
// the red/black split consecutive cells of a class along a row are adjacent
// elements of a half field, so neighbouring threads read neighbouring
// elements on the planes normal to y and z.
template <typename T, typename TB>
__device__ __forceinline__ void vanka_delta_vals(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                                 int s, const T* __restrict__ kinv, T* __restrict__ out) {
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  const int F = g.field;
  const T* ux = x;
  const T* uy = x + F;
  const T* uz = x + 2 * F;
  const T* p = x + 3 * F;
  const int fb = g.vface_bits(I, J, K);
  T res[7];
  res[0] = (fb & 1) ? (T)b[g.at(s)] - row_u(g, ux, p, s, 1, 0) : T(0);
  res[1] = (fb & 2) ? (T)b[g.at(s + 1)] - row_u(g, ux, p, s + 1, 1, 0) : T(0);
  res[2] = (fb & 4) ? (T)b[F + g.at(s)] - row_u(g, uy, p, s, g.sy, 1) : T(0);
  res[3] = (fb & 8) ? (T)b[F + g.at(s + g.sy)] - row_u(g, uy, p, s + g.sy, g.sy, 1) : T(0);
  res[4] = (fb & 16) ? (T)b[2 * F + g.at(s)] - row_u(g, uz, p, s, g.sz, 2) : T(0);
  res[5] = (fb & 32) ? (T)b[2 * F + g.at(s + g.sz)] - row_u(g, uz, p, s + g.sz, g.sz, 2) : T(0);
  res[6] = (T)b[3 * F + g.at(s)] - row_p(g, ux, uy, uz, p, s, g.gamma);
  const T* km = kinv + g.vtype(I, J, K, fb) * 64;
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < 7; ++j) acc += km[r * 8 + j] * res[j];
    out[r] = acc;
  }
}

template <typename T, typename TB>
__device__ __forceinline__ void vanka_delta_at(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                               int s, const T* __restrict__ kinv, T* __restrict__ delta, int c,
                                               int ncells) {
  T d[7];
  vanka_delta_vals<T, TB>(g, x, b, s, kinv, d);
#pragma unroll
  for (int r = 0; r < 7; ++r) delta[(long)r * ncells + c] = d[r];
}

// x[local DOF r of subdomain c] += delta_r, one thread per subdomain.
template <typename T>
__device__ __forceinline__ void vanka_apply_at(const Geom& g, T* __restrict__ x, int s, const T* __restrict__ delta,
                                               int c, int ncells) {
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  const int F = g.field;
  const T* d = delta + c;
  const long n = ncells;
  const int fb = g.vface_bits(I, J, K);
  if (fb & 1) x[g.at(s)] += d[0];
  if (fb & 2) x[g.at(s + 1)] += d[n];
  if (fb & 4) x[F + g.at(s)] += d[2 * n];
  if (fb & 8) x[F + g.at(s + g.sy)] += d[3 * n];
  if (fb & 16) x[2 * F + g.at(s)] += d[4 * n];
  if (fb & 32) x[2 * F + g.at(s + g.sz)] += d[5 * n];
  x[3 * F + g.at(s)] += d[6 * n];
}

template <typename T, typename TB>
__device__ __forceinline__ void vanka_delta_item(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                                 const int* __restrict__ cells, int ncells, const T* __restrict__ kinv,
                                                 T* __restrict__ delta, int c) {
  if (c < ncells) vanka_delta_at<T, TB>(g, x, b, cells[c], kinv, delta, c, ncells);
}

template <typename T>
__device__ __forceinline__ void vanka_apply_item(const Geom& g, T* __restrict__ x, const int* __restrict__ cells,
                                                 int ncells, const T* __restrict__ delta, int c) {
  if (c < ncells) vanka_apply_at<T>(g, x, cells[c], delta, c, ncells);
}

// The same residuals and products with eight lanes per subdomain: lane r < 7
// evaluates local residual row r and forms delta_r from the group's
// residuals, gathered by shuffles.  Each lane makes about 9 loads where the
// one-thread form makes about 60 in a row, so on levels where a pass is a
// latency chain this form finishes sooner.  Output as above.  Lane t of the
// class (t & 7 must equal threadIdx.x & 7, and the eight lanes of a subdomain
// share a wave); every lane of the wave must call it (shuffles).
// Element (in a state vector) of local unknown r of the subdomain of cell
// (I, J, K) at slot s, whether it is an unknown, and the cell across it.
struct VankaDof {
  int e;
  bool active;
  int nI, nJ, nK;
};

__device__ __forceinline__ VankaDof vanka_dof(const Geom& g, int s, int I, int J, int K, int r) {
  const int F = g.field;
  VankaDof d{0, false, I, J, K};
  const int fb = r < 6 ? g.vface_bits(I, J, K) : 0;
  switch (r) {
    case 0: d.e = g.at(s); d.active = fb & 1; d.nI = I - 1; break;
    case 1: d.e = g.at(s + 1); d.active = fb & 2; d.nI = I + 1; break;
    case 2: d.e = F + g.at(s); d.active = fb & 4; d.nJ = J - 1; break;
    case 3: d.e = F + g.at(s + g.sy); d.active = fb & 8; d.nJ = J + 1; break;
    case 4: d.e = 2 * F + g.at(s); d.active = fb & 16; d.nK = K - 1; break;
    case 5: d.e = 2 * F + g.at(s + g.sz); d.active = fb & 32; d.nK = K + 1; break;
    default: d.e = 3 * F + g.at(s); d.active = true; break;  // the cell's own pressure
  }
  return d;
}

// Local residual row r (0..6, as in vanka_delta_vals) of the subdomain of
// cell (I, J, K) at slot s; zero for an inactive row, r = 7 or !valid.  The
// six velocity rows run one code path (the lane's face and axis picked by r,
// then row_u's loads in row_u's order), so a wave issues the loads of two
// paths rather than seven.
template <typename T, typename TB>
__device__ __forceinline__ T vanka_row_residual(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b, int s,
                                                int I, int J, int K, int r, bool valid) {
  const int F = g.field;
  const int fb = g.vface_bits(I, J, K);
  if (!valid || r > 6 || (r < 6 && !((fb >> r) & 1))) return T(0);
  const T* p = x + 3 * F;
  if (r < 6) {
    const int f = r >> 1;
    const int ps = f == 0 ? 1 : f == 1 ? g.sy : g.sz;
    const int sf = s + (r & 1) * ps;  // the face: minus (own slot) or plus
    return (T)b[f * F + g.at(sf)] - row_u(g, x + f * F, p, sf, ps, f);
  }
  return (T)b[3 * F + g.at(s)] - row_p(g, x, x + F, x + 2 * F, p, s, g.gamma);
}

template <typename T, typename TB>
__device__ __forceinline__ T vanka_delta8_lane(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                               const int* __restrict__ cells, int ncells, const T* __restrict__ kinv,
                                               int t) {
  const int c = t >> 3;
  const int r = t & 7;
  const bool valid = c < ncells;
  const int s = valid ? cells[c] : 0;
  int I = 1, J = 1, K = 1;
  if (valid) slot_ijk(g, s, I, J, K);
  // this lane's row of the local inverse is loaded before the residual
  const T* km = kinv + g.vtype(I, J, K, g.vface_bits(I, J, K)) * 64 + r * 8;
  T kr[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) kr[j] = km[j];
  const T res = vanka_row_residual<T, TB>(g, x, b, s, I, J, K, r, valid);
  const int base = (int)(threadIdx.x & 63) & ~7;
  T acc = T(0);
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const T rj = __shfl(res, base + j, 64);
    acc += kr[j] * rj;
  }
  return acc;
}

template <typename T, typename TB>
__device__ __forceinline__ void vanka_delta8_item(const Geom& g, const T* __restrict__ x, const TB* __restrict__ b,
                                                  const int* __restrict__ cells, int ncells, const T* __restrict__ kinv,
                                                  T* __restrict__ delta, int t) {
  const T acc = vanka_delta8_lane<T, TB>(g, x, b, cells, ncells, kinv, t);
  const int c = t >> 3, r = t & 7;
  if (c < ncells && r < 7) delta[(long)r * ncells + c] = acc;
}

// Residual pass of one class: eight lanes per subdomain, or one thread per
// subdomain for classes of more than VANKA_LANES_MAX cells (there the pass is
// bound by bandwidth, not by its latency chain, and one thread per cell
// issues fewer instructions).
constexpr int VANKA_LANES_MAX = 16384;

template <typename T, typename TB>
__global__ __launch_bounds__(BS) void k_vanka_delta(Geom g, const T* __restrict__ x, const TB* __restrict__ b,
                                                    const int* __restrict__ cells, int ncells,
                                                    const T* __restrict__ kinv, T* __restrict__ delta) {
  vanka_delta8_item<T, TB>(g, x, b, cells, ncells, kinv, delta, blockIdx.x * BS + threadIdx.x);
}

template <typename T, typename TB>
__global__ __launch_bounds__(BS) void k_vanka_delta1(Geom g, const T* __restrict__ x, const TB* __restrict__ b,
                                                     const int* __restrict__ cells, int ncells,
                                                     const T* __restrict__ kinv, T* __restrict__ delta) {
  vanka_delta_item<T, TB>(g, x, b, cells, ncells, kinv, delta, blockIdx.x * BS + threadIdx.x);
}

// Eight lanes per subdomain: lane t = 8 c + r (r < 7) adds delta_r to local
// unknown r of cell c (each add goes to its own element; the values of
// vanka_apply_at).
template <typename T>
__device__ __forceinline__ void vanka_apply8_item(const Geom& g, T* __restrict__ x, const int* __restrict__ cells,
                                                  int ncells, const T* __restrict__ delta, int t) {
  const int c = t >> 3, r = t & 7;
  if (c >= ncells || r == 7) return;
  const int s = cells[c];
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  const VankaDof d = vanka_dof(g, s, I, J, K, r);
  if (d.active) x[d.e] += delta[(long)r * ncells + c];
}

template <typename T>
__global__ __launch_bounds__(BS) void k_vanka_apply(Geom g, T* __restrict__ x, const int* __restrict__ cells,
                                                    int ncells, const T* __restrict__ delta) {
  vanka_apply8_item<T>(g, x, cells, ncells, delta, blockIdx.x * BS + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Multiplicative Vanka on a large box level with the x-slabs set apart.  In
// the x-fastest layout a class of cells on an x = const wall has every cell in
// a row of its own, so each of its loads touches a cache line for one or two
// values.  For the length of a Vanka step the slots of the four padded planes
// at each x end (I <= 3, I >= nx-2: every slot an x-wall cell reads or writes)
// move to a slab with y fastest: element ((f (nz+2) + K) 8 + L) (ny+2) + J,
// layer L = I (low end) or I - nx + 6 (high end).  Every Vanka load and store
// goes to the slab or to the level's array by the slot's I, with the same
// arithmetic as vanka_delta_vals and vanka_apply_at: the results are those
// of the unslabbed passes bit for bit.  Needs nx >= 8 (the two ends apart
// from the cells between) and a box (n_f = 6).
// ---------------------------------------------------------------------------
__host__ __device__ inline long xslab_elems(const Geom& g) { return 4L * (g.nz + 2) * 8 * (g.ny + 2); }

template <typename T>
__device__ __forceinline__ T* xslab_ptr(const Geom& g, T* x, T* xs, int f, int I, int J, int K) {
  if (I <= 3 || I >= g.nx - 2) {
    const int L = I <= 3 ? I : I - g.nx + 6;
    return xs + ((long)(f * (g.nz + 2) + K) * 8 + L) * (g.ny + 2) + J;
  }
  return x + (long)f * g.field + g.at(g.idx(I, J, K));
}

// Slab transfers.  XS_IN: slab = x; XS_ZERO: slab = 0 (x is 0); XS_OUT: x =
// slab on the layers a Vanka step changes (I = 1..3, nx-2..nx; the ghost
// planes I = 0, nx+1 hold no unknown).  (A partial refresh would not pay: a
// row's end slots share their cache lines whatever layers are copied.)
enum XSlabCopy { XS_IN = 0, XS_ZERO = 2, XS_OUT = 3 };

template <typename T>
__global__ __launch_bounds__(BS) void k_xslab_copy(Geom g, T* __restrict__ x, T* __restrict__ xs, int mode) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= xslab_elems(g)) return;
  const int J = (int)(t % (g.ny + 2));
  long r = t / (g.ny + 2);
  const int L = (int)(r % 8);
  r /= 8;
  const int K = (int)(r % (g.nz + 2)), f = (int)(r / (g.nz + 2));
  const int I = L < 4 ? L : g.nx - 6 + L;
  T* m = x + (long)f * g.field + g.at(g.idx(I, J, K));
  if (mode == XS_IN)
    xs[t] = *m;
  else if (mode == XS_ZERO)
    xs[t] = T(0);
  else if (mode == XS_OUT && L >= 1 && L <= 6)
    *m = xs[t];
}

// A class's corrections with eight lanes per subdomain (as k_vanka_delta):
// lane r < 7 forms local residual row r from nine loads that every lane
// issues in the same order (a velocity row: its face, the six lattice
// neighbours, the two pressures across it; the pressure row: the six faces
// and the pressure), then delta_r from the group's residuals by shuffles.
// Same values as vanka_delta_vals on the unslabbed state.
template <typename T, typename TB>
__global__ __launch_bounds__(BS) void k_vanka_delta8_xs(Geom g, T* x, T* xs, const TB* __restrict__ b,
                                                        const int* __restrict__ cells, int ncells,
                                                        const T* __restrict__ kinv, T* __restrict__ delta) {
  const int t = blockIdx.x * BS + threadIdx.x;
  const int c = t >> 3, r = t & 7;
  const bool valid = c < ncells;
  const int s = valid ? cells[c] : 0;
  int I = 1, J = 1, K = 1;
  if (valid) slot_ijk(g, s, I, J, K);
  const int fb = g.vface_bits(I, J, K);
  const T* km = kinv + g.vtype(I, J, K, fb) * 64 + r * 8;
  T kr[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) kr[j] = km[j];
  const bool act = valid && r < 7 && (r == 6 || ((fb >> r) & 1));
  T res = T(0);
  if (act) {
    const int F = g.field;
    T v[9];
    T bv;
    if (r < 6) {
      const int f = r >> 1, o = r & 1;
      const int di = f == 0, dj = f == 1, dk = f == 2;
      const int i = I + o * di, j = J + o * dj, k = K + o * dk;
      v[0] = *xslab_ptr<T>(g, x, xs, f, i, j, k);
      v[1] = *xslab_ptr<T>(g, x, xs, f, i - 1, j, k);
      v[2] = *xslab_ptr<T>(g, x, xs, f, i + 1, j, k);
      v[3] = *xslab_ptr<T>(g, x, xs, f, i, j - 1, k);
      v[4] = *xslab_ptr<T>(g, x, xs, f, i, j + 1, k);
      v[5] = *xslab_ptr<T>(g, x, xs, f, i, j, k - 1);
      v[6] = *xslab_ptr<T>(g, x, xs, f, i, j, k + 1);
      v[7] = *xslab_ptr<T>(g, x, xs, 3, i, j, k);
      v[8] = *xslab_ptr<T>(g, x, xs, 3, i - di, j - dj, k - dk);
      bv = (T)b[(long)f * F + g.at(g.idx(i, j, k))];
      const T lap = T(6) * v[0] - v[1] - v[2] - v[3] - v[4] - v[5] - v[6];
      res = bv - ((T)g.c * lap + (v[7] - v[8]) * (T)g.inv_h);
    } else {
      v[0] = *xslab_ptr<T>(g, x, xs, 0, I + 1, J, K);
      v[1] = *xslab_ptr<T>(g, x, xs, 0, I, J, K);
      v[2] = *xslab_ptr<T>(g, x, xs, 1, I, J + 1, K);
      v[3] = *xslab_ptr<T>(g, x, xs, 1, I, J, K);
      v[4] = *xslab_ptr<T>(g, x, xs, 2, I, J, K + 1);
      v[5] = *xslab_ptr<T>(g, x, xs, 2, I, J, K);
      v[6] = *xslab_ptr<T>(g, x, xs, 3, I, J, K);
      bv = (T)b[3L * F + g.at(s)];
      const T div = (v[0] - v[1]) + (v[2] - v[3]) + (v[4] - v[5]);
      res = bv - (-div * (T)g.inv_h - (T)g.gamma * v[6]);
    }
  }
  const int base = (int)(threadIdx.x & 63) & ~7;
  T acc = T(0);
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const T rj = __shfl(res, base + j, 64);
    acc += kr[j] * rj;
  }
  if (valid && r < 7) delta[(long)r * ncells + c] = acc;
}

// vanka_apply_at with the slab, eight lanes per subdomain: lane r < 7 adds
// delta_r to local unknown r (the order of the seven adds does not matter:
// each goes to its own element).
template <typename T>
__global__ __launch_bounds__(BS) void k_vanka_apply_xs(Geom g, T* x, T* xs, const int* __restrict__ cells,
                                                       int ncells, const T* __restrict__ delta) {
  const int t = blockIdx.x * BS + threadIdx.x;
  const int c = t >> 3, r = t & 7;
  if (c >= ncells || r == 7) return;
  int I, J, K;
  slot_ijk(g, cells[c], I, J, K);
  const int fb = g.vface_bits(I, J, K);
  if (r < 6 && !((fb >> r) & 1)) return;
  const int f = r < 6 ? r >> 1 : 3, o = r < 6 ? r & 1 : 0;
  T* e = xslab_ptr<T>(g, x, xs, f, I + (f == 0) * o, J + (f == 1) * o, K + (f == 2) * o);
  *e += delta[(long)r * ncells + c];
}

// ---------------------------------------------------------------------------
// Multiplicative Vanka with two copies of the level's state (8 classes, levels
// whose passes run as eight-lane launches).  Pass p reads copy R and writes
// copy W: each active local unknown of a cell of the pass becomes R + delta
// in W, so a pass needs no separate correction launch.  W then lacks only the
// previous pass's corrections, which the same launch copies over from R,
// except where a cell of the pass rewrites the unknown itself (a face shared
// with a V1 cell of one of the pass's classes).  The subdomains of one pass
// share no unknown and W is never read, so every element of W has at most one
// writer and no launch reads what it writes.  The values are those of the
// delta/apply passes, bit for bit.  The first pass also brings W up to date
// on the boundary band (vanka_band_copy_item); after the 8 passes the state
// is back in the first copy.
// ---------------------------------------------------------------------------

// Symmetric order of the 8 classes, taken as complementary pairs {q, 7-q}:
// forward {0,7} {1,6} {2,5} {3,4}, then backward {3,4} {2,5} {1,6} {0,7}.
// Complementary classes differ in all three parity bits, so their cells meet
// only at edges and corners: a subdomain's local residuals read no unknown of
// a subdomain of the other class (a face row reaches the faces of face
// neighbours, a pressure row only its own cell's faces) and the two share
// none.  A pair therefore runs as one pass with the values of its two classes
// run one after the other, bit for bit: 8 passes for the 16 class steps.  The
// class lists of a pair are stored one after the other, so a pass reads one
// list.  vanka_pair8(p) is the pair (its lower class q) of pass p;
// vanka_pair8_prev(p) the pair whose corrections pass p copies in the
// two-copy passes: none for the first pass, nor for the second {3,4} pass,
// which rewrites all of the unknowns the first one changed.
constexpr int VANKA_PASSES8 = 8;
__host__ __device__ inline int vanka_pair8(int pass) { return pass < 4 ? pass : 7 - pass; }
__host__ __device__ inline int vanka_pair8_prev(int pass) {
  return pass == 0 || pass == 4 ? -1 : vanka_pair8(pass - 1);
}
// bit mask of the two classes of pair q
__host__ __device__ inline int vanka_pair8_mask(int q) { return (1 << q) | (1 << (7 - q)); }

// Whether unknown f of slot (I, J, K) is an active unknown of a V1 cell of a
// class in kmask: a pressure of its own cell, a face of either cell beside it
// (the minus face of (I, J, K) and the plus face of the cell before it).
__device__ __forceinline__ bool vanka_owned(const Geom& g, int f, int I, int J, int K, int kmask) {
  auto v1 = [&](int i, int j, int k) {
    return i >= 0 && j >= 0 && k >= 0 && g.p_active(i, j, k) && !g.p_v2(i, j, k) &&
           ((kmask >> Geom::vanka_colour(i, j, k)) & 1);
  };
  if (f == 3) return v1(I, J, K);
  const bool act = f == 0 ? g.ux_active(I, J, K) : f == 1 ? g.uy_active(I, J, K) : g.uz_active(I, J, K);
  return act && (v1(I, J, K) || v1(I - (f == 0), J - (f == 1), K - (f == 2)));
}

// W = R on every slot within four cells of the boundary (padded I <= 3 or
// I >= nx-2, and so on): every value a V1 cell's local residuals read, and
// every unknown a Vanka pass writes.  Needs nx, ny, nz >= 8 (else copy the
// whole state).  With kmask, the unknowns of the V1 cells of those classes
// are left out (the first pass of a step writes them in the same launch).  Threads: first the full rows (planes K <= 3 or K >= nz-2,
// then rows J <= 3 or J >= ny-2 of the other planes), nx+2 slots each; then
// the eight band slots of every remaining row.
__host__ __device__ inline long vanka_band_slots(const Geom& g) {
  const long full = 8L * (g.ny + 2) + 8L * (g.nz - 6);
  return full * (g.nx + 2) + 8L * (g.ny - 6) * (g.nz - 6);
}

template <typename T>
__device__ __forceinline__ void vanka_band_copy_item(const Geom& g, const T* __restrict__ R, T* __restrict__ W, long t,
                                                     int kmask = 0) {
  const long full = 8L * (g.ny + 2) + 8L * (g.nz - 6);
  const long nA = full * (g.nx + 2);
  int I, J, K;
  if (t < nA) {
    const int row = (int)(t / (g.nx + 2));
    I = (int)(t - (long)row * (g.nx + 2));
    if (row < 8 * (g.ny + 2)) {
      const int pk = row / (g.ny + 2);
      K = pk < 4 ? pk : g.nz - 6 + pk;
      J = row - pk * (g.ny + 2);
    } else {
      const int r2 = row - 8 * (g.ny + 2);
      K = 4 + r2 / 8;
      const int jj = r2 % 8;
      J = jj < 4 ? jj : g.ny - 6 + jj;
    }
  } else {
    const long u = t - nA;
    if (u >= 8L * (g.ny - 6) * (g.nz - 6)) return;
    const int row = (int)(u / 8), ii = (int)(u % 8);
    K = 4 + row / (g.ny - 6);
    J = 4 + row % (g.ny - 6);
    I = ii < 4 ? ii : g.nx - 6 + ii;
  }
  const int e = g.at(g.idx(I, J, K));
#pragma unroll
  for (int f = 0; f < 4; ++f)
    if (!kmask || !vanka_owned(g, f, I, J, K, kmask)) W[f * g.field + e] = R[f * g.field + e];
}


// Copy unknown r of previous-pass cell s from R to W unless a V1 cell of a
// class in the pass's mask kmask owns it too.
template <typename T>
__device__ __forceinline__ void vanka_copy_dof(const Geom& g, const T* __restrict__ R, T* __restrict__ W, int s,
                                               int r, int kmask) {
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  const VankaDof d = vanka_dof(g, s, I, J, K, r);
  if (!d.active) return;
  if (r < 6 && g.p_active(d.nI, d.nJ, d.nK) && !g.p_v2(d.nI, d.nJ, d.nK) &&
      ((kmask >> Geom::vanka_colour(d.nI, d.nJ, d.nK)) & 1))
    return;
  W[d.e] = R[d.e];
}

// Eight lanes per cell of the pass (lanes [0, copy0), copy0 = 8 ncells
// rounded up to whole waves), then eight lanes per previous-pass cell, then
// (the first pass of a step: nband > 0, no previous pass) one lane per slot
// of the boundary band, which brings W up to date there except on the
// unknowns this pass writes (vanka_band_copy_item in the same launch).
template <typename T, typename TB>
__global__ __launch_bounds__(BS) void k_vanka_pp8(Geom g, const T* __restrict__ R, T* __restrict__ W,
                                                  const TB* __restrict__ b, const int* __restrict__ cells, int ncells,
                                                  const T* __restrict__ kinv, const int* __restrict__ prev, int nprev,
                                                  int kmask, int copy0, int nband) {
  const int t = blockIdx.x * BS + threadIdx.x;
  if (t < copy0) {  // whole waves: the shuffles see only this part's lanes
    const int c = t >> 3, r = t & 7;
    const bool valid = c < ncells;
    const int s = valid ? cells[c] : 0;
    int I = 1, J = 1, K = 1;
    if (valid) slot_ijk(g, s, I, J, K);
    // loads that need only the cell go out before the residual and its shuffles:
    // this lane's row of the local inverse and the value it corrects
    const T* km = kinv + g.vtype(I, J, K, g.vface_bits(I, J, K)) * 64 + r * 8;
    T kr[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) kr[j] = km[j];
    const VankaDof dof = vanka_dof(g, s, I, J, K, r < 7 ? r : 6);
    const bool wr = valid && r < 7 && dof.active;
    const T old = wr ? R[dof.e] : T(0);
    const T res = vanka_row_residual<T, TB>(g, R, b, s, I, J, K, r, valid);
    const int base = (int)(threadIdx.x & 63) & ~7;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const T rj = __shfl(res, base + j, 64);
      acc += kr[j] * rj;
    }
    if (wr) W[dof.e] = old + acc;
  } else if (t < copy0 + 8 * nprev) {
    const int u = t - copy0, c = u >> 3, r = u & 7;
    if (r < 7) vanka_copy_dof<T>(g, R, W, prev[c], r, kmask);
  } else if (t < copy0 + 8 * nprev + nband) {
    vanka_band_copy_item<T>(g, R, W, t - copy0 - 8 * nprev, kmask);
  }
}

// A whole Vanka smoothing step on a small level in one workgroup: the class
// passes of vanka_symmetric (delta, then apply, class by class) with a
// workgroup barrier in place of each kernel boundary.  Within a pass the
// items are independent, so the result is that of the per-class launches,
// bit for bit.  On a level whose classes hold a few thousand cells, a pass
// costs the workgroup one or two memory round trips, where two graph-replayed
// launches cost several microseconds each.
constexpr int VSWEEP_BS = 512;  // 256 VGPRs a thread
constexpr int VSWEEP_MAX_CLASS = 512;  // largest class a level may have to use it (one CU streams it)

struct VSweep {
  Geom g;
  int nc;        // colour classes (8 or 27)
  int additive;  // Eq. av: every class from the same state, then the corrections class by class
  const int* vc[27];
  int nv[27];
  long doff[27];
  const void* kinv;
};

// Multiplicative class passes inside one workgroup, the class lists of an
// 8-class step in LDS for the whole step.  Each subdomain's new values are
// formed from the class-start state before a barrier and written after it
// (the values of the delta and apply passes, bit for bit).
constexpr int VSWEEP_LIST = 8 * VSWEEP_MAX_CLASS;

// The class lists of a step: lists.nc, lists.cells(k), lists.count(k).
struct VSweepLists {
  const VSweep& a;
  int nc;
  __device__ __forceinline__ const int* cells(int k) const { return a.vc[k]; }
  __device__ __forceinline__ int count(int k) const { return a.nv[k]; }
};

template <typename Lists>
__device__ __forceinline__ void vsweep_load_lists(const Lists& a, int* __restrict__ scell) {
  if (a.nc != 8) return;
  for (int k = 0; k < 8; ++k)
    for (int c = threadIdx.x; c < a.count(k); c += blockDim.x) scell[k * VSWEEP_MAX_CLASS + c] = a.cells(k)[c];
  __syncthreads();
}

template <typename Lists>
__device__ __forceinline__ int vsweep_cell(const Lists& a, const int* __restrict__ scell, int k, int c) {
  return a.nc == 8 ? scell[k * VSWEEP_MAX_CLASS + c] : a.cells(k)[c];
}

// One thread per subdomain (a class has at most VSWEEP_MAX_CLASS cells, the
// workgroup as many threads): the seven corrections and the values they add
// to stay in registers.  (Eight lanes per subdomain, with the new values
// waiting in LDS, measured slower here: 93 against 71 us per step at 16^3.)
static_assert(VSWEEP_MAX_CLASS <= VSWEEP_BS, "a thread per subdomain");

// One barrier-separated step of the one-workgroup passes: the subdomains of
// class ka (na cells) and of class kb (nb cells, none when nb = 0), a thread
// each, or two (thread t takes cells t and t + blockDim.x) when there are more
// cells than threads.  Every subdomain's new values are formed from the
// step-start state before the first barrier and written after it (the
// subdomains of a step share no unknown; the two classes of a pair read none
// of each other's, so the step has the values of the classes one after the
// other).
template <typename T, typename Lists>
__device__ __forceinline__ void vsweep_step(const Geom& g, const Lists& a, const int* __restrict__ scell,
                                            T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ sk,
                                            int ka, int na, int kb, int nb) {
  T d[2][7], old[2][7];
  int e[2][7];
  bool act[2][7], mine[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = threadIdx.x + h * blockDim.x;
    mine[h] = c < na + nb;
    if (mine[h]) {
      const int s = c < na ? vsweep_cell(a, scell, ka, c) : vsweep_cell(a, scell, kb, c - na);
      vanka_delta_vals<T, T>(g, x, b, s, sk, d[h]);
      int I, J, K;
      slot_ijk(g, s, I, J, K);
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        const VankaDof v = vanka_dof(g, s, I, J, K, r);
        e[h][r] = v.e;
        act[h][r] = v.active;
        old[h][r] = v.active ? x[v.e] : T(0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (mine[h]) {
#pragma unroll
      for (int r = 0; r < 7; ++r)
        if (act[h][r]) x[e[h][r]] = old[h][r] + d[h][r];
    }
  __syncthreads();
}

// 8 classes: the 8 pair passes (vanka_pair8), one step each (a pair holds at
// most 2 VSWEEP_MAX_CLASS cells: two a thread); 27 classes: 0..26 then 26..0.
template <typename T, typename Lists>
__device__ __forceinline__ void vanka_sweep_passes1(const Geom& g, const Lists& a, T* __restrict__ x,
                                                    const T* __restrict__ b, const T* __restrict__ sk,
                                                    int* __restrict__ scell) {
  vsweep_load_lists(a, scell);
  if (a.nc == 8) {
    for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
      const int q = vanka_pair8(pass);
      vsweep_step<T>(g, a, scell, x, b, sk, q, a.count(q), 7 - q, a.count(7 - q));
    }
    return;
  }
  for (int pass = 0; pass < 2 * a.nc; ++pass) {
    const int k = pass < a.nc ? pass : 2 * a.nc - 1 - pass;
    vsweep_step<T>(g, a, scell, x, b, sk, k, a.count(k), k, 0);
  }
}

template <typename T>
__global__ __launch_bounds__(VSWEEP_BS) void k_vanka_sweep(VSweep a, T* __restrict__ x, const T* __restrict__ b,
                                                          T* __restrict__ vd) {
  // the local inverses live in LDS for the whole step
  __shared__ T sk[64 * 64];
  __shared__ int scell[VSWEEP_LIST];
  const int t = threadIdx.x;
  for (int i = t; i < 64 * 64; i += VSWEEP_BS) sk[i] = ((const T*)a.kinv)[i];
  __syncthreads();
  if (a.additive) {
    for (int k = 0; k < a.nc; ++k)
      for (int c = t; c < a.nv[k]; c += VSWEEP_BS)
        vanka_delta_item<T, T>(a.g, x, b, a.vc[k], a.nv[k], sk, vd + a.doff[k], c);
    __syncthreads();
    for (int k = 0; k < a.nc; ++k) {
      for (int c = t; c < a.nv[k]; c += VSWEEP_BS) vanka_apply_item<T>(a.g, x, a.vc[k], a.nv[k], vd + a.doff[k], c);
      __syncthreads();
    }
    return;
  }
  vanka_sweep_passes1<T>(a.g, VSweepLists{a, a.nc}, x, b, sk, scell);
}

// The multiplicative step of k_vanka_sweep on a level whose whole state fits
// in LDS next to the inverses and the class lists (gfx950: 160 KB per
// workgroup): the state is loaded once, the class passes read and write
// it there, and it is written back at the end.  Same values.
template <typename T>
constexpr int vsweep_lds_elems() {
  return sizeof(T) == 8 ? 12288 : 24576;  // 96 KB of FP64 or of FP32
}

template <typename T>
__global__ __launch_bounds__(VSWEEP_BS) void k_vanka_sweep_lds(VSweep a, T* __restrict__ x,
                                                                  const T* __restrict__ b) {
  __shared__ T sk[64 * 64];
  __shared__ int scell[VSWEEP_LIST];
  __shared__ T sx[vsweep_lds_elems<T>()];
  const int t = threadIdx.x;
  const int n4 = 4 * a.g.field;
  for (int i = t; i < 64 * 64; i += VSWEEP_BS) sk[i] = ((const T*)a.kinv)[i];
  for (int i = t; i < n4; i += VSWEEP_BS) sx[i] = x[i];
  __syncthreads();
  vanka_sweep_passes1<T>(a.g, VSweepLists{a, a.nc}, sx, b, sk, scell);
  for (int i = t; i < n4; i += VSWEEP_BS) x[i] = sx[i];
}

// ---------------------------------------------------------------------------
// Grid transfer (Section 2): R = P^T / 8 with P bilinear per velocity lattice
// (weights 1, 1/2 along the face axis; 3/4, 1/4 across) and constant for p.
// ---------------------------------------------------------------------------
// Restriction: one thread per coarse slot; reads the fine residual r (zero at
// every fine slot that is not an unknown).  A coarse slot I reads the fine
// slots 2I-2 .. 2I+1 of each fine row it touches: 2I-2 and 2I are adjacent
// elements of one half field, 2I-1 and 2I+1 of the other, so a fine row is
// two 16-byte loads (the weighted sums keep their order term by term).
template <typename T>
struct FineRow {
  T r0, r1, r2, r3;  // fine slots 2I-2, 2I-1, 2I, 2I+1 of one row
};

template <typename T>
__device__ __forceinline__ FineRow<T> fine_row(const Geom& f, const T* __restrict__ r, int s) {
  FineRow<T> w;
  if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));
    const d2 a = *(const d2*)(r + f.at(s)), b = *(const d2*)(r + f.at(s + 1));
    w.r0 = a.x; w.r2 = a.y; w.r1 = b.x; w.r3 = b.y;
  } else {
    typedef float f2 __attribute__((ext_vector_type(2), aligned(4)));
    const f2 a = *(const f2*)(r + f.at(s)), b = *(const f2*)(r + f.at(s + 1));
    w.r0 = a.x; w.r2 = a.y; w.r1 = b.x; w.r3 = b.y;
  }
  return w;
}

template <typename T>
__device__ __forceinline__ void restrict_item(const Geom& f, const Geom& c, const T* __restrict__ r,
                                              T* __restrict__ bc, int I, int J, int K) {
  const int s = c.at(c.idx(I, J, K));
  const int Ff = f.field, Fc = c.field;
  const T wf[3] = {0.5, 1.0, 0.5};          // face axis: fine 2I-2, 2I-1, 2I
  const T wc[4] = {0.25, 0.75, 0.75, 0.25};  // cell axis: fine 2J-2 .. 2J+1
  // u_x.  A coarse face on the last face plane (I = nx+1: an unknown only
  // beside an exterior layer) has no fine face beyond the lattice: the third
  // fine face of its stencil is dropped, and so are the two more that the
  // paired loads read past the row.
  const bool xe = I == c.nx + 1, ye = J == c.ny + 1, ze = K == c.nz + 1;
  {
    T acc = T(0);
    if (c.ux_active(I, J, K)) {
      for (int kk = 0; kk < 4; ++kk)
        for (int jj = 0; jj < 4; ++jj) {
          const T w = wc[jj] * wc[kk];
          const FineRow<T> q = fine_row(f, r, f.idx(2 * I - 2, 2 * J - 2 + jj, 2 * K - 2 + kk));
          acc += w * (wf[0] * q.r0 + wf[1] * q.r1 + (xe ? T(0) : wf[2] * q.r2));
        }
    }
    bc[s] = (T)(acc * T(0.125));
  }
  // u_y
  {
    T acc = T(0);
    if (c.uy_active(I, J, K)) {
      for (int kk = 0; kk < 4; ++kk)
        for (int jj = 0; jj < (ye ? 2 : 3); ++jj) {
          const FineRow<T> q = fine_row(f, r + Ff, f.idx(2 * I - 2, 2 * J - 2 + jj, 2 * K - 2 + kk));
          const T rv[4] = {q.r0, q.r1, q.r2, q.r3};
          for (int ii = 0; ii < 4; ++ii) acc += wc[ii] * wf[jj] * wc[kk] * rv[ii];
        }
    }
    bc[Fc + s] = (T)(acc * T(0.125));
  }
  // u_z
  {
    T acc = T(0);
    if (c.uz_active(I, J, K)) {
      for (int kk = 0; kk < (ze ? 2 : 3); ++kk)
        for (int jj = 0; jj < 4; ++jj) {
          const FineRow<T> q = fine_row(f, r + 2 * Ff, f.idx(2 * I - 2, 2 * J - 2 + jj, 2 * K - 2 + kk));
          const T rv[4] = {q.r0, q.r1, q.r2, q.r3};
          for (int ii = 0; ii < 4; ++ii) acc += wc[ii] * wc[jj] * wf[kk] * rv[ii];
        }
    }
    bc[2 * Fc + s] = (T)(acc * T(0.125));
  }
  // p
  {
    T acc = T(0);
    if (c.p_active(I, J, K)) {
      for (int kk = 0; kk < 2; ++kk)
        for (int jj = 0; jj < 2; ++jj) {
          const FineRow<T> q = fine_row(f, r + 3 * Ff, f.idx(2 * I - 2, 2 * J - 1 + jj, 2 * K - 1 + kk));
          acc += q.r1;
          acc += q.r2;
        }
    }
    bc[3 * Fc + s] = (T)(acc * T(0.125));
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_restrict(Geom f, Geom c, const T* __restrict__ r, T* __restrict__ bc) {
  int I, J, K;
  if (!slab_item(c, c.sy, I, J, K)) return;  // consecutive coarse slots: dense fine reads
  restrict_item<T>(f, c, r, bc, I, J, K);
}

// 1D prolongation weights on the cell-centre lattice: fine padded index J
// (1-based cell) takes 3/4 from coarse (j>>1)+1 and 1/4 from the coarse row on
// its side (j = J-1).
__device__ __forceinline__ void cell_w(int J, int& n0, int& n1) {
  const int j = J - 1;
  n0 = (j >> 1) + 1;
  n1 = (j & 1) ? n0 + 1 : n0 - 1;
}
// ... and on the face lattice along the face axis: fine face i = I-1 takes 1
// from coarse face i/2 when even, 1/2 from (i-1)/2 and (i+1)/2 when odd.
__device__ __forceinline__ void face_w(int I, int& n0, int& n1, double& w0, double& w1) {
  const int i = I - 1;
  if ((i & 1) == 0) {
    n0 = i / 2 + 1;
    n1 = n0;
    w0 = 1.0;
    w1 = 0.0;
  } else {
    n0 = (i - 1) / 2 + 1;
    n1 = n0 + 1;
    w0 = 0.5;
    w1 = 0.5;
  }
}

// x_fine += P e_coarse at one fine slot (I, J, K).
template <typename T>
__device__ __forceinline__ void prolong_item(const Geom& f, const Geom& c, const T* __restrict__ e,
                                             T* __restrict__ x, int I, int J, int K) {
  const int s = f.at(f.idx(I, J, K));
  const int Ff = f.field, Fc = c.field;
  if (f.ux_active(I, J, K)) {
    int a0, a1, b0, b1, c0, c1;
    double w0, w1;
    face_w(I, a0, a1, w0, w1);
    cell_w(J, b0, b1);
    cell_w(K, c0, c1);
    auto ev = [&](int i, int j, int k) { return (T)e[c.at(c.idx(i, j, k))]; };
    const T v = (T)w0 * (T(0.75) * (T(0.75) * ev(a0, b0, c0) + T(0.25) * ev(a0, b1, c0)) +
                           T(0.25) * (T(0.75) * ev(a0, b0, c1) + T(0.25) * ev(a0, b1, c1))) +
                     (T)w1 * (T(0.75) * (T(0.75) * ev(a1, b0, c0) + T(0.25) * ev(a1, b1, c0)) +
                           T(0.25) * (T(0.75) * ev(a1, b0, c1) + T(0.25) * ev(a1, b1, c1)));
    x[s] = x[s] + v;
  }
  if (f.uy_active(I, J, K)) {
    int a0, a1, b0, b1, c0, c1;
    double w0, w1;
    face_w(J, b0, b1, w0, w1);
    cell_w(I, a0, a1);
    cell_w(K, c0, c1);
    auto ev = [&](int i, int j, int k) { return (T)e[Fc + c.at(c.idx(i, j, k))]; };
    const T v = (T)w0 * (T(0.75) * (T(0.75) * ev(a0, b0, c0) + T(0.25) * ev(a1, b0, c0)) +
                           T(0.25) * (T(0.75) * ev(a0, b0, c1) + T(0.25) * ev(a1, b0, c1))) +
                     (T)w1 * (T(0.75) * (T(0.75) * ev(a0, b1, c0) + T(0.25) * ev(a1, b1, c0)) +
                           T(0.25) * (T(0.75) * ev(a0, b1, c1) + T(0.25) * ev(a1, b1, c1)));
    x[Ff + s] = x[Ff + s] + v;
  }
  if (f.uz_active(I, J, K)) {
    int a0, a1, b0, b1, c0, c1;
    double w0, w1;
    face_w(K, c0, c1, w0, w1);
    cell_w(I, a0, a1);
    cell_w(J, b0, b1);
    auto ev = [&](int i, int j, int k) { return (T)e[2 * Fc + c.at(c.idx(i, j, k))]; };
    const T v = (T)w0 * (T(0.75) * (T(0.75) * ev(a0, b0, c0) + T(0.25) * ev(a1, b0, c0)) +
                           T(0.25) * (T(0.75) * ev(a0, b1, c0) + T(0.25) * ev(a1, b1, c0))) +
                     (T)w1 * (T(0.75) * (T(0.75) * ev(a0, b0, c1) + T(0.25) * ev(a1, b0, c1)) +
                           T(0.25) * (T(0.75) * ev(a0, b1, c1) + T(0.25) * ev(a1, b1, c1)));
    x[2 * Ff + s] = x[2 * Ff + s] + v;
  }
  if (f.p_active(I, J, K)) {
    const int ci = ((I - 1) >> 1) + 1, cj = ((J - 1) >> 1) + 1, ck = ((K - 1) >> 1) + 1;
    x[3 * Ff + s] = x[3 * Ff + s] + e[3 * Fc + c.at(c.idx(ci, cj, ck))];
  }
}

// The same update, one thread per pair of coarse cells Ic, Ic+1 (Ic odd; the
// second exists when Ic < nx) for their sixteen fine children (padded fine
// I = 2Ic-1 .. 2Ic+2, J = 2Jc-1+dj, K = 2Kc-1+dk, dj, dk in {0, 1}), one field
// at a time.  The children's interpolation stencils overlap, so the coarse
// values are loaded once per pair; and slots Ic-1 and Ic+1 of a coarse row are
// adjacent elements of one half field and Ic, Ic+2 of the other, so a coarse
// row is two 16-byte loads (44 loads for two cells, where one-child threads
// issue about 400).  The four fine children along x are likewise two loads and
// two stores per fine row and field.  Each value is prolong_item's expression
// with its face_w / cell_w indices fixed for the child (same operands, same
// order).  Every fine unknown lies in a child of an interior coarse cell, and
// each child belongs to one thread.  Each field's stage passes its base index
// through an empty asm statement, so its coarse values are the only ones held
// in registers.
template <typename T>
struct Quad {
  T v[4];  // slots i0, i0+1, i0+2, i0+3 of one row
};

template <typename T>
__device__ __forceinline__ Quad<T> load_quad(const Geom& g, const T* __restrict__ a, int s) {
  typedef T t2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  const t2 p = *(const t2*)(a + g.at(s)), q = *(const t2*)(a + g.at(s + 1));
  Quad<T> r;
  r.v[0] = p.x; r.v[2] = p.y; r.v[1] = q.x; r.v[3] = q.y;
  return r;
}

// fine row (J, K) of field `a`, slots 2Ic-1 .. 2Ic+2: add add[k] where act[k]
template <typename T>
__device__ __forceinline__ void add_quad(const Geom& f, T* __restrict__ a, int s, const T* add, const bool* act) {
  typedef T t2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  t2* pa = (t2*)(a + f.at(s));
  t2* pb = (t2*)(a + f.at(s + 1));
  t2 A = *pa, B = *pb;
  if (act[0]) A.x = A.x + add[0];
  if (act[2]) A.y = A.y + add[2];
  if (act[1]) B.x = B.x + add[1];
  if (act[3]) B.y = B.y + add[3];
  if (act[0] && act[2]) {
    *pa = A;
  } else {
    if (act[0]) a[f.at(s)] = A.x;
    if (act[2]) a[f.at(s) + 1] = A.y;
  }
  if (act[1] && act[3]) {
    *pb = B;
  } else {
    if (act[1]) a[f.at(s + 1)] = B.x;
    if (act[3]) a[f.at(s + 1) + 1] = B.y;
  }
}

template <typename T>
__device__ __forceinline__ void prolong_pair_item(const Geom& f, const Geom& c, const T* __restrict__ e,
                                                  T* __restrict__ x, int Ic, int Jc, int Kc) {
  int Fc = c.field, Ff = f.field;
  int base = 0;  // laundered between the field stages
  const int nt = Ic + 1 <= c.nx ? 2 : 1;
  auto stage = [&]() { asm volatile("" : "+v"(base), "+s"(Fc), "+s"(Ff)); };
  // u_x: coarse faces Ic .. Ic+2 (U[a], a = face - Ic), rows Jc-1..Jc+1, planes Kc-1..Kc+1
  {
    T U[3][3][3];
#pragma unroll
    for (int bj = 0; bj < 3; ++bj)
#pragma unroll
      for (int ck = 0; ck < 3; ++ck) {
        const Quad<T> q = load_quad(c, e + base, c.idx(Ic - 1, Jc - 1 + bj, Kc - 1 + ck));
#pragma unroll
        for (int a = 0; a < 3; ++a) U[a][bj][ck] = q.v[a + 1];
      }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int dj = d & 1, dk = d >> 1;
      const int J = 2 * Jc - 1 + dj, K = 2 * Kc - 1 + dk;
      const int n1 = dj ? 2 : 0, m1 = dk ? 2 : 0;
      T add[4];
      bool act[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t = k >> 1, di = k & 1;
        act[k] = t < nt && f.ux_active(2 * Ic - 1 + k, J, K);
        const T w0 = di ? T(0.5) : T(1), w1 = di ? T(0.5) : T(0);
        const int a1 = t + di;
        add[k] = w0 * (T(0.75) * (T(0.75) * U[t][1][1] + T(0.25) * U[t][n1][1]) +
                       T(0.25) * (T(0.75) * U[t][1][m1] + T(0.25) * U[t][n1][m1])) +
                 w1 * (T(0.75) * (T(0.75) * U[a1][1][1] + T(0.25) * U[a1][n1][1]) +
                       T(0.25) * (T(0.75) * U[a1][1][m1] + T(0.25) * U[a1][n1][m1]));
      }
      if (act[0] || act[1] || act[2] || act[3]) add_quad(f, x + base, f.idx(2 * Ic - 1, J, K), add, act);
    }
  }
  stage();
  // u_y: coarse cells Ic-1 .. Ic+2 (Vy[a], a = cell - Ic + 1), faces Jc, Jc+1, planes Kc-1..Kc+1
  {
    T Vy[4][2][3];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int ck = 0; ck < 3; ++ck) {
        const Quad<T> q = load_quad(c, e + Fc + base, c.idx(Ic - 1, Jc + bj, Kc - 1 + ck));
#pragma unroll
        for (int a = 0; a < 4; ++a) Vy[a][bj][ck] = q.v[a];
      }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int dj = d & 1, dk = d >> 1;
      const int J = 2 * Jc - 1 + dj, K = 2 * Kc - 1 + dk;
      const int m1 = dk ? 2 : 0, b1 = dj;
      const T v0 = dj ? T(0.5) : T(1), v1 = dj ? T(0.5) : T(0);
      T add[4];
      bool act[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t = k >> 1, di = k & 1;
        act[k] = t < nt && f.uy_active(2 * Ic - 1 + k, J, K);
        const int l1 = t + (di ? 2 : 0), c1 = t + 1;
        add[k] = v0 * (T(0.75) * (T(0.75) * Vy[c1][0][1] + T(0.25) * Vy[l1][0][1]) +
                       T(0.25) * (T(0.75) * Vy[c1][0][m1] + T(0.25) * Vy[l1][0][m1])) +
                 v1 * (T(0.75) * (T(0.75) * Vy[c1][b1][1] + T(0.25) * Vy[l1][b1][1]) +
                       T(0.25) * (T(0.75) * Vy[c1][b1][m1] + T(0.25) * Vy[l1][b1][m1]));
      }
      if (act[0] || act[1] || act[2] || act[3]) add_quad(f, x + Ff + base, f.idx(2 * Ic - 1, J, K), add, act);
    }
  }
  stage();
  // u_z: coarse cells Ic-1 .. Ic+2, rows Jc-1..Jc+1, faces Kc, Kc+1
  {
    T W[4][3][2];
#pragma unroll
    for (int bj = 0; bj < 3; ++bj)
#pragma unroll
      for (int ck = 0; ck < 2; ++ck) {
        const Quad<T> q = load_quad(c, e + 2 * Fc + base, c.idx(Ic - 1, Jc - 1 + bj, Kc + ck));
#pragma unroll
        for (int a = 0; a < 4; ++a) W[a][bj][ck] = q.v[a];
      }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int dj = d & 1, dk = d >> 1;
      const int J = 2 * Jc - 1 + dj, K = 2 * Kc - 1 + dk;
      const int n1 = dj ? 2 : 0, cz = dk;
      const T z0 = dk ? T(0.5) : T(1), z1 = dk ? T(0.5) : T(0);
      T add[4];
      bool act[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t = k >> 1, di = k & 1;
        act[k] = t < nt && f.uz_active(2 * Ic - 1 + k, J, K);
        const int l1 = t + (di ? 2 : 0), c1 = t + 1;
        add[k] = z0 * (T(0.75) * (T(0.75) * W[c1][1][0] + T(0.25) * W[l1][1][0]) +
                       T(0.25) * (T(0.75) * W[c1][n1][0] + T(0.25) * W[l1][n1][0])) +
                 z1 * (T(0.75) * (T(0.75) * W[c1][1][cz] + T(0.25) * W[l1][1][cz]) +
                       T(0.25) * (T(0.75) * W[c1][n1][cz] + T(0.25) * W[l1][n1][cz]));
      }
      if (act[0] || act[1] || act[2] || act[3]) add_quad(f, x + 2 * Ff + base, f.idx(2 * Ic - 1, J, K), add, act);
    }
  }
  stage();
  // p: constant over the eight children of each coarse cell
  {
    const Quad<T> q = load_quad(c, e + 3 * Fc + base, c.idx(Ic - 1, Jc, Kc));
    const T pc[2] = {q.v[1], q.v[2]};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int J = 2 * Jc - 1 + (d & 1), K = 2 * Kc - 1 + (d >> 1);
      T add[4];
      bool act[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        act[k] = (k >> 1) < nt && f.p_active(2 * Ic - 1 + k, J, K);
        add[k] = pc[k >> 1];
      }
      if (act[0] || act[1] || act[2] || act[3]) add_quad(f, x + 3 * Ff + base, f.idx(2 * Ic - 1, J, K), add, act);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_prolong_pairs(Geom f, Geom c, const T* __restrict__ e, T* __restrict__ x) {
  int X, Jc, Kc;
  if (!slab_item(c, (c.nx + 1) >> 1, X, Jc, Kc)) return;
  if (Jc < 1 || Jc > c.ny || Kc < 1 || Kc > c.nz) return;
  prolong_pair_item<T>(f, c, e, x, 2 * X + 1, Jc, Kc);
}

// The fine faces on the last face plane of each velocity lattice (u_x at
// I = nx+1, u_y at J = ny+1, u_z at K = nz+1), unknowns only beside an
// exterior layer (labelled domains), which the paired items above do not
// reach.  Such a fine face coincides with the coarse face on the coarse last
// plane (weight 1 along its axis) and takes 3/4, 1/4 along the other two.
// One thread per face of the three planes: t < ny nz for u_x, then nx nz for
// u_y, then nx ny for u_z.
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong_edge(Geom f, Geom c, const T* __restrict__ e, T* __restrict__ x) {
  long t = (long)blockIdx.x * BS + threadIdx.x;
  const long nyz = (long)f.ny * f.nz, nxz = (long)f.nx * f.nz, nxy = (long)f.nx * f.ny;
  int a, I, J, K;
  if (t < nyz) {
    a = 0; I = f.nx + 1; J = 1 + (int)(t % f.ny); K = 1 + (int)(t / f.ny);
  } else if ((t -= nyz) < nxz) {
    a = 1; J = f.ny + 1; I = 1 + (int)(t % f.nx); K = 1 + (int)(t / f.nx);
  } else if ((t -= nxz) < nxy) {
    a = 2; K = f.nz + 1; I = 1 + (int)(t % f.nx); J = 1 + (int)(t / f.nx);
  } else {
    return;
  }
  if (!(a == 0 ? f.ux_active(I, J, K) : a == 1 ? f.uy_active(I, J, K) : f.uz_active(I, J, K))) return;
  // coarse index along each axis: the last face plane on axis a, near/far cells (3/4, 1/4) on the others
  int n0[3], n1[3];
  const int fi[3] = {I, J, K};
  const int cl[3] = {c.nx + 1, c.ny + 1, c.nz + 1};
  for (int b = 0; b < 3; ++b) {
    if (b == a) {
      n0[b] = n1[b] = cl[b];
    } else {
      cell_w(fi[b], n0[b], n1[b]);
    }
  }
  const T* ea = e + (long)a * c.field;
  T acc = T(0);
  for (int q = 0; q < 8; ++q) {
    const int ib = q & 1, jb = (q >> 1) & 1, kb = q >> 2;
    if ((a == 0 && ib) || (a == 1 && jb) || (a == 2 && kb)) continue;
    const T w = (a == 0 ? T(1) : (ib ? T(0.25) : T(0.75))) * (a == 1 ? T(1) : (jb ? T(0.25) : T(0.75))) *
                (a == 2 ? T(1) : (kb ? T(0.25) : T(0.75)));
    const int Ic = ib ? n1[0] : n0[0], Jc = jb ? n1[1] : n0[1], Kc = kb ? n1[2] : n0[2];
    acc += w * ea[c.at(c.idx(Ic, Jc, Kc))];
  }
  T* xa = x + (long)a * f.field;
  xa[f.at(f.idx(I, J, K))] += acc;
}

// ---------------------------------------------------------------------------
// Coarsest level: x = L~c^{-1} b with the dense inverse; one wave per row.
// x must be zero beforehand (its ghost slots stay zero).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void coarse_row(const double* __restrict__ kinv, const int* __restrict__ dof, int n,
                                           const T* __restrict__ b, T* __restrict__ x, int row, int lane) {
  double acc = 0.0;
  const double* kr = kinv + (size_t)row * n;
  for (int j = lane; j < n; j += 64) acc += kr[j] * (double)b[dof[j]];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) x[dof[row]] = (T)acc;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_coarse_solve(const double* __restrict__ kinv, const int* __restrict__ dof,
                                                     int n, const T* __restrict__ b, T* __restrict__ x) {
  const int row = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  coarse_row<T>(kinv, dof, n, b, x, row, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// BLAS-1 pieces of SQMR (Alg. 4) on whole state vectors (ghost slots are zero).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BS) void k_fill(T* __restrict__ x, long n, T v) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) x[i] = v;
}

// out = (To) in, elementwise (FP64 <-> FP32 at the V-cycle's entry and exit)
template <typename Ti, typename To>
__global__ __launch_bounds__(BS) void k_convert(const Ti* __restrict__ in, To* __restrict__ out, long n) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) out[i] = (To)in[i];
}

// Pairs of elements (n is even: whole fields of a multiple of 8 elements),
// as doubles: 16-byte accesses of doubles, 8-byte ones of floats (the FP32
// V-cycle's output read where it lies; float -> double is exact).
typedef double pair_d2 __attribute__((ext_vector_type(2), aligned(8)));

template <typename TT>
__device__ __forceinline__ pair_d2 pair_load(const TT* __restrict__ p, long i) {
  if constexpr (sizeof(TT) == 8) {
    return ((const pair_d2*)p)[i];
  } else {
    typedef float f2 __attribute__((ext_vector_type(2), aligned(4)));
    const f2 v = ((const f2*)p)[i];
    pair_d2 r;
    r.x = (double)v.x;
    r.y = (double)v.y;
    return r;
  }
}

// partial[2*blk] = sum a.a, partial[2*blk+1] = sum a.c
template <typename TT>
__global__ __launch_bounds__(BS) void k_dot_aa_ac(const TT* __restrict__ a, const double* __restrict__ c, long n,
                                                  double* __restrict__ partial) {
  const pair_d2* c2 = (const pair_d2*)c;
  double s0 = 0.0, s1 = 0.0;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n / 2; i += (long)gridDim.x * BS) {
    const pair_d2 av = pair_load<TT>(a, i), cv = c2[i];
    s0 += av.x * av.x;
    s0 += av.y * av.y;
    s1 += av.x * cv.x;
    s1 += av.y * cv.y;
  }
  const double t0 = block_sum(s0);
  const double t1 = block_sum(s1);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = t0;
    partial[2 * blockIdx.x + 1] = t1;
  }
}

// sum of p over the cells (for the mean-pressure removal)
static __global__ __launch_bounds__(BS) void k_sum_p(Geom g, const double* __restrict__ x, double* __restrict__ partial) {
  const int s = logical_block() * BS + threadIdx.x;
  double v = 0.0;
  if (s < g.field) {
    int I, J, K;
    slot_ijk(g, s, I, J, K);
    if (g.p_active(I, J, K)) v = x[3 * g.field + g.at(s)];
  }
  const double t = block_sum(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

static __global__ __launch_bounds__(BS) void k_shift_p(Geom g, double* __restrict__ x, double amount) {
  const int s = logical_block() * BS + threadIdx.x;
  if (s >= g.field) return;
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  if (g.p_active(I, J, K)) x[3 * g.field + g.at(s)] -= amount;
}

// Zero the ghost slots of a state vector (the caller's initial guess).
static __global__ __launch_bounds__(BS) void k_clear_ghosts(Geom g, double* __restrict__ x) {
  const int s = logical_block() * BS + threadIdx.x;
  if (s >= g.field) return;
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  const int F = g.field;
  const int e = g.at(s);
  if (!g.ux_active(I, J, K)) x[e] = 0.0;
  if (!g.uy_active(I, J, K)) x[F + e] = 0.0;
  if (!g.uz_active(I, J, K)) x[2 * F + e] = 0.0;
  if (!g.p_active(I, J, K)) x[3 * F + e] = 0.0;
}

// s -= a t; with bf != nullptr also bf = (float) s, the right-hand side of
// the FP32 V-cycle that follows (what k_convert would write)
static __global__ __launch_bounds__(BS) void k_axpy_neg(double* __restrict__ s, const double* __restrict__ t, long n,
                                                 double a, float* __restrict__ bf) {
  typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));  // n even: 16-byte accesses
  typedef float f2 __attribute__((ext_vector_type(2), aligned(4)));
  d2* s2 = (d2*)s;
  const d2* t2 = (const d2*)t;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n / 2; i += (long)gridDim.x * BS) {
    d2 sv = s2[i];
    const d2 tv = t2[i];
    sv.x -= a * tv.x;
    sv.y -= a * tv.y;
    s2[i] = sv;
    if (bf) {
      f2 fv;
      fv.x = (float)sv.x;
      fv.y = (float)sv.y;
      ((f2*)bf)[i] = fv;
    }
  }
}

// d = cd * d + cq * q;  x += d;  q = t + beta * q (the next direction, from the
// same q): the iterate update and the direction update in one pass over q
template <typename TT>
__global__ __launch_bounds__(BS) void k_update_dxq(double* __restrict__ d, double* __restrict__ q,
                                                   double* __restrict__ x, const TT* __restrict__ t, long n,
                                                   double cd, double cq, double bt) {
  typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));  // n even: 16-byte accesses
  d2* d_ = (d2*)d;
  d2* q_ = (d2*)q;
  d2* x_ = (d2*)x;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n / 2; i += (long)gridDim.x * BS) {
    const d2 qv = q_[i], dold = d_[i], tv = pair_load<TT>(t, i);
    d2 xv = x_[i];
    d2 dv;
    dv.x = cd * dold.x + cq * qv.x;
    dv.y = cd * dold.y + cq * qv.y;
    d_[i] = dv;
    xv.x += dv.x;
    xv.y += dv.y;
    x_[i] = xv;
    d2 qn;
    qn.x = tv.x + bt * qv.x;
    qn.y = tv.y + bt * qv.y;
    q_[i] = qn;
  }
}

// out[k] = sum_b partial[b*stride + k], fixed order, single block.
static __global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ partial, int nblk, int stride,
                                                 double* __restrict__ out) {
  __shared__ double sm[16];
  for (int k = 0; k < stride; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 1024) v += partial[(long)b * stride + k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < 16; ++i) t += sm[i];
      out[k] = t;
    }
  }
}

}  // namespace sg
