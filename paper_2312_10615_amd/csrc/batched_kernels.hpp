// Batched launches: one kernel launch covers the work of many independent
// box domains at the same multigrid level.  Each launch reads a table of
// entries (domain, first block), sorted by first block; a block finds its
// entry by binary search, skips the domain when that domain's solve has
// finished, and maps its local block index onto a 2-D tile of the domain's
// (row, x) items.  The per-item arithmetic is the single-domain kernels'.
#pragma once

#include "kernels.hpp"
#include "packed_kernels.hpp"

namespace sg {

struct BEnt {
  int dom;
  int bstart;
};

// Per (domain, level) data read by the batched kernels.
struct BLev {
  Geom g, gc;              // this level and (when the domain has it) the next coarser one
  void* x;                 // level vectors, in the V-cycle's precision
  void* b;
  void* r;
  void* dscr;
  void* xc;                // next level's x and b
  void* bc;
  const void* kinv;        // Vanka inverses of this level
  void* alt;               // second copy of x for the two-copy Vanka passes (boxes not run in one workgroup)
  const int* vc[8];        // V1 cells per colour (classes q and 7-q back to back)
  int nv[8];
  long voff[4];            // this domain's slice of the shared Vanka delta buffer, per class pair
  const double* cinv;      // coarsest level: dense inverse and its DOF slots
  const int* cdof;
  int nc;
};

// Per-domain scalars of the batched SQMR (Alg. 4), device resident.
struct BScal {
  double rho, tau, nu_prev, alpha, beta, cd, cq, bnorm, relres, rtol;
  double red[4];   // reduction results of the current step
  int iters, status, maxit, zero_x;
};
enum { RED0 = 0, RED1 = 1 };

__device__ __forceinline__ int bent_find(const BEnt* __restrict__ t, int n) {
  int lo = 0, hi = n - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].bstart <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// 2-D tiles of BX items along a row times BS/BX rows; planes one after another.
template <int BX>
__host__ __device__ inline int tile_blocks(const Geom& g, int per_row) {
  constexpr int BY = BS / BX;
  return ((per_row + BX - 1) / BX) * ((g.ny + 2 + BY - 1) / BY) * (g.nz + 2);
}

template <int BX>
__device__ __forceinline__ bool tile_item(const Geom& g, int per_row, int lb, int& X, int& J, int& K) {
  constexpr int BY = BS / BX;
  const int tx = (per_row + BX - 1) / BX, ty = (g.ny + 2 + BY - 1) / BY;
  const int bx = lb % tx;
  const int r = lb / tx;
  const int by = r % ty;
  K = r / ty;
  X = bx * BX + (int)(threadIdx.x % BX);
  J = by * BY + (int)(threadIdx.x / BX);
  return X < per_row && J < g.ny + 2 && K < g.nz + 2;
}

// Items laid out flat: item l = (row-major row, x) with per_row items a row.
__host__ __device__ inline int flat_blocks(const Geom& g, int per_row) {
  return (int)(((long)per_row * (g.ny + 2) * (g.nz + 2) + BS - 1) / BS);
}

__device__ __forceinline__ bool flat_item(const Geom& g, int per_row, int lb, int& X, int& J, int& K) {
  const long l = (long)lb * BS + threadIdx.x;
  X = (int)(l % per_row);
  const long r = l / per_row;
  J = (int)(r % (g.ny + 2));
  K = (int)(r / (g.ny + 2));
  return K < g.nz + 2;
}

#define SG_BATCH_ENTRY()                   \
  const int e_ = bent_find(tab, nent);     \
  const int d = tab[e_].dom;               \
  if (done[d]) return;                     \
  const int lb = (int)blockIdx.x - tab[e_].bstart;

// --------------------------------------------------------- V-cycle stencils

template <typename T, int BX>
__global__ __launch_bounds__(BS) void kb_resid(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                               const int* __restrict__ done) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  constexpr int V = 16 / (int)sizeof(T);
  int X, J, K;
  if (!flat_item(g, slot_packs_per_row<V>(g), lb, X, J, K)) return;
  RowPack<V> rp;
  if (slot_pack_at<V>(g, X, J, K, rp))
    apply_pack<AP_RESID, T, T, V>(g, (const T*)lev[d].x, (const T*)lev[d].b, (T*)lev[d].r, g.gamma, rp);
}

// DGS passes: packs of V cells of one colour in a row (the single-box packed
// items; V = 16 bytes / element size).  A row holds few packs (5 to 33 on
// the batch's boxes), so the packs of consecutive rows are laid out flat
// rather than in BX-wide tiles (which would leave most lanes idle); the
// tile width does not matter for these classes.

template <typename T>
__host__ __device__ constexpr int bpack() {
  return 16 / (int)sizeof(T);
}

template <typename T, int BX>
__global__ __launch_bounds__(BS) void kb_dgs_u(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                               const int* __restrict__ done, int colour) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  constexpr int V = bpack<T>();
  int m, J, K;
  if (!flat_item(g, pack_per_row<V>(g), lb, m, J, K)) return;
  RowPack<V> rp;
  if (row_pack_at<V>(g, colour ^ 1, m, J, K, rp)) dgs_u_pack<T, T, V>(g, (T*)lev[d].x, (const T*)lev[d].b, rp);
}

// launch t of the forward pressure sweep (dgs_pf_stage_pack)
template <typename T, int BX>
__global__ __launch_bounds__(BS) void kb_dgs_pf(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                const int* __restrict__ done, int t) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  constexpr int V = bpack<T>();
  int m, J, K;
  if (!flat_item(g, pack_per_row<V>(g), lb, m, J, K)) return;
  RowPack<V> rp;
  if (row_pack_at<V>(g, (t & 1) ^ 1, m, J, K, rp))
    dgs_pf_stage_pack<T, T, V>(g, (T*)lev[d].x, (const T*)lev[d].b, (T*)lev[d].dscr, rp, t);
}

// one stage of the reverse pressure sweep (dgs_pr_stage_pack)
template <typename T, int BX>
__global__ __launch_bounds__(BS) void kb_dgs_pr(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                const int* __restrict__ done, int stage) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  constexpr int V = bpack<T>();
  int m, J, K;
  if (!flat_item(g, pack_per_row<V>(g), lb, m, J, K)) return;
  RowPack<V> rp;
  if (row_pack_at<V>(g, (stage & 1) ^ 1, m, J, K, rp))
    dgs_pr_stage_pack<T, T, V>(g, (T*)lev[d].x, (const T*)lev[d].b, rp, stage);
}

// restriction into the next level: one item per coarse slot
template <typename T, int BX>
__global__ __launch_bounds__(BS) void kb_restrict(const BEnt* __restrict__ tab, int nent,
                                                  const BLev* __restrict__ lev, const int* __restrict__ done) {
  SG_BATCH_ENTRY();
  const Geom gc = lev[d].gc;
  int I, J, K;
  if (!tile_item<BX>(gc, gc.sy, lb, I, J, K)) return;
  restrict_item<T>(lev[d].g, gc, (const T*)lev[d].r, (T*)lev[d].bc, I, J, K);
}

template <typename T, int BX>
__global__ __launch_bounds__(BS) void kb_prolong(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                 const int* __restrict__ done) {
  SG_BATCH_ENTRY();
  const Geom gc = lev[d].gc;
  int X, Jc, Kc;  // one thread per pair of coarse cells for their sixteen fine children, laid out flat
  if (!flat_item(gc, (gc.nx + 1) >> 1, lb, X, Jc, Kc)) return;
  if (Jc < 1 || Jc > gc.ny || Kc < 1 || Kc > gc.nz) return;
  prolong_pair_item<T>(lev[d].g, gc, (const T*)lev[d].xc, (T*)lev[d].x, 2 * X + 1, Jc, Kc);
}

// Vanka, one pair of colour classes of each domain (classes q and 7-q, one
// list: vanka_pair8): eight lanes per V1 cell for the residuals (one thread
// per cell measured no faster on the batch's boxes) and for the corrections
template <typename T>
__global__ __launch_bounds__(BS) void kb_vanka_delta(const BEnt* __restrict__ tab, int nent,
                                                     const BLev* __restrict__ lev, const int* __restrict__ done,
                                                     int q, T* __restrict__ delta) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  vanka_delta8_item<T, T>(g, (const T*)lev[d].x, (const T*)lev[d].b, lev[d].vc[q], lev[d].nv[q] + lev[d].nv[7 - q],
                         (const T*)lev[d].kinv, delta + lev[d].voff[q], lb * BS + (int)threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(BS) void kb_vanka_apply(const BEnt* __restrict__ tab, int nent,
                                                     const BLev* __restrict__ lev, const int* __restrict__ done,
                                                     int q, const T* __restrict__ delta) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  vanka_apply8_item<T>(g, (T*)lev[d].x, lev[d].vc[q], lev[d].nv[q] + lev[d].nv[7 - q], delta + lev[d].voff[q],
                       lb * BS + (int)threadIdx.x);
}

// Two-copy Vanka pass of pair q for every box (k_vanka_pp8; levels whose
// classes, summed over the boxes, are small enough for the passes to be
// latency chains): reads copy `rd` (0: x, 1: alt), writes the other; lanes
// [0, copy0) take the pair's cells eight lanes each (copy0 = 8 cells rounded
// up to whole waves), the rest copy the previous pair qp's corrections
// (qp < 0: none).
template <typename T>
__global__ __launch_bounds__(BS) void kb_vanka_pp(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                  const int* __restrict__ done, int q, int qp, int rd) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  const T* R = (const T*)(rd ? lev[d].alt : lev[d].x);
  T* W = (T*)(rd ? lev[d].x : lev[d].alt);
  const int n = lev[d].nv[q] + lev[d].nv[7 - q];
  const int copy0 = (8 * n + 63) / 64 * 64;
  const int t = lb * BS + (int)threadIdx.x;
  if (t < copy0) {
    const T dv = vanka_delta8_lane<T, T>(g, R, (const T*)lev[d].b, lev[d].vc[q], n, (const T*)lev[d].kinv, t);
    const int c = t >> 3, r = t & 7;
    if (c < n && r < 7) {
      const int s = lev[d].vc[q][c];
      int I, J, K;
      slot_ijk(g, s, I, J, K);
      const VankaDof dof = vanka_dof(g, s, I, J, K, r);
      if (dof.active) W[dof.e] = R[dof.e] + dv;
    }
  } else if (qp >= 0) {
    const int u = t - copy0, c = u >> 3, r = u & 7;
    if (c < lev[d].nv[qp] + lev[d].nv[7 - qp] && r < 7)
      vanka_copy_dof<T>(g, R, W, lev[d].vc[qp][c], r, vanka_pair8_mask(q));
  }
}

// alt = x on the boundary band of every box (vanka_band_copy_item), or on the
// whole state of a box with a side below 8
template <typename T>
__global__ __launch_bounds__(BS) void kb_vanka_band(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                    const int* __restrict__ done) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  const T* R = (const T*)lev[d].x;
  T* W = (T*)lev[d].alt;
  const long t = (long)lb * BS + threadIdx.x;
  if (g.nx < 8 || g.ny < 8 || g.nz < 8) {
    if (t < 4L * g.field) W[t] = R[t];
    return;
  }
  vanka_band_copy_item<T>(g, R, W, t);
}

// The whole symmetric Vanka step of one small box in one workgroup (one block
// per box; k_vanka_sweep's passes with barriers, corrections held in registers).
struct BLevLists {
  const BLev& l;
  int nc;
  __device__ __forceinline__ const int* cells(int k) const { return l.vc[k]; }
  __device__ __forceinline__ int count(int k) const { return l.nv[k]; }
};

template <typename T>
__global__ __launch_bounds__(VSWEEP_BS) void kb_vanka_sweep(const BEnt* __restrict__ tab, int nent,
                                                            const BLev* __restrict__ lev, const int* __restrict__ done) {
  const int d = tab[bent_find(tab, nent)].dom;
  if (done[d]) return;
  const Geom g = lev[d].g;
  __shared__ T sk[64 * 64];  // local inverses
  __shared__ int scell[VSWEEP_LIST];
  for (int i = threadIdx.x; i < 64 * 64; i += VSWEEP_BS) sk[i] = ((const T*)lev[d].kinv)[i];
  __syncthreads();
  vanka_sweep_passes1<T>(g, BLevLists{lev[d], 8}, (T*)lev[d].x, (const T*)lev[d].b, sk, scell);
}

// coarsest level of each domain: one wave per row of its dense inverse
template <typename T>
__global__ __launch_bounds__(BS) void kb_coarse(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                const int* __restrict__ done) {
  SG_BATCH_ENTRY();
  const int row = lb * (BS / 64) + (int)(threadIdx.x >> 6);
  const int n = lev[d].nc;
  if (row >= n) return;
  coarse_row<T>(lev[d].cinv, lev[d].cdof, n, (const T*)lev[d].b, (T*)lev[d].x, row, threadIdx.x & 63);
}

// x = 0 over the level's whole state vector (flat, 4 values per thread)
template <typename T>
__global__ __launch_bounds__(BS) void kb_zero_level(const BEnt* __restrict__ tab, int nent,
                                                    const BLev* __restrict__ lev, const int* __restrict__ done) {
  SG_BATCH_ENTRY();
  const long n = 4L * lev[d].g.field;
  T* x = (T*)lev[d].x;
  const long base = (long)lb * BS * 4 + threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long i = base + (long)k * BS;
    if (i < n) x[i] = T(0);
  }
}

// -------------------------------------------------- level-0 batch vectors
// Domain d's state vector is [voff[d], voff[d] + 4 field_d) of each batch vector.

template <int MODE, int BX>
__global__ __launch_bounds__(BS) void kb_apply_vec(const BEnt* __restrict__ tab, int nent,
                                                   const BLev* __restrict__ lev, const int* __restrict__ done,
                                                   const long* __restrict__ voff, const double* __restrict__ x,
                                                   const double* __restrict__ b, double* __restrict__ y,
                                                   double* __restrict__ partial) {
  SG_BATCH_ENTRY();
  const Geom g = lev[d].g;
  const long o = voff[d];
  double acc = 0.0;
  int X, J, K;
  RowPack<2> rp;
  if (flat_item(g, slot_packs_per_row<2>(g), lb, X, J, K) && slot_pack_at<2>(g, X, J, K, rp))
    acc = apply_pack<MODE, double, double, 2>(g, x + o, b ? b + o : nullptr, y ? y + o : nullptr, 0.0, rp);
  if (MODE == AP_APPLY_DOT || MODE == AP_RESNORM || MODE == AP_BNORM) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// flat element range of domain d handled by this thread: 4 strided values
#define SG_VEC_LOOP(BODY)                                    \
  const long o_ = voff[d], n_ = vlen[d];                     \
  const long base_ = (long)lb * BS * 4 + threadIdx.x;        \
  _Pragma("unroll") for (int k_ = 0; k_ < 4; ++k_) {         \
    const long j_ = base_ + (long)k_ * BS;                   \
    if (j_ < n_) {                                           \
      const long i = o_ + j_;                                \
      BODY;                                                  \
    }                                                        \
  }

// s -= alpha t; with lev != nullptr (FP32 V-cycle) also the domain's float
// level-0 right-hand side = (float) s (what kb_convert would write)
__global__ __launch_bounds__(BS) void kb_axpy_neg(const BEnt* __restrict__ tab, int nent, const int* __restrict__ done,
                                                  const long* __restrict__ voff, const long* __restrict__ vlen,
                                                  const BScal* __restrict__ sc, double* __restrict__ s,
                                                  const double* __restrict__ t, const BLev* __restrict__ lev) {
  SG_BATCH_ENTRY();
  const double a = sc[d].alpha;
  float* bf = lev ? (float*)lev[d].b : nullptr;
  SG_VEC_LOOP(const double v = s[i] - a * t[i]; s[i] = v; if (bf) bf[j_] = (float)v);
}

// d = cd d + cq q; x += d; q = t + beta q (the next direction from the same q);
// with lev != nullptr t is read from the domain's float level-0 result of the
// FP32 V-cycle (float -> double is exact: the values of the converted t)
__global__ __launch_bounds__(BS) void kb_update_dxq(const BEnt* __restrict__ tab, int nent,
                                                    const int* __restrict__ done, const long* __restrict__ voff,
                                                    const long* __restrict__ vlen, const BScal* __restrict__ sc,
                                                    double* __restrict__ dv, double* __restrict__ q,
                                                    double* __restrict__ x, const double* __restrict__ t,
                                                    const BLev* __restrict__ lev) {
  SG_BATCH_ENTRY();
  const double cd = sc[d].cd, cq = sc[d].cq, bt = sc[d].beta;
  const float* tf = lev ? (const float*)lev[d].x : nullptr;
  SG_VEC_LOOP(const double qv = q[i]; const double v = cd * dv[i] + cq * qv; dv[i] = v; x[i] += v;
              q[i] = (tf ? (double)tf[j_] : t[i]) + bt * qv);
}

// q = t, d = 0 (start of SQMR)
__global__ __launch_bounds__(BS) void kb_init_qd(const BEnt* __restrict__ tab, int nent, const int* __restrict__ done,
                                                 const long* __restrict__ voff, const long* __restrict__ vlen,
                                                 double* __restrict__ q, double* __restrict__ dv,
                                                 const double* __restrict__ t) {
  SG_BATCH_ENTRY();
  SG_VEC_LOOP(q[i] = t[i]; dv[i] = 0.0);
}

// x = 0 for the domains whose right-hand side is zero (not gated by done)
__global__ __launch_bounds__(BS) void kb_zero_flagged(const BEnt* __restrict__ tab, int nent,
                                                      const long* __restrict__ voff, const long* __restrict__ vlen,
                                                      const BScal* __restrict__ sc, double* __restrict__ x) {
  const int e_ = bent_find(tab, nent);
  const int d = tab[e_].dom;
  if (!sc[d].zero_x) return;
  const int lb = (int)blockIdx.x - tab[e_].bstart;
  SG_VEC_LOOP(x[i] = 0.0);
}

// partial[2 blk] = sum a.a, partial[2 blk + 1] = sum a.c over the domain's slice
// (with lev != nullptr, a is the domain's float level-0 result, as above)
__global__ __launch_bounds__(BS) void kb_dot2(const BEnt* __restrict__ tab, int nent, const int* __restrict__ done,
                                              const long* __restrict__ voff, const long* __restrict__ vlen,
                                              const double* __restrict__ a, const double* __restrict__ c,
                                              double* __restrict__ partial, const BLev* __restrict__ lev) {
  SG_BATCH_ENTRY();
  double s0 = 0.0, s1 = 0.0;
  const float* af = lev ? (const float*)lev[d].x : nullptr;
  SG_VEC_LOOP(const double av = af ? (double)af[j_] : a[i]; s0 += av * av; s1 += av * c[i]);
  const double t0 = block_sum(s0);
  const double t1 = block_sum(s1);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = t0;
    partial[2 * blockIdx.x + 1] = t1;
  }
}

// FP64 batch slice <-> the domain's level-0 buffer in the V-cycle precision
template <typename Ti, typename To, bool TO_LEVEL>
__global__ __launch_bounds__(BS) void kb_convert(const BEnt* __restrict__ tab, int nent, const int* __restrict__ done,
                                                 const long* __restrict__ voff, const long* __restrict__ vlen,
                                                 const BLev* __restrict__ lev, const Ti* __restrict__ vec,
                                                 To* __restrict__ vout) {
  SG_BATCH_ENTRY();
  const long o_ = voff[d], n_ = vlen[d];
  const long base = (long)lb * BS * 4 + threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long j = base + (long)k * BS;
    if (j < n_) {
      if (TO_LEVEL)
        ((To*)lev[d].b)[j] = (To)vec[o_ + j];
      else
        vout[o_ + j] = (To)((const Ti*)lev[d].x)[j];
    }
  }
}

// zero the slots of x that are not unknowns (level-0 flat slots of each field)
__global__ __launch_bounds__(BS) void kb_clear_ghosts(const BEnt* __restrict__ tab, int nent,
                                                      const BLev* __restrict__ lev, const long* __restrict__ voff,
                                                      double* __restrict__ x) {
  const int e_ = bent_find(tab, nent);
  const int d = tab[e_].dom;
  const int lb = (int)blockIdx.x - tab[e_].bstart;
  const Geom g = lev[d].g;
  const int s = lb * BS + (int)threadIdx.x;
  if (s >= g.field) return;
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  double* xv = x + voff[d];
  const int F = g.field;
  const int e = g.at(s);
  if (!g.ux_active(I, J, K)) xv[e] = 0.0;
  if (!g.uy_active(I, J, K)) xv[F + e] = 0.0;
  if (!g.uz_active(I, J, K)) xv[2 * F + e] = 0.0;
  if (!g.p_active(I, J, K)) xv[3 * F + e] = 0.0;
}

// partial[blk] = sum of active p over the block's slots (pressure mean)
__global__ __launch_bounds__(BS) void kb_sum_p(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                               const int* __restrict__ skip, const long* __restrict__ voff,
                                               const double* __restrict__ x, double* __restrict__ partial) {
  const int e_ = bent_find(tab, nent);
  const int d = tab[e_].dom;
  if (skip[d]) return;
  const int lb = (int)blockIdx.x - tab[e_].bstart;
  const Geom g = lev[d].g;
  const int s = lb * BS + (int)threadIdx.x;
  double v = 0.0;
  if (s < g.field) {
    int I, J, K;
    slot_ijk(g, s, I, J, K);
    if (g.p_active(I, J, K)) v = x[voff[d] + 3L * g.field + g.at(s)];
  }
  const double t = block_sum(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(BS) void kb_shift_p(const BEnt* __restrict__ tab, int nent, const BLev* __restrict__ lev,
                                                 const int* __restrict__ skip, const long* __restrict__ voff,
                                                 const BScal* __restrict__ sc, double* __restrict__ x) {
  const int e_ = bent_find(tab, nent);
  const int d = tab[e_].dom;
  if (skip[d]) return;
  const int lb = (int)blockIdx.x - tab[e_].bstart;
  const Geom g = lev[d].g;
  const int s = lb * BS + (int)threadIdx.x;
  if (s >= g.field) return;
  int I, J, K;
  slot_ijk(g, s, I, J, K);
  const double mean = sc[d].red[RED0] / ((double)g.nx * g.ny * g.nz);
  if (g.p_active(I, J, K)) x[voff[d] + 3L * g.field + g.at(s)] -= mean;
}

// sc[d].red[slot + k] = sum of partial[blk * stride + k] over the domain's blocks, in order
__global__ __launch_bounds__(BS) void kb_seg_reduce(const BEnt* __restrict__ tab, int nent,
                                                    const int* __restrict__ skip, const double* __restrict__ partial,
                                                    int stride, int slot, BScal* __restrict__ sc) {
  const int e = blockIdx.x;
  if (e >= nent) return;
  const int d = tab[e].dom;
  if (skip[d]) return;
  const int b0 = tab[e].bstart;
  const int b1 = e + 1 < nent ? tab[e + 1].bstart : tab[nent].bstart;  // the table carries a closing entry
  for (int k = 0; k < stride; ++k) {
    double v = 0.0;
    for (int b = b0 + (int)threadIdx.x; b < b1; b += BS) v += partial[(long)b * stride + k];
    const double t = block_sum(v);
    if (threadIdx.x == 0) sc[d].red[slot + k] = t;
  }
}

#undef SG_VEC_LOOP
#undef SG_BATCH_ENTRY

}  // namespace sg
