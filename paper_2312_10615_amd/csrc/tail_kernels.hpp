// The small levels of a V-cycle in one launch (opt-in).  One workgroup of
// 1024 threads runs the whole recursion from the first level of <= 16^3 cells
// down to the coarsest and back: the same item bodies as the per-level
// kernels, in the same phase order, with a workgroup barrier between phases.
// Within a phase the items are independent (red/black and colour classes), so
// it computes what the per-level launches compute (those run packed versions
// of the item bodies, whose fused multiply-adds may round differently; the
// results agree to rounding).  Measured: a
// phase costs the workgroup two to four dependent memory round trips (~6 us),
// more than a per-level launch replayed from a graph (~1.7 us), so the
// per-level launches stay the default.
#pragma once

#include "kernels.hpp"

namespace sg {

constexpr int TAIL_BS = 1024;
constexpr int TAIL_MAX = 8;          // levels a tail may hold
constexpr long TAIL_CELLS = 4096;    // a level joins the tail at <= 16^3 cells

struct TailLev {
  Geom g, gc;
  void* x;
  void* b;
  void* r;
  void* dscr;
  const void* kinv;
  const int* vc[8];
  int nv[8];
  const double* cinv;   // coarsest level only
  const int* cdof;
  int nc;
};

struct TailArgs {
  int nt;          // levels in the tail; the last one is the coarsest
  int nu, nb, symmetric;
  void* vdelta;
};

__device__ __forceinline__ void tail_rows(const Geom& g, int per_row, long i, int& X, int& J, int& K) {
  X = (int)(i % per_row);
  const long row = i / per_row;
  J = (int)(row % (g.ny + 2));
  K = (int)(row / (g.ny + 2));
}

template <typename T>
__device__ void tl_zero(const TailLev& L, T* x) {
  const long n = 4L * L.g.field;
  for (long i = threadIdx.x; i < n; i += TAIL_BS) x[i] = T(0);
}

template <typename T>
__device__ void tl_dgs_u(const TailLev& L, T* x, const T* b, int colour) {
  const Geom& g = L.g;
  const int pr = g.sy >> 1;
  const long n = (long)pr * (g.ny + 2) * (g.nz + 2);
  for (long i = threadIdx.x; i < n; i += TAIL_BS) {
    int m, J, K;
    tail_rows(g, pr, i, m, J, K);
    dgs_u_item<T, T>(g, x, b, 2 * m + ((colour + 1 + J + K) & 1), J, K);
  }
}

template <typename T>
__device__ void tl_pf_own(const TailLev& L, T* x, const T* b, int colour) {
  const Geom& g = L.g;
  const int pr = g.sy >> 1;
  const long n = (long)pr * (g.ny + 2) * (g.nz + 2);
  for (long i = threadIdx.x; i < n; i += TAIL_BS) {
    int m, J, K;
    tail_rows(g, pr, i, m, J, K);
    dgs_pf_own_item<T, T>(g, x, b, (T*)L.dscr, 2 * m + ((colour + 1 + J + K) & 1), J, K);
  }
}

template <typename T>
__device__ void tl_pf_nbr(const TailLev& L, T* x, int colour) {
  const Geom& g = L.g;
  const int pr = g.sy >> 1;
  const long n = (long)pr * (g.ny + 2) * (g.nz + 2);
  for (long i = threadIdx.x; i < n; i += TAIL_BS) {
    int m, J, K;
    tail_rows(g, pr, i, m, J, K);
    dgs_pf_nbr_item<T>(g, x, (const T*)L.dscr, 2 * m + (((colour ^ 1) + 1 + J + K) & 1), J, K);
  }
}

template <typename T>
__device__ void tl_pr(const TailLev& L, T* x, const T* b, int colour) {
  const Geom& g = L.g;
  const int pr = g.sy >> 1;
  const long n = (long)pr * (g.ny + 2) * (g.nz + 2);
  for (long i = threadIdx.x; i < n; i += TAIL_BS) {
    int m, J, K;
    tail_rows(g, pr, i, m, J, K);
    dgs_pr_item<T, T>(g, x, b, 2 * m + ((colour + 1 + J + K) & 1), J, K);
  }
}

template <typename T>
__device__ void tl_vanka_symmetric(const TailLev& L, T* x, const T* b, T* vd) {
  for (int pass = 0; pass < 16; ++pass) {
    const int k = pass < 8 ? pass : 15 - pass;
    const int n = L.nv[k];
    if (n == 0) continue;
    for (int c = threadIdx.x; c < n; c += TAIL_BS) vanka_delta_item<T, T>(L.g, x, b, L.vc[k], n, (const T*)L.kinv, vd, c);
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += TAIL_BS) vanka_apply_item<T>(L.g, x, L.vc[k], n, vd, c);
    __syncthreads();
  }
}

template <typename T>
__device__ void tl_dgs_forward(const TailLev& L, T* x, const T* b) {
  for (int col = 0; col < 2; ++col) {
    tl_dgs_u<T>(L, x, b, col);
    __syncthreads();
  }
  for (int col = 0; col < 2; ++col) {
    tl_pf_own<T>(L, x, b, col);
    __syncthreads();
    tl_pf_nbr<T>(L, x, col);
    __syncthreads();
  }
}

template <typename T>
__device__ void tl_dgs_reverse(const TailLev& L, T* x, const T* b) {
  for (int col = 1; col >= 0; --col) {
    tl_pr<T>(L, x, b, col);
    __syncthreads();
  }
  for (int col = 1; col >= 0; --col) {
    tl_dgs_u<T>(L, x, b, col);
    __syncthreads();
  }
}

// Alg. 3 with the interior smoother of the schedule: kind 0 symmetric, 1 reverse, 2 forward
template <typename T>
__device__ void tl_smooth(const TailArgs& a, const TailLev& L, T* x, const T* b, int kind, int sweeps) {
  T* vd = (T*)a.vdelta;
  for (int i = 0; i < a.nb; ++i) tl_vanka_symmetric<T>(L, x, b, vd);
  for (int i = 0; i < sweeps; ++i) {
    if (kind != 2) {
      if (kind == 0) tl_dgs_forward<T>(L, x, b);
      tl_dgs_reverse<T>(L, x, b);
    } else {
      tl_dgs_forward<T>(L, x, b);
    }
  }
  for (int i = 0; i < a.nb; ++i) tl_vanka_symmetric<T>(L, x, b, vd);
}

template <typename T>
__device__ void tl_presmooth(const TailArgs& a, const TailLev& L, T* x, const T* b) {
  if (a.symmetric) {
    for (int i = 0; i < a.nu / 2; ++i) tl_smooth<T>(a, L, x, b, 0, 1);
  } else {
    tl_smooth<T>(a, L, x, b, 1, a.nu);
  }
}

template <typename T>
__device__ void tl_postsmooth(const TailArgs& a, const TailLev& L, T* x, const T* b) {
  if (a.symmetric) {
    for (int i = 0; i < a.nu / 2; ++i) tl_smooth<T>(a, L, x, b, 0, 1);
  } else {
    tl_smooth<T>(a, L, x, b, 2, a.nu);
  }
}

// x0 = V-CYCLE(L~, b0, 0) over the tail levels (Alg. 1), one workgroup.
// x0 / b0 are the first tail level's vectors; deeper levels use lev[l].x / .b.
template <typename T>
__global__ __launch_bounds__(TAIL_BS) void k_tail(TailArgs a, const TailLev* __restrict__ lev, T* __restrict__ x0,
                                                  const T* __restrict__ b0) {
  // going down: zero x, smooth, residual, restrict; the coarsest level solves
  for (int l = 0; l < a.nt; ++l) {
    const TailLev& L = lev[l];
    T* x = l == 0 ? x0 : (T*)L.x;
    const T* b = l == 0 ? b0 : (const T*)L.b;
    tl_zero<T>(L, x);
    __syncthreads();
    if (l == a.nt - 1) {
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      for (int r = wave; r < L.nc; r += TAIL_BS / 64) coarse_row<T>(L.cinv, L.cdof, L.nc, b, x, r, lane);
      __syncthreads();
      break;
    }
    tl_presmooth<T>(a, L, x, b);
    const Geom& g = L.g;
    const long ns = (long)g.sy * (g.ny + 2) * (g.nz + 2);
    for (long i = threadIdx.x; i < ns; i += TAIL_BS) {
      int I, J, K;
      tail_rows(g, g.sy, i, I, J, K);
      apply_item<AP_RESID, T, T>(g, x, b, (T*)L.r, g.gamma, I, J, K);
    }
    __syncthreads();
    const Geom& gc = L.gc;
    const long nc = (long)gc.sy * (gc.ny + 2) * (gc.nz + 2);
    for (long i = threadIdx.x; i < nc; i += TAIL_BS) {
      int I, J, K;
      tail_rows(gc, gc.sy, i, I, J, K);
      restrict_item<T>(g, gc, (const T*)L.r, (T*)lev[l + 1].b, I, J, K);
    }
    __syncthreads();
  }
  // going up: prolong the correction, post-smooth
  for (int l = a.nt - 2; l >= 0; --l) {
    const TailLev& L = lev[l];
    T* x = l == 0 ? x0 : (T*)L.x;
    const T* b = l == 0 ? b0 : (const T*)L.b;
    const Geom& g = L.g;
    const long ns = (long)g.sy * (g.ny + 2) * (g.nz + 2);
    for (long i = threadIdx.x; i < ns; i += TAIL_BS) {
      int I, J, K;
      tail_rows(g, g.sy, i, I, J, K);
      prolong_item<T>(g, L.gc, (const T*)lev[l + 1].x, x, I, J, K);
    }
    __syncthreads();
    tl_postsmooth<T>(a, L, x, b);
  }
}

}  // namespace sg
