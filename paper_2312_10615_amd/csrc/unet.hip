// Kernels of the warm-start U-Net for gfx950: 3x3x3 convolutions and their
// gradients on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, float
// accumulation), the 1x1x1 head, the loss, Adam and the conversions between a
// Stokes state vector and voxel tensors.
//
// Convolution as an implicit GEMM.  A block owns a 16 x 4 x 4 (x, y, z) tile
// of output voxels; wave w owns the z-plane w of the tile and, inside it, four
// 16-voxel rows (the M dimension of four MFMA tiles).  The input halo tile
// (18 x 6 x 6 voxels) is staged channels-last in LDS, one chunk of CC input
// channels at a time.  The K dimension of a chunk is (tap, channel) with the
// channel fastest, taken 8 channels (one 16-byte LDS read) per lane group:
// lane l of the wave supplies voxel row element l % 16 and K octet l / 16 of
// each 16x16x32 product, so a lane's A fragment is the 8 consecutive channels
// of one shifted voxel.  The B fragments (weights) are pre-packed in exactly
// this lane order, so each is one 16-byte load per lane.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "stokes_unet.h"

namespace un {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BS = 256;
constexpr int TX = 16, TY = 4, TZ = 4;  // output tile of a convolution block
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;
constexpr int TV = TX * TY * TZ;        // 256 voxels, one per thread

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// float -> bfloat16, round to nearest even (NaN stays a quiet NaN)
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// double -> bfloat16, round to nearest even in one step (no double rounding
// through float).  Finite inputs within the float range.
__device__ __forceinline__ uint32_t d2bf(double d) {
  if (d == 0.0) return (uint32_t)(__double_as_longlong(d) >> 48) & 0x8000u;
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  const unsigned long long sign = u >> 63;
  // round the 52-bit mantissa to 7 bits, ties to even
  u += (1ull << 44) - 1 + ((u >> 45) & 1ull);
  const int e = (int)((u >> 52) & 0x7ff) - 1023 + 127;
  const uint32_t mant = (uint32_t)((u >> 45) & 0x7f);
  if (e <= 0) return (uint32_t)(sign << 15);  // below the normal range: flush (never reached by the data)
  if (e >= 255) return (uint32_t)(sign << 15) | 0x7f80u;
  return (uint32_t)(sign << 15) | ((uint32_t)e << 7) | mant;
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// ------------------------------------------------------------ input staging

struct Src {
  int mode, nz, ny, nx, ch, c_first;
  const uint16_t* s0;
  const uint16_t* s1;
};

// keep the bf16 halves of d where the gate m is > 0 (sign clear, not zero)
__device__ __forceinline__ uint32_t gate2(uint32_t d, uint32_t m) {
  const uint32_t lo = ((m & 0x8000u) == 0 && (m & 0xffffu) != 0) ? (d & 0xffffu) : 0u;
  const uint32_t hi = ((m & 0x80000000u) == 0 && (m >> 16) != 0) ? (d & 0xffff0000u) : 0u;
  return lo | hi;
}

// 8 channels [c, c+8) of the layer input at voxel (z, y, x), inside the grid.
// MODE >= 0 fixes the source mode at compile time (the kernel then carries
// no registers for the other modes' paths); MODE = -1 reads it from s.
template <int MODE = -1>
__device__ __forceinline__ uint4 load8(const Src& s, int z, int y, int x, int c) {
  const int mode = MODE >= 0 ? MODE : s.mode;
  if (mode == UNET_SRC_DIRECT) {
    return *(const uint4*)(s.s0 + (((size_t)z * s.ny + y) * s.nx + x) * s.ch + c);
  }
  if (mode == UNET_SRC_MASKED) {
    const size_t o = (((size_t)z * s.ny + y) * s.nx + x) * s.ch + c;
    const uint4 d = *(const uint4*)(s.s0 + o);
    const uint4 m = *(const uint4*)(s.s1 + o);
    return uint4{gate2(d.x, m.x), gate2(d.y, m.y), gate2(d.z, m.z), gate2(d.w, m.w)};
  }
  if (mode == UNET_SRC_POOL) {
    const int fy = 2 * s.ny, fx = 2 * s.nx;
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          const uint4 v =
              *(const uint4*)(s.s0 + (((size_t)(2 * z + cz) * fy + (2 * y + cy)) * fx + (2 * x + cx)) * s.ch + c);
          const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            a[2 * k] += bf2f(w[k] & 0xffffu);
            a[2 * k + 1] += bf2f(w[k] >> 16);
          }
        }
    uint32_t r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = f2bf(a[2 * k] * 0.125f) | (f2bf(a[2 * k + 1] * 0.125f) << 16);
    return uint4{r[0], r[1], r[2], r[3]};
  }
  // UNET_SRC_CAT_UP
  if (c < s.c_first) {
    const int cy = s.ny >> 1, cx = s.nx >> 1;
    return *(const uint4*)(s.s0 + (((size_t)(z >> 1) * cy + (y >> 1)) * cx + (x >> 1)) * s.c_first + c);
  }
  const int c2 = s.ch - s.c_first;
  return *(const uint4*)(s.s1 + (((size_t)z * s.ny + y) * s.nx + x) * c2 + (c - s.c_first));
}

__device__ __forceinline__ void tile_origin(const Src& s, int tile, int& x0, int& y0, int& z0) {
  const int tx = (s.nx + TX - 1) / TX, ty = (s.ny + TY - 1) / TY;
  x0 = (tile % tx) * TX;
  tile /= tx;
  y0 = (tile % ty) * TY;
  z0 = (tile / ty) * TZ;
}

// Stage channels [cbase, cbase + CC) of the halo tile around (x0, y0, z0) into
// lds[hv * STR + c]; voxels outside the grid read as zero.
template <int CC, int STR, int MODE = -1>
__device__ __forceinline__ void stage_halo(const Src& s, int x0, int y0, int z0, int cbase, uint16_t* lds) {
  constexpr int OCT = CC / 8;
  for (int i = threadIdx.x; i < HV * OCT; i += BS) {
    const int hv = i / OCT, c8 = i - hv * OCT;
    const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
    uint4 v = uint4{0u, 0u, 0u, 0u};
    if (gx >= 0 && gx < s.nx && gy >= 0 && gy < s.ny && gz >= 0 && gz < s.nz)
      v = load8<MODE>(s, gz, gy, gx, cbase + c8 * 8);
    *(uint4*)(lds + hv * STR + c8 * 8) = v;
  }
}

// --------------------------------------------------------------- conv3 fwd

// K octets and k-steps of one CC-channel chunk
template <int CC>
struct Chunk {
  static constexpr int OCT = CC / 8;
  static constexpr int KOCT = 27 * OCT;
  static constexpr int KS = (KOCT + 3) / 4;
};

template <int CC, int NS, int MODE>
__global__ __launch_bounds__(BS) void k_conv3(Src src, int cout, const uint4* __restrict__ frag,
                                              const float* __restrict__ bias, void* __restrict__ out, int relu,
                                              int out_f32) {
  constexpr int STR = CC + 8;  // padded voxel stride: conflict-free 16-byte row reads
  constexpr int OCT = Chunk<CC>::OCT, KOCT = Chunk<CC>::KOCT, KS = Chunk<CC>::KS;
  __shared__ __align__(16) uint16_t lds[HV * STR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  int x0, y0, z0;
  tile_origin(src, blockIdx.x, x0, y0, z0);
  f32x4 acc[4][NS];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < NS; ++j) acc[s][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = src.ch / CC;
  for (int q = 0; q < nchunks; ++q) {
    __syncthreads();
    stage_halo<CC, STR, MODE>(src, x0, y0, z0, q * CC, lds);
    __syncthreads();
    const uint4* wq = frag + (size_t)q * KS * NS * 64;
    for (int ks = 0; ks < KS; ++ks) {
      const int o = ks * 4 + g;
      const bool valid = o < KOCT;
      const int t = valid ? o / OCT : 0;
      const int c8 = valid ? o - t * OCT : 0;
      const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
      bf16x8 a[4], b[NS];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int hv = ((wave + dz) * HY + (s + dy)) * HX + (m + dx);
        uint4 v = *(const uint4*)(lds + hv * STR + c8 * 8);
        if (!valid) v = uint4{0u, 0u, 0u, 0u};
        a[s] = as_bf16x8(v);
      }
#pragma unroll
      for (int j = 0; j < NS; ++j) b[j] = as_bf16x8(wq[(ks * NS + j) * 64 + lane]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < NS; ++j) acc[s][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], b[j], acc[s][j], 0, 0, 0);
    }
  }
  // lane holds rows 4g..4g+3 (voxels along x) of output channel j*16 + m
  const int z = z0 + wave;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int co = j * 16 + m;
    const float bv = bias ? bias[co] : 0.f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int y = y0 + s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + 4 * g + i;
        if (x < src.nx && y < src.ny && z < src.nz) {
          float v = acc[s][j][i] + bv;
          if (relu) v = fmaxf(v, 0.f);
          const size_t o = (((size_t)z * src.ny + y) * src.nx + x) * cout + co;
          if (out_f32)
            ((float*)out)[o] = v;
          else
            ((uint16_t*)out)[o] = (uint16_t)f2bf(v);
        }
      }
    }
  }
}

// Pack master weights into per-lane fragments: element e of lane l of k-step
// ks, output subtile j, chunk q holds W'[t][ci][co] with K octet
// o = 4 ks + l / 16 = (t, c8), ci = q CC + 8 c8 + e, co = 16 j + l % 16.
// transpose: W'[t][ci][co] = w[26 - t][co][ci] (input-gradient convolution).
__global__ __launch_bounds__(BS) void k_pack(const float* __restrict__ w, int cin, int cout, int transpose, int cc,
                                             uint4* __restrict__ frag, long n_uint4) {
  const long i = (long)blockIdx.x * BS + threadIdx.x;
  if (i >= n_uint4) return;
  const int ci_n = transpose ? cout : cin, co_n = transpose ? cin : cout;
  const int ns = co_n / 16, oct = cc / 8, koct = 27 * oct, ks_n = (koct + 3) / 4;
  const int lane = (int)(i % 64);
  long r = i / 64;
  const int j = (int)(r % ns);
  r /= ns;
  const int ks = (int)(r % ks_n);
  const int q = (int)(r / ks_n);
  const int o = ks * 4 + lane / 16;
  const int co = j * 16 + lane % 16;
  uint32_t h[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float v = 0.f;
    if (o < koct) {
      const int t = o / oct, c8 = o % oct;
      const int ci = q * cc + c8 * 8 + e;
      (void)ci_n;
      v = transpose ? w[((size_t)(26 - t) * cin + co) * cout + ci] : w[((size_t)t * cin + ci) * cout + co];
    }
    h[e] = f2bf(v);
  }
  frag[i] = uint4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
}

// ------------------------------------------------------------ conv3 wgrad

// dW as a sum over voxel tiles of 16x16x32 products with the voxels as K:
// A = dz^T (output channel x voxel), B = shifted input (voxel x input channel).
// blockIdx.y = (chunk q, group of (tap, 16-channel) pairs), blockIdx.x = a
// contiguous range of voxel tiles; each block writes one partial sum.
template <int CC, int NSO>
__global__ __launch_bounds__(BS) void k_wgrad(Src xs, Src ds, int ntiles, int tiles_per_block, int npg,
                                              float* __restrict__ partial, float* __restrict__ bpartial) {
  constexpr int CSUB = (CC + 15) / 16;
  constexpr int PAIRS = 27 * CSUB;
  constexpr int TPW = 16 / NSO;
  constexpr int PPB = 4 * TPW;
  constexpr int COUT = 16 * NSO;
  __shared__ __align__(16) uint16_t lx[HV * CC];
  __shared__ __align__(16) uint16_t ld[TV * COUT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int q = blockIdx.y / npg, pg = blockIdx.y % npg;
  const int cin = xs.ch;
  int pt[TPW], pc[TPW];
  bool pv[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    int p = pg * PPB + wave * TPW + i;
    pv[i] = p < PAIRS;
    p = pv[i] ? p : 0;
    pt[i] = p / CSUB;
    pc[i] = p % CSUB;
  }
  f32x4 acc[TPW][NSO];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int os = 0; os < NSO; ++os) acc[i][os] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // channel tid % COUT over voxels tid / COUT + k BS / COUT of each tile
  const int t0 = blockIdx.x * tiles_per_block;
  const int t1 = min(ntiles, t0 + tiles_per_block);
  for (int tile = t0; tile < t1; ++tile) {
    int x0, y0, z0;
    tile_origin(xs, tile, x0, y0, z0);
    __syncthreads();
    stage_halo<CC, CC>(xs, x0, y0, z0, q * CC, lx);
    for (int i = tid; i < TV * (COUT / 8); i += BS) {
      const int v = i / (COUT / 8), c8 = i - v * (COUT / 8);
      const int x = x0 + (v & 15), y = y0 + ((v >> 4) & 3), z = z0 + (v >> 6);
      uint4 val = uint4{0u, 0u, 0u, 0u};
      if (x < ds.nx && y < ds.ny && z < ds.nz) val = load8(ds, z, y, x, c8 * 8);
      *(uint4*)(ld + v * COUT + c8 * 8) = val;
    }
    __syncthreads();
    if (blockIdx.y == 0)
      for (int v = tid / COUT; v < TV; v += BS / COUT) bsum += bf2f(ld[v * COUT + tid % COUT]);
    for (int kk = 0; kk < TV / 32; ++kk) {
      // this lane group's 8 voxels: one half row of the tile
      const int vb = 32 * kk + 8 * g;
      const int xb = vb & 15, y = (vb >> 4) & 3, z = vb >> 6;
      bf16x8 a[NSO];
#pragma unroll
      for (int os = 0; os < NSO; ++os) {
        uint32_t h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          h[e] = (uint32_t)ld[(vb + 2 * e) * COUT + os * 16 + m] |
                 ((uint32_t)ld[(vb + 2 * e + 1) * COUT + os * 16 + m] << 16);
        a[os] = as_bf16x8(uint4{h[0], h[1], h[2], h[3]});
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        if (!pv[i]) continue;
        const int t = pt[i];
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        const int ci = pc[i] * 16 + m;
        const int hb = ((z + dz) * HY + (y + dy)) * HX + (xb + dx);
        uint32_t h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t lo = ci < CC ? (uint32_t)lx[(hb + 2 * e) * CC + ci] : 0u;
          const uint32_t hi = ci < CC ? (uint32_t)lx[(hb + 2 * e + 1) * CC + ci] : 0u;
          h[e] = lo | (hi << 16);
        }
        const bf16x8 b = as_bf16x8(uint4{h[0], h[1], h[2], h[3]});
#pragma unroll
        for (int os = 0; os < NSO; ++os)
          acc[i][os] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[os], b, acc[i][os], 0, 0, 0);
      }
    }
  }
  float* P = partial + (size_t)blockIdx.x * 27 * cin * COUT;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (!pv[i]) continue;
    const int cl = pc[i] * 16 + m;
    if (cl >= CC) continue;
    const int ci = q * CC + cl;
#pragma unroll
    for (int os = 0; os < NSO; ++os)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[((size_t)pt[i] * cin + ci) * COUT + os * 16 + 4 * g + r] = acc[i][os][r];
  }
  if (blockIdx.y == 0) {
    __shared__ float bred[BS];
    bred[tid] = bsum;
    __syncthreads();
    if (tid < COUT) {
      float s = 0.f;
      for (int r = 0; r < BS / COUT; ++r) s += bred[r * COUT + tid];
      bpartial[(size_t)blockIdx.x * COUT + tid] = s;
    }
  }
}

// out[i] = sum over rows r (in order) of partial[r * stride + i], accumulated in double
__global__ __launch_bounds__(BS) void k_sum_rows(const float* __restrict__ partial, int rows, long stride, long n,
                                                 float* __restrict__ out) {
  const long i = (long)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += (double)partial[(size_t)r * stride + i];
  out[i] = (float)s;
}

// ----------------------------------------------------------- skip links

__global__ __launch_bounds__(BS) void k_up_grad(const uint16_t* __restrict__ fine, int cf, int coff, int c, int nz,
                                                int ny, int nx, uint16_t* __restrict__ coarse) {
  const long i = (long)blockIdx.x * BS + threadIdx.x;
  const long n = (long)nz * ny * nx * c;
  if (i >= n) return;
  const int ch = (int)(i % c);
  long v = i / c;
  const int x = (int)(v % nx);
  v /= nx;
  const int y = (int)(v % ny);
  const int z = (int)(v / ny);
  float s = 0.f;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx)
        s += bf2f(fine[(((size_t)(2 * z + cz) * (2 * ny) + (2 * y + cy)) * (2 * nx) + (2 * x + cx)) * cf + coff + ch]);
  coarse[i] = (uint16_t)f2bf(s);
}

__global__ __launch_bounds__(BS) void k_skip_grad(const uint16_t* __restrict__ fine, int cf, int coff,
                                                  const uint16_t* __restrict__ pooled, int c, int nz, int ny, int nx,
                                                  uint16_t* __restrict__ out) {
  const long i = (long)blockIdx.x * BS + threadIdx.x;
  const long n = (long)nz * ny * nx * c;
  if (i >= n) return;
  const int ch = (int)(i % c);
  long v = i / c;
  const int x = (int)(v % nx);
  v /= nx;
  const int y = (int)(v % ny);
  const int z = (int)(v / ny);
  const float a = bf2f(fine[(((size_t)z * ny + y) * nx + x) * cf + coff + ch]);
  const float p = bf2f(pooled[(((size_t)(z >> 1) * (ny >> 1) + (y >> 1)) * (nx >> 1) + (x >> 1)) * c + ch]);
  out[i] = (uint16_t)f2bf(a + p * 0.125f);
}

// ------------------------------------------------------------------- head

__global__ __launch_bounds__(BS) void k_head_fwd(const uint16_t* __restrict__ d, const float* __restrict__ hw,
                                                 const float* __restrict__ hb, float* __restrict__ out, long nvox) {
  __shared__ float w[64];
  if (threadIdx.x < 64) w[threadIdx.x] = bf2f(f2bf(hw[threadIdx.x]));
  __syncthreads();
  const long v = (long)blockIdx.x * BS + threadIdx.x;
  if (v >= nvox) return;
  const uint4 p0 = *(const uint4*)(d + v * 16), p1 = *(const uint4*)(d + v * 16 + 8);
  const uint32_t wd[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
  float a[16];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[2 * k] = bf2f(wd[k] & 0xffffu);
    a[2 * k + 1] = bf2f(wd[k] >> 16);
  }
  float o[4];
#pragma unroll
  for (int co = 0; co < 4; ++co) {
    float s = 0.f;
#pragma unroll
    for (int ci = 0; ci < 16; ++ci) s = fmaf(a[ci], w[ci * 4 + co], s);
    o[co] = s + hb[co];
  }
  *(float4*)(out + v * 4) = float4{o[0], o[1], o[2], o[3]};
}

// 68 sums per block (dhw 16x4, dhb 4) over a fixed voxel range, reduced in a
// fixed order inside the block
__global__ __launch_bounds__(BS) void k_head_bwd(const uint16_t* __restrict__ d, const float* __restrict__ dout,
                                                 const float* __restrict__ hw, uint16_t* __restrict__ dd,
                                                 float* __restrict__ partial, long nvox, long per_block) {
  __shared__ float w[64];
  __shared__ float red[BS / 64][68];
  if (threadIdx.x < 64) w[threadIdx.x] = bf2f(f2bf(hw[threadIdx.x]));
  __syncthreads();
  float sw[68];
#pragma unroll
  for (int k = 0; k < 68; ++k) sw[k] = 0.f;
  const long v0 = (long)blockIdx.x * per_block;
  const long v1 = v0 + per_block < nvox ? v0 + per_block : nvox;
  for (long v = v0 + threadIdx.x; v < v1; v += BS) {
    const float4 g4 = *(const float4*)(dout + v * 4);
    const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
    const uint4 p0 = *(const uint4*)(d + v * 16), p1 = *(const uint4*)(d + v * 16 + 8);
    const uint32_t wd[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
    uint32_t outw[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float a0 = bf2f(wd[k] & 0xffffu), a1 = bf2f(wd[k] >> 16);
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int co = 0; co < 4; ++co) {
        s0 = fmaf(gv[co], w[(2 * k) * 4 + co], s0);
        s1 = fmaf(gv[co], w[(2 * k + 1) * 4 + co], s1);
        sw[(2 * k) * 4 + co] = fmaf(a0, gv[co], sw[(2 * k) * 4 + co]);
        sw[(2 * k + 1) * 4 + co] = fmaf(a1, gv[co], sw[(2 * k + 1) * 4 + co]);
      }
      outw[k] = f2bf(s0) | (f2bf(s1) << 16);
    }
#pragma unroll
    for (int co = 0; co < 4; ++co) sw[64 + co] += gv[co];
    *(uint4*)(dd + v * 16) = uint4{outw[0], outw[1], outw[2], outw[3]};
    *(uint4*)(dd + v * 16 + 8) = uint4{outw[4], outw[5], outw[6], outw[7]};
  }
  // wave reduction (fixed butterfly), then the 4 waves in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 68; ++k) {
    float s = sw[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 68) {
    float s = 0.f;
    for (int wv = 0; wv < BS / 64; ++wv) s += red[wv][threadIdx.x];
    partial[(size_t)blockIdx.x * 68 + threadIdx.x] = s;
  }
}

// --------------------------------------------------------------- loss, adam

__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double red[BS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BS / 64; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(BS) void k_mse(const float* __restrict__ o, const float* __restrict__ t, int nz, int ny,
                                            int nx, double inv_n, float* __restrict__ dout,
                                            double* __restrict__ partial) {
  const long nvox = (long)nz * ny * nx;
  double acc = 0.0;
  for (long v = (long)blockIdx.x * BS + threadIdx.x; v < nvox; v += (long)gridDim.x * BS) {
    const int x = (int)(v % nx);
    const int y = (int)((v / nx) % ny);
    const int z = (int)(v / ((long)nx * ny));
    const float4 a = *(const float4*)(o + v * 4), b = *(const float4*)(t + v * 4);
    // the difference of two floats is exact in double
    const double df[4] = {(double)a.x - b.x, (double)a.y - b.y, (double)a.z - b.z, (double)a.w - b.w};
    const bool un[4] = {x > 0, y > 0, z > 0, true};
    float g[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      g[c] = un[c] ? (float)(2.0 * df[c] * inv_n) : 0.f;
      if (un[c]) acc += df[c] * df[c];
    }
    *(float4*)(dout + v * 4) = float4{g[0], g[1], g[2], g[3]};
  }
  const double s = block_sum_d(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// single block: out[0] = scale * sum(partial[0..n)) in a fixed order
__global__ __launch_bounds__(BS) void k_finish_sum(const double* __restrict__ partial, int n, double scale,
                                                   int take_sqrt, double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += BS) s += partial[i];
  s = block_sum_d(s);
  if (threadIdx.x == 0) {
    s *= scale;
    out[0] = take_sqrt ? sqrt(s) : s;
  }
}

__global__ __launch_bounds__(BS) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, long n, float lr, float b1,
                                             float b2, float eps, float bc1, float bc2) {
  const long i = (long)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ------------------------------------------------ state <-> voxel tensors

struct Lay {
  int nx, ny, nz;
  long sy, sz, off[4], half;
};

// element (inside a field) of the slot of voxel (i, j, k): padded cell (i+1, j+1, k+1)
__device__ __forceinline__ long slot(const Lay& L, int i, int j, int k) {
  const long s = (long)(i + 1) + L.sy * (j + 1) + L.sz * (k + 1);
  return (s & 1) * L.half + (s >> 1);
}

__global__ __launch_bounds__(BS) void k_vel_sumsq(const double* __restrict__ b, Lay L, double* __restrict__ partial) {
  const long nvox = (long)L.nx * L.ny * L.nz;
  double acc = 0.0;
  for (long v = (long)blockIdx.x * BS + threadIdx.x; v < nvox; v += (long)gridDim.x * BS) {
    const int i = (int)(v % L.nx), j = (int)((v / L.nx) % L.ny), k = (int)(v / ((long)L.nx * L.ny));
    const long s = slot(L, i, j, k);
    // minus faces of the voxel; face 0 of each axis is a wall (not an unknown)
    if (i > 0) acc += b[L.off[0] + s] * b[L.off[0] + s];
    if (j > 0) acc += b[L.off[1] + s] * b[L.off[1] + s];
    if (k > 0) acc += b[L.off[2] + s] * b[L.off[2] + s];
  }
  const double t = block_sum_d(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(BS) void k_state_to_input(const double* __restrict__ b, Lay L,
                                                       const double* __restrict__ scale, uint16_t* __restrict__ in) {
  const long nvox = (long)L.nx * L.ny * L.nz;
  const long v = (long)blockIdx.x * BS + threadIdx.x;
  if (v >= nvox) return;
  const int i = (int)(v % L.nx), j = (int)((v / L.nx) % L.ny), k = (int)(v / ((long)L.nx * L.ny));
  const long s = slot(L, i, j, k);
  const double sc = scale[0];
  uint32_t h[3];
  const bool un[3] = {i > 0, j > 0, k > 0};
#pragma unroll
  for (int c = 0; c < 3; ++c) h[c] = (un[c] && sc > 0.0) ? d2bf(b[L.off[c] + s] / sc) : 0u;
  *(uint4*)(in + v * 8) = uint4{h[0] | (h[1] << 16), h[2], 0u, 0u};
}

__global__ __launch_bounds__(BS) void k_state_to_target(const double* __restrict__ x, Lay L,
                                                        const double* __restrict__ scale,
                                                        const float* __restrict__ sigma, float* __restrict__ t) {
  const long nvox = (long)L.nx * L.ny * L.nz;
  const long v = (long)blockIdx.x * BS + threadIdx.x;
  if (v >= nvox) return;
  const int i = (int)(v % L.nx), j = (int)((v / L.nx) % L.ny), k = (int)(v / ((long)L.nx * L.ny));
  const long s = slot(L, i, j, k);
  const double sc = scale[0];
  const bool un[4] = {i > 0, j > 0, k > 0, true};
  float o[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) o[c] = (un[c] && sc > 0.0) ? (float)(x[L.off[c] + s] / (sc * (double)sigma[c])) : 0.f;
  *(float4*)(t + v * 4) = float4{o[0], o[1], o[2], o[3]};
}

// one thread per padded slot of each field
__global__ __launch_bounds__(BS) void k_output_to_state(const float* __restrict__ out, Lay L,
                                                        const double* __restrict__ scale,
                                                        const float* __restrict__ sigma, double* __restrict__ x,
                                                        long field) {
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= 4 * field) return;
  const int f = (int)(e / field);
  const long r = e - f * field;
  const long rp = r % L.sz;  // slot within its plane
  const int K = (int)(r / L.sz), J = (int)(rp / L.sy), I = (int)(rp % L.sy);
  bool un = I >= 1 && I <= L.nx && J >= 1 && J <= L.ny && K >= 1 && K <= L.nz;
  if (f == 0) un = un && I >= 2;
  if (f == 1) un = un && J >= 2;
  if (f == 2) un = un && K >= 2;
  double val = 0.0;
  if (un) {
    const long v = ((long)(K - 1) * L.ny + (J - 1)) * L.nx + (I - 1);
    val = (double)out[v * 4 + f] * scale[0] * (double)sigma[f];
  }
  x[L.off[f] + (r & 1) * L.half + (r >> 1)] = val;
}

__global__ __launch_bounds__(BS) void k_channel_sumsq(const float* __restrict__ t, long nvox,
                                                      double* __restrict__ partial) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long v = (long)blockIdx.x * BS + threadIdx.x; v < nvox; v += (long)gridDim.x * BS) {
    const float4 a = *(const float4*)(t + v * 4);
    acc[0] += (double)a.x * a.x;
    acc[1] += (double)a.y * a.y;
    acc[2] += (double)a.z * a.z;
    acc[3] += (double)a.w * a.w;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double s = block_sum_d(acc[c]);
    if (threadIdx.x == 0) partial[(size_t)c * gridDim.x + blockIdx.x] = s;
  }
}

}  // namespace un

using namespace un;

// ===================================================================== C ABI

namespace {

constexpr int RED_BLOCKS = 1024;

inline hipStream_t S(void* s) { return (hipStream_t)s; }
inline int grid1(long n) { return (int)((n + BS - 1) / BS); }
inline bool a16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
inline int ret() { return hipGetLastError() == hipSuccess ? UNET_OK : UNET_EDEVICE; }

inline int chunk_channels(int c) { return c % 32 == 0 ? 32 : c % 16 == 0 ? 16 : c % 8 == 0 ? 8 : 0; }

inline size_t ksteps(int cc) { return (size_t)((27 * (cc / 8) + 3) / 4); }

bool src_ok(const unet_source* s) {
  if (!s || s->nz <= 0 || s->ny <= 0 || s->nx <= 0 || s->channels <= 0 || s->channels % 8) return false;
  if (!s->src0 || !a16(s->src0)) return false;
  switch (s->mode) {
    case UNET_SRC_DIRECT:
    case UNET_SRC_POOL:
      return true;
    case UNET_SRC_MASKED:
      return s->src1 && a16(s->src1);
    case UNET_SRC_CAT_UP:
      return s->src1 && a16(s->src1) && s->c_first > 0 && s->c_first % 8 == 0 && s->c_first < s->channels &&
             s->nz % 2 == 0 && s->ny % 2 == 0 && s->nx % 2 == 0;
    default:
      return false;
  }
}

Src to_src(const unet_source* s) {
  return Src{s->mode, s->nz, s->ny, s->nx, s->channels, s->c_first, s->src0, s->src1};
}

long tiles_of(const unet_source* s) {
  return (long)((s->nx + TX - 1) / TX) * ((s->ny + TY - 1) / TY) * ((s->nz + TZ - 1) / TZ);
}

template <int CC, int MODE>
int conv_ns(const Src& s, int ns, int cout, const uint4* frag, const float* bias, void* out, int relu, int f32,
            hipStream_t st, long tiles) {
  switch (ns) {
    case 1: k_conv3<CC, 1, MODE><<<tiles, BS, 0, st>>>(s, cout, frag, bias, out, relu, f32); break;
    case 2: k_conv3<CC, 2, MODE><<<tiles, BS, 0, st>>>(s, cout, frag, bias, out, relu, f32); break;
    case 3: k_conv3<CC, 3, MODE><<<tiles, BS, 0, st>>>(s, cout, frag, bias, out, relu, f32); break;
    case 4: k_conv3<CC, 4, MODE><<<tiles, BS, 0, st>>>(s, cout, frag, bias, out, relu, f32); break;
    case 6: k_conv3<CC, 6, MODE><<<tiles, BS, 0, st>>>(s, cout, frag, bias, out, relu, f32); break;
    default: return UNET_EINVAL;
  }
  return ret();
}

// one kernel per source mode: the staging then holds no registers for the others
template <int CC>
int conv_ns(const Src& s, int ns, int cout, const uint4* frag, const float* bias, void* out, int relu, int f32,
            hipStream_t st, long tiles) {
  switch (s.mode) {
    case UNET_SRC_DIRECT: return conv_ns<CC, UNET_SRC_DIRECT>(s, ns, cout, frag, bias, out, relu, f32, st, tiles);
    case UNET_SRC_POOL: return conv_ns<CC, UNET_SRC_POOL>(s, ns, cout, frag, bias, out, relu, f32, st, tiles);
    case UNET_SRC_CAT_UP: return conv_ns<CC, UNET_SRC_CAT_UP>(s, ns, cout, frag, bias, out, relu, f32, st, tiles);
    case UNET_SRC_MASKED: return conv_ns<CC, UNET_SRC_MASKED>(s, ns, cout, frag, bias, out, relu, f32, st, tiles);
    default: return UNET_EINVAL;
  }
}

// wgrad launch shape: grid.y = chunks x pair groups, grid.x = tile groups
struct WgradShape {
  int cc, nso, npg, gy, gx, tpb;
  long ntiles;
};

bool wgrad_shape(const unet_source* x, int cout, WgradShape& w) {
  w.cc = chunk_channels(x->channels);
  w.nso = cout / 16;
  if (!w.cc || cout % 16 || (w.nso != 1 && w.nso != 2 && w.nso != 4)) return false;
  const int pairs = 27 * ((w.cc + 15) / 16);
  const int ppb = 4 * (16 / w.nso);
  w.npg = (pairs + ppb - 1) / ppb;
  w.gy = (x->channels / w.cc) * w.npg;
  w.ntiles = tiles_of(x);
  long gx = 2048 / w.gy;
  if (gx < 1) gx = 1;
  if (gx > w.ntiles) gx = w.ntiles;
  w.tpb = (int)((w.ntiles + gx - 1) / gx);
  w.gx = (int)((w.ntiles + w.tpb - 1) / w.tpb);
  return true;
}

Lay to_lay(const unet_state_layout* L) {
  return Lay{L->nx, L->ny, L->nz, (long)L->sy, (long)L->sz,
             {(long)L->off[0], (long)L->off[1], (long)L->off[2], (long)L->off[3]}, (long)L->half};
}

bool lay_ok(const unet_state_layout* L) {
  return L && L->nx > 0 && L->ny > 0 && L->nz > 0 && L->sy >= L->nx + 2 && L->sz >= L->sy * (L->ny + 2) &&
         2 * L->half >= L->sz * (L->nz + 2);
}

}  // namespace

extern "C" {

size_t unet_packed_elems(int32_t cin, int32_t cout, int32_t transpose) {
  const int ci = transpose ? cout : cin, co = transpose ? cin : cout;
  const int cc = chunk_channels(ci);
  if (!cc || co % 16 || co <= 0) return 0;
  return (size_t)(ci / cc) * ksteps(cc) * (co / 16) * 64 * 8;
}

int unet_pack_weights(const float* w, int32_t cin, int32_t cout, int32_t transpose, uint16_t* frag, void* stream) {
  const size_t n = unet_packed_elems(cin, cout, transpose);
  if (!n || !w || !frag || !a16(frag)) return UNET_EINVAL;
  const int cc = chunk_channels(transpose ? cout : cin);
  const long n4 = (long)(n / 8);
  k_pack<<<grid1(n4), BS, 0, S(stream)>>>(w, cin, cout, transpose ? 1 : 0, cc, (uint4*)frag, n4);
  return ret();
}

int unet_conv3(const unet_source* src, int32_t cout, const uint16_t* frag, const float* bias, int32_t relu,
               int32_t out_f32, void* out, void* stream) {
  if (!src_ok(src)) return UNET_EINVAL;
  if (!frag || !a16(frag) || !out || cout <= 0 || cout % 16) return UNET_EINVAL;
  const int cc = chunk_channels(src->channels);
  const int ns = cout / 16;
  if (!cc || (ns != 1 && ns != 2 && ns != 3 && ns != 4 && ns != 6)) return UNET_EINVAL;
  const Src s = to_src(src);
  const long tiles = tiles_of(src);
  const uint4* f = (const uint4*)frag;
  switch (cc) {
    case 8: return conv_ns<8>(s, ns, cout, f, bias, out, relu, out_f32, S(stream), tiles);
    case 16: return conv_ns<16>(s, ns, cout, f, bias, out, relu, out_f32, S(stream), tiles);
    default: return conv_ns<32>(s, ns, cout, f, bias, out, relu, out_f32, S(stream), tiles);
  }
}

size_t unet_wgrad_workspace_bytes(const unet_source* x, int32_t cout) {
  WgradShape w;
  if (!x || x->channels <= 0 || x->nx <= 0 || x->ny <= 0 || x->nz <= 0 || !wgrad_shape(x, cout, w)) return 0;
  return sizeof(float) * ((size_t)w.gx * 27 * x->channels * cout + (size_t)w.gx * cout);
}

int unet_conv3_wgrad(const unet_source* x, const unet_source* dz, int32_t cout, float* workspace,
                     size_t workspace_bytes, float* dw, float* db, void* stream) {
  if (!src_ok(x) || !src_ok(dz) || !dw || !db || !workspace) return UNET_EINVAL;
  if (dz->channels != cout || dz->nx != x->nx || dz->ny != x->ny || dz->nz != x->nz) return UNET_EINVAL;
  if (dz->mode != UNET_SRC_DIRECT && dz->mode != UNET_SRC_MASKED) return UNET_EINVAL;
  WgradShape w;
  if (!wgrad_shape(x, cout, w)) return UNET_EINVAL;
  if (workspace_bytes < unet_wgrad_workspace_bytes(x, cout)) return UNET_EINVAL;
  const long nw = 27L * x->channels * cout;
  float* part = workspace;
  float* bpart = workspace + (size_t)w.gx * nw;
  const Src xs = to_src(x), ds = to_src(dz);
  const dim3 grid(w.gx, w.gy);
  hipStream_t st = S(stream);
#define WG(CC, NSO) k_wgrad<CC, NSO><<<grid, BS, 0, st>>>(xs, ds, (int)w.ntiles, w.tpb, w.npg, part, bpart)
  if (w.cc == 8) {
    if (w.nso == 1) WG(8, 1); else if (w.nso == 2) WG(8, 2); else WG(8, 4);
  } else if (w.cc == 16) {
    if (w.nso == 1) WG(16, 1); else if (w.nso == 2) WG(16, 2); else WG(16, 4);
  } else {
    if (w.nso == 1) WG(32, 1); else if (w.nso == 2) WG(32, 2); else WG(32, 4);
  }
#undef WG
  k_sum_rows<<<grid1(nw), BS, 0, st>>>(part, w.gx, nw, nw, dw);
  k_sum_rows<<<grid1(cout), BS, 0, st>>>(bpart, w.gx, cout, cout, db);
  return ret();
}

int unet_up_grad(const uint16_t* fine, int32_t cf, int32_t coff, int32_t c, int32_t nz, int32_t ny, int32_t nx,
                 uint16_t* coarse, void* stream) {
  if (!fine || !coarse || c <= 0 || coff < 0 || coff + c > cf || nz <= 0 || ny <= 0 || nx <= 0) return UNET_EINVAL;
  const long n = (long)nz * ny * nx * c;
  k_up_grad<<<grid1(n), BS, 0, S(stream)>>>(fine, cf, coff, c, nz, ny, nx, coarse);
  return ret();
}

int unet_skip_grad(const uint16_t* fine, int32_t cf, int32_t coff, const uint16_t* pooled, int32_t c, int32_t nz,
                   int32_t ny, int32_t nx, uint16_t* out, void* stream) {
  if (!fine || !pooled || !out || c <= 0 || coff < 0 || coff + c > cf || nz <= 0 || ny <= 0 || nx <= 0 || nz % 2 ||
      ny % 2 || nx % 2)
    return UNET_EINVAL;
  const long n = (long)nz * ny * nx * c;
  k_skip_grad<<<grid1(n), BS, 0, S(stream)>>>(fine, cf, coff, pooled, c, nz, ny, nx, out);
  return ret();
}

int unet_head_forward(const uint16_t* d, const float* hw, const float* hb, float* out, int64_t nvox, void* stream) {
  if (!d || !hw || !hb || !out || nvox <= 0 || !a16(d) || !a16(out)) return UNET_EINVAL;
  k_head_fwd<<<grid1(nvox), BS, 0, S(stream)>>>(d, hw, hb, out, nvox);
  return ret();
}

static long head_blocks(int64_t nvox) {
  long nb = (nvox + 4095) / 4096;
  return nb < 1 ? 1 : nb;
}

size_t unet_head_workspace_bytes(int64_t nvox) { return sizeof(float) * 68 * (size_t)head_blocks(nvox); }

int unet_head_backward(const uint16_t* d, const float* dout, const float* hw, uint16_t* dd, float* workspace,
                       size_t workspace_bytes, float* dhw, float* dhb, int64_t nvox, void* stream) {
  if (!d || !dout || !hw || !dd || !workspace || !dhw || !dhb || nvox <= 0) return UNET_EINVAL;
  if (!a16(d) || !a16(dout) || !a16(dd) || workspace_bytes < unet_head_workspace_bytes(nvox)) return UNET_EINVAL;
  const long nb = head_blocks(nvox);
  hipStream_t st = S(stream);
  k_head_bwd<<<nb, BS, 0, st>>>(d, dout, hw, dd, workspace, nvox, 4096);
  // partial is [nb][68]: dhw = columns 0..63, dhb = columns 64..67
  k_sum_rows<<<1, BS, 0, st>>>(workspace, (int)nb, 68, 64, dhw);
  k_sum_rows<<<1, BS, 0, st>>>(workspace + 64, (int)nb, 68, 4, dhb);
  return ret();
}

size_t unet_mse_workspace_bytes(int64_t) { return sizeof(double) * RED_BLOCKS; }

int unet_mse(const float* out, const float* target, int32_t nz, int32_t ny, int32_t nx, float* dout, void* workspace,
             size_t workspace_bytes, double* loss, void* stream) {
  if (!out || !target || !dout || !workspace || !loss || nz <= 0 || ny <= 0 || nx <= 0) return UNET_EINVAL;
  if (!a16(out) || !a16(target) || !a16(dout) || workspace_bytes < unet_mse_workspace_bytes(0)) return UNET_EINVAL;
  const double n = 4.0 * nz * ny * nx - ((double)ny * nz + (double)nx * nz + (double)nx * ny);
  hipStream_t st = S(stream);
  k_mse<<<RED_BLOCKS, BS, 0, st>>>(out, target, nz, ny, nx, 1.0 / n, dout, (double*)workspace);
  k_finish_sum<<<1, BS, 0, st>>>((const double*)workspace, RED_BLOCKS, 1.0 / n, 0, loss);
  return ret();
}

int unet_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2, float eps,
              int32_t step, void* stream) {
  if (!p || !g || !m || !v || n <= 0 || step < 1) return UNET_EINVAL;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  k_adam<<<grid1(n), BS, 0, S(stream)>>>(p, g, m, v, n, lr, beta1, beta2, eps, bc1, bc2);
  return ret();
}

size_t unet_reduce_workspace_bytes(const unet_state_layout*) { return sizeof(double) * 4 * RED_BLOCKS; }

int unet_state_scale(const double* b, const unet_state_layout* L, void* workspace, size_t workspace_bytes,
                     double* scale, void* stream) {
  if (!b || !lay_ok(L) || !workspace || !scale || workspace_bytes < unet_reduce_workspace_bytes(L))
    return UNET_EINVAL;
  const double nu = (double)(L->nx - 1) * L->ny * L->nz + (double)L->nx * (L->ny - 1) * L->nz +
                    (double)L->nx * L->ny * (L->nz - 1);
  if (nu <= 0) return UNET_EINVAL;
  hipStream_t st = S(stream);
  k_vel_sumsq<<<RED_BLOCKS, BS, 0, st>>>(b, to_lay(L), (double*)workspace);
  k_finish_sum<<<1, BS, 0, st>>>((const double*)workspace, RED_BLOCKS, 1.0 / nu, 1, scale);
  return ret();
}

int unet_state_to_input(const double* b, const unet_state_layout* L, const double* scale, uint16_t* in,
                        void* stream) {
  if (!b || !lay_ok(L) || !scale || !in || !a16(in)) return UNET_EINVAL;
  const long nvox = (long)L->nx * L->ny * L->nz;
  k_state_to_input<<<grid1(nvox), BS, 0, S(stream)>>>(b, to_lay(L), scale, in);
  return ret();
}

int unet_state_to_target(const double* x, const unet_state_layout* L, const double* scale, const float* sigma,
                         float* target, void* stream) {
  if (!x || !lay_ok(L) || !scale || !sigma || !target || !a16(target)) return UNET_EINVAL;
  const long nvox = (long)L->nx * L->ny * L->nz;
  k_state_to_target<<<grid1(nvox), BS, 0, S(stream)>>>(x, to_lay(L), scale, sigma, target);
  return ret();
}

int unet_output_to_state(const float* out, const unet_state_layout* L, const double* scale, const float* sigma,
                         double* x, void* stream) {
  if (!out || !lay_ok(L) || !scale || !sigma || !x) return UNET_EINVAL;
  const long field = 2 * L->half;
  for (int f = 1; f < 4; ++f)
    if (L->off[f] - L->off[f - 1] < field) return UNET_EINVAL;
  k_output_to_state<<<grid1(4 * field), BS, 0, S(stream)>>>(out, to_lay(L), scale, sigma, x, field);
  return ret();
}

int unet_channel_sumsq(const float* t, int64_t nvox, void* workspace, size_t workspace_bytes, double* sumsq,
                       void* stream) {
  if (!t || nvox <= 0 || !workspace || !sumsq || !a16(t) || workspace_bytes < sizeof(double) * 4 * RED_BLOCKS)
    return UNET_EINVAL;
  hipStream_t st = S(stream);
  double* part = (double*)workspace;
  k_channel_sumsq<<<RED_BLOCKS, BS, 0, st>>>(t, nvox, part);
  for (int c = 0; c < 4; ++c) k_finish_sum<<<1, BS, 0, st>>>(part + (size_t)c * RED_BLOCKS, RED_BLOCKS, 1.0, 0, sumsq + c);
  return ret();
}

}  // extern "C"
