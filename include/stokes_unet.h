/*
 * Learned warm start for MG-SQMR on gfx950: the kernels of a small 3D U-Net
 * that maps the forcing of a Stokes problem to an initial guess x0 for SQMR.
 *
 * Alg. 4 (SQMR) accepts any initial guess; the solve itself is unchanged.
 * The network (3 levels, 16/32/64 channels, 3x3x3 convolutions, ReLU, 2x2x2
 * average pooling down, nearest-neighbour upsampling with skip
 * concatenation up, a 1x1x1 head to 4 outputs) is assembled from the calls
 * below; its definition, layer by layer, is in the package's unet module.
 *
 * Conventions shared by every call:
 *   - Voxel tensors are [z][y][x][c]: x fastest, channel innermost, dense.
 *     Activations, their gradients and packed weights are bfloat16, stored as
 *     uint16_t bit patterns, rounded to nearest even.  Master weights, biases,
 *     gradients of parameters, head outputs and loss gradients are float.
 *   - Convolutions and products accumulate in float on the matrix cores
 *     (v_mfma_f32_16x16x32_bf16).
 *   - Every pointer is a device pointer unless stated otherwise; the caller
 *     owns all memory.  The library allocates nothing on the device.
 *   - Each call enqueues its kernels on `stream` (a hipStream_t; NULL = the
 *     null stream) and returns without waiting.
 *   - Return value: UNET_OK, UNET_EINVAL (bad size, channel count, null or
 *     misaligned pointer, workspace too small; nothing is enqueued) or
 *     UNET_EDEVICE (a HIP launch error).
 */
#ifndef STOKES_UNET_H
#define STOKES_UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { UNET_OK = 0, UNET_EINVAL = 1, UNET_EDEVICE = 5 };

/* How a convolution reads its (virtual) input tensor of `channels` channels
 * on the nz x ny x nx grid it runs on. */
enum {
  UNET_SRC_DIRECT = 0, /* src0 is that tensor */
  UNET_SRC_POOL = 1,   /* src0 is 2x finer per axis; each input value is the mean of 8 children, rounded */
  UNET_SRC_CAT_UP = 2, /* channels [0, c_first) from the 2x coarser src0 (nearest neighbour),
                          channels [c_first, channels) from src1 on the grid itself */
  UNET_SRC_MASKED = 3  /* src0 where the gate src1 is > 0, else 0 (the ReLU derivative) */
};

typedef struct {
  int32_t mode;         /* UNET_SRC_* */
  int32_t nz, ny, nx;   /* grid the layer runs on (its output grid) */
  int32_t channels;     /* channels of the input the layer sees; a multiple of 8 */
  int32_t c_first;      /* UNET_SRC_CAT_UP only: channels from src0; a multiple of 8 */
  const uint16_t* src0; /* 16-byte aligned */
  const uint16_t* src1; /* CAT_UP / MASKED only, 16-byte aligned */
} unet_source;

/* Layout of a Stokes state vector (stokes_layout_t in stokes_mgsqmr.h): field
 * f (u_x, u_y, u_z, p) of padded cell (I, J, K), slot s = I + sy J + sz K, is
 * element off[f] + (s & 1) * half + (s >> 1); half = field / 2. */
typedef struct {
  int32_t nx, ny, nz;
  int64_t sy, sz;
  int64_t off[4];
  int64_t half;
} unet_state_layout;

/* ---------------------------------------------------------------- weights */

/* Elements (uint16_t) of the packed fragments of one 3x3x3 layer with
 * cin -> cout channels (both multiples of 8; cout, or cin when transposed,
 * a multiple of 16).  transpose = 1 packs the weights of the input-gradient
 * convolution: taps mirrored, input and output channels swapped. */
size_t unet_packed_elems(int32_t cin, int32_t cout, int32_t transpose);

/* Round the float master weights w[27][cin][cout] (tap t = 9(dz+1) + 3(dy+1)
 * + (dx+1)) to bfloat16 and lay them out in the order in which the
 * convolution kernel's lanes read them. */
int unet_pack_weights(const float* w, int32_t cin, int32_t cout, int32_t transpose, uint16_t* frag,
                      void* stream);

/* ------------------------------------------------------------ convolution */

/* out[v][co] = act(bias[co] + sum_t sum_ci in[v + tap_t][ci] * w[t][ci][co]),
 * zero padding at the grid edges.  act = ReLU when relu != 0.  The result is
 * stored as bfloat16 (out_f32 = 0) or float (out_f32 = 1); bias may be NULL.
 * With `frag` packed by unet_pack_weights(transpose = 1) and src in
 * UNET_SRC_MASKED mode (gradient, activation) this is the input gradient of a
 * layer: d in[v] = sum_t dz[v - tap_t] w[t]^T. */
int unet_conv3(const unet_source* src, int32_t cout, const uint16_t* frag, const float* bias, int32_t relu,
               int32_t out_f32, void* out, void* stream);

/* Bytes of float workspace unet_conv3_wgrad needs for this layer. */
size_t unet_wgrad_workspace_bytes(const unet_source* x, int32_t cout);

/* Parameter gradients of a 3x3x3 layer: dw[t][ci][co] = sum_v x[v + tap_t][ci] dz[v][co]
 * and db[co] = sum_v dz[v][co], where x is the layer input (read as in the
 * forward pass) and dz is read through `dz` (normally UNET_SRC_MASKED of the
 * output gradient gated by the output).  Sums run in a fixed order: the result
 * does not depend on scheduling. */
int unet_conv3_wgrad(const unet_source* x, const unet_source* dz, int32_t cout, float* workspace,
                     size_t workspace_bytes, float* dw, float* db, void* stream);

/* ------------------------------------------------ gradients at skip links */

/* Adjoint of nearest-neighbour upsampling on channels [coff, coff+c) of a
 * fine tensor with cf channels on the (2nz, 2ny, 2nx) grid:
 * coarse[v][c] = bf16(sum over the 8 children of fine[child][coff + c]). */
int unet_up_grad(const uint16_t* fine, int32_t cf, int32_t coff, int32_t c, int32_t nz, int32_t ny, int32_t nx,
                 uint16_t* coarse, void* stream);

/* Gradient of a tensor read both as a skip input and through pooling:
 * out[v][c] = bf16(fine[v][coff + c] + pooled[parent(v)][c] / 8), fine with
 * cf channels on the nz x ny x nx grid (all even), pooled with c channels. */
int unet_skip_grad(const uint16_t* fine, int32_t cf, int32_t coff, const uint16_t* pooled, int32_t c, int32_t nz,
                   int32_t ny, int32_t nx, uint16_t* out, void* stream);

/* ------------------------------------------------------------------- head */

/* out[v][co] = hb[co] + sum_ci d[v][ci] * bf16(hw[ci][co]); 16 -> 4 channels. */
int unet_head_forward(const uint16_t* d, const float* hw, const float* hb, float* out, int64_t nvox, void* stream);

/* Bytes of workspace unet_head_backward needs. */
size_t unet_head_workspace_bytes(int64_t nvox);

/* dd[v][ci] = bf16(sum_co dout[v][co] bf16(hw[ci][co])), dhw = sum_v d[v]^T dout[v],
 * dhb = sum_v dout[v], in a fixed order. */
int unet_head_backward(const uint16_t* d, const float* dout, const float* hw, uint16_t* dd, float* workspace,
                       size_t workspace_bytes, float* dhw, float* dhb, int64_t nvox, void* stream);

/* ------------------------------------------------------- loss, optimizer */

/* Bytes of workspace unet_mse needs. */
size_t unet_mse_workspace_bytes(int64_t nvox);

/* Mean squared error over the unknowns of a 4-channel voxel state (channel c
 * < 3 is not an unknown at the minus wall of its axis): loss = sum (o-t)^2 / n,
 * dout = 2 (o - t) / n on unknowns and 0 elsewhere.  *loss (device double). */
int unet_mse(const float* out, const float* target, int32_t nz, int32_t ny, int32_t nx, float* dout,
             void* workspace, size_t workspace_bytes, double* loss, void* stream);

/* One Adam step (Kingma & Ba 2015, Algorithm 1) on n float parameters:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
int unet_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2, float eps,
              int32_t step, void* stream);

/* ------------------------------------------- state vector <-> voxel tensors */

/* Bytes of workspace the reductions below need. */
size_t unet_reduce_workspace_bytes(const unet_state_layout* L);

/* *scale = sqrt(mean of b^2 over the velocity unknowns) (device double); a
 * zero forcing gives scale 0 and the conversions below then produce zeros. */
int unet_state_scale(const double* b, const unet_state_layout* L, void* workspace, size_t workspace_bytes,
                     double* scale, void* stream);

/* Network input [nz][ny][nx][8]: channels 0..2 = b of the voxel's minus-face
 * u_x, u_y, u_z divided by *scale, channels 3..7 = 0. */
int unet_state_to_input(const double* b, const unet_state_layout* L, const double* scale, uint16_t* in,
                        void* stream);

/* Training target [nz][ny][nx][4]: x of the voxel's minus faces and cell
 * centre divided by (*scale * sigma[c]), sigma a device float[4]. */
int unet_state_to_target(const double* x, const unet_state_layout* L, const double* scale, const float* sigma,
                         float* target, void* stream);

/* Initial guess: every slot of the state vector x is written, unknowns with
 * out[v][c] * *scale * sigma[c], all other slots with 0. */
int unet_output_to_state(const float* out, const unet_state_layout* L, const double* scale, const float* sigma,
                         double* x, void* stream);

/* sumsq[c] = sum over voxels of t[v][c]^2 for a 4-channel float tensor (device double[4]). */
int unet_channel_sumsq(const float* t, int64_t nvox, void* workspace, size_t workspace_bytes, double* sumsq,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif
