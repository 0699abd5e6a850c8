/*
 * lbm_nn.h - C ABI of the learned warm start: BF16 MFMA kernels for a small
 * 3D convolutional network that maps a solid mask (and the driving force
 * direction) to the steady velocity field of the lattice Boltzmann solver.
 * The network is not part of the paper; it provides initial states for the
 * solver, which still decides when the steady state is reached (it runs from the
 * predicted equilibrium until its own residual criterion is met).
 *
 * Conventions:
 *  - Tensors are channels-last (NDHWC): element (b, z, y, x, c) at
 *    (((b*D + z)*H + y)*W + x)*C + c.  bf16 tensors are uint16_t bit
 *    patterns (IEEE binary32 upper half, round-to-nearest-even on
 *    conversion); accumulation is float32 in the MFMA units
 *    (v_mfma_f32_16x16x16_bf16).
 *  - Convolution weights are [taps][c_out][c_in] bf16, taps = 27
 *    (3x3x3, index (kz*3 + ky)*3 + kx, offsets -1..1) or 1 (1x1x1).
 *    Padding is circular (the lattice is periodic).  With stride 2 the
 *    output voxel p reads input voxels 2p + k - 1.
 *  - Channel counts c_in and c_out are multiples of 16 (pad with zero
 *    channels/weights), (c_in/16)*(c_out/16) <= 32; the voxel counts of
 *    the input and output grids are multiples of 16.
 *  - All device pointers are caller-owned; every call only enqueues work on
 *    `stream` (a hipStream_t) and returns 0 or a negative code
 *    (-1 invalid argument, -4 HIP error; see lbm_last_error()).
 *  - Reductions (weight gradients, bias gradients, the loss) are split
 *    into fixed chunks and summed in a fixed order: results are
 *    deterministic run to run.
 */
#ifndef LBM_NN_MI355X_H
#define LBM_NN_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t batch;
  int32_t d, h, w;     /* input grid                                       */
  int32_t c_in;        /* input channels, multiple of 16                   */
  int32_t c_out;       /* output channels computed, multiple of 16 (<= 128)*/
  int32_t c_store;     /* output channels written (<= c_out), forward only */
  int32_t stride;      /* 1 or 2 (taps = 27 only); output grid = input/s   */
  int32_t taps;        /* 27 or 1                                          */
  int32_t act;         /* 0: none, 1: leaky ReLU                           */
  float slope;         /* leaky ReLU slope for negative inputs             */
  int32_t out_f32;     /* forward output type: 1 float32, 0 bf16          */
} nn_conv_desc;

/* y = act(conv(x, w) + bias).  x: [B][D][H][W][c_in] bf16; w: [taps][c_out]
 * [c_in] bf16; bias: c_out float32 or NULL; y: [B][D/s][H/s][W/s][c_store],
 * bf16 or float32. */
int nn_conv3d_fwd(const nn_conv_desc* d, const uint16_t* x, const uint16_t* w,
                  const float* bias, void* y, void* stream);

/* nn_conv3d_fwd of the channel concatenation nn_up_concat would form, read
 * straight from its two parts without forming it (the decoder's first
 * layer at inference).  Input channels 0 .. c_coarse-1 are coarse[b, z/2,
 * y/2, x/2] ([B][D/2][H/2][W/2][c_coarse] bf16), channels c_coarse ..
 * c_in-1 are skip[b, z, y, x] ([B][D][H][W][c_in - c_coarse] bf16); (D, H,
 * W) in d is the fine grid.  Stride 1 and 27 taps only; W a multiple of 16,
 * H and D of 4; c_coarse a multiple of 8 below c_in.  Else returns -1 and
 * nothing is launched; the result equals nn_up_concat followed by
 * nn_conv3d_fwd bit for bit. */
int nn_conv3d_fwd_upcat(const nn_conv_desc* d, const uint16_t* coarse, int32_t c_coarse,
                        const uint16_t* skip, const uint16_t* w, const float* bias, void* y,
                        void* stream);

/* Data gradient: dx (+)= conv^T(dy, w), the gradient with respect to the
 * input of the convolution given dy, the gradient with respect to its
 * pre-activation output ([B][D/s][H/s][W/s][c_out] bf16).  dx: [B][D][H][W]
 * [c_in] float32; accumulate != 0 adds to dx.  w_t: workspace of
 * taps*c_in*c_out bf16, left holding the transposed weights (for stride-1
 * 3x3x3 layers on grids with W % 16, H % 4 and D % 4 == 0, dy and w_t
 * 16-byte aligned, also mirrored through the centre tap); its contents are
 * scratch, not part of the result. */
int nn_conv3d_dgrad(const nn_conv_desc* d, const uint16_t* dy, const uint16_t* w,
                    uint16_t* w_t, float* dx, int32_t accumulate, void* stream);

/* Weight and bias gradients: dw[taps][c_out][c_in] = sum over output voxels
 * of dy (x) x at the tap offset; db[c_out] = sum of dy (db may be NULL).
 * Both float32, overwritten.  workspace: nn_conv3d_wgrad_workspace() bytes. */
int nn_conv3d_wgrad(const nn_conv_desc* d, const uint16_t* x, const uint16_t* dy, float* dw,
                    float* db, float* workspace, void* stream);
int64_t nn_conv3d_wgrad_workspace(const nn_conv_desc* d);

/* dy_pre = bf16(dx * (y > 0 ? 1 : slope)) for n elements (y: the bf16
 * leaky ReLU output, whose sign is that of its input). */
int nn_lrelu_bwd(const float* dx, const uint16_t* y, uint16_t* dy_pre, int64_t n, float slope,
                 void* stream);

/* cat[b,z,y,x] = (coarse[b,z/2,y/2,x/2][0..c1), skip[b,z,y,x][0..c2)):
 * nearest-neighbour upsampling by 2 and channel concatenation; (d, h, w)
 * is the fine grid. */
int nn_up_concat(const uint16_t* coarse, const uint16_t* skip, uint16_t* cat, int32_t batch,
                 int32_t d, int32_t h, int32_t w, int32_t c1, int32_t c2, void* stream);

/* Backward of nn_up_concat: dcoarse = sum over the 8 fine children of the
 * first c1 channels of dcat; dskip = the last c2 channels (both
 * overwritten). */
int nn_split_down(const float* dcat, float* dcoarse, float* dskip, int32_t batch, int32_t d,
                  int32_t h, int32_t w, int32_t c1, int32_t c2, void* stream);

/* Masked mean squared error over fluid voxels (mask == 0) of pred and
 * target ([n][3] float32): loss (float32, one value, device) and its
 * gradient written as the bf16 pre-activation gradient of the 1x1x1 head,
 * dy[n][16] (channels 3..15 zero).  workspace: 4096 floats. */
int nn_masked_mse(const float* pred, const float* target, const uint8_t* mask, int64_t n,
                  uint16_t* dy, float* loss, float* workspace, void* stream);

/* nn_masked_mse without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc): the same kernels and results
 * bit for bit, on a 16 KiB device array inside the library (one per GPU,
 * held until the process ends) instead of the caller's workspace.  It
 * allocates nothing.  Call it with the stream's device current.
 * n <= 2^31 - 1 voxels, else -1 with a message.  Every call on one GPU
 * uses that GPU's array: calls that overlap on one GPU (concurrent
 * streams or host threads) race, and the caller must order them. */
int nn_masked_mse_noalloc(const float* pred, const float* target, const uint8_t* mask,
                          int64_t n, uint16_t* dy, float* loss, void* stream);

/* Adam step (Kingma and Ba) on float32 master weights; writes the bf16
 * copy used by the kernels.  t >= 1 is the step number.  The
 * hyper-parameters are double: the complements 1 - beta and the bias
 * corrections 1 - beta^t are formed in double on the host, then the update
 * runs in float32.  Requires 0 <= beta < 1 and eps > 0, else -1. */
int nn_adam_step(float* param, const float* grad, float* m, float* v, uint16_t* param_bf16,
                 int64_t n, double lr, double beta1, double beta2, double eps, int32_t t,
                 void* stream);

/* Network input from a solid mask: x[n][c_pad] bf16 with channel 0 = solid
 * (1/0), channel 1 = fluid (1/0), other channels zero. */
int nn_prepare_input(const uint8_t* mask, uint16_t* x, int64_t n, int32_t c_pad, void* stream);

/* Network input with distance features, for `batch` periodic cubes of
 * edge n (mask and x voxel-major, x fastest): x[i][c_pad] bf16 with
 * channel 0 = solid, 1 = fluid, 2 = d/dmax, 3 = (d/dmax)^2, other channels
 * zero, where d is the distance to the nearest solid voxel (chamfer
 * distance on the 26-neighbourhood with steps 1, sqrt 2, sqrt 3, periodic
 * wrap), clamped at dmax.  In Stokes flow through a pore the velocity
 * grows with the squared distance from the wall, which a few 3x3x3
 * convolutions cannot measure across a pore.  work: 2*batch*n^3 floats.
 * c_pad >= 4, 1 <= dmax <= 64, else -1. */
int nn_prepare_input_dist(const uint8_t* mask, uint16_t* x, int32_t batch, int32_t n,
                          int32_t c_pad, float dmax, float* work, void* stream);

/* Network labels from solver velocities: out[i][a] = scale * u[a*n + i]
 * on fluid voxels, 0 on solids (float32 [n][3]; u float64 [3][n]): the
 * inverse of nn_velocity_out. */
int nn_velocity_labels(const double* u, const uint8_t* mask, double scale, float* out, int64_t n,
                       void* stream);

/* Velocity for the solver: u[a*n + i] = scale * pred[i][a] on fluid
 * voxels, 0 on solids (float64, component-major [3][n]). */
int nn_velocity_out(const float* pred, const uint8_t* mask, double scale, double* u, int64_t n,
                    void* stream);

/* float32 -> bf16 (round to nearest even), n elements. */
int nn_to_bf16(const float* src, uint16_t* dst, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_NN_MI355X_H */
