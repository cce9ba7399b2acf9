/*
 * wsn.h -- C ABI of the learned warm start of the iterative DVM solver
 * (libdvm_hip.so).  A small 3D U-Net maps (log10 Kn, lid speed, wall mask,
 * cell position) on the cell grid to the macroscopic fields (rho, U, T) of the converged
 * solution; its output seeds the solver's initial equilibrium, which the
 * paper builds from the initial macroscopic fields (Sec. 2.2).  The network
 * is not part of the paper;
 * it is the learned warm start of this implementation.
 *
 * Network: 3 levels, base width B (32): per level two 3x3x3 convolutions
 * with ReLU, 2x2x2 average pooling down, nearest x2 upsampling up with the
 * skip activation concatenated after the upsampled channels, a final 1x1x1
 * convolution.  Convolutions run on the matrix cores (MFMA, BF16 operands,
 * FP32 accumulation); master weights, gradients, Adam state and the loss
 * are FP32.
 *
 * Conventions
 *   - Device pointers are marked d_; they must stay valid for the call and
 *     be 16-byte aligned.  Grids are [D][H][W] with W fastest; D, H, W must
 *     be multiples of 4 and at most the sizes given to wsn_create.
 *   - Parameter vector (FP32, host): for each convolution in order
 *     e1a e1b e2a e2b b1 b2 d2a d2b d1a d1b out: W[tap][c_out][c_in]
 *     (tap = 9(dz+1) + 3(dy+1) + (dx+1); 1 tap for "out") then b[c_out].
 *   - The library allocates its device memory in wsn_create (weights,
 *     optimiser state, activations for the largest grid) and frees it in
 *     wsn_destroy.  All work is issued on the given HIP stream.
 *   - base is a multiple of 8 in [8, 64].
 *   - Every call returns 0 on success, -1 on a bad argument, -4 on a HIP
 *     error; wsn_last_error() describes the failure.
 *   - The number of levels is fixed at 3; wsn_create takes the channel
 *     counts, the base width and the largest grid (where the planned
 *     interface took levels and base).
 */
#ifndef WSN_H
#define WSN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wsn_ctx wsn_ctx;

/* cin input channels (6 for the cavity warm start), cout outputs (5), base
   width (32), largest grid. */
int wsn_create(int cin, int cout, int base, int max_d, int max_h, int max_w, void* hip_stream,
               wsn_ctx** out);
size_t wsn_num_params(const wsn_ctx* ctx);
int wsn_set_params(wsn_ctx* ctx, const float* host_params);
int wsn_get_params(wsn_ctx* ctx, float* host_params);
int wsn_get_grads(wsn_ctx* ctx, float* host_grads);

/* Forward pass: d_input [D][H][W][cin] FP32 -> d_output [D][H][W][cout] FP32. */
int wsn_forward(wsn_ctx* ctx, const float* d_input, int D, int H, int W, float* d_output);

/* Backward of the masked mean-squared error after wsn_forward on the same
   input: L = sum over cells with d_mask != 0 and channels of (y - t)^2
   divided by (cells in mask x cout).  Accumulates dL/dparams into the
   gradient buffer (scaled by weight) and adds weight * L to *host_loss. */
int wsn_backward_mse(wsn_ctx* ctx, const float* d_target, const float* d_mask, float weight,
                     double* host_loss);

int wsn_zero_grad(wsn_ctx* ctx);

/* One Adam step (bias-corrected, step counter kept inside). */
int wsn_adam_step(wsn_ctx* ctx, float lr, float beta1, float beta2, float eps);

/* One training step over a batch of n grids: zero the gradient, forward and
   masked-MSE backward of every item with weight 1/n (the batch's mean
   loss), then one Adam step with learning rate lr (beta1 0.9, beta2 0.999,
   eps 1e-8).  d_inputs[i] [D][H][W][cin], d_targets[i] [D][H][W][cout],
   d_masks[i] [D][H][W] on the device, dims[3 i .. 3 i + 2] = (D, H, W) of
   item i (host).  *host_loss (nullable) = the batch's mean loss before the
   step. */
int wsn_train_step(wsn_ctx* ctx, int n, const float* const* d_inputs, const float* const* d_targets,
                   const float* const* d_masks, const int* dims, float lr, double* host_loss);

/* Parameters and optimiser state (Adam moments and step count) to and from
   a file: magic "WSNET001", int32 cin, cout, base, step, uint64 parameter
   count, then the FP32 parameters, first and second moments.  wsn_load
   refuses (-1) a file of another network shape. */
int wsn_save(wsn_ctx* ctx, const char* path);
int wsn_load(wsn_ctx* ctx, const char* path);

/* Kernel-level checks for the tests: one 3x3x3 (taps = 27) or 1x1x1 (taps =
   1) convolution on BF16-rounded FP32 host arrays, through the same kernels
   the network uses.  x [V][ci], w [taps][co][ci], b [co] (nullable),
   gy [V][co]; outputs y [V][co] (forward, FP32 accumulate), gx [V][ci]
   (input gradient), gw [taps][co][ci] (weight gradient), gb [co]. */
int wsn_test_conv(int D, int H, int W, int ci, int co, int taps, const float* x, const float* w,
                  const float* b, const float* gy, float* y, float* gx, float* gw, float* gb);

/* One 16x16x32 BF16 MFMA tile: a [16][32], b [32][16] -> c [16][16] (FP32). */
int wsn_selftest_mfma(const float* a, const float* b, float* c);

const char* wsn_last_error(void);
void wsn_destroy(wsn_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* WSN_H */
