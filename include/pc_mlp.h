/*
 * pc_mlp.h -- C ABI of the learned closure network (gfx950 matrix cores).
 *
 * Section IV of the paper (Boeuf) closes the quasi-neutral fluid equations
 * (3)-(4) with drift-diffusion electron and energy fluxes, eqs. (12)-(13),
 * whose coefficients come from 0D Boltzmann tables.  This library's closure
 * network predicts the two fluxes from five local moments instead: a
 * multilayer perceptron 5 -> 64 -> 64 -> 64 -> 2 with tanh hidden units
 * (8,834 parameters), trained by mean squared error with Adam.
 *
 * Arithmetic: BF16 operands (inputs, weights, hidden activations and
 * back-propagated gradients are rounded to BF16, nearest-even) with FP32
 * accumulation on the matrix cores; biases, outputs, the loss, gradients and
 * the Adam state are FP32.  Inputs and targets are used as given (the caller
 * normalises them).
 *
 * Memory: every pointer is a device pointer owned by the caller.
 *  - master: float[PC_MLP_PARAMS], flat, row-major W[in][out]:
 *      W1 (5x64), b1 (64), W2 (64x64), b2, W3 (64x64), b3, W4 (64x2), b4 (2)
 *  - packed: pc_mlp_sizes.packed_bytes, the operand layouts the kernels read
 *    (written by pc_mlp_pack or pc_mlp_adam)
 *  - x: float[n][5], y and target: float[n][2], row-major
 *  - scratch: pc_mlp_sizes.scratch_bytes for the largest batch used
 * All calls are asynchronous on the given HIP stream and return PC_OK or a
 * negative pc_status (pc_mlp_last_error() gives the detail).
 */
#ifndef PC_MLP_H
#define PC_MLP_H

#include "pc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PC_MLP_PARAMS 8834

typedef struct pc_mlp_sizes {
    int64_t params;          /* PC_MLP_PARAMS */
    int64_t packed_bytes;    /* bytes of the packed operand block */
    int64_t scratch_bytes;   /* training scratch for max_batch samples */
} pc_mlp_sizes;

/* Sizes for training batches of up to max_batch samples. */
pc_status pc_mlp_query(int64_t max_batch, pc_mlp_sizes* out);

/* Convert the FP32 master parameters into the packed BF16 operand block. */
pc_status pc_mlp_pack(const float* master, void* packed, void* hip_stream);

/* y = network(x) for n samples.  hidden (nullable): uint16 (BF16 bit
 * patterns) [3][n][64], the three hidden activations. */
pc_status pc_mlp_forward(const void* packed, const float* x, int64_t n, float* y, uint16_t* hidden,
                         void* hip_stream);

/* Gradient of the mean squared error over n samples (mean over samples and
 * both outputs) with respect to the master parameters, into grad
 * (float[PC_MLP_PARAMS], overwritten; summed in a fixed order, so repeated
 * calls give identical bits) and the loss into *loss (device float, nullable). */
pc_status pc_mlp_grad(const void* packed, const float* x, const float* target, int64_t n, float* grad,
                      float* loss, void* scratch, size_t scratch_bytes, void* hip_stream);

/* Largest batch of the allocation-free gradient below. */
#define PC_MLP_NOALLOC_MAX_BATCH 16384

/* Allocation-free variant of pc_mlp_grad, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training or serving
 * loops, harnesses that forbid hipMalloc): the same arguments and result
 * (bitwise: the same kernels and the same fixed-order reduction) without the
 * scratch buffer.  The scratch is a device array of the library, one per
 * GPU, sized for PC_MLP_NOALLOC_MAX_BATCH samples (about 22 MB) and held
 * until the process ends; its address is looked up on the first call on
 * each device, which must be the current device of the calling thread and
 * of hip_stream.  n > PC_MLP_NOALLOC_MAX_BATCH returns PC_ERR_INVALID_ARG.
 * Nothing is allocated or freed.  Every call on one GPU shares that array:
 * calls that may overlap on one GPU (different streams without ordering)
 * race and must be serialised by the caller. */
pc_status pc_mlp_grad_noalloc(const void* packed, const float* x, const float* target, int64_t n,
                              float* grad, float* loss, void* hip_stream);

/* One Adam step (Kingma and Ba) on the FP32 master parameters with moment
 * buffers m, v (float[PC_MLP_PARAMS], zero before step 1); step counts from
 * 1.  If packed is non-null it is refreshed from the new parameters. */
pc_status pc_mlp_adam(float* master, float* m, float* v, const float* grad, int64_t step, double lr,
                      double beta1, double beta2, double eps, void* packed, void* hip_stream);

const char* pc_mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
