/*
 * mi355lbm — learned closure network for the gray model, on gfx950 matrix
 * cores (BF16 operands, FP32 accumulation).
 *
 * The network maps a window of 33 planar porosities around a cell of a gray
 * column (Sec. 4 of the paper, Fattahi et al., arXiv 1507.06565: the model's
 * effective viscosity and permeability are local functions of the porous
 * structure; the paper uses nu_eff = nu / eps) to two local coefficients,
 * with eps_c the porosity of the cell itself:
 *     nu_eff / nu = exp((1 - eps_c) o1),   eps nu / K = (1 - eps_c) softplus(o2),
 * so that both are exactly the free-fluid values (nu, 0) where eps_c = 1.
 * Layers: 33 inputs (zero-padded to 64) -> 128 -> 128 -> 128 -> 16 outputs
 * (o1, o2 used), exact-erf GELU between layers, linear output.
 *
 * Parameter vector (FP32, MLP_NPARAM floats), row-major matrices [K][N]:
 *     W1[64][128] b1[128] W2[128][128] b2[128] W3[128][128] b3[128]
 *     W4[128][16] b4[16]
 * The BF16 copy (2 * MLP_NPARAM bf16) holds the same vector twice: first in
 * the layout above, then with every matrix transposed ([N][K]); it is written
 * by mlp_pack_bf16 and by every mlp_adam_step.
 *
 * All pointers are device pointers owned by the caller; B (rows) must be a
 * positive multiple of 64.  Inputs x are BF16 [B][64], outputs y FP32 [B][16].
 * Every call is issued on the caller's stream (hipStream_t cast to void*) and
 * synchronises it before returning; errors as in lbm.h (LBM_E_INVAL for bad
 * arguments, LBM_E_DEVICE for HIP errors).
 */
#ifndef MI355LBM_MLP_H
#define MI355LBM_MLP_H

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_NPARAM 43408

/* Workspace for a training step of B rows: FP32 pre-activations and BF16
 * activations of the three hidden layers, and per-workgroup gradient
 * partials. */
lbm_status mlp_workspace_bytes(int64_t B, int64_t* bytes);

/* params (FP32) -> params_bf16 (both layouts). */
lbm_status mlp_pack_bf16(const float* params, void* params_bf16, void* stream);

/* y = net(x).  ws may be NULL (inference); a training step passes the
 * workspace so that mlp_backward can reuse the activations. */
lbm_status mlp_forward(const float* params, const void* params_bf16, const void* x_bf16, int64_t B, float* y,
                       void* ws, void* stream);

/* Gradient of sum(dy * y) with respect to the parameters (grad, FP32,
 * MLP_NPARAM) and, if dx is not NULL, to the inputs (dx FP32 [B][64]), after
 * mlp_forward with the same ws.  Gradients are reduced in a fixed order. */
lbm_status mlp_backward(const float* params, const void* params_bf16, const void* x_bf16, void* ws, const float* dy,
                        int64_t B, float* grad, float* dx, void* stream);

/* Masked mean-squared error on the two used outputs: with t [B][2] targets
 * and mask [B][2] in {0, 1} (mask_sum = sum of mask, computed by the caller),
 * dy = 2 mask (y - t) / mask_sum (0 for the unused outputs); loss_partials
 * needs ceil(B/256) doubles of device memory; *loss (host, may be NULL)
 * receives the loss. */
lbm_status mlp_loss(const float* y, const float* target, const float* mask, int64_t B, double mask_sum, float* dy,
                    double* loss_partials, double* loss, void* stream);

/* The same as mlp_loss (identical dy and loss, bit for bit) without the
 * loss_partials argument, for callers that cannot allocate device memory or
 * pass a workspace (code under stream capture, serving loops, harnesses that
 * forbid allocation): the per-block partials and their total live in a static
 * device array of the library (MLP_LOSS_NOALLOC_MAX_ROWS / 256 + 1 doubles,
 * 128 KiB, held on each GPU the library runs on until the process ends), so
 * the call allocates nothing.  B above MLP_LOSS_NOALLOC_MAX_ROWS is rejected
 * with LBM_E_INVAL.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (several streams or host threads) race and must be
 * serialised by the caller.  The calling thread's current device must be the
 * one the stream and pointers belong to. */
#define MLP_LOSS_NOALLOC_MAX_ROWS 4194304
lbm_status mlp_loss_noalloc(const float* y, const float* target, const float* mask, int64_t B, double mask_sum,
                            float* dy, double* loss, void* stream);

/* One Adam step with bias correction (step t >= 1) on the FP32 parameters,
 * refreshing the BF16 copy; m and v are FP32 moment buffers. */
lbm_status mlp_adam_step(float* params, void* params_bf16, float* m, float* v, const float* grad, double lr,
                         double b1, double b2, double eps, int64_t t, void* stream);

/* Network inputs for every cell of ncols gray columns of height nz: the 33
 * porosities around the cell, replicate padding at the column ends;
 * eps [ncols*nz] FP64 -> x_bf16 [ncols*nz][64]. */
lbm_status mlp_windows(const double* eps, int32_t ncols, int32_t nz, void* x_bf16, void* stream);

/* Closure coefficients from the outputs of n rows and the cells' own
 * porosities eps[n]: nu_eff = nu exp((1 - eps) o1), drag = (1 - eps)
 * softplus(o2); FP64 outputs. */
lbm_status mlp_closure(const float* y, const double* eps, int64_t n, double nu, double* nu_eff, double* drag,
                       void* stream);

/* Loss of nprof porosity profiles through the steady gray column and its
 * gradient with respect to the network outputs (the training signal of the
 * closure; Sec. 4, eq. (GeneralizedPor2) with the porous force of eq.
 * (PorousForce), Stokes regime).  Rows p*nz + z (z = 0..nz-1) of y [.][16]
 * belong to cell z of profile p; eps and u_target [nprof*nz] FP64 are the
 * planar porosity and the superficial velocity of the pore-scale run; layers
 * 0 and nz-1 are walls (their values are ignored).  With the closure map
 * above, the steady profile U of
 *     d/dz (nu_eff dU/dz) - drag U + eps G = 0,   U = 0 at both walls,
 * (three-point scheme on cells 1..nz-2, face viscosity the mean of the two
 * cells, quadratic one-sided slope at the walls, which reproduces the lattice
 * scheme's parabola exactly) is solved in FP64, and
 *     loss[p] = weight / nprof * sum_z (U - u_target)^2 / sum_z u_target^2.
 * dy receives dL/dy for those rows (columns 0 and 1; other columns and the
 * wall rows 0), by the adjoint of the tridiagonal system.  5 <= nz <= 1024;
 * loss is a device array of nprof doubles.  One workgroup per profile. */
lbm_status mlp_profile_loss(const float* y, const double* eps, const double* u_target, int32_t nprof, int32_t nz,
                            double nu, double G, double weight, float* dy, double* loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif
