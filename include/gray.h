/*
 * mi355lbm — gray (homogenised) lattice Boltzmann columns on AMD MI355X.
 *
 * The single-domain model of Sec. 4 of the paper (Fattahi et al., arXiv
 * 1507.06565): the generalised Navier-Stokes equation (GeneralizedPor2) with
 * the porous body force of eq. (PorousForce), discretised as in the cited
 * Guo & Zhao (2002) lattice Boltzmann model, incompressible variant with
 * populations stored as FP32 shifts g = f - w rho0, TRT collision with the
 * magic parameter Lambda; the Forchheimer term is off by default (the Stokes
 * regime of Sec. 4) and can be set per cell (gray_set_forchheimer).
 *
 * Geometry: ncols independent columns of 1 x 1 x nz cells (3 <= nz <= 704),
 * periodic along x and y.  With walls != 0 the layers z = 0 and z = nz-1 are
 * solid with half-way bounce-back and the top wall moves with velocity lid
 * (Couette driving, Ladd's correction 6 w rho0 e.u_w).  Per cell (arrays of
 * ncols*nz doubles, column-major: column c, cell z at c*nz + z):
 *   eps     porosity in (0, 1] (1 = free fluid)
 *   nu_eff  effective viscosity > 0; tau+ = 3 nu_eff + 1/2
 *   drag    Darcy coefficient eps*nu/K >= 0 (0 = free fluid; nu is the fluid
 *           viscosity, which enters only here)
 * G is the external body force per unit fluid volume; the model applies
 * eps*G.  The velocity returned is the volume-averaged (superficial) one.
 *
 * Memory and streams follow the conventions of lbm.h: one caller-owned
 * device buffer of gray_required_bytes, a caller-owned stream (hipStream_t
 * cast to void*).  Every call returns an lbm_status and synchronises the
 * stream before returning.  Errors: LBM_E_INVAL (arguments, parameters out
 * of range), LBM_E_NOMEM (buffer too small), LBM_E_DEVICE (HIP errors),
 * LBM_E_UNSTABLE (NaN or runaway velocity in a steady-state check).
 */
#ifndef MI355LBM_GRAY_H
#define MI355LBM_GRAY_H

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gray_ctx gray_ctx;

lbm_status gray_required_bytes(int32_t ncols, int32_t nz, int64_t* bytes);

/* Bind a context to dev_buf, upload the per-cell parameters and set every
 * population to rest.  lid may be NULL (no moving wall). */
lbm_status gray_init(int32_t ncols, int32_t nz, int32_t walls, const double* eps, const double* nu_eff,
                     const double* drag, double magic_lambda, double rho0, const double* G, const double* lid,
                     void* dev_buf, int64_t bytes, void* hip_stream, gray_ctx** out);

/* Replace the per-cell parameters (e.g. from a closure model); the state is
 * kept (gray_reset restarts from rest). */
lbm_status gray_set_cells(gray_ctx* ctx, const double* eps, const double* nu_eff, const double* drag);

/* Forchheimer term of eq. (PorousForce): per-cell coefficient
 * phi = eps F_eps / sqrt(K) >= 0 (ncols*nz doubles, column-major like eps),
 * adding -phi |u| u to the porous force; the implicit velocity becomes
 * u = v / (c0 + sqrt(c0^2 + c1 |v|)) with c0 = (1 + drag/2)/2, c1 = phi/2.
 * NULL clears it (the Stokes model, which is also the default).  The state
 * is kept.  Errors: LBM_E_INVAL (negative or non-finite coefficient). */
lbm_status gray_set_forchheimer(gray_ctx* ctx, const double* phi);
lbm_status gray_reset(gray_ctx* ctx);

/* Working precision in which the kernel steps the Sec. 4 model (the paper
 * fixes none): 64 (the default) or 32 bits.  The state
 * is kept in FP64 between calls either way, so the precision may change
 * between runs.  FP64 reaches the steady state of the discrete model (within
 * 1e-10 relative of an FP64 reference); in FP32 a column stops changing once
 * the remaining per-step updates fall below the FP32 resolution of its
 * populations, 1e-4 to 3e-3 (relative) short of it, at 0.7-0.9 of the FP64
 * time per step.  Errors: LBM_E_INVAL (other values). */
lbm_status gray_set_precision(gray_ctx* ctx, int32_t bits);

/* Advance every column exactly nsteps steps (one launch; the state stays in
 * registers and LDS, in the working precision, between the load and the
 * store). */
lbm_status gray_run(gray_ctx* ctx, int64_t nsteps);

/* Advance every column until the FP64 sum of u_x over the column changes by
 * at most rel_tol times its value over check_every steps, or max_steps steps
 * have run; steps_done[ncols] (may be NULL) receives the steps each column
 * ran in total.  One launch; each column stops on its own. */
lbm_status gray_run_to_steady(gray_ctx* ctx, double rel_tol, int64_t check_every, int64_t max_steps,
                              int64_t* steps_done);

/* Velocity profile of column col after the last step: u[3*nz] as
 * (u_x, u_y, u_z) per cell, FP64, 0 in wall layers. */
lbm_status gray_profile(gray_ctx* ctx, int32_t col, double* u);

void gray_destroy(gray_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
