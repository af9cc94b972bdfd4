/*
 * mi355lbm — D3Q19 lattice Boltzmann pore-scale flow on AMD MI355X (gfx950).
 *
 * C ABI of the library.  Plain types only; every entry point returns an
 * lbm_status (0 on success, negative on error) unless stated otherwise, and
 * never aborts or throws across the boundary.  lbm_last_error() returns a
 * thread-local text for the last failure on the calling thread.
 *
 * Method: Fattahi, Waluga, Wohlmuth, Ruede, "Large scale lattice Boltzmann
 * simulation for the coupling of free and porous media flow" (arXiv
 * 1507.06565).  Section/equation names below refer to that paper.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - Lattice units: cell spacing 1, time step 1, c_s^2 = 1/3.
 *  - Cell (x, y, z) has linear index x + nx*(y + ny*z) (x fastest).
 *  - D3Q19 velocity order (the direction index used by lbm_geometry_links):
 *      0 ( 0, 0, 0)
 *      1 (+1, 0, 0)  2 (-1, 0, 0)  3 ( 0,+1, 0)  4 ( 0,-1, 0)
 *      5 ( 0, 0,+1)  6 ( 0, 0,-1)
 *      7 (+1,+1, 0)  8 (-1,-1, 0)  9 (+1,-1, 0) 10 (-1,+1, 0)
 *     11 (+1, 0,+1) 12 (-1, 0,-1) 13 (+1, 0,-1) 14 (-1, 0,+1)
 *     15 ( 0,+1,+1) 16 ( 0,-1,-1) 17 ( 0,+1,-1) 18 ( 0,-1,+1)
 *    weights 1/3, 1/18 (axis), 1/36 (diagonal); opposite of k>0 is k+1 for
 *    odd k and k-1 for even k.
 *  - Populations are stored in FP32 as shifts g_k = f_k - w_k*rho0 and
 *    collided in FP32; moments, plane averages, totals and permeability are
 *    accumulated in FP64.
 *  - "The fields after n steps" are the density fluctuation and velocity of
 *    the n-th collision: drho = sum_k g_k, u = (sum_k e_k g_k + F/2)/rho0
 *    (eq. (Macro), with the half-force term of the forcing scheme).
 *  - Device memory is owned by the caller: the library carves every device
 *    array it needs out of one buffer the caller passes to *_init, sized by
 *    *_required_bytes, and never allocates device memory itself.
 *  - Streams are owned by the caller and passed as a hipStream_t cast to
 *    void*.  Stepping calls are asynchronous on that stream; calls that return
 *    host data synchronise it before returning.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MI355LBM_LBM_H
#define MI355LBM_LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_E_INVAL (-1)    /* bad argument or unsupported geometry/parameters */
#define LBM_E_NOMEM (-2)    /* caller buffer too small, or host allocation failed */
#define LBM_E_DEVICE (-3)   /* HIP runtime error or no usable device */
#define LBM_E_STATE (-4)    /* call not valid in the context's current state */
#define LBM_E_UNSTABLE (-5) /* NaN or |u| >= 0.4 detected in a reduction */

/* boundary schemes for the curved (sphere) surfaces, Sec. 2.2 */
#define LBM_BC_SBB 0     /* simple bounce-back, eq. (noslip) */
#define LBM_BC_CLI 1     /* central linear interpolation, eq. (CLI) */
#define LBM_BC_BOUZIDI 2 /* Bouzidi linear interpolation */

#define LBM_BGK 0 /* single relaxation time: omega- = omega+ */
#define LBM_TRT 1 /* two relaxation times, eq. (TRT) */

#define LBM_LAYOUT_TWOGRID 0 /* two population arrays, pull streaming */
#define LBM_LAYOUT_AA 1      /* one array updated in place, alternating steps */
/* Two arrays with pull streaming over 4x4x4 bricks: only bricks that hold a
 * fluid cell are stored (sparse packings store 15-25 % fewer cells than the
 * dense layouts); needs nx, ny, nz divisible by 4.  Same arithmetic as the
 * two-grid layout: the two give bit-identical fields.  It pays off for states
 * larger than the 256 MB last-level cache; a domain whose single AA grid fits
 * in that cache runs faster in the AA layout. */
#define LBM_LAYOUT_BRICK 2

typedef struct lbm_geometry lbm_geometry;
typedef struct lbm_ctx lbm_ctx;

/* A sphere in lattice units.  Centre and radius must be multiples of 2^-12
 * (so all geometric predicates are exact in binary64); along a periodic axis
 * the centre must lie in [0, n) and the radius below n. */
typedef struct {
    double cx, cy, cz, r;
} lbm_sphere;

/* One domain.  Every axis is either periodic, or bounded by solid wall layers
 * at index 0 and n-1 (wall_lo = wall_hi = 1); the wall surface lies half-way
 * between the wall layer and the first fluid layer (q = 1/2).  A nonzero
 * wall_hi_velocity makes every high wall a moving lid (Couette driving).
 * bc selects the boundary scheme used at sphere surfaces. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];
    int32_t wall_lo[3];
    int32_t wall_hi[3];
    double wall_hi_velocity[3];
    const lbm_sphere* spheres;
    int64_t n_spheres;
    int32_t bc;
} lbm_domain_desc;

/* Collision parameters (Sec. 2.1).  tau_plus = 1/omega+ = 3 nu + 1/2 > 1/2.
 * TRT: omega- follows from the magic parameter
 *      Lambda = (1/omega+ - 1/2)(1/omega- - 1/2)  (3/16: exact bounce-back
 *      wall location for Poiseuille flow; second-order CLI);
 * BGK: omega- = omega+ (magic_lambda ignored).  omega- must lie in (0, 2).
 * force: body force per unit volume applied in every fluid cell (the flow
 * driving of Sec. 3; equivalent to a pressure gradient in a periodic domain).
 * rho0: reference density (1 in the paper).  layout: LBM_LAYOUT_*. */
typedef struct {
    int32_t collision;
    double tau_plus;
    double magic_lambda;
    double rho0;
    double force[3];
    int32_t layout;
} lbm_params;

/* ---------------------------------------------------------------- geometry --
 * lbm_geometry_build: voxelise n_domains domains (host, multi-threaded).
 *   A cell is solid when it is a wall layer or its centre lies in the closed
 *   ball of some sphere (periodic images included).  For every fluid cell x
 *   and direction k whose neighbour x+e_k (wrapped) is not fluid there is a
 *   link (x, k) with wall distance q in (0, 1] (eq. (CLI): q = |x_f - x_w| /
 *   |x_f - x_b|): 1/2 if the neighbour is a wall layer, otherwise the first
 *   entry t of the segment x + t e_k into any sphere, computed in binary64 as
 *       t = (-b - sqrt(b*b - a*c)) / a,
 *       a = |e_k|^2, b = e_k.(x - c_s), c = |x - c_s|^2 - r^2;
 *   a sphere closer than a wall wins, a tie goes to the wall.
 *   The spheres are copied; *out is owned by the caller (lbm_geometry_free).
 *   Errors: LBM_E_INVAL for an invalid descriptor (see lbm_domain_desc and
 *   lbm_sphere), LBM_E_NOMEM if host memory runs out. */
lbm_status lbm_geometry_build(const lbm_domain_desc* domains, int32_t n_domains, lbm_geometry** out);

/* Copy flags of domain dom into host_flags[nx*ny*nz]: 0 fluid, 1 sphere,
 * 2 wall layer. */
lbm_status lbm_geometry_flags(const lbm_geometry* g, int32_t dom, uint8_t* host_flags);

/* Links of domain dom sorted by (cell, k).  *n receives the count; if the
 * arrays are non-NULL they must hold *n entries on input (as returned by a
 * first call with NULL arrays) and receive cell index, direction k (x+e_k is
 * the solid neighbour) and q. */
lbm_status lbm_geometry_links(const lbm_geometry* g, int32_t dom, int64_t* n, int64_t* cell, int8_t* dir,
                              double* q);

/* Number of domains, fluid cells of domain dom. */
lbm_status lbm_geometry_info(const lbm_geometry* g, int32_t dom, int32_t* n_domains, int64_t* n_fluid,
                             int64_t* n_links);

void lbm_geometry_free(lbm_geometry* g);

/* ----------------------------------------------------------- pore-scale run --
 * lbm_required_bytes: size of the device buffer lbm_init needs for geometry g
 * and params p (populations, one partial bounce-back value per link, cell
 * info, link coefficients, reduction scratch).  With more than one domain the
 * batched kernel is used: each domain has its own state, in the brick layout
 * (two grids) when params.layout is LBM_LAYOUT_BRICK, otherwise in the AA
 * layout. */
lbm_status lbm_required_bytes(const lbm_geometry* g, const lbm_params* p, int64_t* bytes);

/* lbm_init: bind a context to the caller's device buffer dev_buf (at least
 * lbm_required_bytes, any alignment >= 256 B) on stream hip_stream, upload the
 * geometry (the geometry object may be freed afterwards) and set every
 * population to rest, g = 0 (f = w rho0).  Asynchronous on the stream.
 * Errors: LBM_E_INVAL (parameters: tau_plus <= 1/2, omega- outside (0,2),
 * unknown collision/layout, brick layout with a size not divisible by 4),
 * LBM_E_NOMEM (bytes too small), LBM_E_DEVICE. */
lbm_status lbm_init(const lbm_geometry* g, const lbm_params* p, void* dev_buf, int64_t bytes, void* hip_stream,
                    lbm_ctx** out);

/* Advance every domain n >= 0 time steps: per fluid cell, stream (pull) with
 * bounce-back of the populations that would come out of the solid (eq.
 * (noslip), eq. (CLI) or Bouzidi, chosen by the domain's bc; a CLI/Bouzidi
 * link whose second fluid node x - e_k is not fluid falls back to simple
 * bounce-back; a moving wall adds 6 w_k rho0 e_k.u_w), moments, incompressible
 * equilibrium (eq. (equilibrium)), TRT collision (eqs. (TRT), (TRT2)) with
 * Guo's forcing split into even and odd parts.  Asynchronous. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Run until the FP64 mean velocity along the force direction U changes by at
 * most rel_tol*|U| over check_every steps, or max_steps are done.  For a
 * batched context every domain converges on its own inside one persistent
 * launch.  steps_done[n_domains] receives the steps each domain ran (and
 * max_steps for domains that did not converge).  Synchronises. */
lbm_status lbm_run_to_steady(lbm_ctx* ctx, double rel_tol, int64_t check_every, int64_t max_steps,
                             int64_t* steps_done);

/* Planar averages (Sec. 3.1: planar average of the stream-wise velocity) of
 * velocity component comp (0,1,2) over planes normal to axis (0,1,2) of
 * domain dom, from the fields after the last step.  Each output array has
 * n_axis entries and may be NULL: u_superficial = sum / plane area,
 * u_intrinsic = sum / fluid cells of the plane (0 if none), porosity = fluid
 * cells / plane area.  FP64 reduction in a fixed order.  Synchronises. */
lbm_status lbm_average_profile(lbm_ctx* ctx, int32_t dom, int32_t axis, int32_t comp, double* u_superficial,
                               double* u_intrinsic, double* porosity);

/* Darcy permeability, eq. (1): K = rho0 nu <U_sup> / G, where <U_sup> is the
 * mean superficial velocity along flow_axis over z-planes [z0, z1) and G the
 * body force along flow_axis (must be nonzero).  Synchronises. */
lbm_status lbm_permeability(lbm_ctx* ctx, int32_t dom, int32_t flow_axis, int32_t z0, int32_t z1, double* k);

/* Fields after the last step, FP64 on the host: host_rho[N] (density
 * fluctuation) and host_u[3*N] (component-major: u_x of all cells, then u_y,
 * then u_z); 0 in solid cells.  Either pointer may be NULL.  Synchronises. */
lbm_status lbm_fields(lbm_ctx* ctx, int32_t dom, double* host_rho, double* host_u);

/* Totals over fluid cells: mass sum(drho) and momentum sum(rho0 u).  FP64.
 * Returns LBM_E_UNSTABLE if any fluid cell holds NaN or |u_i| >= 0.4. */
lbm_status lbm_totals(lbm_ctx* ctx, int32_t dom, double* mass, double momentum[3]);

/* Checkpoint: lbm_state_bytes gives the size of the host image; lbm_save
 * copies populations (in the context's storage order), partial bounce-back
 * values, step counter and layout parity to host_buf; lbm_load
 * restores them into a context built from the same geometry and params.
 * Synchronises.  Restarting from a saved image is bit-identical. */
lbm_status lbm_state_bytes(lbm_ctx* ctx, int64_t* bytes);
lbm_status lbm_save(lbm_ctx* ctx, void* host_buf, int64_t bytes);
lbm_status lbm_load(lbm_ctx* ctx, const void* host_buf, int64_t bytes);

/* Steps run so far. */
lbm_status lbm_steps_done(lbm_ctx* ctx, int64_t* steps);

/* Sweep launch configuration of a single-domain context: cells per workgroup
 * (64, 128, 256, 512 or 1024; the brick layout runs one brick of 64 cells
 * per wavefront) and flags: LBM_LAUNCH_XCD_REMAP deals
 * consecutive tiles to one XCD instead of round-robin, LBM_LAUNCH_NONTEMPORAL
 * marks the aligned population streams non-temporal, LBM_LAUNCH_CELLS_2 /
 * LBM_LAUNCH_CELLS_4 (not both; brick layout only, LBM_E_INVAL otherwise)
 * make each thread update 2 or 4 cells in turn (each workgroup steps that
 * many groups of bricks, group b, b + G, ... for a grid of G workgroups;
 * default one cell per thread).  Every configuration gives bit-identical
 * results.  lbm_autotune times every workgroup size with every combination
 * of the first two flags for steps_per_trial steps on the context itself,
 * then (brick layout) 2 and 4 cells per thread at the best of those, keeps the
 * fastest and restores the state (host copy, or the rest state if no step was
 * taken); the choice is cached per process by (architecture, shape, layout,
 * bc) and reused by later lbm_init calls.  Synchronises. */
#define LBM_LAUNCH_XCD_REMAP 1
#define LBM_LAUNCH_NONTEMPORAL 2
#define LBM_LAUNCH_CELLS_2 4
#define LBM_LAUNCH_CELLS_4 8
lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t block, int32_t flags);
lbm_status lbm_get_launch(lbm_ctx* ctx, int32_t* block, int32_t* flags);
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t steps_per_trial);

/* Layout autotuner.  The candidates are, for one domain, the two-grid, AA
 * and (when nx, ny and nz are divisible by 4) brick layouts; for several
 * domains the AA layout (one persistent launch) and the brick layout (one
 * brick-list launch per step).  lbm_autotune_layout_bytes gives the device
 * memory the tuner needs: the largest lbm_required_bytes over the candidates
 * that can hold the geometry.  lbm_autotune_layout initialises each candidate
 * from rest in dev_buf (caller-owned, at least that many bytes, 256-byte
 * aligned), tunes its launch shape with lbm_autotune, times steps_per_trial
 * steps (rounded up to even) with the tuned shape on the caller's stream, and
 * returns the fastest layout in *layout and its time per step in
 * *ms_per_step (may be NULL); no context is left in dev_buf.  Every layout
 * gives bit-identical fields, so the choice only changes speed.  The choice
 * is cached per process by (architecture, domain count, first domain's shape,
 * total cells, bc, collision); with a cached choice the call returns it at
 * once (dev_buf may then be NULL).  Synchronises. */
lbm_status lbm_autotune_layout_bytes(const lbm_geometry* g, const lbm_params* params, int64_t* bytes);
lbm_status lbm_autotune_layout(const lbm_geometry* g, const lbm_params* params, void* dev_buf, int64_t bytes,
                               void* hip_stream, int32_t steps_per_trial, int32_t* layout, double* ms_per_step);

/* The autotuners' choices (lbm_autotune, lbm_autotune_layout and the batch
 * autotuners) are cached per process; these two calls carry them to a later
 * process.  Text, one entry per line, fields separated by spaces, lines
 * starting with '#' ignored:
 *   sweep ARCH NX NY NZ LAYOUT BC BLOCK FLAGS
 *   layout ARCH DOMAINS NX NY NZ BC COLLISION CELLS LAYOUT MS_PER_STEP
 *   brick-batch ARCH DOMAINS BRICKS BLOCK NONTEMPORAL CELLS_PER_THREAD
 *   aa-batch ARCH DOMAINS CELLS BLOCK WORKGROUPS_PER_DOMAIN
 * (ARCH is the device's architecture name; the other fields are integers
 * with the meanings and ranges of lbm_set_launch, lbm_batch_set_launch and
 * lbm_params, MS_PER_STEP a decimal number.)  lbm_tuning_export writes the
 * text and its terminating NUL to buf when capacity exceeds its length, and
 * the length without the NUL to *length in any case (buf may be NULL with
 * capacity 0 to ask for the length).  lbm_tuning_import adds the entries of
 * a NUL-terminated text to the caches, replacing entries with the same key;
 * a line that is not a valid entry fails the whole call with LBM_E_INVAL
 * (naming the line) and changes nothing.  Host only: no device call. */
lbm_status lbm_tuning_export(char* buf, int64_t capacity, int64_t* length);
lbm_status lbm_tuning_import(const char* text);

/* Streaming ceiling of the brick sweep's access pattern (a measurement aid,
 * not a step of the method): copies nbricks x 64 cells x 19 FP32 values from
 * src to dst with one wavefront per brick and non-temporal stores, exactly
 * the population bytes a sweep of that many bricks reads and writes once,
 * with nothing else.  grouped = 0: the sweep's layout (population k of brick
 * b at element k*64*nbricks + 64*b + lane); grouped = 1: a brick's 19
 * populations contiguous ((19*b + k)*64 + lane).  src and dst are
 * caller-owned device buffers of at least 4864*nbricks bytes each (dst is
 * overwritten); three untimed passes, then passes timed with HIP events on
 * hip_stream; *ms_per_pass receives the average.  Synchronises. */
lbm_status lbm_stream_probe(const void* src, void* dst, int64_t nbricks, int32_t grouped, int32_t passes,
                            void* hip_stream, double* ms_per_pass);

/* Launch shape of a batched context.  AA layout (one persistent kernel):
 * workgroup size (256, 512 or 1024) and workgroups that step one domain
 * together (1..64); the persistent launch holds as many workgroups as can be
 * resident, and teams of workgroups_per_domain pop domains from a
 * largest-first queue.  Brick layout (all domains in one brick array, one
 * brick-sweep launch per step): workgroup size 64..1024 (one brick per
 * wavefront), and the second value is the cells per thread instead (1, 2
 * or 4: each workgroup steps that many groups of bricks in turn).  Results
 * are bit-identical for every shape.  lbm_autotune on a batched context
 * (before any step) times the shapes on steps_per_trial steps of all
 * domains (brick layout: sizes and hints at one cell per thread, then 2 and
 * 4 cells per thread at the best), keeps the fastest and restores the rest
 * state. */
lbm_status lbm_batch_set_launch(lbm_ctx* ctx, int32_t block, int32_t workgroups_per_domain);
lbm_status lbm_batch_get_launch(lbm_ctx* ctx, int32_t* block, int32_t* workgroups_per_domain);

/* Destroy a context (the device buffer stays the caller's). */
void lbm_destroy(lbm_ctx* ctx);

/* Text of the last error on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
