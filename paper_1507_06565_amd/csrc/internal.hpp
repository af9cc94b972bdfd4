// Internal declarations shared by the host C ABI (capi.cpp, geometry.cpp)
// and the HIP kernel launchers (*.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lattice.hpp"

namespace lbm {

// ---------------------------------------------------------------- geometry --
struct DomainGeo {
    lbm_domain_desc desc{};            // spheres pointer re-pointed at `spheres`
    std::vector<lbm_sphere> spheres;
    std::vector<uint8_t> flags;        // nx*ny*nz
    std::vector<int64_t> lcell;        // links sorted by (cell, k)
    std::vector<int8_t> ldir;
    std::vector<double> lq;
    std::vector<int8_t> lsurf;
    int64_t n_fluid = 0;
    int64_t ncells() const { return (int64_t)desc.nx * desc.ny * desc.nz; }
};

lbm_status build_domain(const lbm_domain_desc& d, DomainGeo& out, std::string& err);

// error text for the calling thread (defined with the C ABI); returns s
lbm_status set_error(lbm_status s, const std::string& msg);

// ----------------------------------------------------------- device layout --
// One 32-bit word per stored cell (c: its index in the population arrays):
//   CELL_SOLID_WORD (all ones)  solid cell, not updated;
//   otherwise bits 0..17 are the link mask (bit k-1 set if x + e_k is solid)
//   and bits 18..31 the offset of the cell's first link from the first link
//   of its 512-cell segment; segbase[c >> 9] holds that segment's first link.
//   A segment has at most 512 * 18 = 9216 links, so the offset fits 14 bits.
// Link i of cell c (in increasing k) has its record at lparam[first + i].
constexpr uint32_t CELL_SOLID_WORD = 0xFFFFFFFFu;
constexpr int SEG_SHIFT = 9;
constexpr uint32_t LINK_MASK_BITS = 0x3FFFFu;

// Link coefficients and partial values are addressed by 32-bit byte offsets
// (4 x link index, index < nl + Q with the padding) and segment bases are
// int32, so one domain, or one brick-layout batch, may hold at most
// max_links() = 2^30 - Q links.  The environment variable
// MI355LBM_MAX_LINKS can only lower this limit (for tests of the check).
int64_t max_links();

enum Layout : int { L_TWOGRID = 0, L_AA = 1, L_BRICK = 2 };
enum Parity : int { P_EVEN = 0, P_ODD = 1 };

// collision constants shared by every cell of a run
// Uniform constants of the cell update.  The TRT collision with the split
// Guo forcing is evaluated in a folded form (see collide() in cell.hpp); the
// folded coefficients below are products of the relaxation rates, weights,
// rho0 and the body force, formed once on the host in FP64.
struct CellConsts {
    float wp, wm;         // omega+, omega-
    float cp, cm;         // 1 - omega+/2, 1 - omega-/2
    float rho0, inv_rho0;
    float F[3];
    float fh[3];          // F / (2 rho0)
    float om1;            // 1 - omega+
    float hp, hm;         // -omega+/2, -omega-/2
    float a_uu, a_uF;     // -1.5 omega+ rho0, -3 (1 - omega+/2)
    float beta[2];        // 4.5 omega+ w rho0 for w = 1/18, 1/36
    float delta[2];       // 3 omega- w rho0 for w = 1/18, 1/36
    float gam[9];         // 9 (1 - omega+/2) w_k e_k.F for k = 1, 3, ..., 17
    float zet[9];         // 3 (1 - omega-/2) w_k e_k.F for k = 1, 3, ..., 17
    float wterm[Q];       // 6 w_k rho0 e_k.u_w for the moving wall
};

struct SweepArgs {
    float* A;        // populations (two-grid: source grid; AA: the only grid)
    float* B;        // two-grid destination grid (unused for AA)
    int64_t stride;  // floats between consecutive population arrays
    float* pa[Q];    // A + k*stride (uniform bases, filled per launch)
    float* pb[Q];    // B + k*stride
    const uint32_t* info;
    const int32_t* segbase;
    const float* lparam;  // CLI: kappa; Bouzidi: q; NaN: moving-wall bounce-back;
                          // padded with Q entries so that rank lookups stay in bounds
    float* pva;           // partial bounce-back values read this step (one per link)
    float* pvb;           // ... and written for the next step (AA: pva == pvb)
    int32_t nx, ny, nz, ncells;
    const int32_t* nbr;   // brick layout: 27 neighbour bricks per stored brick
    int32_t nbricks;      // brick layout: bricks to update (entries of `list` when it is set)
    const int32_t* list;  // brick layout, batches: the bricks to update (null: 0 .. nbricks-1)
    double* partial;      // brick layout, batches: per-brick FP64 sum of u_x written on check steps
    CellConsts k;
    int32_t xcd_remap;
    int32_t nt;           // non-temporal hints on the aligned streams
    int32_t cpt;          // cells per thread: tiles (brick groups) each workgroup steps in turn, 1, 2 or 4
};

// Brick layout (4x4x4 bricks, bricks without fluid cells not stored): map
// from the dense brick index (bx + BX (by + BY bz)) to the stored brick
// (-1: not stored) and, per stored brick, the stored neighbours in the 27
// directions j = (dx+1) + 3 (dy+1) + 9 (dz+1), wrapped, with the brick itself
// in place of a brick that is not stored.
constexpr int BRICK = 4;
struct BrickMap {
    int32_t bx = 0, by = 0, bz = 0;  // bricks per axis
    int64_t nstored = 0;
    std::vector<int32_t> id;         // bx*by*bz
    std::vector<int32_t> nbr;        // 27 * nstored
};
bool brick_dims_ok(const lbm_domain_desc& d);
void build_brick_map(const DomainGeo& G, BrickMap& bm, bool with_table);

struct DeviceImages {
    std::vector<uint32_t> info;
    std::vector<int32_t> segbase;
    std::vector<float> lparam;
    std::vector<int64_t> seed_idx;
    std::vector<float> seed_val;
};
// cell words, link records and seeds in the storage order of the layout
// (bm: the brick map for L_BRICK, else unused)
lbm_status build_images(const DomainGeo& G, int layout, const BrickMap& bm, int64_t stride, const CellConsts& K,
                        DeviceImages& im, std::string& err);

CellConsts make_consts(const lbm_params& p, double wp, double wm, const double* wall_velocity);

hipError_t launch_sweep(const SweepArgs& a, int layout, int parity, int bc, int block, hipStream_t s);

// brick sweep over a.list (a.nbricks entries); with check, every updated
// brick's wavefront also stores the fixed-order FP64 sum of its cells' u_x
// in a.partial[brick]
hipError_t launch_sweep_bricks(const SweepArgs& a, int bc, int block, bool check, hipStream_t s);

// out[d] = sum of partial[first[d] .. first[d] + count[d]) in a fixed order
// (one wavefront per domain), for the domains listed in doms[0 .. n)
hipError_t launch_domain_sums(const double* partial, const int32_t* first, const int32_t* count, const int32_t* doms,
                              int n, double* out, hipStream_t s);

struct MomentArgs {
    const float* A;
    int64_t stride;
    const uint32_t* info;
    const int32_t* bmap;     // brick layout: dense brick -> stored brick (-1: none); else null
    int32_t nx, ny, nz;
    int32_t layout, parity;  // parity of the last step taken (AA); -1: no step yet
    double rho0;
    double F[3];
};

// out[p*6 + {0..5}] = {sum drho, sum ux, sum uy, sum uz, fluid cells, bad cells}
// over plane p normal to axis (0,1,2); fixed-order FP64 reduction.
hipError_t launch_plane_sums(const MomentArgs& a, int axis, double* out, hipStream_t s);

// rho[i], u[3][i] (FP64) for cells [c0, c0 + n) into out[4*n]: rho then ux, uy, uz
hipError_t launch_fields(const MomentArgs& a, int64_t c0, int64_t n, double* out, hipStream_t s);

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);

// p[idx[i]] = val[i] for i < n (seeding the moving-wall partial values)
hipError_t launch_scatter(float* p, const int64_t* idx, const float* val, int64_t n, hipStream_t s);

}  // namespace lbm
