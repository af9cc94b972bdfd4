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

// ----------------------------------------------------------- device layout --
// info[c]: INFO_SOLID, INFO_FLUID (no links) or the boundary-cell id b >= 0;
// binfo[b] = {mask, base}: bit (k-1) of mask set if (c, k) is a link, the
// link's record is lparam[base + popcount(mask & ((1 << (k-1)) - 1))].
constexpr int32_t INFO_SOLID = -2;
constexpr int32_t INFO_FLUID = -1;

enum Layout : int { L_TWOGRID = 0, L_AA = 1 };
enum Parity : int { P_EVEN = 0, P_ODD = 1 };

struct SweepArgs {
    float* A;        // populations (two-grid: source grid; AA: the only grid)
    float* B;        // two-grid destination grid (unused for AA)
    int64_t stride;  // floats between consecutive population arrays
    const int32_t* info;
    const uint2* binfo;
    const float* lparam;  // CLI: kappa; Bouzidi: q; NaN: moving-wall bounce-back
    float* side;          // AA: post-collision value of each link's unknown population
    int32_t nx, ny, nz, ncells;
    float wp, wm;         // omega+, omega-
    float cp, cm;         // 1 - omega+/2, 1 - omega-/2
    float rho0, inv_rho0;
    float F[3];
    float wterm[Q];       // 6 w_k rho0 e_k.u_w for the moving wall
    int32_t xcd_remap;
};

hipError_t launch_sweep(const SweepArgs& a, int layout, int parity, int bc, int block, hipStream_t s);

struct MomentArgs {
    const float* A;
    int64_t stride;
    const int32_t* info;
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

}  // namespace lbm
