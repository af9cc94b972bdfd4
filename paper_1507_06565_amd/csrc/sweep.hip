// Fused stream + collide sweep of the D3Q19 TRT lattice Boltzmann method
// (Sec. 2.1, eqs. (LBM), (TRT), (TRT2), (equilibrium), (Macro), (collision),
// (streaming)) with interpolated bounce-back at the solid surfaces (Sec. 2.2,
// eqs. (noslip), (CLI)), for gfx950.
//
// One thread per cell, x fastest, so a 64-wide wavefront reads and writes
// 64 consecutive floats of each population array.  Populations are FP32
// shifts g = f - w rho0.  The pass is HBM-bound: 19 loads + 19 stores of 4 B
// per fluid cell, plus a 4 B cell-info load; solid cells return at once.
//
// Boundary handling is fused into the sweep: a fluid cell x with a link k
// (x + e_k solid) rebuilds its unknown population kbar = opp(k) as
//     g_kbar(x, t+1) = c1 gt_k(x) + c0 gt_k(x - e_k) + cb gt_kbar(x) [+ wall]
// where gt are the post-collision values of step t.  gt_k(x - e_k) is the
// value x pulls for direction k anyway; gt_k(x) and gt_kbar(x) are x's own
// values of the previous step, which each layout keeps where nobody else
// writes them during the step:
//   two-grid   : source grid A[k][x], A[kbar][x]
//   AA, even   : gt_k(x) sits in the solid neighbour's slot A[k][x + e_k]
//                (written by x in the previous odd step, read by nobody else);
//                gt_kbar(x) in the per-link side buffer
//   AA, odd    : gt_k(x) in x's own slot A[kbar][x] (no other cell reads or
//                writes it in an odd step); gt_kbar(x) in the side buffer.
// The arithmetic is the same in every layout, so they agree bit for bit.
//
// AA state locations: after an even step gt_k(x) is stored at A[kbar][x];
// after an odd step at A[k][x + e_k].  An even step reads A[k][x] and writes
// A[kbar][x]; an odd step reads A[kbar][x - e_k] and writes A[k][x + e_k].
// Every slot is read and written by one thread only.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace lbm {
namespace {

using L = D3Q19;

__device__ __forceinline__ int remap_block(int b, int nblocks) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of tiles so that neighbouring tiles share an L2.
    const int per = nblocks >> 3;
    if (b < (per << 3)) return (b & 7) * per + (b >> 3);
    return b;
}

template <int BC>
__device__ __forceinline__ void bb_coeffs(float prm, float& c1, float& c0, float& cb) {
    if (BC == LBM_BC_CLI) {
        c1 = 1.0f; c0 = prm; cb = -prm;
    } else if (BC == LBM_BC_BOUZIDI) {
        if (prm < 0.5f) {
            c1 = 2.0f * prm; c0 = 1.0f - 2.0f * prm; cb = 0.0f;
        } else {
            c1 = 1.0f / (2.0f * prm); c0 = 0.0f; cb = 1.0f - c1;
        }
    } else {
        c1 = 1.0f; c0 = 0.0f; cb = 0.0f;
    }
}

// TRT collision with Guo forcing split into even/odd parts, in place on g.
__device__ __forceinline__ void collide(float (&g)[Q], const SweepArgs& a) {
    float drho = g[0];
    float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int k = 2 * p + 1;
        const float s = g[k] + g[k + 1];
        const float d = g[k] - g[k + 1];
        drho += s;
        if (L::ex[k]) jx += L::ex[k] * d;
        if (L::ey[k]) jy += L::ey[k] * d;
        if (L::ez[k]) jz += L::ez[k] * d;
    }
    const float ux = (jx + 0.5f * a.F[0]) * a.inv_rho0;
    const float uy = (jy + 0.5f * a.F[1]) * a.inv_rho0;
    const float uz = (jz + 0.5f * a.F[2]) * a.inv_rho0;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * a.F[0] + uy * a.F[1] + uz * a.F[2];
    {
        const float w0 = 1.0f / 3.0f;
        const float eq = w0 * (drho - 1.5f * a.rho0 * uu);
        g[0] = g[0] - a.wp * (g[0] - eq) + a.cp * (w0 * (-3.0f * uF));
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int k = 2 * p + 1;
        const float w = (float)weight(k);
        const float eu = L::ex[k] * ux + L::ey[k] * uy + L::ez[k] * uz;
        const float eF = L::ex[k] * a.F[0] + L::ey[k] * a.F[1] + L::ez[k] * a.F[2];
        const float eqp = w * (drho + a.rho0 * (4.5f * eu * eu - 1.5f * uu));
        const float eqm = w * (3.0f * a.rho0 * eu);
        const float gp = 0.5f * (g[k] + g[k + 1]);
        const float gm = 0.5f * (g[k] - g[k + 1]);
        const float sp = w * (9.0f * eu * eF - 3.0f * uF);
        const float sm = w * (3.0f * eF);
        const float dp = -a.wp * (gp - eqp) + a.cp * sp;
        const float dm = -a.wm * (gm - eqm) + a.cm * sm;
        const float gk = g[k], gkb = g[k + 1];
        g[k] = gk + dp + dm;
        g[k + 1] = gkb + dp - dm;
    }
}

template <int LAYOUT, int PARITY, int BC, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_sweep(SweepArgs a) {
    int b = blockIdx.x;
    if (a.xcd_remap) b = remap_block(b, gridDim.x);
    const int c = b * BLOCK + threadIdx.x;
    if (c >= a.ncells) return;
    const int inf = a.info[c];
    if (inf == INFO_SOLID) return;

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int x = c % nx;
    const int t = c / nx;
    const int y = t % ny;
    const int z = t / ny;
    const int X[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
    const int Y[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
    const int Z[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
    // linear index of x + (dx, dy, dz)
#define NB(dx, dy, dz) (X[(dx) + 1] + nx * (Y[(dy) + 1] + ny * Z[(dz) + 1]))

    float* __restrict__ A = a.A;
    const int64_t S = a.stride;

    uint32_t mask = 0;
    int base = 0;
    if (inf >= 0) {
        const uint2 bi = a.binfo[inf];
        mask = bi.x;
        base = (int)bi.y;
    }

    // 1) streaming: pull every population that does not come out of a solid
    float g[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int kb = opp(k);
        const bool link = (k != 0) && (mask & (1u << (kb - 1)));
        float v = 0.0f;
        if (!link) {
            if (LAYOUT == L_TWOGRID)
                v = A[k * S + NB(-L::ex[k], -L::ey[k], -L::ez[k])];
            else if (PARITY == P_EVEN)
                v = A[k * S + c];
            else
                v = A[kb * S + NB(-L::ex[k], -L::ey[k], -L::ez[k])];
        }
        g[k] = v;
    }

    // 2) bounce-back of the populations that would come out of the solid
    if (mask) {
        float h[Q];
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int kk = opp(k);  // link direction: x + e_kk is solid
            h[k] = g[k];
            if (mask & (1u << (kk - 1))) {
                const int li = base + __popc(mask & ((1u << (kk - 1)) - 1u));
                const float prm = a.lparam[li];
                float own_kk, own_k;
                if (LAYOUT == L_TWOGRID) {
                    own_kk = A[kk * S + c];
                    own_k = A[k * S + c];
                } else if (PARITY == P_EVEN) {
                    own_kk = A[kk * S + NB(L::ex[kk], L::ey[kk], L::ez[kk])];
                    own_k = a.side[li];
                } else {
                    own_kk = A[k * S + c];
                    own_k = a.side[li];
                }
                float c1, c0, cb, wt = 0.0f;
                if (prm != prm) {  // moving wall: simple bounce-back + Ladd term
                    c1 = 1.0f; c0 = 0.0f; cb = 0.0f; wt = a.wterm[k];
                } else {
                    bb_coeffs<BC>(prm, c1, c0, cb);
                }
                h[k] = c1 * own_kk + c0 * g[kk] + cb * own_k + wt;
            }
        }
#pragma unroll
        for (int k = 1; k < Q; ++k) g[k] = h[k];
    }

    // 3) collision
    collide(g, a);

    // 4) store
    float* __restrict__ D = (LAYOUT == L_TWOGRID) ? a.B : A;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if (LAYOUT == L_TWOGRID)
            D[k * S + c] = g[k];
        else if (PARITY == P_EVEN)
            D[opp(k) * S + c] = g[k];
        else
            D[k * S + NB(L::ex[k], L::ey[k], L::ez[k])] = g[k];
    }
    if (LAYOUT == L_AA && mask) {
#pragma unroll
        for (int kk = 1; kk < Q; ++kk) {
            if (mask & (1u << (kk - 1))) {
                const int li = base + __popc(mask & ((1u << (kk - 1)) - 1u));
                a.side[li] = g[opp(kk)];
            }
        }
    }
#undef NB
}

template <int LAYOUT, int PARITY, int BC>
hipError_t launch3(const SweepArgs& a, int block, hipStream_t s) {
    const int64_t nb64 = ((int64_t)a.ncells + block - 1) / block;
    const unsigned nb = (unsigned)nb64;
    switch (block) {
        case 128: k_sweep<LAYOUT, PARITY, BC, 128><<<nb, 128, 0, s>>>(a); break;
        case 256: k_sweep<LAYOUT, PARITY, BC, 256><<<nb, 256, 0, s>>>(a); break;
        case 512: k_sweep<LAYOUT, PARITY, BC, 512><<<nb, 512, 0, s>>>(a); break;
        case 1024: k_sweep<LAYOUT, PARITY, BC, 1024><<<nb, 1024, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int LAYOUT, int PARITY>
hipError_t launch2(const SweepArgs& a, int bc, int block, hipStream_t s) {
    switch (bc) {
        case LBM_BC_SBB: return launch3<LAYOUT, PARITY, LBM_BC_SBB>(a, block, s);
        case LBM_BC_CLI: return launch3<LAYOUT, PARITY, LBM_BC_CLI>(a, block, s);
        case LBM_BC_BOUZIDI: return launch3<LAYOUT, PARITY, LBM_BC_BOUZIDI>(a, block, s);
    }
    return hipErrorInvalidValue;
}

__global__ void k_fill_zero(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n; j += stride) p[j] = 0.0f;
}

}  // namespace

hipError_t launch_sweep(const SweepArgs& a, int layout, int parity, int bc, int block, hipStream_t s) {
    if (layout == L_TWOGRID) return launch2<L_TWOGRID, P_EVEN>(a, bc, block, s);
    if (parity == P_EVEN) return launch2<L_AA, P_EVEN>(a, bc, block, s);
    return launch2<L_AA, P_ODD>(a, bc, block, s);
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_fill_zero<<<(unsigned)blocks, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace lbm
