// FP64 moments and plane reductions of the pore-scale state (eq. (Macro);
// planar averages of Sec. 3.1; Darcy's law, eq. (1), is evaluated on the host
// from these sums).
//
// The moments of the n-th collision are recovered from the post-collision
// state the sweep leaves behind: the collision conserves sum_k g_k and adds
// F to sum_k e_k g_k, so drho = sum gt and u = (sum e gt - F/2) / rho0.
// Each plane is reduced by one workgroup with a fixed thread-to-cell map and
// a fixed tree, so the result does not depend on timing or launch shape.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace lbm {
namespace {

using L = D3Q19;

// post-collision population k of cell (x, y, z), stored at index c, in the
// current state
__device__ __forceinline__ float post(const MomentArgs& a, int k, int c, int x, int y, int z) {
    if (a.layout != L_AA || a.parity < 0) return a.A[k * a.stride + c];
    if (a.parity == P_EVEN) return a.A[opp(k) * a.stride + c];
    int xn = x + L::ex[k], yn = y + L::ey[k], zn = z + L::ez[k];
    xn = xn < 0 ? a.nx - 1 : (xn == a.nx ? 0 : xn);
    yn = yn < 0 ? a.ny - 1 : (yn == a.ny ? 0 : yn);
    zn = zn < 0 ? a.nz - 1 : (zn == a.nz ? 0 : zn);
    return a.A[k * a.stride + xn + a.nx * (yn + a.ny * zn)];
}

__device__ __forceinline__ bool cell_moments(const MomentArgs& a, int c, double& rho, double& ux, double& uy,
                                             double& uz) {
    const int x = c % a.nx, t = c / a.nx, y = t % a.ny, z = t / a.ny;
    if (a.bmap) {
        // brick layout: cells of bricks that are not stored are solid
        const int b = a.bmap[(x >> 2) + (a.nx >> 2) * ((y >> 2) + (a.ny >> 2) * (z >> 2))];
        if (b < 0) return false;
        c = b * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3);
    }
    if (a.info[c] == CELL_SOLID_WORD) return false;
    double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const double v = (double)post(a, k, c, x, y, z);
        s += v;
        if (L::ex[k]) jx += L::ex[k] * v;
        if (L::ey[k]) jy += L::ey[k] * v;
        if (L::ez[k]) jz += L::ez[k] * v;
    }
    rho = s;
    ux = (jx - 0.5 * a.F[0]) / a.rho0;
    uy = (jy - 0.5 * a.F[1]) / a.rho0;
    uz = (jz - 0.5 * a.F[2]) / a.rho0;
    return true;
}

constexpr int RB = 256;

__global__ void __launch_bounds__(RB) k_plane_sums(MomentArgs a, int axis, double* out) {
    __shared__ double sh[6][RB];
    const int p = blockIdx.x;
    // plane p normal to `axis`; (i, j) run over the other two axes
    int n0, n1;
    if (axis == 0) { n0 = a.ny; n1 = a.nz; }
    else if (axis == 1) { n0 = a.nx; n1 = a.nz; }
    else { n0 = a.nx; n1 = a.ny; }
    const int64_t m = (int64_t)n0 * n1;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t e = threadIdx.x; e < m; e += RB) {
        const int i = (int)(e % n0), j = (int)(e / n0);
        int x, y, z;
        if (axis == 0) { x = p; y = i; z = j; }
        else if (axis == 1) { x = i; y = p; z = j; }
        else { x = i; y = j; z = p; }
        const int c = x + a.nx * (y + a.ny * z);
        double r, ux, uy, uz;
        if (cell_moments(a, c, r, ux, uy, uz)) {
            acc[0] += r; acc[1] += ux; acc[2] += uy; acc[3] += uz; acc[4] += 1.0;
            const bool ok = fabs(ux) < 0.4 && fabs(uy) < 0.4 && fabs(uz) < 0.4;  // false for NaN
            if (!ok) acc[5] += 1.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[(int64_t)p * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_fields(MomentArgs a, int64_t c0, int64_t n, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = 0, ux = 0, uy = 0, uz = 0;
    cell_moments(a, (int)(c0 + i), r, ux, uy, uz);
    out[i] = r;
    out[n + i] = ux;
    out[2 * n + i] = uy;
    out[3 * n + i] = uz;
}

}  // namespace

hipError_t launch_plane_sums(const MomentArgs& a, int axis, double* out, hipStream_t s) {
    const int np = axis == 0 ? a.nx : (axis == 1 ? a.ny : a.nz);
    k_plane_sums<<<np, RB, 0, s>>>(a, axis, out);
    return hipGetLastError();
}

hipError_t launch_fields(const MomentArgs& a, int64_t c0, int64_t n, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fields<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, c0, n, out);
    return hipGetLastError();
}

}  // namespace lbm
