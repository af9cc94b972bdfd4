// Gray (homogenised) lattice Boltzmann model for flow in and over a porous
// medium: the generalised Navier-Stokes model of Sec. 4, eqs.
// (GeneralizedPor1), (GeneralizedPor2), (PorousForce), discretised as in the
// cited Guo & Zhao (2002) model, in its incompressible variant with shifted
// populations and a TRT collision, Forchheimer coefficient zero (Stokes
// regime of Sec. 4, unless a Forchheimer coefficient is set).
//
// A column is 1 x 1 x nz cells, periodic in x and y, so every population
// streams along z only.  Per cell: porosity eps, effective viscosity nu_eff
// (tau+ = 3 nu_eff + 1/2; omega- from the magic parameter), the Darcy drag
// coefficient D = eps nu / K (0 in free fluid) and, optionally, the
// Forchheimer coefficient phi = eps F_eps / sqrt(K):
//   v      = sum_k e_k g_k / rho0 + eps G / 2
//   u      = v / (c0 + sqrt(c0^2 + c1 |v|)),  c0 = (1 + D/2)/2, c1 = phi/2
//            (u = v - F(u)/2 solved for u; u = v / (1 + D/2) when phi = 0)
//   F      = -D u - phi |u| u + eps G            (eq. (PorousForce))
//   g_eq_k = w_k [drho + rho0 (3 e.u + 4.5 (e.u)^2 / eps - 1.5 u.u / eps)]
//   S_k    = w_k rho0 [3 e.F + 9 (e.u)(e.F) / eps - 3 u.F / eps]
// with S split into even and odd parts relaxed by (1 - omega+/2) and
// (1 - omega-/2).  Optional wall layers at z = 0 and z = nz-1 (half-way
// bounce-back; the top wall may move, Ladd's correction).
//
// One workgroup per column, one thread per cell, the time loop inside the
// kernel.  The nine populations with e_z = 0 never leave their cell in a
// 1 x 1 periodic column, so they stay in registers; the ten with e_z != 0
// pass through two LDS buffers (read one, write the other: one barrier per
// step), each thread pulling from offsets it computes once, wall bounce-back
// included.  Global memory is touched only to load and store the state and to
// write the final profile.  The steady-state test (relative change of the
// FP64 sum of u_x over check_every steps) is evaluated in the kernel with a
// fixed-order workgroup reduction.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gray.h"
#include "internal.hpp"

namespace lbm {

struct GrayArgs {
    float* state;         // ncols x 19 x nz
    const float* cell;    // ncols x nz x 4: eps, omega+, omega-, D
    const float* phi;     // ncols x nz Forchheimer coefficients, or null (all zero)
    double* u;            // ncols x nz x 3
    int64_t* steps;       // per column
    double* uprev;        // per column
    int32_t* status;      // per column: 0 running, 1 converged, -1 unstable
    int32_t nz, walls, steady, check_every, lid;
    int64_t nsteps;
    double tol;
    float rho0, G[3];
    float wterm[Q];
};

namespace {

using L = D3Q19;

// the populations with e_z != 0; slot m holds direction MOVK[m], and
// opposite directions sit in slots m and m ^ 1
constexpr int NMOV = 10;
__device__ constexpr int MOVK[NMOV] = {5, 6, 11, 12, 13, 14, 15, 16, 17, 18};

// per-cell constants of the collision
struct GrayCell {
    float D, phi, wp, wm, cmi, hwp, hwm, omwp, A, c45, c9, m15wp, m3cpl, den;
    float Ge[3], hGe[3];
};

template <int BLOCK>
struct GrayShared {
    float mv[2][NMOV][BLOCK];  // moving populations, two buffers
    double red[BLOCK / 64];    // one partial sum per wavefront
    int stop;
};

// One pull-collide step of every active cell of the column: pull the moving
// populations from buffer B, collide all 19 in registers, write the moving
// post-collision values to buffer 1 - B at the cell itself.
template <int BLOCK, bool FORCH, int B>
__device__ __forceinline__ void gray_step(GrayShared<BLOCK>& sh, float (&g)[Q], const int (&src)[NMOV],
                                          const float (&add)[NMOV], bool lid, const GrayCell& c, float rho_inv,
                                          float w3r_axis, float w3r_edge, int z, float& ux, float& uy, float& uz) {
#pragma clang fp contract(off)
#pragma unroll
    for (int m = 0; m < NMOV; ++m) g[MOVK[m]] = (&sh.mv[B][0][0])[src[m]];
    if (lid) {
#pragma unroll
        for (int m = 0; m < NMOV; ++m) g[MOVK[m]] += add[m];
    }
    float gp2[9], gm2[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        gp2[p] = g[2 * p + 1] + g[2 * p + 2];
        gm2[p] = g[2 * p + 1] - g[2 * p + 2];
    }
    float drho = g[0], jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int k = 2 * p + 1;
        drho += gp2[p];
        if (L::ex[k] > 0) jx += gm2[p];
        if (L::ex[k] < 0) jx -= gm2[p];
        if (L::ey[k] > 0) jy += gm2[p];
        if (L::ey[k] < 0) jy -= gm2[p];
        if (L::ez[k] > 0) jz += gm2[p];
        if (L::ez[k] < 0) jz -= gm2[p];
    }
    const float vx = fmaf(jx, rho_inv, c.hGe[0]), vy = fmaf(jy, rho_inv, c.hGe[1]), vz = fmaf(jz, rho_inv, c.hGe[2]);
    float den = c.den;
    if (FORCH && c.phi != 0.0f) {
        const float c0 = 0.5f * (1.0f + 0.5f * c.D), c1 = 0.5f * c.phi;
        const float vn = sqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
        den = 1.0f / (c0 + sqrtf(fmaf(c0, c0, c1 * vn)));
    }
    ux = vx * den;
    uy = vy * den;
    uz = vz * den;
    float Fx = fmaf(-c.D, ux, c.Ge[0]), Fy = fmaf(-c.D, uy, c.Ge[1]), Fz = fmaf(-c.D, uz, c.Ge[2]);
    const float uu = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
    if (FORCH && c.phi != 0.0f) {
        const float pu = c.phi * sqrtf(uu);
        Fx = fmaf(-pu, ux, Fx);
        Fy = fmaf(-pu, uy, Fy);
        Fz = fmaf(-pu, uz, Fz);
    }
    const float uF = fmaf(ux, Fx, fmaf(uy, Fy, uz * Fz));
    // even part: dp = -wp gp + w [T0 + A (e.u (4.5 wp e.u + 9 cpl e.F) + T1)]
    // odd part:  dm = -wm gm + 3 rho0 w (wm e.u + cmi e.F)
    const float T0 = c.wp * drho;
    const float T1 = fmaf(c.m15wp, uu, c.m3cpl * uF);
    g[0] = fmaf(c.omwp, g[0], fmaf(c.A, T1, T0) * (1.0f / 3.0f));
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int k = 2 * p + 1;
        const float w = (float)weight(k);
        const float w3r = norm2(k) == 1 ? w3r_axis : w3r_edge;
        float eu = 0.0f, eF = 0.0f;
        if (L::ex[k]) { eu = L::ex[k] > 0 ? ux : -ux; eF = L::ex[k] > 0 ? Fx : -Fx; }
        if (L::ey[k]) {
            eu = L::ex[k] ? (L::ey[k] > 0 ? eu + uy : eu - uy) : (L::ey[k] > 0 ? uy : -uy);
            eF = L::ex[k] ? (L::ey[k] > 0 ? eF + Fy : eF - Fy) : (L::ey[k] > 0 ? Fy : -Fy);
        }
        if (L::ez[k]) {
            const bool first = !L::ex[k] && !L::ey[k];
            eu = first ? (L::ez[k] > 0 ? uz : -uz) : (L::ez[k] > 0 ? eu + uz : eu - uz);
            eF = first ? (L::ez[k] > 0 ? Fz : -Fz) : (L::ez[k] > 0 ? eF + Fz : eF - Fz);
        }
        const float X = fmaf(c.c45, eu, c.c9 * eF);
        const float Z = fmaf(c.A, fmaf(eu, X, T1), T0);
        const float dp = fmaf(-c.hwp, gp2[p], w * Z);
        const float dm = fmaf(-c.hwm, gm2[p], w3r * fmaf(c.wm, eu, c.cmi * eF));
        g[k] = (g[k] + dp) + dm;
        g[k + 1] = (g[k + 1] + dp) - dm;
    }
#pragma unroll
    for (int m = 0; m < NMOV; ++m) sh.mv[1 - B][m][z] = g[MOVK[m]];
}

template <int BLOCK, bool FORCH>
__global__ void __launch_bounds__(BLOCK) k_gray(GrayArgs a) {
#pragma clang fp contract(off)
    __shared__ GrayShared<BLOCK> sh;
    const int col = blockIdx.x;
    const int z = threadIdx.x;
    const int nz = a.nz;
    const bool live = z < nz;
    const bool active = live && !(a.walls && (z == 0 || z == nz - 1));
    float* gs = a.state + (int64_t)col * Q * nz;
    float g[Q];
    GrayCell c{};
    {
        float eps = 1.0f, wp = 1.0f, wm = 1.0f, D = 0.0f;
        if (live) {
            const float* cp = a.cell + ((int64_t)col * nz + z) * 4;
            eps = cp[0]; wp = cp[1]; wm = cp[2]; D = cp[3];
            if (FORCH) c.phi = a.phi[(int64_t)col * nz + z];
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) g[k] = live ? gs[k * nz + z] : 0.0f;
        const float cpl = 1.0f - 0.5f * wp;
        c.D = D;
        c.wp = wp;
        c.wm = wm;
        c.cmi = 1.0f - 0.5f * wm;
        c.hwp = 0.5f * wp;
        c.hwm = 0.5f * wm;
        c.omwp = 1.0f - wp;
        c.A = a.rho0 * (1.0f / eps);
        c.c45 = 4.5f * wp;
        c.c9 = 9.0f * cpl;
        c.m15wp = -1.5f * wp;
        c.m3cpl = -3.0f * cpl;
        c.den = 1.0f / (1.0f + 0.5f * D);
        for (int i = 0; i < 3; ++i) {
            c.Ge[i] = eps * a.G[i];
            c.hGe[i] = 0.5f * c.Ge[i];
        }
    }
    // pull sources of the moving populations: the neighbour cell (periodic
    // in z), or this cell's opposite population where the neighbour is a wall
    // layer (half-way bounce-back, plus the moving-wall term at the top)
    int src[NMOV];
    float add[NMOV];
#pragma unroll
    for (int m = 0; m < NMOV; ++m) {
        const int k = MOVK[m];
        int zs = z - L::ez[k];
        add[m] = 0.0f;
        if (!active) {
            src[m] = m * BLOCK + z;
        } else if (a.walls && (zs == 0 || zs == nz - 1)) {
            src[m] = (m ^ 1) * BLOCK + z;
            if (zs == nz - 1) add[m] = a.wterm[k];
        } else {
            zs = zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs);
            src[m] = m * BLOCK + zs;
        }
        sh.mv[0][m][z] = g[k];
    }
    const bool lid = a.lid != 0;
    const float rho_inv = 1.0f / a.rho0;
    const float w3r_axis = 3.0f * a.rho0 * (float)(1.0 / 18.0), w3r_edge = 3.0f * a.rho0 * (float)(1.0 / 36.0);
    float ux = 0.0f, uy = 0.0f, uz = 0.0f;
    const int64_t s0 = a.steps[col];
    int64_t s = s0;
    int until_check = a.check_every;
    bool stop = a.nsteps <= 0 || (a.steady && a.status[col] != 0);
    __syncthreads();
    // after each step: the barrier that orders this step's writes before the
    // next step's reads, and, every check_every steps, the steady-state test
    // on the FP64 sum of u_x (per-wavefront butterflies, then the wavefront
    // sums in order)
    auto finish = [&]() {
        ++s;
        stop = s - s0 >= a.nsteps;
        if (a.steady && --until_check == 0) {
            until_check = a.check_every;
            double v = active ? (double)ux : 0.0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if ((z & 63) == 0) sh.red[z >> 6] = v;
            __syncthreads();
            if (z == 0) {
                double U = 0.0;
                for (int w = 0; w < BLOCK / 64; ++w) U += sh.red[w];
                const double Up = a.uprev[col];
                int st = 0;
                if (!(fabs(U) < 0.4 * nz)) st = -1;
                else if (fabs(U - Up) <= a.tol * fabs(U)) st = 1;
                a.uprev[col] = U;
                if (st != 0) a.status[col] = st;
                sh.stop = st;
            }
            __syncthreads();
            if (sh.stop != 0) stop = true;
        } else {
            __syncthreads();
        }
    };
    while (!stop) {
        if (active) gray_step<BLOCK, FORCH, 0>(sh, g, src, add, lid, c, rho_inv, w3r_axis, w3r_edge, z, ux, uy, uz);
        finish();
        if (stop) break;
        if (active) gray_step<BLOCK, FORCH, 1>(sh, g, src, add, lid, c, rho_inv, w3r_axis, w3r_edge, z, ux, uy, uz);
        finish();
    }
    // every thread holds its own cell's post-collision populations
    if (live) {
#pragma unroll
        for (int k = 0; k < Q; ++k) gs[k * nz + z] = g[k];
        double* uo = a.u + ((int64_t)col * nz + z) * 3;
        uo[0] = ux; uo[1] = uy; uo[2] = uz;
    }
    if (z == 0) a.steps[col] = s;
}

int64_t align_up(int64_t v, int64_t al) { return (v + al - 1) / al * al; }

}  // namespace
}  // namespace lbm

using namespace lbm;

struct gray_ctx {
    int ncols = 0, nz = 0, walls = 0;
    hipStream_t stream = nullptr;
    char* buf = nullptr;
    int64_t off_state = 0, off_cell = 0, off_phi = 0, off_u = 0, off_steps = 0, off_uprev = 0, off_status = 0;
    GrayArgs args{};
    double lambda = 3.0 / 16.0, rho0 = 1.0;
    std::vector<int64_t> steps;
};

namespace {

struct GPlan {
    int64_t state, cell, phi, u, steps, uprev, status, total;
};

GPlan gplan(int ncols, int nz) {
    GPlan P{};
    int64_t o = 0;
    P.state = o; o = align_up(o + (int64_t)ncols * Q * nz * 4, 256);
    P.cell = o; o = align_up(o + (int64_t)ncols * nz * 16, 256);
    P.phi = o; o = align_up(o + (int64_t)ncols * nz * 4, 256);
    P.u = o; o = align_up(o + (int64_t)ncols * nz * 24, 256);
    P.steps = o; o = align_up(o + (int64_t)ncols * 8, 256);
    P.uprev = o; o = align_up(o + (int64_t)ncols * 8, 256);
    P.status = o; o = align_up(o + (int64_t)ncols * 4, 256);
    P.total = o;
    return P;
}

#define GCHK(expr, what)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return set_error(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

lbm_status upload_cells(gray_ctx* c, const double* eps, const double* nu_eff, const double* drag) {
    const int64_t n = (int64_t)c->ncols * c->nz;
    std::vector<float> cell((size_t)n * 4);
    for (int64_t i = 0; i < n; ++i) {
        if (!(eps[i] > 0.0 && eps[i] <= 1.0)) return set_error(LBM_E_INVAL, "porosity must lie in (0, 1]");
        if (!(nu_eff[i] > 0.0) || !std::isfinite(nu_eff[i])) return set_error(LBM_E_INVAL, "nu_eff must be positive");
        if (!(drag[i] >= 0.0) || !std::isfinite(drag[i])) return set_error(LBM_E_INVAL, "drag must be >= 0");
        const double tp = 3.0 * nu_eff[i] + 0.5;
        const double tm = 0.5 + c->lambda / (tp - 0.5);
        const double wp = 1.0 / tp, wm = 1.0 / tm;
        if (!(wm > 0.0 && wm < 2.0)) return set_error(LBM_E_INVAL, "omega- outside (0, 2)");
        cell[4 * i + 0] = (float)eps[i];
        cell[4 * i + 1] = (float)wp;
        cell[4 * i + 2] = (float)wm;
        cell[4 * i + 3] = (float)drag[i];
    }
    GCHK(hipMemcpyAsync(c->buf + c->off_cell, cell.data(), cell.size() * 4, hipMemcpyHostToDevice, c->stream),
         "upload cell parameters");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    return LBM_OK;
}

lbm_status launch(gray_ctx* c) {
    const int block = (int)align_up(c->nz, 64);
    const bool forch = c->args.phi != nullptr;
    hipError_t e;
    switch (block) {
#define GB(B)                                                                       \
    case B:                                                                         \
        if (forch) k_gray<B, true><<<c->ncols, B, 0, c->stream>>>(c->args);         \
        else k_gray<B, false><<<c->ncols, B, 0, c->stream>>>(c->args);              \
        break;
        GB(64) GB(128) GB(192) GB(256) GB(320) GB(384) GB(448) GB(512) GB(576) GB(640) GB(704)
#undef GB
        default: return set_error(LBM_E_INVAL, "column height must be at most 704");
    }
    e = hipGetLastError();
    GCHK(e, "gray launch");
    c->steps.assign(c->ncols, 0);
    GCHK(hipMemcpyAsync(c->steps.data(), c->buf + c->off_steps, c->ncols * 8, hipMemcpyDeviceToHost, c->stream),
         "read steps");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status gray_required_bytes(int32_t ncols, int32_t nz, int64_t* bytes) {
    // two buffers of the ten moving populations (80 B per cell, nz rounded up
    // to a multiple of 64) and the reduction buffer must fit the 64 KB of LDS
    // a workgroup gets without opting in to more
    if (ncols < 1 || nz < 3 || nz > 704 || !bytes) return set_error(LBM_E_INVAL, "need ncols >= 1 and 3 <= nz <= 704");
    *bytes = gplan(ncols, nz).total;
    return LBM_OK;
}

lbm_status gray_init(int32_t ncols, int32_t nz, int32_t walls, const double* eps, const double* nu_eff,
                     const double* drag, double magic_lambda, double rho0, const double* G, const double* lid,
                     void* dev_buf, int64_t bytes, void* hip_stream, gray_ctx** out) {
    if (!out || !eps || !nu_eff || !drag || !G || !dev_buf) return set_error(LBM_E_INVAL, "bad arguments");
    *out = nullptr;
    int64_t need = 0;
    lbm_status s = gray_required_bytes(ncols, nz, &need);
    if (s != LBM_OK) return s;
    if (bytes < need) return set_error(LBM_E_NOMEM, "device buffer smaller than gray_required_bytes");
    if (!(rho0 > 0.0) || !(magic_lambda > 0.0)) return set_error(LBM_E_INVAL, "rho0 and Lambda must be positive");
    auto* c = new gray_ctx;
    c->ncols = ncols; c->nz = nz; c->walls = walls ? 1 : 0;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->buf = reinterpret_cast<char*>(dev_buf);
    c->lambda = magic_lambda; c->rho0 = rho0;
    const GPlan P = gplan(ncols, nz);
    c->off_state = P.state; c->off_cell = P.cell; c->off_u = P.u; c->off_steps = P.steps; c->off_uprev = P.uprev;
    c->off_status = P.status;
    c->off_phi = P.phi;
    GrayArgs& a = c->args;
    a.phi = nullptr;
    a.state = reinterpret_cast<float*>(c->buf + P.state);
    a.cell = reinterpret_cast<const float*>(c->buf + P.cell);
    a.u = reinterpret_cast<double*>(c->buf + P.u);
    a.steps = reinterpret_cast<int64_t*>(c->buf + P.steps);
    a.uprev = reinterpret_cast<double*>(c->buf + P.uprev);
    a.status = reinterpret_cast<int32_t*>(c->buf + P.status);
    a.nz = nz; a.walls = c->walls;
    a.rho0 = (float)rho0;
    for (int i = 0; i < 3; ++i) a.G[i] = (float)G[i];
    const double zero[3] = {0, 0, 0};
    const double* lw = lid ? lid : zero;
    for (int k = 0; k < Q; ++k)
        a.wterm[k] = (float)(6.0 * weight(k) * rho0 * (D3Q19::ex[k] * lw[0] + D3Q19::ey[k] * lw[1] + D3Q19::ez[k] * lw[2]));
    a.lid = (lw[0] != 0.0 || lw[1] != 0.0 || lw[2] != 0.0) ? 1 : 0;
    s = upload_cells(c, eps, nu_eff, drag);
    if (s == LBM_OK) s = gray_reset(c);
    if (s != LBM_OK) { delete c; return s; }
    *out = c;
    return LBM_OK;
}

lbm_status gray_reset(gray_ctx* c) {
    if (!c) return set_error(LBM_E_INVAL, "null context");
    std::vector<double> nanv(c->ncols, NAN);
    GCHK(hipMemsetAsync(c->buf + c->off_state, 0, (size_t)c->ncols * Q * c->nz * 4, c->stream), "zero state");
    GCHK(hipMemsetAsync(c->buf + c->off_u, 0, (size_t)c->ncols * c->nz * 24, c->stream), "zero profile");
    GCHK(hipMemsetAsync(c->buf + c->off_steps, 0, (size_t)c->ncols * 8, c->stream), "zero steps");
    GCHK(hipMemsetAsync(c->buf + c->off_status, 0, (size_t)c->ncols * 4, c->stream), "zero status");
    GCHK(hipMemcpyAsync(c->buf + c->off_uprev, nanv.data(), c->ncols * 8, hipMemcpyHostToDevice, c->stream), "history");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    c->steps.assign(c->ncols, 0);
    return LBM_OK;
}

lbm_status gray_set_cells(gray_ctx* c, const double* eps, const double* nu_eff, const double* drag) {
    if (!c || !eps || !nu_eff || !drag) return set_error(LBM_E_INVAL, "bad arguments");
    return upload_cells(c, eps, nu_eff, drag);
}

lbm_status gray_set_forchheimer(gray_ctx* c, const double* phi) {
    if (!c) return set_error(LBM_E_INVAL, "null context");
    if (!phi) {
        c->args.phi = nullptr;
        return LBM_OK;
    }
    const int64_t n = (int64_t)c->ncols * c->nz;
    std::vector<float> f((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (!(phi[i] >= 0.0) || !std::isfinite(phi[i])) return set_error(LBM_E_INVAL, "Forchheimer coefficients must be >= 0");
        f[i] = (float)phi[i];
    }
    GCHK(hipMemcpyAsync(c->buf + c->off_phi, f.data(), f.size() * 4, hipMemcpyHostToDevice, c->stream),
         "upload Forchheimer coefficients");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    c->args.phi = reinterpret_cast<const float*>(c->buf + c->off_phi);
    return LBM_OK;
}

lbm_status gray_run(gray_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return set_error(LBM_E_INVAL, "bad arguments");
    c->args.steady = 0;
    c->args.nsteps = nsteps;
    c->args.check_every = 1;
    c->args.tol = 0.0;
    return launch(c);
}

lbm_status gray_run_to_steady(gray_ctx* c, double rel_tol, int64_t check_every, int64_t max_steps,
                              int64_t* steps_done) {
    if (!c || !(rel_tol >= 0.0) || check_every < 1 || check_every > (1 << 30) || max_steps < 0)
        return set_error(LBM_E_INVAL, "bad arguments");
    c->args.steady = 1;
    c->args.nsteps = max_steps;
    c->args.check_every = (int32_t)check_every;
    c->args.tol = rel_tol;
    lbm_status s = launch(c);
    if (s != LBM_OK) return s;
    if (steps_done) std::memcpy(steps_done, c->steps.data(), c->ncols * 8);
    std::vector<int32_t> st(c->ncols);
    GCHK(hipMemcpyAsync(st.data(), c->buf + c->off_status, c->ncols * 4, hipMemcpyDeviceToHost, c->stream), "status");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    for (int i = 0; i < c->ncols; ++i)
        if (st[i] < 0) return set_error(LBM_E_UNSTABLE, "gray column " + std::to_string(i) + " became unstable");
    return LBM_OK;
}

lbm_status gray_profile(gray_ctx* c, int32_t col, double* u) {
    if (!c || !u || col < 0 || col >= c->ncols) return set_error(LBM_E_INVAL, "bad arguments");
    GCHK(hipMemcpyAsync(u, c->buf + c->off_u + (int64_t)col * c->nz * 24, (size_t)c->nz * 24, hipMemcpyDeviceToHost,
                        c->stream), "copy profile");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    return LBM_OK;
}

void gray_destroy(gray_ctx* c) { delete c; }

}  // extern "C"
