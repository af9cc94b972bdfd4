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
// kernel.  The working precision is FP64 by default: in FP32 the column
// stops changing 1e-4 to 3e-3 (relative) short of its steady state, once the
// remaining per-step updates fall below the FP32 resolution of the
// populations; FP32 is kept as an option.  Every population stays in its
// thread's registers: the nine with e_z = 0 never leave their cell in a
// 1 x 1 periodic column, and the ten with e_z != 0 move one cell per step
// through LDS (every cell writes them to one of two buffers and pulls its
// neighbours' from the other: one barrier per step; 2 x 10 x 704 x 8 bytes
// at the largest column in FP64, which gfx950's LDS holds).  Global memory
// is touched only to load and store the state and to write the final
// profile.  The steady-state test (relative change of the FP64 sum of u_x
// over check_every steps) is evaluated in the kernel with a fixed-order
// workgroup reduction.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gray.h"
#include "internal.hpp"

namespace lbm {

struct GrayArgs {
    double* state;         // ncols x 19 x nz
    const double* cell;    // ncols x nz x 4: eps, omega+, omega-, D
    const double* phi;     // ncols x nz Forchheimer coefficients, or null (all zero)
    double* u;             // ncols x nz x 3
    int64_t* steps;        // per column
    double* uprev;         // per column
    int32_t* status;       // per column: 0 running, 1 converged, -1 unstable
    int32_t nz, walls, steady, check_every, lid;
    int64_t nsteps;
    double tol;
    double rho0, G[3];
    double wterm[Q];
};

namespace {

using L = D3Q19;

// the populations with e_z = +1 (pulled from the cell below) and, in the same
// order, their opposites with e_z = -1 (pulled from the cell above)
constexpr int NUP = 5;
__host__ __device__ constexpr int upk(int i) { return i == 0 ? 5 : (i == 1 ? 11 : (i == 2 ? 14 : (i == 3 ? 15 : 18))); }
__host__ __device__ constexpr int dnk(int i) { return opp(upk(i)); }

// per-cell constants of the collision
template <class T>
struct GrayCell {
    T D, phi, wp, omwp, A, c45, c9, m15wp, m3cpl, den;
    T hp, hm;                  // (1 - omega+)/2, (1 - omega-)/2
    T wA_axis, wA_edge;        // w A per velocity class
    T wmr_axis, wmr_edge;      // 3 rho0 w wm
    T mF_axis, mF_edge;        // 3 rho0 w cmi
    T Ge[3], hGe[3];
};

// Every cell's moving populations in LDS, two buffers: slot i < NUP holds
// direction upk(i), slot NUP + i direction dnk(i).
template <int BLOCK, class T>
struct GrayShared {
    T mv[2][2 * NUP][BLOCK];
    double red[BLOCK / 64];
    int stop;
};

template <int BLOCK, class T>
__device__ __forceinline__ void publish(GrayShared<BLOCK, T>& sh, int buf, const T (&g)[Q], int z) {
#pragma unroll
    for (int i = 0; i < NUP; ++i) {
        sh.mv[buf][i][z] = g[upk(i)];
        sh.mv[buf][NUP + i][z] = g[dnk(i)];
    }
}

// offu / offd: where an active cell's e_z = +1 / -1 populations come from,
// as offsets of slot 0 / NUP: the neighbour cell (periodic), or, next to a
// wall layer, the cell's own opposite slot (half-way bounce-back)
template <int B, int BLOCK, class T>
__device__ __forceinline__ void pull(GrayShared<BLOCK, T>& sh, T (&g)[Q], bool active, bool lid, const T (&wt)[NUP],
                                     int offu, int offd) {
    if (active) {
        const T* m = &sh.mv[B][0][0];
#pragma unroll
        for (int i = 0; i < NUP; ++i) {
            g[upk(i)] = m[i * BLOCK + offu];
            g[dnk(i)] = m[(NUP + i) * BLOCK + offd];
        }
        // the moving-wall term (zero but in the cell below the top wall);
        // lid is uniform over the launch, so the branch costs nothing
        // without a moving wall
        if (lid) {
#pragma unroll
            for (int i = 0; i < NUP; ++i) g[dnk(i)] += wt[i];
        }
    }
}

// One pull-collide step of the column: the pull from buffer B (plus the
// moving-wall term at the top), the collision of the active cells, and the
// moving post-collision values to buffer 1 - B.
template <int BLOCK, bool FORCH, int B, class T>
__device__ __forceinline__ void gray_step(GrayShared<BLOCK, T>& sh, T (&g)[Q], bool active, bool lid,
                                          const T (&wt)[NUP], int offu, int offd, const GrayCell<T>& c, T rho_inv,
                                          int z, T& ux, T& uy, T& uz) {
#pragma clang fp contract(off)
    pull<B>(sh, g, active, lid, wt, offu, offd);
    if (active) {
        T gp2[9], gm2[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            gp2[p] = g[2 * p + 1] + g[2 * p + 2];
            gm2[p] = g[2 * p + 1] - g[2 * p + 2];
        }
        // momentum: signed sums of the gm2 terms, each started from its
        // first term rather than from zero
        T drho = g[0], j[3] = {T(0), T(0), T(0)};
        bool started[3] = {false, false, false};
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int k = 2 * p + 1;
            drho += gp2[p];
            const int e[3] = {L::ex[k], L::ey[k], L::ez[k]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (e[d] == 0) continue;
                if (!started[d]) j[d] = e[d] > 0 ? gm2[p] : -gm2[p];
                else j[d] = e[d] > 0 ? j[d] + gm2[p] : j[d] - gm2[p];
                started[d] = true;
            }
        }
        const T jx = j[0], jy = j[1], jz = j[2];
        const T vx = fma(jx, rho_inv, c.hGe[0]), vy = fma(jy, rho_inv, c.hGe[1]), vz = fma(jz, rho_inv, c.hGe[2]);
        T den = c.den;
        if (FORCH && c.phi != T(0)) {
            const T c0 = T(0.5) * (T(1) + T(0.5) * c.D), c1 = T(0.5) * c.phi;
            const T vn = sqrt(fma(vx, vx, fma(vy, vy, vz * vz)));
            den = T(1) / (c0 + sqrt(fma(c0, c0, c1 * vn)));
        }
        ux = vx * den;
        uy = vy * den;
        uz = vz * den;
        T Fx = fma(-c.D, ux, c.Ge[0]), Fy = fma(-c.D, uy, c.Ge[1]), Fz = fma(-c.D, uz, c.Ge[2]);
        const T uu = fma(ux, ux, fma(uy, uy, uz * uz));
        if (FORCH && c.phi != T(0)) {
            const T pu = c.phi * sqrt(uu);
            Fx = fma(-pu, ux, Fx);
            Fy = fma(-pu, uy, Fy);
            Fz = fma(-pu, uz, Fz);
        }
        const T uF = fma(ux, Fx, fma(uy, Fy, uz * Fz));
        // Pair (k, kb = opp(k)) with gp = (g_k + g_kb)/2, gm = (g_k - g_kb)/2:
        //   even part dp = -wp gp + Wp,  Wp = w [T0 + A (e.u (4.5 wp e.u + 9 cpl e.F) + T1)]
        //   odd part  dm = -wm gm + Wm,  Wm = 3 rho0 w (wm e.u + cmi e.F)
        //   g_k'  = (gp + dp) + (gm + dm) = P + M
        //   g_kb' = (gp + dp) - (gm + dm) = P - M
        // with P = hp gp2 + Wp, M = hm gm2 + Wm, gp2 = 2 gp, gm2 = 2 gm,
        // hp = (1 - wp)/2, hm = (1 - wm)/2; the weights w and 3 rho0 w are
        // folded into per-class (axis / edge) constants.
        const T T0 = c.wp * drho;
        const T T1 = fma(c.m15wp, uu, c.m3cpl * uF);
        g[0] = fma(c.omwp, g[0], fma(c.A, T1, T0) * T(1.0 / 3.0));
        const T H[3] = {c.c9 * Fx, c.c9 * Fy, c.c9 * Fz};                   // 9 cpl F
        const T Ma[3] = {c.mF_axis * Fx, c.mF_axis * Fy, c.mF_axis * Fz};   // 3 rho0 w cmi F, axis
        const T Me[3] = {c.mF_edge * Fx, c.mF_edge * Fy, c.mF_edge * Fz};   // same, edge
        const T wT0_axis = T(1.0 / 18.0) * T0, wT0_edge = T(1.0 / 36.0) * T0;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int k = 2 * p + 1;
            const bool axis = norm2(k) == 1;
            const int e[3] = {L::ex[k], L::ey[k], L::ez[k]};
            const T uc[3] = {ux, uy, uz};
            // e.u, 9 cpl e.F and 3 rho0 w cmi e.F as signed sums of the nonzero components
            T eu = T(0), hF = T(0), mF = T(0);
            bool first = true;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (e[d] == 0) continue;
                if (first) {
                    eu = e[d] > 0 ? uc[d] : -uc[d];
                    hF = e[d] > 0 ? H[d] : -H[d];
                    mF = e[d] > 0 ? (axis ? Ma[d] : Me[d]) : -(axis ? Ma[d] : Me[d]);
                    first = false;
                } else {
                    eu = e[d] > 0 ? eu + uc[d] : eu - uc[d];
                    hF = e[d] > 0 ? hF + H[d] : hF - H[d];
                    mF = e[d] > 0 ? mF + (axis ? Ma[d] : Me[d]) : mF - (axis ? Ma[d] : Me[d]);
                }
            }
            const T X = fma(c.c45, eu, hF);
            const T Wp = fma(axis ? c.wA_axis : c.wA_edge, fma(eu, X, T1), axis ? wT0_axis : wT0_edge);
            const T Wm = fma(axis ? c.wmr_axis : c.wmr_edge, eu, mF);
            const T P = fma(c.hp, gp2[p], Wp), M = fma(c.hm, gm2[p], Wm);
            g[k] = P + M;
            g[k + 1] = P - M;
        }
    }
    publish(sh, 1 - B, g, z);
}

template <int BLOCK, bool FORCH, class T>
__global__ void __launch_bounds__(BLOCK) k_gray(GrayArgs a) {
#pragma clang fp contract(off)
    __shared__ GrayShared<BLOCK, T> sh;
    const int col = blockIdx.x;
    const int z = threadIdx.x;
    const int nz = a.nz;
    const bool live = z < nz;
    const bool walls = a.walls != 0;
    const bool active = live && !(walls && (z == 0 || z == nz - 1));
    double* gs = a.state + (int64_t)col * Q * nz;
    T g[Q];
    GrayCell<T> c{};
    {
        double eps = 1.0, wp = 1.0, wm = 1.0, D = 0.0;
        if (live) {
            const double* cp = a.cell + ((int64_t)col * nz + z) * 4;
            eps = cp[0]; wp = cp[1]; wm = cp[2]; D = cp[3];
            if (FORCH) c.phi = T(a.phi[(int64_t)col * nz + z]);
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) g[k] = live ? T(gs[k * nz + z]) : T(0);
        // constants formed in FP64, then rounded once to the working precision
        const double cpl = 1.0 - 0.5 * wp, cmi = 1.0 - 0.5 * wm;
        const double r3a = 3.0 * a.rho0 * (1.0 / 18.0), r3e = 3.0 * a.rho0 * (1.0 / 36.0);
        const double A = a.rho0 * (1.0 / eps);
        c.D = T(D);
        c.wp = T(wp);
        c.omwp = T(1.0 - wp);
        c.A = T(A);
        c.c45 = T(4.5 * wp);
        c.c9 = T(9.0 * cpl);
        c.m15wp = T(-1.5 * wp);
        c.m3cpl = T(-3.0 * cpl);
        c.den = T(1.0 / (1.0 + 0.5 * D));
        c.hp = T(0.5 * (1.0 - wp));
        c.hm = T(0.5 * (1.0 - wm));
        c.wA_axis = T((1.0 / 18.0) * A);
        c.wA_edge = T((1.0 / 36.0) * A);
        c.wmr_axis = T(r3a * wm);
        c.wmr_edge = T(r3e * wm);
        c.mF_axis = T(r3a * cmi);
        c.mF_edge = T(r3e * cmi);
        for (int i = 0; i < 3; ++i) {
            c.Ge[i] = T(eps * a.G[i]);
            c.hGe[i] = T(0.5 * eps * a.G[i]);
        }
    }
    const bool lid = a.lid != 0;
    // the moving-wall term of the populations pulled from the top wall, in
    // the cell below it only
    T wt[NUP];
    const bool top = lid && walls && z == nz - 2;
#pragma unroll
    for (int i = 0; i < NUP; ++i) wt[i] = top ? T(a.wterm[dnk(i)]) : T(0);
    int offu = z - 1, offd = z + 1;
    if (walls && offu == 0) offu = NUP * BLOCK + z;
    else if (offu < 0) offu += nz;
    if (walls && offd == nz - 1) offd = z - NUP * BLOCK;
    else if (offd >= nz) offd -= nz;
    const T rho_inv = T(1.0 / a.rho0);
    T ux = T(0), uy = T(0), uz = T(0);
    const int64_t s0 = a.steps[col];
    int64_t s = s0;
    int until_check = a.check_every;
    bool stop = a.nsteps <= 0 || (a.steady && a.status[col] != 0);
    publish(sh, 0, g, z);
    __syncthreads();
    // after each step: the barrier that orders this step's boundary values
    // before the next step's reads, and, every check_every steps, the
    // steady-state test on the FP64 sum of u_x (per-wavefront butterflies,
    // then the wavefront sums in order)
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
        gray_step<BLOCK, FORCH, 0, T>(sh, g, active, lid, wt, offu, offd, c, rho_inv, z, ux, uy, uz);
        finish();
        if (stop) break;
        gray_step<BLOCK, FORCH, 1, T>(sh, g, active, lid, wt, offu, offd, c, rho_inv, z, ux, uy, uz);
        finish();
    }
    // every thread holds its own cell's post-collision populations
    if (live) {
#pragma unroll
        for (int k = 0; k < Q; ++k) gs[k * nz + z] = (double)g[k];
        double* uo = a.u + ((int64_t)col * nz + z) * 3;
        uo[0] = (double)ux; uo[1] = (double)uy; uo[2] = (double)uz;
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
    int precision = 64;  // working precision of the kernel, 64 or 32 bits
    std::vector<int64_t> steps;
};

namespace {

struct GPlan {
    int64_t state, cell, phi, u, steps, uprev, status, total;
};

GPlan gplan(int ncols, int nz) {
    GPlan P{};
    int64_t o = 0;
    P.state = o; o = align_up(o + (int64_t)ncols * Q * nz * 8, 256);
    P.cell = o; o = align_up(o + (int64_t)ncols * nz * 32, 256);
    P.phi = o; o = align_up(o + (int64_t)ncols * nz * 8, 256);
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
    std::vector<double> cell((size_t)n * 4);
    for (int64_t i = 0; i < n; ++i) {
        if (!(eps[i] > 0.0 && eps[i] <= 1.0)) return set_error(LBM_E_INVAL, "porosity must lie in (0, 1]");
        if (!(nu_eff[i] > 0.0) || !std::isfinite(nu_eff[i])) return set_error(LBM_E_INVAL, "nu_eff must be positive");
        if (!(drag[i] >= 0.0) || !std::isfinite(drag[i])) return set_error(LBM_E_INVAL, "drag must be >= 0");
        const double tp = 3.0 * nu_eff[i] + 0.5;
        const double tm = 0.5 + c->lambda / (tp - 0.5);
        const double wp = 1.0 / tp, wm = 1.0 / tm;
        if (!(wm > 0.0 && wm < 2.0)) return set_error(LBM_E_INVAL, "omega- outside (0, 2)");
        cell[4 * i + 0] = eps[i];
        cell[4 * i + 1] = wp;
        cell[4 * i + 2] = wm;
        cell[4 * i + 3] = drag[i];
    }
    GCHK(hipMemcpyAsync(c->buf + c->off_cell, cell.data(), cell.size() * 8, hipMemcpyHostToDevice, c->stream),
         "upload cell parameters");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    return LBM_OK;
}

lbm_status launch(gray_ctx* c) {
    const int block = (int)align_up(c->nz, 64);
    const bool forch = c->args.phi != nullptr;
    const bool fp64 = c->precision == 64;
    hipError_t e;
    switch (block) {
#define GB(B)                                                                                 \
    case B:                                                                                   \
        if (fp64 && forch) k_gray<B, true, double><<<c->ncols, B, 0, c->stream>>>(c->args);   \
        else if (fp64) k_gray<B, false, double><<<c->ncols, B, 0, c->stream>>>(c->args);      \
        else if (forch) k_gray<B, true, float><<<c->ncols, B, 0, c->stream>>>(c->args);       \
        else k_gray<B, false, float><<<c->ncols, B, 0, c->stream>>>(c->args);                 \
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
    // the column is one workgroup of nz rounded up to a multiple of 64
    // threads, at most 704 (eleven wavefronts, three per SIMD)
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
    a.state = reinterpret_cast<double*>(c->buf + P.state);
    a.cell = reinterpret_cast<const double*>(c->buf + P.cell);
    a.u = reinterpret_cast<double*>(c->buf + P.u);
    a.steps = reinterpret_cast<int64_t*>(c->buf + P.steps);
    a.uprev = reinterpret_cast<double*>(c->buf + P.uprev);
    a.status = reinterpret_cast<int32_t*>(c->buf + P.status);
    a.nz = nz; a.walls = c->walls;
    a.rho0 = rho0;
    for (int i = 0; i < 3; ++i) a.G[i] = G[i];
    const double zero[3] = {0, 0, 0};
    const double* lw = lid ? lid : zero;
    for (int k = 0; k < Q; ++k)
        a.wterm[k] = 6.0 * weight(k) * rho0 * (D3Q19::ex[k] * lw[0] + D3Q19::ey[k] * lw[1] + D3Q19::ez[k] * lw[2]);
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
    GCHK(hipMemsetAsync(c->buf + c->off_state, 0, (size_t)c->ncols * Q * c->nz * 8, c->stream), "zero state");
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
    std::vector<double> f((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (!(phi[i] >= 0.0) || !std::isfinite(phi[i])) return set_error(LBM_E_INVAL, "Forchheimer coefficients must be >= 0");
        f[i] = phi[i];
    }
    GCHK(hipMemcpyAsync(c->buf + c->off_phi, f.data(), f.size() * 8, hipMemcpyHostToDevice, c->stream),
         "upload Forchheimer coefficients");
    GCHK(hipStreamSynchronize(c->stream), "synchronise");
    c->args.phi = reinterpret_cast<const double*>(c->buf + c->off_phi);
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

lbm_status gray_set_precision(gray_ctx* c, int32_t bits) {
    if (!c || (bits != 32 && bits != 64)) return set_error(LBM_E_INVAL, "precision must be 32 or 64 bits");
    c->precision = bits;
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
