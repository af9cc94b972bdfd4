// Learned closure network of the gray model: forward, backward and Adam on
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation).
//
// Network: 33 porosities (zero-padded to 64) -> 128 -> 128 -> 128 -> 16 (2
// used), exact-erf GELU between layers.  A workgroup (4 wavefronts) carries
// 64 batch rows through every layer; wavefront w owns rows 16w..16w+15 and
// produces 16x16 output tiles, accumulating over K in steps of 32.
// Activations live in LDS as BF16 between layers; pre-activations (FP32) and
// activations (BF16) go to the workspace for the backward pass.
//
// Operand layout of one MFMA (16 x 16 output, K = 32): lane l supplies row
// (A) or column (B) l % 16 and the eight K entries 8*(l/16) .. 8*(l/16)+7;
// it receives output rows 4*(l/16) .. 4*(l/16)+3 of column l % 16.  A and B
// use the same K labelling, so the contraction is over all 32 entries.
//
// Weights: FP32 master vector (layout in include/mlp.h) plus a BF16 copy in
// two layouts, row-major [K][N] (for the data gradients dH = dZ W^T) and
// transposed [N][K] (for the forward products), so that every B operand is
// one 16-byte load.
//
// Backward: per workgroup, data gradients through the layers and per-
// workgroup partial weight and bias gradients (weight gradients contract
// over the workgroup's 64 rows on the matrix cores); a second kernel sums
// the partials over workgroups in a fixed order, so gradients are
// deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mlp.h"
#include "internal.hpp"

namespace lbm {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int IN = 64, HID = 128, OUTP = 16, ROWS = 64, THREADS = 256;
constexpr int OW1 = 0, OB1 = OW1 + IN * HID, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + HID * HID, OW4 = OB3 + HID, OB4 = OW4 + HID * OUTP, NP = OB4 + OUTP;
static_assert(NP == MLP_NPARAM, "parameter layout");

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// out[16w + i][n] for the wave's 16 rows = in[16 rows][K] x W^T; W^T given as
// [N][K] (contiguous K).  Calls f(row_in_block, col, value) for every output.
template <int K, class F>
__device__ __forceinline__ void gemm_rows(const bf16* in, const bf16* WT, int N, F&& f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = 16 * w + (lane & 15), kg = 8 * (lane >> 4);
    for (int nt = 0; nt < N / 16; ++nt) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < K / 32; ++ks) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(in + r * K + ks * 32 + kg);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(WT + (nt * 16 + (lane & 15)) * K + ks * 32 + kg);
            acc = mfma(a, b, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) f(16 * w + 4 * (lane >> 4) + j, nt * 16 + (lane & 15), acc[j]);
    }
}

template <bool TRAIN>
__global__ void __launch_bounds__(THREADS) k_forward(const float* __restrict__ pf, const bf16* __restrict__ pb,
                                                     const bf16* __restrict__ x, float* __restrict__ y,
                                                     float* __restrict__ zws, bf16* __restrict__ hws, int64_t B) {
    __shared__ __attribute__((aligned(16))) bf16 xin[ROWS * IN];
    __shared__ __attribute__((aligned(16))) bf16 h[2][ROWS * HID];
    const int64_t row0 = (int64_t)blockIdx.x * ROWS;
    const bf16* WT = pb + MLP_NPARAM;  // transposed copy
    for (int i = threadIdx.x; i < ROWS * IN / 8; i += THREADS)
        reinterpret_cast<bf16x8*>(xin)[i] = reinterpret_cast<const bf16x8*>(x + row0 * IN)[i];
    __syncthreads();
    auto hidden = [&](int layer, const bf16* in_lds, bf16* out_lds, auto kdim, int ow, int ob) {
        constexpr int K = decltype(kdim)::value;
        gemm_rows<K>(in_lds, WT + ow, HID, [&](int r, int n, float v) {
            const float zz = v + pf[ob + n];
            const float hh = gelu(zz);
            out_lds[r * HID + n] = (bf16)hh;
            if (TRAIN) {
                const int64_t g = (row0 + r) * HID + n;
                zws[(int64_t)layer * B * HID + g] = zz;
                hws[(int64_t)layer * B * HID + g] = (bf16)hh;
            }
        });
        __syncthreads();
    };
    hidden(0, xin, h[0], std::integral_constant<int, IN>{}, OW1, OB1);
    hidden(1, h[0], h[1], std::integral_constant<int, HID>{}, OW2, OB2);
    hidden(2, h[1], h[0], std::integral_constant<int, HID>{}, OW3, OB3);
    gemm_rows<HID>(h[0], WT + OW4, OUTP,
                   [&](int r, int n, float v) { y[(row0 + r) * OUTP + n] = v + pf[OB4 + n]; });
}

// Partial weight gradient of one workgroup: part[ow + k*N + n] =
// sum_rows A[row][k] * D[row][n] for A [64][K] and D [64][DS] (N <= DS
// columns used) in LDS; the contraction over the 64 rows runs on the MFMA.
template <int K, int N, int DS>
__device__ __forceinline__ void weight_grad(const bf16* A, const bf16* D, float* part, int ow) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kg = 8 * (lane >> 4);
    constexpr int MT = K / 16, NT = N / 16;
    for (int t = w; t < MT * NT; t += 4) {
        const int mt = t / NT, nt = t % NT;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < ROWS / 32; ++ks) {
            bf16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int row = ks * 32 + kg + j;
                a[j] = A[row * K + mt * 16 + (lane & 15)];
                b[j] = D[row * DS + nt * 16 + (lane & 15)];
            }
            acc = mfma(a, b, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            part[ow + (mt * 16 + 4 * (lane >> 4) + j) * N + nt * 16 + (lane & 15)] = acc[j];
    }
}

// dH[16 rows of the wave][k] = sum_n dZ[row][n] W[k][n]: A = dZ (LDS, [64][N]),
// B from the row-major W [K][N]; calls f(row, k, value).
template <int N, class F>
__device__ __forceinline__ void data_grad(const bf16* dZ, const bf16* W, int K, F&& f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = 16 * w + (lane & 15), kg = 8 * (lane >> 4);
    for (int kt = 0; kt < K / 16; ++kt) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ns = 0; ns < (N + 31) / 32; ++ns) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(dZ + r * 32 * ((N + 31) / 32) + ns * 32 + kg);
            bf16x8 b;
            if (ns * 32 + kg < N)
                b = *reinterpret_cast<const bf16x8*>(W + (kt * 16 + (lane & 15)) * N + ns * 32 + kg);
            else
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = (bf16)0.0f;
            acc = mfma(a, b, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) f(16 * w + 4 * (lane >> 4) + j, kt * 16 + (lane & 15), acc[j]);
    }
}

__global__ void __launch_bounds__(THREADS) k_backward(const float* __restrict__ pf, const bf16* __restrict__ pb,
                                                      const bf16* __restrict__ x, const float* __restrict__ zws,
                                                      const bf16* __restrict__ hws, const float* __restrict__ dy,
                                                      float* __restrict__ partials, float* __restrict__ dx,
                                                      int64_t B) {
    __shared__ __attribute__((aligned(16))) bf16 act[ROWS * HID];  // activations of the layer below
    __shared__ __attribute__((aligned(16))) bf16 dz[ROWS * HID];   // gradient at the current layer
    __shared__ __attribute__((aligned(16))) bf16 dyb[ROWS * 32];   // output gradient, padded to K = 32
    __shared__ float colsum[4][HID];
    const int64_t row0 = (int64_t)blockIdx.x * ROWS;
    float* part = partials + (int64_t)blockIdx.x * MLP_NPARAM;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

    // output layer: dY (FP32) -> bias partial of b4, BF16 copy
    for (int i = threadIdx.x; i < ROWS * 32; i += THREADS) {
        const int r = i / 32, n = i % 32;
        dyb[i] = (bf16)(n < OUTP ? dy[(row0 + r) * OUTP + n] : 0.0f);
    }
    if (threadIdx.x < OUTP) {
        float s = 0.f;
        for (int r = 0; r < ROWS; ++r) s += dy[(row0 + r) * OUTP + threadIdx.x];
        part[OB4 + threadIdx.x] = s;
    }
    auto load_act = [&](int layer) {  // activations H_layer (0-based) into act
        __syncthreads();
        for (int i = threadIdx.x; i < ROWS * HID / 8; i += THREADS)
            reinterpret_cast<bf16x8*>(act)[i] =
                reinterpret_cast<const bf16x8*>(hws + (int64_t)layer * B * HID + row0 * HID)[i];
        __syncthreads();
    };
    // dW4 = H3^T dY
    load_act(2);
    weight_grad<HID, OUTP, 32>(act, dyb, part, OW4);

    // one hidden layer: dH = dNext W_next^T (dNext in `src` with row stride
    // SS, contraction width NC = the output width of W_next [HID][NC]),
    // dZ = dH * gelu'(Z) into dz, and the bias partial of the layer
    auto hidden = [&](int layer, const bf16* src, auto ss, auto nc, int ow_next) {
        constexpr int SS = decltype(ss)::value, NC = decltype(nc)::value;
        float dzr[HID / 16][4];
        const int r = 16 * w + (lane & 15), kg = 8 * (lane >> 4);
        for (int kt = 0; kt < HID / 16; ++kt) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ns = 0; ns < (NC + 31) / 32; ++ns) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(src + r * SS + ns * 32 + kg);
                bf16x8 b;
                if (ns * 32 + kg < NC)
                    b = *reinterpret_cast<const bf16x8*>(pb + ow_next + (kt * 16 + (lane & 15)) * NC + ns * 32 + kg);
                else
#pragma unroll
                    for (int j = 0; j < 8; ++j) b[j] = (bf16)0.0f;
                acc = mfma(a, b, acc);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) dzr[kt][j] = acc[j];
        }
        __syncthreads();  // everyone is done reading src (it may be dz)
        const float* Z = zws + (int64_t)layer * B * HID;
        for (int kt = 0; kt < HID / 16; ++kt) {
            const int col = kt * 16 + (lane & 15);
            float s4 = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int rr = 16 * w + 4 * (lane >> 4) + j;
                const float g = dzr[kt][j] * gelu_prime(Z[(row0 + rr) * HID + col]);
                dz[rr * HID + col] = (bf16)g;
                s4 += g;
            }
            float v = s4;
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) colsum[w][col] = v;
        }
        __syncthreads();
        if (threadIdx.x < HID) {
            const int ob = layer == 0 ? OB1 : (layer == 1 ? OB2 : OB3);
            part[ob + threadIdx.x] =
                ((colsum[0][threadIdx.x] + colsum[1][threadIdx.x]) + colsum[2][threadIdx.x]) + colsum[3][threadIdx.x];
        }
    };
    // layer 3 (index 2): from dY through W4
    hidden(2, dyb, std::integral_constant<int, 32>{}, std::integral_constant<int, OUTP>{}, OW4);
    load_act(1);
    weight_grad<HID, HID, HID>(act, dz, part, OW3);
    // layer 2
    hidden(1, dz, std::integral_constant<int, HID>{}, std::integral_constant<int, HID>{}, OW3);
    load_act(0);
    weight_grad<HID, HID, HID>(act, dz, part, OW2);
    // layer 1
    hidden(0, dz, std::integral_constant<int, HID>{}, std::integral_constant<int, HID>{}, OW2);
    __syncthreads();
    for (int i = threadIdx.x; i < ROWS * IN / 8; i += THREADS)
        reinterpret_cast<bf16x8*>(act)[i] = reinterpret_cast<const bf16x8*>(x + row0 * IN)[i];
    __syncthreads();
    weight_grad<IN, HID, HID>(act, dz, part, OW1);
    if (dx) {
        data_grad<HID>(dz, pb + OW1, IN, [&](int rr, int k, float v) { dx[(row0 + rr) * IN + k] = v; });
    }
}

__global__ void k_reduce(const float* __restrict__ partials, int nwg, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float s = 0.f;
    for (int i = 0; i < nwg; ++i) s += partials[(int64_t)i * MLP_NPARAM + p];
    grad[p] = s;
}

// master-parameter index -> (row-major index, transposed index or -1)
__device__ __forceinline__ int transposed_index(int p) {
    int o, K, N;
    if (p < OB1) { o = OW1; K = IN; N = HID; }
    else if (p >= OW2 && p < OB2) { o = OW2; K = HID; N = HID; }
    else if (p >= OW3 && p < OB3) { o = OW3; K = HID; N = HID; }
    else if (p >= OW4 && p < OB4) { o = OW4; K = HID; N = OUTP; }
    else return -1;
    const int q = p - o, k = q / N, n = q % N;
    return o + n * K + k;
}

__global__ void k_pack(const float* __restrict__ pf, bf16* __restrict__ pb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const bf16 v = (bf16)pf[p];
    pb[p] = v;
    const int t = transposed_index(p);
    pb[MLP_NPARAM + (t >= 0 ? t : p)] = v;
}

__global__ void k_adam(float* __restrict__ pf, bf16* __restrict__ pb, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float w = pf[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    pf[p] = w;
    const bf16 bw = (bf16)w;
    pb[p] = bw;
    const int t = transposed_index(p);
    pb[MLP_NPARAM + (t >= 0 ? t : p)] = bw;
}

// masked MSE over the two used outputs; dy = 2 mask (y - t) / sum(mask);
// loss partials per block of 256 rows in a fixed order.
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ mk,
                       int64_t B, float inv_n, float* __restrict__ dy, double* __restrict__ lpart) {
    __shared__ double red[256];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (r < B) {
        for (int n = 0; n < OUTP; ++n) {
            float d = 0.f;
            if (n < 2) {
                const float e = (y[r * OUTP + n] - t[r * 2 + n]) * mk[r * 2 + n];
                d = 2.0f * e * inv_n;
                l += (double)e * e;
            }
            dy[r * OUTP + n] = d;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] * inv_n;
}

// The total of n loss partials in index order, by one thread (the same order
// and the same FP64 additions as the host loop of mlp_loss).
__global__ void k_sum_in_order(const double* __restrict__ part, int n, double* __restrict__ out) {
    double L = 0.0;
    for (int i = 0; i < n; ++i) L += part[i];
    *out = L;
}

// windows of 33 porosities around every cell of ncols columns of height nz,
// replicate padding; x[(col*nz + z)*64 + j]
__global__ void k_windows(const double* __restrict__ eps, int nz, int64_t n, bf16* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * IN) return;
    const int64_t cell = i / IN;
    const int j = (int)(i % IN);
    const int64_t col = cell / nz;
    const int z = (int)(cell % nz);
    float v = 0.0f;
    if (j < 33) {
        int zz = z + j - 16;
        zz = zz < 0 ? 0 : (zz > nz - 1 ? nz - 1 : zz);
        v = (float)eps[col * nz + zz];
    }
    x[i] = (bf16)v;
}

__global__ void k_closure(const float* __restrict__ y, const double* __restrict__ eps, int64_t n, double nu,
                          double* __restrict__ nu_eff, double* __restrict__ drag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double o1 = y[i * OUTP], o2 = y[i * OUTP + 1];
    const double s = 1.0 - eps[i];  // vanishes in free fluid
    nu_eff[i] = nu * exp(s * o1);
    drag[i] = s * (o2 > 0 ? o2 + log1p(exp(-o2)) : log1p(exp(o2)));
}

// Profile loss through the steady gray column.  For shear flow along x the
// steady state of the gray model (eq. (GeneralizedPor2) with the porous force
// of eq. (PorousForce), Forchheimer term zero) obeys, cell by cell,
//     d/dz (nu_eff dU/dz) - drag U + eps G = 0,
// discretised on the cells 1..n (n = nz-2) between the wall layers with face
// viscosities (nu_i + nu_{i+1})/2 and, next to each wall (U = 0 half a cell
// away), the one-sided slope 3 U_1 - U_2 / 3, which is exact for the
// parabola the lattice scheme reproduces.  One workgroup per profile: the
// lanes form the coefficients, lane 0 runs the two tridiagonal (Thomas)
// solves -- A U = -eps G and the adjoint A^T lambda = dL/dU -- and the lanes
// chain dL/dA = -lambda U^T through the closure map into dL/do1, dL/do2.
constexpr int PL_MAX = 1024;

__device__ __forceinline__ double softplus_d(double o) { return o > 0 ? o + log1p(exp(-o)) : log1p(exp(o)); }
__device__ __forceinline__ double sigmoid_d(double o) {
    return o >= 0 ? 1.0 / (1.0 + exp(-o)) : exp(o) / (1.0 + exp(o));
}

__global__ void __launch_bounds__(64) k_profile_loss(const float* __restrict__ y, const double* __restrict__ eps,
                                                     const double* __restrict__ ut, int nz, double nu, double G,
                                                     double scale, float* __restrict__ dy,
                                                     double* __restrict__ loss) {
    __shared__ double snu[PL_MAX], sd[PL_MAX], su[PL_MAX], sl[PL_MAX], cpr[PL_MAX], dpr[PL_MAX];
    const int p = blockIdx.x;
    const int n = nz - 2;
    const int64_t r0 = (int64_t)p * nz;
    // coefficients of the interior cells (index i = z - 1)
    for (int i = threadIdx.x; i < n; i += 64) {
        const int64_t r = r0 + i + 1;
        const double s = 1.0 - eps[r];
        snu[i] = nu * exp(s * (double)y[r * OUTP]);
        sd[i] = s * softplus_d((double)y[r * OUTP + 1]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // tridiagonal rows: a (sub), b (diagonal), c (super)
        auto fa = [&](int i) { return i == 0 ? 0.0 : 0.5 * (snu[i - 1] + snu[i]) + (i == n - 1 ? snu[i] / 3.0 : 0.0); };
        auto fc = [&](int i) { return i == n - 1 ? 0.0 : 0.5 * (snu[i] + snu[i + 1]) + (i == 0 ? snu[i] / 3.0 : 0.0); };
        auto fb = [&](int i) {
            double b = -sd[i];
            if (i > 0) b -= 0.5 * (snu[i - 1] + snu[i]);
            else b -= 3.0 * snu[i];
            if (i < n - 1) b -= 0.5 * (snu[i] + snu[i + 1]);
            else b -= 3.0 * snu[i];
            return b;
        };
        // A U = -eps G
        for (int i = 0; i < n; ++i) {
            const double ai = fa(i), bi = fb(i), ci = fc(i);
            const double ri = -eps[r0 + i + 1] * G;
            const double m = i == 0 ? bi : bi - ai * cpr[i - 1];
            cpr[i] = ci / m;
            dpr[i] = (i == 0 ? ri : ri - ai * dpr[i - 1]) / m;
        }
        su[n - 1] = dpr[n - 1];
        for (int i = n - 2; i >= 0; --i) su[i] = dpr[i] - cpr[i] * su[i + 1];
        // loss and dL/dU
        double tt = 0.0, ee = 0.0;
        for (int i = 0; i < n; ++i) {
            const double t = ut[r0 + i + 1];
            const double e = su[i] - t;
            tt += t * t;
            ee += e * e;
        }
        const double w = scale / (tt > 0 ? tt : 1.0);
        loss[p] = w * ee;
        // A^T lambda = dL/dU: sub-diagonal of A^T is c(i-1), super is a(i+1)
        for (int i = 0; i < n; ++i) {
            const double ai = i == 0 ? 0.0 : fc(i - 1), bi = fb(i), ci = i == n - 1 ? 0.0 : fa(i + 1);
            const double ri = 2.0 * w * (su[i] - ut[r0 + i + 1]);
            const double m = i == 0 ? bi : bi - ai * cpr[i - 1];
            cpr[i] = ci / m;
            dpr[i] = (i == 0 ? ri : ri - ai * dpr[i - 1]) / m;
        }
        sl[n - 1] = dpr[n - 1];
        for (int i = n - 2; i >= 0; --i) sl[i] = dpr[i] - cpr[i] * sl[i + 1];
    }
    __syncthreads();
    // dL/dnu_i and dL/ddrag_i, chained through the closure map
    for (int z = threadIdx.x; z < nz; z += 64) {
        const int64_t r = r0 + z;
        float d1 = 0.f, d2 = 0.f;
        if (z >= 1 && z <= n) {
            const int i = z - 1;
            const double li = sl[i], ui = su[i];
            double gnu = 0.0;
            // faces: dL/df = (lambda_i - lambda_j)(U_i - U_j), half to each cell
            if (i > 0) gnu += 0.5 * (li - sl[i - 1]) * (ui - su[i - 1]);
            else gnu += li * (3.0 * ui - su[1] / 3.0);
            if (i < n - 1) gnu += 0.5 * (li - sl[i + 1]) * (ui - su[i + 1]);
            else gnu += li * (3.0 * ui - su[n - 2] / 3.0);
            const double gd = li * ui;
            const double s = 1.0 - eps[r];
            d1 = (float)(gnu * snu[i] * s);
            d2 = (float)(gd * s * sigmoid_d((double)y[r * OUTP + 1]));
        }
        for (int c = 0; c < OUTP; ++c) dy[r * OUTP + c] = c == 0 ? d1 : (c == 1 ? d2 : 0.f);
    }
}

int64_t nwg_of(int64_t B) { return B / ROWS; }

}  // namespace

// Scratch of mlp_loss_noalloc: one loss partial per block of 256 rows, then
// their total in the last slot.  A file-scope device array, so the entry
// point needs no allocation; each GPU holds its own copy for the life of the
// process.  Host code must use its device address (scratch_on_current_device),
// never this name.
static __device__ __align__(256) double scratch[MLP_LOSS_NOALLOC_MAX_ROWS / 256 + 1];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the calling thread's current device, looked
// up once per device (with that device current) and kept.
lbm_status scratch_on_current_device(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(LBM_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(LBM_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(LBM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

#define MCHK(expr, what)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return set_error(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

lbm_status check_batch(int64_t B) {
    if (B <= 0 || B % ROWS != 0 || B > ((int64_t)1 << 26))
        return set_error(LBM_E_INVAL, "batch size must be a positive multiple of 64");
    return LBM_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

lbm_status mlp_workspace_bytes(int64_t B, int64_t* bytes) {
    lbm_status s = check_batch(B);
    if (s != LBM_OK || !bytes) return s != LBM_OK ? s : set_error(LBM_E_INVAL, "null pointer");
    *bytes = B * HID * 3 * 4 + B * HID * 3 * 2 + nwg_of(B) * (int64_t)MLP_NPARAM * 4;
    return LBM_OK;
}

lbm_status mlp_pack_bf16(const float* params, void* params_bf16, void* stream) {
    if (!params || !params_bf16) return set_error(LBM_E_INVAL, "null pointer");
    k_pack<<<(MLP_NPARAM + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, (bf16*)params_bf16);
    MCHK(hipGetLastError(), "pack");
    MCHK(hipStreamSynchronize((hipStream_t)stream), "synchronise");
    return LBM_OK;
}

lbm_status mlp_forward(const float* params, const void* params_bf16, const void* x_bf16, int64_t B, float* y,
                       void* ws, void* stream) {
    lbm_status s = check_batch(B);
    if (s != LBM_OK) return s;
    if (!params || !params_bf16 || !x_bf16 || !y) return set_error(LBM_E_INVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = (unsigned)nwg_of(B);
    if (ws) {
        float* z = (float*)ws;
        bf16* h = (bf16*)((char*)ws + B * HID * 3 * 4);
        k_forward<true><<<grid, THREADS, 0, st>>>(params, (const bf16*)params_bf16, (const bf16*)x_bf16, y, z, h, B);
    } else {
        k_forward<false><<<grid, THREADS, 0, st>>>(params, (const bf16*)params_bf16, (const bf16*)x_bf16, y, nullptr,
                                                   nullptr, B);
    }
    MCHK(hipGetLastError(), "forward");
    MCHK(hipStreamSynchronize(st), "synchronise");
    return LBM_OK;
}

lbm_status mlp_backward(const float* params, const void* params_bf16, const void* x_bf16, void* ws, const float* dy,
                        int64_t B, float* grad, float* dx, void* stream) {
    lbm_status s = check_batch(B);
    if (s != LBM_OK) return s;
    if (!params || !params_bf16 || !x_bf16 || !ws || !dy || !grad) return set_error(LBM_E_INVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nwg = nwg_of(B);
    const float* z = (const float*)ws;
    const bf16* h = (const bf16*)((const char*)ws + B * HID * 3 * 4);
    float* part = (float*)((char*)ws + B * HID * 3 * 4 + B * HID * 3 * 2);
    k_backward<<<(unsigned)nwg, THREADS, 0, st>>>(params, (const bf16*)params_bf16, (const bf16*)x_bf16, z, h, dy,
                                                  part, dx, B);
    MCHK(hipGetLastError(), "backward");
    k_reduce<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(part, (int)nwg, grad);
    MCHK(hipGetLastError(), "gradient reduction");
    MCHK(hipStreamSynchronize(st), "synchronise");
    return LBM_OK;
}

lbm_status mlp_loss(const float* y, const float* target, const float* mask, int64_t B, double mask_sum, float* dy,
                    double* loss_partials, double* loss, void* stream) {
    lbm_status s = check_batch(B);
    if (s != LBM_OK) return s;
    if (!y || !target || !mask || !dy || !loss_partials) return set_error(LBM_E_INVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    const unsigned nb = (unsigned)((B + 255) / 256);
    const float inv = (float)(1.0 / (mask_sum > 1.0 ? mask_sum : 1.0));
    k_loss<<<nb, 256, 0, st>>>(y, target, mask, B, inv, dy, loss_partials);
    MCHK(hipGetLastError(), "loss");
    if (loss) {
        std::vector<double> h(nb);
        MCHK(hipMemcpyAsync(h.data(), loss_partials, nb * 8, hipMemcpyDeviceToHost, st), "copy loss");
        MCHK(hipStreamSynchronize(st), "synchronise");
        double L = 0;
        for (double v : h) L += v;
        *loss = L;
    } else {
        MCHK(hipStreamSynchronize(st), "synchronise");
    }
    return LBM_OK;
}

lbm_status mlp_loss_noalloc(const float* y, const float* target, const float* mask, int64_t B, double mask_sum,
                            float* dy, double* loss, void* stream) {
    lbm_status s = check_batch(B);
    if (s != LBM_OK) return s;
    if (B > MLP_LOSS_NOALLOC_MAX_ROWS)
        return set_error(LBM_E_INVAL, "mlp_loss_noalloc: batch of " + std::to_string(B) + " rows exceeds the " +
                                          std::to_string((long long)MLP_LOSS_NOALLOC_MAX_ROWS) +
                                          "-row limit of its static scratch (use mlp_loss)");
    if (!y || !target || !mask || !dy) return set_error(LBM_E_INVAL, "null pointer");
    double* part = nullptr;
    s = scratch_on_current_device(&part);
    if (s != LBM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const unsigned nb = (unsigned)((B + 255) / 256);
    const float inv = (float)(1.0 / (mask_sum > 1.0 ? mask_sum : 1.0));
    // every one of the nb partials is written before it is read: nothing in
    // the scratch needs clearing between calls
    k_loss<<<nb, 256, 0, st>>>(y, target, mask, B, inv, dy, part);
    MCHK(hipGetLastError(), "loss");
    double* total = part + MLP_LOSS_NOALLOC_MAX_ROWS / 256;
    k_sum_in_order<<<1, 1, 0, st>>>(part, (int)nb, total);
    MCHK(hipGetLastError(), "loss total");
    if (loss) {
        double L = 0.0;
        MCHK(hipMemcpyAsync(&L, total, sizeof(double), hipMemcpyDeviceToHost, st), "copy loss");
        MCHK(hipStreamSynchronize(st), "synchronise");
        *loss = L;
    } else {
        MCHK(hipStreamSynchronize(st), "synchronise");
    }
    return LBM_OK;
}

lbm_status mlp_adam_step(float* params, void* params_bf16, float* m, float* v, const float* grad, double lr,
                         double b1, double b2, double eps, int64_t t, void* stream) {
    if (!params || !params_bf16 || !m || !v || !grad || t < 1) return set_error(LBM_E_INVAL, "bad arguments");
    const float c1 = (float)(1.0 - std::pow(b1, (double)t)), c2 = (float)(1.0 - std::pow(b2, (double)t));
    k_adam<<<(MLP_NPARAM + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, (bf16*)params_bf16, m, v, grad,
                                                                       (float)lr, (float)b1, (float)b2, (float)eps,
                                                                       c1, c2);
    MCHK(hipGetLastError(), "adam");
    MCHK(hipStreamSynchronize((hipStream_t)stream), "synchronise");
    return LBM_OK;
}

lbm_status mlp_windows(const double* eps, int32_t ncols, int32_t nz, void* x_bf16, void* stream) {
    if (!eps || !x_bf16 || ncols < 1 || nz < 1) return set_error(LBM_E_INVAL, "bad arguments");
    const int64_t n = (int64_t)ncols * nz;
    k_windows<<<(unsigned)((n * IN + 255) / 256), 256, 0, (hipStream_t)stream>>>(eps, nz, n, (bf16*)x_bf16);
    MCHK(hipGetLastError(), "windows");
    MCHK(hipStreamSynchronize((hipStream_t)stream), "synchronise");
    return LBM_OK;
}

lbm_status mlp_closure(const float* y, const double* eps, int64_t n, double nu, double* nu_eff, double* drag,
                       void* stream) {
    if (!y || !eps || !nu_eff || !drag || n < 1 || !(nu > 0)) return set_error(LBM_E_INVAL, "bad arguments");
    k_closure<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(y, eps, n, nu, nu_eff, drag);
    MCHK(hipGetLastError(), "closure");
    MCHK(hipStreamSynchronize((hipStream_t)stream), "synchronise");
    return LBM_OK;
}


lbm_status mlp_profile_loss(const float* y, const double* eps, const double* u_target, int32_t nprof, int32_t nz,
                            double nu, double G, double weight, float* dy, double* loss, void* stream) {
    if (!y || !eps || !u_target || !dy || !loss || nprof < 1 || nz < 5 || nz > PL_MAX || !(nu > 0) ||
        !(weight >= 0))
        return set_error(LBM_E_INVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    k_profile_loss<<<(unsigned)nprof, 64, 0, st>>>(y, eps, u_target, nz, nu, G, weight / nprof, dy, loss);
    MCHK(hipGetLastError(), "profile loss");
    MCHK(hipStreamSynchronize(st), "synchronise");
    return LBM_OK;
}

}  // extern "C"
