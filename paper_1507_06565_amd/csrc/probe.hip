// Streaming-ceiling probe for the brick sweep's memory access pattern: the
// same bytes the sweep's population streams move, with nothing else (no
// neighbour pulls, cell words, links or collision), so that the sweep's
// traffic can be set against what the device streams for this pattern.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/lbm.h"
#include "internal.hpp"

namespace lbm {
namespace {

// One wavefront per 64-cell brick, 16 bricks per workgroup.  SoA (the
// sweep's layout): population k of brick b at a[k * stride + 64 b + lane];
// grouped: a brick's 19 populations contiguous, at a[(19 b + k) * 64 + lane].
template <bool GROUPED>
__global__ void __launch_bounds__(1024) k_stream(const float* __restrict__ a, float* __restrict__ b, int64_t nbricks) {
    const int64_t brick = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6);
    if (brick >= nbricks) return;
    const int64_t lane = threadIdx.x & 63;
    const int64_t stride = nbricks * 64;
    float v[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) v[k] = a[GROUPED ? (brick * Q + k) * 64 + lane : k * stride + brick * 64 + lane];
#pragma unroll
    for (int k = 0; k < Q; ++k)
        __builtin_nontemporal_store(v[k], &b[GROUPED ? (brick * Q + k) * 64 + lane : k * stride + brick * 64 + lane]);
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_stream_probe(const void* src, void* dst, int64_t nbricks, int32_t grouped, int32_t passes,
                                       void* hip_stream, double* ms_per_pass) {
    if (!src || !dst || nbricks < 1 || nbricks > ((int64_t)1 << 31) / 16 || passes < 1 || !ms_per_pass)
        return set_error(LBM_E_INVAL, "bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const unsigned grid = (unsigned)((nbricks + 15) / 16);
    auto launch = [&]() {
        if (grouped) k_stream<true><<<grid, 1024, 0, s>>>((const float*)src, (float*)dst, nbricks);
        else k_stream<false><<<grid, 1024, 0, s>>>((const float*)src, (float*)dst, nbricks);
        return hipGetLastError();
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(LBM_E_DEVICE, "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(LBM_E_DEVICE, "event");
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; i < passes && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return set_error(LBM_E_DEVICE, std::string("stream probe: ") + hipGetErrorString(e));
    *ms_per_pass = ms / passes;
    return LBM_OK;
}
