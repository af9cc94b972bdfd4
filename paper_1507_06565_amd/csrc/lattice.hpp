// D3Q19 velocity set (Sec. 2.1 of the paper): rest, six axis and twelve edge
// velocities, weights 1/3, 1/18, 1/36.  The order is part of the C ABI (the
// link direction index) and is listed in include/lbm.h; opposite pairs are
// adjacent (k, k+1) for odd k.
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#define LBM_HD __host__ __device__
#else
#define LBM_HD
#endif

namespace lbm {

constexpr int Q = 19;

struct D3Q19 {
    static constexpr int ex[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
};

LBM_HD constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }
LBM_HD constexpr int norm2(int k) {
    return D3Q19::ex[k] * D3Q19::ex[k] + D3Q19::ey[k] * D3Q19::ey[k] + D3Q19::ez[k] * D3Q19::ez[k];
}
LBM_HD constexpr double weight(int k) { return norm2(k) == 0 ? 1.0 / 3.0 : (norm2(k) == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }

// cell flags
enum : uint8_t { CELL_FLUID = 0, CELL_SPHERE = 1, CELL_WALL = 2 };
// surface a link ends on
enum : int8_t { SURF_SPHERE = 0, SURF_WALL_LO = 1, SURF_WALL_HI = 2 };

}  // namespace lbm
