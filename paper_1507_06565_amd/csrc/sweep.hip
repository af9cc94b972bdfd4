// Single-domain sweep kernels: map workgroups to cells (dense layouts) or to
// bricks (brick layout) and run the fused stream + collide update of cell.hpp
// on every stored cell of the domain.
#include <hip/hip_runtime.h>

#include "cell.hpp"

namespace lbm {
namespace {

// workgroups for n units (cells or bricks), per_group units per workgroup
// and tile, cpt tiles per workgroup
unsigned grid_size(int64_t n, int per_group, int cpt) {
    const int64_t tiles = (n + per_group - 1) / per_group;
    return (unsigned)((tiles + cpt - 1) / cpt);
}

__device__ __forceinline__ int remap_block(int b, int nblocks) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of tiles so that neighbouring tiles share an L2.
    const int per = nblocks >> 3;
    if (b < (per << 3)) return (b & 7) * per + (b >> 3);
    return b;
}

// ROW: the workgroup size divides nx, so a workgroup covers part of one x-row
// and y, z are uniform (scalar) per workgroup.  NT: non-temporal hints on the
// streams whose wavefront accesses are 256-byte aligned.
template <int LAYOUT, int PARITY, int BC, int BLOCK, bool ROW, bool NT>
__global__ void __launch_bounds__(BLOCK) k_sweep(SweepArgs a) {
    int b = blockIdx.x;
    if (a.xcd_remap) b = remap_block(b, gridDim.x);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    int c, x, y, z;
    if (ROW) {
        const int first = b * BLOCK;          // uniform
        const int row = first / nx;           // uniform
        y = row % ny;
        z = row / ny;
        x = first - row * nx + threadIdx.x;
        c = first + threadIdx.x;
    } else {
        c = b * BLOCK + threadIdx.x;
        if (c >= a.ncells) return;
        x = c % nx;
        const int t = c / nx;
        y = t % ny;
        z = t / ny;
    }
    const CellHead h = load_head(a.info, a.segbase, c);
    const DenseNb nbi(nx, ny, nz, x, y, z);
    (void)cell_update<LAYOUT, PARITY, BC, NT, false>(PopBases{a.pa}, PopBases{a.pb}, h, a.lparam, a.pva, a.pvb,
                                                     a.k, nbi, c);
}

// Brick layout: one wavefront per stored brick, lane l = cell l of the brick
// (lx + 4 ly + 16 lz); the pull goes through the brick's neighbour table and
// the store is aligned, as in the two-grid layout.  LIST: the bricks come
// from a.list (a batch of domains stored as one brick array, each domain's
// neighbour table wrapping onto itself); CHECK: the wavefront also stores the
// sum of its cells' u_x (fixed butterfly) for the steady-state test.
template <int BC, bool NT, bool LIST, bool CHECK, class PA>
__device__ __forceinline__ void brick_pass(const SweepArgs& a, int slot, int l, PA pa, PA pb) {
    const int brick = LIST ? __builtin_amdgcn_readfirstlane(a.list[slot]) : slot;
    // the neighbour table and the cell's head are read together: each lane
    // then issues only the pulls it uses (masked: none for a solid cell, and
    // none across a link), and the link records' addresses are known as soon
    // as the pulls have arrived
    const int tab = a.nbr[(int64_t)brick * 27 + (l < 27 ? l : 13)];
    const CellHead h = load_head(a.info, a.segbase, brick * 64 + l);
    // all three have arrived before the pulls are addressed (the table is
    // needed for that anyway), so the compiler cannot defer the head loads
    asm volatile("" ::"v"(tab), "v"(h.inf), "s"(h.seg));
    const BrickNb nbi(tab, brick, l);
    const float ux = cell_update<L_TWOGRID, P_EVEN, BC, NT, false, PA, BrickNb, true>(
        pa, pb, h, a.lparam, a.pva, a.pvb, a.k, nbi, brick * 64 + l);
    if (CHECK) {
        double v = (double)ux;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (l == 0) a.partial[brick] = v;
    }
}

// MULTI: each workgroup steps a.cpt groups of BLOCK / 64 bricks in turn
// (cells per thread), groups b, b + G, b + 2G, ... for a grid of G
// workgroups, so that at any time the grid works on one contiguous run of
// bricks.  The loop is a separate instantiation: the straight-line kernel
// (one group per workgroup) keeps its register allocation.
template <int BC, int BLOCK, bool NT, bool LIST, bool CHECK, bool MULTI>
__global__ void __launch_bounds__(BLOCK) k_sweep_brick(SweepArgs a) {
    int b0 = blockIdx.x;
    if (a.xcd_remap) b0 = remap_block(b0, gridDim.x);
    if constexpr (!MULTI) {
        const int slot = b0 * (BLOCK / 64) + (int)(threadIdx.x >> 6);  // uniform per wavefront
        if (slot >= a.nbricks) return;
        brick_pass<BC, NT, LIST, CHECK>(a, slot, (int)(threadIdx.x & 63), PopBases{a.pa}, PopBases{a.pb});
    } else {
#pragma clang loop unroll(disable)
        for (int j = 0; j < a.cpt; ++j) {
            const int slot = (b0 + j * (int)gridDim.x) * (BLOCK / 64) + (int)(threadIdx.x >> 6);
            if (slot >= a.nbricks) break;
            // the lane index and the grids' bases are made opaque to the
            // compiler in each pass, so that what derives from them (the
            // pull offsets, the 38 array bases) is formed where it is used
            // instead of being held in registers across passes
            int l = (int)(threadIdx.x & 63);
            uint64_t A = (uint64_t)a.A, B = (uint64_t)a.B, sb = (uint64_t)a.stride * 4u;
            asm volatile("" : "+v"(l), "+s"(A), "+s"(B), "+s"(sb));
            brick_pass<BC, NT, LIST, CHECK>(a, slot, l, PopWide{A, sb}, PopWide{B, sb});
        }
    }
}

__global__ void __launch_bounds__(64) k_domain_sums(const double* __restrict__ partial,
                                                    const int32_t* __restrict__ first,
                                                    const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ doms, double* __restrict__ out) {
    const int d = doms[blockIdx.x];
    const int f = first[d], n = count[d];
    double v = 0.0;
    for (int i = (int)threadIdx.x; i < n; i += 64) v += partial[f + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) out[d] = v;
}

template <int LAYOUT, int PARITY, int BC, int BLOCK>
hipError_t launch4(const SweepArgs& a, hipStream_t s) {
    if constexpr (LAYOUT == L_BRICK) {
        const unsigned nb = grid_size((int64_t)a.nbricks, BLOCK / 64, a.cpt);
        if (nb == 0) return hipSuccess;
        const bool multi = a.cpt > 1;
        if (a.nt && multi) k_sweep_brick<BC, BLOCK, true, false, false, true><<<nb, BLOCK, 0, s>>>(a);
        else if (a.nt) k_sweep_brick<BC, BLOCK, true, false, false, false><<<nb, BLOCK, 0, s>>>(a);
        else if (multi) k_sweep_brick<BC, BLOCK, false, false, false, true><<<nb, BLOCK, 0, s>>>(a);
        else k_sweep_brick<BC, BLOCK, false, false, false, false><<<nb, BLOCK, 0, s>>>(a);
        return hipGetLastError();
    } else {
        const unsigned nb = (unsigned)(((int64_t)a.ncells + BLOCK - 1) / BLOCK);
        const bool row = (a.nx % BLOCK) == 0;
        if (row && a.nt)
            k_sweep<LAYOUT, PARITY, BC, BLOCK, true, true><<<nb, BLOCK, 0, s>>>(a);
        else if (row)
            k_sweep<LAYOUT, PARITY, BC, BLOCK, true, false><<<nb, BLOCK, 0, s>>>(a);
        else if (a.nt)
            k_sweep<LAYOUT, PARITY, BC, BLOCK, false, true><<<nb, BLOCK, 0, s>>>(a);
        else
            k_sweep<LAYOUT, PARITY, BC, BLOCK, false, false><<<nb, BLOCK, 0, s>>>(a);
        return hipGetLastError();
    }
}

template <int LAYOUT, int PARITY, int BC>
hipError_t launch3(const SweepArgs& a, int block, hipStream_t s) {
    switch (block) {
        case 64: return launch4<LAYOUT, PARITY, BC, 64>(a, s);
        case 128: return launch4<LAYOUT, PARITY, BC, 128>(a, s);
        case 256: return launch4<LAYOUT, PARITY, BC, 256>(a, s);
        case 512: return launch4<LAYOUT, PARITY, BC, 512>(a, s);
        case 1024: return launch4<LAYOUT, PARITY, BC, 1024>(a, s);
        default: return hipErrorInvalidValue;
    }
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

__global__ void k_scatter(float* p, const int64_t* idx, const float* val, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[idx[i]] = val[i];
}

}  // namespace

hipError_t launch_scatter(float* p, const int64_t* idx, const float* val, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_scatter<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, idx, val, n);
    return hipGetLastError();
}

template <int BC, int BLOCK, bool MULTI>
hipError_t launch_list_m(const SweepArgs& a, bool check, unsigned nb, hipStream_t s) {
    if (a.nt) {
        if (check) k_sweep_brick<BC, BLOCK, true, true, true, MULTI><<<nb, BLOCK, 0, s>>>(a);
        else k_sweep_brick<BC, BLOCK, true, true, false, MULTI><<<nb, BLOCK, 0, s>>>(a);
    } else {
        if (check) k_sweep_brick<BC, BLOCK, false, true, true, MULTI><<<nb, BLOCK, 0, s>>>(a);
        else k_sweep_brick<BC, BLOCK, false, true, false, MULTI><<<nb, BLOCK, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <int BC, int BLOCK>
hipError_t launch_list(const SweepArgs& a, bool check, hipStream_t s) {
    const unsigned nb = grid_size((int64_t)a.nbricks, BLOCK / 64, a.cpt);
    if (nb == 0) return hipSuccess;
    return a.cpt > 1 ? launch_list_m<BC, BLOCK, true>(a, check, nb, s) : launch_list_m<BC, BLOCK, false>(a, check, nb, s);
}

template <int BC>
hipError_t launch_list_bc(const SweepArgs& a, int block, bool check, hipStream_t s) {
    switch (block) {
        case 64: return launch_list<BC, 64>(a, check, s);
        case 128: return launch_list<BC, 128>(a, check, s);
        case 256: return launch_list<BC, 256>(a, check, s);
        case 512: return launch_list<BC, 512>(a, check, s);
        case 1024: return launch_list<BC, 1024>(a, check, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_bricks(const SweepArgs& a, int bc, int block, bool check, hipStream_t s) {
    if (a.cpt != 1 && a.cpt != 2 && a.cpt != 4) return hipErrorInvalidValue;
    switch (bc) {
        case LBM_BC_SBB: return launch_list_bc<LBM_BC_SBB>(a, block, check, s);
        case LBM_BC_CLI: return launch_list_bc<LBM_BC_CLI>(a, block, check, s);
        case LBM_BC_BOUZIDI: return launch_list_bc<LBM_BC_BOUZIDI>(a, block, check, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_domain_sums(const double* partial, const int32_t* first, const int32_t* count, const int32_t* doms,
                              int n, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_domain_sums<<<(unsigned)n, 64, 0, s>>>(partial, first, count, doms, out);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& a, int layout, int parity, int bc, int block, hipStream_t s) {
    if (a.cpt != 1 && a.cpt != 2 && a.cpt != 4) return hipErrorInvalidValue;
    if (a.cpt != 1 && layout != L_BRICK) return hipErrorInvalidValue;  // dense layouts: one cell per thread
    if (layout == L_TWOGRID) return launch2<L_TWOGRID, P_EVEN>(a, bc, block, s);
    if (layout == L_BRICK) return launch2<L_BRICK, P_EVEN>(a, bc, block, s);
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
