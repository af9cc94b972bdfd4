// Batched pore-scale runs: many independent small domains (REV samples of
// uneven size) advanced by ONE persistent cooperative launch.
//
// (This file runs batches in the AA layout; batches in the brick layout are
// stepped by the brick sweep itself over one brick array that holds every
// domain, brick_batch.cpp.)
//
// The grid holds as many workgroups as can be resident at once.  They form
// teams of W consecutive workgroups; a team pops the next domain from a
// largest-first queue (one atomic counter), steps it with the same per-cell
// update as the single-domain sweep (AA layout, cell.hpp), synchronising its
// W workgroups after every time step with a counter barrier, and every
// `check_every` steps evaluates the steady-state test on the FP64 mean
// x-velocity of the domain.  When the domain converges (or reaches its step
// cap) the team pops the next one; the launch ends when the queue is empty.
//
// Determinism: every cell's arithmetic is that of the single-domain sweep,
// and the steady-state sum is a fixed-order reduction over 64-cell chunks
// (independent of the workgroup size and of W), so every launch shape
// produces bit-identical fields, step counts and outputs.
//
// Liveness: the launch is cooperative (all workgroups resident or the launch
// fails); every barrier wait is bounded by a spin limit, after which the
// workgroup raises an error flag and leaves, and every workgroup leaves when
// it sees the flag, so the grid always drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "batch.hpp"
#include "tuning.hpp"
#include "cell.hpp"

namespace lbm {

struct BatchDom {
    float* pa[Q];
    uint32_t stride;  // floats between population arrays
    const uint32_t* info;
    const int32_t* segbase;
    const float* lparam;
    float* pv;        // partial bounce-back values, one per link
    double* partial;  // one FP64 partial sum per 64-cell chunk
    int32_t nx, ny, nz, ncells;
};

struct BatchArgs {
    const BatchDom* doms;
    int32_t ndom;
    const int32_t* order;  // queue: domains sorted largest first
    int32_t* queue;        // next queue position
    uint32_t* bar;         // barrier counter per team
    int32_t* slot;         // per team: {domain of even pops, domain of odd pops, stop flag, unused}
    int64_t* steps;        // per domain: steps run so far
    double* uprev;         // per domain: last checked sum of u_x
    int32_t* status;       // per domain: 0 running, 1 converged, -1 unstable
    int32_t* err;          // global: barrier timeout
    CellConsts k;
    double tol;
    int64_t max_steps;     // steady: cap on this launch's steps per domain; fixed: exact count
    int32_t check_every;
    int32_t steady;
    int32_t W;
    int32_t spin_limit;
};

namespace {

__device__ __forceinline__ uint32_t load_acq(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_acq(int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier of the W workgroups of one team; `target` = generation * W.
// Returns false (for the whole workgroup) when the error flag is raised or
// the wait exceeds the spin limit.
__device__ bool team_barrier(const BatchArgs& a, int team, uint32_t target, int* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // release this workgroup's writes
        atomicAdd(&a.bar[team], 1u);
        int ok = 1;
        int it = 0;
        while (load_acq(&a.bar[team]) < target) {
            if (load_acq(a.err) != 0) { ok = 0; break; }
            if (++it > a.spin_limit) {
                atomicExch(a.err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();  // acquire the other workgroups' writes
        if (load_acq(a.err) != 0) ok = 0;
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

__device__ __forceinline__ double wave_sum(double v) {
    // fixed butterfly over the 64 lanes of a wavefront
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int BC, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_batch(BatchArgs a) {
    __shared__ int s_ok, s_dom, s_stop;
    const int W = a.W;
    const int team = blockIdx.x / W, rank = blockIdx.x % W;
    uint32_t gen = 0;
    // The popped domain alternates between two slots: a domain that needs no
    // step (already steady) passes no barrier before the next pop, so a
    // single slot could be overwritten before a slow team member has read it.
    // The next write to the same slot needs the next pop's barrier, which
    // every member reaches only after reading.
    for (uint32_t npop = 0;; ++npop) {
        int32_t* dslot = &a.slot[4 * team + (npop & 1)];
        if (rank == 0 && threadIdx.x == 0) {
            const int q = atomicAdd(a.queue, 1);
            __hip_atomic_store(dslot, q < a.ndom ? a.order[q] : -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!team_barrier(a, team, ++gen * (uint32_t)W, &s_ok)) return;
        if (threadIdx.x == 0) s_dom = load_acq(dslot);
        __syncthreads();
        // uniform across the workgroup: keep it (and everything derived from
        // it, like the 19 population bases) in scalar registers
        const int d = __builtin_amdgcn_readfirstlane(s_dom);
        if (d < 0) return;
        const BatchDom* D = a.doms + d;
        const int N = __builtin_amdgcn_readfirstlane(D->ncells), nx = __builtin_amdgcn_readfirstlane(D->nx),
                  ny = __builtin_amdgcn_readfirstlane(D->ny), nz = __builtin_amdgcn_readfirstlane(D->nz);
        const PopStrided pa{uniform_ptr(D->pa[0]), (uint32_t)__builtin_amdgcn_readfirstlane((int)D->stride)};
        const uint32_t* info = uniform_ptr(D->info);
        const int32_t* segbase = uniform_ptr(D->segbase);
        const float* lparam = uniform_ptr(D->lparam);
        float* pv = uniform_ptr(D->pv);
        double* partial = uniform_ptr(D->partial);
        const int nchunk = (N + 63) >> 6;
        const int64_t s0 = a.steps[d];
        int64_t s = s0;
        bool done = a.steady ? (a.status[d] != 0) : false;
        if (a.max_steps <= 0) done = true;
        while (!done) {
            const bool check = a.steady && ((s + 1 - s0) % a.check_every == 0);
            const bool even = (s & 1) == 0;
            for (int tile = rank; tile * BLOCK < N; tile += W) {
                const int c = tile * BLOCK + threadIdx.x;
                float ux = 0.0f;
                if (c < N) {
                    const int x = c % nx, t = c / nx, y = t % ny, z = t / ny;
                    const CellHead h = load_head(info, segbase, c);
                    const DenseNb nbi(nx, ny, nz, x, y, z);
                    if (even)
                        ux = cell_update<L_AA, P_EVEN, BC, false, true>(pa, pa, h, lparam, pv, pv, a.k, nbi, c);
                    else
                        ux = cell_update<L_AA, P_ODD, BC, false, true>(pa, pa, h, lparam, pv, pv, a.k, nbi, c);
                }
                if (check) {
                    const double w = wave_sum((double)ux);
                    const int chunk = (tile * BLOCK + (threadIdx.x & ~63)) >> 6;
                    if ((threadIdx.x & 63) == 0 && chunk < nchunk) partial[chunk] = w;
                }
            }
            ++s;
            if (!team_barrier(a, team, ++gen * (uint32_t)W, &s_ok)) return;
            bool stop = s - s0 >= a.max_steps;
            if (check) {
                if (rank == 0 && threadIdx.x < 64) {
                    double acc = 0.0;
                    for (int ch = threadIdx.x; ch < nchunk; ch += 64) acc += partial[ch];
                    acc = wave_sum(acc);
                    if (threadIdx.x == 0) {
                        const double U = acc;
                        const double Up = a.uprev[d];
                        int st = 0;
                        if (!(fabs(U) < 0.4 * (double)N)) st = -1;  // NaN or runaway velocity
                        else if (fabs(U - Up) <= a.tol * fabs(U)) st = 1;
                        a.uprev[d] = U;
                        __hip_atomic_store(&a.slot[4 * team + 2], st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                if (!team_barrier(a, team, ++gen * (uint32_t)W, &s_ok)) return;
                if (threadIdx.x == 0) s_stop = load_acq(&a.slot[4 * team + 2]);
                __syncthreads();
                if (s_stop != 0) {
                    stop = true;
                    if (rank == 0 && threadIdx.x == 0) a.status[d] = s_stop;
                }
            }
            done = stop;
        }
        if (rank == 0 && threadIdx.x == 0) a.steps[d] = s;
        // the next pop's barrier publishes these writes
    }
}

template <int BC, int BLOCK>
hipError_t launch_batch(const BatchArgs& args, int grid, hipStream_t s) {
    BatchArgs a = args;
    void* params[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch<BC, BLOCK>), dim3(grid), dim3(BLOCK),
                                      params, 0, s);
}

template <int BC, int BLOCK>
int max_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_batch<BC, BLOCK>), BLOCK,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct DomPlan {
    int64_t N, stride, nl, nchunk, nseed;
    int64_t grid;  // floats of the state block: Q population arrays + partial values
    int64_t off_pop, off_info, off_segbase, off_lparam, off_partial, off_seed;
};

struct TuneKey {
    std::string arch;
    int ndom;
    int64_t cells;
    bool operator<(const TuneKey& o) const { return std::tie(arch, ndom, cells) < std::tie(o.arch, o.ndom, o.cells); }
};
std::mutex g_mu;
std::map<TuneKey, std::pair<int, int>> g_cache;

}  // namespace

struct BatchCtx {
    int ndom = 0;
    lbm_params p{};
    CellConsts k{};
    int bc = 0;
    hipStream_t stream = nullptr;
    char* buf = nullptr;
    int64_t bytes = 0;
    std::vector<DomPlan> plans;
    std::vector<lbm_domain_desc> desc;
    int64_t off_table = 0, off_order = 0, off_queue = 0, off_bar = 0, off_slot = 0, off_steps = 0, off_uprev = 0,
            off_status = 0, off_err = 0, off_red = 0, off_fields = 0;
    int64_t max_teams = 0, max_np = 0, chunk = 0;
    std::vector<int64_t> steps;  // host copy
    std::vector<int32_t> status;
    std::string arch;
    int cus = 0;
    int block = 512, W = 4;
    BrickBatch* flat = nullptr;  // brick layout: every call goes to brick_batch.cpp
};

namespace {

lbm_status plan(const std::vector<DomainGeo>& doms, const lbm_params& p, BatchCtx& b) {
    if (p.force[1] != 0.0 || p.force[2] != 0.0)
        return set_error(LBM_E_INVAL, "batched runs drive the flow along x (force[1] = force[2] = 0)");
    const auto& d0 = doms[0].desc;
    int64_t o = 0;
    b.plans.clear();
    b.desc.clear();
    for (const auto& G : doms) {
        const auto& d = G.desc;
        if (d.bc != d0.bc) return set_error(LBM_E_INVAL, "all domains of a batch must use the same boundary scheme");
        for (int a = 0; a < 3; ++a)
            if (d.wall_hi_velocity[a] != d0.wall_hi_velocity[a])
                return set_error(LBM_E_INVAL, "all domains of a batch must share the wall velocity");
        DomPlan P{};
        P.N = G.ncells();
        P.stride = align_up(P.N, 64) + 64;
        P.nl = (int64_t)G.lcell.size();
        P.nchunk = (P.N + 63) / 64;
        P.nseed = 0;
        const bool moving = d.wall_hi_velocity[0] != 0.0 || d.wall_hi_velocity[1] != 0.0 || d.wall_hi_velocity[2] != 0.0;
        if (moving)
            for (auto s : G.lsurf)
                if (s == SURF_WALL_HI) ++P.nseed;
        P.grid = Q * P.stride + align_up(P.nl + Q, 64);
        if (P.grid * 4 >= ((int64_t)1 << 32))
            return set_error(LBM_E_INVAL, "a batched domain's state must stay below 4 GiB (fewer than ~50 M cells)");
        P.off_pop = o; o = align_up(o + P.grid * 4, 256);
        P.off_info = o; o = align_up(o + P.N * 4, 256);
        P.off_segbase = o; o = align_up(o + ((P.N >> SEG_SHIFT) + 1) * 4, 256);
        P.off_lparam = o; o = align_up(o + (P.nl + Q) * 4, 256);
        P.off_partial = o; o = align_up(o + P.nchunk * 8, 256);
        P.off_seed = o; o = align_up(o + std::max<int64_t>(P.nseed, 1) * 12, 256);
        b.plans.push_back(P);
        b.desc.push_back(d);
        b.max_np = std::max<int64_t>(b.max_np, std::max(d.nx, std::max(d.ny, d.nz)));
        b.chunk = std::max<int64_t>(b.chunk, std::min<int64_t>(P.N, std::max<int64_t>((int64_t)d.nx * d.ny, 1 << 20)));
    }
    const int64_t nd = (int64_t)doms.size();
    b.max_teams = 4096;
    b.off_table = o; o = align_up(o + nd * (int64_t)sizeof(BatchDom), 256);
    b.off_order = o; o = align_up(o + nd * 4, 256);
    b.off_queue = o; o = align_up(o + 4, 256);
    b.off_bar = o; o = align_up(o + b.max_teams * 4, 256);
    b.off_slot = o; o = align_up(o + b.max_teams * 16, 256);
    b.off_steps = o; o = align_up(o + nd * 8, 256);
    b.off_uprev = o; o = align_up(o + nd * 8, 256);
    b.off_status = o; o = align_up(o + nd * 4, 256);
    b.off_err = o; o = align_up(o + 4, 256);
    b.off_red = o; o = align_up(o + b.max_np * 6 * 8, 256);
    b.off_fields = o; o = align_up(o + b.chunk * 4 * 8, 256);
    b.bytes = o;
    b.ndom = (int)nd;
    b.bc = d0.bc;
    return LBM_OK;
}

#define HIPCHK(expr, what)                                                               \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return set_error(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

// rest state of every domain (zero populations, moving-wall seeds), step
// counters and convergence bookkeeping cleared
lbm_status reset(BatchCtx* b) {
    for (int d = 0; d < b->ndom; ++d) {
        const DomPlan& P = b->plans[d];
        float* pop = reinterpret_cast<float*>(b->buf + P.off_pop);
        HIPCHK(launch_fill_zero(pop, P.grid, b->stream), "zero populations");
        if (P.nseed > 0)
            HIPCHK(launch_scatter(pop, reinterpret_cast<const int64_t*>(b->buf + P.off_seed),
                                  reinterpret_cast<const float*>(b->buf + P.off_seed + P.nseed * 8), P.nseed,
                                  b->stream),
                   "seed moving walls");
    }
    b->steps.assign(b->ndom, 0);
    b->status.assign(b->ndom, 0);
    std::vector<double> nanv(b->ndom, NAN);
    HIPCHK(hipMemsetAsync(b->buf + b->off_steps, 0, b->ndom * 8, b->stream), "clear steps");
    HIPCHK(hipMemsetAsync(b->buf + b->off_status, 0, b->ndom * 4, b->stream), "clear status");
    HIPCHK(hipMemcpyAsync(b->buf + b->off_uprev, nanv.data(), b->ndom * 8, hipMemcpyHostToDevice, b->stream),
           "clear history");
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

// one persistent launch; steady = 0 runs exactly n steps on every domain
lbm_status run(BatchCtx* b, int steady, double tol, int64_t check_every, int64_t n, int block, int W) {
    int per_cu = 0;
    switch (block) {
        case 256: per_cu = b->bc == LBM_BC_SBB ? max_blocks_per_cu<LBM_BC_SBB, 256>() : b->bc == LBM_BC_CLI ? max_blocks_per_cu<LBM_BC_CLI, 256>() : max_blocks_per_cu<LBM_BC_BOUZIDI, 256>(); break;
        case 512: per_cu = b->bc == LBM_BC_SBB ? max_blocks_per_cu<LBM_BC_SBB, 512>() : b->bc == LBM_BC_CLI ? max_blocks_per_cu<LBM_BC_CLI, 512>() : max_blocks_per_cu<LBM_BC_BOUZIDI, 512>(); break;
        case 1024: per_cu = b->bc == LBM_BC_SBB ? max_blocks_per_cu<LBM_BC_SBB, 1024>() : b->bc == LBM_BC_CLI ? max_blocks_per_cu<LBM_BC_CLI, 1024>() : max_blocks_per_cu<LBM_BC_BOUZIDI, 1024>(); break;
        default: return set_error(LBM_E_INVAL, "batched workgroup size must be 256, 512 or 1024");
    }
    if (per_cu < 1) return set_error(LBM_E_DEVICE, "batched kernel cannot be resident");
    int64_t grid = (int64_t)per_cu * b->cus;
    grid = grid / W * W;
    if (grid / W > b->max_teams) grid = b->max_teams * W;
    if (grid < W) return set_error(LBM_E_INVAL, "more workgroups per team than resident workgroups");
    // queue order: largest domain first (ties by index), reset counters
    std::vector<int32_t> order(b->ndom);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->plans[x].N > b->plans[y].N; });
    HIPCHK(hipMemcpyAsync(b->buf + b->off_order, order.data(), b->ndom * 4, hipMemcpyHostToDevice, b->stream),
           "queue order");
    HIPCHK(hipMemsetAsync(b->buf + b->off_queue, 0, 4, b->stream), "reset queue");
    HIPCHK(hipMemsetAsync(b->buf + b->off_bar, 0, b->max_teams * 4, b->stream), "reset barriers");
    HIPCHK(hipMemsetAsync(b->buf + b->off_err, 0, 4, b->stream), "reset error flag");
    BatchArgs a{};
    a.doms = reinterpret_cast<const BatchDom*>(b->buf + b->off_table);
    a.ndom = b->ndom;
    a.order = reinterpret_cast<const int32_t*>(b->buf + b->off_order);
    a.queue = reinterpret_cast<int32_t*>(b->buf + b->off_queue);
    a.bar = reinterpret_cast<uint32_t*>(b->buf + b->off_bar);
    a.slot = reinterpret_cast<int32_t*>(b->buf + b->off_slot);
    a.steps = reinterpret_cast<int64_t*>(b->buf + b->off_steps);
    a.uprev = reinterpret_cast<double*>(b->buf + b->off_uprev);
    a.status = reinterpret_cast<int32_t*>(b->buf + b->off_status);
    a.err = reinterpret_cast<int32_t*>(b->buf + b->off_err);
    a.k = b->k;
    a.tol = tol;
    a.max_steps = n;
    a.check_every = (int32_t)std::max<int64_t>(1, check_every);
    a.steady = steady;
    a.W = W;
    a.spin_limit = 1 << 22;
    hipError_t e = hipSuccess;
#define BL(BC)                                                              \
    switch (block) {                                                        \
        case 256: e = launch_batch<BC, 256>(a, (int)grid, b->stream); break;  \
        case 512: e = launch_batch<BC, 512>(a, (int)grid, b->stream); break;  \
        default: e = launch_batch<BC, 1024>(a, (int)grid, b->stream); break; \
    }
    if (b->bc == LBM_BC_SBB) { BL(LBM_BC_SBB) }
    else if (b->bc == LBM_BC_CLI) { BL(LBM_BC_CLI) }
    else { BL(LBM_BC_BOUZIDI) }
#undef BL
    HIPCHK(e, "persistent batched launch");
    int32_t err = 0;
    HIPCHK(hipMemcpyAsync(&err, b->buf + b->off_err, 4, hipMemcpyDeviceToHost, b->stream), "read error flag");
    HIPCHK(hipMemcpyAsync(b->steps.data(), b->buf + b->off_steps, b->ndom * 8, hipMemcpyDeviceToHost, b->stream),
           "read steps");
    HIPCHK(hipMemcpyAsync(b->status.data(), b->buf + b->off_status, b->ndom * 4, hipMemcpyDeviceToHost, b->stream),
           "read status");
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    if (err) return set_error(LBM_E_DEVICE, "batched launch: a team barrier timed out");
    return LBM_OK;
}

MomentArgs dom_moments(BatchCtx* b, int d) {
    const DomPlan& P = b->plans[d];
    MomentArgs m{};
    m.A = reinterpret_cast<const float*>(b->buf + P.off_pop);
    m.stride = P.stride;
    m.info = reinterpret_cast<const uint32_t*>(b->buf + P.off_info);
    m.nx = b->desc[d].nx; m.ny = b->desc[d].ny; m.nz = b->desc[d].nz;
    m.layout = L_AA;
    m.parity = b->steps[d] == 0 ? -1 : ((b->steps[d] - 1) % 2 == 0 ? P_EVEN : P_ODD);
    m.rho0 = b->p.rho0;
    for (int a = 0; a < 3; ++a) m.F[a] = b->p.force[a];
    return m;
}

lbm_status dom_plane_sums(BatchCtx* b, int d, int axis, std::vector<double>& out) {
    const auto& D = b->desc[d];
    const int np = axis == 0 ? D.nx : (axis == 1 ? D.ny : D.nz);
    double* red = reinterpret_cast<double*>(b->buf + b->off_red);
    HIPCHK(launch_plane_sums(dom_moments(b, d), axis, red, b->stream), "plane reduction");
    out.assign((size_t)np * 6, 0.0);
    HIPCHK(hipMemcpyAsync(out.data(), red, out.size() * 8, hipMemcpyDeviceToHost, b->stream), "copy plane sums");
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

}  // namespace

lbm_status batch_required_bytes(const std::vector<DomainGeo>& doms, const lbm_params& p, int64_t* bytes) {
    if (p.layout == LBM_LAYOUT_BRICK) return bbatch_required_bytes(doms, p, bytes);
    BatchCtx b;
    lbm_status s = plan(doms, p, b);
    if (s != LBM_OK) return s;
    *bytes = b.bytes;
    return LBM_OK;
}

lbm_status batch_init(const std::vector<DomainGeo>& doms, const lbm_params& p, double wp, double wm, char* buf,
                      int64_t bytes, hipStream_t s, BatchCtx** out) {
    if (p.layout == LBM_LAYOUT_BRICK) {
        BrickBatch* f = nullptr;
        lbm_status st = bbatch_init(doms, p, wp, wm, buf, bytes, s, &f);
        if (st != LBM_OK) return st;
        auto* b = new BatchCtx;
        b->flat = f;
        *out = b;
        return LBM_OK;
    }
    auto* b = new BatchCtx;
    lbm_status st = plan(doms, p, *b);
    if (st != LBM_OK) { delete b; return st; }
    if (bytes < b->bytes) { delete b; return set_error(LBM_E_NOMEM, "device buffer smaller than lbm_required_bytes"); }
    b->p = p;
    b->buf = buf;
    b->stream = s;
    b->k = make_consts(p, wp, wm, doms[0].desc.wall_hi_velocity);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete b;
        return set_error(LBM_E_DEVICE, "no HIP device");
    }
    b->cus = prop.multiProcessorCount;
    b->arch = prop.gcnArchName;
    int coop = 0;
    hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (!coop) { delete b; return set_error(LBM_E_DEVICE, "device does not support cooperative launches"); }
    std::vector<BatchDom> table(b->ndom);
    for (int d = 0; d < b->ndom; ++d) {
        const DomPlan& P = b->plans[d];
        DeviceImages im;
        std::string err;
        st = build_images(doms[d], LBM_LAYOUT_AA, BrickMap{}, P.stride, b->k, im, err);
        if (st != LBM_OK) { delete b; return set_error(st, err); }
        BatchDom& T = table[d];
        for (int k = 0; k < Q; ++k) T.pa[k] = reinterpret_cast<float*>(buf + P.off_pop) + k * P.stride;
        T.stride = (uint32_t)P.stride;
        T.info = reinterpret_cast<const uint32_t*>(buf + P.off_info);
        T.segbase = reinterpret_cast<const int32_t*>(buf + P.off_segbase);
        T.lparam = reinterpret_cast<const float*>(buf + P.off_lparam);
        T.pv = reinterpret_cast<float*>(buf + P.off_pop) + Q * P.stride;
        T.partial = reinterpret_cast<double*>(buf + P.off_partial);
        T.nx = doms[d].desc.nx; T.ny = doms[d].desc.ny; T.nz = doms[d].desc.nz; T.ncells = (int32_t)P.N;
        hipError_t e = hipMemcpyAsync(buf + P.off_info, im.info.data(), im.info.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(buf + P.off_segbase, im.segbase.data(), im.segbase.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(buf + P.off_lparam, im.lparam.data(), im.lparam.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && P.nseed > 0) {
            e = hipMemcpyAsync(buf + P.off_seed, im.seed_idx.data(), P.nseed * 8, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(buf + P.off_seed + P.nseed * 8, im.seed_val.data(), P.nseed * 4,
                                   hipMemcpyHostToDevice, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // host images go out of scope
        if (e != hipSuccess) {
            delete b;
            return set_error(LBM_E_DEVICE, std::string("batched upload: ") + hipGetErrorString(e));
        }
    }
    if (hipMemcpyAsync(buf + b->off_table, table.data(), table.size() * sizeof(BatchDom), hipMemcpyHostToDevice, s) !=
        hipSuccess) {
        delete b;
        return set_error(LBM_E_DEVICE, "upload domain table");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        int64_t cells = 0;
        for (auto& P : b->plans) cells += P.N;
        auto it = g_cache.find({b->arch, b->ndom, cells});
        if (it != g_cache.end()) { b->block = it->second.first; b->W = it->second.second; }
    }
    st = reset(b);
    if (st != LBM_OK) { delete b; return st; }
    *out = b;
    return LBM_OK;
}

lbm_status batch_step(BatchCtx* b, int64_t n) {
    if (b->flat) return bbatch_step(b->flat, n);
    if (n == 0) return LBM_OK;
    return run(b, 0, 0.0, 1, n, b->block, b->W);
}

lbm_status batch_run_to_steady(BatchCtx* b, double rel_tol, int64_t check_every, int64_t max_steps,
                               int64_t* steps_done) {
    if (b->flat) return bbatch_run_to_steady(b->flat, rel_tol, check_every, max_steps, steps_done);
    lbm_status s = run(b, 1, rel_tol, check_every, max_steps, b->block, b->W);
    if (s != LBM_OK) return s;
    for (int d = 0; d < b->ndom; ++d) steps_done[d] = b->steps[d];
    for (int d = 0; d < b->ndom; ++d)
        if (b->status[d] < 0) return set_error(LBM_E_UNSTABLE, "domain " + std::to_string(d) + " became unstable");
    return LBM_OK;
}

lbm_status batch_profile(BatchCtx* b, int dom, int axis, int comp, double* u_sup, double* u_int, double* por) {
    if (b->flat) return bbatch_profile(b->flat, dom, axis, comp, u_sup, u_int, por);
    std::vector<double> ps;
    lbm_status s = dom_plane_sums(b, dom, axis, ps);
    if (s != LBM_OK) return s;
    const auto& D = b->desc[dom];
    const int np = axis == 0 ? D.nx : (axis == 1 ? D.ny : D.nz);
    const double area = (double)b->plans[dom].N / np;
    for (int i = 0; i < np; ++i) {
        const double sum = ps[i * 6 + 1 + comp], nf = ps[i * 6 + 4];
        if (u_sup) u_sup[i] = sum / area;
        if (u_int) u_int[i] = nf > 0 ? sum / nf : 0.0;
        if (por) por[i] = nf / area;
    }
    return LBM_OK;
}

lbm_status batch_permeability(BatchCtx* b, int dom, int fa, int z0, int z1, double* k) {
    if (b->flat) return bbatch_permeability(b->flat, dom, fa, z0, z1, k);
    const auto& D = b->desc[dom];
    if (z0 < 0 || z1 > D.nz || z0 >= z1) return set_error(LBM_E_INVAL, "bad plane range");
    if (b->p.force[fa] == 0.0) return set_error(LBM_E_INVAL, "no body force along the flow axis");
    std::vector<double> sup((size_t)D.nz);
    lbm_status s = batch_profile(b, dom, 2, fa, sup.data(), nullptr, nullptr);
    if (s != LBM_OK) return s;
    double m = 0;
    for (int z = z0; z < z1; ++z) m += sup[z];
    m /= (z1 - z0);
    *k = b->p.rho0 * ((b->p.tau_plus - 0.5) / 3.0) * m / b->p.force[fa];
    return LBM_OK;
}

lbm_status batch_fields(BatchCtx* b, int dom, double* rho, double* u) {
    if (b->flat) return bbatch_fields(b->flat, dom, rho, u);
    const int64_t N = b->plans[dom].N, chunk = b->chunk;
    double* dv = reinterpret_cast<double*>(b->buf + b->off_fields);
    std::vector<double> h((size_t)chunk * 4);
    const MomentArgs m = dom_moments(b, dom);
    for (int64_t c0 = 0; c0 < N; c0 += chunk) {
        const int64_t n = std::min(chunk, N - c0);
        HIPCHK(launch_fields(m, c0, n, dv, b->stream), "fields");
        HIPCHK(hipMemcpyAsync(h.data(), dv, n * 4 * 8, hipMemcpyDeviceToHost, b->stream), "copy fields");
        HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
        if (rho) std::memcpy(rho + c0, h.data(), n * 8);
        if (u)
            for (int a = 0; a < 3; ++a) std::memcpy(u + a * N + c0, h.data() + (a + 1) * n, n * 8);
    }
    return LBM_OK;
}

lbm_status batch_totals(BatchCtx* b, int dom, double* mass, double* mom) {
    if (b->flat) return bbatch_totals(b->flat, dom, mass, mom);
    std::vector<double> ps;
    lbm_status s = dom_plane_sums(b, dom, 2, ps);
    if (s != LBM_OK) return s;
    double m = 0, j[3] = {0, 0, 0}, bad = 0;
    for (int z = 0; z < b->desc[dom].nz; ++z) {
        m += ps[z * 6];
        for (int a = 0; a < 3; ++a) j[a] += ps[z * 6 + 1 + a];
        bad += ps[z * 6 + 5];
    }
    if (mass) *mass = m;
    if (mom)
        for (int a = 0; a < 3; ++a) mom[a] = b->p.rho0 * j[a];
    if (bad > 0) return set_error(LBM_E_UNSTABLE, "NaN or |u| >= 0.4 in the flow field");
    return LBM_OK;
}

// image: 4 int64 header {magic, steps of domain 0, ndom, 0}, then per domain
// {steps, status, uprev} and its populations
static const int64_t kBatchMagic = 0x4c424d4241544348;  // "LBMBATCH"

lbm_status batch_state_bytes(BatchCtx* b, int64_t* bytes) {
    if (b->flat) return bbatch_state_bytes(b->flat, bytes);
    int64_t n = 32;
    for (auto& P : b->plans) n += 24 + P.grid * 4;
    *bytes = n;
    return LBM_OK;
}

lbm_status batch_save(BatchCtx* b, void* host, int64_t bytes, int64_t steps) {
    if (b->flat) return bbatch_save(b->flat, host, bytes, steps);
    (void)bytes;
    int64_t* h = reinterpret_cast<int64_t*>(host);
    h[0] = kBatchMagic; h[1] = steps; h[2] = b->ndom; h[3] = 0;
    char* o = reinterpret_cast<char*>(host) + 32;
    std::vector<double> up(b->ndom);
    HIPCHK(hipMemcpyAsync(up.data(), b->buf + b->off_uprev, b->ndom * 8, hipMemcpyDeviceToHost, b->stream), "save");
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    for (int d = 0; d < b->ndom; ++d) {
        const DomPlan& P = b->plans[d];
        int64_t meta[3] = {b->steps[d], b->status[d], 0};
        std::memcpy(&meta[2], &up[d], 8);
        std::memcpy(o, meta, 24);
        o += 24;
        HIPCHK(hipMemcpyAsync(o, b->buf + P.off_pop, P.grid * 4, hipMemcpyDeviceToHost, b->stream), "save");
        o += P.grid * 4;
    }
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

lbm_status batch_load(BatchCtx* b, const void* host, int64_t bytes) {
    if (b->flat) return bbatch_load(b->flat, host, bytes);
    (void)bytes;
    const int64_t* h = reinterpret_cast<const int64_t*>(host);
    if (h[0] != kBatchMagic || h[2] != b->ndom) return set_error(LBM_E_INVAL, "not a state image of this batch");
    const char* o = reinterpret_cast<const char*>(host) + 32;
    std::vector<double> up(b->ndom);
    for (int d = 0; d < b->ndom; ++d) {
        const DomPlan& P = b->plans[d];
        int64_t meta[3];
        std::memcpy(meta, o, 24);
        o += 24;
        b->steps[d] = meta[0];
        b->status[d] = (int32_t)meta[1];
        std::memcpy(&up[d], &meta[2], 8);
        HIPCHK(hipMemcpyAsync(b->buf + P.off_pop, o, P.grid * 4, hipMemcpyHostToDevice, b->stream), "load");
        o += P.grid * 4;
    }
    HIPCHK(hipMemcpyAsync(b->buf + b->off_steps, b->steps.data(), b->ndom * 8, hipMemcpyHostToDevice, b->stream),
           "load");
    HIPCHK(hipMemcpyAsync(b->buf + b->off_status, b->status.data(), b->ndom * 4, hipMemcpyHostToDevice, b->stream),
           "load");
    HIPCHK(hipMemcpyAsync(b->buf + b->off_uprev, up.data(), b->ndom * 8, hipMemcpyHostToDevice, b->stream), "load");
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

lbm_status batch_autotune(BatchCtx* b, int32_t steps_per_trial) {
    if (b->flat) return bbatch_autotune(b->flat, steps_per_trial);
    for (int d = 0; d < b->ndom; ++d)
        if (b->steps[d] != 0) return set_error(LBM_E_STATE, "autotune a batch before stepping it");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "event");
    HIPCHK(hipEventCreate(&e1), "event");
    float best = 1e30f;
    int bb = b->block, bw = b->W;
    lbm_status s = LBM_OK;
    for (int block : {256, 512, 1024})
        for (int W : {1, 2, 4, 8, 16}) {
            s = reset(b);
            if (s != LBM_OK) break;
            hipEventRecord(e0, b->stream);
            s = run(b, 0, 0.0, 1, steps_per_trial, block, W);
            hipEventRecord(e1, b->stream);
            hipEventSynchronize(e1);
            if (s != LBM_OK) break;
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; bb = block; bw = W; }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    lbm_status s2 = reset(b);
    if (s != LBM_OK) return s;
    if (s2 != LBM_OK) return s2;
    b->block = bb;
    b->W = bw;
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t cells = 0;
    for (auto& P : b->plans) cells += P.N;
    g_cache[{b->arch, b->ndom, cells}] = {bb, bw};
    return LBM_OK;
}

lbm_status batch_set_launch(BatchCtx* b, int32_t block, int32_t W) {
    if (b->flat) return bbatch_set_launch(b->flat, block, W);
    if (block != 256 && block != 512 && block != 1024) return set_error(LBM_E_INVAL, "block must be 256, 512 or 1024");
    if (W < 1 || W > 64) return set_error(LBM_E_INVAL, "workgroups per domain must be in [1, 64]");
    b->block = block;
    b->W = W;
    return LBM_OK;
}

lbm_status batch_get_launch(BatchCtx* b, int32_t* block, int32_t* W) {
    if (b->flat) return bbatch_get_launch(b->flat, block, W);
    if (block) *block = b->block;
    if (W) *W = b->W;
    return LBM_OK;
}

void batch_destroy(BatchCtx* b) {
    if (b && b->flat) bbatch_destroy(b->flat);
    delete b;
}

// "aa-batch ARCH DOMAINS CELLS BLOCK WORKGROUPS_PER_DOMAIN"
void abatch_tuning_export(std::string& out) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_cache)
        out += "aa-batch " + kv.first.arch + " " + std::to_string(kv.first.ndom) + " " +
               std::to_string(kv.first.cells) + " " + std::to_string(kv.second.first) + " " +
               std::to_string(kv.second.second) + "\n";
}

int abatch_tuning_import(const std::vector<std::string>& f, bool apply) {
    if (f.empty() || f[0] != "aa-batch") return 0;
    int64_t nd = 0, cells = 0, block = 0, w = 0;
    if (f.size() != 6 || f[1].empty() || !parse_i64(f[2], nd) || !parse_i64(f[3], cells) || !parse_i64(f[4], block) ||
        !parse_i64(f[5], w))
        return -1;
    if (nd < 1 || cells < 1 || (block != 256 && block != 512 && block != 1024) || w < 1 || w > 64) return -1;
    if (apply) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[{f[1], (int)nd, cells}] = {(int)block, (int)w};
    }
    return 1;
}

}  // namespace lbm
