// C ABI of the pore-scale solver: geometry objects, contexts bound to a
// caller-owned device buffer and stream, stepping, FP64 reductions,
// checkpointing and the sweep autotuner.  Single-domain contexts run the
// fused sweep (two-grid, AA or brick); multi-domain contexts run the batched
// persistent kernel (batch.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <limits>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"
#include "tuning.hpp"

using namespace lbm;

struct lbm_geometry {
    std::vector<DomainGeo> doms;
};

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const std::string& m) {
    g_err = m;
    return s;
}

lbm_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_E_DEVICE;
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Relaxation rates (Sec. 2.1): 1/omega+ = tau+ = 3 nu + 1/2; TRT omega- from
// Lambda = (tau+ - 1/2)(tau- - 1/2); BGK omega- = omega+.
lbm_status rates(const lbm_params& p, double& wp, double& wm) {
    if (p.collision != LBM_BGK && p.collision != LBM_TRT) return fail(LBM_E_INVAL, "unknown collision model");
    if (!(p.tau_plus > 0.5) || !std::isfinite(p.tau_plus)) return fail(LBM_E_INVAL, "tau_plus must exceed 1/2");
    if (!(p.rho0 > 0.0)) return fail(LBM_E_INVAL, "rho0 must be positive");
    for (double f : p.force)
        if (!std::isfinite(f)) return fail(LBM_E_INVAL, "force must be finite");
    const double tm = (p.collision == LBM_TRT) ? 0.5 + p.magic_lambda / (p.tau_plus - 0.5) : p.tau_plus;
    wp = 1.0 / p.tau_plus;
    wm = 1.0 / tm;
    if (!(wm > 0.0 && wm < 2.0)) return fail(LBM_E_INVAL, "omega- must lie in (0, 2)");
    if (p.layout != LBM_LAYOUT_TWOGRID && p.layout != LBM_LAYOUT_AA && p.layout != LBM_LAYOUT_BRICK)
        return fail(LBM_E_INVAL, "unknown layout");
    return LBM_OK;
}

// --------------------------------------------------------- memory plan --
struct Plan {
    int64_t N = 0, stride = 0, nb = 0, nl = 0, np = 0, chunk = 0, nseed = 0;
    int64_t NS = 0;            // stored cells (N, or 64 per stored brick)
    int64_t nbricks = 0, nbmap = 0;  // brick layout: stored bricks, entries of the brick map
    int64_t grid = 0;  // floats per state block: Q population arrays + the partial values
    int64_t off_pop = 0, off_info = 0, off_segbase = 0, off_lparam = 0, off_seed = 0, off_red = 0, off_fields = 0;
    int64_t off_nbr = 0, off_bmap = 0;
    int64_t total = 0;
};

// bm: the brick map (counts only) for the brick layout, else unused
Plan plan_single(const DomainGeo& g, const lbm_params& p, const BrickMap& bm) {
    Plan P;
    const auto& d = g.desc;
    P.N = g.ncells();
    const bool brick = p.layout == LBM_LAYOUT_BRICK;
    P.NS = brick ? bm.nstored * 64 : P.N;
    if (brick) {
        P.nbricks = bm.nstored;
        P.nbmap = (int64_t)bm.bx * bm.by * bm.bz;
    }
    // pad each population array so that the 19 arrays do not start on the
    // same power-of-two boundary (HBM channel interleave)
    P.stride = align_up(P.NS, 256) + 320;
    P.nl = (int64_t)g.lcell.size();
    int64_t nb = 0;
    for (size_t i = 0; i < g.lcell.size(); ++i)
        if (i == 0 || g.lcell[i] != g.lcell[i - 1]) ++nb;
    P.nb = nb;
    const bool moving = d.wall_hi_velocity[0] != 0.0 || d.wall_hi_velocity[1] != 0.0 || d.wall_hi_velocity[2] != 0.0;
    if (moving)
        for (size_t i = 0; i < g.lsurf.size(); ++i)
            if (g.lsurf[i] == SURF_WALL_HI) ++P.nseed;
    P.np = std::max(d.nx, std::max(d.ny, d.nz));
    P.chunk = std::min<int64_t>(P.N, std::max<int64_t>((int64_t)d.nx * d.ny, 1 << 20));
    int64_t o = 0;
    const int64_t ngrid = (p.layout == LBM_LAYOUT_AA) ? 1 : 2;
    P.grid = Q * P.stride + align_up(P.nl + Q, 64);
    P.off_pop = o; o = align_up(o + ngrid * P.grid * 4, 256);
    P.off_info = o; o = align_up(o + P.NS * 4, 256);
    P.off_segbase = o; o = align_up(o + ((P.NS >> SEG_SHIFT) + 1) * 4, 256);
    P.off_nbr = o; o = align_up(o + P.nbricks * 27 * 4, 256);
    P.off_bmap = o; o = align_up(o + P.nbmap * 4, 256);
    P.off_lparam = o; o = align_up(o + (P.nl + Q) * 4, 256);
    P.off_seed = o; o = align_up(o + std::max<int64_t>(P.nseed, 1) * 12, 256);
    P.off_red = o; o = align_up(o + P.np * 6 * 8, 256);
    P.off_fields = o; o = align_up(o + P.chunk * 4 * 8, 256);
    P.total = o;
    return P;
}

struct TuneKey {
    std::string arch;
    int nx, ny, nz, layout, bc;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, nx, ny, nz, layout, bc) < std::tie(o.arch, o.nx, o.ny, o.nz, o.layout, o.bc);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;

// layout autotuner cache: (architecture, domains, first domain's shape, total
// cells, bc, collision) -> (layout, ms per step)
struct LayoutKey {
    std::string arch;
    int ndom, nx, ny, nz, bc, collision;
    int64_t cells;
    bool operator<(const LayoutKey& o) const {
        return std::tie(arch, ndom, nx, ny, nz, bc, collision, cells) <
               std::tie(o.arch, o.ndom, o.nx, o.ny, o.nz, o.bc, o.collision, o.cells);
    }
};
std::map<LayoutKey, std::pair<int, double>> g_layout_cache;

}  // namespace

lbm_status lbm::set_error(lbm_status s, const std::string& msg) { return fail(s, msg); }

int64_t lbm::max_links() {
    const int64_t hard = ((int64_t)1 << 30) - Q;
    const char* e = std::getenv("MI355LBM_MAX_LINKS");
    if (e && *e) {
        const long long v = std::strtoll(e, nullptr, 10);
        if (v >= 0 && v < hard) return (int64_t)v;
    }
    return hard;
}

struct lbm_ctx {
    int ndom = 1;
    lbm_params p{};
    double wp = 0, wm = 0;
    hipStream_t stream = nullptr;
    char* buf = nullptr;
    int64_t bytes = 0;
    int64_t steps = 0;
    // single domain
    lbm_domain_desc d{};
    Plan P;
    int cur = 0;       // two-grid: which grid holds the state
    int parity = -1;   // AA: parity of the last step (-1 none)
    int block = 256;
    int xcd_remap = 1;
    int nt = 0;
    int cpt = 1;  // cells per thread: tiles each workgroup steps in turn
    SweepArgs sa{};
    int64_t n_fluid = 0;
    std::string arch;
    // batched
    BatchCtx* batch = nullptr;
};

namespace {

// launch flags (LBM_LAUNCH_*) <-> context fields; flags are validated by
// the caller
void set_flags(lbm_ctx* c, int flags) {
    c->xcd_remap = (flags & LBM_LAUNCH_XCD_REMAP) ? 1 : 0;
    c->nt = (flags & LBM_LAUNCH_NONTEMPORAL) ? 1 : 0;
    c->cpt = (flags & LBM_LAUNCH_CELLS_4) ? 4 : ((flags & LBM_LAUNCH_CELLS_2) ? 2 : 1);
}

int get_flags(const lbm_ctx* c) {
    return (c->xcd_remap ? LBM_LAUNCH_XCD_REMAP : 0) | (c->nt ? LBM_LAUNCH_NONTEMPORAL : 0) |
           (c->cpt == 2 ? LBM_LAUNCH_CELLS_2 : 0) | (c->cpt == 4 ? LBM_LAUNCH_CELLS_4 : 0);
}

MomentArgs moment_args(const lbm_ctx* c) {
    MomentArgs m{};
    m.A = reinterpret_cast<const float*>(c->buf + c->P.off_pop) + (int64_t)c->cur * c->P.grid;
    m.stride = c->P.stride;
    m.info = reinterpret_cast<const uint32_t*>(c->buf + c->P.off_info);
    m.bmap = c->p.layout == LBM_LAYOUT_BRICK ? reinterpret_cast<const int32_t*>(c->buf + c->P.off_bmap) : nullptr;
    m.nx = c->d.nx; m.ny = c->d.ny; m.nz = c->d.nz;
    m.layout = c->p.layout;
    m.parity = c->parity;
    m.rho0 = c->p.rho0;
    for (int a = 0; a < 3; ++a) m.F[a] = c->p.force[a];
    return m;
}

lbm_status plane_sums(lbm_ctx* c, int axis, std::vector<double>& out) {
    const int np = axis == 0 ? c->d.nx : (axis == 1 ? c->d.ny : c->d.nz);
    double* red = reinterpret_cast<double*>(c->buf + c->P.off_red);
    HIP_TRY(launch_plane_sums(moment_args(c), axis, red, c->stream), "plane reduction launch");
    out.assign((size_t)np * 6, 0.0);
    HIP_TRY(hipMemcpyAsync(out.data(), red, out.size() * 8, hipMemcpyDeviceToHost, c->stream), "copy plane sums");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
    return LBM_OK;
}

}  // namespace

CellConsts lbm::make_consts(const lbm_params& p, double wp, double wm, const double* wall_velocity) {
    CellConsts k{};
    k.wp = (float)wp;
    k.wm = (float)wm;
    k.cp = (float)(1.0 - 0.5 * wp);
    k.cm = (float)(1.0 - 0.5 * wm);
    k.rho0 = (float)p.rho0;
    k.inv_rho0 = (float)(1.0 / p.rho0);
    for (int i = 0; i < 3; ++i) k.F[i] = (float)p.force[i];
    for (int i = 0; i < 3; ++i) k.fh[i] = (float)(0.5 * p.force[i] / p.rho0);
    const double cp = 1.0 - 0.5 * wp, cm = 1.0 - 0.5 * wm;
    k.om1 = (float)(1.0 - wp);
    k.hp = (float)(-0.5 * wp);
    k.hm = (float)(-0.5 * wm);
    k.a_uu = (float)(-1.5 * wp * p.rho0);
    k.a_uF = (float)(-3.0 * cp);
    for (int c = 0; c < 2; ++c) {
        const double w = c == 0 ? 1.0 / 18.0 : 1.0 / 36.0;
        k.beta[c] = (float)(4.5 * wp * w * p.rho0);
        k.delta[c] = (float)(3.0 * wm * w * p.rho0);
    }
    for (int pr = 0; pr < 9; ++pr) {
        const int j = 2 * pr + 1;
        const double eF = D3Q19::ex[j] * p.force[0] + D3Q19::ey[j] * p.force[1] + D3Q19::ez[j] * p.force[2];
        k.gam[pr] = (float)(9.0 * cp * weight(j) * eF);
        k.zet[pr] = (float)(3.0 * cm * weight(j) * eF);
    }
    for (int j = 0; j < Q; ++j) {
        const double eu = D3Q19::ex[j] * wall_velocity[0] + D3Q19::ey[j] * wall_velocity[1] +
                          D3Q19::ez[j] * wall_velocity[2];
        k.wterm[j] = (float)(6.0 * weight(j) * p.rho0 * eu);
    }
    return k;
}

namespace {

int flow_axis(const lbm_params& p) {
    int a = 0;
    for (int i = 1; i < 3; ++i)
        if (std::fabs(p.force[i]) > std::fabs(p.force[a])) a = i;
    return a;
}

lbm_status check_ctx(lbm_ctx* c, int32_t dom) {
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (dom < 0 || dom >= c->ndom) return fail(LBM_E_INVAL, "domain index out of range");
    return LBM_OK;
}

lbm_status step_single(lbm_ctx* c, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        SweepArgs a = c->sa;
        float* base = reinterpret_cast<float*>(c->buf + c->P.off_pop);
        int par = P_EVEN;
        if (c->p.layout != LBM_LAYOUT_AA) {
            a.A = base + (int64_t)c->cur * c->P.grid;
            a.B = base + (int64_t)(1 - c->cur) * c->P.grid;
        } else {
            a.A = base;
            a.B = nullptr;
            par = (c->steps % 2 == 0) ? P_EVEN : P_ODD;
        }
        for (int k = 0; k < Q; ++k) {
            a.pa[k] = a.A + k * c->P.stride;
            a.pb[k] = a.B ? a.B + k * c->P.stride : nullptr;
        }
        a.pva = a.A + Q * c->P.stride;
        a.pvb = a.B ? a.B + Q * c->P.stride : a.pva;
        a.xcd_remap = c->xcd_remap;
        a.nt = c->nt;
        a.cpt = c->cpt;
        hipError_t e = launch_sweep(a, c->p.layout, par, c->d.bc, c->block, c->stream);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
        if (c->p.layout != LBM_LAYOUT_AA) c->cur = 1 - c->cur;
        else c->parity = par;
        ++c->steps;
    }
    return LBM_OK;
}

// rest state: every population and partial value zero (f = w rho0), the
// moving-wall partial values seeded
hipError_t reset_state(lbm_ctx* c) {
    const int64_t ngrid = (c->p.layout == LBM_LAYOUT_AA) ? 1 : 2;
    float* pop = reinterpret_cast<float*>(c->buf + c->P.off_pop);
    hipError_t e = launch_fill_zero(pop, ngrid * c->P.grid, c->stream);
    if (e == hipSuccess && c->P.nseed > 0)
        e = launch_scatter(pop, reinterpret_cast<const int64_t*>(c->buf + c->P.off_seed),
                           reinterpret_cast<const float*>(c->buf + c->P.off_seed + c->P.nseed * 8), c->P.nseed,
                           c->stream);
    c->steps = 0;
    c->cur = 0;
    c->parity = -1;
    return e;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_geometry_build(const lbm_domain_desc* domains, int32_t n_domains, lbm_geometry** out) {
    if (!domains || !out || n_domains < 1) return fail(LBM_E_INVAL, "bad arguments");
    *out = nullptr;
    try {
        auto* g = new lbm_geometry;
        g->doms.resize(n_domains);
        for (int i = 0; i < n_domains; ++i) {
            std::string err;
            lbm_status s = build_domain(domains[i], g->doms[i], err);
            if (s != LBM_OK) {
                delete g;
                return fail(s, "domain " + std::to_string(i) + ": " + err);
            }
        }
        *out = g;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_E_NOMEM, "host memory exhausted while building the geometry");
    }
}

lbm_status lbm_geometry_flags(const lbm_geometry* g, int32_t dom, uint8_t* host_flags) {
    if (!g || !host_flags || dom < 0 || dom >= (int)g->doms.size()) return fail(LBM_E_INVAL, "bad arguments");
    const auto& f = g->doms[dom].flags;
    std::memcpy(host_flags, f.data(), f.size());
    return LBM_OK;
}

lbm_status lbm_geometry_links(const lbm_geometry* g, int32_t dom, int64_t* n, int64_t* cell, int8_t* dir,
                              double* q) {
    if (!g || !n || dom < 0 || dom >= (int)g->doms.size()) return fail(LBM_E_INVAL, "bad arguments");
    const auto& D = g->doms[dom];
    const int64_t nl = (int64_t)D.lcell.size();
    if (cell || dir || q) {
        if (*n < nl) { *n = nl; return fail(LBM_E_NOMEM, "link arrays too small"); }
        if (cell) std::memcpy(cell, D.lcell.data(), nl * sizeof(int64_t));
        if (dir) std::memcpy(dir, D.ldir.data(), nl);
        if (q) std::memcpy(q, D.lq.data(), nl * sizeof(double));
    }
    *n = nl;
    return LBM_OK;
}

lbm_status lbm_geometry_info(const lbm_geometry* g, int32_t dom, int32_t* n_domains, int64_t* n_fluid,
                             int64_t* n_links) {
    if (!g || dom < 0 || dom >= (int)g->doms.size()) return fail(LBM_E_INVAL, "bad arguments");
    if (n_domains) *n_domains = (int32_t)g->doms.size();
    if (n_fluid) *n_fluid = g->doms[dom].n_fluid;
    if (n_links) *n_links = (int64_t)g->doms[dom].lcell.size();
    return LBM_OK;
}

void lbm_geometry_free(lbm_geometry* g) { delete g; }

lbm_status lbm_required_bytes(const lbm_geometry* g, const lbm_params* p, int64_t* bytes) {
    if (!g || !p || !bytes) return fail(LBM_E_INVAL, "bad arguments");
    double wp, wm;
    lbm_status s = rates(*p, wp, wm);
    if (s != LBM_OK) return s;
    if (g->doms.size() == 1) {
        BrickMap bm;
        if (p->layout == LBM_LAYOUT_BRICK) {
            if (!brick_dims_ok(g->doms[0].desc)) return fail(LBM_E_INVAL, "brick layout needs nx, ny, nz divisible by 4");
            build_brick_map(g->doms[0], bm, false);
        }
        if ((int64_t)g->doms[0].lcell.size() > max_links())
            return fail(LBM_E_INVAL, "too many boundary links in one domain (limit 2^30 - 19)");
        *bytes = plan_single(g->doms[0], *p, bm).total;
        return LBM_OK;
    }
    return batch_required_bytes(g->doms, *p, bytes);
}

lbm_status lbm_init(const lbm_geometry* g, const lbm_params* p, void* dev_buf, int64_t bytes, void* hip_stream,
                    lbm_ctx** out) {
    if (!g || !p || !dev_buf || !out) return fail(LBM_E_INVAL, "bad arguments");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256 != 0) return fail(LBM_E_INVAL, "device buffer must be 256-byte aligned");
    double wp, wm;
    lbm_status s = rates(*p, wp, wm);
    if (s != LBM_OK) return s;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "no HIP device");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "device properties");
    auto* c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_E_NOMEM, "host allocation");
    c->p = *p;
    c->wp = wp;
    c->wm = wm;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->buf = reinterpret_cast<char*>(dev_buf);
    c->bytes = bytes;
    c->arch = prop.gcnArchName;
    c->ndom = (int)g->doms.size();
    if (c->ndom > 1) {
        s = batch_init(g->doms, *p, wp, wm, c->buf, bytes, c->stream, &c->batch);
        if (s != LBM_OK) { delete c; return s; }
        *out = c;
        return LBM_OK;
    }
    const DomainGeo& G = g->doms[0];
    if ((int64_t)G.lcell.size() > max_links()) {
        delete c;
        return fail(LBM_E_INVAL, "too many boundary links in one domain (limit 2^30 - 19)");
    }
    BrickMap bm;
    if (p->layout == LBM_LAYOUT_BRICK) {
        if (!brick_dims_ok(G.desc)) {
            delete c;
            return fail(LBM_E_INVAL, "brick layout needs nx, ny, nz divisible by 4");
        }
        try {
            build_brick_map(G, bm, true);
        } catch (const std::bad_alloc&) {
            delete c;
            return fail(LBM_E_NOMEM, "host memory for the brick map");
        }
    }
    c->d = G.desc;
    c->d.spheres = nullptr;
    c->d.n_spheres = 0;
    c->P = plan_single(G, *p, bm);
    c->n_fluid = G.n_fluid;
    if (bytes < c->P.total) {
        delete c;
        return fail(LBM_E_NOMEM, "device buffer smaller than lbm_required_bytes");
    }
    // host images of the cell info, boundary-cell records and link parameters
    const int64_t N = c->P.N;
    DeviceImages im;
    {
        std::string err;
        lbm_status st = LBM_OK;
        try {
            st = build_images(G, p->layout, bm, c->P.stride, make_consts(*p, wp, wm, G.desc.wall_hi_velocity), im,
                              err);
        } catch (const std::bad_alloc&) {
            st = LBM_E_NOMEM;
            err = "host memory for the device images";
        }
        if (st != LBM_OK) {
            delete c;
            return fail(st, err);
        }
    }
    const int nx = G.desc.nx, ny = G.desc.ny, nz = G.desc.nz;
    SweepArgs& a = c->sa;
    a.stride = c->P.stride;
    a.info = reinterpret_cast<const uint32_t*>(c->buf + c->P.off_info);
    a.segbase = reinterpret_cast<const int32_t*>(c->buf + c->P.off_segbase);
    a.lparam = reinterpret_cast<const float*>(c->buf + c->P.off_lparam);
    a.nx = nx; a.ny = ny; a.nz = nz; a.ncells = (int32_t)N;
    a.nbr = reinterpret_cast<const int32_t*>(c->buf + c->P.off_nbr);
    a.nbricks = (int32_t)c->P.nbricks;
    a.k = make_consts(*p, wp, wm, G.desc.wall_hi_velocity);
    // launch configuration from the tuning cache, if any
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find({c->arch, nx, ny, nz, p->layout, G.desc.bc});
        if (it != g_tune_cache.end()) {
            c->block = it->second.first;
            set_flags(c, it->second.second);
        }
    }
    hipError_t e = hipSuccess;
    const auto& seed_idx = im.seed_idx;
    const auto& seed_val = im.seed_val;
    const auto& info = im.info;
    const auto& segbase = im.segbase;
    const auto& lparam = im.lparam;
    if ((int64_t)seed_idx.size() != c->P.nseed) {
        e = hipErrorInvalidValue;
    } else if (c->P.nseed > 0) {
        e = hipMemcpyAsync(c->buf + c->P.off_seed, seed_idx.data(), seed_idx.size() * 8, hipMemcpyHostToDevice,
                           c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->buf + c->P.off_seed + c->P.nseed * 8, seed_val.data(), seed_val.size() * 4,
                               hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess) e = reset_state(c);
    if (e == hipSuccess && (int64_t)info.size() != c->P.NS) e = hipErrorInvalidValue;
    if (e == hipSuccess && c->P.NS > 0)
        e = hipMemcpyAsync(c->buf + c->P.off_info, info.data(), c->P.NS * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->P.nbricks > 0)
        e = hipMemcpyAsync(c->buf + c->P.off_nbr, bm.nbr.data(), bm.nbr.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->P.nbmap > 0)
        e = hipMemcpyAsync(c->buf + c->P.off_bmap, bm.id.data(), bm.id.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->buf + c->P.off_segbase, segbase.data(), segbase.size() * 4, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->buf + c->P.off_lparam, lparam.data(), lparam.size() * 4, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host images go out of scope
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "context upload");
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return fail(LBM_E_INVAL, "bad arguments");
    if (c->batch) {
        lbm_status s = batch_step(c->batch, n);
        if (s == LBM_OK) c->steps += n;
        return s;
    }
    return step_single(c, n);
}

lbm_status lbm_run_to_steady(lbm_ctx* c, double rel_tol, int64_t check_every, int64_t max_steps,
                             int64_t* steps_done) {
    if (!c || !(rel_tol >= 0) || check_every < 1 || max_steps < 0 || !steps_done)
        return fail(LBM_E_INVAL, "bad arguments");
    if (c->batch) return batch_run_to_steady(c->batch, rel_tol, check_every, max_steps, steps_done);
    const int fa = flow_axis(c->p);
    double prev = NAN;
    int64_t done = 0;
    std::vector<double> ps;
    while (done < max_steps) {
        const int64_t n = std::min(check_every, max_steps - done);
        lbm_status s = step_single(c, n);
        if (s != LBM_OK) return s;
        done += n;
        s = plane_sums(c, 2, ps);
        if (s != LBM_OK) return s;
        double U = 0.0, bad = 0.0;
        for (int z = 0; z < c->d.nz; ++z) { U += ps[z * 6 + 1 + fa]; bad += ps[z * 6 + 5]; }
        if (bad > 0) { *steps_done = done; return fail(LBM_E_UNSTABLE, "NaN or |u| >= 0.4 in the flow field"); }
        if (n == check_every && std::isfinite(prev) && std::fabs(U - prev) <= rel_tol * std::fabs(U)) {
            *steps_done = done;
            return LBM_OK;
        }
        prev = U;
    }
    *steps_done = max_steps;
    return LBM_OK;
}

lbm_status lbm_average_profile(lbm_ctx* c, int32_t dom, int32_t axis, int32_t comp, double* u_sup, double* u_int,
                               double* porosity) {
    lbm_status s = check_ctx(c, dom);
    if (s != LBM_OK) return s;
    if (axis < 0 || axis > 2 || comp < 0 || comp > 2) return fail(LBM_E_INVAL, "axis and comp must be 0, 1 or 2");
    if (c->batch) return batch_profile(c->batch, dom, axis, comp, u_sup, u_int, porosity);
    std::vector<double> ps;
    s = plane_sums(c, axis, ps);
    if (s != LBM_OK) return s;
    const int np = axis == 0 ? c->d.nx : (axis == 1 ? c->d.ny : c->d.nz);
    const double area = (double)c->P.N / np;
    for (int i = 0; i < np; ++i) {
        const double sum = ps[i * 6 + 1 + comp], nf = ps[i * 6 + 4];
        if (u_sup) u_sup[i] = sum / area;
        if (u_int) u_int[i] = nf > 0 ? sum / nf : 0.0;
        if (porosity) porosity[i] = nf / area;
    }
    return LBM_OK;
}

lbm_status lbm_permeability(lbm_ctx* c, int32_t dom, int32_t fa, int32_t z0, int32_t z1, double* k) {
    lbm_status s = check_ctx(c, dom);
    if (s != LBM_OK) return s;
    if (!k || fa < 0 || fa > 2) return fail(LBM_E_INVAL, "bad arguments");
    if (c->batch) return batch_permeability(c->batch, dom, fa, z0, z1, k);
    if (z0 < 0 || z1 > c->d.nz || z0 >= z1) return fail(LBM_E_INVAL, "bad plane range");
    if (c->p.force[fa] == 0.0) return fail(LBM_E_INVAL, "no body force along the flow axis");
    std::vector<double> sup((size_t)c->d.nz);
    s = lbm_average_profile(c, dom, 2, fa, sup.data(), nullptr, nullptr);
    if (s != LBM_OK) return s;
    double m = 0;
    for (int z = z0; z < z1; ++z) m += sup[z];
    m /= (z1 - z0);
    const double nu = (c->p.tau_plus - 0.5) / 3.0;
    *k = c->p.rho0 * nu * m / c->p.force[fa];
    return LBM_OK;
}

lbm_status lbm_fields(lbm_ctx* c, int32_t dom, double* host_rho, double* host_u) {
    lbm_status s = check_ctx(c, dom);
    if (s != LBM_OK) return s;
    if (c->batch) return batch_fields(c->batch, dom, host_rho, host_u);
    const int64_t N = c->P.N, chunk = c->P.chunk;
    double* dv = reinterpret_cast<double*>(c->buf + c->P.off_fields);
    std::vector<double> h((size_t)chunk * 4);
    for (int64_t c0 = 0; c0 < N; c0 += chunk) {
        const int64_t n = std::min(chunk, N - c0);
        HIP_TRY(launch_fields(moment_args(c), c0, n, dv, c->stream), "fields launch");
        HIP_TRY(hipMemcpyAsync(h.data(), dv, n * 4 * 8, hipMemcpyDeviceToHost, c->stream), "copy fields");
        HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
        if (host_rho) std::memcpy(host_rho + c0, h.data(), n * 8);
        if (host_u)
            for (int a = 0; a < 3; ++a) std::memcpy(host_u + a * N + c0, h.data() + (a + 1) * n, n * 8);
    }
    return LBM_OK;
}

lbm_status lbm_totals(lbm_ctx* c, int32_t dom, double* mass, double momentum[3]) {
    lbm_status s = check_ctx(c, dom);
    if (s != LBM_OK) return s;
    if (c->batch) return batch_totals(c->batch, dom, mass, momentum);
    std::vector<double> ps;
    s = plane_sums(c, 2, ps);
    if (s != LBM_OK) return s;
    double m = 0, j[3] = {0, 0, 0}, bad = 0;
    for (int z = 0; z < c->d.nz; ++z) {
        m += ps[z * 6];
        for (int a = 0; a < 3; ++a) j[a] += ps[z * 6 + 1 + a];
        bad += ps[z * 6 + 5];
    }
    if (mass) *mass = m;
    if (momentum)
        for (int a = 0; a < 3; ++a) momentum[a] = c->p.rho0 * j[a];
    if (bad > 0) return fail(LBM_E_UNSTABLE, "NaN or |u| >= 0.4 in the flow field");
    return LBM_OK;
}

// checkpoint image: 4 int64 header {magic, steps, parity, cur} + the current
// state block (populations and partial bounce-back values)
static const int64_t kMagic = 0x4c424d53544154;  // "LBMSTAT"

lbm_status lbm_state_bytes(lbm_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return fail(LBM_E_INVAL, "bad arguments");
    if (c->batch) return batch_state_bytes(c->batch, bytes);
    *bytes = 32 + c->P.grid * 4;
    return LBM_OK;
}

lbm_status lbm_save(lbm_ctx* c, void* host_buf, int64_t bytes) {
    int64_t need = 0;
    lbm_status s = lbm_state_bytes(c, &need);
    if (s != LBM_OK) return s;
    if (!host_buf || bytes < need) return fail(LBM_E_NOMEM, "host buffer too small");
    if (c->batch) return batch_save(c->batch, host_buf, bytes, c->steps);
    int64_t* h = reinterpret_cast<int64_t*>(host_buf);
    h[0] = kMagic; h[1] = c->steps; h[2] = c->parity; h[3] = 0;
    char* dst = reinterpret_cast<char*>(host_buf) + 32;
    const char* pop = c->buf + c->P.off_pop + (int64_t)c->cur * c->P.grid * 4;
    HIP_TRY(hipMemcpyAsync(dst, pop, c->P.grid * 4, hipMemcpyDeviceToHost, c->stream), "save populations");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
    return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* c, const void* host_buf, int64_t bytes) {
    int64_t need = 0;
    lbm_status s = lbm_state_bytes(c, &need);
    if (s != LBM_OK) return s;
    if (!host_buf || bytes < need) return fail(LBM_E_INVAL, "state image too small");
    const int64_t* h = reinterpret_cast<const int64_t*>(host_buf);
    if (c->batch) {
        s = batch_load(c->batch, host_buf, bytes);
        if (s == LBM_OK) c->steps = h[1];
        return s;
    }
    if (h[0] != kMagic) return fail(LBM_E_INVAL, "not a state image");
    const char* src = reinterpret_cast<const char*>(host_buf) + 32;
    c->cur = 0;
    HIP_TRY(hipMemcpyAsync(c->buf + c->P.off_pop, src, c->P.grid * 4, hipMemcpyHostToDevice, c->stream),
            "load populations");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
    c->steps = h[1];
    c->parity = (int)h[2];
    return LBM_OK;
}

lbm_status lbm_steps_done(lbm_ctx* c, int64_t* steps) {
    if (!c || !steps) return fail(LBM_E_INVAL, "bad arguments");
    *steps = c->steps;
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_ctx* c, int32_t block, int32_t flags) {
    if (!c || c->batch) return fail(LBM_E_INVAL, "launch shape applies to single-domain contexts");
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return fail(LBM_E_INVAL, "block must be 64, 128, 256, 512 or 1024");
    if (flags & ~(LBM_LAUNCH_XCD_REMAP | LBM_LAUNCH_NONTEMPORAL | LBM_LAUNCH_CELLS_2 | LBM_LAUNCH_CELLS_4))
        return fail(LBM_E_INVAL, "unknown launch flags");
    if ((flags & LBM_LAUNCH_CELLS_2) && (flags & LBM_LAUNCH_CELLS_4))
        return fail(LBM_E_INVAL, "LBM_LAUNCH_CELLS_2 and LBM_LAUNCH_CELLS_4 exclude each other");
    if ((flags & (LBM_LAUNCH_CELLS_2 | LBM_LAUNCH_CELLS_4)) && c->p.layout != LBM_LAYOUT_BRICK)
        return fail(LBM_E_INVAL, "more than one cell per thread needs the brick layout");
    c->block = block;
    set_flags(c, flags);
    return LBM_OK;
}

lbm_status lbm_get_launch(lbm_ctx* c, int32_t* block, int32_t* flags) {
    if (!c || c->batch) return fail(LBM_E_INVAL, "launch shape applies to single-domain contexts");
    if (block) *block = c->block;
    if (flags) *flags = get_flags(c);
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t steps_per_trial) {
    if (!c || steps_per_trial < 2) return fail(LBM_E_INVAL, "bad arguments");
    if (c->batch) return batch_autotune(c->batch, steps_per_trial);
    // the trials advance the state: keep a host copy unless it is the rest state
    const bool at_rest = c->steps == 0;
    int64_t sb = 0;
    std::vector<char> saved;
    lbm_status s = LBM_OK;
    if (!at_rest) {
        s = lbm_state_bytes(c, &sb);
        if (s != LBM_OK) return s;
        try {
            saved.resize((size_t)sb);
        } catch (const std::bad_alloc&) {
            return fail(LBM_E_NOMEM, "host memory for the autotuner's state copy");
        }
        s = lbm_save(c, saved.data(), sb);
        if (s != LBM_OK) return s;
    }
    const int blocks[] = {64, 128, 256, 512, 1024};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    float best = 1e30f;
    int bb = c->block, bf = get_flags(c);
    auto trial = [&](int blk, int fl) {
        c->block = blk;
        set_flags(c, fl);
        s = step_single(c, 2);  // warm-up (even + odd for AA)
        if (s != LBM_OK) return;
        hipEventRecord(e0, c->stream);
        s = step_single(c, steps_per_trial);
        if (s != LBM_OK) return;
        hipEventRecord(e1, c->stream);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; bb = blk; bf = fl; }
    };
    // workgroup size, XCD remap and hints at one cell per thread, then (brick
    // layout) two and four cells per thread at the best of those
    for (int blk : blocks)
        for (int fl = 0; fl < 4 && s == LBM_OK; ++fl) trial(blk, fl);
    const int b1 = bb, f1 = bf;
    if (c->p.layout == LBM_LAYOUT_BRICK)
        for (int cells : {LBM_LAUNCH_CELLS_2, LBM_LAUNCH_CELLS_4})
            if (s == LBM_OK) trial(b1, f1 | cells);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->block = bb;
    set_flags(c, bf);
    lbm_status s2 = LBM_OK;
    if (at_rest) {
        hipError_t e = reset_state(c);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) s2 = hip_fail(e, "reset after autotuning");
    } else {
        s2 = lbm_load(c, saved.data(), sb);
    }
    if (s != LBM_OK) return s;
    if (s2 != LBM_OK) return s2;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[{c->arch, c->d.nx, c->d.ny, c->d.nz, c->p.layout, c->d.bc}] = {bb, bf};
    return LBM_OK;
}

}  // extern "C"

namespace {

// candidate layouts of a geometry: single domain two-grid, AA and (when the
// brick dimensions allow it) brick; batches AA (persistent launch) and brick
std::vector<int> layout_candidates(const lbm_geometry* g) {
    bool bricks = true;
    for (const auto& D : g->doms) bricks = bricks && brick_dims_ok(D.desc);
    std::vector<int> c;
    if (g->doms.size() == 1) c.push_back(LBM_LAYOUT_TWOGRID);
    c.push_back(LBM_LAYOUT_AA);
    if (bricks) c.push_back(LBM_LAYOUT_BRICK);
    return c;
}

LayoutKey layout_key(const lbm_geometry* g, const lbm_params* p, const std::string& arch) {
    int64_t cells = 0;
    for (const auto& D : g->doms) cells += D.ncells();
    const auto& d = g->doms[0].desc;
    return {arch, (int)g->doms.size(), d.nx, d.ny, d.nz, d.bc, p->collision, cells};
}

}  // namespace

namespace {

// "sweep ARCH NX NY NZ LAYOUT BC BLOCK FLAGS" and
// "layout ARCH DOMAINS NX NY NZ BC COLLISION CELLS LAYOUT MS_PER_STEP"
void single_tuning_export(std::string& out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune_cache) {
        const TuneKey& k = kv.first;
        out += "sweep " + k.arch + " " + std::to_string(k.nx) + " " + std::to_string(k.ny) + " " + std::to_string(k.nz) +
               " " + std::to_string(k.layout) + " " + std::to_string(k.bc) + " " + std::to_string(kv.second.first) + " " +
               std::to_string(kv.second.second) + "\n";
    }
    for (const auto& kv : g_layout_cache) {
        const LayoutKey& k = kv.first;
        char ms[32];
        std::snprintf(ms, sizeof ms, "%.17g", kv.second.second);
        out += "layout " + k.arch + " " + std::to_string(k.ndom) + " " + std::to_string(k.nx) + " " +
               std::to_string(k.ny) + " " + std::to_string(k.nz) + " " + std::to_string(k.bc) + " " +
               std::to_string(k.collision) + " " + std::to_string(k.cells) + " " + std::to_string(kv.second.first) +
               " " + ms + "\n";
    }
}

int single_tuning_import(const std::vector<std::string>& f, bool apply) {
    if (f.empty()) return 0;
    if (f[0] == "sweep") {
        int64_t v[7];
        if (f.size() != 9 || f[1].empty()) return -1;
        for (int i = 0; i < 7; ++i)
            if (!parse_i64(f[2 + i], v[i])) return -1;
        const int64_t nx = v[0], ny = v[1], nz = v[2], layout = v[3], bc = v[4], block = v[5], flags = v[6];
        const bool ok_block = block == 64 || block == 128 || block == 256 || block == 512 || block == 1024;
        const int64_t cells = LBM_LAUNCH_CELLS_2 | LBM_LAUNCH_CELLS_4;
        if (nx < 1 || ny < 1 || nz < 1 || layout < 0 || layout > 2 || bc < 0 || bc > 2 || !ok_block ||
            (flags & ~(LBM_LAUNCH_XCD_REMAP | LBM_LAUNCH_NONTEMPORAL | cells)) || (flags & cells) == cells ||
            ((flags & cells) && layout != LBM_LAYOUT_BRICK))
            return -1;
        if (apply) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[{f[1], (int)nx, (int)ny, (int)nz, (int)layout, (int)bc}] = {(int)block, (int)flags};
        }
        return 1;
    }
    if (f[0] == "layout") {
        int64_t v[8];
        double ms = 0.0;
        if (f.size() != 11 || f[1].empty()) return -1;
        for (int i = 0; i < 8; ++i)
            if (!parse_i64(f[2 + i], v[i])) return -1;
        if (!parse_f64(f[10], ms)) return -1;
        const int64_t nd = v[0], nx = v[1], ny = v[2], nz = v[3], bc = v[4], coll = v[5], cells = v[6], layout = v[7];
        if (nd < 1 || nx < 1 || ny < 1 || nz < 1 || bc < 0 || bc > 2 || coll < 0 || coll > 1 || cells < 1 ||
            layout < 0 || layout > 2 || ms < 0.0)
            return -1;
        if (apply) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_layout_cache[{f[1], (int)nd, (int)nx, (int)ny, (int)nz, (int)bc, (int)coll, cells}] = {(int)layout, ms};
        }
        return 1;
    }
    return 0;
}

}  // namespace

extern "C" {

lbm_status lbm_tuning_export(char* buf, int64_t capacity, int64_t* length) {
    if (!length || capacity < 0 || (capacity > 0 && !buf)) return fail(LBM_E_INVAL, "bad arguments");
    std::string out = "# mi355lbm tuning cache v1\n";
    single_tuning_export(out);
    bbatch_tuning_export(out);
    abatch_tuning_export(out);
    *length = (int64_t)out.size();
    if (buf && capacity > (int64_t)out.size()) std::memcpy(buf, out.c_str(), out.size() + 1);
    return LBM_OK;
}

lbm_status lbm_tuning_import(const char* text) {
    if (!text) return fail(LBM_E_INVAL, "bad arguments");
    std::vector<std::vector<std::string>> lines;
    {
        std::string cur;
        std::vector<std::string> f;
        for (const char* q = text;; ++q) {
            const char ch = *q;
            if (ch == ' ' || ch == '\t' || ch == '\n' || ch == '\r' || ch == '\0') {
                if (!cur.empty()) f.push_back(cur);
                cur.clear();
                if (ch == '\n' || ch == '\0') {
                    lines.push_back(f);
                    f.clear();
                }
                if (ch == '\0') break;
            } else {
                cur += ch;
            }
        }
    }
    // check every line first, so that a malformed text changes nothing
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t i = 0; i < lines.size(); ++i) {
            const auto& f = lines[i];
            if (f.empty() || f[0][0] == '#') continue;
            const bool apply = pass == 1;
            int r = single_tuning_import(f, apply);
            if (r == 0) r = bbatch_tuning_import(f, apply);
            if (r == 0) r = abatch_tuning_import(f, apply);
            if (r != 1) return fail(LBM_E_INVAL, "tuning text, line " + std::to_string(i + 1) + ": " +
                                                     (r == 0 ? "unknown entry kind" : "malformed entry"));
        }
    }
    return LBM_OK;
}

}  // extern "C"

extern "C" {

lbm_status lbm_autotune_layout_bytes(const lbm_geometry* g, const lbm_params* p, int64_t* bytes) {
    if (!g || !p || !bytes || g->doms.empty()) return fail(LBM_E_INVAL, "bad arguments");
    int64_t most = 0;
    int ok = 0;
    for (int lay : layout_candidates(g)) {
        lbm_params q = *p;
        q.layout = lay;
        int64_t b = 0;
        if (lbm_required_bytes(g, &q, &b) != LBM_OK) continue;
        most = std::max(most, b);
        ++ok;
    }
    if (!ok) return fail(LBM_E_INVAL, "no layout can hold this geometry");
    *bytes = most;
    return LBM_OK;
}

lbm_status lbm_autotune_layout(const lbm_geometry* g, const lbm_params* p, void* dev_buf, int64_t bytes,
                               void* hip_stream, int32_t steps_per_trial, int32_t* layout, double* ms_per_step) {
    if (!g || !p || !layout || g->doms.empty() || steps_per_trial < 2) return fail(LBM_E_INVAL, "bad arguments");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "no HIP device");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "device properties");
    const LayoutKey key = layout_key(g, p, prop.gcnArchName);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_layout_cache.find(key);
        if (it != g_layout_cache.end()) {
            *layout = it->second.first;
            if (ms_per_step) *ms_per_step = it->second.second;
            return LBM_OK;
        }
    }
    if (!dev_buf) return fail(LBM_E_INVAL, "no device buffer (and no cached choice)");
    int64_t need = 0;
    lbm_status s = lbm_autotune_layout_bytes(g, p, &need);
    if (s != LBM_OK) return s;
    if (bytes < need) return fail(LBM_E_NOMEM, "device buffer smaller than lbm_autotune_layout_bytes");
    const int64_t nsteps = steps_per_trial + (steps_per_trial & 1);  // even: whole AA step pairs
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(LBM_E_DEVICE, "event");
    }
    int best = -1;
    double best_ms = 0.0;
    for (int lay : layout_candidates(g)) {
        lbm_params q = *p;
        q.layout = lay;
        int64_t b = 0;
        if (lbm_required_bytes(g, &q, &b) != LBM_OK) continue;  // e.g. beyond a layout's limits
        lbm_ctx* c = nullptr;
        s = lbm_init(g, &q, dev_buf, bytes, hip_stream, &c);
        if (s == LBM_OK) s = lbm_autotune(c, (int32_t)nsteps);
        if (s == LBM_OK) s = lbm_step(c, 2);
        float ms = 0.0f;
        if (s == LBM_OK) {
            hipEventRecord(e0, st);
            s = lbm_step(c, nsteps);
            hipEventRecord(e1, st);
            if (s == LBM_OK && hipEventSynchronize(e1) != hipSuccess) s = fail(LBM_E_DEVICE, "timing event");
            if (s == LBM_OK) hipEventElapsedTime(&ms, e0, e1);
        }
        if (c) lbm_destroy(c);
        if (s != LBM_OK) break;
        const double per = (double)ms / (double)nsteps;
        if (best < 0 || per < best_ms) {
            best = lay;
            best_ms = per;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s != LBM_OK) return s;
    if (best < 0) return fail(LBM_E_INVAL, "no layout can hold this geometry");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_layout_cache[key] = {best, best_ms};
    }
    *layout = best;
    if (ms_per_step) *ms_per_step = best_ms;
    return LBM_OK;
}

lbm_status lbm_batch_set_launch(lbm_ctx* c, int32_t block, int32_t workgroups_per_domain) {
    if (!c || !c->batch) return fail(LBM_E_INVAL, "not a batched context");
    return batch_set_launch(c->batch, block, workgroups_per_domain);
}

lbm_status lbm_batch_get_launch(lbm_ctx* c, int32_t* block, int32_t* workgroups_per_domain) {
    if (!c || !c->batch) return fail(LBM_E_INVAL, "not a batched context");
    return batch_get_launch(c->batch, block, workgroups_per_domain);
}

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    if (c->batch) batch_destroy(c->batch);
    delete c;
}

}  // extern "C"
