// Batched pore-scale runs in the brick layout.
//
// Every domain of the batch is cut into 4x4x4 bricks and its bricks that
// hold fluid are stored in ONE brick array shared by all domains (each
// domain's range padded to a multiple of 8 bricks, so that the 512-cell link
// segments never straddle two domains).  A brick's neighbour table wraps
// inside its own domain, so the brick sweep of the single-domain path
// (sweep.hip) steps the whole batch in one ordinary launch per time step,
// over a list of the bricks of the domains still running.  Two grids; a
// domain's state is in grid (steps & 1), and domains of both parities are
// stepped by two launches over two lists.
//
// Steady-state test (as for the persistent AA batch): every check_every
// steps of a call, the check step's launch stores each brick's FP64 sum of
// u_x (fixed butterfly over its wavefront), a second kernel sums each
// domain's bricks in index order, and a domain whose sum changed by at most
// tol of itself since its previous check stops; its status and last sum
// persist between calls.  Every cell's arithmetic is that of the
// single-domain sweep, so each domain's fields equal a single-domain run bit
// for bit, for every launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "tuning.hpp"

namespace lbm {

namespace {

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Dom {
    lbm_domain_desc desc{};
    int64_t N = 0;                    // dense cells
    int32_t first = 0, nbricks = 0;   // first stored brick of the domain, its stored bricks
    int64_t link0 = 0, nl = 0;        // first link of the domain, its links
    int64_t bmap_off = 0, nbmap = 0;  // its dense brick map in the shared map
};

struct TuneKey {
    std::string arch;
    int ndom;
    int64_t bricks;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, ndom, bricks) < std::tie(o.arch, o.ndom, o.bricks);
    }
};
std::mutex g_mu;
std::map<TuneKey, std::pair<int, int>> g_cache;  // block, nt | W << 1

#define HIPCHK(expr, what)                                                                                  \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) return set_error(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct BrickBatch {
    int ndom = 0;
    lbm_params p{};
    CellConsts k{};
    int bc = 0;
    hipStream_t stream = nullptr;
    char* buf = nullptr;
    int64_t bytes = 0;
    std::vector<Dom> doms;
    int64_t nb = 0, NS = 0, stride = 0, nl = 0, grid = 0, nseed = 0, max_np = 0, chunk = 0, nbmap = 0;
    int64_t off_pop = 0, off_info = 0, off_segbase = 0, off_lparam = 0, off_nbr = 0, off_bmap = 0, off_partial = 0,
            off_list = 0, off_first = 0, off_count = 0, off_dlist = 0, off_usum = 0, off_seed = 0, off_red = 0,
            off_fields = 0;
    std::vector<int64_t> steps;
    std::vector<int32_t> status;
    std::vector<double> uprev;
    int block = 1024, nt = 1, W = 1;  // W: cells per thread of the brick sweep (1, 2 or 4)
    std::string arch;
};

namespace {

lbm_status plan(const std::vector<DomainGeo>& G, const lbm_params& p, BrickBatch& b) {
    if (p.force[1] != 0.0 || p.force[2] != 0.0)
        return set_error(LBM_E_INVAL, "batched runs drive the flow along x (force[1] = force[2] = 0)");
    const auto& d0 = G[0].desc;
    b.doms.clear();
    int64_t nb = 0, nl = 0, nbmap = 0, nseed = 0;
    for (const auto& g : G) {
        const auto& d = g.desc;
        if (d.bc != d0.bc) return set_error(LBM_E_INVAL, "all domains of a batch must use the same boundary scheme");
        for (int a = 0; a < 3; ++a)
            if (d.wall_hi_velocity[a] != d0.wall_hi_velocity[a])
                return set_error(LBM_E_INVAL, "all domains of a batch must share the wall velocity");
        if (!brick_dims_ok(d)) return set_error(LBM_E_INVAL, "brick layout needs nx, ny, nz divisible by 4 in every domain");
        BrickMap bm;
        build_brick_map(g, bm, false);
        Dom D;
        D.desc = d;
        D.desc.spheres = nullptr;
        D.desc.n_spheres = 0;
        D.N = g.ncells();
        D.first = (int32_t)nb;
        D.nbricks = (int32_t)bm.nstored;
        D.link0 = nl;
        D.nl = (int64_t)g.lcell.size();
        D.bmap_off = nbmap;
        D.nbmap = (int64_t)bm.bx * bm.by * bm.bz;
        nb += align_up(bm.nstored, 8);
        nl += D.nl;
        nbmap += D.nbmap;
        const bool moving = d.wall_hi_velocity[0] != 0.0 || d.wall_hi_velocity[1] != 0.0 || d.wall_hi_velocity[2] != 0.0;
        if (moving)
            for (auto s : g.lsurf)
                if (s == SURF_WALL_HI) ++nseed;
        b.max_np = std::max<int64_t>(b.max_np, std::max(d.nx, std::max(d.ny, d.nz)));
        b.chunk = std::max<int64_t>(b.chunk, std::min<int64_t>(D.N, std::max<int64_t>((int64_t)d.nx * d.ny, 1 << 20)));
        b.doms.push_back(D);
    }
    b.nb = nb;
    b.NS = nb * 64;
    if (b.NS >= ((int64_t)1 << 30))
        return set_error(LBM_E_INVAL, "a brick-layout batch must store fewer than 2^30 cells");
    if (nl > max_links()) return set_error(LBM_E_INVAL, "too many boundary links in one batch (limit 2^30 - 19)");
    b.nl = nl;
    b.nbmap = nbmap;
    b.nseed = nseed;
    b.stride = align_up(b.NS, 256) + 320;
    b.grid = Q * b.stride + align_up(nl + Q, 64);
    const int64_t nd = (int64_t)G.size();
    int64_t o = 0;
    b.off_pop = o; o = align_up(o + 2 * b.grid * 4, 256);
    b.off_info = o; o = align_up(o + b.NS * 4, 256);
    b.off_segbase = o; o = align_up(o + ((b.NS >> SEG_SHIFT) + 1) * 4, 256);
    b.off_lparam = o; o = align_up(o + (nl + Q) * 4, 256);
    b.off_nbr = o; o = align_up(o + nb * 27 * 4, 256);
    b.off_bmap = o; o = align_up(o + std::max<int64_t>(nbmap, 1) * 4, 256);
    b.off_partial = o; o = align_up(o + std::max<int64_t>(nb, 1) * 8, 256);
    b.off_list = o; o = align_up(o + 2 * std::max<int64_t>(nb, 1) * 4, 256);  // two lists (parities)
    b.off_first = o; o = align_up(o + nd * 4, 256);
    b.off_count = o; o = align_up(o + nd * 4, 256);
    b.off_dlist = o; o = align_up(o + nd * 4, 256);
    b.off_usum = o; o = align_up(o + nd * 8, 256);
    b.off_seed = o; o = align_up(o + std::max<int64_t>(nseed, 1) * 12, 256);
    b.off_red = o; o = align_up(o + b.max_np * 6 * 8, 256);
    b.off_fields = o; o = align_up(o + b.chunk * 4 * 8, 256);
    b.bytes = o;
    b.ndom = (int)nd;
    b.bc = d0.bc;
    return LBM_OK;
}

float* grid_base(BrickBatch* b, int g) { return reinterpret_cast<float*>(b->buf + b->off_pop) + g * b->grid; }

lbm_status reset(BrickBatch* b) {
    HIPCHK(launch_fill_zero(grid_base(b, 0), 2 * b->grid, b->stream), "zero populations");
    if (b->nseed > 0)
        HIPCHK(launch_scatter(grid_base(b, 0), reinterpret_cast<const int64_t*>(b->buf + b->off_seed),
                              reinterpret_cast<const float*>(b->buf + b->off_seed + b->nseed * 8), b->nseed,
                              b->stream),
               "seed moving walls");
    b->steps.assign(b->ndom, 0);
    b->status.assign(b->ndom, 0);
    b->uprev.assign(b->ndom, NAN);
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

// device lists of the bricks of the given domains, by parity of their step
// count: list p holds the domains whose state is in grid p
struct Lists {
    int64_t n[2] = {0, 0};
};

lbm_status upload_lists(BrickBatch* b, const std::vector<int>& ds, Lists& L) {
    std::vector<int32_t> h[2];
    for (int d : ds) {
        const Dom& D = b->doms[d];
        auto& v = h[b->steps[d] & 1];
        for (int32_t i = 0; i < D.nbricks; ++i) v.push_back(D.first + i);
    }
    int32_t* dev = reinterpret_cast<int32_t*>(b->buf + b->off_list);
    for (int q = 0; q < 2; ++q) {
        L.n[q] = (int64_t)h[q].size();
        if (!h[q].empty())
            HIPCHK(hipMemcpyAsync(dev + q * std::max<int64_t>(b->nb, 1), h[q].data(), h[q].size() * 4,
                                  hipMemcpyHostToDevice, b->stream),
                   "brick list");
    }
    // the host vectors go out of scope: the copies must have completed
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

// one time step of the listed bricks; `shift` = number of steps already run
// in this call (the domains of list q are at parity q ^ (shift & 1))
lbm_status sweep_step(BrickBatch* b, const Lists& L, int64_t shift, bool check) {
    for (int q = 0; q < 2; ++q) {
        if (L.n[q] == 0) continue;
        const int cur = (int)((q + shift) & 1);
        SweepArgs a{};
        a.A = grid_base(b, cur);
        a.B = grid_base(b, 1 - cur);
        a.stride = b->stride;
        for (int k = 0; k < Q; ++k) {
            a.pa[k] = a.A + k * b->stride;
            a.pb[k] = a.B + k * b->stride;
        }
        a.pva = a.A + Q * b->stride;
        a.pvb = a.B + Q * b->stride;
        a.info = reinterpret_cast<const uint32_t*>(b->buf + b->off_info);
        a.segbase = reinterpret_cast<const int32_t*>(b->buf + b->off_segbase);
        a.lparam = reinterpret_cast<const float*>(b->buf + b->off_lparam);
        a.nbr = reinterpret_cast<const int32_t*>(b->buf + b->off_nbr);
        a.list = reinterpret_cast<const int32_t*>(b->buf + b->off_list) + q * std::max<int64_t>(b->nb, 1);
        a.nbricks = (int32_t)L.n[q];
        a.partial = reinterpret_cast<double*>(b->buf + b->off_partial);
        a.k = b->k;
        a.xcd_remap = 0;
        a.nt = b->nt;
        a.cpt = b->W;
        HIPCHK(launch_sweep_bricks(a, b->bc, b->block, check, b->stream), "brick batch sweep");
    }
    return LBM_OK;
}

MomentArgs dom_moments(BrickBatch* b, int d) {
    const Dom& D = b->doms[d];
    MomentArgs m{};
    m.A = grid_base(b, (int)(b->steps[d] & 1));
    m.stride = b->stride;
    m.info = reinterpret_cast<const uint32_t*>(b->buf + b->off_info);
    m.bmap = reinterpret_cast<const int32_t*>(b->buf + b->off_bmap) + D.bmap_off;
    m.nx = D.desc.nx; m.ny = D.desc.ny; m.nz = D.desc.nz;
    m.layout = L_BRICK;
    m.parity = -1;
    m.rho0 = b->p.rho0;
    for (int a = 0; a < 3; ++a) m.F[a] = b->p.force[a];
    return m;
}

lbm_status dom_plane_sums(BrickBatch* b, int d, int axis, std::vector<double>& out) {
    const auto& D = b->doms[d].desc;
    const int np = axis == 0 ? D.nx : (axis == 1 ? D.ny : D.nz);
    double* red = reinterpret_cast<double*>(b->buf + b->off_red);
    HIPCHK(launch_plane_sums(dom_moments(b, d), axis, red, b->stream), "plane reduction");
    out.assign((size_t)np * 6, 0.0);
    HIPCHK(hipMemcpyAsync(out.data(), red, out.size() * 8, hipMemcpyDeviceToHost, b->stream), "copy plane sums");
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

const int64_t kMagic = 0x4c424d4252494b53;  // "LBMBRIKS"

}  // namespace

lbm_status bbatch_required_bytes(const std::vector<DomainGeo>& doms, const lbm_params& p, int64_t* bytes) {
    BrickBatch b;
    lbm_status s = plan(doms, p, b);
    if (s != LBM_OK) return s;
    *bytes = b.bytes;
    return LBM_OK;
}

lbm_status bbatch_init(const std::vector<DomainGeo>& doms, const lbm_params& p, double wp, double wm, char* buf,
                       int64_t bytes, hipStream_t s, BrickBatch** out) {
    auto* b = new BrickBatch;
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
    b->arch = prop.gcnArchName;
    // global images: every domain's records moved to its brick and link ranges
    std::vector<uint32_t> info;
    std::vector<int32_t> segbase, nbr, bmap, first(b->ndom), count(b->ndom);
    std::vector<float> lparam;
    std::vector<int64_t> seed_idx;
    std::vector<float> seed_val;
    try {
        info.assign((size_t)b->NS, CELL_SOLID_WORD);
        segbase.assign((size_t)((b->NS >> SEG_SHIFT) + 1), (int32_t)b->nl);
        lparam.assign((size_t)(b->nl + Q), 0.0f);
        nbr.resize((size_t)(b->nb * 27));
        for (int64_t i = 0; i < b->nb; ++i)
            for (int j = 0; j < 27; ++j) nbr[(size_t)(i * 27 + j)] = (int32_t)i;  // padding bricks: themselves
        bmap.assign((size_t)std::max<int64_t>(b->nbmap, 1), -1);
        for (int d = 0; d < b->ndom; ++d) {
            const Dom& D = b->doms[d];
            BrickMap bm;
            build_brick_map(doms[d], bm, true);
            DeviceImages im;
            std::string err;
            st = build_images(doms[d], LBM_LAYOUT_BRICK, bm, b->stride, b->k, im, err);
            if (st != LBM_OK) { delete b; return set_error(st, "domain " + std::to_string(d) + ": " + err); }
            const int64_t c0 = (int64_t)D.first * 64;
            std::copy(im.info.begin(), im.info.end(), info.begin() + c0);
            const int64_t nseg = ((int64_t)D.nbricks * 64 + 511) / 512;  // segments the domain covers
            for (int64_t g = 0; g < nseg; ++g) segbase[(size_t)(c0 / 512 + g)] = (int32_t)(D.link0 + im.segbase[g]);
            std::copy(im.lparam.begin(), im.lparam.begin() + D.nl, lparam.begin() + D.link0);
            for (int64_t i = 0; i < (int64_t)bm.nbr.size(); ++i) nbr[(size_t)(c0 / 64 * 27 + i)] = D.first + bm.nbr[i];
            for (int64_t i = 0; i < D.nbmap; ++i)
                bmap[(size_t)(D.bmap_off + i)] = bm.id[i] < 0 ? -1 : D.first + bm.id[i];
            for (size_t i = 0; i < im.seed_idx.size(); ++i) {
                seed_idx.push_back(im.seed_idx[i] + D.link0);  // Q * stride + global link
                seed_val.push_back(im.seed_val[i]);
            }
            first[d] = D.first;
            count[d] = D.nbricks;
        }
    } catch (const std::bad_alloc&) {
        delete b;
        return set_error(LBM_E_NOMEM, "host memory for the batch images");
    }
    if ((int64_t)seed_idx.size() != b->nseed) { delete b; return set_error(LBM_E_INVAL, "internal: seed count"); }
    hipError_t e = hipSuccess;
    auto up = [&](int64_t off, const void* src, size_t n) {
        if (e == hipSuccess && n > 0) e = hipMemcpyAsync(buf + off, src, n, hipMemcpyHostToDevice, s);
    };
    up(b->off_info, info.data(), info.size() * 4);
    up(b->off_segbase, segbase.data(), segbase.size() * 4);
    up(b->off_lparam, lparam.data(), lparam.size() * 4);
    up(b->off_nbr, nbr.data(), nbr.size() * 4);
    up(b->off_bmap, bmap.data(), bmap.size() * 4);
    up(b->off_first, first.data(), first.size() * 4);
    up(b->off_count, count.data(), count.size() * 4);
    up(b->off_seed, seed_idx.data(), seed_idx.size() * 8);
    up(b->off_seed + b->nseed * 8, seed_val.data(), seed_val.size() * 4);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host images go out of scope
    if (e != hipSuccess) {
        delete b;
        return set_error(LBM_E_DEVICE, std::string("brick batch upload: ") + hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find({b->arch, b->ndom, b->nb});
        if (it != g_cache.end()) {
            b->block = it->second.first;
            b->nt = it->second.second & 1;
            b->W = it->second.second >> 1;
        }
    }
    st = reset(b);
    if (st != LBM_OK) { delete b; return st; }
    *out = b;
    return LBM_OK;
}

lbm_status bbatch_step(BrickBatch* b, int64_t n) {
    if (n <= 0) return LBM_OK;
    std::vector<int> all(b->ndom);
    for (int d = 0; d < b->ndom; ++d) all[d] = d;
    Lists L;
    lbm_status s = upload_lists(b, all, L);
    if (s != LBM_OK) return s;
    for (int64_t i = 0; i < n; ++i) {
        s = sweep_step(b, L, i, false);
        if (s != LBM_OK) return s;
    }
    for (auto& v : b->steps) v += n;
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

lbm_status bbatch_run_to_steady(BrickBatch* b, double tol, int64_t check_every, int64_t max_steps,
                                int64_t* steps_done) {
    std::vector<int> active;
    for (int d = 0; d < b->ndom; ++d)
        if (b->status[d] == 0) active.push_back(d);
    int64_t it = 0;
    std::vector<double> usum(b->ndom);
    Lists L;
    bool stale = true;   // the device lists no longer match `active`
    int64_t since = 0;   // steps run since the lists were uploaded
    while (it < max_steps && !active.empty()) {
        lbm_status s = LBM_OK;
        if (stale) {
            s = upload_lists(b, active, L);
            if (s != LBM_OK) return s;
            stale = false;
            since = 0;
        }
        const int64_t n = std::min(check_every - it % check_every, max_steps - it);
        const bool check = (it + n) % check_every == 0;
        for (int64_t j = 0; j < n; ++j) {
            s = sweep_step(b, L, since + j, check && j == n - 1);
            if (s != LBM_OK) return s;
        }
        since += n;
        it += n;
        for (int d : active) b->steps[d] += n;
        if (check) {
            HIPCHK(hipMemcpyAsync(b->buf + b->off_dlist, active.data(), active.size() * 4, hipMemcpyHostToDevice,
                                  b->stream),
                   "domain list");
            HIPCHK(launch_domain_sums(reinterpret_cast<const double*>(b->buf + b->off_partial),
                                      reinterpret_cast<const int32_t*>(b->buf + b->off_first),
                                      reinterpret_cast<const int32_t*>(b->buf + b->off_count),
                                      reinterpret_cast<const int32_t*>(b->buf + b->off_dlist), (int)active.size(),
                                      reinterpret_cast<double*>(b->buf + b->off_usum), b->stream),
                   "domain sums");
            HIPCHK(hipMemcpyAsync(usum.data(), b->buf + b->off_usum, b->ndom * 8, hipMemcpyDeviceToHost, b->stream),
                   "copy domain sums");
            HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
            std::vector<int> still;
            for (int d : active) {
                const double U = usum[d], Up = b->uprev[d];
                int st = 0;
                if (!(std::fabs(U) < 0.4 * (double)b->doms[d].N)) st = -1;  // NaN or runaway velocity
                else if (std::fabs(U - Up) <= tol * std::fabs(U)) st = 1;
                b->uprev[d] = U;
                b->status[d] = st;
                if (st == 0) still.push_back(d);
            }
            if (still.size() != active.size()) stale = true;
            active.swap(still);
        }
    }
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    for (int d = 0; d < b->ndom; ++d) steps_done[d] = b->steps[d];
    for (int d = 0; d < b->ndom; ++d)
        if (b->status[d] < 0) return set_error(LBM_E_UNSTABLE, "domain " + std::to_string(d) + " became unstable");
    return LBM_OK;
}

lbm_status bbatch_profile(BrickBatch* b, int dom, int axis, int comp, double* u_sup, double* u_int, double* por) {
    std::vector<double> ps;
    lbm_status s = dom_plane_sums(b, dom, axis, ps);
    if (s != LBM_OK) return s;
    const auto& D = b->doms[dom].desc;
    const int np = axis == 0 ? D.nx : (axis == 1 ? D.ny : D.nz);
    const double area = (double)b->doms[dom].N / np;
    for (int i = 0; i < np; ++i) {
        const double sum = ps[i * 6 + 1 + comp], nf = ps[i * 6 + 4];
        if (u_sup) u_sup[i] = sum / area;
        if (u_int) u_int[i] = nf > 0 ? sum / nf : 0.0;
        if (por) por[i] = nf / area;
    }
    return LBM_OK;
}

lbm_status bbatch_permeability(BrickBatch* b, int dom, int fa, int z0, int z1, double* k) {
    const auto& D = b->doms[dom].desc;
    if (z0 < 0 || z1 > D.nz || z0 >= z1) return set_error(LBM_E_INVAL, "bad plane range");
    if (b->p.force[fa] == 0.0) return set_error(LBM_E_INVAL, "no body force along the flow axis");
    std::vector<double> sup((size_t)D.nz);
    lbm_status s = bbatch_profile(b, dom, 2, fa, sup.data(), nullptr, nullptr);
    if (s != LBM_OK) return s;
    double m = 0;
    for (int z = z0; z < z1; ++z) m += sup[z];
    m /= (z1 - z0);
    *k = b->p.rho0 * ((b->p.tau_plus - 0.5) / 3.0) * m / b->p.force[fa];
    return LBM_OK;
}

lbm_status bbatch_fields(BrickBatch* b, int dom, double* rho, double* u) {
    const int64_t N = b->doms[dom].N, chunk = b->chunk;
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

lbm_status bbatch_totals(BrickBatch* b, int dom, double* mass, double* mom) {
    std::vector<double> ps;
    lbm_status s = dom_plane_sums(b, dom, 2, ps);
    if (s != LBM_OK) return s;
    double m = 0, j[3] = {0, 0, 0}, bad = 0;
    for (int z = 0; z < b->doms[dom].desc.nz; ++z) {
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

// image: 4 int64 header {magic, steps of the context, ndom, 0}, then per
// domain {steps, status, last sum} and its Q population ranges and its
// partial bounce-back values, from the grid that holds its state
lbm_status bbatch_state_bytes(BrickBatch* b, int64_t* bytes) {
    int64_t n = 32;
    for (auto& D : b->doms) n += 24 + ((int64_t)Q * D.nbricks * 64 + D.nl) * 4;
    *bytes = n;
    return LBM_OK;
}

lbm_status bbatch_save(BrickBatch* b, void* host, int64_t bytes, int64_t steps) {
    (void)bytes;
    int64_t* h = reinterpret_cast<int64_t*>(host);
    h[0] = kMagic; h[1] = steps; h[2] = b->ndom; h[3] = 0;
    char* o = reinterpret_cast<char*>(host) + 32;
    for (int d = 0; d < b->ndom; ++d) {
        const Dom& D = b->doms[d];
        int64_t meta[3] = {b->steps[d], b->status[d], 0};
        std::memcpy(&meta[2], &b->uprev[d], 8);
        std::memcpy(o, meta, 24);
        o += 24;
        const float* g = grid_base(b, (int)(b->steps[d] & 1));
        const int64_t nc = (int64_t)D.nbricks * 64;
        for (int k = 0; k < Q; ++k) {
            HIPCHK(hipMemcpyAsync(o, g + k * b->stride + (int64_t)D.first * 64, nc * 4, hipMemcpyDeviceToHost,
                                  b->stream),
                   "save");
            o += nc * 4;
        }
        HIPCHK(hipMemcpyAsync(o, g + Q * b->stride + D.link0, D.nl * 4, hipMemcpyDeviceToHost, b->stream), "save");
        o += D.nl * 4;
    }
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

lbm_status bbatch_load(BrickBatch* b, const void* host, int64_t bytes) {
    (void)bytes;
    const int64_t* h = reinterpret_cast<const int64_t*>(host);
    if (h[0] != kMagic || h[2] != b->ndom) return set_error(LBM_E_INVAL, "not a state image of this batch");
    const char* o = reinterpret_cast<const char*>(host) + 32;
    for (int d = 0; d < b->ndom; ++d) {
        const Dom& D = b->doms[d];
        int64_t meta[3];
        std::memcpy(meta, o, 24);
        o += 24;
        b->steps[d] = meta[0];
        b->status[d] = (int32_t)meta[1];
        std::memcpy(&b->uprev[d], &meta[2], 8);
        float* g = grid_base(b, (int)(b->steps[d] & 1));
        const int64_t nc = (int64_t)D.nbricks * 64;
        for (int k = 0; k < Q; ++k) {
            HIPCHK(hipMemcpyAsync(g + k * b->stride + (int64_t)D.first * 64, o, nc * 4, hipMemcpyHostToDevice,
                                  b->stream),
                   "load");
            o += nc * 4;
        }
        HIPCHK(hipMemcpyAsync(g + Q * b->stride + D.link0, o, D.nl * 4, hipMemcpyHostToDevice, b->stream), "load");
        o += D.nl * 4;
    }
    HIPCHK(hipStreamSynchronize(b->stream), "synchronise");
    return LBM_OK;
}

lbm_status bbatch_autotune(BrickBatch* b, int32_t steps_per_trial) {
    for (int d = 0; d < b->ndom; ++d)
        if (b->steps[d] != 0) return set_error(LBM_E_STATE, "autotune a batch before stepping it");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "event");
    HIPCHK(hipEventCreate(&e1), "event");
    float best = 1e30f;
    int bb = b->block, bn = b->nt, bw = b->W;
    lbm_status s = LBM_OK;
    auto trial = [&](int block, int nt, int W) {
        b->block = block;
        b->nt = nt;
        b->W = W;
        s = reset(b);
        if (s != LBM_OK) return;
        (void)hipEventRecord(e0, b->stream);
        s = bbatch_step(b, steps_per_trial);
        (void)hipEventRecord(e1, b->stream);
        (void)hipEventSynchronize(e1);
        if (s != LBM_OK) return;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; bb = block; bn = nt; bw = W; }
    };
    // workgroup size and hints at one cell per thread, then cells per
    // thread at the best of those
    for (int block : {256, 512, 1024})
        for (int nt = 0; nt < 2 && s == LBM_OK; ++nt) trial(block, nt, 1);
    const int b1 = bb, n1 = bn;
    for (int W : {2, 4})
        if (s == LBM_OK) trial(b1, n1, W);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->block = bb;
    b->nt = bn;
    b->W = bw;
    lbm_status s2 = reset(b);
    if (s != LBM_OK) return s;
    if (s2 != LBM_OK) return s2;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[{b->arch, b->ndom, b->nb}] = {bb, bn | (bw << 1)};
    return LBM_OK;
}

// block: threads per workgroup of the brick sweep (one brick per wavefront);
// W: cells per thread, i.e. groups of block / 64 bricks each workgroup steps
// in turn (1, 2 or 4)
lbm_status bbatch_set_launch(BrickBatch* b, int32_t block, int32_t W) {
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return set_error(LBM_E_INVAL, "block must be 64, 128, 256, 512 or 1024");
    if (W != 1 && W != 2 && W != 4) return set_error(LBM_E_INVAL, "brick batches take 1, 2 or 4 cells per thread");
    b->block = block;
    b->W = W;
    return LBM_OK;
}

lbm_status bbatch_get_launch(BrickBatch* b, int32_t* block, int32_t* W) {
    if (block) *block = b->block;
    if (W) *W = b->W;
    return LBM_OK;
}

void bbatch_destroy(BrickBatch* b) { delete b; }

// "brick-batch ARCH DOMAINS BRICKS BLOCK NT CELLS_PER_THREAD"
void bbatch_tuning_export(std::string& out) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_cache)
        out += "brick-batch " + kv.first.arch + " " + std::to_string(kv.first.ndom) + " " +
               std::to_string(kv.first.bricks) + " " + std::to_string(kv.second.first) + " " +
               std::to_string(kv.second.second & 1) + " " + std::to_string(kv.second.second >> 1) + "\n";
}

int bbatch_tuning_import(const std::vector<std::string>& f, bool apply) {
    if (f.empty() || f[0] != "brick-batch") return 0;
    int64_t nd = 0, nb = 0, block = 0, nt = 0, w = 0;
    if (f.size() != 7 || f[1].empty() || !parse_i64(f[2], nd) || !parse_i64(f[3], nb) || !parse_i64(f[4], block) ||
        !parse_i64(f[5], nt) || !parse_i64(f[6], w))
        return -1;
    const bool ok_block = block == 64 || block == 128 || block == 256 || block == 512 || block == 1024;
    if (nd < 1 || nb < 0 || !ok_block || (nt != 0 && nt != 1) || (w != 1 && w != 2 && w != 4)) return -1;
    if (apply) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[{f[1], (int)nd, nb}] = {(int)block, (int)(nt | (w << 1))};
    }
    return 1;
}

}  // namespace lbm
