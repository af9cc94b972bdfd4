// Host geometry build: voxelisation of spheres and wall layers into cell
// flags, and the boundary-link list with wall distances q (Sec. 2.2, eq.
// (CLI): q = |x_f1 - x_w| / |x_f1 - x_b|).
//
// Sphere data are dyadic (multiples of 2^-12), so every squared distance and
// every discriminant formed here is exact in binary64; q needs one correctly
// rounded square root.  The result is therefore a plain function of the input,
// independent of thread count and traversal order.
//
// Work is split into z-slabs over host threads.  Sphere candidates for a cell
// come from a uniform bucket grid in which each sphere image is registered in
// every bucket its (r + 1)-expanded box touches: a unit-step segment from x
// can only meet a ball whose expanded box contains x.
#include <algorithm>
#include <cmath>
#include <thread>

#include "internal.hpp"

namespace lbm {
namespace {

using L = D3Q19;

struct Img {
    double cx, cy, cz, r;
};

bool is_dyadic(double v) {
    const double s = v * 4096.0;
    return std::isfinite(s) && std::floor(s) == s && std::fabs(s) < 9.0e15;
}

int n_threads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min(h, 32u);
}

template <class F>
void parallel_slabs(int nz, F&& fn) {
    const int T = std::max(1, std::min(n_threads(), nz));
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        const int za = (int)((int64_t)nz * t / T), zb = (int)((int64_t)nz * (t + 1) / T);
        th.emplace_back([&fn, t, za, zb] { fn(t, za, zb); });
    }
    for (auto& x : th) x.join();
}

}  // namespace

lbm_status build_domain(const lbm_domain_desc& din, DomainGeo& out, std::string& err) {
    lbm_domain_desc d = din;
    const int n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1 || n[a] > (1 << 20)) { err = "domain size out of range"; return LBM_E_INVAL; }
        const bool per = d.periodic[a] != 0;
        const bool lo = d.wall_lo[a] != 0, hi = d.wall_hi[a] != 0;
        if (per ? (lo || hi) : !(lo && hi)) {
            err = "every axis must be periodic or bounded by wall layers on both sides";
            return LBM_E_INVAL;
        }
        if (!per && n[a] < 3) { err = "a walled axis needs at least 3 cells"; return LBM_E_INVAL; }
    }
    const int64_t N = (int64_t)d.nx * d.ny * d.nz;
    if (N > (int64_t)1 << 30) { err = "more than 2^30 cells in one domain"; return LBM_E_INVAL; }
    if (d.bc < LBM_BC_SBB || d.bc > LBM_BC_BOUZIDI) { err = "unknown boundary scheme"; return LBM_E_INVAL; }
    if (d.n_spheres < 0 || (d.n_spheres > 0 && !d.spheres)) { err = "bad sphere array"; return LBM_E_INVAL; }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d.wall_hi_velocity[a])) { err = "bad wall velocity"; return LBM_E_INVAL; }

    out.spheres.assign(d.spheres, d.spheres + d.n_spheres);
    for (const auto& s : out.spheres) {
        const double c[3] = {s.cx, s.cy, s.cz};
        if (!(s.r > 0.0) || !is_dyadic(s.r) || s.r > 1024.0) { err = "sphere radius must be a positive multiple of 2^-12"; return LBM_E_INVAL; }
        for (int a = 0; a < 3; ++a) {
            if (!is_dyadic(c[a]) || std::fabs(c[a]) > 65536.0) { err = "sphere centre must be a multiple of 2^-12"; return LBM_E_INVAL; }
            if (d.periodic[a] && !(c[a] >= 0.0 && c[a] < n[a] && s.r < n[a])) {
                err = "sphere centre must lie in [0, n) and r < n along a periodic axis";
                return LBM_E_INVAL;
            }
        }
    }
    d.spheres = out.spheres.data();
    out.desc = d;

    // sphere images: shifts of -n, 0, +n along periodic axes
    std::vector<Img> imgs;
    for (const auto& s : out.spheres) {
        const double c[3] = {s.cx, s.cy, s.cz};
        for (int i = -1; i <= 1; ++i)
            for (int j = -1; j <= 1; ++j)
                for (int l = -1; l <= 1; ++l) {
                    const int sh[3] = {i, j, l};
                    bool ok = true;
                    double p[3];
                    for (int a = 0; a < 3; ++a) {
                        if (sh[a] != 0 && !d.periodic[a]) { ok = false; break; }
                        p[a] = c[a] + (double)sh[a] * n[a];
                        // keep only images whose expanded box meets the domain
                        if (p[a] + s.r + 1.0 < 0.0 || p[a] - s.r - 1.0 > n[a] - 1) { ok = false; break; }
                    }
                    if (ok) imgs.push_back({p[0], p[1], p[2], s.r});
                }
    }

    // ---- flags
    out.flags.assign((size_t)N, CELL_FLUID);
    uint8_t* F = out.flags.data();
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    auto wall_layer = [&](int x, int y, int z) {
        return (d.wall_lo[0] && x == 0) || (d.wall_hi[0] && x == nx - 1) || (d.wall_lo[1] && y == 0) ||
               (d.wall_hi[1] && y == ny - 1) || (d.wall_lo[2] && z == 0) || (d.wall_hi[2] && z == nz - 1);
    };
    parallel_slabs(nz, [&](int, int za, int zb) {
        for (int z = za; z < zb; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    if (wall_layer(x, y, z)) F[x + (int64_t)nx * (y + (int64_t)ny * z)] = CELL_WALL;
        for (const auto& s : imgs) {
            const int z0 = std::max(za, (int)std::ceil(s.cz - s.r));
            const int z1 = std::min(zb - 1, (int)std::floor(s.cz + s.r));
            if (z0 > z1) continue;
            const int y0 = std::max(0, (int)std::ceil(s.cy - s.r)), y1 = std::min(ny - 1, (int)std::floor(s.cy + s.r));
            const int x0 = std::max(0, (int)std::ceil(s.cx - s.r)), x1 = std::min(nx - 1, (int)std::floor(s.cx + s.r));
            const double r2 = s.r * s.r;
            for (int z = z0; z <= z1; ++z) {
                const double dz = (double)z - s.cz;
                for (int y = y0; y <= y1; ++y) {
                    const double dy = (double)y - s.cy;
                    const double dyz = dy * dy + dz * dz;
                    if (dyz > r2) continue;
                    uint8_t* row = F + (int64_t)nx * (y + (int64_t)ny * z);
                    for (int x = x0; x <= x1; ++x) {
                        const double dx = (double)x - s.cx;
                        // same predicate as |x - c|^2 <= r^2 (all terms exact)
                        if (row[x] == CELL_FLUID && dx * dx + dy * dy + dz * dz <= r2) row[x] = CELL_SPHERE;
                    }
                }
            }
        }
    });

    // ---- bucket grid of sphere images for the link pass
    const int B = 8;
    const int gb[3] = {(nx + B - 1) / B, (ny + B - 1) / B, (nz + B - 1) / B};
    std::vector<std::vector<int>> bucket((size_t)gb[0] * gb[1] * gb[2]);
    for (int i = 0; i < (int)imgs.size(); ++i) {
        const auto& s = imgs[i];
        const double c[3] = {s.cx, s.cy, s.cz};
        int lo[3], hi[3];
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::max(0, (int)std::ceil(c[a] - s.r - 1.0));
            hi[a] = std::min(n[a] - 1, (int)std::floor(c[a] + s.r + 1.0));
            if (lo[a] > hi[a]) ok = false;
        }
        if (!ok) continue;
        for (int bz = lo[2] / B; bz <= hi[2] / B; ++bz)
            for (int by = lo[1] / B; by <= hi[1] / B; ++by)
                for (int bx = lo[0] / B; bx <= hi[0] / B; ++bx)
                    bucket[bx + (size_t)gb[0] * (by + (size_t)gb[1] * bz)].push_back(i);
    }

    // ---- links, per slab, concatenated in slab order
    const int T = std::max(1, std::min(n_threads(), nz));
    struct Part {
        std::vector<int64_t> cell;
        std::vector<int8_t> dir;
        std::vector<double> q;
        std::vector<int8_t> surf;
        int64_t fluid = 0;
    };
    std::vector<Part> parts(T);
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        const int za = (int)((int64_t)nz * t / T), zb = (int)((int64_t)nz * (t + 1) / T);
        th.emplace_back([&, t, za, zb] {
            Part& P = parts[t];
            for (int z = za; z < zb; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        const int64_t c = x + (int64_t)nx * (y + (int64_t)ny * z);
                        if (F[c] != CELL_FLUID) continue;
                        ++P.fluid;
                        const std::vector<int>& cand = bucket[x / B + (size_t)gb[0] * (y / B + (size_t)gb[1] * (z / B))];
                        for (int k = 1; k < Q; ++k) {
                            int xn = x + L::ex[k], yn = y + L::ey[k], zn = z + L::ez[k];
                            xn = xn < 0 ? nx - 1 : (xn == nx ? 0 : xn);
                            yn = yn < 0 ? ny - 1 : (yn == ny ? 0 : yn);
                            zn = zn < 0 ? nz - 1 : (zn == nz ? 0 : zn);
                            const uint8_t fn = F[xn + (int64_t)nx * (yn + (int64_t)ny * zn)];
                            if (fn == CELL_FLUID) continue;
                            double q = INFINITY;
                            int8_t surf = SURF_SPHERE;
                            if (wall_layer(xn, yn, zn)) {
                                q = 0.5;
                                const bool hi = (d.wall_hi[0] && xn == nx - 1) || (d.wall_hi[1] && yn == ny - 1) ||
                                                (d.wall_hi[2] && zn == nz - 1);
                                surf = hi ? SURF_WALL_HI : SURF_WALL_LO;
                            }
                            const double a2 = (double)norm2(k);
                            for (int i : cand) {
                                const Img& s = imgs[i];
                                const double dx = (double)x - s.cx, dy = (double)y - s.cy, dz = (double)z - s.cz;
                                const double b = L::ex[k] * dx + L::ey[k] * dy + L::ez[k] * dz;
                                const double c0 = dx * dx + dy * dy + dz * dz - s.r * s.r;
                                const double disc = b * b - a2 * c0;
                                if (disc < 0.0) continue;
                                const double tq = (-b - std::sqrt(disc)) / a2;
                                if (tq > 0.0 && tq <= 1.0 && tq < q) {
                                    q = tq;
                                    surf = SURF_SPHERE;
                                }
                            }
                            P.cell.push_back(c);
                            P.dir.push_back((int8_t)k);
                            P.q.push_back(q);
                            P.surf.push_back(surf);
                        }
                    }
        });
    }
    for (auto& x : th) x.join();
    size_t total = 0;
    out.n_fluid = 0;
    for (auto& P : parts) { total += P.cell.size(); out.n_fluid += P.fluid; }
    out.lcell.resize(total); out.ldir.resize(total); out.lq.resize(total); out.lsurf.resize(total);
    size_t o = 0;
    for (auto& P : parts) {
        std::copy(P.cell.begin(), P.cell.end(), out.lcell.begin() + o);
        std::copy(P.dir.begin(), P.dir.end(), out.ldir.begin() + o);
        std::copy(P.q.begin(), P.q.end(), out.lq.begin() + o);
        std::copy(P.surf.begin(), P.surf.end(), out.lsurf.begin() + o);
        o += P.cell.size();
    }
    for (size_t i = 0; i < total; ++i)
        if (!(out.lq[i] > 0.0 && out.lq[i] <= 1.0)) {
            err = "internal: a solid neighbour without a surface on its link";
            return LBM_E_INVAL;
        }
    return LBM_OK;
}

}  // namespace lbm
