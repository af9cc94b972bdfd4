// Host images of the device-side geometry records of one domain: the cell
// words, the per-segment link bases, the per-link bounce-back coefficients
// (eq. (noslip), eq. (CLI), Bouzidi) and the seeds of the moving-wall partial
// values, in the storage order of the layout (dense: the cell index; brick:
// stored brick * 64 + local index), plus the brick map of the brick layout.
#include <limits>

#include "internal.hpp"

namespace lbm {

bool brick_dims_ok(const lbm_domain_desc& d) {
    return d.nx % BRICK == 0 && d.ny % BRICK == 0 && d.nz % BRICK == 0;
}

void build_brick_map(const DomainGeo& G, BrickMap& bm, bool with_table) {
    const int nx = G.desc.nx, ny = G.desc.ny;
    bm.bx = G.desc.nx / BRICK;
    bm.by = G.desc.ny / BRICK;
    bm.bz = G.desc.nz / BRICK;
    const int64_t nb = (int64_t)bm.bx * bm.by * bm.bz;
    bm.id.assign((size_t)nb, -1);
    int64_t ns = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int X = (int)(b % bm.bx), Y = (int)((b / bm.bx) % bm.by), Z = (int)(b / ((int64_t)bm.bx * bm.by));
        bool fluid = false;
        for (int l = 0; l < 64 && !fluid; ++l) {
            const int x = X * BRICK + (l & 3), y = Y * BRICK + ((l >> 2) & 3), z = Z * BRICK + (l >> 4);
            fluid = G.flags[x + (int64_t)nx * (y + (int64_t)ny * z)] == CELL_FLUID;
        }
        if (fluid) bm.id[b] = (int32_t)ns++;
    }
    bm.nstored = ns;
    bm.nbr.clear();
    if (!with_table) return;
    bm.nbr.resize((size_t)(27 * ns));
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t me = bm.id[b];
        if (me < 0) continue;
        const int X = (int)(b % bm.bx), Y = (int)((b / bm.bx) % bm.by), Z = (int)(b / ((int64_t)bm.bx * bm.by));
        for (int j = 0; j < 27; ++j) {
            const int Xn = (X + j % 3 - 1 + bm.bx) % bm.bx;
            const int Yn = (Y + j / 3 % 3 - 1 + bm.by) % bm.by;
            const int Zn = (Z + j / 9 - 1 + bm.bz) % bm.bz;
            const int32_t o = bm.id[Xn + (int64_t)bm.bx * (Yn + (int64_t)bm.by * Zn)];
            bm.nbr[(size_t)me * 27 + j] = o < 0 ? me : o;
        }
    }
}

lbm_status build_images(const DomainGeo& G, int layout, const BrickMap& bm, int64_t stride, const CellConsts& K,
                        DeviceImages& im, std::string& err) {
    const int nx = G.desc.nx, ny = G.desc.ny, nz = G.desc.nz;
    const int64_t N = G.ncells();
    const int64_t nl = (int64_t)G.lcell.size();
    const bool brick = layout == L_BRICK;
    const int64_t NS = brick ? bm.nstored * 64 : N;  // stored cells
    // storage index of a (stored) dense cell
    auto sidx = [&](int64_t cell) -> int64_t {
        if (!brick) return cell;
        const int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((int64_t)nx * ny));
        const int32_t b = bm.id[x / BRICK + (int64_t)bm.bx * (y / BRICK + (int64_t)bm.by * (z / BRICK))];
        return b < 0 ? -1 : (int64_t)b * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3);
    };
    im.info.assign((size_t)NS, CELL_SOLID_WORD);
    if (brick) {
        for (int64_t b = 0; b < (int64_t)bm.id.size(); ++b) {
            const int32_t s = bm.id[b];
            if (s < 0) continue;
            const int X = (int)(b % bm.bx), Y = (int)((b / bm.bx) % bm.by), Z = (int)(b / ((int64_t)bm.bx * bm.by));
            for (int l = 0; l < 64; ++l) {
                const int x = X * BRICK + (l & 3), y = Y * BRICK + ((l >> 2) & 3), z = Z * BRICK + (l >> 4);
                if (G.flags[x + (int64_t)nx * (y + (int64_t)ny * z)] == CELL_FLUID) im.info[(size_t)s * 64 + l] = 0u;
            }
        }
    } else {
        for (int64_t i = 0; i < N; ++i) im.info[i] = G.flags[i] == CELL_FLUID ? 0u : CELL_SOLID_WORD;
    }
    // links in storage order: the geometry lists them by (cell, k); within a
    // brick the dense order of its cells is the local order (z, then y, then
    // x), so a stable counting sort by stored brick gives (storage index, k)
    std::vector<int64_t> order;
    if (brick) {
        std::vector<int64_t> start((size_t)bm.nstored + 1, 0);
        std::vector<int64_t> lb((size_t)nl);
        for (int64_t i = 0; i < nl; ++i) {
            const int64_t s = sidx(G.lcell[i]);
            if (s < 0) {
                err = "internal: link of a cell outside the stored bricks";
                return LBM_E_INVAL;
            }
            lb[i] = s >> 6;
            ++start[lb[i] + 1];
        }
        for (int64_t b = 0; b < bm.nstored; ++b) start[b + 1] += start[b];
        order.resize((size_t)nl);
        for (int64_t i = 0; i < nl; ++i) order[start[lb[i]]++] = i;
    }
    auto link_at = [&](int64_t j) { return brick ? order[j] : j; };
    const int64_t nseg = (NS >> SEG_SHIFT) + 1;
    im.segbase.assign((size_t)nseg, 0);
    im.lparam.assign((size_t)(nl + Q), 0.0f);
    im.seed_idx.clear();
    im.seed_val.clear();
    const bool moving = G.desc.wall_hi_velocity[0] != 0.0 || G.desc.wall_hi_velocity[1] != 0.0 ||
                        G.desc.wall_hi_velocity[2] != 0.0;
    {
        // first link of every segment (links are in storage order)
        int64_t j = 0;
        for (int64_t sg = 0; sg < nseg; ++sg) {
            while (j < nl && (sidx(G.lcell[link_at(j)]) >> SEG_SHIFT) < sg) ++j;
            im.segbase[sg] = (int32_t)j;
        }
    }
    int64_t prev = -1;
    for (int64_t j = 0; j < nl; ++j) {
        const int64_t i = link_at(j);
        const int64_t cell = G.lcell[i];
        const int64_t s = sidx(cell);
        const int kk = G.ldir[i];
        if (s != prev) {
            const int64_t off = j - im.segbase[s >> SEG_SHIFT];
            if (off < 0 || off >= (1 << 14)) {
                err = "internal: link offset outside its segment";
                return LBM_E_INVAL;
            }
            im.info[s] = (uint32_t)off << 18;
            prev = s;
        }
        im.info[s] |= 1u << (kk - 1);
        // second fluid node x - e_kk decides the interpolation fallback
        const int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((int64_t)nx * ny));
        int x2 = x - D3Q19::ex[kk], y2 = y - D3Q19::ey[kk], z2 = z - D3Q19::ez[kk];
        x2 = (x2 + nx) % nx; y2 = (y2 + ny) % ny; z2 = (z2 + nz) % nz;
        const bool f2 = G.flags[x2 + (int64_t)nx * (y2 + (int64_t)ny * z2)] == CELL_FLUID;
        const double q = G.lq[i];
        float prm = 0.0f;
        const bool mw = moving && G.lsurf[i] == SURF_WALL_HI;
        if (mw) {
            prm = std::numeric_limits<float>::quiet_NaN();
        } else if (G.desc.bc == LBM_BC_CLI) {
            prm = f2 ? (float)((1.0 - 2.0 * q) / (1.0 + 2.0 * q)) : 0.0f;
        } else if (G.desc.bc == LBM_BC_BOUZIDI) {
            prm = (q < 0.5 && !f2) ? 0.5f : (float)q;
        }
        im.lparam[j] = prm;
        if (mw) {
            // moving-wall links start from the wall term alone: the partial
            // value that the first step reads (state block 0, after the Q
            // population arrays)
            im.seed_idx.push_back((int64_t)Q * stride + j);
            im.seed_val.push_back(K.wterm[opp(kk)]);
        }
    }
    return LBM_OK;
}

}  // namespace lbm
