// Host images of the device-side geometry records of one domain: the cell
// words, the per-segment link bases, the per-link bounce-back coefficients
// (eq. (noslip), eq. (CLI), Bouzidi) and the seeds of the moving-wall partial
// values.
#include <limits>

#include "internal.hpp"

namespace lbm {

lbm_status build_images(const DomainGeo& G, int /*layout*/, int64_t stride, const CellConsts& K, DeviceImages& im,
                        std::string& err) {
    const int64_t N = G.ncells();
    const int64_t nl = (int64_t)G.lcell.size();
    im.info.assign((size_t)N, 0u);
    for (int64_t i = 0; i < N; ++i) im.info[i] = G.flags[i] == CELL_FLUID ? 0u : CELL_SOLID_WORD;
    const int64_t nseg = (N >> SEG_SHIFT) + 1;
    im.segbase.assign((size_t)nseg, 0);
    im.lparam.assign((size_t)(nl + Q), 0.0f);
    im.seed_idx.clear();
    im.seed_val.clear();
    const bool moving = G.desc.wall_hi_velocity[0] != 0.0 || G.desc.wall_hi_velocity[1] != 0.0 ||
                        G.desc.wall_hi_velocity[2] != 0.0;
    const int nx = G.desc.nx, ny = G.desc.ny, nz = G.desc.nz;
    {
        // first link of every segment (links are sorted by cell)
        int64_t li = 0;
        for (int64_t sg = 0; sg < nseg; ++sg) {
            while (li < nl && (G.lcell[li] >> SEG_SHIFT) < sg) ++li;
            im.segbase[sg] = (int32_t)li;
        }
    }
    for (int64_t i = 0; i < nl; ++i) {
        const int64_t cell = G.lcell[i];
        const int kk = G.ldir[i];
        if (i == 0 || cell != G.lcell[i - 1]) {
            const int64_t off = i - im.segbase[cell >> SEG_SHIFT];
            if (off < 0 || off >= (1 << 14)) {
                err = "internal: link offset outside its segment";
                return LBM_E_INVAL;
            }
            im.info[cell] = (uint32_t)off << 18;
        }
        im.info[cell] |= 1u << (kk - 1);
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
        im.lparam[i] = prm;
        if (mw) {
            // moving-wall links start from the wall term alone: the partial
            // value that the first step reads (state block 0, after the Q
            // population arrays)
            im.seed_idx.push_back((int64_t)Q * stride + i);
            im.seed_val.push_back(K.wterm[opp(kk)]);
        }
    }
    return LBM_OK;
}

}  // namespace lbm
