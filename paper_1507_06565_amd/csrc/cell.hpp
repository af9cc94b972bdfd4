// Fused stream + collide sweep of the D3Q19 TRT lattice Boltzmann method
// (Sec. 2.1, eqs. (LBM), (TRT), (TRT2), (equilibrium), (Macro), (collision),
// (streaming)) with interpolated bounce-back at the solid surfaces (Sec. 2.2,
// eqs. (noslip), (CLI)), for gfx950.
//
// One thread per cell, x fastest, so a 64-wide wavefront reads and writes
// 64 consecutive floats of each population array.  Populations are FP32
// shifts g = f - w rho0.  The pass is HBM-bound: 19 loads + 19 stores of 4 B
// per fluid cell, plus a 4 B cell-info load; solid cells return at once.
//
// Boundary handling is fused into the sweep.  A fluid cell x with a link kk
// (x + e_kk solid) rebuilds its unknown population k = opp(kk) as
//     g_k(x, t+1) = c1 gt_kk(x) + c0 gt_kk(x - e_kk) + cb gt_k(x) [+ wall]
// (eq. (noslip), eq. (CLI), or Bouzidi), gt being post-collision values of
// step t.  At the end of step t the cell itself owns gt_kk(x) and gt_k(x), so
// it stores the partial value P = c1 gt_kk(x) + cb gt_k(x) [+ wall] in a
// per-link buffer (one float per link, in link order, so the values of a
// wavefront's cells are contiguous); at step t+1 the cell reads P back and
// adds c0 gt_kk(x - e_kk), which is the value it pulls for direction kk.
// The per-link data read is the link coefficient and P.  Each link's P is
// read and written by its own cell only.
//
// Solid cells are not updated, but a solid cell whose 32-cell group (one
// 128-byte line of every population array) contains fluid cells stores zeros
// into its own slots, so that the group's stores cover whole lines: partial
// lines cost extra HBM cycles.  No cell reads a solid cell's slots (the pull
// of a link direction is replaced by P), so the zeros are never used.
//
// Brick layout: the cells of every 4x4x4 brick that holds a fluid cell are
// stored together (local index lx + 4 ly + 16 lz, so a 32-lane group is one
// 4x4x2 half-brick and one 128-byte line); bricks without fluid are not
// stored.  It streams like the two-grid layout (pull from x - e_k, aligned
// store at x), with the source found through the brick's neighbour table.
//
// AA state locations: after an even step gt_k(x) is stored at A[kbar][x];
// after an odd step at A[k][x + e_k].  An even step reads A[k][x] and writes
// A[kbar][x]; an odd step reads A[kbar][x - e_k] and writes A[k][x + e_k].
// Every slot is read and written by one thread only.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace lbm {

using L = D3Q19;

// (c1, c0, cb) of a link from its coefficient word: CLI stores kappa =
// (1 - 2q)/(1 + 2q), Bouzidi stores q, NaN marks a moving-wall link (simple
// bounce-back plus the wall term).
template <int BC>
__device__ __forceinline__ void bb_coeffs(float prm, float& c1, float& c0, float& cb) {
#pragma clang fp contract(off)
    if (prm != prm) {
        c1 = 1.0f; c0 = 0.0f; cb = 0.0f;
    } else if (BC == LBM_BC_CLI) {
        c1 = 1.0f; c0 = prm; cb = -prm;
    } else if (BC == LBM_BC_BOUZIDI) {
        if (prm < 0.5f) {
            c1 = 2.0f * prm; c0 = 1.0f - 2.0f * prm; cb = 0.0f;
        } else {
            c1 = 1.0f / (2.0f * prm); c0 = 0.0f; cb = 1.0f - c1;
        }
    } else {
        c1 = 1.0f; c0 = 0.0f; cb = 0.0f;
    }
}

// TRT collision with the Guo forcing split into even and odd parts
// (eqs. (TRT), (TRT2), (equilibrium), (collision)), in place on g.
//
// With s = g_k + g_kbar, d = g_k - g_kbar, eu = e_k.u and w the weight of k,
// the post-collision pair is g_k + P + M and g_kbar + P - M, where
//   P = -omega+/2 s + w a + eu (4.5 omega+ w rho0 eu + 9 (1-omega+/2) w e_k.F)
//   M = -omega-/2 d + 3 omega- w rho0 eu + 3 (1-omega-/2) w e_k.F
//   a = omega+ drho - 1.5 omega+ rho0 u.u - 3 (1-omega+/2) u.F,
// which is the textbook form -omega+(g+ - eq+) + (1-omega+/2) S+ and
// -omega-(g- - eq-) + (1-omega-/2) S- with the uniform factors folded; the
// rest population becomes (1-omega+) g_0 + a/3.  FMAs are explicit and no
// other contraction is allowed, so every kernel that inlines this rounds
// identically and all of them agree bit for bit.
__device__ __forceinline__ float collide(float (&g)[Q], const CellConsts& a) {
#pragma clang fp contract(off)
    float drho = g[0];
    float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int k = 2 * p + 1;
        const float s = g[k] + g[k + 1];
        const float d = g[k] - g[k + 1];
        drho += s;
        if (L::ex[k]) jx = L::ex[k] > 0 ? jx + d : jx - d;
        if (L::ey[k]) jy = L::ey[k] > 0 ? jy + d : jy - d;
        if (L::ez[k]) jz = L::ez[k] > 0 ? jz + d : jz - d;
    }
    const float ux = __builtin_fmaf(jx, a.inv_rho0, a.fh[0]);
    const float uy = __builtin_fmaf(jy, a.inv_rho0, a.fh[1]);
    const float uz = __builtin_fmaf(jz, a.inv_rho0, a.fh[2]);
    const float uu = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
    const float uF = __builtin_fmaf(ux, a.F[0], __builtin_fmaf(uy, a.F[1], uz * a.F[2]));
    const float aa = __builtin_fmaf(a.a_uu, uu, __builtin_fmaf(a.a_uF, uF, a.wp * drho));
    const float al0 = aa * (1.0f / 3.0f);
    const float al1 = aa * (1.0f / 18.0f);
    const float al2 = aa * (1.0f / 36.0f);
    g[0] = __builtin_fmaf(a.om1, g[0], al0);
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int k = 2 * p + 1;
        const int c = p < 3 ? 0 : 1;
        float eu = 0.0f;
        if (L::ex[k]) eu = L::ex[k] > 0 ? eu + ux : eu - ux;
        if (L::ey[k]) eu = L::ey[k] > 0 ? eu + uy : eu - uy;
        if (L::ez[k]) eu = L::ez[k] > 0 ? eu + uz : eu - uz;
        const float gk = g[k], gkb = g[k + 1];
        const float s = gk + gkb;
        const float d = gk - gkb;
        const float P = __builtin_fmaf(eu, __builtin_fmaf(a.beta[c], eu, a.gam[p]),
                                       __builtin_fmaf(a.hp, s, c == 0 ? al1 : al2));
        const float M = __builtin_fmaf(a.hm, d, __builtin_fmaf(a.delta[c], eu, a.zet[p]));
        g[k] = (gk + P) + M;
        g[k + 1] = (gkb + P) - M;
    }
    return ux;
}

typedef __attribute__((address_space(1))) float gfloat;

// Population array bases.  PopBases: one pointer per direction (the
// single-domain sweep passes them as kernel arguments).  PopStrided: one base
// and the distance between arrays, for kernels that would otherwise hold 19
// pointers in scalar registers (the batched kernel); byte offsets
// 4 (k stride + cell) must stay below 2^32, which the host checks.
struct PopBases {
    float* const* p;
    __device__ __forceinline__ __attribute__((address_space(1))) char* at(int k, uint32_t idx) const {
        return (__attribute__((address_space(1))) char*)p[k] + (idx << 2);
    }
};
// PopWide: one base and the distance between arrays in bytes (64-bit); the
// array base is formed in scalar registers where it is used, so a loop over
// several bricks keeps two values live instead of 19 pointers.
struct PopWide {
    uint64_t base, sbytes;
    __device__ __forceinline__ __attribute__((address_space(1))) char* at(int k, uint32_t idx) const {
        return (__attribute__((address_space(1))) char*)(base + (uint64_t)k * sbytes) + (idx << 2);
    }
};
struct PopStrided {
    float* base;
    uint32_t stride;  // floats between consecutive arrays
    __device__ __forceinline__ __attribute__((address_space(1))) char* at(int k, uint32_t idx) const {
        return (__attribute__((address_space(1))) char*)base + (((uint32_t)k * stride + idx) << 2);
    }
};

template <bool NT>
__device__ __forceinline__ float ld(const gfloat* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st(gfloat* p, float v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// a pointer that is the same in every lane, kept in scalar registers
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Index of the neighbour x + (dx, dy, dz) of a cell in the dense layouts
// (x fastest, every axis wrapped; walls are solid cells of the grid).  All
// indices are below 2^31.
struct DenseNb {
    unsigned X[3], Y[3], Z[3], nx, ny;
    __device__ __forceinline__ DenseNb(int nx_, int ny_, int nz_, int x, int y, int z) {
        X[0] = (unsigned)(x == 0 ? nx_ - 1 : x - 1); X[1] = (unsigned)x; X[2] = (unsigned)(x == nx_ - 1 ? 0 : x + 1);
        Y[0] = (unsigned)(y == 0 ? ny_ - 1 : y - 1); Y[1] = (unsigned)y; Y[2] = (unsigned)(y == ny_ - 1 ? 0 : y + 1);
        Z[0] = (unsigned)(z == 0 ? nz_ - 1 : z - 1); Z[1] = (unsigned)z; Z[2] = (unsigned)(z == nz_ - 1 ? 0 : z + 1);
        nx = (unsigned)nx_;
        ny = (unsigned)ny_;
    }
    __device__ __forceinline__ unsigned operator()(int dx, int dy, int dz) const {
        return X[dx + 1] + nx * (Y[dy + 1] + ny * Z[dz + 1]);
    }
};

// Same in the brick layout: lane l of a wavefront is cell l of its brick,
// and lane j < 27 holds the stored index of the neighbouring brick in
// direction (j % 3 - 1, j / 3 % 3 - 1, j / 9 - 1) (wrapped; a brick without
// fluid is replaced by the brick itself, whose values are then never used:
// a fluid cell pulls from a cell of such a brick only along a link).  A cell
// on a face of its brick can only leave it through that face, so each lane
// needs at most six neighbour bricks (its x, y and z sides and their three
// pairwise edges); they are fetched once, across lanes, by the constructor,
// which every lane of the wavefront must run together.
struct BrickNb {
    int own;               // this brick
    int lx, ly, lz;        // local coordinates, 0..3
    int sx, sy, sz;        // side of the brick the cell touches per axis: -1, 0 or +1
    int bX, bY, bZ, bXY, bXZ, bYZ;
    __device__ __forceinline__ BrickNb(int table, int own_, int l) {
        own = own_;
        lx = l & 3; ly = (l >> 2) & 3; lz = l >> 4;
        sx = lx == 0 ? -1 : (lx == 3 ? 1 : 0);
        sy = ly == 0 ? -1 : (ly == 3 ? 1 : 0);
        sz = lz == 0 ? -1 : (lz == 3 ? 1 : 0);
        bX = __shfl(table, 13 + sx, 64);
        bY = __shfl(table, 13 + 3 * sy, 64);
        bZ = __shfl(table, 13 + 9 * sz, 64);
        bXY = __shfl(table, 13 + sx + 3 * sy, 64);
        bXZ = __shfl(table, 13 + sx + 9 * sz, 64);
        bYZ = __shfl(table, 13 + 3 * sy + 9 * sz, 64);
    }
    __device__ __forceinline__ unsigned operator()(int dx, int dy, int dz) const {
        const bool cx = dx != 0 && dx == sx, cy = dy != 0 && dy == sy, cz = dz != 0 && dz == sz;
        const int src = cx ? (cy ? bXY : (cz ? bXZ : bX)) : (cy ? (cz ? bYZ : bY) : (cz ? bZ : own));
        return (unsigned)src * 64u + (unsigned)(((lx + dx) & 3) + 4 * ((ly + dy) & 3) + 16 * ((lz + dz) & 3));
    }
};

// The cell word of a cell and the first link of its 512-cell link segment.
// Callers load them as early as they can: the link records' addresses
// depend on both.
struct CellHead {
    uint32_t inf;
    int32_t seg;
};

// Loads the head of cell c.  A wavefront covers 64 consecutive, 64-aligned
// cells (every layout and launch shape), so c >> SEG_SHIFT is the same in
// all its lanes and the segment base is one uniform load.
__device__ __forceinline__ CellHead load_head(const uint32_t* __restrict__ info, const int32_t* __restrict__ segbase,
                                              int c) {
    CellHead h;
    h.inf = info[c];
    h.seg = segbase[__builtin_amdgcn_readfirstlane((uint32_t)c >> SEG_SHIFT)];
    return h;
}

// One cell of one time step: pull (with the partial bounce-back values),
// link correction, collision, push and the next step's partial values.
// Returns the x-velocity of this step's moments (0 for a solid cell).  c is
// the cell's index in the population arrays, nbi(dx, dy, dz) that of its
// neighbour (DenseNb or BrickNb), h its head (load_head).
//
// MASKED (the head must already be in registers): a lane loads only the
// pulls it uses; a solid lane, and a fluid lane for a direction whose source
// is solid (a link: the pulled value is replaced by the partial value), load
// nothing, so a wavefront does not fetch lines only such lanes would touch.
template <int LAYOUT, int PARITY, int BC, bool NT, bool RELOAD, class PA, class NBI, bool MASKED = false>
__device__ __forceinline__ float cell_update(PA pa, PA pb, CellHead h, const float* __restrict__ lparam,
                                             const float* pva, float* pvb, const CellConsts& K, const NBI& nbi,
                                             int c) {
#pragma clang fp contract(off)
    static_assert(!MASKED || LAYOUT == L_TWOGRID, "masked pulls exist for the pull layouts only");
    const unsigned uc = (unsigned)c;
#define NB(dx, dy, dz) nbi((dx), (dy), (dz))

    // Addressing: population k of cell i is at byte offset 4*i from the
    // array base A + k*stride (uniform); 4*i fits 32 bits (the host limits a
    // domain to 2^30 cells), so loads use a scalar base + 32-bit offset.
#define AT(bases, k, idx) (*(__attribute__((address_space(1))) float*)(bases).at((k), (uint32_t)(idx)))

    // 1) streaming: all 19 pulls are issued together; the empty asm pins
    //    them ahead of the solid-cell branch, so a wavefront waits for memory
    //    once
    const uint32_t inf = h.inf;
    // pulls a lane does not need (MASKED): none if solid, else the link ones
    const uint32_t skip = inf == CELL_SOLID_WORD ? 0xFFFFFFFFu : (inf & LINK_MASK_BITS);
    float g[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if (MASKED) {
            // the source of pull k is x - e_k = x + e_opp(k): a link of x when
            // bit opp(k) - 1 of the mask is set
            const bool need = k == 0 ? skip != 0xFFFFFFFFu : !(skip & (1u << (opp(k) - 1)));
            if (need)
                g[k] = AT(pa, k, NB(-L::ex[k], -L::ey[k], -L::ez[k]));
            else
                g[k] = 0.0f;
        } else if (LAYOUT == L_TWOGRID)
            g[k] = AT(pa, k, NB(-L::ex[k], -L::ey[k], -L::ez[k]));
        else if (PARITY == P_EVEN)
            g[k] = ld<NT>(&AT(pa, k, uc));
        else
            g[k] = AT(pa, opp(k), NB(-L::ex[k], -L::ey[k], -L::ez[k]));
    }
    const __attribute__((address_space(1))) char* lp = (const __attribute__((address_space(1))) char*)lparam;
    const __attribute__((address_space(1))) char* vp = (const __attribute__((address_space(1))) char*)pva;
    float prm[Q], pv[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) asm volatile("" ::"v"(g[k]));
    // a solid cell whose 32-cell group holds fluid runs along with the fluid
    // lanes and stores zeros in the same store instructions (see above)
    const bool solid = inf == CELL_SOLID_WORD;
    const uint64_t fluid_lanes = __ballot(!solid);
    if (solid) {
        const uint32_t grp = (__lane_id() & 32) ? (uint32_t)(fluid_lanes >> 32) : (uint32_t)fluid_lanes;
        if (grp == 0u) return 0.0f;
    }
    const uint32_t mask = solid ? 0u : (inf & LINK_MASK_BITS);
    const int base = h.seg + (int)(inf >> 18);

    // 2) links: the unknown population is the partial value P stored last
    //    step plus c0 times the second node's value
    if (mask) {
        // every coefficient and partial-value load is issued before any is
        // used, each only by the lanes that have that link: a wavefront skips
        // the directions none of its lanes links along, and a load serves
        // only the lanes that need its value
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int kk = opp(k);
            prm[k] = 0.0f;
            pv[k] = 0.0f;
            if (mask & (1u << (kk - 1))) {
                const uint32_t li = (uint32_t)base + __popc(mask & ((1u << (kk - 1)) - 1u));
                prm[k] = *(const __attribute__((address_space(1))) float*)(lp + (li << 2));
                pv[k] = *(const __attribute__((address_space(1))) float*)(vp + (li << 2));
            }
        }
        // in place: g[kk] is read only when c0 != 0, i.e. when x + e_k is
        // fluid, so (x, k) is not itself a link and g[kk] is its pulled value
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int kk = opp(k);
            if (mask & (1u << (kk - 1))) {
                float c1, c0, cb;
                bb_coeffs<BC>(prm[k], c1, c0, cb);
                g[k] = (c0 != 0.0f) ? pv[k] + c0 * g[kk] : pv[k];
            }
        }
    }

    // 3) collision
    const float ux = collide(g, K);

    // 4) store
    const PA D = (LAYOUT == L_TWOGRID) ? pb : pa;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const float v = solid ? 0.0f : g[k];
        if (LAYOUT == L_TWOGRID)
            st<NT>(&AT(D, k, uc), v);
        else if (PARITY == P_EVEN)
            st<NT>(&AT(D, opp(k), uc), v);
        else
            AT(D, k, NB(L::ex[k], L::ey[k], L::ez[k])) = v;
    }
    // 5) partial bounce-back values for the next step; with RELOAD the
    //    coefficients are read again (a cache hit) rather than held in
    //    registers across the collision, for kernels short of registers
    if (mask) {
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int kk = opp(k);
            if (mask & (1u << (kk - 1))) {
                const uint32_t li = (uint32_t)base + __popc(mask & ((1u << (kk - 1)) - 1u));
                float pk = prm[k];
                if (RELOAD) pk = __builtin_nontemporal_load((const __attribute__((address_space(1))) float*)(lp + (li << 2)));
                float c1, c0, cb;
                bb_coeffs<BC>(pk, c1, c0, cb);
                const float P = c1 * g[kk] + cb * g[k] + (pk != pk ? K.wterm[k] : 0.0f);
                *(__attribute__((address_space(1))) float*)((__attribute__((address_space(1))) char*)pvb + (li << 2)) = P;
            }
        }
    }
    return solid ? 0.0f : ux;
#undef NB
#undef AT
}

}  // namespace lbm
