"""Seeded synthetic inputs for the pore-scale and gray-column workloads.

This module is the single source of inputs for both the GPU library and the
CPU oracle.  It holds no lattice Boltzmann arithmetic: it only draws sphere
packings, domain descriptors and porosity profiles.

The paper builds its porous beds with a rigid-body code that drops spheres
under gravity (Sec. 3.1); the packings here are a seeded stand-in with the
same structure: polydisperse spheres (radii uniform in a range, as in
Sec. 3.1 where radii vary by up to 50% of a mean diameter), non-overlapping,
filling a bed below a free channel, with spheres allowed to reach below the
bottom wall so that the wall does not create a high-porosity layer (the
set-up fix described in Sec. 3.1).

Sphere centres and radii are quantised to multiples of 2**-12 lattice units,
so that every squared distance and every ray/sphere discriminant a geometry
builder forms from them is exact in binary64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DYADIC = 4096.0  # 2**12: sphere data are multiples of 1/DYADIC


def quantise(a: np.ndarray) -> np.ndarray:
    return np.round(np.asarray(a, dtype=np.float64) * DYADIC) / DYADIC


@dataclass
class Domain:
    """Pore-scale domain: a box of nx*ny*nz cells (x fastest in memory).

    walls are solid node layers at index 0 (lo) and n-1 (hi) of an axis; the
    wall surface is half-way between the wall layer and the first fluid layer.
    """
    nx: int
    ny: int
    nz: int
    periodic: tuple = (1, 1, 0)
    wall_lo: tuple = (0, 0, 1)
    wall_hi: tuple = (0, 0, 1)
    wall_hi_velocity: tuple = (0.0, 0.0, 0.0)
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    bc: str = "cli"  # "sbb" | "cli" | "bouzidi"
    name: str = ""

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Params:
    """Collision parameters in lattice units (rho0 = 1 unless stated)."""
    collision: str = "trt"  # "bgk" | "trt"
    tau_plus: float = 0.7
    magic_lambda: float = 3.0 / 16.0
    rho0: float = 1.0
    force: tuple = (1e-6, 0.0, 0.0)
    layout: str = "twogrid"  # "twogrid" | "aa" | "brick" | "auto" (timed by the layout autotuner)


# ----------------------------------------------------------------------------
# sphere packing: random placement + collective rearrangement (push-apart)
# ----------------------------------------------------------------------------

def _pairs(tree, rmax2):
    return tree.query_pairs(rmax2, output_type="ndarray")


def pack_spheres(seed: int, box: tuple, periodic: tuple, r_range: tuple,
                 solid_volume: float, zc_bounds=None, gap: float = 2.0 ** -9,
                 max_iter: int = 3000, shrink: float = 0.995, relax_tol: float = 0.02):
    """Random non-overlapping polydisperse spheres.

    box: (Lx, Ly, Lz) extent of the placement region; centres x,y in [0, L),
    z in zc range.  periodic: per-axis periodicity of the placement box.
    solid_volume: target total sphere volume (continuous).
    zc_bounds: callable(r) -> (zmin, zmax) constraint on the centre height
    for non-periodic z (None: z in [0, Lz) periodic or free).
    Returns an (n, 4) float64 array (cx, cy, cz, r) of dyadic values with
    pairwise distances >= r_i + r_j (periodic images included), exactly.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    a, b = r_range
    radii = []
    vol = 0.0
    while vol < solid_volume:
        r = rng.uniform(a, b)
        radii.append(r)
        vol += 4.0 / 3.0 * math.pi * r ** 3
    if radii and vol - solid_volume > 0.5 * 4.0 / 3.0 * math.pi * radii[-1] ** 3:
        radii.pop()
    R = np.array(sorted(radii, reverse=True), dtype=np.float64)
    n = len(R)
    L = np.array(box, dtype=np.float64)
    per = np.array(periodic, dtype=bool)
    P = rng.uniform(0.0, 1.0, size=(n, 3)) * L
    if zc_bounds is not None:
        lo, hi = zc_bounds(R)
        P[:, 2] = lo + rng.uniform(0.0, 1.0, size=n) * np.maximum(hi - lo, 0.0)

    boxsize = np.where(per, L, 1e9)

    def clamp(P):
        for ax in range(3):
            if per[ax]:
                P[:, ax] = np.mod(P[:, ax], L[ax])
        if zc_bounds is not None:
            lo, hi = zc_bounds(R)
            P[:, 2] = np.clip(P[:, 2], lo, hi)
        return P

    def min_image(d):
        for ax in range(3):
            if per[ax]:
                d[:, ax] -= L[ax] * np.round(d[:, ax] / L[ax])
        return d

    P = clamp(P)

    def overlaps(P, R):
        rmax = 2.0 * R.max() + gap
        tree = cKDTree(np.where(per, np.mod(P, L), P + 1e4), boxsize=boxsize)
        pr = _pairs(tree, rmax)
        if len(pr) == 0:
            return (np.zeros(0, int),) * 2 + (np.zeros((0, 3)), np.zeros(0), np.zeros(0))
        i, j = pr[:, 0], pr[:, 1]
        d = min_image(P[j] - P[i])
        dist = np.sqrt((d * d).sum(1))
        ov = R[i] + R[j] + gap - dist
        m = ov > 0
        return i[m], j[m], d[m], dist[m], ov[m]

    # collective rearrangement: push overlapping pairs apart (Jacobi sweeps)
    # until the largest overlap is below relax_tol ...
    for it in range(max_iter):
        i, j, d, dist, ov = overlaps(P, R)
        if len(ov) == 0 or ov.max() <= relax_tol:
            break
        dist = np.maximum(dist, 1e-12)
        u = d / dist[:, None]
        wi = R[j] ** 3 / (R[i] ** 3 + R[j] ** 3)  # heavier spheres move less
        wj = 1.0 - wi
        disp = np.zeros_like(P)
        np.add.at(disp, i, -(ov * wi * 0.55)[:, None] * u)
        np.add.at(disp, j, (ov * wj * 0.55)[:, None] * u)
        P = clamp(P + disp)
        if (it + 1) % 500 == 0:
            R *= shrink  # jammed: shrink all radii slightly and continue
    # ... then remove what is left by shrinking the spheres involved
    for _ in range(200):
        i, j, d, dist, ov = overlaps(P, R)
        if len(ov) == 0:
            break
        cut = np.zeros(n)
        np.maximum.at(cut, i, 0.5 * ov + gap)
        np.maximum.at(cut, j, 0.5 * ov + gap)
        R = R - cut

    S = np.empty((n, 4))
    S[:, :3] = P
    S[:, 3] = R
    S = quantise(S)
    for ax in range(3):
        if per[ax]:
            S[:, ax] = np.mod(S[:, ax], L[ax])
    S = _fix_exact(S, L, per, zc_bounds)
    return S


def _fix_exact(S, L, per, zc_bounds):
    """Shrink any sphere pair that overlaps after quantisation (exact test)."""
    from scipy.spatial import cKDTree

    boxsize = np.where(per, L, 1e9)
    for _ in range(100):
        tree = cKDTree(np.where(per, S[:, :3], S[:, :3] + 1e4), boxsize=boxsize)
        pr = _pairs(tree, 2.0 * S[:, 3].max() + 1e-6)
        if len(pr) == 0:
            return S
        i, j = pr[:, 0], pr[:, 1]
        d = S[j, :3] - S[i, :3]
        for ax in range(3):
            if per[ax]:
                d[:, ax] -= L[ax] * np.round(d[:, ax] / L[ax])
        d2 = (d * d).sum(1)              # exact: dyadic with <= 24 frac bits
        rs = S[i, 3] + S[j, 3]
        bad = d2 < rs * rs
        if not bad.any():
            return S
        for k in np.unique(np.concatenate([i[bad], j[bad]])):
            S[k, 3] -= 1.0 / DYADIC
    raise RuntimeError("could not remove overlaps after quantisation")


def check_non_overlap(S, L, per) -> bool:
    """Exact pairwise non-overlap test (brute force, small inputs)."""
    n = len(S)
    for a in range(n):
        d = S[a + 1:, :3] - S[a, :3]
        for ax in range(3):
            if per[ax]:
                d[:, ax] -= L[ax] * np.round(d[:, ax] / L[ax])
        d2 = (d * d).sum(1)
        rs = S[a + 1:, 3] + S[a, 3]
        if np.any(d2 < rs * rs):
            return False
    return True


def voxel_solid_count(S, shape, periodic, z_range=None) -> int:
    """Approximate-free count of lattice points inside any sphere (closed ball),
    restricted to z in z_range; used only to steer the generator's porosity."""
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), dtype=bool)
    for cx, cy, cz, r in S:
        shifts = []
        for ax, (c, n) in enumerate(((cx, nx), (cy, ny), (cz, nz))):
            s = [0.0]
            if periodic[ax]:
                s = [-float(n), 0.0, float(n)]
            shifts.append(s)
        for sx in shifts[0]:
            for sy in shifts[1]:
                for sz in shifts[2]:
                    c = (cx + sx, cy + sy, cz + sz)
                    lo = [max(0, math.ceil(c[i] - r)) for i in range(3)]
                    hi = [min(n - 1, math.floor(c[i] + r)) for i, n in enumerate((nx, ny, nz))]
                    if any(lo[i] > hi[i] for i in range(3)):
                        continue
                    xs = np.arange(lo[0], hi[0] + 1) - c[0]
                    ys = np.arange(lo[1], hi[1] + 1) - c[1]
                    zs = np.arange(lo[2], hi[2] + 1) - c[2]
                    d2 = zs[:, None, None] ** 2 + ys[None, :, None] ** 2 + xs[None, None, :] ** 2
                    solid[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] |= d2 <= r * r
    if z_range is not None:
        solid = solid[z_range[0]:z_range[1]]
    return int(solid.sum())


class PackingError(RuntimeError):
    """No attempt of the generator met the porosity and radius tolerances."""


# Jam shrinking and overlap repair may take radii somewhat below the lower end
# of the drawn range; an attempt is accepted only if no radius fell below this
# fraction of it.
R_SHRINK_MIN = 0.95
# further seeds tried (seed + RESEED * k) when the volume-steered attempts miss
RESEED = 1_000_000
RESEED_TRIES = 24


def packing_ok(S, r_range, eps, porosity, tol):
    """Acceptance of a packing: voxel porosity within tol of the target and
    every radius in [R_SHRINK_MIN * r_lo, r_hi]."""
    if abs(eps - porosity) > tol:
        return False
    if len(S) == 0:
        return True
    return bool(S[:, 3].min() >= R_SHRINK_MIN * r_range[0] and S[:, 3].max() <= r_range[1])


def porous_bed(seed, nx, ny, nz, bed_top, r_range, porosity, tol=0.01, max_tries=6, reseeds=RESEED_TRIES):
    """Spheres filling the bed layers [1, bed_top) of a channel with wall
    layers at z = 0 and z = nz-1, periodic in x and y.

    Centre heights obey z_c + r <= bed_top and z_c - r >= 0.5 - 2*rbar, so
    spheres may be cut by the bottom wall (no wall-induced porosity layer).
    The voxel porosity of layers [1, bed_top) is steered to the target by
    rescaling the sphere volume over max_tries attempts (the first three with
    the given seed); if none is accepted (packing_ok), further seeds
    seed + RESEED * k (k = 1 .. reseeds) are tried; PackingError if every
    attempt misses.
    """
    rbar = 0.5 * (r_range[0] + r_range[1])
    bed_cells = nx * ny * (bed_top - 1)
    z_lo_plane = 0.5 - 2.0 * rbar

    def zc_bounds(R):
        return z_lo_plane + R, bed_top - R

    target_solid = (1.0 - porosity) * bed_cells

    def attempt(sd, vol):
        S = pack_spheres(sd, (nx, ny, bed_top), (1, 1, 0), r_range, vol, zc_bounds=zc_bounds)
        solid = voxel_solid_count(S, (nx, ny, nz), (1, 1, 0), (1, bed_top))
        return S, 1.0 - solid / bed_cells, solid

    vol = target_solid
    for k in range(max_tries):
        S, eps, solid = attempt(seed + 1000003 * k if k >= 3 else seed, vol)
        if packing_ok(S, r_range, eps, porosity, tol):
            return S, eps
        vol *= target_solid / max(solid, 1.0)
    for k in range(1, reseeds + 1):
        vol = target_solid
        for _ in range(3):
            S, eps, solid = attempt(seed + RESEED * k, vol)
            if packing_ok(S, r_range, eps, porosity, tol):
                return S, eps
            vol *= target_solid / max(solid, 1.0)
    raise PackingError(f"bed {nx}x{ny}x{nz} (seed {seed}): no packing within {tol} of porosity {porosity}")


def rev_cube(seed, edge, r_range, porosity, tol=0.02, max_tries=6, reseeds=RESEED_TRIES):
    """Periodic cube of edge cells filled to a target voxel porosity: the
    sphere volume is rescaled over max_tries attempts with the given seed,
    then further seeds seed + RESEED * k (k = 1 .. reseeds) are tried;
    PackingError if no attempt meets packing_ok."""
    cells = edge ** 3
    target_solid = (1.0 - porosity) * cells

    def attempt(sd, vol):
        S = pack_spheres(sd, (edge, edge, edge), (1, 1, 1), r_range, vol)
        solid = voxel_solid_count(S, (edge,) * 3, (1, 1, 1))
        return S, 1.0 - solid / cells, solid

    for k in range(reseeds + 1):
        vol = target_solid
        for _ in range(max_tries if k == 0 else 3):
            S, eps, solid = attempt(seed + RESEED * k, vol)
            if packing_ok(S, r_range, eps, porosity, tol):
                return S, eps
            vol *= target_solid / max(solid, 1.0)
    raise PackingError(f"REV cube {edge}^3 (seed {seed}): no packing within {tol} of porosity {porosity}")


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def channel_c0():
    """32^3 plain channel: periodic x,y; wall layers z=0, z=31; no spheres."""
    d = Domain(32, 32, 32, name="channel-32^3")
    d.bc = "sbb"
    p = Params(collision="bgk", tau_plus=0.8, magic_lambda=(0.8 - 0.5) ** 2,
               force=(1e-6, 0.0, 0.0))
    return d, p


def coupled_c1(seed=1, bc="bouzidi", porosity=0.6):
    """128x64x256 free channel over a sphere bed in layers [1,128)."""
    S, eps = porous_bed(seed, 128, 64, 256, 128, (6.0, 10.0), porosity)
    d = Domain(128, 64, 256, spheres=S, bc=bc, name="coupled-128x64x256")
    p = Params(collision="trt", tau_plus=0.7, magic_lambda=3.0 / 16.0,
               force=(1e-6, 0.0, 0.0))
    return d, p, eps


def large_c2(seed=2):
    """512x256x1024 free channel over a sphere bed in layers [1,512)."""
    S, eps = porous_bed(seed, 512, 256, 1024, 512, (8.0, 16.0), 0.45)
    d = Domain(512, 256, 1024, spheres=S, bc="cli", name="large-512x256x1024")
    p = Params(collision="trt", tau_plus=0.7, magic_lambda=3.0 / 16.0,
               force=(5e-7, 0.0, 0.0), layout="aa")
    return d, p, eps


def rev_sample_c3(i, edges=(32, 48, 64, 96)):
    """i-th periodic REV cube: edge uniform in edges, porosity U[0.35,0.9]."""
    rng = np.random.default_rng(1000 + i)
    edge = int(edges[rng.integers(0, len(edges))])
    target = float(rng.uniform(0.35, 0.9))
    S, eps = rev_cube(1000 + i, edge, (3.0, 10.0), target)
    d = Domain(edge, edge, edge, periodic=(1, 1, 1), wall_lo=(0, 0, 0),
               wall_hi=(0, 0, 0), spheres=S, bc="cli", name=f"rev-{i}-{edge}")
    p = Params(collision="trt", tau_plus=1.0, magic_lambda=3.0 / 16.0,
               force=(1e-6, 0.0, 0.0))
    return d, p, target, eps


def smoothed_step_porosity(nz, seed):
    """Column porosity: 1 in the upper half, eps_p below, joined by a smoothed
    step S(s) = 3s^2 - 2s^3 of width w centred at nz/2."""
    rng = np.random.default_rng(2000 + seed)
    eps_p = float(rng.uniform(0.4, 0.8))
    w = float(rng.uniform(4.0, 32.0))
    z = np.arange(nz, dtype=np.float64)
    s = np.clip((z - nz / 2 + w / 2) / w, 0.0, 1.0)
    S = 3 * s * s - 2 * s ** 3
    return eps_p + (1.0 - eps_p) * S, eps_p, w


def cubic_array(L, a):
    """Simple-cubic array: one sphere of radius a centred in a periodic cube."""
    c = L / 2.0 + 0.0
    S = quantise(np.array([[c + 0.25, c + 0.125, c + 0.375, a]]))
    return Domain(L, L, L, periodic=(1, 1, 1), wall_lo=(0, 0, 0), wall_hi=(0, 0, 0),
                  spheres=S, bc="cli", name=f"sc-{L}-{a}")
