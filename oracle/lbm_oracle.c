/*
 * Plain FP64 CPU oracle for the pore-scale lattice Boltzmann hot path and the
 * gray (Brinkman) column model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It is written for clarity, not speed:
 * every step follows the paper's definitions in the order the paper gives
 * them, in binary64, with no blocking or fusion.
 *
 * Passages followed (Fattahi, Waluga, Wohlmuth, Ruede, arXiv:1507.06565):
 *   - lattice Boltzmann equation with a source term, eq. (LBM), Sec. 2.1
 *   - D3Q19 velocity set, Sec. 2.1
 *   - TRT collision and its symmetric/antisymmetric split, eqs. (TRT), (TRT2)
 *   - relaxation rates 1/omega+ = 3 nu + 1/2, omega- in (0,2), Sec. 2.1
 *   - incompressible equilibrium with density fluctuation, eq. (equilibrium)
 *   - moments, eq. (Macro); collision / streaming split, eqs. (collision),
 *     (streaming)
 *   - magic parameter Lambda, Sec. 2.1
 *   - simple bounce-back, eq. (noslip); central linear interpolation (CLI)
 *     bounce-back and the wall distance q, eq. (CLI), Sec. 2.2
 *   - generalised (gray) model for porous media, eqs. (GeneralizedPor1),
 *     (GeneralizedPor2), (PorousForce), (SteadyVelocity), Sec. 4; its
 *     discretisation is that of the cited Guo & Zhao (2002) model.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes): populations are stored shifted, g = f - w*rho0 (the paper's
 * equilibrium is written for the density fluctuation); the body force enters
 * through Guo's source term split into its even and odd parts with
 * (1 - omega+/2) and (1 - omega-/2); the velocity is u = (sum e g + F/2)/rho0;
 * the second-node CLI term falls back to simple bounce-back when the second
 * node is not fluid; Bouzidi's linear interpolation is offered beside CLI;
 * the moving-wall correction is Ladd's 6 w rho0 e.u_w.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* --------------------------------------------------------------------------
 * D3Q19 velocity set (Sec. 2.1): one rest velocity, six axis velocities and
 * twelve edge diagonals.  Weights: 1/3, 1/18, 1/36 by |e|^2 = 0, 1, 2; they
 * sum to one.  The opposite index is found by search, not assumed.
 * -------------------------------------------------------------------------- */
static const int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double W[19];
static int OPP[19];
static int tables_ready = 0;

static void tables(void) {
    if (tables_ready) return;
    for (int k = 0; k < 19; ++k) {
        int e2 = EX[k] * EX[k] + EY[k] * EY[k] + EZ[k] * EZ[k];
        W[k] = (e2 == 0) ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        for (int j = 0; j < 19; ++j)
            if (EX[j] == -EX[k] && EY[j] == -EY[k] && EZ[j] == -EZ[k]) OPP[k] = j;
    }
    tables_ready = 1;
}

void orc_lattice(int32_t* e /*19*3*/, double* w /*19*/, int32_t* opp /*19*/) {
    tables();
    for (int k = 0; k < 19; ++k) {
        e[3 * k] = EX[k]; e[3 * k + 1] = EY[k]; e[3 * k + 2] = EZ[k];
        w[k] = W[k]; opp[k] = OPP[k];
    }
}

/* --------------------------------------------------------------------------
 * Domain description (shared layout with the Python side of the oracle only).
 * -------------------------------------------------------------------------- */
typedef struct {
    int32_t n[3];
    int32_t periodic[3];
    int32_t wall_lo[3];
    int32_t wall_hi[3];
    double wall_hi_vel[3];
    const double* spheres; /* nsph * (cx, cy, cz, r) */
    int64_t nsph;
    int32_t bc; /* 0 simple bounce-back, 1 CLI, 2 Bouzidi linear */
} odomain;

enum { ORC_OK = 0, ORC_INVAL = -1, ORC_UNSTABLE = -5 };
enum { FLUID = 0, SPHERE = 1, WALL = 2 };
enum { SURF_SPHERE = 0, SURF_WALL_LO = 1, SURF_WALL_HI = 2 };

static int64_t cell_index(const odomain* d, int x, int y, int z) {
    return (int64_t)x + (int64_t)d->n[0] * ((int64_t)y + (int64_t)d->n[1] * z);
}

static int valid_domain(const odomain* d) {
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) return 0;
        if (d->periodic[a] && (d->wall_lo[a] || d->wall_hi[a])) return 0;
        if (!d->periodic[a] && !(d->wall_lo[a] && d->wall_hi[a])) return 0;
    }
    for (int64_t s = 0; s < d->nsph; ++s) {
        double r = d->spheres[4 * s + 3];
        if (!(r > 0.0)) return 0;
        for (int a = 0; a < 3; ++a)
            if (d->periodic[a] && !(r < d->n[a])) return 0;
    }
    return 1;
}

static int in_wall_layer(const odomain* d, const int c[3]) {
    for (int a = 0; a < 3; ++a) {
        if (d->wall_lo[a] && c[a] == 0) return 1;
        if (d->wall_hi[a] && c[a] == d->n[a] - 1) return 1;
    }
    return 0;
}

/* image shifts of a sphere along axis a: {-n, 0, n} if periodic, else {0} */
static int shifts(const odomain* d, int a, double* s) {
    if (d->periodic[a]) { s[0] = -d->n[a]; s[1] = 0.0; s[2] = d->n[a]; return 3; }
    s[0] = 0.0; return 1;
}

/* Solid predicate: a cell centre is solid when it lies in the closed ball of
 * some sphere image.  With dyadic sphere data every term is exact. */
static int inside(double x, double y, double z, double cx, double cy, double cz, double r) {
    double dx = x - cx, dy = y - cy, dz = z - cz;
    return dx * dx + dy * dy + dz * dz <= r * r;
}

/* Flags by marking each sphere image's bounding box. */
int orc_flags(const odomain* d, uint8_t* flags) {
    if (!valid_domain(d)) return ORC_INVAL;
    const int nx = d->n[0], ny = d->n[1], nz = d->n[2];
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int c[3] = {x, y, z};
                flags[cell_index(d, x, y, z)] = in_wall_layer(d, c) ? WALL : FLUID;
            }
    double sx[3], sy[3], sz[3];
    int nsx = shifts(d, 0, sx), nsy = shifts(d, 1, sy), nsz = shifts(d, 2, sz);
    for (int64_t s = 0; s < d->nsph; ++s) {
        const double* S = d->spheres + 4 * s;
        for (int i = 0; i < nsx; ++i)
            for (int j = 0; j < nsy; ++j)
                for (int l = 0; l < nsz; ++l) {
                    double cx = S[0] + sx[i], cy = S[1] + sy[j], cz = S[2] + sz[l], r = S[3];
                    int x0 = (int)ceil(cx - r), x1 = (int)floor(cx + r);
                    int y0 = (int)ceil(cy - r), y1 = (int)floor(cy + r);
                    int z0 = (int)ceil(cz - r), z1 = (int)floor(cz + r);
                    x0 = x0 < 0 ? 0 : x0;
                    y0 = y0 < 0 ? 0 : y0;
                    z0 = z0 < 0 ? 0 : z0;
                    x1 = x1 > nx - 1 ? nx - 1 : x1;
                    y1 = y1 > ny - 1 ? ny - 1 : y1;
                    z1 = z1 > nz - 1 ? nz - 1 : z1;
                    for (int z = z0; z <= z1; ++z)
                        for (int y = y0; y <= y1; ++y)
                            for (int x = x0; x <= x1; ++x) {
                                int64_t id = cell_index(d, x, y, z);
                                if (flags[id] == FLUID && inside(x, y, z, cx, cy, cz, r)) flags[id] = SPHERE;
                            }
                }
    }
    return ORC_OK;
}

/* Flags by testing every cell against every sphere image (small inputs). */
int orc_flags_bruteforce(const odomain* d, uint8_t* flags) {
    if (!valid_domain(d)) return ORC_INVAL;
    double sx[3], sy[3], sz[3];
    int nsx = shifts(d, 0, sx), nsy = shifts(d, 1, sy), nsz = shifts(d, 2, sz);
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                int c[3] = {x, y, z};
                uint8_t f = in_wall_layer(d, c) ? WALL : FLUID;
                for (int64_t s = 0; s < d->nsph && f == FLUID; ++s) {
                    const double* S = d->spheres + 4 * s;
                    for (int i = 0; i < nsx; ++i)
                        for (int j = 0; j < nsy; ++j)
                            for (int l = 0; l < nsz; ++l)
                                if (inside(x, y, z, S[0] + sx[i], S[1] + sy[j], S[2] + sz[l], S[3])) f = SPHERE;
                }
                flags[cell_index(d, x, y, z)] = f;
            }
    return ORC_OK;
}

/* neighbour of (x,y,z) along e_k, wrapped on periodic axes; returns 0 if the
 * neighbour falls outside a non-periodic axis */
static int neighbour(const odomain* d, const int c[3], int k, int out[3]) {
    int e[3] = {EX[k], EY[k], EZ[k]};
    for (int a = 0; a < 3; ++a) {
        int v = c[a] + e[a];
        if (v < 0 || v >= d->n[a]) {
            if (!d->periodic[a]) return 0;
            v = (v + d->n[a]) % d->n[a];
        }
        out[a] = v;
    }
    return 1;
}

/* A link (x, k) exists for a fluid cell x whose neighbour x + e_k is not
 * fluid.  Links are enumerated in increasing (cell, k) order. */
int64_t orc_count_links(const odomain* d, const uint8_t* flags) {
    tables();
    int64_t n = 0;
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                int c[3] = {x, y, z}, nb[3];
                if (flags[cell_index(d, x, y, z)] != FLUID) continue;
                for (int k = 1; k < 19; ++k) {
                    if (!neighbour(d, c, k, nb)) return -1;
                    if (flags[cell_index(d, nb[0], nb[1], nb[2])] != FLUID) ++n;
                }
            }
    return n;
}

/* Smallest t in (0,1] at which x + t e_k enters the closed ball (c, r); the
 * root of |d + t e|^2 = r^2 with d = x - c, written a t^2 + 2 b t + c0 = 0,
 * a = |e|^2, b = e.d, c0 = |d|^2 - r^2, taking the smaller root
 * t = (-b - sqrt(b^2 - a c0)) / a.  Returns +inf if there is none. */
static double entry(int x, int y, int z, int k, double cx, double cy, double cz, double r) {
    double dx = x - cx, dy = y - cy, dz = z - cz;
    double a = (double)(EX[k] * EX[k] + EY[k] * EY[k] + EZ[k] * EZ[k]);
    double b = EX[k] * dx + EY[k] * dy + EZ[k] * dz;
    double c0 = dx * dx + dy * dy + dz * dz - r * r;
    double disc = b * b - a * c0;
    if (disc < 0.0) return INFINITY;
    double t = (-b - sqrt(disc)) / a;
    if (t > 0.0 && t <= 1.0) return t;
    return INFINITY;
}

/* The wall distance q of every link (eq. (CLI): q is the distance from the
 * fluid node to the wall over the node spacing along the link).  For a wall
 * layer the surface is half-way, q = 1/2; for a sphere it is the first entry
 * of the link segment into any sphere image.  The first surface along the
 * segment wins; a sphere must be strictly closer than a wall to win. */
int orc_links(const odomain* d, const uint8_t* flags, int64_t nlinks,
              int64_t* cell, int8_t* dir, double* q, int8_t* surf) {
    tables();
    if (!valid_domain(d)) return ORC_INVAL;
    const int64_t N = (int64_t)d->n[0] * d->n[1] * d->n[2];
    int64_t* first = (int64_t*)malloc(sizeof(int64_t) * N);
    if (!first) return ORC_INVAL;
    int64_t l = 0;
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                int64_t id = cell_index(d, x, y, z);
                first[id] = -1;
                if (flags[id] != FLUID) continue;
                int c[3] = {x, y, z}, nb[3];
                for (int k = 1; k < 19; ++k) {
                    if (!neighbour(d, c, k, nb)) { free(first); return ORC_INVAL; }
                    if (flags[cell_index(d, nb[0], nb[1], nb[2])] == FLUID) continue;
                    if (l >= nlinks) { free(first); return ORC_INVAL; }
                    if (first[id] < 0) first[id] = l;
                    cell[l] = id;
                    dir[l] = (int8_t)k;
                    if (in_wall_layer(d, nb)) {
                        int hi = 0;
                        for (int a = 0; a < 3; ++a)
                            if (d->wall_hi[a] && nb[a] == d->n[a] - 1) hi = 1;
                        q[l] = 0.5;
                        surf[l] = hi ? SURF_WALL_HI : SURF_WALL_LO;
                    } else {
                        q[l] = INFINITY;
                        surf[l] = SURF_SPHERE;
                    }
                    ++l;
                }
            }
    if (l != nlinks) { free(first); return ORC_INVAL; }
    double sx[3], sy[3], sz[3];
    int nsx = shifts(d, 0, sx), nsy = shifts(d, 1, sy), nsz = shifts(d, 2, sz);
    for (int64_t s = 0; s < d->nsph; ++s) {
        const double* S = d->spheres + 4 * s;
        for (int i = 0; i < nsx; ++i)
            for (int j = 0; j < nsy; ++j)
                for (int m = 0; m < nsz; ++m) {
                    double cx = S[0] + sx[i], cy = S[1] + sy[j], cz = S[2] + sz[m], r = S[3];
                    /* a segment of unit steps from x can touch the ball only if
                     * every coordinate of x is within r + 1 of the centre */
                    int x0 = (int)ceil(cx - r - 1), x1 = (int)floor(cx + r + 1);
                    int y0 = (int)ceil(cy - r - 1), y1 = (int)floor(cy + r + 1);
                    int z0 = (int)ceil(cz - r - 1), z1 = (int)floor(cz + r + 1);
                    x0 = x0 < 0 ? 0 : x0;
                    y0 = y0 < 0 ? 0 : y0;
                    z0 = z0 < 0 ? 0 : z0;
                    if (x1 > d->n[0] - 1) x1 = d->n[0] - 1;
                    if (y1 > d->n[1] - 1) y1 = d->n[1] - 1;
                    if (z1 > d->n[2] - 1) z1 = d->n[2] - 1;
                    for (int z = z0; z <= z1; ++z)
                        for (int y = y0; y <= y1; ++y)
                            for (int x = x0; x <= x1; ++x) {
                                int64_t id = cell_index(d, x, y, z);
                                if (first[id] < 0) continue;
                                for (int64_t t = first[id]; t < nlinks && cell[t] == id; ++t) {
                                    double e = entry(x, y, z, dir[t], cx, cy, cz, r);
                                    if (e < q[t]) { q[t] = e; surf[t] = SURF_SPHERE; }
                                }
                            }
                }
    }
    free(first);
    for (int64_t t = 0; t < nlinks; ++t)
        if (!(q[t] > 0.0 && q[t] <= 1.0)) return ORC_INVAL;
    return ORC_OK;
}

/* Same root by bisection on the segment (test check of the closed form). */
double orc_entry_bisect(int x, int y, int z, int k, double cx, double cy, double cz, double r, int iters) {
    tables();
    double lo = 0.0, hi = 1.0;
    double ex = EX[k], ey = EY[k], ez = EZ[k];
    /* requires the end point inside and the start outside */
    for (int i = 0; i < iters; ++i) {
        double t = 0.5 * (lo + hi);
        double px = x + t * ex - cx, py = y + t * ey - cy, pz = z + t * ez - cz;
        if (px * px + py * py + pz * pz <= r * r) hi = t; else lo = t;
    }
    return hi;
}

double orc_entry(int x, int y, int z, int k, double cx, double cy, double cz, double r) {
    tables();
    return entry(x, y, z, k, cx, cy, cz, r);
}

/* --------------------------------------------------------------------------
 * Relaxation rates (Sec. 2.1): 1/omega+ = 3 nu + 1/2 = tau+; the magic
 * parameter Lambda = (1/omega+ - 1/2)(1/omega- - 1/2) fixes omega-.  BGK is
 * the TRT with omega- = omega+.  omega- must lie in (0, 2).
 * -------------------------------------------------------------------------- */
int orc_rates(int trt, double tau_plus, double lambda, double* wp, double* wm) {
    if (!(tau_plus > 0.5)) return ORC_INVAL;
    double tau_minus = trt ? 0.5 + lambda / (tau_plus - 0.5) : tau_plus;
    *wp = 1.0 / tau_plus;
    *wm = 1.0 / tau_minus;
    if (!(*wm > 0.0 && *wm < 2.0) || !(*wp > 0.0 && *wp < 2.0)) return ORC_INVAL;
    return ORC_OK;
}

/* Interpolated bounce-back coefficients (c1, c0, cb) of
 *   g_kbar(x, t+1) = c1 gt_k(x) + c0 gt_k(x - e_k) + cb gt_kbar(x)
 * for a link k from fluid x into the solid (eq. (noslip) and eq. (CLI)).
 * f2 tells whether the second fluid node x - e_k is fluid. */
static void coefficients(int bc, double q, int f2, double* c1, double* c0, double* cb) {
    *c1 = 1.0; *c0 = 0.0; *cb = 0.0;                    /* simple bounce-back */
    if (bc == 1 && f2) {                                /* CLI */
        double kappa = (1.0 - 2.0 * q) / (1.0 + 2.0 * q);
        *c1 = 1.0; *c0 = kappa; *cb = -kappa;
    } else if (bc == 2) {                               /* Bouzidi linear */
        if (q < 0.5) {
            if (f2) { *c1 = 2.0 * q; *c0 = 1.0 - 2.0 * q; *cb = 0.0; }
        } else {
            *c1 = 1.0 / (2.0 * q); *c0 = 0.0; *cb = (2.0 * q - 1.0) / (2.0 * q);
        }
    }
}

void orc_coefficients(int bc, double q, int f2, double* c) { coefficients(bc, q, f2, c, c + 1, c + 2); }

/* --------------------------------------------------------------------------
 * The pore-scale time step on a window of the domain (two grids, pull).
 *
 * State between steps: post-collision shifted populations gt_k(x).
 * Window: cells org + [0, win) in global coordinates (x fastest).  Along an
 * axis the window wraps if it spans a whole periodic axis; otherwise a value
 * read from outside the window is NaN, so that only cells far enough from the
 * window edge are exact after n steps (one cell per step).
 *
 *  wflags[M]          flags of the window cells
 *  wq[19*M]           q of link (x, k) (x + e_k not fluid), NaN if no link
 *  wsurf[19*M]        surface of that link (sphere / low wall / high wall)
 *  ga, gb [19*M]      state; the result is returned in ga
 *  rho[M], u[3*M]     moments of the last step (0 in solid cells)
 * -------------------------------------------------------------------------- */
typedef struct {
    int32_t trt;
    double tau_plus, magic_lambda, rho0, force[3];
} oparams;

int orc_run(const odomain* d, const oparams* p, const int32_t org[3], const int32_t win[3],
            const uint8_t* wflags, const double* wq, const int8_t* wsurf,
            double* ga, double* gb, int64_t nsteps, double* rho, double* u) {
    tables();
    if (!valid_domain(d)) return ORC_INVAL;
    double wp, wm;
    if (orc_rates(p->trt, p->tau_plus, p->magic_lambda, &wp, &wm) != ORC_OK) return ORC_INVAL;
    const int wx = win[0], wy = win[1], wz = win[2];
    const int64_t M = (int64_t)wx * wy * wz;
    int wrap[3];
    for (int a = 0; a < 3; ++a) wrap[a] = (win[a] == d->n[a]) && d->periodic[a];
    const double r0 = p->rho0, F[3] = {p->force[0], p->force[1], p->force[2]};
    const double* uw = d->wall_hi_vel;
    double* src = ga;
    double* dst = gb;
    int unstable = 0;
    for (int64_t step = 0; step < nsteps; ++step) {
        #pragma omp parallel for schedule(static)
        for (int z = 0; z < wz; ++z) {
            for (int y = 0; y < wy; ++y)
                for (int x = 0; x < wx; ++x) {
                    const int64_t id = x + (int64_t)wx * (y + (int64_t)wy * z);
                    if (wflags[id] != FLUID) {
                        for (int k = 0; k < 19; ++k) dst[k * M + id] = 0.0;
                        if (step == nsteps - 1) { rho[id] = 0; u[id] = u[M + id] = u[2 * M + id] = 0; }
                        continue;
                    }
                    /* window index of x + s*e_k, or -1 if outside the window */
                    #define NB(kk, s, out)                                                     \
                        do {                                                                   \
                            int cc[3] = {x + (s) * EX[kk], y + (s) * EY[kk], z + (s) * EZ[kk]}; \
                            int ok = 1;                                                        \
                            for (int a = 0; a < 3; ++a) {                                      \
                                if (cc[a] < 0 || cc[a] >= win[a]) {                            \
                                    if (wrap[a]) cc[a] = (cc[a] + win[a]) % win[a];            \
                                    else ok = 0;                                               \
                                }                                                              \
                            }                                                                  \
                            out = ok ? cc[0] + (int64_t)wx * (cc[1] + (int64_t)wy * cc[2]) : -1; \
                        } while (0)
                    double g[19];
                    /* streaming (eq. (streaming)), pull form, with bounce-back
                     * for the populations that would come out of the solid */
                    for (int kd = 0; kd < 19; ++kd) {
                        const int k = OPP[kd];          /* link direction into the solid */
                        const double qq = (kd == 0) ? NAN : wq[k * M + id];
                        if (kd != 0 && !isnan(qq)) {
                            int64_t f2;
                            NB(k, -1, f2);              /* second fluid node x - e_k */
                            int f2fluid = (f2 < 0) ? 1 : (wflags[f2] == FLUID);
                            double c1, c0, cb;
                            coefficients(d->bc, qq, f2fluid, &c1, &c0, &cb);
                            double v2 = (f2 < 0) ? NAN : src[k * M + f2];
                            double val = c1 * src[k * M + id] + cb * src[kd * M + id];
                            if (c0 != 0.0) val += c0 * v2;
                            if (wsurf[k * M + id] == SURF_WALL_HI) {
                                double eu = EX[kd] * uw[0] + EY[kd] * uw[1] + EZ[kd] * uw[2];
                                val += 6.0 * W[kd] * r0 * eu;   /* moving wall */
                            }
                            g[kd] = val;
                        } else {
                            int64_t s;
                            NB(kd, -1, s);
                            g[kd] = (s < 0) ? NAN : src[kd * M + s];
                        }
                    }
                    #undef NB
                    /* moments (eq. (Macro)) with the half-force velocity */
                    double drho = 0, jx = 0, jy = 0, jz = 0;
                    for (int k = 0; k < 19; ++k) {
                        drho += g[k];
                        jx += EX[k] * g[k]; jy += EY[k] * g[k]; jz += EZ[k] * g[k];
                    }
                    const double ux = (jx + 0.5 * F[0]) / r0, uy = (jy + 0.5 * F[1]) / r0, uz = (jz + 0.5 * F[2]) / r0;
                    const double uu = ux * ux + uy * uy + uz * uz;
                    if (step == nsteps - 1) { rho[id] = drho; u[id] = ux; u[M + id] = uy; u[2 * M + id] = uz; }
                    if (!(fabs(ux) < 0.4 && fabs(uy) < 0.4 && fabs(uz) < 0.4) && !isnan(ux)) unstable = 1;
                    /* incompressible equilibrium (eq. (equilibrium)), c_s^2 = 1/3 */
                    double geq[19], S[19];
                    for (int k = 0; k < 19; ++k) {
                        const double eu = EX[k] * ux + EY[k] * uy + EZ[k] * uz;
                        geq[k] = W[k] * (drho + r0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
                        /* Guo source: w [3 (e - u).F + 9 (e.u)(e.F)] */
                        const double eF = EX[k] * F[0] + EY[k] * F[1] + EZ[k] * F[2];
                        const double uF = ux * F[0] + uy * F[1] + uz * F[2];
                        S[k] = W[k] * (3.0 * (eF - uF) + 9.0 * eu * eF);
                    }
                    /* TRT collision (eqs. (TRT), (TRT2), (collision)) */
                    for (int k = 0; k < 19; ++k) {
                        const int kb = OPP[k];
                        const double gp = 0.5 * (g[k] + g[kb]), gm = 0.5 * (g[k] - g[kb]);
                        const double ep = 0.5 * (geq[k] + geq[kb]), em = 0.5 * (geq[k] - geq[kb]);
                        const double sp = 0.5 * (S[k] + S[kb]), sm = 0.5 * (S[k] - S[kb]);
                        dst[k * M + id] = g[k] - wp * (gp - ep) - wm * (gm - em)
                                          + (1.0 - 0.5 * wp) * sp + (1.0 - 0.5 * wm) * sm;
                    }
                }
        }
        double* t = src; src = dst; dst = t;
    }
    if (src != ga) memcpy(ga, src, sizeof(double) * 19 * M);
    return unstable ? ORC_UNSTABLE : ORC_OK;
}

/* --------------------------------------------------------------------------
 * Gray (generalised Navier-Stokes / Brinkman) model on a 1 x 1 x nz column,
 * Sec. 4, eqs. (GeneralizedPor2), (PorousForce), discretised as in the cited
 * Guo & Zhao (2002) model in its incompressible (shifted) variant with a TRT
 * collision; the Forchheimer coefficient is zero (Stokes regime, Sec. 4).
 *
 * Per cell: porosity eps, effective viscosity nu_eff (sets tau+ = 3 nu_eff +
 * 1/2, tau- from Lambda), drag coefficient D = eps nu / K (0 in free fluid).
 *   equilibrium  g_eq = w [drho + rho0 (3 e.u + 4.5 (e.u)^2/eps - 1.5 u.u/eps)]
 *   force        F = -D u + eps G
 *   source       w rho0 [3 e.F + 9 (e.u)(e.F)/eps - 3 u.F/eps]
 *   velocity     v = sum e g / rho0 + eps G / 2,  u = v / (1 + D/2)
 * Walls (if walls != 0): solid layers z = 0 and z = nz-1 with half-way
 * bounce-back; the top wall moves with velocity uw (Ladd's correction).
 * The column is periodic along x and y, so every population streams along z
 * only.  g[19*nz] holds post-collision populations; it is advanced nsteps;
 * u_out[3*nz] returns the velocity of the last step.
 * -------------------------------------------------------------------------- */
int orc_gray_run(int nz, int walls, const double* eps, const double* nu_eff, const double* drag,
                 const double* forch, double lambda, double rho0, const double G[3], const double uw[3],
                 double* g, int64_t nsteps, double* u_out) {
    tables();
    if (nz < 3) return ORC_INVAL;
    double* src = g;
    double* dst = (double*)calloc((size_t)19 * nz, sizeof(double));
    if (!dst) return ORC_INVAL;
    int unstable = 0;
    for (int64_t step = 0; step < nsteps; ++step) {
        for (int z = 0; z < nz; ++z) {
            int solid = walls && (z == 0 || z == nz - 1);
            if (solid) {
                for (int k = 0; k < 19; ++k) dst[k * nz + z] = 0.0;
                if (step == nsteps - 1) u_out[3 * z] = u_out[3 * z + 1] = u_out[3 * z + 2] = 0.0;
                continue;
            }
            double wp, wm;
            if (orc_rates(1, 3.0 * nu_eff[z] + 0.5, lambda, &wp, &wm) != ORC_OK) { free(dst); return ORC_INVAL; }
            double gg[19];
            for (int kd = 0; kd < 19; ++kd) {
                int zs = z - EZ[kd];
                if (zs < 0 || zs >= nz) {
                    if (walls) { free(dst); return ORC_INVAL; }
                    zs = (zs + nz) % nz;
                }
                if (walls && (zs == 0 || zs == nz - 1)) {
                    double val = src[OPP[kd] * nz + z];       /* half-way bounce-back */
                    if (zs == nz - 1) val += 6.0 * W[kd] * rho0 * (EX[kd] * uw[0] + EY[kd] * uw[1] + EZ[kd] * uw[2]);
                    gg[kd] = val;
                } else {
                    gg[kd] = src[kd * nz + zs];
                }
            }
            double drho = 0, j[3] = {0, 0, 0};
            for (int k = 0; k < 19; ++k) {
                drho += gg[k];
                j[0] += EX[k] * gg[k]; j[1] += EY[k] * gg[k]; j[2] += EZ[k] * gg[k];
            }
            const double e = eps[z], D = drag[z], phi = forch ? forch[z] : 0.0;
            double uu = 0, v[3], uv[3], Ft[3];
            for (int a = 0; a < 3; ++a) v[a] = j[a] / rho0 + 0.5 * e * G[a];
            /* the velocity is implicit in the porous force F = -D u - phi |u| u + eps G
               (eq. PorousForce): u = v - F(u)/2 solved for u */
            double den = 1.0 + 0.5 * D;
            if (phi != 0.0) {
                const double c0 = 0.5 * (1.0 + 0.5 * D), c1 = 0.5 * phi;
                const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                den = c0 + sqrt(c0 * c0 + c1 * vn);
            }
            for (int a = 0; a < 3; ++a) uv[a] = v[a] / den;
            const double un = sqrt(uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2]);
            for (int a = 0; a < 3; ++a) { Ft[a] = -D * uv[a] - phi * un * uv[a] + e * G[a]; uu += uv[a] * uv[a]; }
            if (step == nsteps - 1) { u_out[3 * z] = uv[0]; u_out[3 * z + 1] = uv[1]; u_out[3 * z + 2] = uv[2]; }
            if (!(fabs(uv[0]) < 0.4) && !isnan(uv[0])) unstable = 1;
            double geq[19], S[19];
            for (int k = 0; k < 19; ++k) {
                double eu = EX[k] * uv[0] + EY[k] * uv[1] + EZ[k] * uv[2];
                double eF = EX[k] * Ft[0] + EY[k] * Ft[1] + EZ[k] * Ft[2];
                double uF = uv[0] * Ft[0] + uv[1] * Ft[1] + uv[2] * Ft[2];
                geq[k] = W[k] * (drho + rho0 * (3.0 * eu + 4.5 * eu * eu / e - 1.5 * uu / e));
                S[k] = W[k] * rho0 * (3.0 * eF + 9.0 * eu * eF / e - 3.0 * uF / e);
            }
            for (int k = 0; k < 19; ++k) {
                int kb = OPP[k];
                double gp = 0.5 * (gg[k] + gg[kb]), gm = 0.5 * (gg[k] - gg[kb]);
                double ep = 0.5 * (geq[k] + geq[kb]), em = 0.5 * (geq[k] - geq[kb]);
                double sp = 0.5 * (S[k] + S[kb]), sm = 0.5 * (S[k] - S[kb]);
                dst[k * nz + z] = gg[k] - wp * (gp - ep) - wm * (gm - em) + (1.0 - 0.5 * wp) * sp + (1.0 - 0.5 * wm) * sm;
            }
        }
        double* t = src; src = dst; dst = t;
    }
    if (src != g) { memcpy(g, src, sizeof(double) * 19 * nz); free(src); }
    else free(dst);
    return unstable ? ORC_UNSTABLE : ORC_OK;
}
