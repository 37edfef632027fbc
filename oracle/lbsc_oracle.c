/*
 * Plain FP64 CPU oracle of the two-component D3Q19 Shan-Chen lattice
 * Boltzmann step with the mass-conserving evaporation sink of Hessling, Xie
 * and Harting, "Diffusion dominated evaporation in multicomponent lattice
 * Boltzmann simulations" (arXiv:1701.03637).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * Everything is double precision, plain loops, no blocking and no fusion.
 * OpenMP only splits independent per-node loops over z-planes; every sum runs
 * serially in node order, so results do not depend on the thread count.
 *
 * Canonical step (state S(t) = post-stream, post-sink populations):
 *   1. moments rho^c = sum_i f_i^c, j^c = sum_i f_i^c e_i, psi^c = psi(rho^c)
 *      (Sec. II A, definitions after Eq. (eqdis); Eq. (psifunc))
 *   2. Shan-Chen force F^c = -psi^c g sum_i w_i psi^cbar(x+e_i) e_i (Eq. (sc))
 *   3. common velocity u' = sum_c rho^c u^c / sum_c rho^c (Sec. II A) and the
 *      force shift u_eq^c = u' + tau^c F^c / rho^c (Sec. II B)
 *   4. BGK relaxation towards f^eq(rho^c, u_eq^c) (Eqs. (LBM), (eqdis));
 *      sink nodes do not collide (Sec. II C: forces act in the bulk only)
 *   5. pull streaming with periodic wrap (Sec. II A); optional half-way
 *      bounce-back wall at the z seam ("inverting velocities", Sec. II A)
 *   6. evaporation sink (Sec. II C): component A is reset to f^eq(rho_H, 0),
 *      component B to f^eq(rhoA_pre + rhoB_pre - rho_H, 0), where the "pre"
 *      densities are those streamed in during this step; the evaporated mass
 *      E accumulates rhoA_pre - rho_H.
 *
 * Readings of points the paper leaves open (each is listed with its reason in
 * the design notes of the repository):
 *   - direction order: 0 rest, 1-6 = +-x, +-y, +-z, 7-18 the twelve face
 *     diagonals with opposites adjacent (the paper fixes only the weights);
 *   - the seam wall mirrors psi across the seam (psi(z=-1) := psi(z=0)), so
 *     a wall next to a uniform fluid exerts no force (neutral wetting);
 *   - a solid wall (Sec. III A, III B: "a wall of thickness 2 with simple
 *     bounce back") is a layer of solid nodes: every population a fluid node
 *     would pull from a solid node is its own reflected one (half-way
 *     bounce-back); solid nodes hold no fluid and enter the force of Eq. (sc)
 *     with psi of given wall densities (0: no interaction with the wall);
 *   - at rho^c = 0 the force shift is taken as zero (f^eq is then zero for
 *     any finite velocity);
 *   - a sink switched on mid-run is skipped by the next collision and resets
 *     its nodes at the end of that step;
 *   - the single-component multiphase form (Sec. I: the method carries over to
 *     "the multiphase pseudopotential method"): one component whose force of
 *     Eq. (sc) takes itself as the partner with the coupling g (negative for
 *     attraction); the evaporation boundary holds it at rho_H with zero
 *     velocity, and with no partner to take the difference the removed mass
 *     leaves the system and is booked as E (Sec. II C: the model extends to
 *     situations where mass is not conserved).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19

/* D3Q19 lattice velocities e_i (Sec. II A). */
static const int EX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

enum { ORC_PSI_RHO = 0, ORC_PSI_EXP = 1 };
enum { ORC_SINK_NONE = 0, ORC_SINK_ZMAX = 1, ORC_SINK_FACES = 2, ORC_SINK_SPHERE = 3 };

typedef struct {
    int nx, ny, nz;
    int wall_z;        /* 1: bounce-back wall at the z seam (below z = 0) */
    double tau[2];     /* relaxation times tau^A, tau^B */
    double g;          /* g^{AB} = g^{BA} */
    int psi_kind;      /* ORC_PSI_RHO or ORC_PSI_EXP */
    int sink_kind;     /* ORC_SINK_* */
    double rho_h;      /* density imposed on component A at sink nodes */
    double sink_radius;
    double center[3];
    double phi_delta[2]; /* (rhoA - rhoB) inside / outside a droplet */
    int solid_z;       /* solid wall nodes at z = 0 .. solid_z - 1 (0: none) */
    double wall_rho[2];  /* densities whose psi the solid nodes carry */
    int ncomp;         /* components: 2 (also 0) or 1 (single-component multiphase) */
} orc_params;

typedef struct {
    long long step;
    double mass[2];
    double evaporated;
    double evap_rate;
    double momentum[3];
    double z_interface;
    double r_droplet;
    long long nonfinite;
    long long nonpositive;
} orc_diag;

typedef struct {
    orc_params p;
    long long n;      /* nodes */
    double *f;        /* S(t): f[(c*NQ + i)*n + node] */
    double *fs;       /* post-collision populations f* */
    double *rho;      /* rho[c*n + node] */
    double *psi;      /* psi[c*n + node] */
    double *flux;     /* per-node sink flux of the last reset (NaN: no sink node) */
    double evaporated;
    double evap_rate;
    long long step;
} orc_lattice;

/* ---- lattice constants ------------------------------------------------- */

/* Weight w_i from |e_i|^2: 1/3, 1/18, 1/36 (Sec. II A, after Eq. (eqdis)). */
static double weight(int i)
{
    int e2 = EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i];
    if (e2 == 0) return 1.0 / 3.0;
    if (e2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* The direction j with e_j = -e_i, found by search. */
static int opposite(int i)
{
    for (int j = 0; j < NQ; ++j)
        if (EX[j] == -EX[i] && EY[j] == -EY[i] && EZ[j] == -EZ[i]) return j;
    return -1;
}

void orc_lattice_tables(int *ex, int *ey, int *ez, double *w, int *opp)
{
    for (int i = 0; i < NQ; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        ez[i] = EZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Second-order equilibrium, Eq. (eqdis), with c_s^2 = 1/3. */
static double feq(int i, double rho, double ux, double uy, double uz)
{
    const double cs2 = 1.0 / 3.0;
    double eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
    double uu = ux * ux + uy * uy + uz * uz;
    return weight(i) * rho * (1.0 + eu / cs2 - uu / (2.0 * cs2) + eu * eu / (2.0 * cs2 * cs2));
}

void orc_feq(double rho, double ux, double uy, double uz, double *out19)
{
    for (int i = 0; i < NQ; ++i) out19[i] = feq(i, rho, ux, uy, uz);
}

/* Effective mass, Eq. (psifunc) with rho_0 = 1, or psi = rho. */
static double psi_of(const orc_params *p, double rho)
{
    if (p->psi_kind == ORC_PSI_EXP) return 1.0 - exp(-rho);
    return rho;
}

/* ---- geometry ------------------------------------------------------------ */

static long long node_index(const orc_lattice *L, int x, int y, int z)
{
    return ((long long)z * L->p.ny + y) * L->p.nx + x;
}

/* Periodic wrap of a coordinate one step outside [0, n) (every caller steps
 * by at most one node). */
static int wrap(int a, int n)
{
    if (a < 0) return a + n;
    if (a >= n) return a - n;
    return a;
}

static int is_sink(const orc_params *p, int x, int y, int z)
{
    switch (p->sink_kind) {
    case ORC_SINK_ZMAX:
        return z == p->nz - 1;
    case ORC_SINK_FACES:
        return x == 0 || y == 0 || z == 0 || x == p->nx - 1 || y == p->ny - 1 || z == p->nz - 1;
    case ORC_SINK_SPHERE: {
        double dx = x - p->center[0], dy = y - p->center[1], dz = z - p->center[2];
        return dx * dx + dy * dy + dz * dz >= p->sink_radius * p->sink_radius;
    }
    default:
        return 0;
    }
}

/* Components stepped: 1 or 2. With one, component 1 stays empty. */
static int ncomp(const orc_params *p) { return p->ncomp == 1 ? 1 : 2; }

/* The partner in the force of Eq. (sc): the other component, or with one
 * component the component itself. */
static int partner(const orc_params *p, int c) { return ncomp(p) == 1 ? c : 1 - c; }

/* Solid wall node (the layer z < solid_z). */
static int is_solid(const orc_params *p, int z) { return z < p->solid_z; }

/* ---- lifecycle ----------------------------------------------------------- */

orc_lattice *orc_create(const orc_params *p)
{
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return NULL;
    if (p->solid_z < 0 || p->solid_z >= p->nz || (p->solid_z > 0 && p->wall_z)) return NULL;
    if (p->ncomp != 0 && p->ncomp != 1 && p->ncomp != 2) return NULL;
    orc_lattice *L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    if (!L) return NULL;
    L->p = *p;
    L->n = (long long)p->nx * p->ny * p->nz;
    L->f = (double *)calloc((size_t)(2 * NQ * L->n), sizeof(double));
    L->fs = (double *)calloc((size_t)(2 * NQ * L->n), sizeof(double));
    L->rho = (double *)calloc((size_t)(2 * L->n), sizeof(double));
    L->psi = (double *)calloc((size_t)(2 * L->n), sizeof(double));
    L->flux = (double *)calloc((size_t)L->n, sizeof(double));
    if (!L->f || !L->fs || !L->rho || !L->psi || !L->flux) {
        free(L->f); free(L->fs); free(L->rho); free(L->psi); free(L->flux); free(L);
        return NULL;
    }
    return L;
}

void orc_destroy(orc_lattice *L)
{
    if (!L) return;
    free(L->f); free(L->fs); free(L->rho); free(L->psi); free(L->flux);
    free(L);
}

/* ---- the sink (Sec. II C) ------------------------------------------------ */

/* Resets every sink node of the post-stream state in L->f and returns
 * sum over sink nodes of (rhoA_pre - rho_H), summed serially in node order.
 * The per-node resets are independent and run in parallel; each node's
 * flux is kept in L->flux (NaN at nodes outside the sink) for the sum. */
static double apply_sink(orc_lattice *L)
{
    const orc_params *p = &L->p;
    const long long n = L->n;
    double flux = 0.0;
    if (p->sink_kind == ORC_SINK_NONE) return 0.0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long long k = node_index(L, x, y, z);
                L->flux[k] = NAN;
                if (!is_sink(p, x, y, z) || is_solid(p, z)) continue;
                double ra = 0.0, rb = 0.0;
                for (int i = 0; i < NQ; ++i) {
                    ra += L->f[(0 * NQ + i) * n + k];
                    rb += L->f[(1 * NQ + i) * n + k];
                }
                double rb_h = ra + rb - p->rho_h;
                for (int i = 0; i < NQ; ++i) {
                    L->f[(0 * NQ + i) * n + k] = feq(i, p->rho_h, 0.0, 0.0, 0.0);
                    if (ncomp(p) == 2) L->f[(1 * NQ + i) * n + k] = feq(i, rb_h, 0.0, 0.0, 0.0);
                }
                L->flux[k] = ra - p->rho_h;
            }
    for (long long k = 0; k < n; ++k)
        if (!isnan(L->flux[k])) flux += L->flux[k];
    return flux;
}

/* ---- initialisation ------------------------------------------------------ */

/* Solid nodes hold no fluid: their populations are zero; so are those of an
 * absent second component. */
static void clear_solid(orc_lattice *L)
{
    const long long n = L->n, plane = (long long)L->p.nx * L->p.ny;
    for (int q = 0; q < 2 * NQ; ++q)
        for (long long k = 0; k < (long long)L->p.solid_z * plane; ++k) L->f[q * n + k] = 0.0;
    if (ncomp(&L->p) == 1)
        for (long long q = NQ * n; q < 2 * NQ * n; ++q) L->f[q] = 0.0;
}

/* f = f^eq(rho, 0) at every node, then the initial sink reset, which is not
 * counted as evaporated mass. */
void orc_init_from_density(orc_lattice *L, const double *rhoA, const double *rhoB)
{
    const long long n = L->n;
    for (long long k = 0; k < n; ++k)
        for (int i = 0; i < NQ; ++i) {
            L->f[(0 * NQ + i) * n + k] = feq(i, rhoA[k], 0.0, 0.0, 0.0);
            L->f[(1 * NQ + i) * n + k] = feq(i, rhoB[k], 0.0, 0.0, 0.0);
        }
    clear_solid(L);
    L->evap_rate = apply_sink(L);
    L->evaporated = 0.0;
    L->step = 0;
}

/* Arbitrary populations f[(c*19 + i)*n + node], then the uncounted reset. */
void orc_init_from_populations(orc_lattice *L, const double *f)
{
    memcpy(L->f, f, sizeof(double) * (size_t)(2 * NQ * L->n));
    clear_solid(L);
    L->evap_rate = apply_sink(L);
    L->evaporated = 0.0;
    L->step = 0;
}

void orc_set_sink(orc_lattice *L, int kind, double rho_h, double radius)
{
    L->p.sink_kind = kind;
    L->p.rho_h = rho_h;
    L->p.sink_radius = radius;
}

/* ---- moments and force --------------------------------------------------- */

/* Densities and psi at every node; solid nodes carry psi(wall_rho[c]). */
static void compute_density_psi(orc_lattice *L)
{
    const long long n = L->n, solid_end = (long long)L->p.solid_z * L->p.nx * L->p.ny;
#pragma omp parallel for schedule(static)
    for (long long k = 0; k < n; ++k)
        for (int c = 0; c < 2; ++c) {
            double r = 0.0;
            for (int i = 0; i < NQ; ++i) r += L->f[(c * NQ + i) * n + k];
            L->rho[c * n + k] = r;
            L->psi[c * n + k] = k < solid_end ? psi_of(&L->p, L->p.wall_rho[c]) : psi_of(&L->p, r);
        }
}

/* psi of component c at the neighbour (x,y,z) + e_i: periodic wrap, or the
 * mirror psi(z=-1) := psi(z=0) across a wall at the z seam. */
static double psi_neighbour(const orc_lattice *L, int c, int x, int y, int z, int i)
{
    int xn = wrap(x + EX[i], L->p.nx);
    int yn = wrap(y + EY[i], L->p.ny);
    int zn = z + EZ[i];
    if (zn < 0 || zn >= L->p.nz) zn = L->p.wall_z ? z : wrap(zn, L->p.nz);
    return L->psi[c * L->n + node_index(L, xn, yn, zn)];
}

/* Eq. (sc) with one partner component: F^c = -psi^c g sum_i w_i psi^cbar e_i. */
static void sc_force(const orc_lattice *L, int c, int x, int y, int z, double F[3])
{
    int cb = partner(&L->p, c);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = 1; i < NQ; ++i) {
        double ps = psi_neighbour(L, cb, x, y, z, i);
        sx += weight(i) * ps * EX[i];
        sy += weight(i) * ps * EY[i];
        sz += weight(i) * ps * EZ[i];
    }
    double pc = L->psi[c * L->n + node_index(L, x, y, z)];
    F[0] = -pc * L->p.g * sx;
    F[1] = -pc * L->p.g * sy;
    F[2] = -pc * L->p.g * sz;
}

static void momentum_of(const orc_lattice *L, int c, long long k, double j[3])
{
    j[0] = j[1] = j[2] = 0.0;
    for (int i = 0; i < NQ; ++i) {
        double fi = L->f[(c * NQ + i) * L->n + k];
        j[0] += fi * EX[i];
        j[1] += fi * EY[i];
        j[2] += fi * EZ[i];
    }
}

/* ---- one time step ------------------------------------------------------- */

static void collide(orc_lattice *L)
{
    const orc_params *p = &L->p;
    const long long n = L->n;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long long k = node_index(L, x, y, z);
                if (is_solid(p, z)) {
                    for (int q = 0; q < 2 * NQ; ++q) L->fs[q * n + k] = 0.0;
                    continue;
                }
                if (is_sink(p, x, y, z)) {
                    for (int q = 0; q < 2 * NQ; ++q) L->fs[q * n + k] = L->f[q * n + k];
                    continue;
                }
                const int nc = ncomp(p);
                double rho[2] = {0.0, 0.0}, j[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}}, F[2][3];
                for (int c = 0; c < nc; ++c) {
                    rho[c] = L->rho[c * n + k];
                    momentum_of(L, c, k, j[c]);
                    sc_force(L, c, x, y, z, F[c]);
                }
                /* u' = sum_c rho^c u^c / sum_c rho^c = sum_c j^c / sum_c rho^c */
                double rt = rho[0] + rho[1];
                double up[3];
                for (int d = 0; d < 3; ++d) up[d] = (j[0][d] + j[1][d]) / rt;
                for (int q = nc * NQ; q < 2 * NQ; ++q) L->fs[q * n + k] = 0.0;
                for (int c = 0; c < nc; ++c) {
                    double u[3];
                    for (int d = 0; d < 3; ++d)
                        u[d] = up[d] + (rho[c] != 0.0 ? p->tau[c] * F[c][d] / rho[c] : 0.0);
                    for (int i = 0; i < NQ; ++i) {
                        double fi = L->f[(c * NQ + i) * n + k];
                        double fe = feq(i, rho[c], u[0], u[1], u[2]);
                        L->fs[(c * NQ + i) * n + k] = fi - (fi - fe) / p->tau[c];
                    }
                }
            }
}

/* Pull streaming, one (component, direction) plane at a time. A population
 * that would come across the seam wall or out of a solid node is the node's
 * own reflected one; solid nodes stay empty. */
static void stream(orc_lattice *L)
{
    const orc_params *p = &L->p;
    const long long n = L->n;
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < NQ; ++i) {
            const int io = opposite(i);
#pragma omp parallel for schedule(static)
            for (int z = 0; z < p->nz; ++z) {
                int zs = z - EZ[i];
                int across_wall = p->wall_z && (zs < 0 || zs >= p->nz);
                int from_solid = !p->wall_z && is_solid(p, wrap(zs, p->nz));
                for (int y = 0; y < p->ny; ++y)
                    for (int x = 0; x < p->nx; ++x) {
                        long long k = node_index(L, x, y, z);
                        double v;
                        if (is_solid(p, z)) {
                            v = 0.0;
                        } else if (across_wall || from_solid) {
                            v = L->fs[(c * NQ + io) * n + k];
                        } else {
                            long long ks = node_index(L, wrap(x - EX[i], p->nx), wrap(y - EY[i], p->ny),
                                                      wrap(zs, p->nz));
                            v = L->fs[(c * NQ + i) * n + ks];
                        }
                        L->f[(c * NQ + i) * n + k] = v;
                    }
            }
        }
}

void orc_step(orc_lattice *L, long long nsteps)
{
    for (long long s = 0; s < nsteps; ++s) {
        compute_density_psi(L);
        collide(L);
        stream(L);
        double flux = apply_sink(L);
        L->evap_rate = flux;
        L->evaporated += flux;
        L->step += 1;
    }
}

/* ---- read-outs ----------------------------------------------------------- */

void orc_get_populations(const orc_lattice *L, double *out)
{
    memcpy(out, L->f, sizeof(double) * (size_t)(2 * NQ * L->n));
}

void orc_get_density(orc_lattice *L, double *rhoA, double *rhoB)
{
    compute_density_psi(L);
    memcpy(rhoA, L->rho, sizeof(double) * (size_t)L->n);
    memcpy(rhoB, L->rho + L->n, sizeof(double) * (size_t)L->n);
}

/* Barycentric velocity U of Eq. (velw):
 * U = (sum_c rho^c u^c + (F^A + F^B)/2) / (rho^A + rho^B); no force acts at
 * sink nodes; solid nodes have U = 0.  out3[d*n + node]. */
void orc_get_velocity(orc_lattice *L, double *out3)
{
    const orc_params *p = &L->p;
    const long long n = L->n;
    compute_density_psi(L);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long long k = node_index(L, x, y, z);
                double num[3] = {0.0, 0.0, 0.0};
                if (is_solid(p, z)) {
                    for (int d = 0; d < 3; ++d) out3[d * n + k] = 0.0;
                    continue;
                }
                for (int c = 0; c < ncomp(p); ++c) {
                    double j[3], F[3] = {0.0, 0.0, 0.0};
                    momentum_of(L, c, k, j);
                    if (!is_sink(p, x, y, z)) sc_force(L, c, x, y, z, F);
                    for (int d = 0; d < 3; ++d) num[d] += j[d] + 0.5 * F[d];
                }
                double rt = L->rho[k] + L->rho[n + k];
                for (int d = 0; d < 3; ++d) out3[d * n + k] = num[d] / rt;
            }
}

/* Total Shan-Chen force summed over all fluid nodes and both components. */
void orc_total_force(orc_lattice *L, double out[3])
{
    const orc_params *p = &L->p;
    compute_density_psi(L);
    out[0] = out[1] = out[2] = 0.0;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int c = 0; c < ncomp(p); ++c) {
                    double F[3];
                    if (is_solid(p, z)) continue;
                    sc_force(L, c, x, y, z, F);
                    for (int d = 0; d < 3; ++d) out[d] += F[d];
                }
}

/* Mass, evaporated mass, momentum, interface height and droplet radius, over
 * the fluid nodes. */
void orc_diagnostics(orc_lattice *L, orc_diag *out)
{
    const orc_params *p = &L->p;
    const long long n = L->n;
    compute_density_psi(L);
    memset(out, 0, sizeof(*out));
    out->step = L->step;
    out->evaporated = L->evaporated;
    out->evap_rate = L->evap_rate;
    double *prof = (double *)calloc((size_t)p->nz, sizeof(double));
    double phisum = 0.0;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long long k = node_index(L, x, y, z);
                if (is_solid(p, z)) continue;
                double ra = L->rho[k], rb = L->rho[n + k];
                out->mass[0] += ra;
                out->mass[1] += rb;
                for (int c = 0; c < 2; ++c) {
                    double j[3];
                    momentum_of(L, c, k, j);
                    for (int d = 0; d < 3; ++d) out->momentum[d] += j[d];
                }
                if (!isfinite(ra) || !isfinite(rb)) out->nonfinite += 1;
                if (ra <= 0.0 || (ncomp(p) == 2 && rb <= 0.0)) out->nonpositive += 1;
                /* the order parameter: rhoA - rhoB, or with one component its
                 * density, against the midpoint of the two phases */
                double q = ncomp(p) == 2 ? ra - rb : ra;
                prof[z] += ncomp(p) == 2 ? q : q - 0.5 * (p->phi_delta[0] + p->phi_delta[1]);
                double phi = (q - p->phi_delta[1]) / (p->phi_delta[0] - p->phi_delta[1]);
                if (phi < 0.0) phi = 0.0;
                if (phi > 1.0) phi = 1.0;
                phisum += phi;
            }
    /* Interface: first sign change of the plane-averaged order parameter
     * (rhoA - rhoB, or one component's density minus the midpoint of its
     * phases) scanning up from the lowest fluid plane, located by linear
     * interpolation. */
    out->z_interface = NAN;
    double area = (double)p->nx * p->ny;
    for (int z = p->solid_z; z + 1 < p->nz; ++z) {
        double a = prof[z] / area, b = prof[z + 1] / area;
        if ((a > 0.0 && b <= 0.0) || (a < 0.0 && b >= 0.0)) {
            out->z_interface = z + a / (a - b);
            break;
        }
    }
    out->r_droplet = cbrt(3.0 * phisum / (4.0 * M_PI));
    free(prof);
}

double orc_evaporated(const orc_lattice *L) { return L->evaporated; }
long long orc_step_count(const orc_lattice *L) { return L->step; }

/* Threads the per-node loops use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of the per-node loops (results do not depend on it). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
