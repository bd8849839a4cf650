/*
 * fsl_oracle.c -- plain, slow, FP64 CPU oracle of the free-surface lattice
 * Boltzmann step for liquid-gas-solid flow (Bogner, Harting & Ruede 2017).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product library.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * The step follows the paper's method section in its own order:
 *   1. streaming, Eq. (LBE1), with the missing populations reconstructed by
 *      half-way bounce-back at box walls, by the moving-wall bounce-back rule
 *      Eq. (bbrule) at particle links and by the free-surface condition Eq. (fsk)
 *      at gas links; momentum exchange Eqs. (netforce), (torque),
 *      (momentum_transfer) at particle links, at links from nodes of another
 *      particle and (a reading) at links from beyond the box faces, and at the
 *      no-slip faces themselves (the plate force);
 *   2. moments (Sec. 2.1), with the Guo half-force shift of the velocity;
 *   3. interface mass exchange Eqs. (massExchange), (massExchangeb);
 *   4. TRT collision Eq. (LBE2) with the equilibrium Eq. (equilibrium) and the
 *      magic parameterisation of Sec. 2.1;
 *   5. cell conversions of Fig. (cellConversions) with the closure of the
 *      interface layer, equilibrium initialisation of new interface cells and
 *      excess-mass redistribution;
 *   6. particle update: lubrication correction Eq. (lubrication) between
 *      spheres and (a reading) at no-slip faces, a contact spring (a reading),
 *      and up to ten substeps per lattice step (Sec. 2.3), then the
 *      obstacle-coverage update;
 *   7. bubble model (end of Sec. 2.2): per-bubble volume, constant gas mass,
 *      gas density = mass / volume; a bubble whose gas falls apart splits.
 * Where the paper is silent the reading used is stated at the place it is used.
 * Parity-pinned parts are listed in the tests; the conversion rules (reading
 * of the fill thresholds, conflict rule, G->I initial state, excess split), the
 * bubble merge and the cover/uncover bookkeeping next to gas are "parity
 * unpinned" beyond conservation and the invariants checked in the tests (the
 * cover/uncover bookkeeping in liquid is pinned on a closed form).
 *
 * Build: cc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no intrinsics).
 */
#define _GNU_SOURCE
#include "fsl_oracle.h"

#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- D3Q19 velocity set (Sec. 2.1), typed out for the oracle ---------------- */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static double W[19];
static int OPP[19];

static void init_lattice_tables(void)
{
    for (int q = 0; q < 19; ++q) {
        int n2 = CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q];
        W[q] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        for (int p = 0; p < 19; ++p)
            if (CX[p] == -CX[q] && CY[p] == -CY[q] && CZ[p] == -CZ[q]) OPP[q] = p;
    }
}

enum { GAS = 0, LIQ = 1, IFC = 2, SOL = 3 };
enum { ERR_LG = 1u, ERR_NAN = 2u, ERR_CAP = 4u, ERR_VOL = 8u, ERR_ARG = 16u, ERR_PART = 32u };
enum { CV_NONE = 0, CV_F = 1, CV_E0 = 2, CV_E = 3, CV_NEWG = 4, CV_NEWL = 5 };

struct orc_ctx {
    orc_config cfg;
    int nx, ny, nz, N;
    double lp, lm;          /* lambda_plus, lambda_minus */
    uint8_t *flag;
    double *f, *fn;         /* post-collision state at t, work/next state */
    double *rho_new, *u_new;/* collision moments of the last step [N], [3][N] */
    double *m, *phi, *phi_new;
    int *bub, *pid, *claim;
    uint8_t *conv;
    double ledger;
    uint32_t err;
    /* particles */
    int np;
    double *px, *pu, *pw, *pR, *prho, *pF, *pT, *pFp, *pTp;
    int have_prev;          /* a previous step's force exists */
    double wallF[18];       /* force on each no-slip face [2 axis + side][comp], last step */
    double wallP[18];       /* the part of it from links into particle nodes (force_pass) */
    /* bubbles */
    int nb;
    double *bM, *bV, *bV0, *bcent, *brho;
    int *broot, *balive;
    int64_t *bngas, *bnif;
};

/* ---- small helpers ------------------------------------------------------------ */
static int wrap_or_wall(int v, int n, int periodic)
{
    if (v >= 0 && v < n) return v;
    if (!periodic) return -1;
    v %= n;
    if (v < 0) v += n;
    return v;
}

/* neighbour of cell (i,j,k) displaced by (dx,dy,dz); -1 outside a wall.  The face
 * index of the first non-periodic axis that is left is returned in *face as
 * 2*axis + (0 low / 1 high). */
static int nbr(const orc_ctx *c, int i, int j, int k, int dx, int dy, int dz, int *face)
{
    int a = wrap_or_wall(i + dx, c->nx, c->cfg.periodic[0]);
    int b = wrap_or_wall(j + dy, c->ny, c->cfg.periodic[1]);
    int d = wrap_or_wall(k + dz, c->nz, c->cfg.periodic[2]);
    if (a < 0 || b < 0 || d < 0) {
        if (face) {
            if (a < 0) *face = (i + dx < 0) ? 0 : 1;
            else if (b < 0) *face = (j + dy < 0) ? 2 : 3;
            else *face = (k + dz < 0) ? 4 : 5;
        }
        return -1;
    }
    return a + c->nx * (b + c->ny * d);
}

/* Free-slip faces (specular reflection at the half-way wall).  Reading: a link whose
 * far end lies beyond faces of the box reflects specularly when every face it
 * crosses is free-slip, and bounces back when any of them is no-slip.  The reflected
 * link reaches cell (i,j,k) + d along q from the cell (i,j,k) + d' with the crossed
 * components of d removed, travelling along q with the crossed components reversed.
 * crossed_axes returns the bit set of the non-periodic axes that (i,j,k) + d leaves
 * (bit a for axis a) and whether all of them slip. */
static int crossed_axes(const orc_ctx *c, int i, int j, int k, int dx, int dy, int dz, int *all_slip)
{
    const int v[3] = {i + dx, j + dy, k + dz}, n[3] = {c->nx, c->ny, c->nz};
    int m = 0;
    for (int a = 0; a < 3; ++a)
        if (!c->cfg.periodic[a] && (v[a] < 0 || v[a] >= n[a])) m |= 1 << a;
    int slip = m != 0;
    for (int a = 0; a < 3; ++a)
        if (((m >> a) & 1) && !c->cfg.freeslip[a]) slip = 0;
    *all_slip = slip;
    return m;
}

/* direction q with the components of the axes in m reversed */
static int mirror_dir(int q, int m)
{
    const int e[3] = {(m & 1) ? -CX[q] : CX[q], (m & 2) ? -CY[q] : CY[q], (m & 4) ? -CZ[q] : CZ[q]};
    for (int p = 0; p < 19; ++p)
        if (CX[p] == e[0] && CY[p] == e[1] && CZ[p] == e[2]) return p;
    return q;
}

/* Periodic images of the spheres: along a periodic axis a displacement is taken as
 * its nearest image, in [-n/2, n/2); along a walled axis as it is. */
static double min_image(const orc_ctx *c, int a, double d)
{
    if (!c->cfg.periodic[a]) return d;
    const double n = c->cfg.n[a];
    return d - n * floor(d / n + 0.5);
}

/* a coordinate along a periodic axis taken into [0, n) */
static double wrap_coord(const orc_ctx *c, int a, double v)
{
    if (!c->cfg.periodic[a]) return v;
    const double n = c->cfg.n[a];
    v -= n * floor(v / n);
    return v < n ? v : 0.0; /* v just below 0 can round up to n */
}

static void cell_ijk(const orc_ctx *c, int x, int *i, int *j, int *k)
{
    *i = x % c->nx;
    *j = (x / c->nx) % c->ny;
    *k = x / (c->nx * c->ny);
}

/* Eq. (equilibrium) with c_s^2 = 1/3 */
void orc_equilibrium(double rho, const double u[3], double e[19])
{
    if (W[0] == 0.0) init_lattice_tables();
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < 19; ++q) {
        double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
        e[q] = rho * W[q] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* even part e^+_q(rho,u) */
static double eq_plus(int q, double rho, const double u[3])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
    return rho * W[q] * (1.0 + 4.5 * cu * cu - 1.5 * uu);
}

/* lambda_- from the TRT constraint of Sec. 2.1:
 * (1/lp + 1/2)(1/lm + 1/2) = Lambda with lp = -1/tau */
double orc_lambda_minus(double tau, double magic, int trt)
{
    double lp = -1.0 / tau;
    if (!trt) return lp;
    double a = 1.0 / lp + 0.5;       /* = -(tau - 1/2) */
    double b = magic / a;            /* = 1/lm + 1/2 */
    return 1.0 / (b - 0.5);
}

static int find_root(const orc_ctx *c, int b)
{
    while (c->broot[b] != b) b = c->broot[b];
    return b;
}

/* moments of the stored post-collision populations of cell x: rho and the
 * velocity u = (sum_q c_q f*_q - F/2)/rho with F = rho g.  The collision with
 * the Guo force adds F to the first moment, so this is the velocity of the
 * collision that produced f* (reading: velocity used by Eq. (fsk) and density
 * used by Eq. (bbrule) are these moments of the boundary cell at time t). */
static void post_moments(const orc_ctx *c, const double *f, int x, double *rho, double u[3])
{
    double r = 0, jx = 0, jy = 0, jz = 0;
    for (int q = 0; q < 19; ++q) {
        double v = f[(size_t)q * c->N + x];
        r += v;
        jx += CX[q] * v;
        jy += CY[q] * v;
        jz += CZ[q] * v;
    }
    *rho = r;
    u[0] = jx / r - 0.5 * c->cfg.g[0];
    u[1] = jy / r - 0.5 * c->cfg.g[1];
    u[2] = jz / r - 0.5 * c->cfg.g[2];
}

/* rigid-body velocity of particle P at point p (arm to the nearest image) */
static void rigid_velocity(const orc_ctx *c, int P, const double p[3], double uw[3])
{
    const double *xp = c->px + 3 * P, *up = c->pu + 3 * P, *wp = c->pw + 3 * P;
    double r0 = min_image(c, 0, p[0] - xp[0]), r1 = min_image(c, 1, p[1] - xp[1]), r2 = min_image(c, 2, p[2] - xp[2]);
    uw[0] = up[0] + (wp[1] * r2 - wp[2] * r1);
    uw[1] = up[1] + (wp[2] * r0 - wp[0] * r2);
    uw[2] = up[2] + (wp[0] * r1 - wp[1] * r0);
}

/* Eq. (bbrule) written for the pulled direction q whose source x - c_q is covered
 * by particle P: f_q(x,t+1) = f*_qbar(x,t) + 6 w_q rho_w (c_q . u_w), with u_w the
 * particle surface velocity at the link midpoint x_w = x - c_q/2 and rho_w the
 * density of the fluid node at time t. */
static double bb_particle(const orc_ctx *c, const double *f, int x, int q, int P, double rho_w)
{
    int i, j, k;
    cell_ijk(c, x, &i, &j, &k);
    double xw[3] = {i - 0.5 * CX[q], j - 0.5 * CY[q], k - 0.5 * CZ[q]};
    double uw[3];
    rigid_velocity(c, P, xw, uw);
    double cu = CX[q] * uw[0] + CY[q] * uw[1] + CZ[q] * uw[2];
    return f[(size_t)OPP[q] * c->N + x] + 6.0 * W[q] * rho_w * cu;
}

static double bubble_rho(const orc_ctx *c, int b)
{
    return c->brho[find_root(c, b)];
}

/* ---- creation / destruction --------------------------------------------------- */
static void *xcalloc(size_t n, size_t s)
{
    void *p = calloc(n ? n : 1, s);
    return p;
}

void orc_destroy(orc_ctx *c)
{
    if (!c) return;
    free(c->flag); free(c->f); free(c->fn); free(c->rho_new); free(c->u_new);
    free(c->m); free(c->phi); free(c->phi_new); free(c->bub); free(c->pid); free(c->claim);
    free(c->conv);
    free(c->px); free(c->pu); free(c->pw); free(c->pR); free(c->prho); free(c->pF); free(c->pT); free(c->pFp); free(c->pTp);
    free(c->bM); free(c->bV); free(c->bV0); free(c->bcent); free(c->brho); free(c->broot);
    free(c->balive); free(c->bngas); free(c->bnif);
    free(c);
}

static void bubbles_recompute(orc_ctx *c);
static int split_bubbles(orc_ctx *c);

/* Initial state (reading of the configs; the same specification is implemented
 * independently by the library):
 *  - fill level = fraction of the 8^3 sub-points (offsets (a+1/2)/8 - 1/2) that lie
 *    below the pool height and outside every gas sphere (strict comparisons);
 *  - phi = 1 -> liquid, phi = 0 -> gas, otherwise interface; then every liquid cell
 *    with a gas neighbour becomes interface (closure of the layer, Sec. 2.2);
 *  - bubble id of a gas sub-point: 0 above the pool, else 1 + index of the first
 *    gas sphere holding it; a cell takes the smallest id of its gas sub-points;
 *  - liquid density rho_g0 (1 - 3 g_z (zs - z)) (linear hydrostatic profile), or 1
 *    for a fully liquid box; u = 0; f* = equilibrium; interface mass m = phi rho;
 *  - bubble mass M_b = rho_g(b) V_b(0). */
orc_ctx *orc_create(const orc_config *cfg)
{
    init_lattice_tables();
    orc_ctx *c = (orc_ctx *)xcalloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->cfg = *cfg;
    if (c->cfg.n_sub <= 0) c->cfg.n_sub = 10;
    if (c->cfg.max_bubbles <= 0) c->cfg.max_bubbles = 64;
    if (c->cfg.max_bubbles < cfg->n_gas_spheres + 1) c->cfg.max_bubbles = cfg->n_gas_spheres + 1;
    c->nx = cfg->n[0]; c->ny = cfg->n[1]; c->nz = cfg->n[2];
    c->N = c->nx * c->ny * c->nz;
    c->lp = -1.0 / cfg->tau;
    c->lm = orc_lambda_minus(cfg->tau, cfg->magic, cfg->trt);
    size_t N = (size_t)c->N;
    c->flag = (uint8_t *)xcalloc(N, 1);
    c->f = (double *)xcalloc(19 * N, sizeof(double));
    c->fn = (double *)xcalloc(19 * N, sizeof(double));
    c->rho_new = (double *)xcalloc(N, sizeof(double));
    c->u_new = (double *)xcalloc(3 * N, sizeof(double));
    c->m = (double *)xcalloc(N, sizeof(double));
    c->phi = (double *)xcalloc(N, sizeof(double));
    c->phi_new = (double *)xcalloc(N, sizeof(double));
    c->bub = (int *)xcalloc(N, sizeof(int));
    c->pid = (int *)xcalloc(N, sizeof(int));
    c->claim = (int *)xcalloc(N, sizeof(int));
    c->conv = (uint8_t *)xcalloc(N, 1);
    int mp = cfg->max_particles > 0 ? cfg->max_particles : 1;
    c->px = (double *)xcalloc(3 * mp, sizeof(double));
    c->pu = (double *)xcalloc(3 * mp, sizeof(double));
    c->pw = (double *)xcalloc(3 * mp, sizeof(double));
    c->pF = (double *)xcalloc(3 * mp, sizeof(double));
    c->pT = (double *)xcalloc(3 * mp, sizeof(double));
    c->pFp = (double *)xcalloc(3 * mp, sizeof(double));
    c->pTp = (double *)xcalloc(3 * mp, sizeof(double));
    c->pR = (double *)xcalloc(mp, sizeof(double));
    c->prho = (double *)xcalloc(mp, sizeof(double));
    int MB = c->cfg.max_bubbles;
    c->bM = (double *)xcalloc(MB, sizeof(double));
    c->bV = (double *)xcalloc(MB, sizeof(double));
    c->bV0 = (double *)xcalloc(MB, sizeof(double));
    c->brho = (double *)xcalloc(MB, sizeof(double));
    c->bcent = (double *)xcalloc(3 * MB, sizeof(double));
    c->broot = (int *)xcalloc(MB, sizeof(int));
    c->balive = (int *)xcalloc(MB, sizeof(int));
    c->bngas = (int64_t *)xcalloc(MB, sizeof(int64_t));
    c->bnif = (int64_t *)xcalloc(MB, sizeof(int64_t));
    if (!c->flag || !c->f || !c->fn || !c->rho_new || !c->u_new || !c->m || !c->phi ||
        !c->phi_new || !c->bub || !c->pid || !c->claim || !c->conv || !c->bM || !c->bV) {
        orc_destroy(c);
        return NULL;
    }
    for (int x = 0; x < c->N; ++x) c->pid[x] = -1;

    const double zs = cfg->zs;
    const int full = zs < 0.0;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                int x = i + c->nx * (j + c->ny * k);
                int nliq = 0, gid = 1 << 30;
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b)
                        for (int d = 0; d < 8; ++d) {
                            double p0 = i + (2 * a + 1 - 8) / 16.0;
                            double p1 = j + (2 * b + 1 - 8) / 16.0;
                            double p2 = k + (2 * d + 1 - 8) / 16.0;
                            int below = full || p2 < zs;
                            int id = below ? -1 : 0;
                            for (int s = 0; s < cfg->n_gas_spheres && id < 0; ++s) {
                                const double *S = cfg->gas_spheres[s];
                                double d0 = p0 - S[0], d1 = p1 - S[1], d2 = p2 - S[2];
                                if ((d0 * d0 + d1 * d1) + d2 * d2 < S[3] * S[3]) id = s + 1;
                            }
                            if (id < 0) ++nliq;
                            else if (id < gid) gid = id;
                        }
                double phi = nliq / 512.0;
                c->phi[x] = phi;
                c->flag[x] = nliq == 512 ? LIQ : (nliq == 0 ? GAS : IFC);
                c->bub[x] = nliq == 512 ? 0 : gid;
            }
    /* closure: liquid cells next to gas become interface */
    for (int x = 0; x < c->N; ++x) c->conv[x] = 0;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                int x = i + c->nx * (j + c->ny * k);
                if (c->flag[x] != LIQ) continue;
                for (int q = 1; q < 19; ++q) {
                    int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                    if (n >= 0 && c->flag[n] == GAS) {
                        c->conv[x] = 1;
                        c->bub[x] = c->bub[n];
                        break;
                    }
                }
            }
    for (int x = 0; x < c->N; ++x)
        if (c->conv[x]) { c->flag[x] = IFC; c->conv[x] = 0; }
    /* hydrostatic density and equilibrium populations */
    for (int x = 0; x < c->N; ++x) {
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        if (c->flag[x] == LIQ || c->flag[x] == IFC) {
            double rho = full ? 1.0 : cfg->rho_g0 * (1.0 - 3.0 * cfg->g[2] * (zs - k));
            double u0[3] = {0, 0, 0}, e[19];
            orc_equilibrium(rho, u0, e);
            for (int q = 0; q < 19; ++q) c->f[(size_t)q * N + x] = e[q];
            c->rho_new[x] = rho;
            if (c->flag[x] == IFC) c->m[x] = c->phi[x] * rho;
            else c->phi[x] = 1.0;
        }
    }
    /* bubbles */
    c->nb = cfg->n_gas_spheres + 1;
    for (int b = 0; b < c->nb; ++b) {
        c->broot[b] = b;
        c->balive[b] = 1;
        c->brho[b] = (b == 0) ? cfg->rho_g0 : cfg->gas_spheres[b - 1][4];
    }
    c->bM[0] = 0;
    bubbles_recompute(c);
    for (int b = 0; b < c->nb; ++b) {
        double rg = (b == 0) ? cfg->rho_g0 : cfg->gas_spheres[b - 1][4];
        c->bV0[b] = c->bV[b];
        c->bM[b] = rg * c->bV[b];
        c->balive[b] = c->bV[b] > 0.0;
        c->brho[b] = rg;
    }
    bubbles_recompute(c);
    split_bubbles(c);
    return c;
}

int orc_num_cells(const orc_ctx *c) { return c->N; }
uint32_t orc_error(const orc_ctx *c) { return c->err; }

/* ---- bubble model (end of Sec. 2.2) -------------------------------------------
 * Reading: isothermal ideal gas per bubble, M_b = rho_b V_b constant; the volume is
 * the number of gas cells plus the gas fraction (1 - phi) of interface cells that
 * carry the bubble's id; bubbles merged earlier are looked up through their root. */
static void bubbles_recompute(orc_ctx *c)
{
    for (int b = 0; b < c->nb; ++b) {
        c->bV[b] = 0;
        c->bngas[b] = 0;
        c->bnif[b] = 0;
        c->bcent[3 * b] = c->bcent[3 * b + 1] = c->bcent[3 * b + 2] = 0;
    }
    for (int x = 0; x < c->N; ++x) {
        int fl = c->flag[x];
        if (fl != GAS && fl != IFC) continue;
        int b = find_root(c, c->bub[x]);
        double w = (fl == GAS) ? 1.0 : 1.0 - c->phi[x];
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        c->bV[b] += w;
        c->bcent[3 * b] += w * i;
        c->bcent[3 * b + 1] += w * j;
        c->bcent[3 * b + 2] += w * k;
        if (fl == GAS) c->bngas[b]++;
        else c->bnif[b]++;
    }
    for (int b = 0; b < c->nb; ++b) {
        if (c->broot[b] != b || !c->balive[b]) continue;
        if (b == 0 && c->cfg.open_atmosphere) {
            /* pressure outlet (reading): the gas above the pool keeps rho_g0 and its
             * mass follows its volume */
            c->brho[0] = c->cfg.rho_g0;
            c->bM[0] = c->cfg.rho_g0 * c->bV[0];
            if (c->bV[0] > 0.0)
                for (int a = 0; a < 3; ++a) c->bcent[a] /= c->bV[0];
            continue;
        }
        if (c->bV[b] > 0.0) {
            c->brho[b] = c->bM[b] / c->bV[b];
            for (int a = 0; a < 3; ++a) c->bcent[3 * b + a] /= c->bV[b];
        } else if (c->bM[b] > 0.0) {
            /* reading: a bubble whose gas volume has vanished no longer exists; its
             * gas mass leaves the system (the liquid mass ledger is not involved) */
            c->balive[b] = 0;
            c->bM[b] = 0.0;
        }
    }
}

/* ---- bubble splitting (bubble model, end of Sec. 2.2) ----------------------------
 * A bubble is a connected region of gas.  Readings: two gas cells are connected when
 * they are D3Q19 neighbours (the neighbourhood of the merge rule) and belong to the
 * same root bubble.  When the gas cells of a root fall into several components, the
 * component holding the lowest cell index keeps the bubble; every other component,
 * in order of its lowest cell index, becomes a bubble with the lowest id that is not
 * alive (never used, or merged away: merges relabel the cells to their root).  An
 * interface cell of the root goes with the component of its gas neighbours of that
 * root (the one with the lowest cell index if they differ); one without such a
 * neighbour stays with the bubble.  The gas mass is shared in proportion to the
 * volumes of the parts (gas cells plus 1 - phi of their interface cells), so every
 * part starts at the density of the bubble it came from.  The volumes of the
 * bubble table must be those of the current state.  Returns the number of new
 * bubbles; a full table sets ERR_CAP and stops. */
static int split_bubbles(orc_ctx *c)
{
    const int N = c->N, MB = c->cfg.max_bubbles;
    int *lab = (int *)xcalloc((size_t)N, sizeof(int));   /* lowest cell index of the component */
    int *nid = (int *)xcalloc((size_t)N, sizeof(int));   /* per component (at that cell): new id or -1 */
    int *stack = (int *)xcalloc((size_t)N, sizeof(int));
    int *newb = (int *)xcalloc((size_t)N, sizeof(int));  /* per cell: new id or -1 */
    int *parent = (int *)xcalloc((size_t)MB, sizeof(int));
    double *Vn = (double *)xcalloc((size_t)MB, sizeof(double));
    unsigned char *seen = (unsigned char *)xcalloc((size_t)MB, 1);
    unsigned char *isnew = (unsigned char *)xcalloc((size_t)MB, 1);  /* ids taken by this split */
    int created = 0;
    for (int x = 0; x < N; ++x) lab[x] = nid[x] = newb[x] = -1;
    /* components: flood fill from the lowest unlabelled gas cell */
    for (int x = 0; x < N; ++x) {
        if (c->flag[x] != GAS || lab[x] >= 0) continue;
        const int r = find_root(c, c->bub[x]);
        int top = 0;
        stack[top++] = x;
        lab[x] = x;
        while (top) {
            int y = stack[--top], i, j, k;
            cell_ijk(c, y, &i, &j, &k);
            for (int q = 1; q < 19; ++q) {
                int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                if (n < 0 || c->flag[n] != GAS || lab[n] >= 0 || find_root(c, c->bub[n]) != r) continue;
                lab[n] = x;
                stack[top++] = n;
            }
        }
    }
    /* the first component of each root keeps it; the others take new ids */
    for (int x = 0; x < N; ++x) {
        if (lab[x] != x) continue;
        const int r = find_root(c, c->bub[x]);
        if (r == 0 && c->cfg.open_atmosphere) continue;  /* every part stays at the outlet */
        if (!seen[r]) {
            seen[r] = 1;
            continue;
        }
        /* the lowest id that is not alive: never used, or merged away */
        int b = 1;
        while (b < MB && (c->balive[b] || isnew[b])) ++b;
        if (b >= MB) {
            c->err |= ERR_CAP;
            break;
        }
        nid[x] = b;
        isnew[b] = 1;
        if (b >= c->nb) c->nb = b + 1;
        parent[b] = r;
        ++created;
    }
    if (created) {
        /* interface cells first: they look at the ids of their gas neighbours */
        for (int x = 0; x < N; ++x) {
            if (c->flag[x] != IFC) continue;
            const int r = find_root(c, c->bub[x]);
            int best = -1, i, j, k;
            cell_ijk(c, x, &i, &j, &k);
            for (int q = 1; q < 19; ++q) {
                int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                if (n < 0 || c->flag[n] != GAS || find_root(c, c->bub[n]) != r) continue;
                if (best < 0 || lab[n] < best) best = lab[n];
            }
            if (best >= 0 && nid[best] >= 0) {
                newb[x] = nid[best];
                Vn[nid[best]] += 1.0 - c->phi[x];
            }
        }
        for (int x = 0; x < N; ++x) {
            if (c->flag[x] != GAS || nid[lab[x]] < 0) continue;
            newb[x] = nid[lab[x]];
            Vn[newb[x]] += 1.0;
        }
        for (int x = 0; x < N; ++x)
            if (newb[x] >= 0) c->bub[x] = newb[x];
        /* masses: each new part at the density of its bubble (new ids in increasing
         * order, which is the order of the parts) */
        for (int r = 0; r < MB; ++r) {
            if (!seen[r]) continue;
            const double Mr = c->bM[r];
            double taken = 0.0;
            for (int b = 1; b < MB; ++b) {
                if (!isnew[b] || parent[b] != r) continue;
                c->bM[b] = Mr * Vn[b] / c->bV[r];
                c->bV0[b] = Vn[b];
                c->broot[b] = b;
                c->balive[b] = 1;
                taken += c->bM[b];
            }
            c->bM[r] = Mr - taken;
        }
        bubbles_recompute(c);
    }
    free(lab);
    free(nid);
    free(stack);
    free(newb);
    free(parent);
    free(Vn);
    free(seen);
    free(isnew);
    return created;
}

int orc_split(orc_ctx *c)
{
    int n = split_bubbles(c);
    return (c->err & ERR_CAP) ? -1 : n;
}

/* ---- coverage update (Sec. 2.3: nodes inside a particle are obstacle nodes) ----
 * Readings: a node is inside P iff ((dx*dx + dy*dy) + dz*dz) <= R*R in FP64; when
 * two particles cover a node the lower index owns it.  Covered fluid cells hand
 * their mass (rho for liquid, m for interface) to the ledger.  An uncovered node
 * takes f* = e(rho_bar, u_rigid), rho_bar = mean density of its liquid/interface
 * neighbours (pre-uncover flags, not counting nodes uncovered in the same pass),
 * 1 if there are none; it becomes liquid if it has a liquid/interface neighbour
 * and no gas neighbour, interface (m = rho_bar, id of the first gas neighbour) if
 * it has both, gas if it has only gas neighbours and liquid otherwise; the
 * ledger pays rho_bar for liquid and interface.  A final closure turns uncovered
 * liquid cells that touch gas into interface cells. */
static void coverage_update(orc_ctx *c)
{
    const size_t N = (size_t)c->N;
    for (int x = 0; x < c->N; ++x) c->claim[x] = -1;
    for (int P = 0; P < c->np; ++P) {
        const double *xp = c->px + 3 * P;
        double R = c->pR[P];
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int)floor(xp[a] - R);
            hi[a] = (int)ceil(xp[a] + R);
            if (c->cfg.periodic[a]) continue; /* nodes of the images across the faces */
            if (lo[a] < 0) lo[a] = 0;
            if (hi[a] > c->cfg.n[a] - 1) hi[a] = c->cfg.n[a] - 1;
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    double d0 = i - xp[0], d1 = j - xp[1], d2 = k - xp[2];
                    if ((d0 * d0 + d1 * d1) + d2 * d2 <= R * R) {
                        int x = wrap_or_wall(i, c->nx, 1) + c->nx * (wrap_or_wall(j, c->ny, 1) + c->ny * wrap_or_wall(k, c->nz, 1));
                        if (c->claim[x] < 0) c->claim[x] = P;
                    }
                }
    }
    /* covers and owner transfers */
    int n_unc = 0;
    for (int x = 0; x < c->N; ++x) {
        int cl = c->claim[x];
        if (c->flag[x] == SOL) {
            if (cl >= 0) c->pid[x] = cl;
            else { c->conv[x] = 1; ++n_unc; }
            continue;
        }
        if (cl < 0) continue;
        if (c->flag[x] == LIQ) {
            double r = 0;
            for (int q = 0; q < 19; ++q) r += c->f[(size_t)q * N + x];
            c->ledger += r;
        } else if (c->flag[x] == IFC) {
            c->ledger += c->m[x];
        }
        c->flag[x] = SOL;
        c->pid[x] = cl;
        c->phi[x] = 0;
    }
    if (!n_unc) return;
    /* uncovers: decide with the flags as they are now (uncovered nodes are still SOL) */
    int *dec = (int *)calloc((size_t)n_unc, sizeof(int) * 3);
    double *drho = (double *)calloc((size_t)n_unc, sizeof(double));
    int *ux = (int *)calloc((size_t)n_unc, sizeof(int));
    int u = 0;
    for (int x = 0; x < c->N; ++x) {
        if (!c->conv[x]) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        int nli = 0, gfirst = -1;
        double rs = 0;
        for (int q = 1; q < 19; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n < 0) continue;
            int fl = c->flag[n];
            if (fl == LIQ || fl == IFC) {
                double r = 0;
                for (int p = 0; p < 19; ++p) r += c->f[(size_t)p * N + n];
                rs += r;
                ++nli;
            } else if (fl == GAS && gfirst < 0) {
                gfirst = n;
            }
        }
        int type;
        if (nli > 0) type = gfirst >= 0 ? IFC : LIQ;
        else type = gfirst >= 0 ? GAS : LIQ;
        ux[u] = x;
        dec[3 * u] = type;
        dec[3 * u + 1] = gfirst >= 0 ? c->bub[gfirst] : 0;
        drho[u] = nli > 0 ? rs / nli : 1.0;
        ++u;
    }
    for (u = 0; u < n_unc; ++u) {
        int x = ux[u], type = dec[3 * u];
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        int P = c->pid[x];
        double p[3] = {i, j, k}, ur[3], e[19];
        rigid_velocity(c, P, p, ur);
        c->conv[x] = 0;
        c->pid[x] = -1;
        c->flag[x] = (uint8_t)type;
        if (type == GAS) {
            c->bub[x] = dec[3 * u + 1];
            c->phi[x] = 0;
            for (int q = 0; q < 19; ++q) c->f[(size_t)q * N + x] = 0;
            continue;
        }
        orc_equilibrium(drho[u], ur, e);
        for (int q = 0; q < 19; ++q) c->f[(size_t)q * N + x] = e[q];
        c->ledger -= drho[u];
        if (type == IFC) {
            c->m[x] = drho[u];
            c->phi[x] = 1.0;
            c->bub[x] = dec[3 * u + 1];
        } else {
            c->phi[x] = 1.0;
        }
    }
    /* closure among uncovered nodes */
    for (u = 0; u < n_unc; ++u) {
        int x = ux[u];
        if (c->flag[x] != LIQ) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        for (int q = 1; q < 19; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n >= 0 && c->flag[n] == GAS) {
                c->flag[x] = IFC;
                c->m[x] = drho[u];
                c->phi[x] = 1.0;
                c->bub[x] = c->bub[n];
                break;
            }
        }
    }
    free(dec);
    free(drho);
    free(ux);
}

/* ---- particles ---------------------------------------------------------------- */
/* Sphere positions: every component finite; on a walled axis the centre lies in the
 * box (faces at -1/2 and n - 1/2); on a periodic axis anywhere (the centre is kept
 * in [0, n), and the sphere acts through its nearest images), the axis longer than
 * 2R + 4 so that every node within a link of the sphere is nearer to the centre than
 * half the box. */
static int position_ok(const orc_ctx *c, const double *x, double R)
{
    for (int a = 0; a < 3; ++a) {
        double v = x[a];
        if (!isfinite(v)) return 0;
        if (c->cfg.periodic[a]) {
            if (!(c->cfg.n[a] > 2.0 * R + 4.0)) return 0;
        } else if (v < -0.5 || v > c->cfg.n[a] - 0.5) {
            return 0;
        }
    }
    return 1;
}

int orc_particles_set(orc_ctx *c, int n, const double *x, const double *u,
                      const double *omega, const double *R, const double *rho_p)
{
    if (n < 0 || n > c->cfg.max_particles) { c->err |= ERR_ARG; return -1; }
    for (int P = 0; P < n; ++P) {
        if (!(R[P] > 0.0) || !(rho_p[P] > 0.0) || !position_ok(c, x + 3 * P, R[P])) {
            c->err |= ERR_ARG;
            return -1;
        }
        for (int a = 0; a < 3; ++a)
            if ((u && !isfinite(u[3 * P + a])) || (omega && !isfinite(omega[3 * P + a]))) {
                c->err |= ERR_ARG;
                return -1;
            }
    }
    c->np = n;
    c->have_prev = 0;
    for (int P = 0; P < n; ++P) {
        for (int a = 0; a < 3; ++a) {
            c->px[3 * P + a] = wrap_coord(c, a, x[3 * P + a]);
            c->pu[3 * P + a] = u ? u[3 * P + a] : 0.0;
            c->pw[3 * P + a] = omega ? omega[3 * P + a] : 0.0;
            c->pF[3 * P + a] = 0;
            c->pT[3 * P + a] = 0;
        }
        c->pR[P] = R[P];
        c->prho[P] = rho_p[P];
    }
    coverage_update(c);
    bubbles_recompute(c);
    split_bubbles(c);
    return 0;
}

int orc_walls_get(const orc_ctx *c, double F[18])
{
    for (int a = 0; a < 18; ++a) F[a] = c->wallF[a];
    return 0;
}

int orc_particles_get(orc_ctx *c, int n, double *x, double *u, double *omega, double *F, double *T)
{
    if (n > c->np) n = c->np;
    for (int P = 0; P < n; ++P)
        for (int a = 0; a < 3; ++a) {
            if (x) x[3 * P + a] = c->px[3 * P + a];
            if (u) u[3 * P + a] = c->pu[3 * P + a];
            if (omega) omega[3 * P + a] = c->pw[3 * P + a];
            if (F) F[3 * P + a] = c->pF[3 * P + a];
            if (T) T[3 * P + a] = c->pT[3 * P + a];
        }
    return n;
}

/* Contact between overlapping spheres.  The paper gives no contact model (its
 * lubrication force is cut off at small gaps); reading: a linear repulsive spring
 * of stiffness k along the line of centres, F1 = -k (R1 + R2 - |d|) d/|d| for
 * |d| < R1 + R2 (d = x2 - x1), equal and opposite on particle 2; k = 0 switches it
 * off.  Returns 1 when a force is applied. */
int orc_contact(const double x1[3], const double x2[3], double R1, double R2, double k, double F1[3])
{
    double d[3] = {x2[0] - x1[0], x2[1] - x1[1], x2[2] - x1[2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    F1[0] = F1[1] = F1[2] = 0;
    if (!(k > 0.0) || !(dist < R1 + R2) || dist <= 0.0) return 0;
    double s = -k * (R1 + R2 - dist) / dist;
    for (int a = 0; a < 3; ++a) F1[a] = s * d[a];
    return 1;
}

/* Eq. (lubrication) with the gap limited from below by 0.2 Delta_c and applied only
 * for gaps smaller than Delta_c = 2/3; returns 1 when a force is applied.  F1 is the
 * force on particle 1; particle 2 receives -F1. */
int orc_lubrication(const double x1[3], const double x2[3], const double u1[3],
                    const double u2[3], double R1, double R2, double mu, double F1[3])
{
    const double dc = 2.0 / 3.0;
    double d[3] = {x2[0] - x1[0], x2[1] - x1[1], x2[2] - x1[2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    F1[0] = F1[1] = F1[2] = 0;
    double gap = dist - R1 - R2;
    if (!(gap < dc) || dist <= 0.0) return 0;
    if (gap < 0.2 * dc) gap = 0.2 * dc;
    double n[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
    double rr = R1 * R2;
    double coef = -6.0 * M_PI * mu * (rr * rr) / ((R1 + R2) * (R1 + R2)) * (1.0 / gap - 1.0 / dc);
    double vn = n[0] * (u1[0] - u2[0]) + n[1] * (u1[1] - u2[1]) + n[2] * (u1[2] - u2[2]);
    for (int a = 0; a < 3; ++a) F1[a] = coef * vn * n[a];
    return 1;
}

/* A sphere at a no-slip face (axes a with noslip[a], faces at -1/2 and n[a] - 1/2).
 * The paper states Eq. (lubrication) and needs a contact rule only for pairs of
 * particles; reading: a face acts as a resting sphere of infinite radius touching the
 * face plane.  Then (R1 R2)^2 / (R1 + R2)^2 tends to R^2, the line of centres is the
 * face normal and the gap is h - R (h: distance of the centre from the face), so for
 * gaps below Delta_c = 2/3, limited from below by 0.2 Delta_c, the sphere takes
 * -6 pi mu R^2 (1/gap - 1/Delta_c) times its velocity component normal to the face,
 * along that normal; with k > 0 an overlapping sphere (h < R) is pushed off the face
 * by k (R - h).  Adds to F; returns the number of faces that applied a force. */
int orc_face_force(const int n[3], const int noslip[3], const double x[3], const double u[3],
                   double R, double mu, double k, double F[3])
{
    const double dc = 2.0 / 3.0;
    int hits = 0;
    for (int a = 0; a < 3; ++a) {
        if (!noslip[a]) continue;
        for (int side = 0; side < 2; ++side) {
            /* distance from the face and the direction pointing away from it */
            double h = side ? (n[a] - 0.5) - x[a] : x[a] + 0.5;
            double away = side ? -1.0 : 1.0;
            int hit = 0;
            if (k > 0.0 && h < R) {
                F[a] += away * k * (R - h);
                hit = 1;
            }
            double gap = h - R;
            if (gap < dc) {
                if (gap < 0.2 * dc) gap = 0.2 * dc;
                /* normal n = -away e_a towards the face: -c (n.u) n = -c u_a e_a */
                F[a] -= 6.0 * M_PI * mu * R * R * (1.0 / gap - 1.0 / dc) * u[a];
                hit = 1;
            }
            hits += hit;
        }
    }
    return hits;
}

/* Semi-implicit Euler with n_sub substeps (Sec. 2.3, "up to 10" read as a fixed
 * count; the paper does not give the scheme).  The hydrodynamic force and torque
 * are held constant over the substeps and are the mean of the momentum-exchange
 * values of this and the previous lattice step (the two-step average of Ladd's
 * suspension method, which removes the period-two oscillation of the momentum
 * exchange that otherwise drives explicit coupling unstable at density ratio
 * 2.5); right after the particle table is set, this step's value alone.  The
 * lubrication force is recomputed every substep, gravity m_P g (buoyancy comes
 * through the fluid pressure), m_P = rho_P 4/3 pi R^3, I = 2/5 m_P R^2.  The pair
 * forces (lubrication, contact) take the nearest periodic image of the partner;
 * the no-slip faces act on each sphere as in orc_face_force, at the position and
 * velocity the substep starts from.  Velocity is updated before position; along a periodic axis the position is kept
 * in [0, n).  A sphere closer than R to a wall face while moving towards it has
 * that velocity component reversed. */
static void particles_integrate(orc_ctx *c)
{
    const int np = c->np, ns = c->cfg.n_sub;
    const double dt = 1.0 / ns;
    const double mu = (c->cfg.tau - 0.5) / 3.0;
    int noslip[3];
    for (int a = 0; a < 3; ++a) noslip[a] = !c->cfg.periodic[a] && !c->cfg.freeslip[a];
    double *Fl = (double *)calloc((size_t)3 * np + 3, sizeof(double));
    for (int s = 0; s < ns; ++s) {
        memset(Fl, 0, sizeof(double) * 3 * np);
        for (int a = 0; a < np; ++a)
            for (int b = a + 1; b < np; ++b) {
                double F1[3], xb[3];
                for (int d = 0; d < 3; ++d)
                    xb[d] = c->px[3 * a + d] + min_image(c, d, c->px[3 * b + d] - c->px[3 * a + d]);
                if (orc_lubrication(c->px + 3 * a, xb, c->pu + 3 * a, c->pu + 3 * b,
                                    c->pR[a], c->pR[b], mu, F1)) {
                    for (int d = 0; d < 3; ++d) {
                        Fl[3 * a + d] += F1[d];
                        Fl[3 * b + d] -= F1[d];
                    }
                }
                if (orc_contact(c->px + 3 * a, xb, c->pR[a], c->pR[b], c->cfg.contact_k, F1)) {
                    for (int d = 0; d < 3; ++d) {
                        Fl[3 * a + d] += F1[d];
                        Fl[3 * b + d] -= F1[d];
                    }
                }
            }
        for (int P = 0; P < np; ++P)
            orc_face_force(c->cfg.n, noslip, c->px + 3 * P, c->pu + 3 * P, c->pR[P], mu, c->cfg.contact_k,
                           Fl + 3 * P);
        for (int P = 0; P < np; ++P) {
            double R = c->pR[P];
            double mP = c->prho[P] * (4.0 / 3.0) * M_PI * R * R * R;
            double IP = 0.4 * mP * R * R;
            for (int d = 0; d < 3; ++d) {
                double Fh = c->pF[3 * P + d], Th = c->pT[3 * P + d];
                if (c->have_prev) {
                    Fh = 0.5 * (Fh + c->pFp[3 * P + d]);
                    Th = 0.5 * (Th + c->pTp[3 * P + d]);
                }
                double F = Fh + mP * c->cfg.g[d] + Fl[3 * P + d];
                c->pu[3 * P + d] += dt * F / mP;
                c->px[3 * P + d] = wrap_coord(c, d, c->px[3 * P + d] + dt * c->pu[3 * P + d]);
                c->pw[3 * P + d] += dt * Th / IP;
                if (!c->cfg.periodic[d]) {
                    if (c->px[3 * P + d] < R - 0.5 && c->pu[3 * P + d] < 0)
                        c->pu[3 * P + d] = -c->pu[3 * P + d];
                    if (c->px[3 * P + d] > c->cfg.n[d] - 0.5 - R && c->pu[3 * P + d] > 0)
                        c->pu[3 * P + d] = -c->pu[3 * P + d];
                }
            }
        }
    }
    free(Fl);
    for (int k = 0; k < 3 * np; ++k) {
        c->pFp[k] = c->pF[k];
        c->pTp[k] = c->pT[k];
    }
    c->have_prev = 1;
    for (int P = 0; P < np; ++P)
        if (!position_ok(c, c->px + 3 * P, c->pR[P])) c->err |= ERR_PART;
}

/* ---- one lattice step ----------------------------------------------------------- */

/* momentum exchange over all particle links (Eqs. netforce, torque,
 * momentum_transfer) and the mass that moving bounce-back adds to a liquid cell,
 * which the ledger pays (an interface cell's mass is m, which only the exchange of
 * Eq. massExchangeb changes, so its moving-wall term is not charged).  Reading: the momentum Delta j_q(x) = c_q f*_q(x,t) -
 * c_qbar f_qbar(x,t+1) with f_qbar(x,t+1) from Eq. (bbrule); the torque arm is the
 * node x.  A solid node of another particle P' with a link into P contributes
 * with equilibrium populations at rho = 1 and the rigid velocity of P' at that
 * node: Delta j = 2 c_q e^+_q(1, u_P'(x)).  Reading for the faces of the box, which
 * the paper does not treat: a link into P from beyond a non-periodic face is taken
 * the same way, with the velocity of the first no-slip face it crosses (at rest when
 * it crosses free-slip faces only), and that no-slip face takes -Delta j.  The
 * constant parts 2 w_q c_q of the links into a closed node set cancel exactly; without
 * the face links a sphere that covers nodes of a face layer would miss them over the
 * cut and be pulled into the face by the lattice pressure 1/3.  Gas contributes
 * nothing.  The torque arm runs from the nearest image of the centre to the far end
 * of the link. */
static void force_pass(orc_ctx *c)
{
    const size_t N = (size_t)c->N;
    for (int a = 0; a < 18; ++a) c->wallP[a] = 0.0;
    for (int P = 0; P < c->np; ++P)
        for (int a = 0; a < 3; ++a) c->pF[3 * P + a] = c->pT[3 * P + a] = 0;
    if (c->np == 0) return;
    for (int x = 0; x < c->N; ++x) {
        int fl = c->flag[x];
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        if (fl == LIQ || fl == IFC) {
            int any = 0;
            for (int q = 1; q < 19 && !any; ++q) {
                int s = nbr(c, i, j, k, -CX[q], -CY[q], -CZ[q], NULL);
                if (s >= 0 && c->flag[s] == SOL) any = 1;
            }
            if (!any) continue;
            double rho, u[3];
            post_moments(c, c->f, x, &rho, u);
            for (int q = 1; q < 19; ++q) {
                int s = nbr(c, i, j, k, -CX[q], -CY[q], -CZ[q], NULL);
                if (s < 0 || c->flag[s] != SOL) continue;
                int P = c->pid[s];
                double fout = c->f[(size_t)OPP[q] * N + x];
                double fin = bb_particle(c, c->f, x, q, P, rho);
                /* link x -> x + c_qbar enters P; Delta j = c_qbar (fout + fin) */
                double dj[3] = {-CX[q] * (fout + fin), -CY[q] * (fout + fin), -CZ[q] * (fout + fin)};
                double r[3] = {min_image(c, 0, i - c->px[3 * P]), min_image(c, 1, j - c->px[3 * P + 1]),
                               min_image(c, 2, k - c->px[3 * P + 2])};
                c->pF[3 * P] += dj[0];
                c->pF[3 * P + 1] += dj[1];
                c->pF[3 * P + 2] += dj[2];
                c->pT[3 * P] += r[1] * dj[2] - r[2] * dj[1];
                c->pT[3 * P + 1] += r[2] * dj[0] - r[0] * dj[2];
                c->pT[3 * P + 2] += r[0] * dj[1] - r[1] * dj[0];
                if (fl == LIQ) c->ledger -= fin - fout; /* interface mass is m, not rho */
            }
        } else if (fl == SOL) {
            int Pp = c->pid[x];
            if (Pp >= 0)
                for (int q = 1; q < 19; ++q) {
                    /* a link into this node of Pp from beyond the faces of the box */
                    if (nbr(c, i, j, k, -CX[q], -CY[q], -CZ[q], NULL) >= 0) continue;
                    int slip = 0;
                    const int cross = crossed_axes(c, i, j, k, -CX[q], -CY[q], -CZ[q], &slip);
                    double uw[3] = {0.0, 0.0, 0.0};
                    int face = -1;
                    if (!slip) {
                        int a = 0;
                        while (!((cross >> a) & 1) || c->cfg.freeslip[a]) ++a;
                        const int v = a == 0 ? i - CX[q] : (a == 1 ? j - CY[q] : k - CZ[q]);
                        face = 2 * a + (v < 0 ? 0 : 1);
                        for (int d = 0; d < 3; ++d) uw[d] = c->cfg.wall_u[a][v < 0 ? 0 : 1][d];
                    }
                    double ep = 2.0 * eq_plus(q, 1.0, uw);
                    double dj[3] = {CX[q] * ep, CY[q] * ep, CZ[q] * ep};
                    double r[3] = {min_image(c, 0, i - CX[q] - c->px[3 * Pp]),
                                   min_image(c, 1, j - CY[q] - c->px[3 * Pp + 1]),
                                   min_image(c, 2, k - CZ[q] - c->px[3 * Pp + 2])};
                    c->pF[3 * Pp] += dj[0];
                    c->pF[3 * Pp + 1] += dj[1];
                    c->pF[3 * Pp + 2] += dj[2];
                    c->pT[3 * Pp] += r[1] * dj[2] - r[2] * dj[1];
                    c->pT[3 * Pp + 1] += r[2] * dj[0] - r[0] * dj[2];
                    c->pT[3 * Pp + 2] += r[0] * dj[1] - r[1] * dj[0];
                    if (face >= 0)
                        for (int d = 0; d < 3; ++d) c->wallP[3 * face + d] -= dj[d];
                }
            for (int q = 1; q < 19; ++q) {
                int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                if (n < 0 || c->flag[n] != SOL) continue;
                int P = c->pid[n];
                if (P == Pp) continue;
                double p[3] = {i, j, k}, ur[3];
                rigid_velocity(c, Pp, p, ur);
                double ep = 2.0 * eq_plus(q, 1.0, ur);
                double dj[3] = {CX[q] * ep, CY[q] * ep, CZ[q] * ep};
                double r[3] = {min_image(c, 0, i - c->px[3 * P]), min_image(c, 1, j - c->px[3 * P + 1]),
                               min_image(c, 2, k - c->px[3 * P + 2])};
                c->pF[3 * P] += dj[0];
                c->pF[3 * P + 1] += dj[1];
                c->pF[3 * P + 2] += dj[2];
                c->pT[3 * P] += r[1] * dj[2] - r[2] * dj[1];
                c->pT[3 * P + 1] += r[2] * dj[0] - r[0] * dj[2];
                c->pT[3 * P + 2] += r[0] * dj[1] - r[1] * dj[0];
            }
        }
    }
}

/* TRT collision Eq. (LBE2) with Guo forcing split into even and odd parts:
 * f* = f + lp (f+ - e+) + lm (f- - e-) + (1 + lp/2) F+ + (1 + lm/2) F-,
 * F_q = w_q [3 (c_q - u) + 9 (c_q . u) c_q] . F, F = rho g. */
static void collide_cell(const orc_ctx *c, double fcell[19], double rho, const double u[3])
{
    double e[19], Fq[19], fs[19];
    const double *g = c->cfg.g;
    double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
    orc_equilibrium(rho, u, e);
    for (int q = 0; q < 19; ++q) {
        double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
        double t0 = 3.0 * ((CX[q] - u[0]) * F[0] + (CY[q] - u[1]) * F[1] + (CZ[q] - u[2]) * F[2]);
        double t1 = 9.0 * cu * (CX[q] * F[0] + CY[q] * F[1] + CZ[q] * F[2]);
        Fq[q] = W[q] * (t0 + t1);
    }
    for (int q = 0; q < 19; ++q) {
        int o = OPP[q];
        double fp = 0.5 * (fcell[q] + fcell[o]), fm = 0.5 * (fcell[q] - fcell[o]);
        double ep = 0.5 * (e[q] + e[o]), em = 0.5 * (e[q] - e[o]);
        double Fp = 0.5 * (Fq[q] + Fq[o]), Fm = 0.5 * (Fq[q] - Fq[o]);
        fs[q] = fcell[q] + c->lp * (fp - ep) + c->lm * (fm - em) + (1.0 + 0.5 * c->lp) * Fp +
                (1.0 + 0.5 * c->lm) * Fm;
    }
    for (int q = 0; q < 19; ++q) fcell[q] = fs[q];
}

/* ---- surface tension: interface curvature (end of Sec. 2.2) ---------------------- */
/* The fill level as the curvature sees it: liquid 1, gas 0, interface its fill
 * level, particle nodes 1 (reading of perfect wettability: the liquid spreads on the
 * particles); a position beyond a wall takes the value of the nearest cell inside
 * the box, so the normal has no component into the wall. */
static int clamp_axis(int v, int n, int periodic)
{
    if (periodic) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

static double phi_eff(const orc_ctx *c, int i, int j, int k)
{
    i = clamp_axis(i, c->nx, c->cfg.periodic[0]);
    j = clamp_axis(j, c->ny, c->cfg.periodic[1]);
    k = clamp_axis(k, c->nz, c->cfg.periodic[2]);
    int x = i + c->nx * (j + c->ny * k);
    switch (c->flag[x]) {
    case GAS: return 0.0;
    case IFC: return c->phi[x];
    default: return 1.0; /* liquid and particle nodes */
    }
}

/* weight of a cell displaced along the differentiation axis when its two other
 * offsets are a and b (Parker and Youngs): 4, 2 or 1 for 0, 1 or 2 of them nonzero */
static double py_weight(int a, int b)
{
    return (a == 0 && b == 0) ? 4.0 : ((a == 0 || b == 0) ? 2.0 : 1.0);
}

/* n = grad phi by the weighted central differences over the 3x3x3 block (the
 * weights of one axis sum to 16 over a distance of 2, hence 1/32) */
static void py_gradient(const orc_ctx *c, int i, int j, int k, double n[3])
{
    n[0] = n[1] = n[2] = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                double v = phi_eff(c, i + dx, j + dy, k + dz);
                if (dx) n[0] += dx * py_weight(dy, dz) * v;
                if (dy) n[1] += dy * py_weight(dx, dz) * v;
                if (dz) n[2] += dz * py_weight(dx, dy) * v;
            }
    n[0] /= 32.0;
    n[1] /= 32.0;
    n[2] /= 32.0;
}

/* kappa = -(1/2) div(n/|n|) with the same weighted differences.  Reading: the paper
 * writes kappa = -div(n/|n|) together with p_w = p_g + 2 sigma kappa; the Laplace
 * jump 2 sigma / R of a spherical bubble needs kappa to be the mean curvature, half
 * the divergence.  With n pointing into the liquid, a gas bubble has kappa = -1/R. */
static double curvature_at(const orc_ctx *c, int i, int j, int k)
{
    double div = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                int a = clamp_axis(i + dx, c->nx, c->cfg.periodic[0]);
                int b = clamp_axis(j + dy, c->ny, c->cfg.periodic[1]);
                int d = clamp_axis(k + dz, c->nz, c->cfg.periodic[2]);
                double n[3];
                py_gradient(c, a, b, d, n);
                double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                if (nn == 0.0) continue;
                if (dx) div += dx * py_weight(dy, dz) * n[0] / nn;
                if (dy) div += dy * py_weight(dx, dz) * n[1] / nn;
                if (dz) div += dz * py_weight(dx, dy) * n[2] / nn;
            }
    return -0.5 * div / 32.0;
}

int orc_curvature(orc_ctx *c, double *kappa)
{
    for (int x = 0; x < c->N; ++x) {
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        kappa[x] = c->flag[x] == IFC ? curvature_at(c, i, j, k) : 0.0;
    }
    return 0;
}

static void stream_collide(orc_ctx *c)
{
    const size_t N = (size_t)c->N;
    const double *g = c->cfg.g;
    int nerr = 0;
    double wf[18];
    for (int a = 0; a < 18; ++a) wf[a] = c->wallP[a];  /* links into particle nodes */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : nerr) reduction(+ : wf[:18]) num_threads(c->cfg.n_threads > 0 ? c->cfg.n_threads : omp_get_max_threads())
#endif
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                int x = i + c->nx * (j + c->ny * k);
                int fl = c->flag[x];
                if (fl != LIQ && fl != IFC) {
                    c->phi_new[x] = 0.0;
                    continue;
                }
                double fc[19];
                double rho_t = 0, u_t[3] = {0, 0, 0};
                int have_t = 0;
                double kappa = 0.0;
                int have_kappa = 0;
                fc[0] = c->f[x];
                for (int q = 1; q < 19; ++q) {
                    int s = nbr(c, i, j, k, -CX[q], -CY[q], -CZ[q], NULL);
                    int sf = s >= 0 ? c->flag[s] : -1;
                    if (sf == LIQ || sf == IFC) {
                        fc[q] = c->f[(size_t)q * N + s];
                        continue;
                    }
                    if (!have_t) {
                        post_moments(c, c->f, x, &rho_t, u_t);
                        have_t = 1;
                    }
                    int slip = 0, cross = s < 0 ? crossed_axes(c, i, j, k, -CX[q], -CY[q], -CZ[q], &slip) : 0;
                    if (s < 0 && slip) {
                        /* free slip: specular reflection from the cell beside x along the
                         * wall; gas there gives the free-surface condition, a particle
                         * node plain bounce-back */
                        const int sp = nbr(c, i, j, k, (cross & 1) ? 0 : -CX[q], (cross & 2) ? 0 : -CY[q],
                                           (cross & 4) ? 0 : -CZ[q], NULL);
                        const int spf = c->flag[sp];
                        if (spf == LIQ || spf == IFC) {
                            fc[q] = c->f[(size_t)mirror_dir(q, cross) * N + sp];
                        } else if (spf == GAS) {
                            double rg = bubble_rho(c, c->bub[sp]);
                            if (c->cfg.sigma != 0.0) {
                                if (!have_kappa) {
                                    kappa = curvature_at(c, i, j, k);
                                    have_kappa = 1;
                                }
                                rg += 6.0 * c->cfg.sigma * kappa;
                            }
                            fc[q] = -c->f[(size_t)OPP[q] * N + x] + 2.0 * eq_plus(q, rg, u_t);
                        } else {
                            fc[q] = c->f[(size_t)OPP[q] * N + x];
                        }
                    } else if (s < 0) { /* half-way no-slip wall, optionally moving */
                        /* the moving-wall term of the first crossed no-slip face */
                        int a = 0;
                        while (!((cross >> a) & 1) || c->cfg.freeslip[a]) ++a;
                        const int v = a == 0 ? i - CX[q] : (a == 1 ? j - CY[q] : k - CZ[q]);
                        const int side = v < 0 ? 0 : 1;
                        const double *uw = c->cfg.wall_u[a][side];
                        double cu = CX[q] * uw[0] + CY[q] * uw[1] + CZ[q] * uw[2];
                        const double fout = c->f[(size_t)OPP[q] * N + x];
                        fc[q] = fout + 6.0 * W[q] * rho_t * cu;
                        /* momentum exchange with that face (as for particle links):
                         * Delta j = c_qbar (f*_qbar(x,t) + f_q(x,t+1)) */
                        wf[3 * (2 * a + side)] -= CX[q] * (fout + fc[q]);
                        wf[3 * (2 * a + side) + 1] -= CY[q] * (fout + fc[q]);
                        wf[3 * (2 * a + side) + 2] -= CZ[q] * (fout + fc[q]);
                    } else if (sf == SOL) {
                        fc[q] = bb_particle(c, c->f, x, q, c->pid[s], rho_t);
                    } else { /* gas: Eq. (fsk) with p_w = p_g of the neighbour's bubble */
                        if (fl == LIQ) nerr |= ERR_LG;
                        double rg = bubble_rho(c, c->bub[s]);
                        /* Laplace pressure jump p_w = p_g + 2 sigma kappa, rho = 3 p */
                        if (c->cfg.sigma != 0.0) {
                            if (!have_kappa) {
                                kappa = curvature_at(c, i, j, k);
                                have_kappa = 1;
                            }
                            rg += 6.0 * c->cfg.sigma * kappa;
                        }
                        fc[q] = -c->f[(size_t)OPP[q] * N + x] + 2.0 * eq_plus(q, rg, u_t);
                    }
                }
                double rho = 0, jx = 0, jy = 0, jz = 0;
                for (int q = 0; q < 19; ++q) {
                    rho += fc[q];
                    jx += CX[q] * fc[q];
                    jy += CY[q] * fc[q];
                    jz += CZ[q] * fc[q];
                }
                double u[3] = {(jx + 0.5 * rho * g[0]) / rho, (jy + 0.5 * rho * g[1]) / rho,
                               (jz + 0.5 * rho * g[2]) / rho};
                if (!(rho == rho) || !(u[0] == u[0])) nerr |= ERR_NAN;
                if (fl == IFC) {
                    /* Eqs. (massExchange, massExchangeb), mass form: m += sum_q dm_q,
                     * phi = m / rho(t+1); post-collision populations of time t on both
                     * sides of the link; phi(t) on both sides for interface links */
                    double dm = 0;
                    for (int q = 1; q < 19; ++q) {
                        int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                        int qin = OPP[q];  /* the population arriving at x against c_q */
                        if (n < 0) {
                            /* across free-slip faces the partner is the cell beside x
                             * along the wall, whose reflected population arrives here */
                            int slip = 0;
                            const int cross = crossed_axes(c, i, j, k, CX[q], CY[q], CZ[q], &slip);
                            if (!slip) continue;
                            n = nbr(c, i, j, k, (cross & 1) ? 0 : CX[q], (cross & 2) ? 0 : CY[q],
                                    (cross & 4) ? 0 : CZ[q], NULL);
                            qin = mirror_dir(OPP[q], cross);
                        }
                        int nf = c->flag[n];
                        if (nf != LIQ && nf != IFC) continue;
                        double d = c->f[(size_t)qin * N + n] - c->f[(size_t)q * N + x];
                        if (nf == IFC) d *= 0.5 * (c->phi[n] + c->phi[x]);
                        dm += d;
                    }
                    c->m[x] += dm;
                    c->phi_new[x] = c->m[x] / rho;
                } else {
                    c->phi_new[x] = 1.0;
                }
                c->rho_new[x] = rho;
                c->u_new[x] = u[0];
                c->u_new[N + x] = u[1];
                c->u_new[2 * N + x] = u[2];
                collide_cell(c, fc, rho, u);
                for (int q = 0; q < 19; ++q) c->fn[(size_t)q * N + x] = fc[q];
            }
    c->err |= (uint32_t)nerr;
    for (int a = 0; a < 18; ++a) c->wallF[a] = wf[a];
    double *t = c->f; c->f = c->fn; c->fn = t;
    t = c->phi; c->phi = c->phi_new; c->phi_new = t;
}

/* Cell conversions (Fig. cellConversions and the text after Eq. massExchangeb).
 * Readings: an interface cell fills when phi >= 1 - eps_c and empties when
 * phi <= eps_c; an emptying cell with a filling D3Q19 neighbour stays interface for
 * this step; gas neighbours of filled cells and liquid neighbours of emptied
 * cells become interface; a gas cell turned interface starts from the equilibrium
 * at the mean density and velocity of its neighbours that were liquid or
 * interface before the conversion, with m = 0; a liquid cell turned interface
 * keeps m = rho and takes the bubble id of its first emptied neighbour; the excess
 * mass (m - rho of a filled cell, m of an emptied cell) is shared equally by the
 * neighbours that are interface after the conversion, or goes to the ledger when
 * there are none; emptied cells whose gas neighbours belong to other bubbles merge
 * those bubbles (root = lower id, masses add). */
static void conversions(orc_ctx *c)
{
    const size_t N = (size_t)c->N;
    const double eps = c->cfg.eps_c;
    int nF = 0, nE = 0;
    for (int x = 0; x < c->N; ++x) {
        c->conv[x] = CV_NONE;
        if (c->flag[x] != IFC) continue;
        if (c->phi[x] >= 1.0 - eps) { c->conv[x] = CV_F; ++nF; }
        else if (c->phi[x] <= eps) { c->conv[x] = CV_E0; ++nE; }
    }
    if (!nF && !nE) return;
    /* conflict rule */
    for (int x = 0; x < c->N; ++x) {
        if (c->conv[x] != CV_E0) continue;
        int i, j, k, keep = 1;
        cell_ijk(c, x, &i, &j, &k);
        for (int q = 1; q < 19 && keep; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n >= 0 && c->conv[n] == CV_F) keep = 0;
        }
        c->conv[x] = keep ? CV_E : CV_NONE;
    }
    /* closure marks */
    for (int x = 0; x < c->N; ++x) {
        int cv = c->conv[x];
        if (cv != CV_F && cv != CV_E) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        for (int q = 1; q < 19; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n < 0) continue;
            if (cv == CV_F && c->flag[n] == GAS) c->conv[n] = CV_NEWG;
            if (cv == CV_E && c->flag[n] == LIQ) c->conv[n] = CV_NEWL;
        }
    }
    /* initialise new interface cells (old flags still in place) */
    for (int x = 0; x < c->N; ++x) {
        int cv = c->conv[x];
        if (cv != CV_NEWG && cv != CV_NEWL) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        if (cv == CV_NEWG) {
            double rs = 0, us[3] = {0, 0, 0};
            int cnt = 0;
            for (int q = 1; q < 19; ++q) {
                int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                if (n < 0 || (c->flag[n] != LIQ && c->flag[n] != IFC)) continue;
                rs += c->rho_new[n];
                us[0] += c->u_new[n];
                us[1] += c->u_new[N + n];
                us[2] += c->u_new[2 * N + n];
                ++cnt;
            }
            double rb = rs / cnt, ub[3] = {us[0] / cnt, us[1] / cnt, us[2] / cnt}, e[19];
            orc_equilibrium(rb, ub, e);
            for (int q = 0; q < 19; ++q) c->f[(size_t)q * N + x] = e[q];
            c->rho_new[x] = rb;
            c->u_new[x] = ub[0];
            c->u_new[N + x] = ub[1];
            c->u_new[2 * N + x] = ub[2];
            c->m[x] = 0.0;
        } else {
            c->m[x] = c->rho_new[x];
            for (int q = 1; q < 19; ++q) {
                int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                if (n >= 0 && c->conv[n] == CV_E) { c->bub[x] = c->bub[n]; break; }
            }
        }
    }
    /* finalise flags */
    for (int x = 0; x < c->N; ++x) {
        switch (c->conv[x]) {
        case CV_F: c->flag[x] = LIQ; break;
        case CV_E: c->flag[x] = GAS; break;
        case CV_NEWG:
        case CV_NEWL: c->flag[x] = IFC; break;
        default: break;
        }
    }
    /* excess mass */
    for (int x = 0; x < c->N; ++x) {
        int cv = c->conv[x];
        if (cv != CV_F && cv != CV_E) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        double ex = (cv == CV_F) ? c->m[x] - c->rho_new[x] : c->m[x];
        int rec[18], nr = 0;
        for (int q = 1; q < 19; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n >= 0 && c->flag[n] == IFC) rec[nr++] = n;
        }
        if (nr == 0) c->ledger += ex;
        else
            for (int r = 0; r < nr; ++r) c->m[rec[r]] += ex / nr;
        c->m[x] = 0.0;
    }
    for (int x = 0; x < c->N; ++x) {
        if (c->flag[x] == IFC) c->phi[x] = c->m[x] / c->rho_new[x];
        else if (c->flag[x] == LIQ) c->phi[x] = 1.0;
        else if (c->flag[x] == GAS) c->phi[x] = 0.0;
    }
    /* bubble merge through emptied cells */
    int merged = 0;
    for (int x = 0; x < c->N; ++x) {
        if (c->conv[x] != CV_E) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        for (int q = 1; q < 19; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n < 0 || c->flag[n] != GAS) continue;
            int a = find_root(c, c->bub[x]), b = find_root(c, c->bub[n]);
            if (a == b) continue;
            int lo = a < b ? a : b, hi = a < b ? b : a;
            c->broot[hi] = lo;
            c->bM[lo] += c->bM[hi];
            c->balive[hi] = 0;
            merged = 1;
        }
    }
    /* after a merge every gas and interface cell carries its root id, so that the
     * merged ids hold no cells and can be taken again by a split */
    if (merged)
        for (int x = 0; x < c->N; ++x)
            if (c->flag[x] == GAS || c->flag[x] == IFC) c->bub[x] = find_root(c, c->bub[x]);
    for (int x = 0; x < c->N; ++x) c->conv[x] = CV_NONE;
}

static void check_invariant(orc_ctx *c)
{
    for (int x = 0; x < c->N; ++x) {
        if (c->flag[x] != LIQ) continue;
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        for (int q = 1; q < 19; ++q) {
            int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
            if (n >= 0 && c->flag[n] == GAS) { c->err |= ERR_LG; return; }
        }
    }
}

int orc_step(orc_ctx *c, int nsteps)
{
    for (int s = 0; s < nsteps; ++s) {
        force_pass(c);
        stream_collide(c);
        conversions(c);
        if (c->np > 0 && c->cfg.integrate) {
            particles_integrate(c);
            coverage_update(c);
        }
        bubbles_recompute(c);
        split_bubbles(c);
        check_invariant(c);
    }
    return c->err ? -1 : 0;
}

/* ---- reporting ----------------------------------------------------------------- */
static void neumaier_add(double *s, double *comp, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *comp += (*s - t) + v;
    else *comp += (v - t) + *s;
    *s = t;
}

void orc_mass_get(orc_ctx *c, double *total, double *ledger)
{
    double s = 0, comp = 0;
    for (int x = 0; x < c->N; ++x) {
        if (c->flag[x] == LIQ) {
            for (int q = 0; q < 19; ++q) neumaier_add(&s, &comp, c->f[(size_t)q * c->N + x]);
        } else if (c->flag[x] == IFC) {
            neumaier_add(&s, &comp, c->m[x]);
        }
    }
    neumaier_add(&s, &comp, c->ledger);
    if (total) *total = s + comp;
    if (ledger) *ledger = c->ledger;
}

int orc_bubbles_get(orc_ctx *c, orc_bubble *out, int cap, int *n)
{
    int k = 0;
    for (int b = 0; b < c->nb && k < cap; ++b, ++k) {
        orc_bubble *o = out + k;
        int r = find_root(c, b);
        o->id = b;
        o->alive = c->balive[b] && r == b;
        o->V = c->bV[r];
        o->M = c->bM[r];
        o->rho_g = c->brho[r];
        for (int a = 0; a < 3; ++a) o->centroid[a] = c->bcent[3 * r + a];
        o->V0 = c->bV0[b];
        o->n_gas = c->bngas[r];
        o->n_iface = c->bnif[r];
    }
    if (n) *n = c->nb;
    return 0;
}

int orc_bubbles_set(orc_ctx *c, int n, const double *M, const int *root, const int *alive)
{
    if (n > c->cfg.max_bubbles) return -1;
    c->nb = n;
    for (int b = 0; b < n; ++b) {
        c->bM[b] = M[b];
        c->broot[b] = root[b];
        c->balive[b] = alive[b];
    }
    bubbles_recompute(c);
    split_bubbles(c);
    return (c->err & ERR_CAP) ? -1 : 0;
}

int orc_field_get(orc_ctx *c, int which, void *out)
{
    const size_t N = (size_t)c->N;
    switch (which) {
    case ORC_FLAGS: memcpy(out, c->flag, N); break;
    case ORC_MASS: memcpy(out, c->m, N * sizeof(double)); break;
    case ORC_PHI: memcpy(out, c->phi, N * sizeof(double)); break;
    case ORC_F: memcpy(out, c->f, 19 * N * sizeof(double)); break;
    case ORC_BUBBLE_ID: memcpy(out, c->bub, N * sizeof(int)); break;
    case ORC_PID: memcpy(out, c->pid, N * sizeof(int)); break;
    case ORC_RHO:
    case ORC_U: {
        double *o = (double *)out;
        for (int x = 0; x < c->N; ++x) {
            double r = 0, u[3] = {0, 0, 0};
            if (c->flag[x] == LIQ || c->flag[x] == IFC) post_moments(c, c->f, x, &r, u);
            if (which == ORC_RHO) o[x] = r;
            else {
                o[x] = u[0];
                o[N + x] = u[1];
                o[2 * N + x] = u[2];
            }
        }
        break;
    }
    default: return -1;
    }
    return 0;
}

int orc_field_set(orc_ctx *c, int which, const void *in)
{
    const size_t N = (size_t)c->N;
    switch (which) {
    case ORC_FLAGS: memcpy(c->flag, in, N); break;
    case ORC_MASS: memcpy(c->m, in, N * sizeof(double)); break;
    case ORC_PHI: memcpy(c->phi, in, N * sizeof(double)); break;
    case ORC_F: memcpy(c->f, in, 19 * N * sizeof(double)); break;
    case ORC_BUBBLE_ID: memcpy(c->bub, in, N * sizeof(int)); break;
    case ORC_PID: memcpy(c->pid, in, N * sizeof(int)); break;
    default: return -1;
    }
    return 0;
}

/* ---- differentiation form: summed drag over a frozen window ------------------ */
/* d lambda_- / d tau of the TRT constraint (Sec. 2.1); for SRT lambda_- = lambda_+ */
static double dlm_dtau(double tau, double magic, int trt)
{
    if (!trt) return 1.0 / (tau * tau);
    double a = 0.5 - tau;            /* 1/lp + 1/2 */
    double lm = orc_lambda_minus(tau, magic, trt);
    return -lm * lm * magic / (a * a);
}

/* J_t of the window: -sum_P uhat_P . F_P with F_P the momentum exchange of
 * force_pass (fluid links and the equilibrium links of other particles) evaluated
 * on the state s; its tangents along the four parameter directions from ds.  Wall
 * links carry no particle force.  Serial, in cell order. */
static void window_drag(const orc_ctx *c, const double *s, const double *ds, const double *uhat,
                        double *J, double dJ[4])
{
    const size_t N = (size_t)c->N;
    for (int x = 0; x < c->N; ++x) {
        int i, j, k;
        cell_ijk(c, x, &i, &j, &k);
        if (c->flag[x] == LIQ) {
            double rw = 0, drw[4] = {0, 0, 0, 0};
            for (int q = 0; q < 19; ++q) {
                rw += s[(size_t)q * N + x];
                for (int d = 0; d < 4; ++d) drw[d] += ds[((size_t)d * 19 + q) * N + x];
            }
            for (int q = 1; q < 19; ++q) {
                int src = nbr(c, i, j, k, -CX[q], -CY[q], -CZ[q], NULL);
                if (src < 0 || c->flag[src] != SOL) continue;
                int P = c->pid[src];
                const double *uh = uhat + 3 * P;
                double xw[3] = {i - 0.5 * CX[q], j - 0.5 * CY[q], k - 0.5 * CZ[q]}, uw[3];
                rigid_velocity(c, P, xw, uw);
                double cu = CX[q] * uw[0] + CY[q] * uw[1] + CZ[q] * uw[2];
                double cuh = CX[q] * uh[0] + CY[q] * uh[1] + CZ[q] * uh[2];
                int o = OPP[q];
                /* Delta j = -c_q (f*_qbar + f_q(t+1)), f_q(t+1) from Eq. (bbrule) */
                double fout = s[(size_t)o * N + x];
                double fin = fout + 6.0 * W[q] * rw * cu;
                *J += cuh * (fout + fin);
                for (int d = 0; d < 4; ++d) {
                    double dfo = ds[((size_t)d * 19 + o) * N + x];
                    dJ[d] += cuh * (2.0 * dfo + 6.0 * W[q] * drw[d] * cu);
                }
            }
        } else if (c->flag[x] == SOL) {
            int Pp = c->pid[x];
            for (int q = 1; q < 19; ++q) {
                int n = nbr(c, i, j, k, CX[q], CY[q], CZ[q], NULL);
                if (n < 0 || c->flag[n] != SOL) continue;
                int P = c->pid[n];
                if (P == Pp) continue;
                double p[3] = {i, j, k}, ur[3];
                rigid_velocity(c, Pp, p, ur);
                const double *uh = uhat + 3 * P;
                double cuh = CX[q] * uh[0] + CY[q] * uh[1] + CZ[q] * uh[2];
                *J -= cuh * 2.0 * eq_plus(q, 1.0, ur);
            }
        }
    }
}

/* Summed drag J = sum_{t<T} J_t over T frozen-flag steps from the current state
 * and its tangent-linear (forward-mode) derivatives along tau and g, found by
 * differentiating each part of the step -- streaming with bounce-back (Eq. bbrule,
 * including its density rho_w), moments with the half-force shift and the TRT
 * collision with Guo forcing (Eq. LBE2) -- with respect to the parameters, the
 * window's initial state held fixed.  Every non-solid cell must be liquid and the
 * spheres kinematic (integrate off), so the cell types cannot change.  The
 * oracle's own state is left as it was. */
int orc_window_J(orc_ctx *c, int T, double *J, double *dJ)
{
    const size_t N = (size_t)c->N;
    if (T < 0 || !J) return -1;
    if (c->cfg.integrate && c->np > 0) return -1;
    for (int a = 0; a < 3; ++a)  /* the window's links are no-slip or periodic */
        if (c->cfg.freeslip[a] && !c->cfg.periodic[a]) return -1;
    for (int x = 0; x < c->N; ++x)
        if (c->flag[x] == GAS || c->flag[x] == IFC) return -1;
    double *s = (double *)malloc(sizeof(double) * 19 * N);
    double *sn = (double *)malloc(sizeof(double) * 19 * N);
    double *ds = (double *)calloc(4 * 19 * N, sizeof(double));
    double *dsn = (double *)calloc(4 * 19 * N, sizeof(double));
    double *uhat = (double *)calloc(3 * (size_t)(c->np > 0 ? c->np : 1), sizeof(double));
    if (!s || !sn || !ds || !dsn || !uhat) {
        free(s); free(sn); free(ds); free(dsn); free(uhat);
        return -1;
    }
    memcpy(s, c->f, sizeof(double) * 19 * N);
    memcpy(sn, c->f, sizeof(double) * 19 * N);
    for (int P = 0; P < c->np; ++P) {
        const double *u = c->pu + 3 * P;
        double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        if (nu > 0)
            for (int a = 0; a < 3; ++a) uhat[3 * P + a] = u[a] / nu;
    }
    const double *g = c->cfg.g;
    const double lp = c->lp, lm = c->lm;
    /* derivatives of the rates and of g along direction d: d = 0 tau, d = 1..3 g */
    double dlp[4] = {1.0 / (c->cfg.tau * c->cfg.tau), 0, 0, 0};
    double dlmv[4] = {dlm_dtau(c->cfg.tau, c->cfg.magic, c->cfg.trt), 0, 0, 0};
    double dg[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double Jv = 0, dJv[4] = {0, 0, 0, 0};

    for (int t = 0; t < T; ++t) {
        window_drag(c, s, ds, uhat, &Jv, dJv);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(c->cfg.n_threads > 0 ? c->cfg.n_threads : omp_get_max_threads())
#endif
        for (int x = 0; x < c->N; ++x) {
            if (c->flag[x] != LIQ) continue;
            int i, j, k;
            cell_ijk(c, x, &i, &j, &k);
            /* streaming with reconstruction, and its tangent */
            double fc[19], dfc[4][19];
            double rt = 0, drt[4] = {0, 0, 0, 0};
            for (int q = 0; q < 19; ++q) {
                rt += s[(size_t)q * N + x];
                for (int d = 0; d < 4; ++d) drt[d] += ds[((size_t)d * 19 + q) * N + x];
            }
            for (int q = 0; q < 19; ++q) {
                int face = -1;
                int src = q == 0 ? x : nbr(c, i, j, k, -CX[q], -CY[q], -CZ[q], &face);
                int o = OPP[q];
                if (src >= 0 && c->flag[src] == LIQ) {
                    fc[q] = s[(size_t)q * N + src];
                    for (int d = 0; d < 4; ++d) dfc[d][q] = ds[((size_t)d * 19 + q) * N + src];
                    continue;
                }
                double uw[3] = {0, 0, 0};
                if (src < 0) {
                    const double *w = c->cfg.wall_u[face / 2][face % 2];
                    uw[0] = w[0]; uw[1] = w[1]; uw[2] = w[2];
                } else {
                    double xw[3] = {i - 0.5 * CX[q], j - 0.5 * CY[q], k - 0.5 * CZ[q]};
                    rigid_velocity(c, c->pid[src], xw, uw);
                }
                double cu = CX[q] * uw[0] + CY[q] * uw[1] + CZ[q] * uw[2];
                fc[q] = s[(size_t)o * N + x] + 6.0 * W[q] * rt * cu;
                for (int d = 0; d < 4; ++d)
                    dfc[d][q] = ds[((size_t)d * 19 + o) * N + x] + 6.0 * W[q] * drt[d] * cu;
            }
            /* moments: rho, u = (j + rho g / 2) / rho */
            double rho = 0, jm[3] = {0, 0, 0};
            for (int q = 0; q < 19; ++q) {
                rho += fc[q];
                jm[0] += CX[q] * fc[q];
                jm[1] += CY[q] * fc[q];
                jm[2] += CZ[q] * fc[q];
            }
            double u[3] = {(jm[0] + 0.5 * rho * g[0]) / rho, (jm[1] + 0.5 * rho * g[1]) / rho,
                           (jm[2] + 0.5 * rho * g[2]) / rho};
            double e[19], Fq[19], F[3] = {rho * g[0], rho * g[1], rho * g[2]};
            orc_equilibrium(rho, u, e);
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            for (int q = 0; q < 19; ++q) {
                double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
                double cF = CX[q] * F[0] + CY[q] * F[1] + CZ[q] * F[2];
                Fq[q] = W[q] * (3.0 * (cF - (u[0] * F[0] + u[1] * F[1] + u[2] * F[2])) + 9.0 * cu * cF);
            }
            for (int d = 0; d < 4; ++d) {
                /* tangent of the moments */
                double drho = 0, dj[3] = {0, 0, 0};
                for (int q = 0; q < 19; ++q) {
                    drho += dfc[d][q];
                    dj[0] += CX[q] * dfc[d][q];
                    dj[1] += CY[q] * dfc[d][q];
                    dj[2] += CZ[q] * dfc[d][q];
                }
                double du[3], dF[3];
                for (int a = 0; a < 3; ++a) {
                    du[a] = (dj[a] - (jm[a] / rho) * drho) / rho + 0.5 * dg[d][a];
                    dF[a] = drho * g[a] + rho * dg[d][a];
                }
                double udu = u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
                double de[19], dFq[19];
                for (int q = 0; q < 19; ++q) {
                    double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
                    double dcu = CX[q] * du[0] + CY[q] * du[1] + CZ[q] * du[2];
                    de[q] = W[q] * (drho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) +
                                    rho * (3.0 * dcu + 9.0 * cu * dcu - 3.0 * udu));
                    double cF = CX[q] * F[0] + CY[q] * F[1] + CZ[q] * F[2];
                    double cdF = CX[q] * dF[0] + CY[q] * dF[1] + CZ[q] * dF[2];
                    double duF = du[0] * F[0] + du[1] * F[1] + du[2] * F[2];
                    double udF = u[0] * dF[0] + u[1] * dF[1] + u[2] * dF[2];
                    dFq[q] = W[q] * (3.0 * (cdF - duF - udF) + 9.0 * (dcu * cF + cu * cdF));
                }
                /* tangent of f* = f + lp (f+ - e+) + lm (f- - e-) + (1 + lp/2) F+ + (1 + lm/2) F- */
                for (int q = 0; q < 19; ++q) {
                    int o = OPP[q];
                    double fp = 0.5 * (fc[q] + fc[o]), fm = 0.5 * (fc[q] - fc[o]);
                    double ep = 0.5 * (e[q] + e[o]), em = 0.5 * (e[q] - e[o]);
                    double Fp = 0.5 * (Fq[q] + Fq[o]), Fm = 0.5 * (Fq[q] - Fq[o]);
                    double dfp = 0.5 * (dfc[d][q] + dfc[d][o]), dfm = 0.5 * (dfc[d][q] - dfc[d][o]);
                    double dep = 0.5 * (de[q] + de[o]), dem = 0.5 * (de[q] - de[o]);
                    double dFp = 0.5 * (dFq[q] + dFq[o]), dFm = 0.5 * (dFq[q] - dFq[o]);
                    dsn[((size_t)d * 19 + q) * N + x] =
                        dfc[d][q] + dlp[d] * (fp - ep) + lp * (dfp - dep) + dlmv[d] * (fm - em) +
                        lm * (dfm - dem) + 0.5 * dlp[d] * Fp + (1.0 + 0.5 * lp) * dFp +
                        0.5 * dlmv[d] * Fm + (1.0 + 0.5 * lm) * dFm;
                }
            }
            /* primal: the oracle's own collision */
            collide_cell(c, fc, rho, u);
            for (int q = 0; q < 19; ++q) sn[(size_t)q * N + x] = fc[q];
        }
        double *tp = s; s = sn; sn = tp;
        tp = ds; ds = dsn; dsn = tp;
    }
    *J = Jv;
    if (dJ)
        for (int d = 0; d < 4; ++d) dJ[d] = dJv[d];
    free(s); free(sn); free(ds); free(dsn); free(uhat);
    return 0;
}
