/*
 * fsl_oracle.h -- interface of the plain FP64 CPU oracle of the free-surface
 * lattice Boltzmann step (liquid-gas-solid, Bogner, Harting & Ruede 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no source with the HIP path: constants,
 * geometry rules and every arithmetic step are typed out here independently.
 *
 * Conventions (common to both implementations by specification, not by code):
 *   direction order  0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *                    7..18 = (+-1,+-1,0),(+-1,0,+-1),(0,+-1,+-1) in the sign
 *                    order (+,+),(+,-),(-,+),(-,-)
 *   cell index       i + nx*(j + ny*k); node (i,j,k) sits at (i,j,k); the
 *                    no-slip walls are half-way, at -1/2 and n-1/2
 *   flag values      0 gas, 1 liquid, 2 interface, 3 particle-covered
 *   populations      exchanged unshifted, q-major: f[q*N + cell]
 */
#ifndef FSL_ORACLE_H
#define FSL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_GAS_SPHERES 16

typedef struct {
    int n[3];                 /* box size in cells                          */
    int periodic[3];          /* 1 = periodic axis, 0 = half-way no-slip wall */
    int trt;                  /* 0 = single relaxation time, 1 = two-relaxation-time */
    double tau;               /* tau = -1/lambda_plus                        */
    double magic;             /* Lambda of the TRT constraint (3/16)         */
    double g[3];              /* body-force acceleration                     */
    double zs;                /* pool height in node coordinates, <0: fully liquid */
    double rho_g0;            /* initial gas density of the atmosphere       */
    int n_gas_spheres;
    double gas_spheres[ORC_MAX_GAS_SPHERES][5]; /* cx, cy, cz, r, rho_g      */
    double eps_c;             /* conversion threshold slack                  */
    int integrate;            /* 1 = particles move, 0 = kinematic           */
    int n_sub;                /* particle substeps per lattice step          */
    int max_particles;
    int max_bubbles;
    double wall_u[3][2][3];   /* velocity of each box face [axis][low/high][comp] */
    int n_threads;            /* OpenMP threads for the per-cell loops (0 = default) */
    double sigma;             /* surface tension (0: no Laplace pressure jump)  */
    int freeslip[3];          /* 1 = the faces of a non-periodic axis reflect
                                 specularly (free slip) instead of bouncing back */
    int open_atmosphere;      /* 1 = bubble 0 (the gas above the pool) is held at
                                 rho_g0 (pressure outlet) instead of a fixed mass */
    double contact_k;         /* stiffness of the sphere contact spring (0 = none) */
} orc_config;

typedef struct {
    int id, alive;
    double V, M, rho_g, centroid[3], V0;
    int64_t n_gas, n_iface;
} orc_bubble;

typedef struct orc_ctx orc_ctx;

orc_ctx *orc_create(const orc_config *cfg);
void orc_destroy(orc_ctx *c);
int orc_step(orc_ctx *c, int nsteps);
int orc_particles_set(orc_ctx *c, int n, const double *x, const double *u,
                      const double *omega, const double *R, const double *rho_p);
int orc_particles_get(orc_ctx *c, int n, double *x, double *u, double *omega,
                      double *F, double *T);
int orc_bubbles_get(orc_ctx *c, orc_bubble *out, int cap, int *n);
/* force of the fluid on each no-slip face over the last step (momentum exchange of
 * its half-way bounce-back links), F[3 (2 axis + side) + comp], side 0 = low face;
 * a link beyond several faces counts for the first no-slip one; free-slip and
 * periodic faces read 0 */
int orc_walls_get(const orc_ctx *c, double F[18]);
void orc_mass_get(orc_ctx *c, double *total, double *ledger);

enum { ORC_FLAGS = 0, ORC_MASS = 1, ORC_PHI = 2, ORC_F = 3, ORC_BUBBLE_ID = 4, ORC_PID = 5,
       ORC_RHO = 6, ORC_U = 7 };
/* FLAGS u8, MASS f64, PHI f64, F f64[19][N], BUBBLE_ID i32, PID i32,
 * RHO f64 (moments of the stored post-collision state), U f64[3][N] */
int orc_field_get(orc_ctx *c, int which, void *out);
int orc_field_set(orc_ctx *c, int which, const void *in);
/* bubble table import: n records of (M, root, alive); volumes recomputed */
int orc_bubbles_set(orc_ctx *c, int n, const double *M, const int *root, const int *alive);
uint32_t orc_error(const orc_ctx *c);
int orc_num_cells(const orc_ctx *c);

/* Frozen-flag window (differentiation form): every non-solid cell liquid,
 * kinematic spheres (integrate off).  Runs T steps from the current state, which
 * it leaves unchanged, and returns J = sum_t sum_P (-F_P(t) . u_P/|u_P|), F_P(t)
 * the force reported by step t.  When dJ is non-null it also returns the
 * forward-mode (tangent-linear) derivatives dJ/dtau and dJ/dg[3] in dJ[0..3].
 * Returns -1 when the state does not allow a frozen window. */
int orc_window_J(orc_ctx *c, int T, double *J, double *dJ);

/* Interface curvature of the current state (the kappa of the Laplace pressure
 * jump): kappa[x] for every interface cell x, 0 elsewhere. */
int orc_curvature(orc_ctx *c, double *kappa);
/* Bubble splitting of the current state (also part of every step and of particles_set,
 * bubbles_set and create): returns the number of new bubbles, -1 with a full table. */
int orc_split(orc_ctx *c);

/* exposed pieces of the method for unit checks */
void orc_equilibrium(double rho, const double u[3], double e[19]);
int orc_lubrication(const double x1[3], const double x2[3], const double u1[3],
                    const double u2[3], double R1, double R2, double mu, double F1[3]);
int orc_contact(const double x1[3], const double x2[3], double R1, double R2, double k, double F1[3]);
int orc_face_force(const int n[3], const int noslip[3], const double x[3], const double u[3],
                   double R, double mu, double k, double F[3]);
double orc_lambda_minus(double tau, double magic, int trt);

#ifdef __cplusplus
}
#endif
#endif
