/*
 * fsl.h -- C ABI of the MI355X (gfx950) free-surface lattice Boltzmann library
 * for liquid-gas-solid flow (Bogner, Harting & Ruede, "Direct simulation of
 * liquid-gas-solid flow with a free surface lattice Boltzmann method").
 *
 * The library advances one simulation state on one GPU.  It never allocates
 * device memory: the caller passes one device workspace of
 * fsl_workspace_bytes(cfg) bytes (with fsl_init_static, the state part only) and
 * a HIP stream; every kernel runs on that stream.  The library allocates only its small host context (freed by
 * fsl_destroy, which never frees the workspace).  Host arrays passed to the
 * get/set calls are owned by the caller, row-major, FP64 unless stated.
 *
 * Problem statement (Sec. 2): the box is split into three disjoint regions
 * (liquid, gas, solid).  Liquid is simulated by a D3Q19 lattice Boltzmann model
 * (Sec. 2.1); the liquid-gas boundary is captured by fill levels and cell types
 * (Sec. 2.2); every gas region (bubble) holds a constant gas mass that sets its
 * pressure; spheres described by radius, density, position, velocity and
 * angular velocity (Sec. 2.3) block the nodes they cover and couple through
 * moving-wall bounce-back and momentum exchange.
 *
 * Conventions (shared with the oracle by specification):
 *   cell index     i + nx*(j + ny*k); node (i,j,k) sits at (i,j,k); walls (no-slip
 *                  or free-slip) are half-way, at -1/2 and n-1/2 on non-periodic axes
 *   directions     0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (+-1,+-1,0),
 *                  (+-1,0,+-1), (0,+-1,+-1) in sign order (+,+),(+,-),(-,+),(-,-)
 *   flag values    0 gas, 1 liquid, 2 interface, 3 particle-covered
 *
 * Error convention: every int-returning call returns FSL_OK (0) or a negative
 * FSL_E_* code.  Errors raised inside kernels (list overflow, NaN, a liquid cell
 * next to gas) are latched on the device and reported by the next synchronising
 * call (fsl_sync, the get calls).  fsl_error_string gives the text of the last
 * error.  No C++ exception crosses this boundary.
 */
#ifndef FSL_H
#define FSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSL_OK 0
#define FSL_E_ARG (-1)       /* invalid argument or configuration            */
#define FSL_E_HIP (-2)       /* a HIP runtime call failed                     */
#define FSL_E_CAPACITY (-3)  /* a conversion/event list or table overflowed   */
#define FSL_E_NUMERIC (-4)   /* NaN/Inf density or velocity                   */
#define FSL_E_INVARIANT (-5) /* a liquid cell has a gas neighbour             */

#define FSL_NOSLIP 0
#define FSL_PERIODIC 1
#define FSL_FREESLIP 2  /* both faces reflect specularly (set-up of Sec. 3.2) */

#define FSL_SRT 0
#define FSL_TRT 1

/* population storage (form 1): FP32, or f - w_q stored as IEEE binary16 /
 * bfloat16 (round to nearest even); the collision always runs in FP32 */
#define FSL_STORE_F32 0
#define FSL_STORE_F16S 1
#define FSL_STORE_BF16S 2

#define FSL_MAX_GAS_SPHERES 16

typedef struct {
    int n[3];                   /* box size in cells, each >= 1                       */
    int boundary[3];            /* FSL_NOSLIP, FSL_PERIODIC or FSL_FREESLIP per axis.
                                   A link whose far end lies beyond faces of the box
                                   reflects specularly when every face it crosses is
                                   free-slip: it arrives from the cell beside the node
                                   along the wall with the crossed components of its
                                   direction reversed (gas there: the free-surface
                                   condition; a particle node: bounce-back).  Any
                                   no-slip face crossed: half-way bounce-back.  The
                                   interface mass exchange pairs a cell with the cell
                                   whose reflected populations it receives.          */
    int collision;              /* FSL_SRT or FSL_TRT                                 */
    double tau;                 /* relaxation time, lambda_+ = -1/tau (Sec. 2.1)      */
    double magic;               /* TRT constant Lambda (3/16 in the paper)            */
    double g[3];                /* body-force acceleration, lattice units             */
    double zs;                  /* pool height (node coordinates); < 0: fully liquid  */
    double rho_g0;              /* gas density of the atmosphere above the pool      */
    int n_gas_spheres;          /* spherical gas bubbles in the initial state         */
    double gas_spheres[FSL_MAX_GAS_SPHERES][5]; /* cx, cy, cz, r, rho_g                */
    int max_particles;          /* particle table capacity                            */
    int n_sub;                  /* particle substeps per lattice step (10)            */
    int integrate;              /* 1: particles move; 0: kinematic (fixed x, u, omega)*/
    int storage;                /* FSL_STORE_*                                        */
    double eps_c;               /* interface fills at phi >= 1-eps_c, empties at <= eps_c */
    int list_capacity;          /* per-step conversion/event list capacity, 0 = auto  */
    int max_bubbles;            /* bubble table capacity, 0 = auto (64)               */
    int window_steps;           /* differentiation window length T (0 = no window)    */
    int window_every;           /* checkpoint interval k of the window                */
    double sigma;               /* surface tension: the free-surface condition takes
                                   p_w = p_g + 2 sigma kappa (0 = none)                */
    double wall_u[3][2][3];     /* velocity of each non-periodic box face
                                   [axis][low, high][component]; the half-way
                                   bounce-back at a face takes the moving-wall form of
                                   Eq. bbrule (all zero: resting walls)                */
    int open_atmosphere;        /* 1: bubble 0 (the gas above the pool) is held at
                                   rho_g0, its mass following its volume, and is never
                                   split: a pressure outlet (Sec. 3.2)               */
    double contact_k;           /* stiffness of the contact spring between overlapping
                                   spheres, F = k (R1 + R2 - |d|) along the line of
                                   centres (0 = none; the paper gives no contact
                                   model, its lubrication force is cut off)          */
    int no_face_forces;         /* 1: the force on each no-slip face (fsl_walls_get) is
                                   not computed, which saves a pass over the face
                                   layers per step; fsl_walls_get then fails with
                                   FSL_E_ARG.  0 (the default): computed every step */
} fsl_config;

typedef struct {
    int id, alive;              /* alive: a root bubble (merged ones point to a root) */
    double V, M, rho_g;         /* gas volume (cells), constant gas mass, M/V         */
    double centroid[3];         /* gas-volume centroid                                */
    double V0;                  /* volume at initialisation                           */
    int64_t n_gas, n_iface;     /* gas and interface cells carrying the id            */
} fsl_bubble;

typedef struct fsl_ctx fsl_ctx;

/* Bytes of device workspace needed for cfg; 0 if cfg is invalid. */
size_t fsl_workspace_bytes(const fsl_config *cfg);

/* Build the initial state (Sec. 2.2 cell types and fill levels of a flat pool
 * with spherical gas bubbles, liquid at hydrostatic equilibrium) in the caller's
 * workspace d_ws (device pointer, >= fsl_workspace_bytes(cfg) bytes, 256-byte
 * aligned) and return a context bound to hip_stream (a hipStream_t, may be 0).
 * The workspace must outlive the context.  FSL_E_ARG on a bad configuration. */
int fsl_init(const fsl_config *cfg, void *d_ws, size_t bytes, void *hip_stream, fsl_ctx **out);

/* Bytes of device working memory that the library holds on each device for the
 * contexts of fsl_init_static (a file-scope device array, kept until the process
 * ends). */
#define FSL_STATIC_SCRATCH_BYTES (128u << 20)

/* fsl_init for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) once the state
 * exists.  The workspace of fsl_init has two parts: the state, which lives from
 * one call to the next (fields, particle and bubble tables, counters, error word,
 * stored densities, differentiation window), and the working memory that each
 * call writes before it reads it (conversion and event lists, particle pairs and
 * candidate grid, splitting labels, field staging, tile lists).  Here the caller
 * passes the state only; the working memory is the library's array of
 * FSL_STATIC_SCRATCH_BYTES on the current device, which must be the device of
 * hip_stream.
 *   d_state NULL: *bytes receives the state bytes cfg needs; nothing else happens.
 *   otherwise:    d_state (device, 256-byte aligned, *bytes >= that size, owned by
 *                 the caller and outliving the context) receives the initial state
 *                 and *out the context, used like one from fsl_init.
 * FSL_E_ARG if cfg is invalid or needs more working memory than the array holds
 * (roughly 15 bytes per cell with particles, 8 without), with the text from
 * fsl_error_string(NULL); FSL_E_HIP if the array's address cannot be found.  Every
 * context made here on one device shares the array: calls on such contexts that
 * overlap in time (other streams, other threads) race and give wrong results;
 * calls that follow one another on the device are independent.  No call allocates
 * device memory. */
int fsl_init_static(const fsl_config *cfg, void *d_state, size_t *bytes, void *hip_stream, fsl_ctx **out);

/* Enqueue n lattice steps on the stream (asynchronous).  One step: streaming with
 * wall / moving-particle / free-surface reconstruction, moments, interface mass
 * exchange, collision (Eqs. LBE1, LBE2, fsk, bbrule, massExchange, massExchangeb),
 * momentum exchange (Eqs. netforce, torque), cell conversions, particle update
 * (Eq. lubrication, substeps) and the bubble model (end of Sec. 2.2): gas volumes
 * and densities, merges, and splitting: where the gas of a bubble falls apart
 * (D3Q19 neighbours of one root bubble), the part with the lowest cell index keeps
 * the id, the others take the lowest ids that are not alive, in order of their
 * lowest cell index, interface cells follow the part of their gas neighbours, and
 * the gas mass is shared by volume.  After a merge every gas and interface cell
 * carries its root id, so merged ids are free again.  A bubble whose gas volume
 * vanishes no longer exists (its gas mass leaves).  A split that needs more live
 * bubbles than max_bubbles, or a state with more than 1024 separate gas parts, is
 * reported as FSL_E_CAPACITY by the next synchronising call.
 * For n >= 8 on a stream other than the null stream, once the stored densities
 * are valid and the particle update is past its first step (and profiling is
 * off), the steps are replayed from a HIP graph of two captured steps: the same
 * kernels in the same order, without the per-launch cost.  Every setter, the
 * window calls and fsl_profile_enable drop the graph. */
int fsl_step(fsl_ctx *ctx, int n);

/* Replace the particle table with n spheres (Sec. 2.3; arrays n x 3: centres in
 * node coordinates, velocities, angular velocities; n: radii, specific densities;
 * u / omega may be NULL for zero) and recompute node coverage.  Newly covered
 * cells hand their liquid mass to the ledger, uncovered cells are re-initialised.
 * Along a periodic axis a sphere may lie across the faces: its centre is taken into
 * [0, n) and it acts through its nearest images (coverage, links, lever arms, pair
 * forces); the axis must be longer than 2R + 4.  FSL_E_ARG if n > max_particles, a
 * radius is not in (0, 60] cells, a density is not positive, a value is not finite,
 * a centre lies outside a walled axis (faces at -1/2 and n - 1/2) or a periodic axis
 * is too short.  A sphere whose centre leaves a walled box later is reported as
 * FSL_E_INVARIANT by the next synchronising call. */
int fsl_particles_set(fsl_ctx *ctx, int n, const double *x, const double *u,
                      const double *omega, const double *R, const double *rho_p);

/* Copy the first n particles' state (any pointer may be NULL) to the host.
 * F and T are the momentum-exchange force and torque of the last completed step
 * (Eqs. netforce, torque).  Synchronises the stream. */
int fsl_particles_get(fsl_ctx *ctx, int n, double *x, double *u, double *omega,
                      double *F, double *T);

/* Force of the fluid on each no-slip face of the box over the last completed step:
 * the momentum exchange (Eqs. netforce, momentum_transfer) of the face's half-way
 * bounce-back links, resting or moving (Eq. bbrule), as for particle links; the
 * plate force of the sheared suspension (Sec. 3.1, mu_s = F_x / (A gamma)).  A
 * sphere node on a face layer takes the links from beyond the face as links from
 * inside another particle (Eq. momentum_transfer: equilibrium at rho = 1, here with
 * the face's velocity); the face takes the opposite momentum of those too.
 * F[3 (2 axis + side) + component], side 0 the low face; a link whose source lies
 * beyond several faces counts for the first no-slip one; free-slip and periodic
 * faces read 0.  The normal components include the fluid pressure (rho c_s^2 per
 * unit area at rest).  Synchronises.  FSL_E_ARG
 * when the context was made with no_face_forces. */
int fsl_walls_get(fsl_ctx *ctx, double F[18]);

/* Copy up to cap bubble records (the bubble model of Sec. 2.2: gas mass M, volume V
 * from the fill levels, rho_g = M / V) to out; *n receives the number of ids in use
 * (splits add ids).  Synchronises. */
int fsl_bubbles_get(fsl_ctx *ctx, fsl_bubble *out, int cap, int *n);

/* Import the bubble table of Sec. 2.2 (gas masses, merge roots, alive flags) for
 * n ids (the others become unused), recompute volumes and gas densities rho_g =
 * M / V from the current fields and split bubbles whose gas is not connected. */
int fsl_bubbles_set(fsl_ctx *ctx, int n, const double *M, const int *root, const int *alive);

/* Field exchange for tests and checkpoints.  Host layouts:
 *   FSL_FIELD_FLAGS u8[N]; FSL_FIELD_MASS f64[N] (interface mass m);
 *   FSL_FIELD_PHI f64[N]; FSL_FIELD_F f64[19][N] post-collision populations,
 *   unshifted; FSL_FIELD_BUBBLE_ID i32[N]; FSL_FIELD_PID i32[N] (-1 = none);
 *   FSL_FIELD_KAPPA f64[N] (get only, sigma != 0): interface curvature of the
 *   current state, the one the next step uses; 0 outside interface cells.
 * fields_get synchronises; fields_set is stream-ordered and synchronises. */
#define FSL_FIELD_FLAGS 0
#define FSL_FIELD_MASS 1
#define FSL_FIELD_PHI 2
#define FSL_FIELD_F 3
#define FSL_FIELD_BUBBLE_ID 4
#define FSL_FIELD_PID 5
#define FSL_FIELD_KAPPA 6
int fsl_fields_get(fsl_ctx *ctx, int field, void *host);
int fsl_fields_set(fsl_ctx *ctx, int field, const void *host);

/* Total mass sum_liquid rho + sum_interface m + ledger (FP64) and the ledger alone
 * (mass held by covered cells, by excess without recipients and paid by moving
 * bounce-back).  Synchronises. */
int fsl_mass_get(fsl_ctx *ctx, double *total, double *ledger);

/* Wait for the stream and report a latched device error (FSL_E_*). */
int fsl_sync(fsl_ctx *ctx);

/* Text of the last error of ctx (never NULL); with ctx NULL, of the last call on
 * this thread that failed before it had a context (fsl_init_static). */
const char *fsl_error_string(const fsl_ctx *ctx);

/* Free the host context (not the workspace). */
void fsl_destroy(fsl_ctx *ctx);

/* Per-phase timing with HIP events on the library's stream.  When enabled, each
 * phase of a step is bracketed by events; fsl_profile_get writes, for phase k < n
 * (0 = fused stream-collide kernel, 1 = cell conversions, 2 = bubble volumes,
 * 3 = particle pairs and forces, 4 = particle substeps, 5 = coverage update,
 * 6 = interface curvature, run only with sigma > 0, 7 = bubble splitting test and
 * pass), the summed milliseconds and counts since the last call, resets them,
 * synchronises and returns the number of phases (8).  Off by default. */
int fsl_profile_enable(fsl_ctx *ctx, int on);
int fsl_profile_get(fsl_ctx *ctx, double *ms, long long *count, int n);

/* Differentiation form: the summed drag over a window with frozen cell types and
 * its gradient with respect to the relaxation time and the body force.
 *
 * fsl_window_forward runs T ordinary steps (Sec. 2.1 stream-collide with the
 * bounce-back of Eq. bbrule) from the current state and returns, in FP64,
 *   J = sum_{t=1..T} sum_P (-F_P(t) . u_P/|u_P|),
 * F_P(t) the momentum-exchange force of step t (Eqs. netforce, momentum_transfer);
 * particles at rest do not contribute.  It keeps the state at t = 0, k, 2k, ... as
 * checkpoints in the workspace; afterwards the state is the state after T steps.
 * Requirements (FSL_E_ARG otherwise): the configuration reserved the window
 * (cfg.window_steps >= T, cfg.window_every >= k, ceil(T/k) <= ceil(window_steps /
 * window_every)), FP32 storage, spheres kinematic (integrate = 0), no free-slip
 * faces, and every non-solid cell liquid, so that no cell type can change.
 *
 * fsl_window_backward returns dJ/dtau (total derivative, including lambda_- of the
 * TRT constraint) and dJ/dg[3], both multiplied by the seed dJ, by a reverse sweep
 * that recomputes each segment of k steps from its checkpoint.  It needs a
 * completed fsl_window_forward with no fsl_params_set, fsl_particles_set or
 * fsl_fields_set since (FSL_E_ARG otherwise) and does not change the state.
 * Both synchronise the stream. */
int fsl_window_forward(fsl_ctx *ctx, int T, int k, double *J);
int fsl_window_backward(fsl_ctx *ctx, double dJ, double *dJ_dtau, double dJ_dg[3]);

/* Replace the relaxation time tau (> 1/2; lambda_- follows the TRT constraint with
 * the configured magic parameter) and the body force g for the following steps
 * (Sec. 2.1).  Invalidates a recorded window.  Asynchronous. */
int fsl_params_set(fsl_ctx *ctx, double tau, const double g[3]);

#ifdef __cplusplus
}
#endif
#endif
