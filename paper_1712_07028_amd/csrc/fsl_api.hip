// fsl_api.hip -- host runtime and C ABI of the free-surface LBM library.
//
// The caller's workspace is carved into the state (two population lattices,
// cell types, fill levels, interface mass, bubble ids, particle ids), the
// per-step lists, the particle and bubble tables and a staging area for host
// exchange.  Every kernel is enqueued on the caller's stream; a step never
// returns control to the host, device-side errors are latched in one word and
// read at the next synchronising call.
#include <hip/hip_runtime.h>

#include <math.h>

#include <cmath>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/fsl.h"
#include "k_init.hpp"
#include "k_particles.hpp"
#include "k_split.hpp"
#include "k_stream_collide.hpp"
#include "k_adjoint.hpp"
#include "k_walls.hpp"

using namespace fsl;

namespace {

constexpr size_t ALIGN = 256;
constexpr int LIST_BLOCKS = 1024;  // list kernels: enough waves to hide the latency of their gathers
constexpr int NPROF = 8;

size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// The workspace has two parts.  The state (offsets from the workspace) holds what
// lives from one call to the next: fields, tables, counters, the error word, stored
// densities, curvature tile flags and the differentiation window.  The working
// memory (offsets from its own base) holds what one call writes before it reads it:
// conversion and event lists, particle pairs and candidate grid, splitting labels,
// field staging and the general-path tile list; their lengths are counters in the
// state.  fsl_init puts the working memory right after the state.
struct Layout {
    size_t fA, fB, flags, cv, phiA, phiB, m, bub, pid, claim;
    size_t counters, ctl, ptab, pacc, pFT, pFTp, pFl, pmir;
    size_t btab, bacc, broot, balive, rhog, kappa, ktf, klist, kcount, wallu;
    size_t rhow;  // densities of the liquid and interface cells for the next launch
    size_t wallF; // force on each no-slip face over the last step
    size_t win;   // differentiation window storage
    // working memory
    size_t lF, lE0, lE, lNG, lNL, lCov, lUnc, uncRho, uncDec, merges, pairs;
    size_t gStart, gCount, gIdx, gBsum, stage;
    size_t slab, scomp, scid, spar, svol;  // bubble splitting
    size_t glist;  // tiles of the general path of the stream-collide step
    size_t state, work, total;
    long long S;
    int cap, capEv, pcap, maxP, maxB, ncellMax, nTiles;
    int ktx, kty, nKT;  // curvature tiles
    size_t stageBytes, winBytes;
};

int esize(int storage) { return storage == FSL_STORE_F32 ? 4 : 2; }

bool valid(const fsl_config *c) {
    if (!c) return false;
    for (int a = 0; a < 3; ++a)
        if (c->n[a] < 1 || (c->boundary[a] != FSL_NOSLIP && c->boundary[a] != FSL_PERIODIC &&
                            c->boundary[a] != FSL_FREESLIP))
            return false;
    long long N = (long long)c->n[0] * c->n[1] * c->n[2];
    if (N >= (1LL << 31) - 4096) return false;
    if (!(c->tau > 0.5)) return false;
    if (c->collision != FSL_SRT && c->collision != FSL_TRT) return false;
    if (c->collision == FSL_TRT && !(c->magic > 0.0)) return false;
    if (c->storage < 0 || c->storage > 2) return false;
    if (c->n_gas_spheres < 0 || c->n_gas_spheres > FSL_MAX_GAS_SPHERES) return false;
    if (c->max_particles < 0 || c->n_sub < 0) return false;
    if (c->max_bubbles < 0 || c->max_bubbles > 64) return false;
    if (c->n_gas_spheres + 1 > (c->max_bubbles ? c->max_bubbles : 64)) return false;
    if (c->window_steps < 0 || c->window_every < 0) return false;
    if (!(c->sigma >= 0.0) || !(c->sigma < 1.0)) return false;
    return true;
}

// stage_cap: the most bytes of field staging (chunks of a field pass through it)
Layout layout_of(const fsl_config *c, size_t stage_cap = (size_t)64 << 20) {
    Layout L{};
    long long N = (long long)c->n[0] * c->n[1] * c->n[2];
    L.S = (N + 255) / 256 * 256;
    L.cap = c->list_capacity > 0 ? c->list_capacity : (int)std::max<long long>(65536, N / 16);
    // coverage events: replacing a whole particle table covers up to the solid
    // fraction of the box at once
    L.capEv = c->max_particles > 0 ? (int)std::max<long long>(L.cap, N / 3 + 65536) : L.cap;
    L.maxP = std::max(1, c->max_particles);
    L.pcap = 16 * L.maxP;
    L.maxB = c->max_bubbles > 0 ? c->max_bubbles : 64;
    L.ncellMax = ((c->n[0] + 2) / 3) * ((c->n[1] + 2) / 3) * ((c->n[2] + 2) / 3) + 1;
    L.stageBytes = std::min<size_t>(stage_cap, std::max<size_t>((size_t)L.S * 8, 1 << 20));
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
    size_t lat = (size_t)Q * L.S * esize(c->storage);
    L.fA = take(lat);
    L.fB = take(lat);
    L.flags = take(L.S);
    L.cv = take(L.S);
    L.phiA = take(L.S * 8);
    L.phiB = take(L.S * 8);
    L.m = take(L.S * 8);
    L.bub = take(L.S * 2);
    L.pid = take(L.S * 4);
    L.claim = take(L.S * 4);
    L.counters = take(64 * 4);
    L.ctl = take(64 * 8);  // [0] err word, [8] ledger, [16..] mass sums
    L.ptab = take((size_t)L.maxP * P_STRIDE * 8);
    L.pacc = take((size_t)L.maxP * ACC_COPIES * ACC_STRIDE * 8);
    L.pFT = take((size_t)L.maxP * 6 * 8);
    L.pFTp = take((size_t)L.maxP * 6 * 8);
    L.pFl = take((size_t)L.maxP * 3 * 8);
    L.pmir = take((size_t)L.maxP * 64);
    L.rhow = take(c->max_particles > 0 ? (size_t)L.S * 4 : 0);
    L.btab = take((size_t)L.maxB * B_STRIDE * 8);
    L.bacc = take((size_t)L.maxB * BACC_STRIDE * 8);
    L.broot = take((size_t)L.maxB * 4);
    L.balive = take((size_t)L.maxB * 4);
    L.rhog = take((size_t)L.maxB * 4);
    L.kappa = take(c->sigma != 0.0 ? (size_t)L.S * 4 : 0);
    L.ktx = (c->n[0] + KTX - 1) / KTX;
    L.kty = (c->n[1] + KTY - 1) / KTY;
    L.nKT = c->sigma != 0.0 ? L.ktx * L.kty * c->n[2] : 0;
    L.ktf = take((size_t)L.nKT * 4);
    L.klist = take((size_t)L.nKT * 4);
    L.kcount = take(c->sigma != 0.0 ? 4 : 0);
    L.wallu = take(18 * 4);
    L.wallF = take(18 * 8);
    L.nTiles = ((c->n[0] + TX - 1) / TX) * ((c->n[1] + TY - 1) / TY) * c->n[2];
    L.winBytes = adjoint_window_bytes(c->window_steps, c->window_every, (size_t)L.S, c->max_particles,
                                      L.nTiles);
    L.win = take(L.winBytes);
    L.state = o;
    o = 0;  // working memory
    L.lF = take((size_t)L.cap * 4);
    L.lE0 = take((size_t)L.cap * 4);
    L.lE = take((size_t)L.cap * 4);
    L.lNG = take((size_t)L.cap * 4);
    L.lNL = take((size_t)L.cap * 4);
    L.lCov = take((size_t)L.capEv * 8);
    L.lUnc = take((size_t)L.capEv * 8);
    L.uncRho = take((size_t)L.capEv * 8);
    L.uncDec = take((size_t)L.capEv * 4);
    L.merges = take((size_t)L.cap * 8);
    L.pairs = take((size_t)L.pcap * 8);
    L.gStart = take((size_t)(L.ncellMax + 1) * 4);
    L.gCount = take((size_t)L.ncellMax * 4);
    L.gIdx = take((size_t)L.maxP * 4);
    L.gBsum = take(1025 * 4);
    L.slab = take(L.S * 4);
    L.scomp = take(SPLIT_MAXC * 4);
    L.scid = take(SPLIT_MAXC * 4);
    L.spar = take(SPLIT_MAXC * 4);
    L.svol = take(SPLIT_MAXC * 8);
    L.stage = take(L.stageBytes);
    L.glist = take((size_t)L.nTiles * 4);
    L.work = o;
    L.total = L.state + L.work;
    return L;
}

}  // namespace

struct fsl_ctx {
    fsl_config cfg;
    Layout L;
    Geom G;
    Phys Ph;
    Dev D;
    SplitBuf SB;
    hipStream_t st;
    char *ws;  // state
    char *xs;  // working memory
    char err[256];
    double Rmax;
    PGrid PG;
    FaceSet FS;  // the no-slip face layers for the face forces
    int ncell;
    int tilesX, tilesY, nTiles;
    int profiling;
    int have_prev;  // a previous step's hydrodynamic force exists (particle update)
    int stamp;      // stamp of the next stream-collide launch (>= 1)
    int rhow_ok;    // the density words of stamp - 1 hold the densities of the populations in A
    // two steps captured as a HIP graph from a steady state (stored densities valid, the
    // particle update past its first step): fsl_step replays it while lattice A is the
    // buffer it was captured with; any setter drops it
    hipGraphExec_t gexec;
    void *gfA;
    int gstate;  // 0 usable, -1 capture failed on this context (eager steps only)
    std::vector<hipEvent_t> evpool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> evlog;
    double prof_ms[NPROF];
    long long prof_n[NPROF];
    AdjointState adj;
};

namespace {

int fail(fsl_ctx *c, int code, const char *msg) {
    if (c) snprintf(c->err, sizeof(c->err), "%s", msg);
    return code;
}

#define HIPCHK(ctx, call)                                                           \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            char b_[200];                                                           \
            snprintf(b_, sizeof b_, "%s: %s", #call, hipGetErrorString(e_));       \
            return fail(ctx, FSL_E_HIP, b_);                                        \
        }                                                                           \
    } while (0)

#define LAUNCHCHK(ctx)                                                              \
    do {                                                                            \
        hipError_t e_ = hipGetLastError();                                          \
        if (e_ != hipSuccess) return fail(ctx, FSL_E_HIP, hipGetErrorString(e_));  \
    } while (0)

hipEvent_t ev_get(fsl_ctx *c) {
    if (!c->evpool.empty()) {
        hipEvent_t e = c->evpool.back();
        c->evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    fsl_ctx *c;
    int k;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(fsl_ctx *ctx, int kind) : c(ctx), k(kind) {
        if (c->profiling) {
            a = ev_get(c);
            b = ev_get(c);
            if (a) (void)hipEventRecord(a, c->st);
        }
    }
    ~ProfScope() {
        if (c->profiling && a && b) {
            (void)hipEventRecord(b, c->st);
            c->evlog.push_back({k, {a, b}});
        }
    }
};

int grid_for(long long n, int block = 256, int cap = 8192) {
    long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void set_phys(fsl_ctx *c) {
    const fsl_config &f = c->cfg;
    c->Ph.lp = (float)(-1.0 / f.tau);
    double lp = -1.0 / f.tau;
    double lm = lp;
    if (f.collision == FSL_TRT) {
        double a = 1.0 / lp + 0.5;
        double b = f.magic / a;
        lm = 1.0 / (b - 0.5);
    }
    c->Ph.lm = (float)lm;
    for (int a = 0; a < 3; ++a) c->Ph.g[a] = (float)f.g[a];
    c->Ph.eps = f.eps_c;
    c->Ph.scale = f.storage == FSL_STORE_F16S ? 1024.0f : 1.0f;
    c->Ph.s6 = (float)(6.0 * f.sigma);
    c->Ph.moving_walls = 0;
    for (int a = 0; a < 3; ++a)
        for (int sd = 0; sd < 2; ++sd)
            for (int d = 0; d < 3; ++d)
                if (f.boundary[a] == FSL_NOSLIP && f.wall_u[a][sd][d] != 0.0) c->Ph.moving_walls = 1;
    for (int a = 0; a < 3; ++a) {
        c->Ph.slip[a] = f.boundary[a] == FSL_FREESLIP;
        if (c->Ph.slip[a]) c->Ph.moving_walls = 1;
    }
    c->Ph.open_atm = f.open_atmosphere != 0;
    c->Ph.inv = 1.0f / c->Ph.scale;
    // FSL_WIDE_OFFSETS=1 takes the 64-bit form on any box (a test of that form)
    const char *wide = getenv("FSL_WIDE_OFFSETS");
    c->Ph.wide = c->G.S >= (1ll << 30) || (wide && wide[0] == '1');
}

// one lattice update of every cell: the marching pass over the liquid cells, then the
// general path over the tiles it listed (interface cells, liquid cells next to gas or
// a moving or slipping face)
template <int ST, bool MW, bool PER>
void launch_stream_collide_mw(fsl_ctx *c, const Dev &Dv) {
    int *glist = (int *)(c->xs + c->L.glist), *ngen = Dv.counters + C_NGEN;
    // planes per block: NZC, fewer on small boxes so that the launch still fills the
    // device (at least 2,048 blocks)
    const long long cols = (long long)c->tilesX * c->tilesY;
    int nzc = NZC;
    while (nzc > 2 && cols * ((c->G.nz + nzc - 1) / nzc) < 2048) nzc /= 2;
    const int nChunks = (c->G.nz + nzc - 1) / nzc;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->st, ngen, 1LL, 0);
    hipLaunchKernelGGL((k_stream_collide<ST, MW, PER>), dim3(c->tilesX * c->tilesY * nChunks), dim3(256), 0, c->st,
                       c->G, c->Ph, Dv, c->tilesX, c->tilesY, nChunks, nzc, glist, ngen);
    hipLaunchKernelGGL((k_general<ST, MW>), dim3(std::min(c->nTiles, 4096)), dim3(256), 0, c->st, c->G, c->Ph, Dv,
                       c->tilesX, c->tilesY, (const int *)glist, (const int *)ngen);
}
template <int ST>
void launch_stream_collide(fsl_ctx *c, const Dev &Dv) {
    // the lever arms of particle links take nearest images only on boxes with a
    // periodic axis
    const bool per = c->G.per[0] || c->G.per[1] || c->G.per[2];
    if (c->Ph.moving_walls) {
        if (per) launch_stream_collide_mw<ST, true, true>(c, Dv);
        else launch_stream_collide_mw<ST, true, false>(c, Dv);
    } else {
        if (per) launch_stream_collide_mw<ST, false, true>(c, Dv);
        else launch_stream_collide_mw<ST, false, false>(c, Dv);
    }
}

template <int ST> int enqueue_steps(fsl_ctx *c, int n, int split = 1);
template <int ST> int enqueue_integration(fsl_ctx *c);
template <int ST> int enqueue_pair_forces(fsl_ctx *c);
template <int ST> int enqueue_coverage_step(fsl_ctx *c);
template <int ST> int enqueue_coverage_full(fsl_ctx *c);
template <int ST> int enqueue_bubbles(fsl_ctx *c, double *phi, int init);

template <int ST>
int enqueue_bubbles(fsl_ctx *c, double *phi, int init) {
    ProfScope ps(c, 2);
    Dev &D = c->D;
    hipLaunchKernelGGL(k_bubble_zero, dim3(1), dim3(256), 0, c->st, D, (const int *)nullptr);
    hipLaunchKernelGGL(k_bubble_accum, dim3(grid_for((c->G.N + 15) / 16, 256, 2048)), dim3(256), 0,
                       c->st, c->G, D, (const double *)phi, (const int *)nullptr);
    hipLaunchKernelGGL(k_bubble_finalize, dim3(1), dim3(64), 0, c->st, D, init, (const int *)nullptr,
                       c->Ph.open_atm);
    LAUNCHCHK(c);
    return FSL_OK;
}

// bubble splitting at the end of a step (force = 0: labelling only where the local
// test of a cell that left the gas fails) or of the current state (force = 1);
// phi is the state's fill level.  Every kernel after the test reads the flag the
// test leaves and returns at once when there is nothing to do.
template <int ST>
int enqueue_split(fsl_ctx *c, const double *phi, int force) {
    ProfScope ps(c, 7);
    const Dev &D = c->D;
    const SplitBuf &B = c->SB;
    const dim3 gl(LIST_BLOCKS), b(256), gn(grid_for(c->G.N, 256, 2048));
    if (force) hipLaunchKernelGGL(k_split_force, dim3(1), dim3(64), 0, c->st, D);
    else hipLaunchKernelGGL(k_split_test, gl, b, 0, c->st, c->G, D);
    hipLaunchKernelGGL(k_ccl_init, gn, b, 0, c->st, c->G, D, B);
    hipLaunchKernelGGL(k_ccl_union, gn, b, 0, c->st, c->G, D, B);
    hipLaunchKernelGGL(k_ccl_flatten, gn, b, 0, c->st, c->G, D, B);
    hipLaunchKernelGGL(k_split_plan, dim3(1), dim3(1024), 0, c->st, D, B, c->Ph.open_atm);
    hipLaunchKernelGGL(k_split_ifc, gn, b, 0, c->st, c->G, D, B, phi);
    hipLaunchKernelGGL(k_split_gas, dim3(grid_for((c->G.N + 15) / 16, 256, 2048)), b, 0, c->st, c->G, D, B);
    hipLaunchKernelGGL(k_split_mass, dim3(1), dim3(256), 0, c->st, D, B);
    const int *gate = D.counters + C_SPLIT;  // 2: some bubble split, volumes again
    hipLaunchKernelGGL(k_bubble_accum, dim3(grid_for((c->G.N + 15) / 16, 256, 2048)), dim3(256), 0,
                       c->st, c->G, D, phi, gate);
    hipLaunchKernelGGL(k_bubble_finalize, dim3(1), dim3(64), 0, c->st, D, 0, gate, c->Ph.open_atm);
    LAUNCHCHK(c);
    return FSL_OK;
}

template <int ST>
int enqueue_conversions(fsl_ctx *c) {
    ProfScope ps(c, 1);
    Dev &D = c->D;
    dim3 g(LIST_BLOCKS), b(256);
    hipLaunchKernelGGL(k_conv_mark, g, b, 0, c->st, D);
    hipLaunchKernelGGL(k_conv_closure, g, b, 0, c->st, c->G, D);
    hipLaunchKernelGGL(k_conv_init<ST>, g, b, 0, c->st, c->G, c->Ph, D);
    hipLaunchKernelGGL(k_conv_finalize, g, b, 0, c->st, D);
    hipLaunchKernelGGL(k_conv_excess<ST>, g, b, 0, c->st, c->G, c->Ph, D);
    hipLaunchKernelGGL(k_conv_fill<ST>, g, b, 0, c->st, c->G, c->Ph, D);
    hipLaunchKernelGGL(k_bubble_merge, dim3(1), dim3(64), 0, c->st, D);
    hipLaunchKernelGGL(k_bubble_relabel, dim3(grid_for(c->G.N, 256, 2048)), b, 0, c->st, c->G, D);
    LAUNCHCHK(c);
    return FSL_OK;
}

// cover / uncover events with the lattice lat and fill levels phi as "current"
template <int ST>
int enqueue_cover_events(fsl_ctx *c, const Dev &Dv, double *phi) {
    dim3 g(LIST_BLOCKS), b(256);
    hipLaunchKernelGGL(k_cov_apply<ST>, g, b, 0, c->st, c->G, c->Ph, Dv, phi);
    hipLaunchKernelGGL(k_unc_decide<ST>, g, b, 0, c->st, c->G, c->Ph, Dv);
    hipLaunchKernelGGL(k_unc_apply<ST>, g, b, 0, c->st, c->G, c->Ph, Dv, phi);
    hipLaunchKernelGGL(k_unc_closure, g, b, 0, c->st, c->G, Dv, phi);
    LAUNCHCHK(c);
    return FSL_OK;
}

template <int ST>
int enqueue_particles(fsl_ctx *c) {
    int rc = enqueue_pair_forces<ST>(c);
    if (rc || !c->cfg.integrate) return rc;
    rc = enqueue_integration<ST>(c);
    if (rc) return rc;
    return enqueue_coverage_step<ST>(c);
}

template <int ST>
int enqueue_pair_forces(fsl_ctx *c) {
    Dev &D = c->D;
    const int np = D.np;
    ProfScope ps(c, 3);
    // candidate pairs (positions at t): particle-particle links and lubrication
    hipLaunchKernelGGL(k_grid_zero, dim3(grid_for(c->ncell)), dim3(256), 0, c->st, D, c->ncell);
    hipLaunchKernelGGL(k_grid_count, dim3(grid_for(np)), dim3(256), 0, c->st, D, c->PG);
    {
        const int chunk = std::max(256, (c->ncell + 1023) / 1024 + 255) / 256 * 256;
        const int nb = (c->ncell + chunk - 1) / chunk;
        int *bsum = (int *)(c->xs + c->L.gBsum);
        hipLaunchKernelGGL(k_gscan_sum, dim3(nb), dim3(256), 0, c->st, D, c->ncell, chunk, bsum);
        hipLaunchKernelGGL(k_gscan_top, dim3(1), dim3(1024), 0, c->st, D, c->ncell, nb, bsum);
        hipLaunchKernelGGL(k_gscan_apply, dim3(nb), dim3(256), 0, c->st, D, c->ncell, chunk, (const int *)bsum);
    }
    hipLaunchKernelGGL(k_grid_fill, dim3(grid_for(np)), dim3(256), 0, c->st, D, c->PG);
    hipLaunchKernelGGL(k_pairs, dim3(grid_for((long long)np * 27, 256, 2048)), dim3(256), 0, c->st, D, c->PG, c->L.pcap);
    hipLaunchKernelGGL(k_solid_pairs, dim3(grid_for(c->L.pcap, 4, 8192)), dim3(256), 0, c->st, c->G, D, c->L.pcap);
    if (!c->G.per[0] || !c->G.per[1] || !c->G.per[2])
        hipLaunchKernelGGL(k_face_links, dim3((np + 3) / 4), dim3(256), 0, c->st, c->G, c->Ph, D);
    hipLaunchKernelGGL(k_part_forces, dim3((np + 255) / 256), dim3(256), 0, c->st, D, c->cfg.integrate);
    LAUNCHCHK(c);
    return FSL_OK;
}

template <int ST>
int enqueue_integration(fsl_ctx *c) {
    Dev &D = c->D;
    const int np = D.np;
    ProfScope ps(c, 4);
    const int ns = c->cfg.n_sub > 0 ? c->cfg.n_sub : 10;
    const double mu = (c->cfg.tau - 0.5) / 3.0;
    int wmask = 0;  // axes whose faces are no-slip walls
    for (int a = 0; a < 3; ++a)
        if (c->cfg.boundary[a] == FSL_NOSLIP) wmask |= 1 << a;
    if (np <= INT_BLOCK_MAX) {  // small tables: every substep in one block
        hipLaunchKernelGGL(k_integrate_block, dim3(1), dim3(1024), 0, c->st, c->G, D, ns, mu, c->cfg.contact_k,
                           c->L.pcap, c->cfg.g[0], c->cfg.g[1], c->cfg.g[2], c->have_prev, wmask);
    } else {
        for (int s = 0; s < ns; ++s) {
            hipLaunchKernelGGL(k_lub, dim3(grid_for(c->L.pcap, 256, 1024)), dim3(256), 0, c->st, c->G, D, mu,
                               c->cfg.contact_k, c->L.pcap);
            hipLaunchKernelGGL(k_substep, dim3(grid_for(np)), dim3(256), 0, c->st, D, c->G, 1.0 / ns,
                               c->cfg.g[0], c->cfg.g[1], c->cfg.g[2], c->have_prev, mu, c->cfg.contact_k, wmask);
        }
    }
    c->have_prev = 1;
    LAUNCHCHK(c);
    return FSL_OK;
}

template <int ST>
int enqueue_coverage_step(fsl_ctx *c) {
    Dev &D = c->D;
    const int np = D.np;
    ProfScope ps(c, 5);
    dim3 pw((np + 3) / 4);
    hipLaunchKernelGGL(k_cov_flag_init, dim3(grid_for(np)), dim3(256), 0, c->st, c->G, D);
    hipLaunchKernelGGL(k_cov_flag_pairs, dim3(grid_for(c->L.pcap, 256, 1024)), dim3(256), 0, c->st, c->G, D,
                       c->L.pcap);
    hipLaunchKernelGGL(k_cov_claim, pw, dim3(256), 0, c->st, c->G, D, 0);
    hipLaunchKernelGGL(k_cov_scan, pw, dim3(256), 0, c->st, c->G, D);
    int rc = enqueue_cover_events<ST>(c, D, D.phi_nxt);
    if (rc) return rc;
    hipLaunchKernelGGL(k_cov_reset, pw, dim3(256), 0, c->st, c->G, D);
    hipLaunchKernelGGL(k_part_mirror, dim3(grid_for(np)), dim3(256), 0, c->st, D);
    LAUNCHCHK(c);
    return FSL_OK;
}

// curvature at the interface cells of the current state (phi_cur, flags)
void enqueue_curvature(fsl_ctx *c) {
    const Layout &L = c->L;
    char *w = c->ws;
    unsigned *tf = (unsigned *)(w + L.ktf);
    int *tl = (int *)(w + L.klist), *tc = (int *)(w + L.kcount);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->st, tc, 1LL, 0);
    hipLaunchKernelGGL(k_curv_mark, dim3(grid_for((c->G.N + 15) / 16, 256, 8192)), dim3(256), 0, c->st, c->G,
                       c->D, tf, tl, tc, L.ktx, L.kty);
    hipLaunchKernelGGL(k_curv_tiles, dim3(std::min(L.nKT, 1024)), dim3(256), 0, c->st, c->G, c->D,
                       (const double *)c->D.phi_cur, tf, (const int *)tl, (const int *)tc, L.ktx, L.kty);
}

// split = 0 leaves out the bubble-splitting test (a state without gas cells: the
// differentiation window)
template <int ST>
int enqueue_steps(fsl_ctx *c, int n, int split) {
    for (int s = 0; s < n; ++s) {
        Dev &D = c->D;
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, c->st, D);
        if (D.wallF) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, D.wallF, 18LL, 0.0);
        if (c->FS.n > 0 && D.wallF)  // face forces from the state at t
            hipLaunchKernelGGL(k_wall_forces<ST>, dim3(grid_for(c->FS.start[c->FS.n], 256, 1024)), dim3(256), 0, c->st,
                               c->G, c->Ph, D, c->FS);
        if (D.kappa) {  // curvature of the interface at t for the Laplace jump
            ProfScope ps(c, 6);
            enqueue_curvature(c);
        }
        if (!c->rhow_ok && D.rhow) {  // densities of the current populations for rho_w
            hipLaunchKernelGGL(k_rhow_fill<ST>, dim3(grid_for(c->G.N, 256, 8192)), dim3(256), 0, c->st, c->G,
                               c->Ph, D, c->stamp - 1);
            c->rhow_ok = 1;
        }
        D.st_prev = c->rhow_ok ? c->stamp - 1 : -1;
        D.st_cur = c->stamp;
        {
            ProfScope ps(c, 0);
            launch_stream_collide<ST>(c, D);
        }
        LAUNCHCHK(c);
        if (++c->stamp >= (1 << 30)) {  // restart the stamps on entries that all read 0
            c->stamp = 1;
            c->rhow_ok = 0;
            if (D.rhow)
                hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->G.S, 256, 8192)), dim3(256), 0, c->st,
                                   (int *)D.rhow, c->G.S, (int)RHOW_NONE);
        } else {
            c->rhow_ok = 1;
        }
        int rc = enqueue_conversions<ST>(c);
        if (rc) return rc;
        if (D.np > 0) {
            rc = enqueue_particles<ST>(c);
            if (rc) return rc;
        }
        rc = enqueue_bubbles<ST>(c, D.phi_nxt, 0);
        if (rc) return rc;
        if (split) {
            rc = enqueue_split<ST>(c, D.phi_nxt, 0);
            if (rc) return rc;
        }
        std::swap(D.fA, D.fB);
        std::swap(D.phi_cur, D.phi_nxt);
    }
    return FSL_OK;
}

// coverage of a whole new particle table (no previous positions): dense scan
template <int ST>
int enqueue_coverage_full(fsl_ctx *c) {
    Dev Dv = c->D;
    Dv.fB = c->D.fA;  // the current state is in lattice A between steps
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, c->st, Dv);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->G.N, 256, 4096)), dim3(256), 0, c->st, Dv.claim,
                       c->G.N, CLAIM_NONE);
    if (Dv.np > 0) hipLaunchKernelGGL(k_cov_claim, dim3((Dv.np + 3) / 4), dim3(256), 0, c->st, c->G, Dv, 1);
    hipLaunchKernelGGL(k_cov_scan_dense, dim3(grid_for(c->G.N, 256, 4096)), dim3(256), 0, c->st, c->G, Dv);
    int rc = enqueue_cover_events<ST>(c, Dv, Dv.phi_cur);
    if (rc) return rc;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->G.N, 256, 4096)), dim3(256), 0, c->st, Dv.claim,
                       c->G.N, CLAIM_NONE);
    LAUNCHCHK(c);
    rc = enqueue_bubbles<ST>(c, Dv.phi_cur, 0);
    if (rc) return rc;
    return enqueue_split<ST>(c, Dv.phi_cur, 1);
}

template <int ST>
int dispatch_init(fsl_ctx *c, const InitGeo &I) {
    Dev &D = c->D;
    long long N = c->G.N;
    int g = grid_for(N, 256, 8192);
    hipLaunchKernelGGL(k_init_geometry, dim3(g), dim3(256), 0, c->st, c->G, D, I);
    hipLaunchKernelGGL(k_init_closure_mark, dim3(g), dim3(256), 0, c->st, c->G, D);
    hipLaunchKernelGGL(k_init_pdf<ST>, dim3(g), dim3(256), 0, c->st, c->G, c->Ph, D, I);
    LAUNCHCHK(c);
    int rc = enqueue_bubbles<ST>(c, D.phi_cur, 1);
    if (rc) return rc;
    return enqueue_split<ST>(c, D.phi_cur, 1);
}

template <typename Fn>
int by_storage(fsl_ctx *c, Fn &&fn) {
    switch (c->cfg.storage) {
    case FSL_STORE_F32: return fn(std::integral_constant<int, ST_F32>{});
    case FSL_STORE_F16S: return fn(std::integral_constant<int, ST_F16>{});
    default: return fn(std::integral_constant<int, ST_BF16>{});
    }
}

int read_error(fsl_ctx *c) {
    unsigned e = 0;
    HIPCHK(c, hipMemcpyAsync(&e, c->D.err, 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (!e) return FSL_OK;
    if (e & ERR_CAP) return fail(c, FSL_E_CAPACITY, "a list, the bubble table or the gas-part list overflowed");
    if (e & ERR_NAN) return fail(c, FSL_E_NUMERIC, "NaN density or velocity");
    if (e & ERR_LG) return fail(c, FSL_E_INVARIANT, "a liquid cell has a gas neighbour");
    if (e & ERR_PART)
        return fail(c, FSL_E_INVARIANT, "a sphere centre left the box or is not finite");
    return fail(c, FSL_E_NUMERIC, "device error");
}


// ---- differentiation window -------------------------------------------------------
double dlambda_minus_dtau(const fsl_config &f) {
    if (f.collision != FSL_TRT) return 1.0 / (f.tau * f.tau);
    // lambda_- = 1 / (Lambda / (1/lambda_+ + 1/2) - 1/2), 1/lambda_+ + 1/2 = 1/2 - tau
    const double a = 0.5 - f.tau;
    const double lm = 1.0 / (f.magic / a - 0.5);
    return -lm * lm * f.magic / (a * a);
}

int window_forward(fsl_ctx *c, int T, int k, double *J) {
    AdjointState &A = c->adj;
    Dev &D = c->D;
    A.ready = 0;
    if (!A.bytes) return fail(c, FSL_E_ARG, "window_forward: no window in the workspace (set window_steps and window_every)");
    if (c->cfg.storage != FSL_STORE_F32) return fail(c, FSL_E_ARG, "window_forward: the window runs on FP32 storage");
    if (T < 1 || k < 1 || T > A.Tmax || k > A.kmax || (T + k - 1) / k > A.ncp)
        return fail(c, FSL_E_ARG, "window_forward: T or k exceed the window reserved in the workspace");
    if (c->cfg.integrate && D.np > 0) return fail(c, FSL_E_ARG, "window_forward: spheres must be kinematic (integrate off)");
    for (int a = 0; a < 3; ++a)
        if (c->cfg.boundary[a] == FSL_FREESLIP) return fail(c, FSL_E_ARG, "window_forward: free-slip faces");
    // the adjoint transposes resting walls only (plain bounce-back)
    if (c->Ph.moving_walls) return fail(c, FSL_E_ARG, "window_forward: moving box faces");
    int *bad = (int *)(A.acc + 32);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, A.acc, 64LL, 0.0);
    hipLaunchKernelGGL(k_win_check, dim3(grid_for(c->G.N, 256, 2048)), dim3(256), 0, c->st, c->G, D, bad);
    int nbad = 0;
    HIPCHK(c, hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (nbad) return fail(c, FSL_E_ARG, "window_forward: the box holds gas or interface cells");
    if (D.np > 0) hipLaunchKernelGGL(k_win_uhat, dim3(grid_for(D.np)), dim3(256), 0, c->st, D, A.uh);
    const size_t st = (size_t)Q * c->G.S * 4, stride = adj_up(st) / 4;
    HIPCHK(c, hipMemcpyAsync(A.cp, D.fA, st, hipMemcpyDeviceToDevice, c->st));
    for (int t = 0; t < T; ++t) {
        int rc = enqueue_steps<ST_F32>(c, 1, 0);  // no gas in the window
        if (rc) return rc;
        if (D.np > 0) hipLaunchKernelGGL(k_win_J, dim3(1), dim3(256), 0, c->st, D, A.acc);
        if ((t + 1) % k == 0 && t + 1 < T)
            HIPCHK(c, hipMemcpyAsync(A.cp + (size_t)((t + 1) / k) * stride, c->D.fA, st, hipMemcpyDeviceToDevice, c->st));
    }
    LAUNCHCHK(c);
    double Jh = 0;
    HIPCHK(c, hipMemcpyAsync(&Jh, A.acc, 8, hipMemcpyDeviceToHost, c->st));
    int rc = read_error(c);
    if (rc) return rc;
    if (J) *J = Jh;
    A.T = T;
    A.k = k;
    A.lp_tau = 1.0 / (c->cfg.tau * c->cfg.tau);
    A.lm_tau = dlambda_minus_dtau(c->cfg);
    A.ready = 1;
    return FSL_OK;
}

int window_backward(fsl_ctx *c, double dJ, double *dJ_dtau, double *dJ_dg) {
    AdjointState &A = c->adj;
    if (!A.ready) return fail(c, FSL_E_ARG, "window_backward: no completed window_forward since the last change of state or parameters");
    const int T = A.T, k = A.k;
    const size_t stride = adj_up((size_t)Q * c->G.S * 4) / 4;
    const long long lat = (long long)Q * c->G.S;
    Dev Dr = c->D;
    Dr.st_prev = Dr.st_cur = -1;  // recomputed segments neither use nor leave stored densities
    Dr.pacc = A.dummy;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)A.nTiles * ADJ_NPART)), dim3(256), 0, c->st, A.part,
                       (long long)A.nTiles * ADJ_NPART, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)c->L.maxP * ACC_COPIES * ACC_STRIDE)), dim3(256), 0, c->st, A.dummy,
                       (long long)c->L.maxP * ACC_COPIES * ACC_STRIDE, 0.0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(lat, 256, 8192)), dim3(256), 0, c->st, (int *)A.mu[0], lat, 0);
    int cur = 0;  // mu[cur] holds mu_{t+1}
    const int nseg = (T + k - 1) / k;
    for (int j = nseg - 1; j >= 0; --j) {
        const int t0 = j * k;
        const int thi = std::min(std::min(T, t0 + k), T - 1);  // last adjoint step using this segment
        if (thi < t0 + 1) continue;
        auto slot = [&](int i) -> float * { return i == 0 ? A.cp + (size_t)j * stride : A.seg + (size_t)(i - 1) * stride; };
        // recompute s_{t0+1} .. s_{thi-1} from the checkpoint s_{t0}
        for (int i = 1; i <= thi - 1 - t0; ++i) {
            Dr.fA = slot(i - 1);
            Dr.fB = slot(i);
            ProfScope ps(c, 0);
            launch_stream_collide<ST_F32>(c, Dr);
        }
        for (int t = thi; t >= t0 + 1; --t) {
            hipLaunchKernelGGL(k_adj_step, dim3(c->nTiles), dim3(256), 0, c->st, c->G, c->Ph, Dr,
                               (const float *)slot(t - 1 - t0), (const float *)A.mu[cur], A.mu[1 - cur],
                               (const float4 *)A.uh, A.part, c->tilesX, c->tilesY, c->nTiles);
            cur ^= 1;
        }
        LAUNCHCHK(c);
    }
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, c->st, (const double *)A.part, A.nTiles, A.acc);
    LAUNCHCHK(c);
    double r[6];
    HIPCHK(c, hipMemcpyAsync(r, A.acc, sizeof r, hipMemcpyDeviceToHost, c->st));
    int rc = read_error(c);
    if (rc) return rc;
    if (dJ_dtau) *dJ_dtau = dJ * (r[1] * A.lp_tau + r[2] * A.lm_tau);
    if (dJ_dg)
        for (int a = 0; a < 3; ++a) dJ_dg[a] = dJ * r[3 + a];
    return FSL_OK;
}

}  // namespace

// ==================================================================================
// Working memory of the contexts made by fsl_init_static: one copy on each device the
// library runs on, held until the process ends and shared by every such context on
// that device.  Host code never names it: it uses the device address looked up once
// per device.
static __device__ __align__(256) unsigned char scratch[FSL_STATIC_SCRATCH_BYTES];

namespace {
constexpr size_t STATIC_STAGE_BYTES = (size_t)8 << 20;  // field staging within the array
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char *scratch_ptr[MAX_DEVICES];             // the array's device address on each device
thread_local char noctx_err[256] = "null context";  // last error of a call without context

int fail_noctx(int code, const char *msg) {
    snprintf(noctx_err, sizeof noctx_err, "%s", msg);
    return code;
}

// the array's address on the current device, looked up on first use
char *static_work(int *code) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        *code = fail_noctx(FSL_E_HIP, "init_static: no current device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char b[200];
            snprintf(b, sizeof b, "init_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
            *code = fail_noctx(FSL_E_HIP, b);
            return nullptr;
        }
        scratch_ptr[dev] = (char *)p;
    }
    return scratch_ptr[dev];
}
}  // namespace

extern "C" {

size_t fsl_workspace_bytes(const fsl_config *cfg) {
    if (!valid(cfg)) return 0;
    return layout_of(cfg).total;
}

// a context on the state d_ws and the working memory d_work, both laid out by L
static int init_ctx(const fsl_config *cfg, const Layout &L, char *d_ws, char *d_work, void *hip_stream,
                    fsl_ctx **out) {
    fsl_ctx *c = new (std::nothrow) fsl_ctx();
    if (!c) return FSL_E_ARG;
    c->cfg = *cfg;
    if (c->cfg.n_sub <= 0) c->cfg.n_sub = 10;
    c->L = L;
    c->st = (hipStream_t)hip_stream;
    c->ws = d_ws;
    c->xs = d_work;
    c->err[0] = 0;
    Geom &G = c->G;
    G.nx = cfg->n[0];
    G.ny = cfg->n[1];
    G.nz = cfg->n[2];
    for (int a = 0; a < 3; ++a) G.per[a] = cfg->boundary[a] == FSL_PERIODIC;
    G.N = (long long)G.nx * G.ny * G.nz;
    G.S = L.S;
    set_phys(c);
    Dev &D = c->D;
    char *w = c->ws, *x = c->xs;
    D.fA = w + L.fA;
    D.fB = w + L.fB;
    D.flags = (uint8_t *)(w + L.flags);
    D.cv = (uint8_t *)(w + L.cv);
    D.phi_cur = (double *)(w + L.phiA);
    D.phi_nxt = (double *)(w + L.phiB);
    D.m = (double *)(w + L.m);
    D.bub = (uint16_t *)(w + L.bub);
    D.pid = (int *)(w + L.pid);
    D.claim = (int *)(w + L.claim);
    D.lF = (int *)(x + L.lF);
    D.lE0 = (int *)(x + L.lE0);
    D.lE = (int *)(x + L.lE);
    D.lNG = (int *)(x + L.lNG);
    D.lNL = (int *)(x + L.lNL);
    D.lCov = (int *)(x + L.lCov);
    D.lUnc = (int *)(x + L.lUnc);
    D.uncRho = (double *)(x + L.uncRho);
    D.uncDec = (int *)(x + L.uncDec);
    D.merges = (int2 *)(x + L.merges);
    D.pairs = (int2 *)(x + L.pairs);
    D.counters = (int *)(w + L.counters);
    D.err = (unsigned *)(w + L.ctl);
    D.ledger = (double *)(w + L.ctl + 8);
    D.ptab = (double *)(w + L.ptab);
    D.pacc = (double *)(w + L.pacc);
    D.pFT = (double *)(w + L.pFT);
    D.pFTp = (double *)(w + L.pFTp);
    D.pFl = (double *)(w + L.pFl);
    D.pmir = (float4 *)(w + L.pmir);
    D.gridStart = (int *)(x + L.gStart);
    D.gridCount = (int *)(x + L.gCount);
    D.gridIdx = (int *)(x + L.gIdx);
    D.btab = (double *)(w + L.btab);
    D.bacc = (double *)(w + L.bacc);
    D.broot = (int *)(w + L.broot);
    D.balive = (int *)(w + L.balive);
    D.rhog = (float *)(w + L.rhog);
    D.kappa = cfg->sigma != 0.0 ? (float *)(w + L.kappa) : nullptr;
    D.wallu = (float *)(w + L.wallu);
    D.wallF = cfg->no_face_forces ? nullptr : (double *)(w + L.wallF);
    D.rhow = cfg->max_particles > 0 ? (unsigned *)(w + L.rhow) : nullptr;
    D.st_prev = D.st_cur = -1;
    c->stamp = 1;
    c->rhow_ok = 0;
    if (D.rhow)  // no density held
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(L.S, 256, 8192)), dim3(256), 0, c->st, (int *)D.rhow, L.S,
                           (int)RHOW_NONE);
    {
        // face velocities (a periodic axis has no face)
        float wv[18];
        for (int a = 0; a < 3; ++a)
            for (int sd = 0; sd < 2; ++sd)
                for (int d = 0; d < 3; ++d)
                    wv[(a * 2 + sd) * 3 + d] = cfg->boundary[a] != FSL_NOSLIP ? 0.0f : (float)cfg->wall_u[a][sd][d];
        if (hipMemcpyAsync(D.wallu, wv, sizeof wv, hipMemcpyHostToDevice, c->st) != hipSuccess ||
            hipStreamSynchronize(c->st) != hipSuccess) {
            delete c;
            return FSL_E_HIP;
        }
    }
    D.cap = L.cap;
    D.capEv = L.capEv;
    D.maxP = L.maxP;
    D.maxB = L.maxB;
    D.np = 0;
    D.nb = L.maxB;  // kernels walk the whole table; unused ids hold no cells
    c->SB = SplitBuf{(int *)(x + L.slab), (int *)(x + L.scomp), (int *)(x + L.scid), (int *)(x + L.spar),
                     (double *)(x + L.svol)};
    c->Rmax = 0;
    c->ncell = 1;
    c->PG = PGrid{{1, 1, 1}, {(double)G.nx, (double)G.ny, (double)G.nz}, 2.0 / 3.0 + 1.0, {G.nx, G.ny, G.nz},
                  {G.per[0], G.per[1], G.per[2]}};
    {
        FaceSet &F = c->FS;
        F.n = 0;
        F.start[0] = 0;
        const long long nn[3] = {G.nx, G.ny, G.nz};
        for (int a = 0; a < 3; ++a) {
            if (cfg->boundary[a] != FSL_NOSLIP) continue;
            for (int sd = 0; sd < 2; ++sd) {
                F.axis[F.n] = a;
                F.side[F.n] = sd;
                F.start[F.n + 1] = F.start[F.n] + nn[a == 0 ? 1 : 0] * nn[a == 2 ? 1 : 2];
                ++F.n;
            }
        }
    }
    c->tilesX = (G.nx + TX - 1) / TX;
    c->tilesY = (G.ny + TY - 1) / TY;
    c->nTiles = c->tilesX * c->tilesY * G.nz;
    c->profiling = 0;
    for (int k = 0; k < NPROF; ++k) { c->prof_ms[k] = 0; c->prof_n[k] = 0; }
    adjoint_bind(c->adj, w + L.win, L.winBytes, cfg->window_steps, cfg->window_every, L.S, L.maxP, L.nTiles);

    // control block, tables, accumulators
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, (double *)(w + L.ctl), 64LL, 0.0);
    if (D.wallF) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, D.wallF, 18LL, 0.0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->st, D.counters, 64LL, 0);
    {
        const int used = cfg->n_gas_spheres + 1;  // bubble ids in use: atmosphere and gas spheres
        if (hipMemcpyAsync(D.counters + C_BUSED, &used, 4, hipMemcpyHostToDevice, c->st) != hipSuccess ||
            hipStreamSynchronize(c->st) != hipSuccess) {
            delete c;
            return FSL_E_HIP;
        }
    }
    if (L.nKT > 0)  // curvature tile flags: zero between steps
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(L.nKT)), dim3(256), 0, c->st, (int *)(w + L.ktf),
                           (long long)L.nKT, 0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)L.maxP * ACC_COPIES * ACC_STRIDE)), dim3(256), 0, c->st,
                       D.pacc, (long long)L.maxP * ACC_COPIES * ACC_STRIDE, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)L.maxP * 6)), dim3(256), 0, c->st, D.pFT,
                       (long long)L.maxP * 6, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)L.maxP * 6)), dim3(256), 0, c->st, D.pFTp,
                       (long long)L.maxP * 6, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)L.maxP * 3)), dim3(256), 0, c->st, D.pFl,
                       (long long)L.maxP * 3, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)L.maxB * B_STRIDE)), dim3(256), 0, c->st, D.btab,
                       (long long)L.maxB * B_STRIDE, 0.0);
    // lattice B starts cleared so that unused cells hold finite values
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((long long)Q * L.S * esize(cfg->storage) / 4, 256, 8192)),
                       dim3(256), 0, c->st, (int *)D.fB, (long long)Q * L.S * esize(cfg->storage) / 4, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((long long)Q * L.S * esize(cfg->storage) / 4, 256, 8192)),
                       dim3(256), 0, c->st, (int *)D.fA, (long long)Q * L.S * esize(cfg->storage) / 4, 0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(L.S, 256, 8192)), dim3(256), 0, c->st, D.phi_nxt, (long long)L.S, 0.0);
    // bubble merge table: every id its own root, before any kernel follows it
    {
        std::vector<int> root(L.maxB), alive(L.maxB, 1);
        for (int b = 0; b < L.maxB; ++b) root[b] = b;
        hipError_t e1 = hipMemcpyAsync(D.broot, root.data(), L.maxB * 4, hipMemcpyHostToDevice, c->st);
        hipError_t e2 = hipMemcpyAsync(D.balive, alive.data(), L.maxB * 4, hipMemcpyHostToDevice, c->st);
        hipError_t e3 = hipStreamSynchronize(c->st);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) { delete c; return FSL_E_HIP; }
    }
    // bubble densities of the initial state in the density slot of the table
    std::vector<double> rho0(D.nb);
    rho0[0] = cfg->rho_g0;
    for (int s = 0; s < cfg->n_gas_spheres; ++s) rho0[s + 1] = cfg->gas_spheres[s][4];
    for (int b = 0; b < D.nb; ++b) {
        hipError_t e = hipMemcpyAsync(D.btab + b * B_STRIDE + B_RHO, &rho0[b], 8, hipMemcpyHostToDevice, c->st);
        if (e != hipSuccess) { delete c; return FSL_E_HIP; }
    }
    InitGeo I{};
    I.zs = cfg->zs;
    I.rho_g0 = cfg->rho_g0;
    I.gz = cfg->g[2];
    I.ns = cfg->n_gas_spheres;
    for (int s = 0; s < I.ns; ++s)
        for (int a = 0; a < 5; ++a) I.sph[s][a] = cfg->gas_spheres[s][a];
    int rc = by_storage(c, [&](auto st) { return dispatch_init<decltype(st)::value>(c, I); });
    if (rc == FSL_OK) rc = read_error(c);
    if (rc != FSL_OK) {
        delete c;
        return rc;
    }
    *out = c;
    return FSL_OK;
}

int fsl_init(const fsl_config *cfg, void *d_ws, size_t bytes, void *hip_stream, fsl_ctx **out) {
    if (!out) return FSL_E_ARG;
    *out = nullptr;
    if (!valid(cfg) || !d_ws || ((uintptr_t)d_ws % ALIGN)) return FSL_E_ARG;
    Layout L = layout_of(cfg);
    if (bytes < L.total) return FSL_E_ARG;
    return init_ctx(cfg, L, (char *)d_ws, (char *)d_ws + L.state, hip_stream, out);
}

int fsl_init_static(const fsl_config *cfg, void *d_state, size_t *bytes, void *hip_stream, fsl_ctx **out) {
    if (out) *out = nullptr;
    if (!bytes) return fail_noctx(FSL_E_ARG, "init_static: bytes is NULL");
    if (!valid(cfg)) return fail_noctx(FSL_E_ARG, "init_static: invalid configuration");
    const Layout L = layout_of(cfg, STATIC_STAGE_BYTES);
    if (L.work > (size_t)FSL_STATIC_SCRATCH_BYTES) {
        char b[200];
        snprintf(b, sizeof b, "init_static: the configuration needs %zu bytes of working memory, above the %zu held",
                 L.work, (size_t)FSL_STATIC_SCRATCH_BYTES);
        return fail_noctx(FSL_E_ARG, b);
    }
    if (!d_state) {
        *bytes = L.state;
        return FSL_OK;
    }
    if (!out || ((uintptr_t)d_state % ALIGN))
        return fail_noctx(FSL_E_ARG, "init_static: out is NULL or the state is not 256-byte aligned");
    if (*bytes < L.state) return fail_noctx(FSL_E_ARG, "init_static: state buffer too small");
    int rc = FSL_OK;
    char *work = static_work(&rc);
    if (!work) return rc;
    return init_ctx(cfg, L, (char *)d_state, work, hip_stream, out);
}

}  // extern "C"

// Steps as a HIP graph: launch-bound small boxes issue about 60 kernels per step.  Two
// steps are captured (lattice and fill-level buffers swap back, and the stored-density
// parities alternate as in eager steps); the host state that the capture advanced is
// restored, and each replay advances it by two steps.
template <int ST>
static int capture_pair(fsl_ctx *c) {
    const Dev D0 = c->D;
    const int stamp0 = c->stamp, rhow0 = c->rhow_ok, prev0 = c->have_prev;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->st, hipStreamCaptureModeRelaxed) != hipSuccess) {
        c->gstate = -1;
        (void)hipGetLastError();
        return FSL_OK;
    }
    const int rc = enqueue_steps<ST>(c, 2);
    const hipError_t e = hipStreamEndCapture(c->st, &g);
    c->D = D0;
    c->stamp = stamp0;
    c->rhow_ok = rhow0;
    c->have_prev = prev0;
    if (rc != FSL_OK || e != hipSuccess || !g || hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        c->gexec = nullptr;
        c->gstate = -1;
        (void)hipGetLastError();
    } else {
        c->gfA = c->D.fA;
    }
    if (g) (void)hipGraphDestroy(g);
    return FSL_OK;
}

static void drop_graph(fsl_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
}

extern "C" {

int fsl_step(fsl_ctx *c, int n) {
    if (!c || n < 0) return FSL_E_ARG;
    return by_storage(c, [&](auto st) -> int {
        constexpr int ST = decltype(st)::value;
        while (n > 0) {
            const bool steady = n >= 8 && c->gstate == 0 && c->st != nullptr && !c->profiling && c->rhow_ok &&
                                (c->D.np == 0 || !c->cfg.integrate || c->have_prev) && c->stamp < (1 << 29);
            if (steady && !c->gexec) {
                const int rc = capture_pair<ST>(c);
                if (rc) return rc;
            }
            if (steady && c->gexec && c->D.fA == c->gfA) {
                const int k = n / 2;
                for (int i = 0; i < k; ++i) HIPCHK(c, hipGraphLaunch(c->gexec, c->st));
                c->stamp += 2 * k;
                n -= 2 * k;
                continue;
            }
            const int rc = enqueue_steps<ST>(c, 1);
            if (rc) return rc;
            --n;
        }
        return FSL_OK;
    });
}

int fsl_particles_set(fsl_ctx *c, int n, const double *x, const double *u, const double *omega,
                      const double *R, const double *rho_p) {
    if (!c || n < 0 || n > c->cfg.max_particles || (n > 0 && (!x || !R || !rho_p)))
        return fail(c, FSL_E_ARG, "particles_set: bad arguments");
    c->rhow_ok = 0;  // the stored densities may not match the populations any more
    drop_graph(c);
    c->adj.ready = 0;
    std::vector<double> tab((size_t)std::max(n, 1) * P_STRIDE, 0.0);
    double Rmax = 0;
    for (int P = 0; P < n; ++P) {
        double *t = &tab[(size_t)P * P_STRIDE];
        for (int a = 0; a < 3; ++a) {
            const double v = c->G.per[a] && std::isfinite(x[3 * P + a]) ? wrap_coord(x[3 * P + a], c->cfg.n[a])
                                                                          : x[3 * P + a];
            t[P_X + a] = v;
            t[P_XOLD + a] = v;
            t[P_U + a] = u ? u[3 * P + a] : 0.0;
            t[P_W + a] = omega ? omega[3 * P + a] : 0.0;
        }
        if (!(R[P] > 0.0) || !(rho_p[P] > 0.0)) return fail(c, FSL_E_ARG, "particles_set: radius and density must be > 0");
        if (R[P] > 60.0) return fail(c, FSL_E_ARG, "particles_set: radius above 60 cells");
        if (!sphere_supported(t + P_X, R[P], c->cfg.n, c->G.per))
            return fail(c, FSL_E_ARG, "particles_set: a centre is not finite or outside a walled axis, or a "
                                      "periodic axis is not longer than 2R + 4");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(t[P_U + a]) || !std::isfinite(t[P_W + a]))
                return fail(c, FSL_E_ARG, "particles_set: a velocity is not finite");
        t[P_R] = R[P];
        t[P_RHO] = rho_p[P];
        Rmax = std::max(Rmax, R[P]);
    }
    if (n > 0) HIPCHK(c, hipMemcpyAsync(c->D.ptab, tab.data(), (size_t)n * P_STRIDE * 8, hipMemcpyHostToDevice, c->st));
    Dev &D = c->D;
    D.np = n;
    c->have_prev = 0;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)c->L.maxP * ACC_COPIES * ACC_STRIDE)), dim3(256), 0, c->st,
                       D.pacc, (long long)c->L.maxP * ACC_COPIES * ACC_STRIDE, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)c->L.maxP * 6)), dim3(256), 0, c->st, D.pFT,
                       (long long)c->L.maxP * 6, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)c->L.maxP * 6)), dim3(256), 0, c->st, D.pFTp,
                       (long long)c->L.maxP * 6, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((long long)c->L.maxP * 3)), dim3(256), 0, c->st, D.pFl,
                       (long long)c->L.maxP * 3, 0.0);
    // lubrication candidate grid: cells no smaller than the largest pair reach
    c->Rmax = Rmax;
    const double reach = 2.0 / 3.0 + 1.0;
    const double cell = std::max(2.0 * Rmax + reach, 3.0);
    long long tot = 1;
    for (int a = 0; a < 3; ++a) {
        c->PG.g[a] = std::max(1, (int)floor(c->cfg.n[a] / cell));
        c->PG.cs[a] = (double)c->cfg.n[a] / c->PG.g[a];
        tot *= c->PG.g[a];
    }
    c->PG.reach = reach;
    if (tot > c->L.ncellMax) return fail(c, FSL_E_ARG, "particles_set: radius too small for the pair grid");
    c->ncell = (int)tot;
    if (n > 0) hipLaunchKernelGGL(k_part_mirror, dim3(grid_for(n)), dim3(256), 0, c->st, D);
    int rc = by_storage(c, [&](auto st) { return enqueue_coverage_full<decltype(st)::value>(c); });
    if (rc) return rc;
    return read_error(c);
}

int fsl_walls_get(fsl_ctx *c, double F[18]) {
    if (!c || !F) return FSL_E_ARG;
    if (!c->D.wallF) return fail(c, FSL_E_ARG, "walls_get: the context was made with no_face_forces");
    HIPCHK(c, hipMemcpyAsync(F, c->D.wallF, 18 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return read_error(c);
}

int fsl_particles_get(fsl_ctx *c, int n, double *x, double *u, double *omega, double *F, double *T) {
    if (!c || n < 0) return FSL_E_ARG;
    if (n > c->D.np) n = c->D.np;
    if (n == 0) return fsl_sync(c);
    std::vector<double> tab((size_t)n * P_STRIDE), ft((size_t)n * 6);
    HIPCHK(c, hipMemcpyAsync(tab.data(), c->D.ptab, tab.size() * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(ft.data(), c->D.pFT, ft.size() * 8, hipMemcpyDeviceToHost, c->st));
    int rc = read_error(c);
    for (int P = 0; P < n; ++P)
        for (int a = 0; a < 3; ++a) {
            if (x) x[3 * P + a] = tab[(size_t)P * P_STRIDE + P_X + a];
            if (u) u[3 * P + a] = tab[(size_t)P * P_STRIDE + P_U + a];
            if (omega) omega[3 * P + a] = tab[(size_t)P * P_STRIDE + P_W + a];
            if (F) F[3 * P + a] = ft[(size_t)P * 6 + a];
            if (T) T[3 * P + a] = ft[(size_t)P * 6 + 3 + a];
        }
    return rc;
}

int fsl_bubbles_get(fsl_ctx *c, fsl_bubble *out, int cap, int *n) {
    if (!c || (cap > 0 && !out)) return FSL_E_ARG;
    const int nt = c->D.nb;
    std::vector<double> tab((size_t)nt * B_STRIDE);
    std::vector<int> root(nt), alive(nt);
    int nb = 0;
    HIPCHK(c, hipMemcpyAsync(tab.data(), c->D.btab, tab.size() * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(root.data(), c->D.broot, nt * 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(alive.data(), c->D.balive, nt * 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(&nb, c->D.counters + C_BUSED, 4, hipMemcpyDeviceToHost, c->st));
    int rc = read_error(c);
    nb = std::min(std::max(nb, 0), nt);
    if (n) *n = nb;
    for (int b = 0; b < nb && b < cap; ++b) {
        int r = b;
        for (int it = 0; it < 64 && root[r] != r; ++it) r = root[r];
        const double *t = &tab[(size_t)r * B_STRIDE];
        fsl_bubble &o = out[b];
        o.id = b;
        o.alive = alive[b] && r == b;
        o.V = t[B_V];
        o.M = t[B_M];
        o.rho_g = t[B_RHO];
        for (int a = 0; a < 3; ++a) o.centroid[a] = t[B_C + a];
        o.V0 = tab[(size_t)b * B_STRIDE + B_V0];
        o.n_gas = (int64_t)llround(t[B_NGAS]);
        o.n_iface = (int64_t)llround(t[B_NIF]);
    }
    return rc;
}

int fsl_bubbles_set(fsl_ctx *c, int n, const double *M, const int *root, const int *alive) {
    if (!c || n < 1 || n > c->L.maxB || !M || !root || !alive) return fail(c, FSL_E_ARG, "bubbles_set: bad arguments");
    c->rhow_ok = 0;  // the stored densities may not match the populations any more
    drop_graph(c);
    for (int b = 0; b < n; ++b)
        if (root[b] < 0 || root[b] >= n) return fail(c, FSL_E_ARG, "bubbles_set: bad root");
    // ids from n on become unused: no mass, their own root, not alive
    const int nt = c->L.maxB;
    std::vector<double> tab((size_t)nt * B_STRIDE);
    std::vector<int> rt(nt), al(nt, 0);
    HIPCHK(c, hipMemcpyAsync(tab.data(), c->D.btab, tab.size() * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (int b = 0; b < nt; ++b) {
        rt[b] = b < n ? root[b] : b;
        al[b] = b < n ? alive[b] : 0;
        if (b >= n) std::fill(&tab[(size_t)b * B_STRIDE], &tab[(size_t)(b + 1) * B_STRIDE], 0.0);
        else tab[(size_t)b * B_STRIDE + B_M] = M[b];
    }
    HIPCHK(c, hipMemcpyAsync(c->D.btab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->D.broot, rt.data(), nt * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->D.balive, al.data(), nt * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->D.counters + C_BUSED, &n, 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    // the lists a step leaves are not read again: the splitting pass below clears no marks
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, c->st, c->D);
    int rc = by_storage(c, [&](auto st) {
        int r = enqueue_bubbles<decltype(st)::value>(c, c->D.phi_cur, 0);
        return r ? r : enqueue_split<decltype(st)::value>(c, c->D.phi_cur, 1);
    });
    if (rc) return rc;
    return read_error(c);
}

int fsl_fields_get(fsl_ctx *c, int field, void *host) {
    if (!c || !host) return FSL_E_ARG;
    const long long N = c->G.N;
    Dev &D = c->D;
    double *stage = (double *)(c->xs + c->L.stage);
    const long long chunk = (long long)(c->L.stageBytes / 8);
    switch (field) {
    case FSL_FIELD_FLAGS: HIPCHK(c, hipMemcpyAsync(host, D.flags, N, hipMemcpyDeviceToHost, c->st)); break;
    case FSL_FIELD_MASS: HIPCHK(c, hipMemcpyAsync(host, D.m, N * 8, hipMemcpyDeviceToHost, c->st)); break;
    case FSL_FIELD_PHI: HIPCHK(c, hipMemcpyAsync(host, D.phi_cur, N * 8, hipMemcpyDeviceToHost, c->st)); break;
    case FSL_FIELD_PID: HIPCHK(c, hipMemcpyAsync(host, D.pid, N * 4, hipMemcpyDeviceToHost, c->st)); break;
    case FSL_FIELD_KAPPA: {
        if (!D.kappa) return fail(c, FSL_E_ARG, "fields_get: no surface tension configured");
        double *stage = (double *)(c->xs + c->L.stage);
        const long long chunk = (long long)(c->L.stageBytes / 8);
        enqueue_curvature(c);  // of the current state: the one the next step uses
        LAUNCHCHK(c);
        std::vector<uint8_t> fl(N);
        HIPCHK(c, hipMemcpyAsync(fl.data(), D.flags, N, hipMemcpyDeviceToHost, c->st));
        for (long long c0 = 0; c0 < N; c0 += chunk) {
            const long long n = std::min(chunk, N - c0);
            hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, c->st, (const float *)D.kappa + c0, n, stage);
            HIPCHK(c, hipMemcpyAsync((double *)host + c0, stage, n * 8, hipMemcpyDeviceToHost, c->st));
            HIPCHK(c, hipStreamSynchronize(c->st));
        }
        for (long long i = 0; i < N; ++i)
            if (fl[i] != IFC) ((double *)host)[i] = 0.0;
        break;
    }
    case FSL_FIELD_BUBBLE_ID:
        for (long long c0 = 0; c0 < N; c0 += chunk / 2) {
            long long n = std::min(chunk / 2, N - c0);
            hipLaunchKernelGGL(k_u16_to_i32, dim3(grid_for(n)), dim3(256), 0, c->st, D.bub + c0, n, (int *)stage);
            HIPCHK(c, hipMemcpyAsync((int *)host + c0, stage, n * 4, hipMemcpyDeviceToHost, c->st));
            HIPCHK(c, hipStreamSynchronize(c->st));
        }
        break;
    case FSL_FIELD_F: {
        int rc = by_storage(c, [&](auto st) -> int {
            constexpr int ST = decltype(st)::value;
            for (int q = 0; q < Q; ++q)
                for (long long c0 = 0; c0 < N; c0 += chunk) {
                    long long n = std::min(chunk, N - c0);
                    hipLaunchKernelGGL(k_pop_to_f64<ST>, dim3(grid_for(n)), dim3(256), 0, c->st, c->G, c->Ph,
                                       (const void *)D.fA, q, c0, n, stage);
                    HIPCHK(c, hipMemcpyAsync((double *)host + (long long)q * N + c0, stage, n * 8,
                                             hipMemcpyDeviceToHost, c->st));
                    HIPCHK(c, hipStreamSynchronize(c->st));
                }
            return FSL_OK;
        });
        if (rc) return rc;
        break;
    }
    default: return fail(c, FSL_E_ARG, "fields_get: unknown field");
    }
    return read_error(c);
}

int fsl_fields_set(fsl_ctx *c, int field, const void *host) {
    if (!c || !host) return FSL_E_ARG;
    c->rhow_ok = 0;  // the stored densities may not match the populations any more
    drop_graph(c);
    c->adj.ready = 0;
    const long long N = c->G.N;
    Dev &D = c->D;
    double *stage = (double *)(c->xs + c->L.stage);
    const long long chunk = (long long)(c->L.stageBytes / 8);
    switch (field) {
    case FSL_FIELD_FLAGS: HIPCHK(c, hipMemcpyAsync(D.flags, host, N, hipMemcpyHostToDevice, c->st)); break;
    case FSL_FIELD_MASS: HIPCHK(c, hipMemcpyAsync(D.m, host, N * 8, hipMemcpyHostToDevice, c->st)); break;
    case FSL_FIELD_PHI: HIPCHK(c, hipMemcpyAsync(D.phi_cur, host, N * 8, hipMemcpyHostToDevice, c->st)); break;
    case FSL_FIELD_PID: HIPCHK(c, hipMemcpyAsync(D.pid, host, N * 4, hipMemcpyHostToDevice, c->st)); break;
    case FSL_FIELD_BUBBLE_ID:
        for (long long c0 = 0; c0 < N; c0 += chunk / 2) {
            long long n = std::min(chunk / 2, N - c0);
            HIPCHK(c, hipMemcpyAsync(stage, (const int *)host + c0, n * 4, hipMemcpyHostToDevice, c->st));
            hipLaunchKernelGGL(k_i32_to_u16, dim3(grid_for(n)), dim3(256), 0, c->st, (const int *)stage, n, D.bub + c0);
            HIPCHK(c, hipStreamSynchronize(c->st));
        }
        break;
    case FSL_FIELD_F: {
        int rc = by_storage(c, [&](auto st) -> int {
            constexpr int ST = decltype(st)::value;
            for (int q = 0; q < Q; ++q)
                for (long long c0 = 0; c0 < N; c0 += chunk) {
                    long long n = std::min(chunk, N - c0);
                    HIPCHK(c, hipMemcpyAsync(stage, (const double *)host + (long long)q * N + c0, n * 8,
                                             hipMemcpyHostToDevice, c->st));
                    hipLaunchKernelGGL(k_pop_from_f64<ST>, dim3(grid_for(n)), dim3(256), 0, c->st, c->G, c->Ph,
                                       D.fA, q, c0, n, (const double *)stage);
                    HIPCHK(c, hipStreamSynchronize(c->st));
                }
            return FSL_OK;
        });
        if (rc) return rc;
        break;
    }
    default: return fail(c, FSL_E_ARG, "fields_set: unknown field");
    }
    return read_error(c);
}

int fsl_mass_get(fsl_ctx *c, double *total, double *ledger) {
    if (!c) return FSL_E_ARG;
    double *out = (double *)(c->ws + c->L.ctl) + 2;
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, out, 2LL, 0.0);
    int rc = by_storage(c, [&](auto st) -> int {
        constexpr int ST = decltype(st)::value;
        hipLaunchKernelGGL(k_mass<ST>, dim3(grid_for(c->G.N, 256, 2048)), dim3(256), 0, c->st, c->G, c->Ph, c->D, out);
        LAUNCHCHK(c);
        return FSL_OK;
    });
    if (rc) return rc;
    double h[3];
    HIPCHK(c, hipMemcpyAsync(h, (double *)(c->ws + c->L.ctl) + 1, 24, hipMemcpyDeviceToHost, c->st));
    rc = read_error(c);
    if (ledger) *ledger = h[0];
    if (total) *total = h[2] + h[1] + h[0];
    return rc;
}

int fsl_sync(fsl_ctx *c) {
    if (!c) return FSL_E_ARG;
    return read_error(c);
}

const char *fsl_error_string(const fsl_ctx *c) {
    if (!c) return noctx_err;
    return c->err;
}

void fsl_destroy(fsl_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (auto &e : c->evlog) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    delete c;
}

int fsl_profile_enable(fsl_ctx *c, int on) {
    if (!c) return FSL_E_ARG;
    drop_graph(c);
    c->profiling = on ? 1 : 0;
    return FSL_OK;
}

int fsl_profile_get(fsl_ctx *c, double *ms, long long *count, int n) {
    if (!c || n < 0) return FSL_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (auto &e : c->evlog) {
        float t = 0;
        if (hipEventElapsedTime(&t, e.second.first, e.second.second) == hipSuccess) {
            c->prof_ms[e.first] += t;
            c->prof_n[e.first] += 1;
        }
        c->evpool.push_back(e.second.first);
        c->evpool.push_back(e.second.second);
    }
    c->evlog.clear();
    for (int k = 0; k < NPROF; ++k) {
        if (ms && k < n) ms[k] = c->prof_ms[k];
        if (count && k < n) count[k] = c->prof_n[k];
        c->prof_ms[k] = 0;
        c->prof_n[k] = 0;
    }
    return NPROF;
}

int fsl_window_forward(fsl_ctx *c, int T, int k, double *J) {
    if (!c) return FSL_E_ARG;
    c->rhow_ok = 0;  // the stored densities may not match the populations any more
    drop_graph(c);
    return window_forward(c, T, k, J);
}

int fsl_window_backward(fsl_ctx *c, double dJ, double *dJ_dtau, double dJ_dg[3]) {
    if (!c) return FSL_E_ARG;
    c->rhow_ok = 0;  // the stored densities may not match the populations any more
    drop_graph(c);
    return window_backward(c, dJ, dJ_dtau, dJ_dg);
}

int fsl_params_set(fsl_ctx *c, double tau, const double g[3]) {
    if (!c || !(tau > 0.5) || !g) return fail(c, FSL_E_ARG, "params_set: tau must exceed 1/2");
    c->rhow_ok = 0;  // the stored densities may not match the populations any more
    drop_graph(c);
    if (c->cfg.collision == FSL_TRT && !(tau != 0.5)) return fail(c, FSL_E_ARG, "params_set: bad tau");
    c->cfg.tau = tau;
    for (int a = 0; a < 3; ++a) c->cfg.g[a] = g[a];
    set_phys(c);
    c->adj.ready = 0;
    return FSL_OK;
}

}  // extern "C"
