// fsl_device.hpp -- device-side definitions of the free-surface LBM library:
// D3Q19 velocity set, population storage formats, workspace pointers and the
// wave-level helpers shared by the kernels.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsl {

// ---- D3Q19 (Sec. 2.1): rest, six axis directions, twelve diagonals -------------
// Order: 0 rest; 1..6 +x,-x,+y,-y,+z,-z; 7..18 (+-1,+-1,0),(+-1,0,+-1),(0,+-1,+-1)
// with sign pairs (+,+),(+,-),(-,+),(-,-).
constexpr int Q = 19;
__host__ __device__ constexpr int cx(int q) {
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
    return v[q];
}
__host__ __device__ constexpr int cy(int q) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
    return v[q];
}
__host__ __device__ constexpr int cz(int q) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    return v[q];
}
__host__ __device__ constexpr int opp(int q) {
    constexpr int v[Q] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return v[q];
}

// directions whose component along axis A (0 x, 1 y, 2 z) equals V, as a bit set
template <int A, int V>
__host__ __device__ constexpr uint32_t dir_mask() {
    uint32_t m = 0;
    for (int q = 1; q < Q; ++q)
        if ((A == 0 ? cx(q) : A == 1 ? cy(q) : cz(q)) == V) m |= 1u << q;
    return m;
}
__host__ __device__ constexpr float wq(int q) {
    return q == 0 ? 1.0f / 3.0f : (q <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr double wqd(int q) {
    return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// cell types
constexpr uint8_t GAS = 0, LIQ = 1, IFC = 2, SOL = 3, WALL = 4;

// device error bits (latched, reported by the host at the next sync)
constexpr unsigned ERR_LG = 1u, ERR_NAN = 2u, ERR_CAP = 4u, ERR_VOL = 8u;
// a sphere centre left the box, or came closer than R + 1 to a periodic face (the
// coverage, pair search and lever arms do not wrap)
constexpr unsigned ERR_PART = 16u;

// conversion marks (one byte per cell, zero outside the conversion phase)
constexpr uint8_t CV_F = 1, CV_E0 = 2, CV_E = 4, CV_NEWG = 8, CV_NEWL = 16;
// a gas cell that left the gas phase in this step (became interface or was covered);
// set until the splitting test at the end of the step
constexpr uint8_t CV_GRM = 32;
// a cell that entered the gas phase in this step (emptied or uncovered as gas)
constexpr uint8_t CV_GAD = 64;

// counters in the control block
enum Counter {
    C_NF = 0, C_NE0, C_NE, C_NNG, C_NNL, C_NMERGE, C_NCOVER, C_NUNCOVER, C_NPAIRS, C_COVALL,
    C_SPLIT,  // splitting pass: 1 = label the gas, 2 = some bubble splits
    C_NCOMP,  // gas components listed by the splitting pass
    C_MERGED, // some bubbles merged in this step: cells are relabelled to their roots
    C_NGEN,   // tiles listed for the general path of the stream-collide step
    C_COUNT
};
// persistent slot (not reset per step): number of bubble ids in use
constexpr int C_BUSED = 63;

// particle table: 16 doubles per particle
// P_OVL: 1 when the coverage update must resolve overlaps through claims (a sphere
// within one cell of another, or one that moved half a cell or more in a step)
enum PSlot { P_X = 0, P_U = 3, P_W = 6, P_R = 9, P_RHO = 10, P_XOLD = 11, P_OVL = 14, P_STRIDE = 16 };
// particle accumulators: F(3) T(3) dm(1) pad -> 8 doubles
constexpr int ACC_STRIDE = 8;
// copies of each particle's accumulator: the waves that touch one sphere add into
// different copies (by block), so their FP64 atomics do not queue on one cache line;
// the force pass sums the copies in a fixed order
constexpr int ACC_COPIES = 8;
__host__ __device__ constexpr long long acc_at(int P, int copy) {
    return ((long long)P * ACC_COPIES + copy) * ACC_STRIDE;
}
// bubble table: 16 doubles per id
enum BSlot { B_M = 0, B_V = 1, B_RHO = 2, B_C = 3, B_V0 = 6, B_NGAS = 7, B_NIF = 8, B_STRIDE = 16 };
// bubble accumulators: V, Vx, Vy, Vz, n_gas, n_iface
constexpr int BACC_STRIDE = 6;

// ---- population storage (form 1) ----------------------------------------------
// Populations are always stored shifted, h_q = f_q - w_q, so that density
// deviations of O(1e-3) never round at O(1).  FP32 stores h directly; the 16-bit
// formats store h * scale (a power of two) with round-to-nearest-even.
enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

template <int S> struct Store;
// enc() gives the stored word, dec() the value it represents, so that the
// value a kernel will read back is known when it writes (rnd = dec(enc(v))).
template <> struct Store<ST_F32> {
    using T = float;
    static __device__ __forceinline__ T enc(float v, float) { return v; }
    static __device__ __forceinline__ float dec(T w, float) { return w; }
    static __device__ __forceinline__ float ld(const T *p, float inv) { return dec(*p, inv); }
    static __device__ __forceinline__ void st(T *p, float v, float sc) { *p = enc(v, sc); }
};
template <> struct Store<ST_F16> {
    using T = _Float16;
    static __device__ __forceinline__ T enc(float v, float sc) { return (_Float16)(v * sc); }
    static __device__ __forceinline__ float dec(T w, float inv) { return (float)w * inv; }
    static __device__ __forceinline__ float ld(const T *p, float inv) { return dec(*p, inv); }
    static __device__ __forceinline__ void st(T *p, float v, float sc) { *p = enc(v, sc); }
};
template <> struct Store<ST_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ T enc(float v, float sc) {
        uint32_t u = __float_as_uint(v * sc);
        if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);  // RNE
        return (uint16_t)(u >> 16);
    }
    static __device__ __forceinline__ float dec(T w, float inv) {
        return __uint_as_float(((uint32_t)w) << 16) * inv;
    }
    static __device__ __forceinline__ float ld(const T *p, float inv) { return dec(*p, inv); }
    static __device__ __forceinline__ void st(T *p, float v, float sc) { *p = enc(v, sc); }
};

// ---- geometry / parameters passed by value ------------------------------------
struct Geom {
    int nx, ny, nz;
    int per[3];
    long long N;  // cells
    long long S;  // plane stride of one population (>= N, multiple of 256)
};

struct Phys {
    float lp, lm;      // lambda_+, lambda_-
    float g[3];
    double eps;        // conversion threshold slack
    float scale, inv;  // 16-bit storage scale and its inverse
    float s6;          // 6 sigma: density form of the Laplace jump 2 sigma kappa (rho = 3 p)
    int moving_walls;  // some face moves (velocities in Dev::wallu) or slips: wall links
                       // then take the general path
    int slip[3];       // the faces of axis a are free-slip
    int open_atm;      // bubble 0 is held at its density (pressure outlet)
    int wide;          // the march's bounce-back pulls take 64-bit offsets (S >= 2^30,
                       // where an offset within a pair of planes leaves 32 bits)
};

struct Dev {
    void *fA, *fB;            // post-collision populations at t (A), next (B)
    uint8_t *flags, *cv;
    double *phi_cur, *phi_nxt, *m;
    uint16_t *bub;
    int *pid, *claim;
    int *lF, *lE0, *lE, *lNG, *lNL;  // conversion lists
    int *lCov, *lUnc;                // coverage events (cell, particle) pairs
    double *uncRho;                  // per uncover event: decided density
    int *uncDec;                     // per uncover event: type | bubble << 8
    int2 *merges, *pairs;
    int *counters;
    unsigned *err;
    double *ledger;                  // [0] ledger
    double *wallF;                   // force on each no-slip face over the last step [18]
    double *ptab, *pacc, *pFT, *pFTp, *pFl; // particles (pFTp: previous step's F, T)
    float4 *pmir;                    // FP32 mirror per particle (PMir: anchor, fraction, u, omega)
    int *gridStart, *gridCount, *gridIdx;
    double *btab, *bacc;
    int *broot, *balive;
    float *rhog;                     // FP32 gas density per bubble id (through root)
    float *kappa;                    // interface curvature (null without surface tension)
    float *wallu;                    // face velocities [axis][low, high][component]
    // density of every liquid and interface cell as computed from its populations by
    // the last launch (null without particles), for Eq. bbrule's rho_w in the next
    // launch: see rhow_word; a launch reads words of stamp st_prev and writes words of
    // stamp st_cur (< 0: none)
    unsigned *rhow;
    int st_prev, st_cur;
    int cap;                         // conversion list capacity
    int capEv;                       // coverage event list capacity
    int maxP, maxB;
    int np, nb;
};

// FP32 mirror of a particle for the kernels that need its rigid-body velocity at a node:
// anchor a = floor(x_P) (exact integers), fraction x_P - a, u_P, omega_P; 12 floats in
// the first three float4 of the particle's 64-byte record
struct PMir {
    float ax, ay, az, fx, fy, fz, ux, uy, uz, wx, wy, wz;
};
__device__ __forceinline__ PMir pmir_load(const float4 *pmir, int P) {
    const float4 *m = pmir + 4LL * P;
    const float4 a = m[0], b = m[1], c = m[2];
    return PMir{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
}

// The sphere positions the library handles: every component finite; on a
// non-periodic axis the centre inside the box (faces at -1/2 and n - 1/2); on a
// periodic axis anywhere (the centre is kept in [0, n) and the sphere acts through its
// nearest images), the axis longer than 2R + 4, so that every node within a link of
// the sphere lies less than n/2 from its centre and the sphere never meets its own
// image.
__host__ __device__ inline bool sphere_supported(const double x[3], double R, const int n[3], const int per[3]) {
    for (int a = 0; a < 3; ++a) {
        const double v = x[a];
        if (!(v == v) || v - v != 0.0) return false;  // NaN or infinite
        if (per[a]) {
            if (!(n[a] > 2.0 * R + 4.0)) return false;
        } else if (!(v >= -0.5 && v <= n[a] - 0.5)) {
            return false;
        }
    }
    return true;
}

// a coordinate along a periodic axis taken into [0, n)
__host__ __device__ inline double wrap_coord(double v, int n) {
    v -= n * floor(v / n);
    return v < n ? v : 0.0;  // v just below 0 can round up to n
}

// a displacement along an axis, the nearest image along a periodic one: [-n/2, n/2)
__host__ __device__ inline double min_img(double d, int n, int per) {
    return per ? d - n * floor(d / n + 0.5) : d;
}

// lever arm x - x_P along one axis from the FP32 mirror: the integer part x - anchor
// taken to its nearest image along a periodic axis (exactly: it is an integer below n
// in size), minus the fraction
__device__ __forceinline__ float mirror_arm(int x, float anchor, float frac, int n, int per) {
    float d = (float)x - anchor;
    if (per) d -= (float)n * rintf(d / (float)n);
    return d - frac;
}

// Stored density word: the FP32 density with its lowest mantissa bit replaced by the
// parity of the stamp of the launch that wrote it (a change of at most one unit in the
// last place); RHOW_NONE (a NaN) where no density is held.  A reader takes the word
// only with the parity of the stamp it expects.
constexpr unsigned RHOW_NONE = 0x7fc00000u;
__device__ __forceinline__ unsigned rhow_word(float rho, int stamp) {
    return (__float_as_uint(rho) & ~1u) | (unsigned)(stamp & 1);
}
__device__ __forceinline__ bool rhow_valid(unsigned w, int stamp) {
    return stamp >= 0 && (w & 0x7f800000u) != 0x7f800000u && (w & 1u) == (unsigned)(stamp & 1);
}

// ---- small helpers ---------------------------------------------------------------
__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// append the lanes with pred to a list: one atomic per wave
__device__ __forceinline__ void wave_append(bool pred, int value, int *list, int *counter,
                                            int cap, unsigned *err) {
    unsigned long long mask = __ballot(pred);
    if (!mask) return;
    int n = __popcll(mask);
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(counter, n);
    base = __shfl(base, leader);
    if (pred) {
        int off = __popcll(mask & ((1ull << lane_id()) - 1ull));
        int slot = base + off;
        if (slot < cap) list[slot] = value;
        else atomicOr(err, ERR_CAP);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace fsl
