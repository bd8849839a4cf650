// k_stream_collide.hpp -- the fused per-cell step of the free-surface LBM:
// pull streaming (Eq. LBE1) with reconstruction of the populations whose source
// is not fluid -- half-way bounce-back at walls, moving-wall bounce-back at
// particle links (Eq. bbrule), the free-surface condition at gas links
// (Eq. fsk) -- then moments, interface mass exchange and fill level
// (Eqs. massExchange, massExchangeb, mass form), TRT collision with Guo forcing
// (Eq. LBE2 with Eq. equilibrium), detection of filled / emptied interface cells
// and the momentum-exchange force and torque (Eqs. netforce, torque,
// momentum_transfer) accumulated per particle in FP64.
//
// One thread per cell, 256-thread blocks covering a 64(x) x 4(y) x 1(z) tile;
// the neighbours' cell types are staged in LDS with a one-cell halo; populations
// are read and written as coalesced SoA rows h[q][z][y][x] (h = f - w).  Tiles
// are handed to the eight XCDs in contiguous ranges so that the row overlap of
// neighbouring tiles stays inside one L2.
#pragma once

#include "fsl_device.hpp"

namespace fsl {

constexpr int TX = 64, TY = 4;

// Per-lane momentum-exchange accumulator for the links of one particle.
// Delta j of a link (Eq. momentum_transfer) is -c_q (h*_qbar + h_q + 2 w_q) in
// shifted populations; the small shifted parts are summed in FP32 and the
// constant parts 2 w_q c_q are counted exactly as integer direction sums (axis
// links 2w = 1/9, diagonal links 2w = 1/18).  All links of a lane share the node
// x; the lever arm x - x_P is split into the integer part x - a (a = floor x_P)
// and the fraction f = x_P - a, so torque sums stay exact integers or small FP32
// values until the wave total is formed in FP64.
struct LinkAcc {
    int P;
    float fs[3];   // sum of -c_q (h*_qbar + h_q)
    int ca[3];     // sum of -c_q over axis links
    int cd[3];     // sum of -c_q over diagonal links
    float dm;      // mass added by moving bounce-back at a liquid cell
    float an[3];   // anchor a of particle P (integers stored exactly)
    float fr[3];   // fraction x_P - a
};

__device__ __forceinline__ void acc_zero(LinkAcc &L) {
    L.fs[0] = L.fs[1] = L.fs[2] = 0.f;
    L.ca[0] = L.ca[1] = L.ca[2] = 0;
    L.cd[0] = L.cd[1] = L.cd[2] = 0;
    L.dm = 0.f;
}

// rare path: one lane's links of a particle straight to the accumulators.  Takes
// the sums by value so that the accumulator never needs an address (it stays in
// registers; only this call, when taken, uses the stack).
__device__ __noinline__ void acc_flush_v(double *pacc, int P, float fs0, float fs1, float fs2, int ca0,
                                         int ca1, int ca2, int cd0, int cd1, int cd2, float dm, float rx,
                                         float ry, float rz) {
    const double F[3] = {(double)fs0 + (ca0 * (1.0 / 9.0) + cd0 * (1.0 / 18.0)),
                         (double)fs1 + (ca1 * (1.0 / 9.0) + cd1 * (1.0 / 18.0)),
                         (double)fs2 + (ca2 * (1.0 / 9.0) + cd2 * (1.0 / 18.0))};
    const double a[7] = {F[0], F[1], F[2], ry * F[2] - rz * F[1], rz * F[0] - rx * F[2],
                         rx * F[1] - ry * F[0], (double)dm};
    double *dst = pacc + acc_at(P, blockIdx.x & (ACC_COPIES - 1));
    for (int k = 0; k < 7; ++k) unsafeAtomicAdd(dst + k, a[k]);
}
__device__ __forceinline__ void acc_flush(const Geom &G, const Dev &D, const LinkAcc &L, int x, int y, int z) {
    if (L.P < 0) return;
    // lever arm x - x_P = (x - a) - f, to the nearest image
    acc_flush_v(D.pacc, L.P, L.fs[0], L.fs[1], L.fs[2], L.ca[0], L.ca[1], L.ca[2], L.cd[0], L.cd[1],
                L.cd[2], L.dm, mirror_arm(x, L.an[0], L.fr[0], G.nx, G.per[0]),
                mirror_arm(y, L.an[1], L.fr[1], G.ny, G.per[1]), mirror_arm(z, L.an[2], L.fr[2], G.nz, G.per[2]));
}

// wave64 sums with DPP: pairs, quads, half-row and row mirrors leave every lane of a
// row of 16 with the row sum; row_bcast:15 on rows 1 and 3 then adds the sum of the
// row before (lane 31 = rows 0+1, lane 63 = rows 2+3), row_bcast:31 on rows 2 and 3
// adds lane 31 (lane 63 = whole wave).  Every lane of the wave must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_add_i(int v) {
    return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add_f(float f) {
    const int v = __float_as_int(f);
    return f + __int_as_float(__builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ int wave_total_i(int v) {
    v = dpp_add_i<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_add_i<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_add_i<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add_i<0x140, 0xF>(v);  // row_mirror
    v = dpp_add_i<0x142, 0xA>(v);  // row_bcast:15
    v = dpp_add_i<0x143, 0xC>(v);  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
// FP32 sums of 32 lanes, the two halves added in FP64
__device__ __forceinline__ double wave_total_f(float f) {
    f = dpp_add_f<0xB1, 0xF>(f);
    f = dpp_add_f<0x4E, 0xF>(f);
    f = dpp_add_f<0x141, 0xF>(f);
    f = dpp_add_f<0x140, 0xF>(f);
    f = dpp_add_f<0x142, 0xA>(f);
    const int v = __float_as_int(f);
    return (double)__int_as_float(__builtin_amdgcn_readlane(v, 31)) +
           (double)__int_as_float(__builtin_amdgcn_readlane(v, 63));
}
// two small integers (|value| < 2^15 after the wave sum) in one 32-bit word
__device__ __forceinline__ int pack2(int hi, int lo) { return hi * 65536 + lo; }
__device__ __forceinline__ void unpack2(int p, int &hi, int &lo) {
    lo = (int)(short)(p & 0xffff);
    hi = (p - lo) / 65536;
}

// wave-level reduction of the lanes' accumulators, segmented by particle id:
// one FP64 atomic per (wave, particle, component).  Lanes must be converged.
// integer arm x - a along one axis, to the nearest image along a periodic axis (the
// nodes next to a sphere lie within R + 2 of its centre, less than n/2)
__device__ __forceinline__ int anchor_arm(int x, float anchor, int n, int per) {
    int d = x - (int)anchor;
    if (per) {
        if (2 * d > n) d -= n;
        else if (2 * d < -n) d += n;
    }
    return d;
}

__device__ __forceinline__ void acc_reduce_wave(const Geom &G, const Dev &D, const LinkAcc &L, int x, int y,
                                                int z) {
    int key = L.P;
    if (!__ballot(key >= 0)) return;
    // lane parts: forces, torques about the anchor, mass
    const int dx = anchor_arm(x, L.an[0], G.nx, G.per[0]), dy = anchor_arm(y, L.an[1], G.ny, G.per[1]),
              dz = anchor_arm(z, L.an[2], G.nz, G.per[2]);
    const float ts0 = dy * L.fs[2] - dz * L.fs[1], ts1 = dz * L.fs[0] - dx * L.fs[2], ts2 = dx * L.fs[1] - dy * L.fs[0];
    const int ta0 = dy * L.ca[2] - dz * L.ca[1], ta1 = dz * L.ca[0] - dx * L.ca[2], ta2 = dx * L.ca[1] - dy * L.ca[0];
    const int td0 = dy * L.cd[2] - dz * L.cd[1], td1 = dz * L.cd[0] - dx * L.cd[2], td2 = dx * L.cd[1] - dy * L.cd[0];
    // direction counts per lane and component are at most 2 (axis) and 4 (diagonal),
    // so their wave sums fit 16 bits; torque counts are bounded by the lever arm
    // (|x - a| <= R + 2 for the nodes next to a sphere of radius R <= 60): the
    // diagonal ones stay below 2^15 in a wave sum, the axis ones far below 2^15
    const int p0 = pack2(L.ca[0], L.cd[0]), p1 = pack2(L.ca[1], L.cd[1]), p2 = pack2(L.ca[2], L.cd[2]);
    const int r0 = pack2(ta0, td0), r1 = pack2(ta1, td1), r2 = pack2(ta2, td2);
    while (true) {
        const unsigned long long act = __ballot(key >= 0);
        if (!act) break;
        const int leader = __ffsll((long long)act) - 1;
        const int k0 = __builtin_amdgcn_readlane(key, leader);
        const bool mine = key == k0;
        const double F0s = wave_total_f(mine ? L.fs[0] : 0.f), F1s = wave_total_f(mine ? L.fs[1] : 0.f),
                     F2s = wave_total_f(mine ? L.fs[2] : 0.f);
        const double T0s = wave_total_f(mine ? ts0 : 0.f), T1s = wave_total_f(mine ? ts1 : 0.f),
                     T2s = wave_total_f(mine ? ts2 : 0.f);
        const double dms = wave_total_f(mine ? L.dm : 0.f);
        const int q0 = wave_total_i(mine ? p0 : 0), q1 = wave_total_i(mine ? p1 : 0), q2 = wave_total_i(mine ? p2 : 0);
        const int s0 = wave_total_i(mine ? r0 : 0), s1 = wave_total_i(mine ? r1 : 0), s2 = wave_total_i(mine ? r2 : 0);
        // the sums are uniform; lanes 0-6 each add one component, so one atomic
        // instruction serves the segment (the fraction is the leader's particle's)
        const float fl0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(L.fr[0]), leader));
        const float fl1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(L.fr[1]), leader));
        const float fl2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(L.fr[2]), leader));
        const int ln = (int)lane_id();
        if (ln < 7) {
            int a0, d0, a1, d1, a2, d2, ta, tb, tc, te, tf, tg;
            unpack2(q0, a0, d0);
            unpack2(q1, a1, d1);
            unpack2(q2, a2, d2);
            unpack2(s0, ta, tb);
            unpack2(s1, tc, te);
            unpack2(s2, tf, tg);
            const double F[3] = {F0s + (a0 * (1.0 / 9.0) + d0 * (1.0 / 18.0)),
                                 F1s + (a1 * (1.0 / 9.0) + d1 * (1.0 / 18.0)),
                                 F2s + (a2 * (1.0 / 9.0) + d2 * (1.0 / 18.0))};
            // sum over lanes of (x - a) x F_lane, then shift the arm by the fraction
            const double Ta[3] = {T0s + (ta * (1.0 / 9.0) + tb * (1.0 / 18.0)),
                                  T1s + (tc * (1.0 / 9.0) + te * (1.0 / 18.0)),
                                  T2s + (tf * (1.0 / 9.0) + tg * (1.0 / 18.0))};
            const double f0 = fl0, f1 = fl1, f2 = fl2;
            const double v = ln == 0 ? F[0]
                           : ln == 1 ? F[1]
                           : ln == 2 ? F[2]
                           : ln == 3 ? Ta[0] - (f1 * F[2] - f2 * F[1])
                           : ln == 4 ? Ta[1] - (f2 * F[0] - f0 * F[2])
                           : ln == 5 ? Ta[2] - (f0 * F[1] - f1 * F[0])
                                     : dms;
            unsafeAtomicAdd(D.pacc + acc_at(k0, blockIdx.x & (ACC_COPIES - 1)) + ln, v);
        }
        if (mine) key = -1;
    }
}

// ---- moments and collision of one cell ------------------------------------------
// Populations come in shifted (h = f - w).  The D3Q19 opposite pairs (q, opp(q)) with
// q < opp(q) are (1,2) (3,4) (5,6) (7,10) (8,9) (11,14) (12,13) (15,18) (16,17); the
// sums below are written as short trees over these pairs so that no long chain of
// dependent additions forms.
struct Moments {
    double drho;    // rho - 1 in FP64 (the FP32 terms are summed without loss that matters)
    float j0, j1, j2;
};
__device__ __forceinline__ Moments cell_moments(const float (&h)[Q]) {
    auto dp = [&](int q, int o) { return (double)h[q] + (double)h[o]; };
    const double a = ((double)h[0] + dp(1, 2)) + (dp(3, 4) + dp(5, 6));
    const double b = (dp(7, 10) + dp(8, 9)) + (dp(11, 14) + dp(12, 13));
    const double c = dp(15, 18) + dp(16, 17);
    const float d1 = h[1] - h[2], d3 = h[3] - h[4], d5 = h[5] - h[6], d7 = h[7] - h[10], d8 = h[8] - h[9];
    const float d11 = h[11] - h[14], d12 = h[12] - h[13], d15 = h[15] - h[18], d16 = h[16] - h[17];
    Moments M;
    M.drho = (a + b) + c;
    M.j0 = ((d1 + d7) + (d8 + d11)) + d12;
    M.j1 = ((d3 + d7) + (d15 + d16)) - d8;
    M.j2 = ((d5 + d11) + (d15 - d16)) - d12;
    return M;
}

// TRT collision with Guo forcing (Eq. LBE2) in shifted form, written to B at cell c.
// The rest population is stored as the exact mass balance of the collision,
// h*_0 = sum_q h_q - sum_{q>0} h*_q with the stored moving values summed in FP64:
// in exact arithmetic it is the same population, and FP32 rounding of the weights
// then cannot bias the mass.  Returns false on a NaN density or velocity.
template <int ST, bool NT = false>
__device__ __forceinline__ bool collide_store(const Phys &Ph, const float (&fi)[Q], const Moments &M,
                                              typename Store<ST>::T *B, long long S, unsigned c, bool store = true) {
    using SS = Store<ST>;
    using T = typename SS::T;
    const float inv = Ph.inv, sc = Ph.scale;
    const float drho = (float)M.drho;
    const float rho = 1.0f + drho;
    const float irho = __builtin_amdgcn_rcpf(rho);
    const float u0 = M.j0 * irho + 0.5f * Ph.g[0];
    const float u1 = M.j1 * irho + 0.5f * Ph.g[1];
    const float u2 = M.j2 * irho + 0.5f * Ph.g[2];
    const float F0 = rho * Ph.g[0], F1 = rho * Ph.g[1], F2 = rho * Ph.g[2];
    const float uu = u0 * u0 + u1 * u1 + u2 * u2;
    const float uF = u0 * F0 + u1 * F1 + u2 * F2;
    const float lp = Ph.lp, lm = Ph.lm;
    const float ap = 1.0f + 0.5f * lp, am = 1.0f + 0.5f * lm;
    double sp[9];
    T out[Q];
    int k = 0;
#pragma unroll
    for (int q = 1; q < Q; q += 1) {
        if (opp(q) < q) continue;
        const int o = opp(q);
        const float w = wq(q);
        const float cu = cx(q) * u0 + cy(q) * u1 + cz(q) * u2;
        const float cF = cx(q) * F0 + cy(q) * F1 + cz(q) * F2;
        const float ep = w * (drho + rho * (4.5f * cu * cu - 1.5f * uu));
        const float em = w * rho * 3.0f * cu;
        const float Fp = w * (-3.0f * uF + 9.0f * cu * cF);
        const float Fm = w * 3.0f * cF;
        const float hp = 0.5f * (fi[q] + fi[o]) - ep;
        const float hm = 0.5f * (fi[q] - fi[o]) - em;
        const float even = lp * hp + ap * Fp, odd = lm * hm + am * Fm;
        const T vq = SS::enc(fi[q] + even + odd, sc), vo = SS::enc(fi[o] + even - odd, sc);
        sp[k] = (double)SS::dec(vq, inv) + (double)SS::dec(vo, inv);
        out[q] = vq;
        out[o] = vo;
        ++k;
    }
    const double sout = (((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]))) + sp[8];
    out[0] = SS::enc((float)(M.drho - sout), sc);
    if (store) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (NT) __builtin_nontemporal_store(out[q], B + q * S + c);
            else B[q * S + c] = out[q];
        }
    }
    return rho == rho && u0 == u0 && u1 == u1 && u2 == u2;
}

// Specular reflection at free-slip faces: the link q of cell (x, y, z) whose source
// lies beyond the faces of the axes marked o* arrives from the cell beside it along
// the wall, with the crossed components of its direction reversed.  Gas there gives
// the free-surface condition (Eq. fsk) with that cell's bubble; a particle node
// gives plain bounce-back (fbb, the cell's own opposite population).
__device__ __forceinline__ int mirror_q(int q, bool ox, bool oy, bool oz) {
    const int ex = ox ? -cx(q) : cx(q), ey = oy ? -cy(q) : cy(q), ez = oz ? -cz(q) : cz(q);
    int r = q;
#pragma unroll
    for (int p = 1; p < Q; ++p)
        if (cx(p) == ex && cy(p) == ey && cz(p) == ez) r = p;
    return r;
}

template <int ST>
__device__ __noinline__ float slip_link(const Geom &G, const Phys &Ph, const Dev &D,
                                        const uint8_t (&tile)[3][TY + 2][TX + 2], int lx, int ly, int x, int y,
                                        int z, int c, int q, bool ox, bool oy, bool oz, float ut0, float ut1,
                                        float ut2, float fbb) {
    using SS = Store<ST>;
    const int dx = ox ? 0 : cx(q), dy = oy ? 0 : cy(q), dz = oz ? 0 : cz(q);
    const uint8_t sf = tile[1 - dz][ly + 1 - dy][lx + 1 - dx];
    const int sp = wrapc(x - dx, G.nx) + G.nx * wrapc(y - dy, G.ny) + G.nx * G.ny * wrapc(z - dz, G.nz);
    if (sf == LIQ || sf == IFC)
        return SS::ld((const typename SS::T *)D.fA + mirror_q(q, ox, oy, oz) * G.S + (unsigned)sp, Ph.inv);
    if (sf == GAS) {
        const int bid = D.bub[sp];
        const float rg = D.rhog[bid < D.maxB ? bid : 0] + (D.kappa ? Ph.s6 * D.kappa[c] : 0.f);
        const float cu = cx(q) * ut0 + cy(q) * ut1 + cz(q) * ut2;
        const float uu = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
        return -fbb + 2.0f * wq(q) * ((rg - 1.0f) + rg * (4.5f * cu * cu - 1.5f * uu));
    }
    return fbb;
}

// One boundary cell of the fused step (a cell with an interface, gas or particle
// next to it, or an interface cell).  INTERIOR: the tile and its halo lie inside
// the box, so a source is the cell index minus a uniform offset (no wrap, no wall).
// Lanes without a cell (inb false) stay in the wave with nothing to do, because the
// wave-level sums below read every lane.  MW: some box face moves (its wall links
// then take the moving-wall form of Eq. bbrule).
template <int ST, bool INTERIOR, bool MW>
__device__ __forceinline__ void sc_cell(const Geom &G, const Phys &Ph, const Dev &D,
                                        const uint8_t (&tile)[3][TY + 2][TX + 2],
                                        const double (&ph)[3][TY + 2][TX + 2], int lx, int ly, int x, int y,
                                        int z, bool inb) {
    using SS = Store<ST>;
    using T = typename SS::T;
    const int nx = G.nx, ny = G.ny, nz = G.nz, nxy = nx * ny;
    const int c = inb ? x + nx * y + nxy * z : 0;
    const uint8_t fl = inb ? tile[1][ly + 1][lx + 1] : WALL;
    const T *A = (const T *)D.fA;
    T *B = (T *)D.fB;
    const long long S = G.S;
    const float inv = Ph.inv;
    auto src = [&](int q) -> int {
        if (INTERIOR) return c - (cx(q) + cy(q) * nx + cz(q) * nxy);
        const int sx = wrapc(x - cx(q), nx), sy = wrapc(y - cy(q), ny), sz = wrapc(z - cz(q), nz);
        return sx + nx * sy + nxy * sz;
    };

    LinkAcc acc;
    acc.P = -1;
    acc_zero(acc);
    acc.an[0] = acc.an[1] = acc.an[2] = 0.f;
    acc.fr[0] = acc.fr[1] = acc.fr[2] = 0.f;
    bool isF = false, isE = false;

    if (fl == LIQ || fl == IFC) {
        uint32_t gm = 0, sm = 0, wm = 0;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const uint8_t sf = tile[1 - cz(q)][ly + 1 - cy(q)][lx + 1 - cx(q)];
            gm |= (uint32_t)(sf == GAS) << q;
            sm |= (uint32_t)(sf == SOL) << q;
            if (!INTERIOR) wm |= (uint32_t)(sf == WALL) << q;
        }
        const uint32_t miss = gm | sm | wm;
        bool needOwn = (fl == IFC) || gm || (MW && wm);
        float fi[Q];
        // density and velocity of this cell at t from its own populations, which are
        // then reloaded where a rule needs one (a compiler barrier keeps the two
        // groups of loads apart, so that both arrays are never live together).  A
        // cell whose only missing links lead to particles needs the density alone
        // (Eq. bbrule): the previous launch stored it when it took this path too.
        float rho_t = 1.0f, ut0 = 0.f, ut1 = 0.f, ut2 = 0.f;
        if (!needOwn && sm) {
            bool have = false;
            if (D.rhow != nullptr && D.st_prev >= 0) {
                const unsigned e = D.rhow[c];
                have = rhow_valid(e, D.st_prev);
                rho_t = __uint_as_float(e);
            }
            needOwn = !have;
        }
        if (needOwn) {
            float fa[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) fa[q] = SS::ld(A + q * S + (unsigned)c, inv);
            const Moments Mt = cell_moments(fa);
            rho_t = 1.0f + (float)Mt.drho;
            const float ir = __builtin_amdgcn_rcpf(rho_t);
            ut0 = Mt.j0 * ir - 0.5f * Ph.g[0];
            ut1 = Mt.j1 * ir - 0.5f * Ph.g[1];
            ut2 = Mt.j2 * ir - 0.5f * Ph.g[2];
        }
        __asm__ volatile("" ::: "memory");
        auto fo = [&](int q) { return SS::ld(A + q * S + (unsigned)c, inv); };
        fi[0] = fo(0);
#pragma unroll
        for (int q = 1; q < Q; ++q)
            if (!((miss >> q) & 1u)) fi[q] = SS::ld(A + q * S + (unsigned)src(q), inv);
        // particle ids of the solid sources: one batch of loads, reduced to the first
        // id P0 and the mask of links whose particle is P0
        int P0 = -1;
        uint32_t same = 0;
        if (sm) {
            int pq[Q];
#pragma unroll
            for (int q = 1; q < Q; ++q) pq[q] = ((sm >> q) & 1u) ? D.pid[src(q)] : -1;
#pragma unroll
            for (int q = Q - 1; q >= 1; --q)
                if ((sm >> q) & 1u) P0 = pq[q];
#pragma unroll
            for (int q = 1; q < Q; ++q) same |= (uint32_t)(((sm >> q) & 1u) && pq[q] == P0) << q;
        }
        if (miss) {
            // rigid-body velocity of the lane's particle at the node: c_q . u_w at
            // the link midpoint x - c_q/2 equals c_q . (u_P + omega x (x - x_P))
            // because c_q . (omega x c_q) = 0, so one velocity serves all links
            float un0 = 0.f, un1 = 0.f, un2 = 0.f;
            auto node_velocity = [&](int P) {
                const PMir m = pmir_load(D.pmir, P);
                acc.an[0] = m.ax; acc.an[1] = m.ay; acc.an[2] = m.az;
                acc.fr[0] = m.fx; acc.fr[1] = m.fy; acc.fr[2] = m.fz;
                const float rx = mirror_arm(x, m.ax, m.fx, G.nx, G.per[0]);
                const float ry = mirror_arm(y, m.ay, m.fy, G.ny, G.per[1]);
                const float rz = mirror_arm(z, m.az, m.fz, G.nz, G.per[2]);
                un0 = m.ux + (m.wy * rz - m.wz * ry);
                un1 = m.uy + (m.wz * rx - m.wx * rz);
                un2 = m.uz + (m.wx * ry - m.wy * rx);
            };
            if ((unsigned)P0 < (unsigned)D.np) {
                acc.P = P0;
                node_velocity(P0);
            }
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const int o = opp(q);
                if (!INTERIOR && ((wm >> q) & 1u)) {
                    // half-way bounce-back; a moving face adds 6 w_q rho_t (c_q . u_w)
                    // (Eq. bbrule), the face being the first crossed no-slip face.  A
                    // link that crosses free-slip faces only reflects specularly.
                    float add = 0.f;
                    if (MW) {
                        const int sx = x - cx(q), sy = y - cy(q), sz = z - cz(q);
                        const bool ox = !G.per[0] && (sx < 0 || sx >= nx);
                        const bool oy = !G.per[1] && (sy < 0 || sy >= ny);
                        const bool oz = !G.per[2] && (sz < 0 || sz >= nz);
                        if ((!ox || Ph.slip[0]) && (!oy || Ph.slip[1]) && (!oz || Ph.slip[2])) {
                            fi[q] = slip_link<ST>(G, Ph, D, tile, lx, ly, x, y, z, c, q, ox, oy, oz, ut0, ut1, ut2,
                                                  fo(o));
                            continue;
                        }
                        int a = 2, sd = sz < 0 ? 0 : 1;
                        if (ox && !Ph.slip[0]) { a = 0; sd = sx < 0 ? 0 : 1; }
                        else if (oy && !Ph.slip[1]) { a = 1; sd = sy < 0 ? 0 : 1; }
                        const float *uw = D.wallu + (a * 2 + sd) * 3;
                        add = 6.0f * wq(q) * rho_t * (cx(q) * uw[0] + cy(q) * uw[1] + cz(q) * uw[2]);
                    }
                    fi[q] = fo(o) + add;
                } else if ((sm >> q) & 1u) {
                    if (!((same >> q) & 1u) || acc.P != P0) {  // another particle (rare)
                        const int P = D.pid[src(q)];
                        if ((unsigned)P >= (unsigned)D.np) {  // inconsistent state: plain wall
                            fi[q] = fo(o);
                            atomicOr(D.err, ERR_LG);
                            continue;
                        }
                        if (P != acc.P) {
                            acc_flush(G, D, acc, x, y, z);
                            acc.P = P;
                            acc_zero(acc);
                            node_velocity(P);
                        }
                    }
                    const float cu = cx(q) * un0 + cy(q) * un1 + cz(q) * un2;
                    const float fin = fo(o) + 6.0f * wq(q) * rho_t * cu;  // Eq. (bbrule)
                    fi[q] = fin;
                    const float s2 = fo(o) + fin;
                    acc.fs[0] -= cx(q) * s2;
                    acc.fs[1] -= cy(q) * s2;
                    acc.fs[2] -= cz(q) * s2;
                    if (q <= 6) {
                        acc.ca[0] -= cx(q); acc.ca[1] -= cy(q); acc.ca[2] -= cz(q);
                    } else {
                        acc.cd[0] -= cx(q); acc.cd[1] -= cy(q); acc.cd[2] -= cz(q);
                    }
                    // the ledger pays the moving-wall mass of liquid cells only: an
                    // interface cell's mass is m, which the link does not change
                    if (fl == LIQ) acc.dm += fin - fo(o);
                } else if ((gm >> q) & 1u) {
                    if (fl == LIQ) atomicOr(D.err, ERR_LG);
                    const int bid = D.bub[src(q)];
                    // Laplace jump p_w = p_g + 2 sigma kappa in density form
                    const float rg = D.rhog[bid < D.maxB ? bid : 0] + (D.kappa ? Ph.s6 * D.kappa[c] : 0.f);
                    const float cu = cx(q) * ut0 + cy(q) * ut1 + cz(q) * ut2;
                    const float uu = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
                    // Eq. (fsk) in shifted form: -h*_qbar + 2 (e+_q(rho_g, u) - w_q)
                    fi[q] = -fo(o) + 2.0f * wq(q) * ((rg - 1.0f) + rg * (4.5f * cu * cu - 1.5f * uu));
                }
            }
        }
        // moments; the density deviation in FP64
        const Moments M = cell_moments(fi);
        const double drho_d = M.drho;
        if (fl == IFC) {
            // Eqs. (massExchange, massExchangeb), mass form, FP64
            const double phx = ph[1][ly + 1][lx + 1];
            double dm = 0.0;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const uint8_t nf = tile[1 + cz(q)][ly + 1 + cy(q)][lx + 1 + cx(q)];
                if (nf == LIQ || nf == IFC) {
                    double d = (double)fi[opp(q)] - (double)fo(q);
                    if (nf == IFC) d *= 0.5 * (ph[1 + cz(q)][ly + 1 + cy(q)][lx + 1 + cx(q)] + phx);
                    dm += d;
                } else if (MW && !INTERIOR && nf == WALL) {
                    // across free-slip faces the partner is the cell beside this one
                    // along the wall: its reflected population arrives as fi[opp(q)]
                    const int ex = x + cx(q), ey = y + cy(q), ez = z + cz(q);
                    const bool ox = !G.per[0] && (ex < 0 || ex >= nx);
                    const bool oy = !G.per[1] && (ey < 0 || ey >= ny);
                    const bool oz = !G.per[2] && (ez < 0 || ez >= nz);
                    if ((!ox || Ph.slip[0]) && (!oy || Ph.slip[1]) && (!oz || Ph.slip[2])) {
                        const int dx = ox ? 0 : cx(q), dy = oy ? 0 : cy(q), dz = oz ? 0 : cz(q);
                        const uint8_t pf = tile[1 + dz][ly + 1 + dy][lx + 1 + dx];
                        if (pf == LIQ || pf == IFC) {
                            double d = (double)fi[opp(q)] - (double)fo(q);
                            if (pf == IFC) d *= 0.5 * (ph[1 + dz][ly + 1 + dy][lx + 1 + dx] + phx);
                            dm += d;
                        }
                    }
                }
            }
            const double mnew = D.m[c] + dm;
            D.m[c] = mnew;
            const double phin = mnew / (1.0 + drho_d);
            D.phi_nxt[c] = phin;
            isF = phin >= 1.0 - Ph.eps;
            isE = !isF && phin <= Ph.eps;
        }

        // the density of the populations stored below (the collision keeps the
        // mass), for the next launch
        if (D.rhow != nullptr && D.st_cur >= 0) D.rhow[c] = rhow_word(1.0f + (float)drho_d, D.st_cur);
        if (!collide_store<ST>(Ph, fi, M, B, S, (unsigned)c)) atomicOr(D.err, ERR_NAN);
    }

    wave_append(isF, c, D.lF, D.counters + C_NF, D.cap, D.err);
    wave_append(isE, c, D.lE0, D.counters + C_NE0, D.cap, D.err);
    if (D.np > 0) acc_reduce_wave(G, D, acc, x, y, z);
}

// Cell types of a 64 x 4 x 1 tile and its one-cell halo (WALL outside a
// non-periodic face): 3 x 6 rows of 66 bytes, 1,188 bytes, at most five per thread.
// All loads of a thread are issued before the first is written, so that their
// latencies overlap.  The caller syncs.
__device__ __forceinline__ void stage_flag_tile(const Geom &G, const uint8_t *flags,
                                                uint8_t (&tile)[3][TY + 2][TX + 2], int x0, int y0,
                                                int z, bool interior) {
    constexpr int NE = 3 * (TY + 2) * (TX + 2);
    constexpr int K = (NE + 255) / 256;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    uint8_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = threadIdx.x + 256 * k;
        v[k] = WALL;
        if (e < NE) {
            const int lx = e % (TX + 2), r = e / (TX + 2);
            const int ly = r % (TY + 2), lz = r / (TY + 2);
            int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z + lz - 1;
            if (interior) {
                v[k] = flags[gx + (long long)nx * (gy + (long long)ny * gz)];
            } else {
                bool ok = true;
                if (gx < 0 || gx >= nx) { if (G.per[0]) gx = wrapc(gx, nx); else ok = false; }
                if (gy < 0 || gy >= ny) { if (G.per[1]) gy = wrapc(gy, ny); else ok = false; }
                if (gz < 0 || gz >= nz) { if (G.per[2]) gz = wrapc(gz, nz); else ok = false; }
                if (ok) v[k] = flags[gx + (long long)nx * (gy + (long long)ny * gz)];
            }
        }
    }
    uint8_t *flat = &tile[0][0][0];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = threadIdx.x + 256 * k;
        if (e < NE) flat[e] = v[k];
    }
}

// tile t of a launch over the tiles of the box: XCD-contiguous ranges when the tile
// count allows
__device__ __forceinline__ int tile_of_block(int b, int nTiles) {
    return (nTiles % 8 == 0) ? (b % 8) * (nTiles / 8) + b / 8 : b;
}

// Exact integer counts of the constant parts 2 w_q c_q of Delta j (Eq.
// momentum_transfer in shifted populations), in units of 1/18 (axis links 2,
// diagonal links 1): three components packed 10 bits apart, each |v| < 512
__host__ __device__ constexpr int kpack(int a, int b, int c) { return a + 1024 * b + 1048576 * c; }
__device__ __forceinline__ int sext10(int v) { return v >= 512 ? v - 1024 : v; }
__device__ __forceinline__ void kunpack(int p, int &a, int &b, int &c) {
    a = sext10(p & 1023);
    p = (p - a) / 1024;
    b = sext10(p & 1023);
    c = (p - b) / 1024;
}
__device__ __forceinline__ int kconst(int q) {
    const int m = q <= 6 ? 2 : 1;
    return kpack(-cx(q) * m, -cy(q) * m, -cz(q) * m);
}

// ---- the marching kernel ------------------------------------------------------------
// A block takes a 64 x 4 column of cells through nzc consecutive planes (NZC, fewer on
// small boxes).  Each wave
// takes one row of the column; each lane one x.  The cell types and the particle ids
// of the particle nodes of four planes (z-1 .. z+2) stay in LDS rings, refilled one
// plane ahead from loads issued a plane earlier, so that a plane costs one barrier.
constexpr int NZC = 16;
#ifndef WPE_MARCH
#define WPE_MARCH 4
#endif
constexpr int HX = TX + 2, HY = TY + 2;  // a staged plane: 6 rows of 66 cells

// bitmasks of a staged row (cells x0-1 .. x0+64): bit l of a "3" mask is set when one
// of the cells x-1, x, x+1 of lane l is of the kind, of a "1" mask when the cell x is.
// nf: not liquid or interface (gas, particle node, wall); bad: gas and, with moving
// or slipping faces, walls.
enum { MK_NF3 = 0, MK_NF1, MK_BAD3, MK_BAD1, MK_N };

struct MarchLds {
    uint8_t ft[4][HY][HX];              // cell types, slot z & 3
    int pt[4][HY][HX];                  // particle ids (particle nodes only), slot z & 3
    unsigned long long mk[4][MK_N][HY]; // row masks, slot z & 3
    int genflag[2];                     // the plane holds cells for the general path
    // each lane's link sums for one particle over the planes of the march: force and
    // torque about the particle's centre (Eqs. netforce, torque, momentum_transfer) in
    // FP64, and the mass that moving bounce-back added (paid by the ledger)
    double acc[7][256];
    int accP[256];
};

// Staging of the ring: wave wv loads rows wv and wv + 4 (waves 0, 1) of a plane, lane l
// the cell x0-1+l and lanes 0, 1 also x0+63+l.  The lane's column and row offsets
// (periodic faces wrapped, -1 beyond a non-periodic face) are fixed for the march; a
// plane adds a uniform offset.  Indices fit 32 bits (the box holds < 2^31 cells).
struct StageIdx {
    int xm, xe;  // column of the lane's main and extra cell, or -1
    int yo[2];   // (row y) * nx of the wave's two rows, or -1
};
__device__ __forceinline__ int stage_wrap(int v, int n, int per) {
    return (v >= 0 && v < n) ? v : (per ? wrapc(v, n) : -1);
}
__device__ __forceinline__ StageIdx stage_idx(const Geom &G, int x0, int y0) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    StageIdx s;
    s.xm = stage_wrap(x0 - 1 + lane, G.nx, G.per[0]);
    s.xe = lane < 2 ? stage_wrap(x0 + 63 + lane, G.nx, G.per[0]) : -1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = wv + 4 * k;
        const int yy = r < HY ? stage_wrap(y0 - 1 + r, G.ny, G.per[1]) : -1;
        s.yo[k] = yy >= 0 ? yy * G.nx : -1;
    }
    return s;
}
// the plane offset z * nx * ny, or -1 beyond a non-periodic face
__device__ __forceinline__ int stage_zo(const Geom &G, int z) {
    const int zz = stage_wrap(z, G.nz, G.per[2]);
    return zz >= 0 ? zz * G.nx * G.ny : -1;
}

// the rows of a plane that wave wv stages
struct RowPre {
    int f[2];  // cell types: lane's main cell (bits 0-7), extra cell (bits 8-15)
    int p[2];  // particle id of the main cell (particle nodes), -1 otherwise
    int pe[2]; // ... of the extra cell
};

__device__ __forceinline__ void pre_flags(const uint8_t *flags, const StageIdx &I, RowPre &R, int zo) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const bool row = I.yo[k] >= 0 && zo >= 0;
        const int v = (row && I.xm >= 0) ? flags[I.xm + I.yo[k] + zo] : WALL;
        const int e = (row && I.xe >= 0) ? flags[I.xe + I.yo[k] + zo] : WALL;
        R.f[k] = v | (e << 8);
    }
}

// particle ids of the particle nodes among the rows whose types R holds; -1 at every
// other cell, and a particle node without a valid id reads as INT_MAX (an id that no
// particle has, so its links report the inconsistency)
__device__ __forceinline__ int ring_id(int p) { return p >= 0 ? p : 0x7fffffff; }
__device__ __forceinline__ void pre_pids(const int *pid, const StageIdx &I, RowPre &R, int zo) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        R.p[k] = (R.f[k] & 0xff) == SOL ? ring_id(pid[I.xm + I.yo[k] + zo]) : -1;
        R.pe[k] = ((R.f[k] >> 8) & 0xff) == SOL ? ring_id(pid[I.xe + I.yo[k] + zo]) : -1;
    }
}

// write the staged rows of a plane into ring slot sl and form their masks (ballots
// over the wave's registers); the caller syncs before the slot is read
__device__ __forceinline__ void pre_store(MarchLds &L, const RowPre &R, int sl, bool wall_bad) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = wv + 4 * k;
        if (r >= HY) continue;  // uniform over the wave
        const int a = R.f[k] & 0xff, b = (R.f[k] >> 8) & 0xff;
        L.ft[sl][r][lane] = (uint8_t)a;
        L.pt[sl][r][lane] = R.p[k];
        if (lane < 2) {
            L.ft[sl][r][64 + lane] = (uint8_t)b;
            L.pt[sl][r][64 + lane] = R.pe[k];
        }
        const bool hl = lane < 2;
        const unsigned long long nlo = __ballot(a != LIQ && a != IFC);
        const unsigned long long nhi = __ballot(hl && b != LIQ && b != IFC) & 3ull;
        const unsigned long long blo = __ballot(a == GAS || (wall_bad && a == WALL));
        const unsigned long long bhi = __ballot(hl && (b == GAS || (wall_bad && b == WALL))) & 3ull;
        if (lane == 0) {
            const unsigned long long n1 = (nlo >> 1) | (nhi << 63), n2 = (nlo >> 2) | (nhi << 62);
            const unsigned long long b1 = (blo >> 1) | (bhi << 63), b2 = (blo >> 2) | (bhi << 62);
            L.mk[sl][MK_NF3][r] = nlo | n1 | n2;
            L.mk[sl][MK_NF1][r] = n1;
            L.mk[sl][MK_BAD3][r] = blo | b1 | b2;
            L.mk[sl][MK_BAD1][r] = b1;
        }
    }
}

// D3Q19 neighbourhood of lane l in row ly of the plane in slot s0 (planes z-1, z+1 in
// slots sm, sp): the OR of the masks of kind K3 (x-1..x+1) and K1 (x) over the 3 x 3
// square of the plane and the plus shape of the planes beside it
template <int K3, int K1>
__device__ __forceinline__ bool nbr_any(const MarchLds &L, int sm, int s0, int sp, int ly, int lx) {
    const unsigned long long m = L.mk[s0][K3][ly] | L.mk[s0][K3][ly + 1] | L.mk[s0][K3][ly + 2] |
                                 L.mk[sm][K3][ly + 1] | L.mk[sp][K3][ly + 1] | L.mk[sm][K1][ly] |
                                 L.mk[sm][K1][ly + 2] | L.mk[sp][K1][ly] | L.mk[sp][K1][ly + 2];
    return (m >> lx) & 1ull;
}

__device__ __forceinline__ void lds_add(double *p, double v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// one lane's sums (in LDS) straight to its particle (a lane that moves on to another
// particle), then cleared
__device__ __forceinline__ void macc_atomic(const Dev &D, MarchLds &L, int t) {
    double *dst = D.pacc + acc_at(L.accP[t], blockIdx.x & (ACC_COPIES - 1));
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        unsafeAtomicAdd(dst + k, L.acc[k][t]);
        L.acc[k][t] = 0.0;
    }
}

// FP64 wave sum with DPP on the two 32-bit halves (same pattern as wave_total_f)
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
    return v + __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_total_d(double v) {
    v = dpp_add_d<0xB1, 0xF>(v);
    v = dpp_add_d<0x4E, 0xF>(v);
    v = dpp_add_d<0x141, 0xF>(v);
    v = dpp_add_d<0x140, 0xF>(v);
    v = dpp_add_d<0x142, 0xA>(v);
    v = dpp_add_d<0x143, 0xC>(v);
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// the lanes' remaining sums at the end of a march, segmented by particle: one FP64
// atomic instruction per (wave, particle).  Every lane of the wave must be active.
__device__ __forceinline__ void macc_wave_flush(const Dev &D, const MarchLds &L) {
    const int t = threadIdx.x;
    int key = L.accP[t];
    const double a0 = L.acc[0][t], a1 = L.acc[1][t], a2 = L.acc[2][t], a3 = L.acc[3][t], a4 = L.acc[4][t],
                 a5 = L.acc[5][t], a6 = L.acc[6][t];
    while (true) {
        const unsigned long long act = __ballot(key >= 0);
        if (!act) break;
        const int leader = __ffsll((long long)act) - 1;
        const int k0 = __builtin_amdgcn_readlane(key, leader);
        const bool mine = key == k0;
        const double s0 = wave_total_d(mine ? a0 : 0.0), s1 = wave_total_d(mine ? a1 : 0.0),
                     s2 = wave_total_d(mine ? a2 : 0.0), s3 = wave_total_d(mine ? a3 : 0.0),
                     s4 = wave_total_d(mine ? a4 : 0.0), s5 = wave_total_d(mine ? a5 : 0.0),
                     s6 = wave_total_d(mine ? a6 : 0.0);
        const int ln = (int)lane_id();
        if (ln < 7) {
            const double v = ln == 0 ? s0 : ln == 1 ? s1 : ln == 2 ? s2 : ln == 3 ? s3 : ln == 4 ? s4 : ln == 5 ? s5 : s6;
            unsafeAtomicAdd(D.pacc + acc_at(k0, blockIdx.x & (ACC_COPIES - 1)) + ln, v);
        }
        if (mine) key = -1;
    }
}

// density of a cell's own populations (a cell whose density from the launch before
// is not stored): kept out of line, so that its loads never share registers with
// the pulled populations
template <int ST>
__device__ __noinline__ float own_density(const void *A, long long S, int c, float inv) {
    using SS = Store<ST>;
    const typename SS::T *p = (const typename SS::T *)A;
    float fa[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) fa[q] = SS::ld(p + q * S + (unsigned)c, inv);
    return 1.0f + (float)cell_moments(fa).drho;
}

// Source offsets of a lane's pulls: the cell x - c_q is c + dx[c_x] + dy[c_y] + dz[c_z]
// with dx[1] the step to x-1 and dx[-1] the step to x+1 (and so on), wrapped at periodic
// faces.  Beyond a non-periodic face the step is 0: that pull reads the cell itself,
// and the link takes bounce-back instead.  dx is per lane, dy per wave row, dz per plane.
struct SrcOff {
    int xm, xp, ym, yp, zm, zp;
};
template <int Q_>
__device__ __forceinline__ int src_off(const SrcOff &o) {
    return (cx(Q_) == 1 ? o.xm : cx(Q_) == -1 ? o.xp : 0) + (cy(Q_) == 1 ? o.ym : cy(Q_) == -1 ? o.yp : 0) +
           (cz(Q_) == 1 ? o.zm : cz(Q_) == -1 ? o.zp : 0);
}
__device__ __forceinline__ int step_to(int v, int d, int n, int per, int stride) {
    const int w = v + d;
    if (w >= 0 && w < n) return d * stride;
    return per ? (wrapc(w, n) - v) * stride : 0;
}

// One cell of a row in the marching pass: a liquid cell whose neighbours are liquid,
// interface, particle nodes or resting walls (act).  Pull streaming (Eq. LBE1); a
// source beyond a resting wall gives half-way bounce-back, a particle node the
// moving-wall rule (Eq. bbrule) with rho_w the density of the cell at t and u_w the
// particle's rigid-body velocity, and its momentum exchange (Eqs. netforce, torque,
// momentum_transfer) joins the lane's sums; then the collision (Eq. LBE2).  Lanes with
// store set and act clear (gas and particle nodes of the row) write values that no
// rule reads, so that every row of every population is written whole and once;
// interface cells and lanes outside the box leave their words to the general path.
template <int ST, bool PER>
__device__ __forceinline__ void march_cell(const Geom &G, const Phys &Ph, const Dev &D, MarchLds &L,
                                           int sm1, int s0, int sp1, int lx, int ly, int x, int y, int z, int c,
                                           const SrcOff &so, bool act, bool store, bool nbnf, const void *Av,
                                           void *Bv, long long S, const StageIdx &SI, RowPre &R, int zo2,
                                           int &curP) {
    using SS = Store<ST>;
    using T = typename SS::T;
    const T *A = (const T *)Av;
    T *B = (T *)Bv;
    const float inv = Ph.inv;
    auto slot = [&](int q) { return cz(q) == 1 ? sm1 : (cz(q) == -1 ? sp1 : s0); };  // plane z - c_z
    // bounce-back sources: particle nodes (sm, from the staged cell types) and resting
    // walls (wm: the sources beyond a non-periodic face, from the cell's position)
    uint32_t sm = 0, wm = 0;
    if (act) {
        if (!G.per[0]) wm |= (x == 0 ? dir_mask<0, 1>() : 0u) | (x == G.nx - 1 ? dir_mask<0, -1>() : 0u);
        if (!G.per[1]) wm |= (y == 0 ? dir_mask<1, 1>() : 0u) | (y == G.ny - 1 ? dir_mask<1, -1>() : 0u);
        if (!G.per[2]) wm |= (z == 0 ? dir_mask<2, 1>() : 0u) | (z == G.nz - 1 ? dir_mask<2, -1>() : 0u);
        if (nbnf) {
#pragma unroll
            for (int q = 1; q < Q; ++q) sm |= (uint32_t)(L.ft[slot(q)][ly + 1 - cy(q)][lx + 1 - cx(q)] == SOL) << q;
        }
    }
    const uint32_t bb = sm | wm;
    // the particle P of the particle-node links and whether some link leads to another:
    // over the 18 staged ids (-1 at every cell that is no particle node) the smallest as
    // an unsigned value and the largest as a signed one agree exactly when every
    // particle node among them has the same id
    int P = -1;
    bool multi = false;
    if (sm) {
        unsigned pmin = 0xffffffffu;
        int pmax = -1;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const int p = L.pt[slot(q)][ly + 1 - cy(q)][lx + 1 - cx(q)];
            pmin = min(pmin, (unsigned)p);
            pmax = max(pmax, p);
        }
        P = (int)pmin;
        multi = (int)pmin != pmax;
    }
    const bool okP = (unsigned)P < (unsigned)D.np;
    // rho_w of Eq. bbrule: the density of this cell at t, as the launch before stored it
    unsigned e = RHOW_NONE;
    if (sm && D.rhow != nullptr && D.st_prev >= 0) e = D.rhow[c];
    PMir pm{};
    if (sm && okP) pm = pmir_load(D.pmir, P);
    // pulls; a bounce-back link takes the cell's own opposite population instead (the
    // source address is selected, so every population is one load)
    float fi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) fi[q] = 0.f;
    if (act) {  // lanes without a liquid cell load nothing
        if (__ballot(bb) == 0ull) {
#define FSL_PULL(QQ) fi[QQ] = SS::ld(A + QQ * S + (unsigned)(c + src_off<QQ>(so)), inv);
            FSL_PULL(0) FSL_PULL(1) FSL_PULL(2) FSL_PULL(3) FSL_PULL(4) FSL_PULL(5) FSL_PULL(6)
            FSL_PULL(7) FSL_PULL(8) FSL_PULL(9) FSL_PULL(10) FSL_PULL(11) FSL_PULL(12) FSL_PULL(13)
            FSL_PULL(14) FSL_PULL(15) FSL_PULL(16) FSL_PULL(17) FSL_PULL(18)
#undef FSL_PULL
        } else if (!Ph.wide) {
            // the planes q and opp(q) share the base of the lower one; the lane's offset
            // from it (at most 4 S) stays within 32 bits
            const unsigned S32 = (unsigned)S;
            fi[0] = SS::ld(A + (unsigned)c, inv);
#define FSL_PULL(QQ)                                                                                      \
    {                                                                                                     \
        constexpr int lo_ = QQ < opp(QQ) ? QQ : opp(QQ);                                                  \
        const int so_ = src_off<QQ>(so);                                                                  \
        const unsigned m_ = (unsigned)__builtin_amdgcn_sbfe((int)bb, QQ, 1); /* all ones on a link */     \
        unsigned o_ = (unsigned)(QQ - lo_) * S32 + (unsigned)(c + so_) +                                   \
                      (((unsigned)(opp(QQ) - QQ) * S32 - (unsigned)so_) & m_);                            \
        __asm__("" : "+v"(o_));                                                                           \
        fi[QQ] = SS::ld(A + lo_ * S + o_, inv);                                                           \
    }
            FSL_PULL(1) FSL_PULL(2) FSL_PULL(3) FSL_PULL(4) FSL_PULL(5) FSL_PULL(6)
            FSL_PULL(7) FSL_PULL(8) FSL_PULL(9) FSL_PULL(10) FSL_PULL(11) FSL_PULL(12) FSL_PULL(13)
            FSL_PULL(14) FSL_PULL(15) FSL_PULL(16) FSL_PULL(17) FSL_PULL(18)
#undef FSL_PULL
        } else {
            fi[0] = SS::ld(A + (unsigned)c, inv);
#define FSL_PULL(QQ)                                                                                       \
    {                                                                                                      \
        const bool b_ = (bb >> QQ) & 1u;                                                                   \
        fi[QQ] = SS::ld((b_ ? A + opp(QQ) * S : A + QQ * S) + (unsigned)(b_ ? c : c + src_off<QQ>(so)), inv); \
    }
            FSL_PULL(1) FSL_PULL(2) FSL_PULL(3) FSL_PULL(4) FSL_PULL(5) FSL_PULL(6)
            FSL_PULL(7) FSL_PULL(8) FSL_PULL(9) FSL_PULL(10) FSL_PULL(11) FSL_PULL(12) FSL_PULL(13)
            FSL_PULL(14) FSL_PULL(15) FSL_PULL(16) FSL_PULL(17) FSL_PULL(18)
#undef FSL_PULL
        }
    }
    // particle ids of plane z+2 for the ring (its cell types were loaded before)
    pre_pids(D.pid, SI, R, zo2);
    if (sm) {
        const float rho_t = rhow_valid(e, D.st_prev) ? __uint_as_float(e) : own_density<ST>(Av, S, c, inv);
        const int t = threadIdx.x;
        // the links mk of particle Pk (mirror m): moving-wall rule and momentum exchange.
        // With rho u = rho_w u_w the link adds a_q = 6 w_q c_q . rho u to the bounced
        // population, and Delta j = -c_q (h*_qbar + h_q + 2 w_q) with h_q = h*_qbar + a_q.
        auto particle_links = [&](int Pk, uint32_t mk, const PMir &m) {
            if (Pk != curP) {  // the lane's sums move on to another particle
                if (curP >= 0) macc_atomic(D, L, t);
                curP = Pk;
                L.accP[t] = Pk;
            }
            // rigid-body velocity at the node: c_q . u_w at the link midpoint equals
            // c_q . (u_P + omega x (x - x_P)) because c_q . (omega x c_q) = 0
            // nearest image only when the box has periodic axes (a compile-time case)
            const float rx = mirror_arm(x, m.ax, m.fx, G.nx, PER && G.per[0]),
                        ry = mirror_arm(y, m.ay, m.fy, G.ny, PER && G.per[1]),
                        rz = mirror_arm(z, m.az, m.fz, G.nz, PER && G.per[2]);
            const float ru0 = rho_t * (m.ux + (m.wy * rz - m.wz * ry));
            const float ru1 = rho_t * (m.uy + (m.wz * rx - m.wx * rz));
            const float ru2 = rho_t * (m.uz + (m.wx * ry - m.wy * rx));
            // a_q for axis links (6 w = 1/3) and diagonal links (6 w = 1/6)
            const float ax = ru0 * (1.0f / 3.0f), ay = ru1 * (1.0f / 3.0f), az = ru2 * (1.0f / 3.0f);
            const float hxy_p = (ru0 + ru1) * (1.0f / 6.0f), hxy_m = (ru0 - ru1) * (1.0f / 6.0f);
            const float hxz_p = (ru0 + ru2) * (1.0f / 6.0f), hxz_m = (ru0 - ru2) * (1.0f / 6.0f);
            const float hyz_p = (ru1 + ru2) * (1.0f / 6.0f), hyz_m = (ru1 - ru2) * (1.0f / 6.0f);
            auto aq = [&](int q) -> float {  // 6 w_q c_q . rho u
                if (q <= 6) return (cx(q) ? cx(q) * ax : 0.f) + (cy(q) ? cy(q) * ay : 0.f) + (cz(q) ? cz(q) * az : 0.f);
                if (cz(q) == 0) return cx(q) == cy(q) ? cx(q) * hxy_p : cx(q) * hxy_m;
                if (cy(q) == 0) return cx(q) == cz(q) ? cx(q) * hxz_p : cx(q) * hxz_m;
                return cy(q) == cz(q) ? cy(q) * hyz_p : cy(q) * hyz_m;
            };
            // sum over the links of -c_q (h*_qbar + h_q), FP32
            float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const bool b = (mk >> q) & 1u;
                const float a = b ? aq(q) : 0.f;
                const float s2 = b ? 2.0f * fi[q] + a : 0.f;
                if (cx(q)) f0 -= cx(q) * s2;
                if (cy(q)) f1 -= cy(q) * s2;
                if (cz(q)) f2 -= cz(q) * s2;
                fi[q] += a;
            }
            // the constant parts 2 w_q c_q as exact counts (units of 1/18) from the link
            // mask: axis links count 2, diagonal links 1; and the added mass sum a_q
            // (bit q set for the directions with c_q = -1 and = +1 along each axis)
            const int kx = 2 * (__popc(mk & 0x4u) - __popc(mk & 0x2u)) + __popc(mk & 0x6600u) - __popc(mk & 0x1980u);
            const int ky = 2 * (__popc(mk & 0x10u) - __popc(mk & 0x8u)) + __popc(mk & 0x60500u) - __popc(mk & 0x18280u);
            const int kz = 2 * (__popc(mk & 0x40u) - __popc(mk & 0x20u)) + __popc(mk & 0x55000u) - __popc(mk & 0x2a800u);
            // sum_q a_q = rho u . sum_q 6 w_q c_q = -(rho u . k) / 6 with k = -sum c_q m_q
            const float dm = -(ru0 * (float)kx + ru1 * (float)ky + ru2 * (float)kz) * (1.0f / 6.0f);
            const double F0 = (double)f0 + kx * (1.0 / 18.0), F1 = (double)f1 + ky * (1.0 / 18.0),
                         F2 = (double)f2 + kz * (1.0 / 18.0);
            const double dx = rx, dy = ry, dz = rz;
            // LDS atomic adds without return: the lane's own slots, so nothing waits
            lds_add(&L.acc[0][t], F0);
            lds_add(&L.acc[1][t], F1);
            lds_add(&L.acc[2][t], F2);
            lds_add(&L.acc[3][t], dy * F2 - dz * F1);
            lds_add(&L.acc[4][t], dz * F0 - dx * F2);
            lds_add(&L.acc[5][t], dx * F1 - dy * F0);
            lds_add(&L.acc[6][t], (double)dm);
        };
        if (!multi && okP) {
            particle_links(P, sm, pm);
        } else {
            // links into more than one particle, or an inconsistent owner (rare): one
            // particle at a time
            uint32_t rest = sm;
            while (rest) {
                const int q0 = __ffs(rest) - 1;
                int Pk = -1;
#pragma unroll
                for (int q = 1; q < Q; ++q)
                    if (q == q0) Pk = L.pt[slot(q)][ly + 1 - cy(q)][lx + 1 - cx(q)];
                uint32_t mk = 0;
#pragma unroll
                for (int q = 1; q < Q; ++q)
                    mk |= (uint32_t)(((rest >> q) & 1u) && L.pt[slot(q)][ly + 1 - cy(q)][lx + 1 - cx(q)] == Pk) << q;
                rest &= ~mk;
                if ((unsigned)Pk >= (unsigned)D.np) {  // not a particle: plain bounce-back
                    atomicOr(D.err, ERR_LG);
                    continue;
                }
                particle_links(Pk, mk, pmir_load(D.pmir, Pk));
            }
        }
    }
    const Moments M = cell_moments(fi);
    if (D.rhow != nullptr && D.st_cur >= 0 && store) {
        // the density for a liquid cell, none for the row's other cells
        const unsigned w = act ? rhow_word(1.0f + (float)M.drho, D.st_cur) : RHOW_NONE;
        __builtin_nontemporal_store(w, D.rhow + c);
    }
    if (!collide_store<ST, true>(Ph, fi, M, B, S, (unsigned)c, store) && act) atomicOr(D.err, ERR_NAN);
}

// tiles of the march: blocks go to the eight XCDs round-robin; each XCD takes whole
// chunks of planes (every eighth chunk), all tile columns of a chunk in turn
__device__ __forceinline__ void march_of_block(int b, int nCols, int nChunks, int &col, int &chunk) {
    if (nChunks % 8 == 0) {
        const int i = b >> 3;
        col = i % nCols;
        chunk = (b & 7) + 8 * (i / nCols);
    } else {
        col = b % nCols;
        chunk = b / nCols;
    }
}

// The fused step (Eqs. LBE1, LBE2, bbrule, netforce, torque, momentum_transfer) for the
// liquid cells of a 64 x 4 column through nzc planes.  Interface cells and liquid
// cells next to gas or a moving or slipping face are left to k_general: each plane of
// the column that holds one is appended to the list gen.
template <int ST, bool MW, bool PER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE_MARCH))) void k_stream_collide(
    Geom G, Phys Ph, Dev D, int tilesX, int tilesY, int nChunks, int nzc, int *gen, int *ngen) {
    __shared__ MarchLds L;
    int col, chunk;
    march_of_block(blockIdx.x, tilesX * tilesY, nChunks, col, chunk);
    const int x0 = (col % tilesX) * TX, y0 = (col / tilesX) * TY;
    const int zs = chunk * nzc, ze = min(zs + nzc, G.nz);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lx = lane, ly = wv;
    const int x = x0 + lx, y = y0 + ly;
    const bool inb = x < G.nx && y < G.ny;

    // planes zs-1 .. zs+1 into the ring
    const StageIdx SI = stage_idx(G, x0, y0);
    RowPre R;
    for (int p = zs - 1; p <= zs + 1; ++p) {
        const int zo = stage_zo(G, p);
        pre_flags(D.flags, SI, R, zo);
        pre_pids(D.pid, SI, R, zo);
        pre_store(L, R, p & 3, MW);
    }
    if (threadIdx.x < 2) L.genflag[threadIdx.x] = 0;
    L.accP[threadIdx.x] = -1;
    int curP = -1;  // the particle of the lane's sums (a copy of L.accP)
#pragma unroll
    for (int k = 0; k < 7; ++k) L.acc[k][threadIdx.x] = 0.0;
    __syncthreads();

    for (int z = zs; z < ze; ++z) {
        // the ring's next plane z+2: cell types now, particle ids once the pulls of this
        // plane are issued
        const int zo2 = stage_zo(G, z + 2);
        pre_flags(D.flags, SI, R, zo2);
        const int s0 = z & 3, sm1 = (z - 1) & 3, sp1 = (z + 1) & 3;
        // values the compiler would otherwise keep for the whole march (per-direction
        // address terms of the lane, plane bases): recomputed in every plane instead
        int xl = x, yl = y;
        long long Sl = G.S;
        __asm__ volatile("" : "+v"(xl), "+v"(yl));
        // the lane's cell for addresses (lanes beyond the box take the last one)
        const int xc = min(xl, G.nx - 1), yc = min(yl, G.ny - 1);
        __asm__ volatile("" : "+s"(Sl));
        const void *Av = D.fA;
        void *Bv = D.fB;
        const uint8_t fl = inb ? L.ft[s0][ly + 1][lx + 1] : WALL;
        const bool nbnf = nbr_any<MK_NF3, MK_NF1>(L, sm1, s0, sp1, ly, lx);
        const bool nbbad = nbr_any<MK_BAD3, MK_BAD1>(L, sm1, s0, sp1, ly, lx);
        const bool gen_c = inb && (fl == IFC || (fl == LIQ && nbbad));
        const bool act = inb && fl == LIQ && !nbbad;
        if (__ballot(gen_c) && lane == 0) L.genflag[z & 1] = 1;
        if (__ballot(act)) {
            const int nxy = G.nx * G.ny;
            SrcOff so;
            so.xm = step_to(xc, -1, G.nx, G.per[0], 1);
            so.xp = step_to(xc, 1, G.nx, G.per[0], 1);
            so.ym = step_to(yc, -1, G.ny, G.per[1], G.nx);
            so.yp = step_to(yc, 1, G.ny, G.per[1], G.nx);
            so.zm = step_to(z, -1, G.nz, G.per[2], nxy);
            so.zp = step_to(z, 1, G.nz, G.per[2], nxy);
            const int c = xc + G.nx * yc + nxy * z;
            march_cell<ST, PER>(G, Ph, D, L, sm1, s0, sp1, lx, ly, xl, yl, z, c, so, act, inb && !gen_c, nbnf, Av, Bv, Sl,
                           SI, R, zo2, curP);
        } else {
            pre_pids(D.pid, SI, R, zo2);
        }
        pre_store(L, R, (z + 2) & 3, MW);
        __syncthreads();
        if (threadIdx.x == 0 && L.genflag[z & 1]) {
            L.genflag[z & 1] = 0;
            const int slot = atomicAdd(ngen, 1);
            gen[slot] = col + tilesX * tilesY * z;  // list capacity: every tile of the box
        }
    }
    if (D.np > 0) macc_wave_flush(D, L);
}

// Row masks of the staged tile for the general path's selection (gas and, with moving
// or slipping faces, walls).  One ballot per row; the caller syncs before and after.
__device__ __forceinline__ void build_bad_masks(const uint8_t (&tile)[3][TY + 2][TX + 2],
                                                unsigned long long (&b3)[3 * (TY + 2)],
                                                unsigned long long (&b1)[3 * (TY + 2)], bool wall_bad) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = wv; r < 3 * (TY + 2); r += 4) {
        const int lz = r / (TY + 2), ly = r - lz * (TY + 2);
        const uint8_t a = tile[lz][ly][lane], b = tile[lz][ly][TX + (lane & 1)];
        const unsigned long long lo = __ballot(a == GAS || (wall_bad && a == WALL));
        const unsigned long long hi = __ballot(lane < 2 && (b == GAS || (wall_bad && b == WALL))) & 3ull;
        if (lane == 0) {
            const unsigned long long s1 = (lo >> 1) | (hi << 63), s2 = (lo >> 2) | (hi << 62);
            b3[r] = lo | s1 | s2;
            b1[r] = s1;
        }
    }
}

// Fill levels of the staged tile's interface cells, with the tile's one-cell halo:
// Eqs. (massExchange, massExchangeb) weight a link to an interface neighbour by the
// mean of the two fill levels, so each level is read once per tile into LDS rather
// than once per link.  Reads the staged cell types; other entries are left 0.
__device__ __forceinline__ void stage_phi_tile(const Geom &G, const double *phi,
                                               const uint8_t (&tile)[3][TY + 2][TX + 2],
                                               double (&ph)[3][TY + 2][TX + 2], int x0, int y0, int z,
                                               bool interior) {
    constexpr int NE = 3 * (TY + 2) * (TX + 2);
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const uint8_t *ft = &tile[0][0][0];
    double *fp = &ph[0][0][0];
    for (int e = threadIdx.x; e < NE; e += 256) {
        double v = 0.0;
        if (ft[e] == IFC) {
            const int lx = e % (TX + 2), r = e / (TX + 2);
            int gx = x0 + lx - 1, gy = y0 + r % (TY + 2) - 1, gz = z + r / (TY + 2) - 1;
            if (!interior) {  // beyond a face only along a periodic axis (a wall stages WALL)
                gx = wrapc(gx, nx);
                gy = wrapc(gy, ny);
                gz = wrapc(gz, nz);
            }
            v = phi[gx + (long long)nx * (gy + (long long)ny * gz)];
        }
        fp[e] = v;
    }
}

// The general path: interface cells and liquid cells next to gas or a moving or
// slipping face, for the tiles (64 x 4 of one plane) that k_stream_collide listed.
// A tile's cells are compacted and handled by as few waves as they fill (sc_cell).
template <int ST, bool MW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MW ? 1 : 5))) void k_general(
    Geom G, Phys Ph, Dev D, int tilesX, int tilesY, const int *gen, const int *ngen) {
    __shared__ uint8_t tile[3][TY + 2][TX + 2];
    __shared__ double ph[3][TY + 2][TX + 2];
    __shared__ unsigned long long b3[3 * (TY + 2)], b1[3 * (TY + 2)];
    __shared__ uint8_t list[TX * TY];
    __shared__ int wcount[4];
    const int n = *ngen;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int t = gen[i];
        const int x0 = (t % tilesX) * TX;
        const int rest = t / tilesX;
        const int y0 = (rest % tilesY) * TY;
        const int z = rest / tilesY;
        const bool interior = x0 >= 1 && x0 + TX + 1 <= G.nx && y0 >= 1 && y0 + TY + 1 <= G.ny && z >= 1 &&
                              z + 2 <= G.nz;
        stage_flag_tile(G, D.flags, tile, x0, y0, z, interior);
        __syncthreads();
        build_bad_masks(tile, b3, b1, MW);
        stage_phi_tile(G, (const double *)D.phi_cur, tile, ph, x0, y0, z, interior);
        __syncthreads();
        const int lx = lane, ly = wv;
        const bool inb = x0 + lx < G.nx && y0 + ly < G.ny;
        const uint8_t fl = inb ? tile[1][ly + 1][lx + 1] : WALL;
        constexpr int R6 = TY + 2;
        const unsigned long long bad = b3[R6 + ly + 1] | b3[R6 + ly] | b3[R6 + ly + 2] | b3[ly + 1] |
                                       b3[2 * R6 + ly + 1] | b1[ly] | b1[ly + 2] | b1[2 * R6 + ly] |
                                       b1[2 * R6 + ly + 2];
        const bool g = inb && (fl == IFC || (fl == LIQ && ((bad >> lx) & 1ull)));
        const unsigned long long m = __ballot(g);
        if (lane == 0) wcount[wv] = (int)__popcll(m);
        __syncthreads();
        int base = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int k = wcount[w];
            base += w < wv ? k : 0;
            total += k;
        }
        if (g) list[base + (int)__popcll(m & ((1ull << lane) - 1ull))] = (uint8_t)threadIdx.x;
        __syncthreads();
        if (wv * 64 < total) {
            const bool has = (int)threadIdx.x < total;
            const int e = has ? list[threadIdx.x] : 0;
            const int ex = e & (TX - 1), ey = e >> 6;
            if (interior) sc_cell<ST, true, MW>(G, Ph, D, tile, ph, ex, ey, x0 + ex, y0 + ey, z, has);
            else sc_cell<ST, false, MW>(G, Ph, D, tile, ph, ex, ey, x0 + ex, y0 + ey, z, has);
        }
        __syncthreads();
    }
}

// the density word of every liquid and interface cell from its populations in A, for
// the first launch after the populations were set from outside
template <int ST>
__global__ void k_rhow_fill(Geom G, Phys Ph, Dev D, int stamp) {
    using SS = Store<ST>;
    const typename SS::T *A = (const typename SS::T *)D.fA;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        const uint8_t f = D.flags[c];
        unsigned w = RHOW_NONE;
        if (f == LIQ || f == IFC) {
            float fa[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) fa[q] = SS::ld(A + q * G.S + c, Ph.inv);
            w = rhow_word(1.0f + (float)cell_moments(fa).drho, stamp);
        }
        D.rhow[c] = w;
    }
}

}  // namespace fsl
