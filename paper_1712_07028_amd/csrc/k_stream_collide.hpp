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
__device__ __forceinline__ void acc_flush(const Dev &D, const LinkAcc &L, int x, int y, int z) {
    if (L.P < 0) return;
    // lever arm x - x_P = (x - a) - f
    acc_flush_v(D.pacc, L.P, L.fs[0], L.fs[1], L.fs[2], L.ca[0], L.ca[1], L.ca[2], L.cd[0], L.cd[1],
                L.cd[2], L.dm, ((float)x - L.an[0]) - L.fr[0], ((float)y - L.an[1]) - L.fr[1],
                ((float)z - L.an[2]) - L.fr[2]);
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
__device__ __forceinline__ void acc_reduce_wave(const Dev &D, const LinkAcc &L, int x, int y, int z) {
    int key = L.P;
    if (!__ballot(key >= 0)) return;
    // lane parts: forces, torques about the anchor, mass
    const int dx = x - (int)L.an[0], dy = y - (int)L.an[1], dz = z - (int)L.an[2];
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
template <int ST>
__device__ __forceinline__ bool collide_store(const Phys &Ph, const float (&fi)[Q], const Moments &M,
                                              typename Store<ST>::T *B, long long S, unsigned c) {
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
        sp[k++] = (double)SS::dec(vq, inv) + (double)SS::dec(vo, inv);
        B[q * S + c] = vq;
        B[o * S + c] = vo;
    }
    const double sout = (((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]))) + sp[8];
    SS::st(B + c, (float)(M.drho - sout), sc);
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
                                        const uint8_t (&tile)[3][TY + 2][TX + 2], int lx, int ly,
                                        int x, int y, int z, bool inb) {
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
    auto nbr = [&](int q) -> int {
        if (INTERIOR) return c + (cx(q) + cy(q) * nx + cz(q) * nxy);
        const int sx = wrapc(x + cx(q), nx), sy = wrapc(y + cy(q), ny), sz = wrapc(z + cz(q), nz);
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
                const int2 e = D.rhow[c];
                have = e.y == D.st_prev;
                rho_t = __int_as_float(e.x);
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
                const float4 *pm = D.pmir + 4LL * P;
                const float4 an = pm[0], fr = pm[1], up = pm[2], wp = pm[3];
                acc.an[0] = an.x; acc.an[1] = an.y; acc.an[2] = an.z;
                acc.fr[0] = fr.x; acc.fr[1] = fr.y; acc.fr[2] = fr.z;
                const float rx = ((float)x - an.x) - fr.x;
                const float ry = ((float)y - an.y) - fr.y;
                const float rz = ((float)z - an.z) - fr.z;
                un0 = up.x + (wp.y * rz - wp.z * ry);
                un1 = up.y + (wp.z * rx - wp.x * rz);
                un2 = up.z + (wp.x * ry - wp.y * rx);
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
                            acc_flush(D, acc, x, y, z);
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
            const double phx = D.phi_cur[c];
            double dm = 0.0;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const uint8_t nf = tile[1 + cz(q)][ly + 1 + cy(q)][lx + 1 + cx(q)];
                if (nf == LIQ || nf == IFC) {
                    double d = (double)fi[opp(q)] - (double)fo(q);
                    if (nf == IFC) d *= 0.5 * (D.phi_cur[nbr(q)] + phx);
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
                            if (pf == IFC) {
                                const int pc = wrapc(x + dx, nx) + nx * wrapc(y + dy, ny) + nxy * wrapc(z + dz, nz);
                                d *= 0.5 * (D.phi_cur[pc] + phx);
                            }
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
        if (D.rhow != nullptr && D.st_cur >= 0)
            D.rhow[c] = make_int2(__float_as_int(1.0f + (float)drho_d), D.st_cur);
        if (!collide_store<ST>(Ph, fi, M, B, S, (unsigned)c)) atomicOr(D.err, ERR_NAN);
    }

    wave_append(isF, c, D.lF, D.counters + C_NF, D.cap, D.err);
    wave_append(isE, c, D.lE0, D.counters + C_NE0, D.cap, D.err);
    if (D.np > 0) acc_reduce_wave(D, acc, x, y, z);
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

// Per row of the staged tile (3 planes x 6 rows of 66 cells): w3 bit i is set when
// one of the columns i, i+1, i+2 (the cells x-1, x, x+1 of lane i) is neither liquid
// nor a resting wall, w1 bit i when column i+1 (the cell x of lane i) is neither.
// One ballot per row; the caller syncs before and after.
__device__ __forceinline__ void build_row_masks(const uint8_t (&tile)[3][TY + 2][TX + 2],
                                                unsigned long long (&w3)[3 * (TY + 2)],
                                                unsigned long long (&w1)[3 * (TY + 2)], bool wall_ok) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = wv; r < 3 * (TY + 2); r += 4) {
        const int lz = r / (TY + 2), ly = r - lz * (TY + 2);
        const uint8_t a = tile[lz][ly][lane], b = tile[lz][ly][TX + (lane & 1)];
        const unsigned long long lo = __ballot(a != LIQ && !(a == WALL && wall_ok));
        const unsigned long long hi = __ballot(lane < 2 && b != LIQ && !(b == WALL && wall_ok)) & 3ull;
        const unsigned long long s1 = (lo >> 1) | (hi << 63);
        const unsigned long long s2 = (lo >> 2) | (hi << 62);
        if (lane == 0) {
            w3[r] = lo | s1 | s2;
            w1[r] = s1;
        }
    }
}

// tile t of the launch: XCD-contiguous ranges when the tile count allows
__device__ __forceinline__ int tile_of_block(int b, int nTiles) {
    return (nTiles % 8 == 0) ? (b % 8) * (nTiles / 8) + b / 8 : b;
}

// A liquid cell whose 18 neighbours are liquid or beyond a wall: plain pull
// (Eq. LBE1) with half-way bounce-back at walls, then the collision (Eq. LBE2).
template <int ST, bool INTERIOR>
__device__ __forceinline__ void lean_cell(const Geom &G, const Phys &Ph, const Dev &D,
                                          const uint8_t (&tile)[3][TY + 2][TX + 2], int lx, int ly, int x,
                                          int y, int z) {
    using SS = Store<ST>;
    using T = typename SS::T;
    const int nx = G.nx, ny = G.ny, nz = G.nz, nxy = nx * ny;
    const int c = x + nx * y + nxy * z;
    const T *A = (const T *)D.fA;
    T *B = (T *)D.fB;
    const long long S = G.S;
    float fi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T *p;
        if (INTERIOR || q == 0) {
            p = A + q * S + (unsigned)(c - (cx(q) + cy(q) * nx + cz(q) * nxy));
        } else {
            const bool wall = tile[1 - cz(q)][ly + 1 - cy(q)][lx + 1 - cx(q)] == WALL;
            const int s = wrapc(x - cx(q), nx) + nx * wrapc(y - cy(q), ny) + nxy * wrapc(z - cz(q), nz);
            p = wall ? A + opp(q) * S + (unsigned)c : A + q * S + (unsigned)s;
        }
        fi[q] = SS::ld(p, Ph.inv);
    }
    const Moments M = cell_moments(fi);
    if (!collide_store<ST>(Ph, fi, M, B, S, (unsigned)c)) atomicOr(D.err, ERR_NAN);
}

// The fused step of one 64 x 4 tile of a plane: the cell types of the tile and its
// halo are staged in LDS; lean cells (liquid, with liquid or wall neighbours only)
// take the plain path in place; the other liquid and interface cells of the tile
// are compacted into a list and handled by as few waves as they fill, so that the
// boundary work (bounce-back, free surface, mass exchange, forces, lists) is not
// repeated by every wave that holds one such cell.
template <int ST, bool MW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MW ? 1 : 5))) void k_stream_collide(Geom G, Phys Ph, Dev D, int tilesX,
                                                        int tilesY, int nTiles) {
    __shared__ uint8_t tile[3][TY + 2][TX + 2];
    __shared__ unsigned long long w3[3 * (TY + 2)], w1[3 * (TY + 2)];
    __shared__ uint8_t list[TX * TY];
    __shared__ int wcount[4];

    const int t = tile_of_block(blockIdx.x, nTiles);
    const int x0 = (t % tilesX) * TX;
    const int rest = t / tilesX;
    const int y0 = (rest % tilesY) * TY;
    const int z = rest / tilesY;
    const bool interior = x0 >= 1 && x0 + TX + 1 <= G.nx && y0 >= 1 && y0 + TY + 1 <= G.ny && z >= 1 &&
                          z + 2 <= G.nz;
    stage_flag_tile(G, D.flags, tile, x0, y0, z, interior);
    __syncthreads();
    build_row_masks(tile, w3, w1, !MW);
    __syncthreads();

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lx = lane, ly = wv;
    const int x = x0 + lx, y = y0 + ly;
    const bool inb = x < G.nx && y < G.ny;
    const uint8_t fl = inb ? tile[1][ly + 1][lx + 1] : WALL;
    // any neighbour of the wave's cells that is neither liquid nor a wall (same
    // plane: the 3 x 3 square; planes z +- 1: the plus shape)
    constexpr int R6 = TY + 2;
    const unsigned long long nb = w3[R6 + ly + 1] | w3[R6 + ly] | w3[R6 + ly + 2] | w3[ly + 1] |
                                  w3[2 * R6 + ly + 1] | w1[ly] | w1[ly + 2] | w1[2 * R6 + ly] |
                                  w1[2 * R6 + ly + 2];
    const bool lean = inb && fl == LIQ && !((nb >> lx) & 1ull);
    if (lean) {
        if (interior) lean_cell<ST, true>(G, Ph, D, tile, lx, ly, x, y, z);
        else lean_cell<ST, false>(G, Ph, D, tile, lx, ly, x, y, z);
    }

    // the tile's boundary cells, in lane order
    const bool need = inb && !lean && (fl == LIQ || fl == IFC);
    const unsigned long long m = __ballot(need);
    if (lane == 0) wcount[wv] = (int)__popcll(m);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int n = wcount[w];
        base += w < wv ? n : 0;
        total += n;
    }
    if (need) list[base + (int)__popcll(m & ((1ull << lane) - 1ull))] = (uint8_t)threadIdx.x;
    __syncthreads();
    if (wv * 64 < total) {
        const bool has = (int)threadIdx.x < total;
        const int e = has ? list[threadIdx.x] : 0;
        const int ex = e & (TX - 1), ey = e >> 6;
        if (interior) sc_cell<ST, true, MW>(G, Ph, D, tile, ex, ey, x0 + ex, y0 + ey, z, has);
        else sc_cell<ST, false, MW>(G, Ph, D, tile, ex, ey, x0 + ex, y0 + ey, z, has);
    }
}

}  // namespace fsl
