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
// constant parts 2 w_q c_q are counted exactly as integer direction sums
// (axis links 2w = 1/9, diagonal links 2w = 1/18).  All links of a lane share
// the node x, so the torque (x - x_P) x F is formed once per lane in FP64.
struct LinkAcc {
    int P;
    float fs[3];   // sum of -c_q (h*_qbar + h_q)
    int ca[3];     // sum of -c_q over axis links
    int cd[3];     // sum of -c_q over diagonal links
    float dm;      // mass added by moving bounce-back at a liquid cell
};

__device__ __forceinline__ void acc_zero(LinkAcc &L) {
    L.fs[0] = L.fs[1] = L.fs[2] = 0.f;
    L.ca[0] = L.ca[1] = L.ca[2] = 0;
    L.cd[0] = L.cd[1] = L.cd[2] = 0;
    L.dm = 0.f;
}

// FP64 force, torque and mass of the lane's links (a[0..6])
__device__ __forceinline__ void acc_expand(const Dev &D, const LinkAcc &L, int x, int y, int z, double a[7]) {
    double F[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = (double)L.fs[k] + (L.ca[k] * (1.0 / 9.0) + L.cd[k] * (1.0 / 18.0));
    const double *pt = D.ptab + (long long)L.P * P_STRIDE;
    const double rx = x - pt[P_X], ry = y - pt[P_X + 1], rz = z - pt[P_X + 2];
    a[0] = F[0];
    a[1] = F[1];
    a[2] = F[2];
    a[3] = ry * F[2] - rz * F[1];
    a[4] = rz * F[0] - rx * F[2];
    a[5] = rx * F[1] - ry * F[0];
    a[6] = (double)L.dm;
}

__device__ __noinline__ void acc_flush(const Dev &D, const LinkAcc &L, int x, int y, int z) {
    if (L.P < 0) return;
    double a[7];
    acc_expand(D, L, x, y, z, a);
    double *dst = D.pacc + (long long)L.P * ACC_STRIDE;
#pragma unroll
    for (int k = 0; k < 7; ++k) unsafeAtomicAdd(dst + k, a[k]);
}

// wave-level reduction of the lanes' accumulators, segmented by particle id:
// one FP64 atomic per (wave, particle, component)
__device__ __forceinline__ void acc_reduce_wave(const Dev &D, const LinkAcc &L, int x, int y, int z) {
    int key = L.P;
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    if (key >= 0) acc_expand(D, L, x, y, z, a);
    while (true) {
        unsigned long long act = __ballot(key >= 0);
        if (!act) break;
        int leader = __ffsll((long long)act) - 1;
        int k0 = __shfl(key, leader);
        bool mine = key == k0;
        double *dst = D.pacc + (long long)k0 * ACC_STRIDE;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            double v = wave_sum(mine ? a[k] : 0.0);
            if ((int)lane_id() == leader) unsafeAtomicAdd(dst + k, v);
        }
        if (mine) key = -1;
    }
}

// One cell of the fused step.  INTERIOR: the tile and its halo lie inside the box,
// so a source is the cell index minus a uniform offset (no wrap, no wall).
template <int ST, bool INTERIOR>
__device__ __forceinline__ void sc_cell(const Geom &G, const Phys &Ph, const Dev &D,
                                        const uint8_t (&tile)[3][TY + 2][TX + 2], int lx, int ly,
                                        int x, int y, int z) {
    using SS = Store<ST>;
    using T = typename SS::T;
    const int nx = G.nx, ny = G.ny, nz = G.nz, nxy = nx * ny;
    const int c = x + nx * y + nxy * z;
    const uint8_t fl = tile[1][ly + 1][lx + 1];
    const T *A = (const T *)D.fA;
    T *B = (T *)D.fB;
    const long long S = G.S;
    const float inv = Ph.inv, sc = Ph.scale;
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
        const bool needOwn = (fl == IFC) || gm || sm;
        float fo[Q], fi[Q];
        // all independent loads first: own populations, pulled populations, ids
        if (needOwn) {
#pragma unroll
            for (int q = 0; q < Q; ++q) fo[q] = SS::ld(A + q * S + c, inv);
        }
        fi[0] = needOwn ? fo[0] : SS::ld(A + c, inv);
#pragma unroll
        for (int q = 1; q < Q; ++q)
            if (!((miss >> q) & 1u)) fi[q] = SS::ld(A + q * S + src(q), inv);
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
        float rho_t = 1.0f, ut0 = 0.f, ut1 = 0.f, ut2 = 0.f;
        if (needOwn) {
            float d = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                d += fo[q];
                j0 += cx(q) * fo[q];
                j1 += cy(q) * fo[q];
                j2 += cz(q) * fo[q];
            }
            rho_t = 1.0f + d;
            ut0 = j0 / rho_t - 0.5f * Ph.g[0];
            ut1 = j1 / rho_t - 0.5f * Ph.g[1];
            ut2 = j2 / rho_t - 0.5f * Ph.g[2];
        }
        if (miss) {
            // rigid-body velocity of the lane's particle at the node: c_q . u_w at
            // the link midpoint x - c_q/2 equals c_q . (u_P + omega x (x - x_P))
            // because c_q . (omega x c_q) = 0, so one velocity serves all links
            float un0 = 0.f, un1 = 0.f, un2 = 0.f;
            auto node_velocity = [&](int P) {
                const float4 *pm = D.pmir + 4LL * P;
                const float4 an = pm[0], fr = pm[1], up = pm[2], wp = pm[3];
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
                    fi[q] = needOwn ? fo[o] : SS::ld(A + o * S + c, inv);
                } else if ((sm >> q) & 1u) {
                    if (!((same >> q) & 1u) || acc.P != P0) {  // another particle (rare)
                        const int P = D.pid[src(q)];
                        if ((unsigned)P >= (unsigned)D.np) {  // inconsistent state: plain wall
                            fi[q] = fo[o];
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
                    const float fin = fo[o] + 6.0f * wq(q) * rho_t * cu;  // Eq. (bbrule)
                    fi[q] = fin;
                    const float s2 = fo[o] + fin;
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
                    if (fl == LIQ) acc.dm += fin - fo[o];
                } else if ((gm >> q) & 1u) {
                    if (fl == LIQ) atomicOr(D.err, ERR_LG);
                    const int bid = D.bub[src(q)];
                    const float rg = D.rhog[bid < D.maxB ? bid : 0];
                    const float cu = cx(q) * ut0 + cy(q) * ut1 + cz(q) * ut2;
                    const float uu = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
                    // Eq. (fsk) in shifted form: -h*_qbar + 2 (e+_q(rho_g, u) - w_q)
                    fi[q] = -fo[o] + 2.0f * wq(q) * ((rg - 1.0f) + rg * (4.5f * cu * cu - 1.5f * uu));
                }
            }
        }
        // moments; the density deviation is summed in FP64 (exact for 19 FP32 terms)
        double drho_d = 0.0;
        float j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            drho_d += (double)fi[q];
            j0 += cx(q) * fi[q];
            j1 += cy(q) * fi[q];
            j2 += cz(q) * fi[q];
        }
        const float drho = (float)drho_d;
        const float rho = 1.0f + drho;
        const float u0 = j0 / rho + 0.5f * Ph.g[0];
        const float u1 = j1 / rho + 0.5f * Ph.g[1];
        const float u2 = j2 / rho + 0.5f * Ph.g[2];
        if (!(rho == rho) || !(u0 == u0) || !(u1 == u1) || !(u2 == u2)) atomicOr(D.err, ERR_NAN);

        if (fl == IFC) {
            // Eqs. (massExchange, massExchangeb), mass form, FP64
            const double phx = D.phi_cur[c];
            double dm = 0.0;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const uint8_t nf = tile[1 + cz(q)][ly + 1 + cy(q)][lx + 1 + cx(q)];
                if (nf == LIQ || nf == IFC) {
                    double d = (double)fi[opp(q)] - (double)fo[q];
                    if (nf == IFC) d *= 0.5 * (D.phi_cur[nbr(q)] + phx);
                    dm += d;
                }
            }
            const double mnew = D.m[c] + dm;
            D.m[c] = mnew;
            const double phin = mnew / (1.0 + drho_d);
            D.phi_nxt[c] = phin;
            isF = phin >= 1.0 - Ph.eps;
            isE = !isF && phin <= Ph.eps;
        }

        // TRT collision with Guo forcing (Eq. LBE2), shifted form: e - w and f - w
        const float F0 = rho * Ph.g[0], F1 = rho * Ph.g[1], F2 = rho * Ph.g[2];
        const float uu = u0 * u0 + u1 * u1 + u2 * u2;
        const float uF = u0 * F0 + u1 * F1 + u2 * F2;
        const float lp = Ph.lp, lm = Ph.lm;
        const float ap = 1.0f + 0.5f * lp, am = 1.0f + 0.5f * lm;
        // moving populations; their stored values are summed in FP64 so that the rest
        // population can carry the exact mass balance of the collision (in exact
        // arithmetic the collision conserves mass, so h*_0 = sum_q h_q - sum_{q>0} h*_q
        // is the same population; this only keeps FP32 rounding from biasing the mass)
        double sout = 0.0;
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
            sout += (double)SS::dec(vq, inv) + (double)SS::dec(vo, inv);
            B[q * S + c] = vq;
            B[o * S + c] = vo;
        }
        SS::st(B + c, (float)(drho_d - sout), sc);
    }

    wave_append(isF, c, D.lF, D.counters + C_NF, D.cap, D.err);
    wave_append(isE, c, D.lE0, D.counters + C_NE0, D.cap, D.err);
    if (D.np > 0) acc_reduce_wave(D, acc, x, y, z);
}

template <int ST>
__global__ __launch_bounds__(256) void k_stream_collide(Geom G, Phys Ph, Dev D, int tilesX,
                                                        int tilesY, int nTiles) {
    __shared__ uint8_t tile[3][TY + 2][TX + 2];

    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int b = blockIdx.x;
    const int t = (nTiles % 8 == 0) ? (b % 8) * (nTiles / 8) + b / 8 : b;
    const int x0 = (t % tilesX) * TX;
    const int rest = t / tilesX;
    const int y0 = (rest % tilesY) * TY;
    const int z = rest / tilesY;
    const bool interior = x0 >= 1 && x0 + TX + 1 <= nx && y0 >= 1 && y0 + TY + 1 <= ny && z >= 1 &&
                          z + 2 <= nz;

    for (int i = threadIdx.x; i < 3 * (TY + 2) * (TX + 2); i += 256) {
        int lx = i % (TX + 2), ly = (i / (TX + 2)) % (TY + 2), lz = i / ((TX + 2) * (TY + 2));
        int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z + lz - 1;
        bool ok = true;
        if (gx < 0 || gx >= nx) { if (G.per[0]) gx = wrapc(gx, nx); else ok = false; }
        if (gy < 0 || gy >= ny) { if (G.per[1]) gy = wrapc(gy, ny); else ok = false; }
        if (gz < 0 || gz >= nz) { if (G.per[2]) gz = wrapc(gz, nz); else ok = false; }
        uint8_t v = WALL;
        if (ok) v = D.flags[gx + (long long)nx * (gy + (long long)ny * gz)];
        tile[lz][ly][lx] = v;
    }
    __syncthreads();

    const int lx = threadIdx.x & (TX - 1), ly = threadIdx.x >> 6;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= nx || y >= ny) return;
    if (interior) sc_cell<ST, true>(G, Ph, D, tile, lx, ly, x, y, z);
    else sc_cell<ST, false>(G, Ph, D, tile, lx, ly, x, y, z);
}

}  // namespace fsl
