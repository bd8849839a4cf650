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

struct LinkAcc {
    int P;
    double a[7];  // F(3), T(3), mass added by moving bounce-back
};

__device__ __forceinline__ void acc_flush(const Dev &D, LinkAcc &L) {
    if (L.P < 0) return;
    double *dst = D.pacc + (long long)L.P * ACC_STRIDE;
#pragma unroll
    for (int k = 0; k < 7; ++k) unsafeAtomicAdd(dst + k, L.a[k]);
}

__device__ __forceinline__ void acc_add(const Dev &D, LinkAcc &L, int P, double djx, double djy,
                                        double djz, double rx, double ry, double rz, double dm) {
    if (P != L.P) {
        acc_flush(D, L);
        L.P = P;
#pragma unroll
        for (int k = 0; k < 7; ++k) L.a[k] = 0.0;
    }
    double jx = djx, jy = djy, jz = djz;
    L.a[0] += jx;
    L.a[1] += jy;
    L.a[2] += jz;
    L.a[3] += ry * jz - rz * jy;
    L.a[4] += rz * jx - rx * jz;
    L.a[5] += rx * jy - ry * jx;
    L.a[6] += dm;
}

// wave-level reduction of the per-lane accumulators, segmented by particle id:
// one FP64 atomic per (wave, particle, component)
__device__ __forceinline__ void acc_reduce_wave(const Dev &D, LinkAcc &L) {
    int key = L.P;
    while (true) {
        unsigned long long act = __ballot(key >= 0);
        if (!act) break;
        int leader = __ffsll((long long)act) - 1;
        int k0 = __shfl(key, leader);
        bool mine = key == k0;
        double *dst = D.pacc + (long long)k0 * ACC_STRIDE;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            double v = wave_sum(mine ? L.a[k] : 0.0);
            if ((int)lane_id() == leader) unsafeAtomicAdd(dst + k, v);
        }
        if (mine) key = -1;
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_stream_collide(Geom G, Phys Ph, Dev D, int tilesX,
                                                        int tilesY, int nTiles) {
    using SS = Store<ST>;
    using T = typename SS::T;
    __shared__ uint8_t tile[3][TY + 2][TX + 2];

    const int nx = G.nx, ny = G.ny, nz = G.nz;
    int b = blockIdx.x;
    int t = (nTiles % 8 == 0) ? (b % 8) * (nTiles / 8) + b / 8 : b;
    const int x0 = (t % tilesX) * TX;
    const int rest = t / tilesX;
    const int y0 = (rest % tilesY) * TY;
    const int z = rest / tilesY;

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
    const int c = x + nx * (y + ny * z);
    const uint8_t fl = tile[1][ly + 1][lx + 1];

    LinkAcc acc;
    acc.P = -1;
#pragma unroll
    for (int k = 0; k < 7; ++k) acc.a[k] = 0.0;
    bool isF = false, isE = false;

    const T *A = (const T *)D.fA;
    T *B = (T *)D.fB;
    const long long S = G.S;
    const float inv = Ph.inv, sc = Ph.scale;

    if (fl == LIQ || fl == IFC) {
        uint32_t gm = 0, sm = 0, wm = 0;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            uint8_t sf = tile[1 - cz(q)][ly + 1 - cy(q)][lx + 1 - cx(q)];
            gm |= (uint32_t)(sf == GAS) << q;
            sm |= (uint32_t)(sf == SOL) << q;
            wm |= (uint32_t)(sf == WALL) << q;
        }
        const bool needOwn = (fl == IFC) || gm || sm;
        float fo[Q], fi[Q];
        if (needOwn) {
#pragma unroll
            for (int q = 0; q < Q; ++q) fo[q] = SS::ld(A + q * S + c, inv);
        }
        fi[0] = needOwn ? fo[0] : SS::ld(A + c, inv);
        const uint32_t miss = gm | sm | wm;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            if (!((miss >> q) & 1u)) {
                int sx = wrapc(x - cx(q), nx), sy = wrapc(y - cy(q), ny), sz = wrapc(z - cz(q), nz);
                fi[q] = SS::ld(A + q * S + (sx + nx * (sy + ny * sz)), inv);
            }
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
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const int o = opp(q);
                if ((wm >> q) & 1u) {
                    fi[q] = needOwn ? fo[o] : SS::ld(A + o * S + c, inv);
                } else if ((sm >> q) & 1u) {
                    int sx = wrapc(x - cx(q), nx), sy = wrapc(y - cy(q), ny), sz = wrapc(z - cz(q), nz);
                    int P = D.pid[sx + nx * (sy + ny * sz)];
                    if ((unsigned)P >= (unsigned)D.np) {  // inconsistent state: plain wall
                        fi[q] = fo[o];
                        atomicOr(D.err, ERR_LG);
                        continue;
                    }
                    const double *pt = D.ptab + (long long)P * P_STRIDE;
                    double rx = (x - 0.5 * cx(q)) - pt[P_X], ry = (y - 0.5 * cy(q)) - pt[P_X + 1],
                           rz = (z - 0.5 * cz(q)) - pt[P_X + 2];
                    double uw0 = pt[P_U] + (pt[P_W + 1] * rz - pt[P_W + 2] * ry);
                    double uw1 = pt[P_U + 1] + (pt[P_W + 2] * rx - pt[P_W] * rz);
                    double uw2 = pt[P_U + 2] + (pt[P_W] * ry - pt[P_W + 1] * rx);
                    float cu = (float)(cx(q) * uw0 + cy(q) * uw1 + cz(q) * uw2);
                    float fin = fo[o] + 6.0f * wq(q) * rho_t * cu;
                    fi[q] = fin;
                    // f*_qbar(x) + f_q(x,t+1) in FP64: shifted parts plus 2 w_q
                    const double s = ((double)fo[o] + (double)fin) + 2.0 * wqd(q);
                    // the ledger pays the moving-wall mass of liquid cells only: an
                    // interface cell's mass is m, which the link does not change
                    acc_add(D, acc, P, -cx(q) * s, -cy(q) * s, -cz(q) * s, x - pt[P_X],
                            y - pt[P_X + 1], z - pt[P_X + 2],
                            fl == LIQ ? (double)fin - (double)fo[o] : 0.0);
                } else if ((gm >> q) & 1u) {
                    if (fl == LIQ) atomicOr(D.err, ERR_LG);
                    int sx = wrapc(x - cx(q), nx), sy = wrapc(y - cy(q), ny), sz = wrapc(z - cz(q), nz);
                    int bid = D.bub[sx + nx * (sy + ny * sz)];
                    float rg = D.rhog[bid < D.maxB ? bid : 0];
                    float cu = cx(q) * ut0 + cy(q) * ut1 + cz(q) * ut2;
                    float uu = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
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
            const double phx = D.phi_cur[c];
            double dm = 0.0;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                uint8_t nf = tile[1 + cz(q)][ly + 1 + cy(q)][lx + 1 + cx(q)];
                if (nf == LIQ || nf == IFC) {
                    double d = (double)fi[opp(q)] - (double)fo[q];
                    if (nf == IFC) {
                        int nxp = wrapc(x + cx(q), nx), nyp = wrapc(y + cy(q), ny), nzp = wrapc(z + cz(q), nz);
                        d *= 0.5 * (D.phi_cur[nxp + nx * (nyp + ny * nzp)] + phx);
                    }
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

        // TRT collision with Guo forcing, shifted form: e - w and f - w
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
    } else if (fl == SOL && D.np > 0) {
        // solid node of particle P' with links into another particle P: equilibrium
        // populations at rho = 1 and the rigid velocity of P' (Sec. 2.3)
        uint32_t nm = 0;
#pragma unroll
        for (int q = 1; q < Q; ++q)
            nm |= (uint32_t)(tile[1 + cz(q)][ly + 1 + cy(q)][lx + 1 + cx(q)] == SOL) << q;
        const int Pp = D.pid[c];
        if (nm && (unsigned)Pp < (unsigned)D.np) {
            const double *pp = D.ptab + (long long)Pp * P_STRIDE;
            double rx = x - pp[P_X], ry = y - pp[P_X + 1], rz = z - pp[P_X + 2];
            double ur0 = pp[P_U] + (pp[P_W + 1] * rz - pp[P_W + 2] * ry);
            double ur1 = pp[P_U + 1] + (pp[P_W + 2] * rx - pp[P_W] * rz);
            double ur2 = pp[P_U + 2] + (pp[P_W] * ry - pp[P_W + 1] * rx);
            double uu = ur0 * ur0 + ur1 * ur1 + ur2 * ur2;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                if (!((nm >> q) & 1u)) continue;
                int nxp = wrapc(x + cx(q), nx), nyp = wrapc(y + cy(q), ny), nzp = wrapc(z + cz(q), nz);
                int P = D.pid[nxp + nx * (nyp + ny * nzp)];
                if (P == Pp || (unsigned)P >= (unsigned)D.np) continue;
                const double *pt = D.ptab + (long long)P * P_STRIDE;
                double cu = cx(q) * ur0 + cy(q) * ur1 + cz(q) * ur2;
                double e2 = 2.0 * wqd(q) * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                acc_add(D, acc, P, cx(q) * e2, cy(q) * e2, cz(q) * e2, x - pt[P_X], y - pt[P_X + 1],
                        z - pt[P_X + 2], 0.0);
            }
        }
    }

    wave_append(isF, c, D.lF, D.counters + C_NF, D.cap, D.err);
    wave_append(isE, c, D.lE0, D.counters + C_NE0, D.cap, D.err);
    if (D.np > 0) acc_reduce_wave(D, acc);
}

}  // namespace fsl
