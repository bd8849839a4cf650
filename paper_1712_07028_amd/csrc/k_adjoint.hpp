// k_adjoint.hpp -- differentiation form: reverse-mode (adjoint) sweep of the step
// over a window in which the cell types are frozen (every non-solid cell liquid,
// spheres kinematic).
//
// State of the window: s_t = post-collision populations after t steps.  The step is
// s_{t+1} = C(S(s_t)) with S the pull streaming with bounce-back (Eq. LBE1, walls and
// Eq. bbrule, whose rho_w is the density of s_t at the fluid node) and C the TRT
// collision with Guo forcing (Eq. LBE2).  The objective is the summed drag
//   J = sum_{t=0}^{T-1} J_t(s_t),  J_t = -sum_P uhat_P . F_P(s_t),
// F_P the momentum exchange of Eqs. (netforce, momentum_transfer), linear in s_t.
//
// With mu_t the adjoint of the pre-collision populations f_t = S(s_{t-1}):
//   sbar_t = S^T mu_{t+1} + dJ_t/ds_t,   mu_t = (dC/df)^T(f_t) sbar_t,
// for t = T-1 .. 1, mu_T = 0, and the parameter gradient collects
//   sum_t sbar_t . dC/dtheta (f_t)
// with theta = (lambda_+, lambda_-, g).  One kernel does one t: it gathers mu_{t+1}
// from the downstream cells (the transpose of the pull), adds the drag source,
// recomputes f_t from s_{t-1}, applies the transposed collision Jacobian and
// reduces the five parameter partials per block in FP64.  Segments of k states are
// recomputed from checkpoints by the ordinary stream-collide kernel.
#pragma once

#include <stdio.h>

#include "fsl_device.hpp"
#include "k_stream_collide.hpp"

namespace fsl {

constexpr int ADJ_NPART = 8;  // doubles per block partial: dL/dlp, dL/dlm, dL/dg[3]

struct AdjointState {
    char *base = nullptr;
    size_t bytes = 0;
    int Tmax = 0, kmax = 0, ncp = 0, nTiles = 0;
    long long S = 0;
    float *cp = nullptr;      // checkpoints s_0, s_k, s_2k, ... [ncp][Q][S]
    float *seg = nullptr;     // recomputed states of one segment [kmax - 1][Q][S]
    float *mu[2] = {nullptr, nullptr};
    double *part = nullptr;   // per-block partials [nTiles][ADJ_NPART]
    double *acc = nullptr;    // [0] J, [1..5] reduced partials
    float4 *uh = nullptr;     // unit direction of motion per particle
    double *dummy = nullptr;  // force accumulator of recomputed steps
    int T = 0, k = 0;         // last forward window
    int ready = 0;            // checkpoints of the last forward window are valid
    double lp_tau = 0, lm_tau = 0;  // d lambda_+- / d tau at the window's tau
};

inline size_t adj_up(size_t v) { return (v + 255) / 256 * 256; }

inline size_t adjoint_window_bytes(int T, int k, size_t S, int maxP, int nTiles) {
    if (T <= 0 || k <= 0) return 0;
    const size_t st = (size_t)Q * S * 4;
    const int ncp = (T + k - 1) / k;
    const int nseg = (k < T ? k : T) - 1;
    return adj_up(st) * (ncp + nseg + 2) + adj_up((size_t)nTiles * ADJ_NPART * 8) + adj_up(64 * 8) +
           adj_up((size_t)(maxP > 0 ? maxP : 1) * 16) + adj_up((size_t)(maxP > 0 ? maxP : 1) * ACC_COPIES * ACC_STRIDE * 8);
}

inline void adjoint_bind(AdjointState &A, char *base, size_t bytes, int T, int k, long long S, int maxP,
                         int nTiles) {
    A = AdjointState{};
    A.base = base;
    A.bytes = bytes;
    if (!bytes) return;
    A.Tmax = T;
    A.kmax = k;
    A.S = S;
    A.nTiles = nTiles;
    A.ncp = (T + k - 1) / k;
    const int nseg = (k < T ? k : T) - 1;
    const size_t st = adj_up((size_t)Q * S * 4);
    char *p = base;
    A.cp = (float *)p;
    p += st * A.ncp;
    A.seg = (float *)p;
    p += st * nseg;
    A.mu[0] = (float *)p;
    p += st;
    A.mu[1] = (float *)p;
    p += st;
    A.part = (double *)p;
    p += adj_up((size_t)nTiles * ADJ_NPART * 8);
    A.acc = (double *)p;
    p += adj_up(64 * 8);
    A.uh = (float4 *)p;
    p += adj_up((size_t)(maxP > 0 ? maxP : 1) * 16);
    A.dummy = (double *)p;
}

// ---- small kernels of the window ---------------------------------------------------
// every non-solid cell must be liquid
__global__ void k_win_check(Geom G, Dev D, int *bad) {
    int n = 0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x)
        n += (D.flags[c] == GAS || D.flags[c] == IFC);
    if (__ballot(n != 0) && n) atomicAdd(bad, n);
}

// unit direction of motion u_P / |u_P| (zero for a particle at rest)
__global__ void k_win_uhat(Dev D, float4 *uh) {
    for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < D.np; P += gridDim.x * blockDim.x) {
        const double *t = D.ptab + (long long)P * P_STRIDE;
        const double n = sqrt(t[P_U] * t[P_U] + t[P_U + 1] * t[P_U + 1] + t[P_U + 2] * t[P_U + 2]);
        const double s = n > 0.0 ? 1.0 / n : 0.0;
        uh[P] = make_float4((float)(t[P_U] * s), (float)(t[P_U + 1] * s), (float)(t[P_U + 2] * s), 0.f);
    }
}

// J += -sum_P uhat_P . F_P of the step just taken (FP64, fixed summation order)
__global__ __launch_bounds__(256) void k_win_J(Dev D, double *acc) {
    __shared__ double red[256];
    double v = 0.0;
    for (int P = threadIdx.x; P < D.np; P += 256) {
        const double *t = D.ptab + (long long)P * P_STRIDE;
        const double n = sqrt(t[P_U] * t[P_U] + t[P_U + 1] * t[P_U + 1] + t[P_U + 2] * t[P_U + 2]);
        if (n > 0.0) {
            const double *F = D.pFT + (long long)P * 6;
            v -= (t[P_U] * F[0] + t[P_U + 1] * F[1] + t[P_U + 2] * F[2]) / n;
        }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[0] += red[0];
}

// sum of the per-block partials in a fixed order: acc[1 + i] = sum_b part[b][i]
__global__ __launch_bounds__(256) void k_adj_reduce(const double *part, int nb, double *acc) {
    __shared__ double red[256];
    for (int i = 0; i < 5; ++i) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) v += part[(long long)b * ADJ_NPART + i];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) acc[1 + i] = red[0];
        __syncthreads();
    }
}

// ---- one adjoint step of one cell ---------------------------------------------------
// gr receives the cell's dL/dlambda_+, dL/dlambda_-, dL/dg[3] with L = sbar . C.
template <bool INTERIOR>
__device__ __forceinline__ void adj_cell(const Geom &G, const Phys &Ph, const Dev &D,
                                         const uint8_t (&tile)[3][TY + 2][TX + 2], int lx, int ly, int x,
                                         int y, int z, bool inb, const float *__restrict__ sPrev,
                                         const float *__restrict__ muN, float *__restrict__ muO,
                                         const float4 *__restrict__ uh, float gr[5]) {
    const int nx = G.nx, ny = G.ny, nz = G.nz, nxy = nx * ny;
    const int c = inb ? x + nx * y + nxy * z : 0;
    const uint8_t fl = inb ? tile[1][ly + 1][lx + 1] : WALL;
    if (fl != LIQ) return;
    const long long S = G.S;
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
    // rigid-body velocity of particle P at this node (the same for all its links,
    // since c_q . (omega x c_q) = 0)
    auto node_velocity = [&](int P, float &u0, float &u1, float &u2) {
        const PMir m = pmir_load(D.pmir, P);
        const float rx = mirror_arm(x, m.ax, m.fx, G.nx, G.per[0]), ry = mirror_arm(y, m.ay, m.fy, G.ny, G.per[1]),
                    rz = mirror_arm(z, m.az, m.fz, G.nz, G.per[2]);
        u0 = m.ux + (m.wy * rz - m.wz * ry);
        u1 = m.uy + (m.wz * rx - m.wx * rz);
        u2 = m.uz + (m.wx * ry - m.wy * rx);
    };

    // links: bit q of sm / wm = the pull source x - c_q is solid / a wall; the
    // outgoing direction opp(q) then points into that obstacle
    uint32_t sm = 0, wm = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const uint8_t sf = tile[1 - cz(q)][ly + 1 - cy(q)][lx + 1 - cx(q)];
        sm |= (uint32_t)(sf == SOL) << q;
        if (!INTERIOR) wm |= (uint32_t)(sf == WALL) << q;
    }
    const uint32_t miss = sm | wm;

    // ---- f_t = S(s_{t-1}) at x: pull with bounce-back (same rules as the step) ----
    float fi[Q];
    float rho_t = 1.0f;
    if (miss) {
        float fo[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) fo[q] = sPrev[q * S + c];
        float d = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) d += fo[q];
        rho_t = 1.0f + d;
        fi[0] = fo[0];
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            if (!((miss >> q) & 1u)) {
                fi[q] = sPrev[q * S + src(q)];
            } else if ((sm >> q) & 1u) {
                const int P = D.pid[src(q)];
                float u0 = 0.f, u1 = 0.f, u2 = 0.f;
                if ((unsigned)P < (unsigned)D.np) node_velocity(P, u0, u1, u2);
                const float cu = cx(q) * u0 + cy(q) * u1 + cz(q) * u2;
                fi[q] = fo[opp(q)] + 6.0f * wq(q) * rho_t * cu;
            } else {
                fi[q] = fo[opp(q)];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) fi[q] = sPrev[q * S + (q ? src(q) : c)];
    }

    // ---- sbar_t = S^T mu_{t+1} + dJ_t/ds_t ----
    // s_q(x) moves to x + c_q; when that cell is an obstacle it is bounced back into
    // the pull direction opp(q) at x, which is the link with bit opp(q) set above
    float sb[Q];
    sb[0] = muN[c];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const int o = opp(q);
        if (!((miss >> o) & 1u)) sb[q] = muN[q * S + nbr(q)];
        else sb[q] = muN[o * S + c];
    }
    if (sm) {
        // moving bounce-back f_o(x) = s_q(x) + 6 w rho_t (c_o . u_w): its density term
        // reaches every s_k(x); the drag of the link is (c_o . uhat)(s_q + f_o)
        float K = 0.f;
#pragma unroll
        for (int o = 1; o < Q; ++o) {
            if (!((sm >> o) & 1u)) continue;
            const int q = opp(o);
            const int P = D.pid[src(o)];
            if ((unsigned)P >= (unsigned)D.np) continue;
            float u0, u1, u2;
            node_velocity(P, u0, u1, u2);
            const float4 e = uh[P];
            const float cu = cx(o) * u0 + cy(o) * u1 + cz(o) * u2;
            const float ce = cx(o) * e.x + cy(o) * e.y + cz(o) * e.z;
            K += 6.0f * wq(o) * cu * (sb[q] + ce);
            sb[q] += 2.0f * ce;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) sb[q] += K;
    }

    // ---- transposed collision Jacobian at f_t ----
    double drd = 0.0;
    float j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        drd += (double)fi[q];
        j0 += cx(q) * fi[q];
        j1 += cy(q) * fi[q];
        j2 += cz(q) * fi[q];
    }
    const float drho = (float)drd, rho = 1.0f + drho, irho = 1.0f / rho;
    const float g0 = Ph.g[0], g1 = Ph.g[1], g2 = Ph.g[2];
    const float u0 = j0 * irho + 0.5f * g0, u1 = j1 * irho + 0.5f * g1, u2 = j2 * irho + 0.5f * g2;
    const float uu = u0 * u0 + u1 * u1 + u2 * u2, ug = u0 * g0 + u1 * g1 + u2 * g2;
    const float lp = Ph.lp, lm = Ph.lm, ap = 1.0f + 0.5f * lp, am = 1.0f + 0.5f * lm;

    // rest population
    float a[Q];
    float Phi, D0, D1, D2, Lp, Lm = 0.f, Gg0, Gg1, Gg2;
    {
        const float w = wq(0);
        a[0] = lp * sb[0];
        const float b0 = ap * sb[0];
        const float P0 = 1.0f - 1.5f * uu, Q0 = -3.0f * ug;
        Phi = w * (-a[0] * P0 + b0 * Q0);
        D0 = w * (3.0f * a[0] * u0 - 3.0f * b0 * g0);
        D1 = w * (3.0f * a[0] * u1 - 3.0f * b0 * g1);
        D2 = w * (3.0f * a[0] * u2 - 3.0f * b0 * g2);
        const float neq = fi[0] - w * (drho + rho * (-1.5f * uu));
        Lp = sb[0] * (neq + 0.5f * rho * w * Q0);
        Gg0 = -3.0f * w * b0 * u0;
        Gg1 = -3.0f * w * b0 * u1;
        Gg2 = -3.0f * w * b0 * u2;
    }
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        if (opp(q) < q) continue;
        const int o = opp(q);
        const float w = wq(q);
        const float sp = 0.5f * (sb[q] + sb[o]), sn = 0.5f * (sb[q] - sb[o]);
        a[q] = lp * sp + lm * sn;
        a[o] = lp * sp - lm * sn;
        const float bp = 2.0f * ap * sp, bn = 2.0f * am * sn;  // b_q + b_o, b_q - b_o
        const float cu = cx(q) * u0 + cy(q) * u1 + cz(q) * u2;
        const float cg = cx(q) * g0 + cy(q) * g1 + cz(q) * g2;
        const float Pe = 1.0f + 4.5f * cu * cu - 1.5f * uu;   // even part of P_q
        const float Qe = -3.0f * ug + 9.0f * cu * cg;         // even part of Q_q
        // Phi = sum_k w_k (-a_k P_k + b_k Q_k)
        Phi += w * (-(2.0f * lp * sp) * Pe - (2.0f * lm * sn) * 3.0f * cu + bp * Qe + bn * 3.0f * cg);
        // dPhi/du / rho = sum_k w_k [-a_k (3 c_k + 9 cu_k c_k - 3 u) + b_k (9 cg_k c_k - 3 g)]
        const float tc = w * (-(2.0f * lm * sn) * 3.0f - (2.0f * lp * sp) * 9.0f * cu + bp * 9.0f * cg);
        const float tu = w * (2.0f * lp * sp) * 3.0f, tg = -w * bp * 3.0f;
        D0 += tc * cx(q) + tu * u0 + tg * g0;
        D1 += tc * cy(q) + tu * u1 + tg * g1;
        D2 += tc * cz(q) + tu * u2 + tg * g2;
        // dL/dlambda: sbar . (f - e + F/2), even and odd parts
        const float ep = w * (drho + rho * (4.5f * cu * cu - 1.5f * uu)), em = w * rho * 3.0f * cu;
        const float Xp = 0.5f * (fi[q] + fi[o]) - ep + 0.5f * rho * w * Qe;
        const float Xm = 0.5f * (fi[q] - fi[o]) - em + 0.5f * rho * w * 3.0f * cg;
        Lp += 2.0f * sp * Xp;
        Lm += 2.0f * sn * Xm;
        // sum_k w_k b_k [3 (c_k - u) + 9 cu_k c_k]
        const float gc = w * (bn * 3.0f + bp * 9.0f * cu), gu = -w * bp * 3.0f;
        Gg0 += gc * cx(q) + gu * u0;
        Gg1 += gc * cy(q) + gu * u1;
        Gg2 += gc * cz(q) + gu * u2;
    }
    // mu_t = sbar + a + dPhi/drho + dPhi/du . du/df,  du/df_q = (c_q - u + g/2) / rho
    const float v0 = -u0 + 0.5f * g0, v1 = -u1 + 0.5f * g1, v2 = -u2 + 0.5f * g2;
    const float base = Phi + D0 * v0 + D1 * v1 + D2 * v2;
#pragma unroll
    for (int q = 0; q < Q; ++q)
        muO[q * S + c] = sb[q] + a[q] + base + (cx(q) * D0 + cy(q) * D1 + cz(q) * D2);
    gr[0] = Lp;
    gr[1] = Lm;
    gr[2] = rho * (0.5f * D0 + Gg0);
    gr[3] = rho * (0.5f * D1 + Gg1);
    gr[4] = rho * (0.5f * D2 + Gg2);
}

// five waves per SIMD (91 VGPRs, no spill): at 256^3 the backward sweep takes 393 ms
// against 425 ms at the four that the register count alone allows; six waves spill
__global__ __launch_bounds__(256, 5) void k_adj_step(Geom G, Phys Ph, Dev D, const float *__restrict__ sPrev,
                                                  const float *__restrict__ muN, float *__restrict__ muO,
                                                  const float4 *__restrict__ uh, double *part, int tilesX,
                                                  int tilesY, int nTiles) {
    __shared__ uint8_t tile[3][TY + 2][TX + 2];
    __shared__ double red[4][5];
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int b = blockIdx.x;
    const int t = tile_of_block(b, nTiles);
    const int x0 = (t % tilesX) * TX;
    const int rest = t / tilesX;
    const int y0 = (rest % tilesY) * TY;
    const int z = rest / tilesY;
    const bool interior = x0 >= 1 && x0 + TX + 1 <= nx && y0 >= 1 && y0 + TY + 1 <= ny && z >= 1 &&
                          z + 2 <= nz;
    stage_flag_tile(G, D.flags, tile, x0, y0, z, interior);
    __syncthreads();
    const int lx = threadIdx.x & (TX - 1), ly = threadIdx.x >> 6;
    const int x = x0 + lx, y = y0 + ly;
    const bool inb = x < nx && y < ny;
    float gr[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (interior) adj_cell<true>(G, Ph, D, tile, lx, ly, x, y, z, inb, sPrev, muN, muO, uh, gr);
    else adj_cell<false>(G, Ph, D, tile, lx, ly, x, y, z, inb, sPrev, muN, muO, uh, gr);
    // block partials in FP64; the block owns its slot, so the sum over launches is
    // taken in launch order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double s = wave_sum((double)gr[i]);
        if (lane == 0) red[wv][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int i = threadIdx.x;
        part[(long long)b * ADJ_NPART + i] += (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
    }
}

}  // namespace fsl
