// k_particles.hpp -- rigid spheres (Sec. 2.3): force/torque hand-over from the
// per-particle FP64 accumulators of the stream-collide kernel, lubrication
// correction (Eq. lubrication) on a candidate-pair list from a uniform grid,
// substep time integration, and the obstacle-coverage update (nodes inside a
// sphere are obstacle nodes; covered / uncovered cells keep the mass ledger).
#pragma once

#include "cov_column.hpp"
#include "k_free_surface.hpp"

namespace fsl {

constexpr int CLAIM_NONE = 0x7fffffff;

// per particle: F, T of the step (reported), mass paid by moving bounce-back to the
// ledger (block reduction then one atomic per block), accumulators cleared
__global__ __launch_bounds__(256) void k_part_forces(Dev D, int integrate) {
    __shared__ double red[256];
    int P = blockIdx.x * blockDim.x + threadIdx.x;
    double dm = 0.0;
    if (P < D.np) {
        double *a = D.pacc + acc_at(P, 0);
        double *o = D.pFT + (long long)P * 6;
        double *op = D.pFTp + (long long)P * 6;
        double s[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) s[k] = a[k];
        for (int j = 1; j < ACC_COPIES; ++j)
#pragma unroll
            for (int k = 0; k < 7; ++k) s[k] += a[j * ACC_STRIDE + k];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            op[k] = o[k];
            o[k] = s[k];
        }
        dm = s[6];
        for (int k = 0; k < ACC_COPIES * ACC_STRIDE; ++k) a[k] = 0.0;
        if (integrate) {
            double *t = D.ptab + (long long)P * P_STRIDE;
            t[P_XOLD] = t[P_X];
            t[P_XOLD + 1] = t[P_X + 1];
            t[P_XOLD + 2] = t[P_X + 2];
            double *fl = D.pFl + (long long)P * 3;
            fl[0] = fl[1] = fl[2] = 0.0;
        }
    }
    red[threadIdx.x] = dm;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0.0) unsafeAtomicAdd(D.ledger, -red[0]);
}

// node box [lo, hi] of a sphere: clipped to the box along walled axes, unwrapped along
// periodic ones (node_at wraps the indices; the box never holds a node twice, see
// sphere_supported); false when nothing is left (a sphere outside the box or not
// finite, which the next synchronising call reports)
__device__ __forceinline__ bool sphere_box(const Geom &G, const double *x, double R, int lo[3], int hi[3]) {
    const int n[3] = {G.nx, G.ny, G.nz};
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const double l = floor(x[a] - R), h = ceil(x[a] + R);
        const bool in = G.per[a] ? (l >= -2.0 * n[a] && h <= 3.0 * n[a]) : (l <= n[a] - 1.0 && h >= 0.0);
        if (!in) {  // also NaN
            lo[a] = 0;
            hi[a] = -1;
            ok = false;
            continue;
        }
        if (G.per[a]) {
            lo[a] = (int)l;
            hi[a] = (int)h;
        } else {
            lo[a] = l < 0.0 ? 0 : (int)l;
            hi[a] = h > n[a] - 1.0 ? n[a] - 1 : (int)h;
        }
    }
    return ok;
}

// cell index of node coordinates that may lie beyond periodic faces (in range along
// walled axes)
__device__ __forceinline__ int node_at(const Geom &G, int i, int j, int k) {
    if (G.per[0]) i = ((i % G.nx) + G.nx) % G.nx;
    if (G.per[1]) j = ((j % G.ny) + G.ny) % G.ny;
    if (G.per[2]) k = ((k % G.nz) + G.nz) % G.nz;
    return i + G.nx * (j + G.ny * k);
}

// position of sphere t's centre as the image nearest to the point p (per axis)
__device__ __forceinline__ void image_near(const Geom &G, const double *t, const double *p, double out[3]) {
    const int n[3] = {G.nx, G.ny, G.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = p[a] + min_img(t[a] - p[a], n[a], G.per[a]);
}

__device__ __forceinline__ bool inside(double i, double j, double k, const double *x, double R) {
    double d0 = i - x[0], d1 = j - x[1], d2 = k - x[2];
    return __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2)) <= __dmul_rn(R, R);
}

// FP32 mirror used by the stream-collide kernel: integer anchor floor(x_P), the
// fraction x_P - anchor, velocity and angular velocity
__global__ void k_part_mirror(Dev D) {
    GRID_STRIDE(P, D.np) {
        const double *t = D.ptab + (long long)P * P_STRIDE;
        float4 *m = D.pmir + 4LL * P;
        double a0 = floor(t[P_X]), a1 = floor(t[P_X + 1]), a2 = floor(t[P_X + 2]);
        // PMir order: anchor, fraction, u, omega
        m[0] = make_float4((float)a0, (float)a1, (float)a2, (float)(t[P_X] - a0));
        m[1] = make_float4((float)(t[P_X + 1] - a1), (float)(t[P_X + 2] - a2), (float)t[P_U], (float)t[P_U + 1]);
        m[2] = make_float4((float)t[P_U + 2], (float)t[P_W], (float)t[P_W + 1], (float)t[P_W + 2]);
        m[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// ---- candidate pairs for lubrication: uniform grid ---------------------------------
struct PGrid {
    int g[3];
    double cs[3];
    double reach;  // pair candidate distance between surfaces
    int n[3], per[3];  // the box, for nearest images across periodic faces
};

__device__ __forceinline__ int pgrid_cell(const PGrid &PG, const double *x, int a) {
    int v = (int)floor(x[a] / PG.cs[a]);
    return v < 0 ? 0 : (v >= PG.g[a] ? PG.g[a] - 1 : v);
}

__global__ void k_grid_zero(Dev D, int ncell) { GRID_STRIDE(i, ncell) D.gridCount[i] = 0; }

__global__ void k_grid_count(Dev D, PGrid PG) {
    GRID_STRIDE(P, D.np) {
        const double *x = D.ptab + (long long)P * P_STRIDE;
        int cell = pgrid_cell(PG, x, 0) + PG.g[0] * (pgrid_cell(PG, x, 1) + PG.g[1] * pgrid_cell(PG, x, 2));
        atomicAdd(D.gridCount + cell, 1);
    }
}

// exclusive scan of the grid counts by one block; gridCount becomes the fill cursor
// exclusive prefix sum of the per-cell counts into gridStart (and the fill cursors
// in gridCount), over many blocks: block sums, a scan of the block sums (at most
// 1,024), then each block scans its own range from its offset
__global__ __launch_bounds__(256) void k_gscan_sum(Dev D, int ncell, int chunk, int *bsum) {
    __shared__ int red[256];
    const int lo = blockIdx.x * chunk, hi = min(ncell, lo + chunk);
    int s = 0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) s += D.gridCount[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(1024) void k_gscan_top(Dev D, int ncell, int nb, int *bsum) {
    __shared__ int v[1024];
    const int t = threadIdx.x;
    const int x = t < nb ? bsum[t] : 0;
    v[t] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int y = t >= o ? v[t - o] : 0;
        __syncthreads();
        v[t] += y;
        __syncthreads();
    }
    if (t < nb) bsum[t] = v[t] - x;
    if (t == 1023) D.gridStart[ncell] = v[t];
}
__global__ __launch_bounds__(256) void k_gscan_apply(Dev D, int ncell, int chunk, const int *bsum) {
    __shared__ int v[256];
    const int lo = blockIdx.x * chunk, hi = min(ncell, lo + chunk);
    const int t = threadIdx.x;
    int carry = bsum[blockIdx.x];
    for (int base = lo; base < hi; base += 256) {
        const int i = base + t;
        const int x = i < hi ? D.gridCount[i] : 0;
        v[t] = x;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int y = t >= o ? v[t - o] : 0;
            __syncthreads();
            v[t] += y;
            __syncthreads();
        }
        if (i < hi) {
            const int st = carry + v[t] - x;
            D.gridStart[i] = st;
            D.gridCount[i] = st;
        }
        carry += v[255];
        __syncthreads();
    }
}

__global__ void k_grid_fill(Dev D, PGrid PG) {
    GRID_STRIDE(P, D.np) {
        const double *x = D.ptab + (long long)P * P_STRIDE;
        int cell = pgrid_cell(PG, x, 0) + PG.g[0] * (pgrid_cell(PG, x, 1) + PG.g[1] * pgrid_cell(PG, x, 2));
        int s = atomicAdd(D.gridCount + cell, 1);
        D.gridIdx[s] = P;
    }
}

// append the pair (a, b) of every active lane with pred to a list of pairs: one
// atomic per wave (the ballot sees the active lanes only, so divergent callers are fine)
__device__ __forceinline__ void wave_push2(bool pred, int a, int b, int *list, int *counter, int cap,
                                           unsigned *err) {
    const unsigned long long mask = __ballot(pred);
    if (!mask) return;
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        const int slot = base + __popcll(mask & ((1ull << lane_id()) - 1ull));
        if (slot < cap) {
            list[2 * slot] = a;
            list[2 * slot + 1] = b;
        } else {
            atomicOr(err, ERR_CAP);
        }
    }
}

// one thread per particle and neighbouring grid cell (27 per particle), so that the
// dependent loads of the cell lists overlap across many threads.  Pairs are sparse
// (about one per wave), so they are gathered per block in LDS and appended with one
// atomic per block: one atomic per pair on the same counter serialises.
constexpr int PAIR_BUF = 1024;

__global__ __launch_bounds__(256) void k_pairs(Dev D, PGrid PG, int pcap) {
    __shared__ int2 buf[PAIR_BUF];
    __shared__ int cnt, base;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int total = D.np * 27;
    // whole blocks take the same rounds, so every thread reaches the barriers below
    for (int r = blockIdx.x * blockDim.x; r < total; r += gridDim.x * blockDim.x) {
        const int idx = r + threadIdx.x;
        if (idx >= total) continue;
        const int P = idx / 27, d = idx - 27 * P;
        const double *x = D.ptab + (long long)P * P_STRIDE;
        const int off[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
        int cc[3];
        bool skip = false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int v = pgrid_cell(PG, x, k) + off[k];
            if (PG.per[k]) {
                // a periodic axis of one or two grid cells holds each neighbour once
                if ((PG.g[k] == 1 && off[k] != 0) || (PG.g[k] == 2 && off[k] < 0)) skip = true;
                v = v < 0 ? v + PG.g[k] : (v >= PG.g[k] ? v - PG.g[k] : v);
            } else if (v < 0 || v >= PG.g[k]) {
                skip = true;
            }
            cc[k] = v;
        }
        if (skip) continue;
        const int cell = cc[0] + PG.g[0] * (cc[1] + PG.g[1] * cc[2]);
        for (int s = D.gridStart[cell]; s < D.gridStart[cell + 1]; ++s) {
            const int Qp = D.gridIdx[s];
            if (Qp <= P) continue;
            const double *y = D.ptab + (long long)Qp * P_STRIDE;
            const double d0 = min_img(y[0] - x[0], PG.n[0], PG.per[0]), d1 = min_img(y[1] - x[1], PG.n[1], PG.per[1]),
                         d2 = min_img(y[2] - x[2], PG.n[2], PG.per[2]);
            const double gap = sqrt(d0 * d0 + d1 * d1 + d2 * d2) - x[P_R] - y[P_R];
            if (gap >= PG.reach) continue;
            const int k = atomicAdd(&cnt, 1);
            if (k < PAIR_BUF) {
                buf[k] = make_int2(P, Qp);
            } else {  // the block's buffer is full: straight to the list
                const int g = atomicAdd(D.counters + C_NPAIRS, 1);
                if (g < pcap) D.pairs[g] = make_int2(P, Qp);
                else atomicOr(D.err, ERR_CAP);
            }
        }
    }
    __syncthreads();
    const int n = min(cnt, PAIR_BUF);
    if (threadIdx.x == 0) base = n ? atomicAdd(D.counters + C_NPAIRS, n) : 0;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        if (base + k < pcap) D.pairs[base + k] = buf[k];
        else atomicOr(D.err, ERR_CAP);
    }
}

// Momentum exchange between two particles (Sec. 2.3): a node inside particle P'
// with a link into particle P contributes with equilibrium populations at rho = 1
// and the rigid velocity of P' at the node, Delta j = 2 c_q e^+_q(1, u_P'(x)), to
// P's force and torque.  Such nodes exist only for pairs closer than sqrt(2), all
// of which are in the candidate list; one wave per pair scans the nodes of each
// particle that lie within one cell of the other's bounding box.
__global__ __launch_bounds__(256) void k_solid_pairs(Geom G, Dev D, int pcap) {
    const int n = min(D.counters[C_NPAIRS], pcap);
    const int lane = threadIdx.x & 63;
    for (int k = blockIdx.x * 4 + (threadIdx.x >> 6); k < n; k += gridDim.x * 4) {
    const int pa = D.pairs[k].x, pb = D.pairs[k].y;
    {
        // nodes of one sphere next to nodes of the other need the centres closer than
        // the radii plus the longest link (sqrt 2); margin 1.5
        const double *ta = D.ptab + (long long)pa * P_STRIDE, *tb = D.ptab + (long long)pb * P_STRIDE;
        const double d0 = min_img(ta[P_X] - tb[P_X], G.nx, G.per[0]), d1 = min_img(ta[P_X + 1] - tb[P_X + 1], G.ny, G.per[1]),
                     d2 = min_img(ta[P_X + 2] - tb[P_X + 2], G.nz, G.per[2]);
        const double reach = ta[P_R] + tb[P_R] + 1.5;
        if (d0 * d0 + d1 * d1 + d2 * d2 > reach * reach) continue;
    }
    for (int side = 0; side < 2; ++side) {
        const int Pp = side ? pb : pa, Po = side ? pa : pb;
        const double *tp = D.ptab + (long long)Pp * P_STRIDE, *tq = D.ptab + (long long)Po * P_STRIDE;
        // the other sphere's centre at its image nearest to this one (node coordinates
        // below stay in this sphere's frame; node_at wraps them)
        double to[3];
        image_near(G, tq + P_X, tp + P_X, to);
        const double Ro = tq[P_R];
        const double ro = (Ro + 1.5) * (Ro + 1.5);
        int lo[3], hi[3], lo2[3], hi2[3];
        sphere_box(G, tp + P_X, tp[P_R], lo, hi);
        sphere_box(G, to, Ro + 1.0, lo2, hi2);
        for (int a = 0; a < 3; ++a) { lo[a] = max(lo[a], lo2[a]); hi[a] = min(hi[a], hi2[a]); }
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        if (lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2]) {
            const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
            const int tot = ex * ey * ez;
            for (int s2 = lane; s2 < tot; s2 += 64) {
                const int i = lo[0] + s2 % ex, j = lo[1] + (s2 / ex) % ey, kk = lo[2] + s2 / (ex * ey);
                {
                    // only nodes within a link of the other sphere can have such links
                    const double e0 = i - to[0], e1 = j - to[1], e2 = kk - to[2];
                    if (e0 * e0 + e1 * e1 + e2 * e2 > ro) continue;
                }
                // a node of Pp lies inside Pp and a node of Po inside Po (coverage takes
                // the same inside test), so cells that fail it need no loads
                if (!inside(i, j, kk, tp + P_X, tp[P_R])) continue;
                const int c = node_at(G, i, j, kk);
                if (D.flags[c] != SOL || D.pid[c] != Pp) continue;
                const double rx = i - tp[P_X], ry = j - tp[P_X + 1], rz = kk - tp[P_X + 2];
                const double ur0 = tp[P_U] + (tp[P_W + 1] * rz - tp[P_W + 2] * ry);
                const double ur1 = tp[P_U + 1] + (tp[P_W + 2] * rx - tp[P_W] * rz);
                const double ur2 = tp[P_U + 2] + (tp[P_W] * ry - tp[P_W + 1] * rx);
                const double uu = ur0 * ur0 + ur1 * ur1 + ur2 * ur2;
                const double ox = i - to[0], oy = j - to[1], oz = kk - to[2];
                for (int q = 1; q < Q; ++q) {
                    if (!inside(i + cx(q), j + cy(q), kk + cz(q), to, Ro)) continue;
                    int iw, jw, kw;
                    cell_xyz(G, c, iw, jw, kw);
                    const int nb = nbr_idx(G, iw, jw, kw, q, 1);
                    if (nb < 0 || D.flags[nb] != SOL || D.pid[nb] != Po) continue;
                    const double cu = cx(q) * ur0 + cy(q) * ur1 + cz(q) * ur2;
                    const double e2 = 2.0 * wqd(q) * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                    const double j0 = cx(q) * e2, j1 = cy(q) * e2, j2 = cz(q) * e2;
                    acc[0] += j0;
                    acc[1] += j1;
                    acc[2] += j2;
                    acc[3] += oy * j2 - oz * j1;
                    acc[4] += oz * j0 - ox * j2;
                    acc[5] += ox * j1 - oy * j0;
                }
            }
        }
        double *dst = D.pacc + acc_at(Po, k & (ACC_COPIES - 1));
        for (int a = 0; a < 6; ++a) {
            const double v = wave_sum(acc[a]);
            if (lane == 0 && v != 0.0) unsafeAtomicAdd(dst + a, v);
        }
    }
    }
}

// Links into a particle's nodes from beyond the faces of the box (Eq. momentum_transfer).
// Reading: the far end is taken as a node inside another particle is, with
// equilibrium populations at rho = 1, here at the velocity of the first no-slip face
// the link crosses (at rest when it crosses free-slip faces only): Delta j = 2 c_q
// e^+_q(1, u_w), and that no-slip face takes -Delta j.  The constant parts 2 w_q c_q
// of the links into a closed node set cancel exactly; without these links a sphere
// that covers nodes of a face layer would miss them over the cut and be pulled into
// the face by the lattice pressure 1/3.  One wave per particle walks the face-layer
// nodes of its node box; the torque arm runs from the centre to the far end of the
// link.
__global__ __launch_bounds__(256) void k_face_links(Geom G, Phys Ph, Dev D) {
    const int P = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (P >= D.np) return;
    const int lane = threadIdx.x & 63;
    const double *t = D.ptab + (long long)P * P_STRIDE;
    const int n[3] = {G.nx, G.ny, G.nz};
    int lo[3], hi[3];
    sphere_box(G, t + P_X, t[P_R], lo, hi);
    bool touch = false;
    for (int a = 0; a < 3; ++a)
        if (!G.per[a] && lo[a] <= hi[a] && (lo[a] == 0 || hi[a] == n[a] - 1)) touch = true;
    if (!touch) return;  // the whole wave: no face layer in reach
    double acc[6] = {0, 0, 0, 0, 0, 0};
    // the face layers of the walled axes that the node box reaches; a node on the
    // layers of two axes is taken with the lower axis
    for (int a = 0; a < 3; ++a) {
        if (G.per[a]) continue;
        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;  // the other two axes
        const int eb = hi[b] - lo[b] + 1, ed = hi[d] - lo[d] + 1;
        for (int side = 0; side < 2; ++side) {
            const int layer = side ? n[a] - 1 : 0;
            if (layer < lo[a] || layer > hi[a] || (side && n[a] == 1)) continue;
            for (int s = lane; s < eb * ed; s += 64) {
                int p[3];
                p[a] = layer;
                p[b] = lo[b] + s % eb;
                p[d] = lo[d] + s / eb;
                bool lower = false;
                for (int k = 0; k < a; ++k)
                    if (!G.per[k] && (p[k] == 0 || p[k] == n[k] - 1)) lower = true;
                if (lower || !inside(p[0], p[1], p[2], t + P_X, t[P_R])) continue;
                const int c = node_at(G, p[0], p[1], p[2]);
                if (D.flags[c] != SOL || D.pid[c] != P) continue;
                for (int q = 1; q < Q; ++q) {
                    const int f[3] = {p[0] - cx(q), p[1] - cy(q), p[2] - cz(q)};  // far end
                    int fa = -1;
                    bool crossed = false;
                    for (int k = 0; k < 3; ++k) {
                        if (G.per[k] || (f[k] >= 0 && f[k] < n[k])) continue;
                        crossed = true;
                        if (fa < 0 && !Ph.slip[k]) fa = k;
                    }
                    if (!crossed) continue;
                    const int sd = fa >= 0 && f[fa] >= 0 ? 1 : 0;
                    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
                    if (fa >= 0) {
                        const float *uw = D.wallu + (fa * 2 + sd) * 3;
                        u0 = uw[0];
                        u1 = uw[1];
                        u2 = uw[2];
                    }
                    const double cu = cx(q) * u0 + cy(q) * u1 + cz(q) * u2;
                    const double e2 = 2.0 * wqd(q) * (1.0 + 4.5 * cu * cu - 1.5 * (u0 * u0 + u1 * u1 + u2 * u2));
                    const double j0 = cx(q) * e2, j1 = cy(q) * e2, j2 = cz(q) * e2;
                    const double r0 = f[0] - t[P_X], r1 = f[1] - t[P_X + 1], r2 = f[2] - t[P_X + 2];
                    acc[0] += j0;
                    acc[1] += j1;
                    acc[2] += j2;
                    acc[3] += r1 * j2 - r2 * j1;
                    acc[4] += r2 * j0 - r0 * j2;
                    acc[5] += r0 * j1 - r1 * j0;
                    if (fa >= 0 && D.wallF) {
                        double *w = D.wallF + 3 * (2 * fa + sd);
                        if (j0 != 0.0) unsafeAtomicAdd(w, -j0);
                        if (j1 != 0.0) unsafeAtomicAdd(w + 1, -j1);
                        if (j2 != 0.0) unsafeAtomicAdd(w + 2, -j2);
                    }
                }
            }
        }
    }
    double *dst = D.pacc + acc_at(P, P & (ACC_COPIES - 1));
    for (int a = 0; a < 6; ++a) {
        const double v = wave_sum(acc[a]);
        if (lane == 0 && v != 0.0) unsafeAtomicAdd(dst + a, v);
    }
}

// Pair force of one candidate pair (x, u of each sphere; f: force on sphere 1, sphere 2
// takes -f).  Contact (the paper gives no contact model; reading): overlapping spheres
// repel by a linear spring of stiffness kc along the line of centres, -kc (R1 + R2 -
// |d|) d/|d|.  Eq. (lubrication): only for gaps below Delta_c = 2/3, the gap limited
// from below by 0.2 Delta_c.  The partner is taken at its nearest periodic image.
// Returns false when there is no force.
__device__ __forceinline__ bool pair_force(const Geom &G, const double *x1, const double *u1, double R1,
                                           const double *x2, const double *u2, double R2, double mu, double kc,
                                           double f[3]) {
    const double dc = 2.0 / 3.0;
    const double d0 = min_img(x2[0] - x1[0], G.nx, G.per[0]), d1 = min_img(x2[1] - x1[1], G.ny, G.per[1]),
                 d2 = min_img(x2[2] - x1[2], G.nz, G.per[2]);
    const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double sR = R1 + R2;
    double gap = dist - sR;
    f[0] = f[1] = f[2] = 0.0;
    if (kc > 0.0 && dist < sR && dist > 0.0) {
        const double s = -kc * (sR - dist) / dist;
        f[0] = s * d0;
        f[1] = s * d1;
        f[2] = s * d2;
    }
    if (gap < dc && dist > 0.0) {
        if (gap < 0.2 * dc) gap = 0.2 * dc;
        const double n0 = d0 / dist, n1 = d1 / dist, n2 = d2 / dist;
        const double rr = R1 * R2;
        const double coef = -6.0 * M_PI * mu * (rr * rr) / (sR * sR) * (1.0 / gap - 1.0 / dc);
        const double vn = n0 * (u1[0] - u2[0]) + n1 * (u1[1] - u2[1]) + n2 * (u1[2] - u2[2]);
        f[0] += coef * vn * n0;
        f[1] += coef * vn * n1;
        f[2] += coef * vn * n2;
    }
    return f[0] != 0.0 || f[1] != 0.0 || f[2] != 0.0;
}

// Force of the no-slip faces (axes with bit a of wmask; faces at -1/2 and n - 1/2) on
// one sphere, added to f.  Eq. (lubrication) and contact are stated for particle
// pairs; reading: a face is a resting sphere of infinite radius touching the face
// plane, so (R1 R2)^2/(R1 + R2)^2 becomes R^2, the pair normal the face normal and
// the gap h - R (h: distance of the centre from the face).  For a gap below Delta_c,
// limited from below by 0.2 Delta_c, that leaves a drag -6 pi mu R^2 (1/gap -
// 1/Delta_c) on the velocity component normal to the face, whichever the side; an
// overlapping sphere (h < R) is pushed off the face by kc (R - h).
__device__ __forceinline__ void face_force(const Geom &G, int wmask, const double *x, const double *u, double R,
                                           double mu, double kc, double f[3]) {
    const double dc = 2.0 / 3.0;
    const int n[3] = {G.nx, G.ny, G.nz};
    for (int a = 0; a < 3; ++a) {
        if (!((wmask >> a) & 1)) continue;
        const double hl = x[a] + 0.5, hh = (n[a] - 0.5) - x[a];
        if (kc > 0.0) {
            if (hl < R) f[a] += kc * (R - hl);
            if (hh < R) f[a] -= kc * (R - hh);
        }
        const double c = 6.0 * M_PI * mu * R * R;
        double gl = hl - R, gh = hh - R;
        if (gl < dc) f[a] -= c * (1.0 / fmax(gl, 0.2 * dc) - 1.0 / dc) * u[a];
        if (gh < dc) f[a] -= c * (1.0 / fmax(gh, 0.2 * dc) - 1.0 / dc) * u[a];
    }
}

__global__ void k_lub(Geom G, Dev D, double mu, double kc, int pcap) {
    int n = min(D.counters[C_NPAIRS], pcap);
    GRID_STRIDE(k, n) {
        const int a = D.pairs[k].x, b = D.pairs[k].y;
        const double *p1 = D.ptab + (long long)a * P_STRIDE, *p2 = D.ptab + (long long)b * P_STRIDE;
        double f[3];
        if (!pair_force(G, p1 + P_X, p1 + P_U, p1[P_R], p2 + P_X, p2 + P_U, p2[P_R], mu, kc, f)) continue;
        unsafeAtomicAdd(D.pFl + 3 * a, f[0]);
        unsafeAtomicAdd(D.pFl + 3 * a + 1, f[1]);
        unsafeAtomicAdd(D.pFl + 3 * a + 2, f[2]);
        unsafeAtomicAdd(D.pFl + 3 * b, -f[0]);
        unsafeAtomicAdd(D.pFl + 3 * b + 1, -f[1]);
        unsafeAtomicAdd(D.pFl + 3 * b + 2, -f[2]);
    }
}

// one semi-implicit Euler substep of particle t (x, u, omega may live elsewhere than
// the table): velocity from F_hyd + m g + F_pair, then position; angular velocity from
// T_hyd; the no-slip faces act through face_force at the position and velocity the
// substep starts from; normal velocity reversed when closer than R to a wall face and
// moving towards it; along a periodic axis the centre kept in [0, n).  F_hyd, T_hyd are the mean of
// this and the previous step's momentum exchange (two-step average that removes the
// period-two oscillation of explicit coupling), or this step's alone after a reset.
__device__ __forceinline__ void substep_one(const Geom &G, const Dev &D, int P, double *x, double *u, double *w,
                                            double *fl, double dt, const double gg[3], int have_prev, double mu,
                                            double kc, int wmask) {
    const double *t = D.ptab + (long long)P * P_STRIDE;
    const double *FTn = D.pFT + (long long)P * 6, *FTp = D.pFTp + (long long)P * 6;
    const double R = t[P_R];
    if (wmask) face_force(G, wmask, x, u, R, mu, kc, fl);
    const double mP = t[P_RHO] * (4.0 / 3.0) * M_PI * R * R * R;
    const double IP = 0.4 * mP * R * R;
    const int n[3] = {G.nx, G.ny, G.nz};
    for (int d = 0; d < 3; ++d) {
        const double Fh = have_prev ? 0.5 * (FTn[d] + FTp[d]) : FTn[d];
        const double Th = have_prev ? 0.5 * (FTn[3 + d] + FTp[3 + d]) : FTn[3 + d];
        const double F = Fh + mP * gg[d] + fl[d];
        u[d] += dt * F / mP;
        x[d] += dt * u[d];
        if (G.per[d]) x[d] = wrap_coord(x[d], n[d]);
        w[d] += dt * Th / IP;
        if (!G.per[d]) {
            if (x[d] < R - 0.5 && u[d] < 0) u[d] = -u[d];
            if (x[d] > n[d] - 0.5 - R && u[d] > 0) u[d] = -u[d];
        }
        fl[d] = 0.0;
    }
}

__global__ void k_substep(Dev D, Geom G, double dt, double g0, double g1, double g2, int have_prev, double mu,
                          double kc, int wmask) {
    GRID_STRIDE(P, D.np) {
        double *t = D.ptab + (long long)P * P_STRIDE;
        const double gg[3] = {g0, g1, g2};
        substep_one(G, D, P, t + P_X, t + P_U, t + P_W, D.pFl + (long long)P * 3, dt, gg, have_prev, mu, kc,
                    wmask);
        const int n[3] = {G.nx, G.ny, G.nz};
        if (!sphere_supported(t + P_X, t[P_R], n, G.per)) atomicOr(D.err, ERR_PART);
    }
}

// All ns substeps in one block for small tables (np <= INT_BLOCK_MAX): centres,
// velocities and pair forces in LDS, so that a substep's pair phase sees the
// previous substep's update after a barrier; the same arithmetic as k_lub and
// k_substep, which take one launch each per substep.
constexpr int INT_BLOCK_MAX = 512;
__global__ __launch_bounds__(1024) void k_integrate_block(Geom G, Dev D, int ns, double mu, double kc, int pcap,
                                                          double g0, double g1, double g2, int have_prev,
                                                          int wmask) {
    __shared__ double sx[INT_BLOCK_MAX][3], su[INT_BLOCK_MAX][3], sf[INT_BLOCK_MAX][3];
    const int np = D.np, npair = min(D.counters[C_NPAIRS], pcap);
    for (int P = threadIdx.x; P < np; P += blockDim.x) {
        const double *t = D.ptab + (long long)P * P_STRIDE;
        for (int d = 0; d < 3; ++d) {
            sx[P][d] = t[P_X + d];
            su[P][d] = t[P_U + d];
            sf[P][d] = D.pFl[3 * P + d];
        }
    }
    __syncthreads();
    const double dt = 1.0 / ns, gg[3] = {g0, g1, g2};
    for (int s = 0; s < ns; ++s) {
        for (int k = threadIdx.x; k < npair; k += blockDim.x) {
            const int a = D.pairs[k].x, b = D.pairs[k].y;
            double f[3];
            if (!pair_force(G, sx[a], su[a], D.ptab[(long long)a * P_STRIDE + P_R], sx[b], su[b],
                            D.ptab[(long long)b * P_STRIDE + P_R], mu, kc, f))
                continue;
            for (int d = 0; d < 3; ++d) {
                atomicAdd(&sf[a][d], f[d]);
                atomicAdd(&sf[b][d], -f[d]);
            }
        }
        __syncthreads();
        for (int P = threadIdx.x; P < np; P += blockDim.x)
            substep_one(G, D, P, sx[P], su[P], D.ptab + (long long)P * P_STRIDE + P_W, sf[P], dt, gg, have_prev, mu,
                        kc, wmask);
        __syncthreads();
    }
    for (int P = threadIdx.x; P < np; P += blockDim.x) {
        double *t = D.ptab + (long long)P * P_STRIDE;
        for (int d = 0; d < 3; ++d) {
            t[P_X + d] = sx[P][d];
            t[P_U + d] = su[P][d];
            D.pFl[3 * P + d] = 0.0;
        }
        const int n[3] = {G.nx, G.ny, G.nz};
        if (!sphere_supported(t + P_X, t[P_R], n, G.per)) atomicOr(D.err, ERR_PART);
    }
}

// ---- coverage update --------------------------------------------------------------
// Which spheres resolve their coverage through claims (lowest index wins an
// overlap): those with a candidate partner whose centre is closer than the radii
// plus one cell at the new positions, and those that moved half a cell or more.
// For every other sphere no node can be inside it and another sphere at once, so
// its cover and uncover events follow from the inside tests at the old and new
// positions alone.
__global__ void k_cov_flag_init(Geom G, Dev D) {
    GRID_STRIDE(P, D.np) {
        double *t = D.ptab + (long long)P * P_STRIDE;
        const double m = fmax(fabs(min_img(t[P_X] - t[P_XOLD], G.nx, G.per[0])),
                              fmax(fabs(min_img(t[P_X + 1] - t[P_XOLD + 1], G.ny, G.per[1])),
                                   fabs(min_img(t[P_X + 2] - t[P_XOLD + 2], G.nz, G.per[2]))));
        t[P_OVL] = 0.0;
        // a sphere that moved half a cell or more in one step may meet partners that
        // the pair list (taken at the old positions) does not hold: then every
        // sphere takes the claim path this step
        if (m >= 0.5) atomicOr(D.counters + C_COVALL, 1);
    }
}
__device__ __forceinline__ bool cov_claims(const Dev &D, const double *t) {
    return t[P_OVL] != 0.0 || D.counters[C_COVALL] != 0;
}
__global__ void k_cov_flag_pairs(Geom G, Dev D, int pcap) {
    const int n = min(D.counters[C_NPAIRS], pcap);
    GRID_STRIDE(k, n) {
        const int a = D.pairs[k].x, b = D.pairs[k].y;
        double *ta = D.ptab + (long long)a * P_STRIDE, *tb = D.ptab + (long long)b * P_STRIDE;
        const double d0 = min_img(ta[P_X] - tb[P_X], G.nx, G.per[0]), d1 = min_img(ta[P_X + 1] - tb[P_X + 1], G.ny, G.per[1]),
                     d2 = min_img(ta[P_X + 2] - tb[P_X + 2], G.nz, G.per[2]);
        const double r = ta[P_R] + tb[P_R] + 1.0;
        if (d0 * d0 + d1 * d1 + d2 * d2 < r * r) {
            ta[P_OVL] = 1.0;
            tb[P_OVL] = 1.0;
        }
    }
}

// one wave per particle walks its bounding box; all = 0 limits the claims to the
// spheres flagged above
__global__ __launch_bounds__(256) void k_cov_claim(Geom G, Dev D, int all) {
    int P = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (P >= D.np) return;
    const double *t = D.ptab + (long long)P * P_STRIDE;
    if (!all && !cov_claims(D, t)) return;
    int lo[3], hi[3];
    sphere_box(G, t + P_X, t[P_R], lo, hi);
    int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    int tot = ex * ey * ez;
    for (int s = threadIdx.x & 63; s < tot; s += 64) {
        int i = lo[0] + s % ex, j = lo[1] + (s / ex) % ey, k = lo[2] + s / (ex * ey);
        if (inside(i, j, k, t + P_X, t[P_R])) atomicMin(D.claim + node_at(G, i, j, k), P);
    }
}

__device__ __forceinline__ int event_len(const Dev &D, int which) {
    int n = D.counters[which];
    return n < D.capEv ? n : D.capEv;
}

__device__ __forceinline__ void push_event(const Dev &D, int *list, int which, int cell, int P) {
    int s = atomicAdd(D.counters + which, 1);
    if (s < D.capEv) { list[2 * s] = cell; list[2 * s + 1] = P; }
    else atomicOr(D.err, ERR_CAP);
}

__device__ __forceinline__ void classify_node(const Dev &D, int c, int P) {
    int cl = D.claim[c];
    uint8_t f = D.flags[c];
    bool owned = (f == SOL) && D.pid[c] == P;
    if (owned && cl == CLAIM_NONE) push_event(D, D.lUnc, C_NUNCOVER, c, P);
    if (cl == P && !owned) {
        if (f == SOL) D.pid[c] = P;  // owner changes to the lower index
        else push_event(D, D.lCov, C_NCOVER, c, P);
    }
}

// walks the union of the old and new bounding boxes
__global__ __launch_bounds__(256) void k_cov_scan(Geom G, Dev D) {
    int P = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (P >= D.np) return;
    const double *t = D.ptab + (long long)P * P_STRIDE;
    // the old centre at its image nearest the new one: both boxes in one frame
    double xo[3];
    image_near(G, t + P_XOLD, t + P_X, xo);
    int lo[3], hi[3], lo2[3], hi2[3];
    const bool inNew = sphere_box(G, t + P_X, t[P_R], lo, hi);
    const bool inOld = sphere_box(G, xo, t[P_R], lo2, hi2);
    if (!inNew && !inOld) return;
    for (int a = 0; a < 3; ++a) {
        lo[a] = !inNew ? lo2[a] : !inOld ? lo[a] : min(lo[a], lo2[a]);
        hi[a] = !inNew ? hi2[a] : !inOld ? hi[a] : max(hi[a], hi2[a]);
    }
    if (cov_claims(D, t)) {
        // by cell index: along a periodic axis n consecutive nodes hold every cell once
        const int n[3] = {G.nx, G.ny, G.nz};
        for (int a = 0; a < 3; ++a)
            if (G.per[a]) hi[a] = min(hi[a], lo[a] + n[a] - 1);
        const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
        const int tot = ex * ey * ez;
        for (int s = threadIdx.x & 63; s < tot; s += 64) {
            int i = lo[0] + s % ex, j = lo[1] + (s / ex) % ey, k = lo[2] + s / (ex * ey);
            classify_node(D, node_at(G, i, j, k), P);
        }
        return;
    }
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1;
    // a sphere alone (it moved less than half a cell): only nodes whose inside test
    // changed between the old and new positions can change owner.  Walked as (x, y) columns: the in-plane part of
    // both squared distances is formed once per column, in the order of inside(), and
    // a column outside both circles is skipped (adding dz^2 cannot bring it inside);
    // cov_column_ranges gives the candidates of the others, and every candidate
    // still takes the exact test.
    const double *xn = t + P_X;
    const double R2 = __dmul_rn(t[P_R], t[P_R]);
    for (int s = threadIdx.x & 63; s < ex * ey; s += 64) {
        const int i = lo[0] + s % ex, j = lo[1] + s / ex;
        const double a0 = i - xn[0], a1 = j - xn[1], b0 = i - xo[0], b1 = j - xo[1];
        const double sn = __dadd_rn(__dmul_rn(a0, a0), __dmul_rn(a1, a1));
        const double so = __dadd_rn(__dmul_rn(b0, b0), __dmul_rn(b1, b1));
        if (sn > R2 && so > R2) continue;
        int r[4];  // candidate ranges of k
        cov_column_ranges(sn, so, R2, xn[2], xo[2], lo[2], hi[2], r);
        const int r1lo = r[0], r2lo = r[2];
        const int n1 = max(r[1] - r1lo + 1, 0), n2 = max(r[3] - r2lo + 1, 0);
        for (int m = 0; m < n1 + n2; ++m) {
            const int k = m < n1 ? r1lo + m : r2lo + (m - n1);
            const double a2 = k - xn[2], b2 = k - xo[2];
            const bool in_new = __dadd_rn(sn, __dmul_rn(a2, a2)) <= R2;
            const bool in_old = __dadd_rn(so, __dmul_rn(b2, b2)) <= R2;
            bool cov = false, unc = false;
            const int c = node_at(G, i, j, k);
            if (in_new != in_old) {
                const uint8_t f = D.flags[c];
                cov = in_new && f != SOL;
                unc = !in_new && f == SOL && D.pid[c] == P;
            }
            wave_push2(cov, c, P, D.lCov, D.counters + C_NCOVER, D.capEv, D.err);
            wave_push2(unc, c, P, D.lUnc, D.counters + C_NUNCOVER, D.capEv, D.err);
        }
    }
}

// full-box variant used when the table is replaced (no previous positions)
__global__ void k_cov_scan_dense(Geom G, Dev D) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        int cl = D.claim[c];
        uint8_t f = D.flags[c];
        if (f == SOL) {
            if (cl == CLAIM_NONE) push_event(D, D.lUnc, C_NUNCOVER, (int)c, D.pid[c]);
            else D.pid[c] = cl;
        } else if (cl != CLAIM_NONE) {
            push_event(D, D.lCov, C_NCOVER, (int)c, cl);
        }
    }
}

// the ledger takes the covered mass summed per wave (one atomic per wave): every
// wave of the block takes the same rounds, so the sums see whole waves
template <int ST>
__global__ void k_cov_apply(Geom G, Phys Ph, Dev D, double *phi) {
    const int n = event_len(D, C_NCOVER);
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int e = base + threadIdx.x;
        double led = 0.0;
        if (e < n) {
            const int c = D.lCov[2 * e], P = D.lCov[2 * e + 1];
            const uint8_t f = D.flags[c];
            if (f == LIQ) led = cell_rho<ST>(G, D, Ph, D.fB, c);
            else if (f == IFC) led = D.m[c];
            else if (f == GAS) D.cv[c] = CV_GRM;  // left the gas: for the splitting test
            D.flags[c] = SOL;
            D.pid[c] = P;
            phi[c] = 0.0;
        }
        led = wave_sum(led);
        if (lane_id() == 0 && led != 0.0) unsafeAtomicAdd(D.ledger, led);
    }
}

// decision with the flags after covering (uncovered nodes are still solid)
template <int ST>
__global__ void k_unc_decide(Geom G, Phys Ph, Dev D) {
    int n = event_len(D, C_NUNCOVER);
    GRID_STRIDE(e, n) {
        int c = D.lUnc[2 * e], x, y, z;
        cell_xyz(G, c, x, y, z);
        int nli = 0, gfirst = -1;
        double rs = 0.0;
        for (int q = 1; q < Q; ++q) {
            int nb = nbr_idx(G, x, y, z, q, 1);
            if (nb < 0) continue;
            uint8_t f = D.flags[nb];
            if (f == LIQ || f == IFC) {
                rs += cell_rho<ST>(G, D, Ph, D.fB, nb);
                ++nli;
            } else if (f == GAS && gfirst < 0) {
                gfirst = nb;
            }
        }
        int type = nli > 0 ? (gfirst >= 0 ? IFC : LIQ) : (gfirst >= 0 ? GAS : LIQ);
        int bub = gfirst >= 0 ? D.bub[gfirst] : 0;
        D.uncDec[e] = type | (bub << 8);
        D.uncRho[e] = nli > 0 ? rs / nli : 1.0;
    }
}

template <int ST>
__global__ void k_unc_apply(Geom G, Phys Ph, Dev D, double *phi) {
    int n = event_len(D, C_NUNCOVER);
    GRID_STRIDE(e, n) {
        int c = D.lUnc[2 * e], P = D.lUnc[2 * e + 1], x, y, z;
        cell_xyz(G, c, x, y, z);
        int type = D.uncDec[e] & 0xff, bub = D.uncDec[e] >> 8;
        double rb = D.uncRho[e];
        D.pid[c] = -1;
        D.flags[c] = (uint8_t)type;
        if (type == GAS) {
            D.bub[c] = (uint16_t)bub;
            phi[c] = 0.0;
            D.cv[c] = CV_GAD;  // new gas: for the splitting test
            continue;
        }
        float u0 = 0.f, u1 = 0.f, u2 = 0.f;
        if ((unsigned)P < (unsigned)D.np) {
            const double *t = D.ptab + (long long)P * P_STRIDE;
            double rx = min_img(x - t[P_X], G.nx, G.per[0]), ry = min_img(y - t[P_X + 1], G.ny, G.per[1]),
                   rz = min_img(z - t[P_X + 2], G.nz, G.per[2]);
            u0 = (float)(t[P_U] + (t[P_W + 1] * rz - t[P_W + 2] * ry));
            u1 = (float)(t[P_U + 1] + (t[P_W + 2] * rx - t[P_W] * rz));
            u2 = (float)(t[P_U + 2] + (t[P_W] * ry - t[P_W + 1] * rx));
        }
        store_equilibrium<ST>(G, Ph, D.fB, c, rb - 1.0, u0, u1, u2);
        // the density of the stored populations, for rho_w (Eq. bbrule) in the next launch
        if (D.rhow != nullptr && D.st_cur >= 0)
            D.rhow[c] = rhow_word((float)cell_rho<ST>(G, D, Ph, D.fB, c), D.st_cur);
        unsafeAtomicAdd(D.ledger, -rb);
        phi[c] = 1.0;
        if (type == IFC) {
            D.m[c] = rb;
            D.bub[c] = (uint16_t)bub;
        }
    }
}

__global__ void k_unc_closure(Geom G, Dev D, double *phi) {
    int n = event_len(D, C_NUNCOVER);
    GRID_STRIDE(e, n) {
        int c = D.lUnc[2 * e], x, y, z;
        if ((D.uncDec[e] & 0xff) != LIQ) continue;
        cell_xyz(G, c, x, y, z);
        for (int q = 1; q < Q; ++q) {
            int nb = nbr_idx(G, x, y, z, q, 1);
            if (nb >= 0 && D.flags[nb] == GAS) {
                D.flags[c] = IFC;
                D.m[c] = D.uncRho[e];
                phi[c] = 1.0;
                D.bub[c] = D.bub[nb];
                break;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_cov_reset(Geom G, Dev D) {
    int P = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (P >= D.np) return;
    const double *t = D.ptab + (long long)P * P_STRIDE;
    if (!cov_claims(D, t)) return;
    int lo[3], hi[3];
    sphere_box(G, t + P_X, t[P_R], lo, hi);
    int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    int tot = ex * ey * ez;
    for (int s = threadIdx.x & 63; s < tot; s += 64) {
        int i = lo[0] + s % ex, j = lo[1] + (s / ex) % ey, k = lo[2] + s / (ex * ey);
        D.claim[node_at(G, i, j, k)] = CLAIM_NONE;
    }
}

}  // namespace fsl
