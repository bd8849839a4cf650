// k_free_surface.hpp -- list-driven cell conversions (Sec. 2.2, Fig.
// cellConversions) and the bubble model (end of Sec. 2.2).
//
// The stream-collide kernel leaves two lists of interface cells: filled
// (phi >= 1 - eps_c) and emptied (phi <= eps_c).  The kernels below, in order:
//   mark     : conversion marks of the listed cells
//   closure  : conflict rule (an emptied cell next to a filled one stays interface),
//              gas neighbours of filled cells and liquid neighbours of emptied cells
//              become new interface cells (one winner per cell by an atomic OR)
//   init     : new interface cells from gas take the equilibrium at the mean density
//              and velocity of their liquid/interface neighbours, m = 0; new
//              interface cells from liquid keep m = rho and take the bubble id of
//              their first emptied neighbour
//   finalize : cell types
//   excess   : excess mass (m - rho, or m) shared equally by the neighbours that are
//              interface now (FP64 atomics), or paid into the ledger
//   fill     : fill levels of the recipients, marks cleared, invariant checked,
//              bubble merges recorded
// Every step of this phase touches only the listed cells and their neighbours.
#pragma once

#include "fsl_device.hpp"

namespace fsl {

__device__ __forceinline__ void cell_xyz(const Geom &G, int c, int &x, int &y, int &z) {
    x = c % G.nx;
    int r = c / G.nx;
    y = r % G.ny;
    z = r / G.ny;
}

// neighbour index of c along q, -1 beyond a wall
__device__ __forceinline__ int nbr_idx(const Geom &G, int x, int y, int z, int q, int sign) {
    int a = x + sign * cx(q), b = y + sign * cy(q), d = z + sign * cz(q);
    if (a < 0 || a >= G.nx) { if (!G.per[0]) return -1; a = wrapc(a, G.nx); }
    if (b < 0 || b >= G.ny) { if (!G.per[1]) return -1; b = wrapc(b, G.ny); }
    if (d < 0 || d >= G.nz) { if (!G.per[2]) return -1; d = wrapc(d, G.nz); }
    return a + G.nx * (b + G.ny * d);
}

template <int ST>
__device__ __forceinline__ double cell_rho(const Geom &G, const Dev &D, const Phys &Ph, const void *F, int c) {
    using SS = Store<ST>;
    const typename SS::T *p = (const typename SS::T *)F;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += (double)SS::ld(p + q * G.S + c, Ph.inv);
    return 1.0 + s;
}

// density deviation drho = rho - 1 and velocity of the post-collision populations
// (first moment minus half the Guo force)
template <int ST>
__device__ __forceinline__ void cell_rho_u(const Geom &G, const Phys &Ph, const void *F, int c,
                                           float &drho, float &u0, float &u1, float &u2) {
    using SS = Store<ST>;
    const typename SS::T *p = (const typename SS::T *)F;
    float d = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float h = SS::ld(p + q * G.S + c, Ph.inv);
        d += h;
        j0 += cx(q) * h;
        j1 += cy(q) * h;
        j2 += cz(q) * h;
    }
    drho = d;
    const float rho = 1.0f + d;
    u0 = j0 / rho - 0.5f * Ph.g[0];
    u1 = j1 / rho - 0.5f * Ph.g[1];
    u2 = j2 / rho - 0.5f * Ph.g[2];
}

// shifted equilibrium e_q(rho,u) - w_q written to cell c; drho = rho - 1 is passed
// separately so that it keeps its own precision
template <int ST>
__device__ __forceinline__ void store_equilibrium(const Geom &G, const Phys &Ph, void *F, int c,
                                                  double drho_d, float u0, float u1, float u2) {
    using SS = Store<ST>;
    typename SS::T *p = (typename SS::T *)F;
    const float drho = (float)drho_d;
    const float rho = 1.0f + drho;
    float uu = u0 * u0 + u1 * u1 + u2 * u2;
    // moving populations in FP32; the rest population carries the exact mass balance
    // sum_q h_q = rho - 1 (the equilibrium's zeroth moment), so that the rounded
    // weights do not bias the mass of the cell
    double s = 0.0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        float cu = cx(q) * u0 + cy(q) * u1 + cz(q) * u2;
        float h = wq(q) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
        const typename SS::T v = SS::enc(h, Ph.scale);
        s += (double)SS::dec(v, Ph.inv);
        p[q * G.S + c] = v;
    }
    SS::st(p + c, (float)(drho_d - s), Ph.scale);
}

__device__ __forceinline__ uint8_t cv_or(uint8_t *cv, int c, uint8_t bits) {
    unsigned *w = (unsigned *)(cv + (c & ~3));
    int sh = 8 * (c & 3);
    unsigned old = atomicOr(w, (unsigned)bits << sh);
    return (uint8_t)(old >> sh);
}

__device__ __forceinline__ int list_len(const Dev &D, int which) {
    int n = D.counters[which];
    return n < D.cap ? n : D.cap;
}

__device__ __forceinline__ void list_push(const Dev &D, int *list, int which, int v) {
    int s = atomicAdd(D.counters + which, 1);
    if (s < D.cap) list[s] = v;
    else atomicOr(D.err, ERR_CAP);
}

#define GRID_STRIDE(i, n) for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

__global__ void k_conv_mark(Dev D) {
    int nF = list_len(D, C_NF), nE = list_len(D, C_NE0);
    GRID_STRIDE(i, nF) D.cv[D.lF[i]] = CV_F;
    GRID_STRIDE(i, nE) D.cv[D.lE0[i]] = CV_E0;
}

__global__ void k_conv_closure(Geom G, Dev D) {
    int nF = list_len(D, C_NF), nE = list_len(D, C_NE0);
    GRID_STRIDE(i, nE) {
        int c = D.lE0[i], x, y, z;
        cell_xyz(G, c, x, y, z);
        bool keep = true;
        for (int q = 1; q < Q && keep; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n >= 0 && D.cv[n] == CV_F) keep = false;
        }
        if (!keep) continue;
        cv_or(D.cv, c, CV_E);
        list_push(D, D.lE, C_NE, c);
        for (int q = 1; q < Q; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n < 0 || D.flags[n] != LIQ) continue;
            if (!(cv_or(D.cv, n, CV_NEWL) & CV_NEWL)) list_push(D, D.lNL, C_NNL, n);
        }
    }
    GRID_STRIDE(i, nF) {
        int c = D.lF[i], x, y, z;
        cell_xyz(G, c, x, y, z);
        for (int q = 1; q < Q; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n < 0 || D.flags[n] != GAS) continue;
            if (!(cv_or(D.cv, n, CV_NEWG) & CV_NEWG)) list_push(D, D.lNG, C_NNG, n);
        }
    }
}

template <int ST>
__global__ void k_conv_init(Geom G, Phys Ph, Dev D) {
    int nG = list_len(D, C_NNG), nL = list_len(D, C_NNL);
    GRID_STRIDE(i, nG) {
        int c = D.lNG[i], x, y, z;
        cell_xyz(G, c, x, y, z);
        float rs = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
        int cnt = 0;
        for (int q = 1; q < Q; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n < 0) continue;
            uint8_t f = D.flags[n];
            if (f != LIQ && f != IFC) continue;
            float r, a, b, e;
            cell_rho_u<ST>(G, Ph, D.fB, n, r, a, b, e);
            rs += r;
            s0 += a;
            s1 += b;
            s2 += e;
            ++cnt;
        }
        float inv = 1.0f / (float)cnt;
        store_equilibrium<ST>(G, Ph, D.fB, c, (double)(rs * inv), s0 * inv, s1 * inv, s2 * inv);
        D.m[c] = 0.0;
    }
    GRID_STRIDE(i, nL) {
        int c = D.lNL[i], x, y, z;
        cell_xyz(G, c, x, y, z);
        D.m[c] = cell_rho<ST>(G, D, Ph, D.fB, c);
        for (int q = 1; q < Q; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n >= 0 && (D.cv[n] & CV_E)) { D.bub[c] = D.bub[n]; break; }
        }
    }
}

__global__ void k_conv_finalize(Dev D) {
    int nF = list_len(D, C_NF), nE = list_len(D, C_NE), nG = list_len(D, C_NNG), nL = list_len(D, C_NNL);
    GRID_STRIDE(i, nF) D.flags[D.lF[i]] = LIQ;
    GRID_STRIDE(i, nE) D.flags[D.lE[i]] = GAS;
    GRID_STRIDE(i, nG) D.flags[D.lNG[i]] = IFC;
    GRID_STRIDE(i, nL) D.flags[D.lNL[i]] = IFC;
}

template <int ST>
__device__ __forceinline__ void share_excess(const Geom &G, const Dev &D, int c, double ex) {
    int x, y, z;
    cell_xyz(G, c, x, y, z);
    int k = 0;
    for (int q = 1; q < Q; ++q) {
        int n = nbr_idx(G, x, y, z, q, 1);
        if (n >= 0 && D.flags[n] == IFC) ++k;
    }
    if (k == 0) {
        unsafeAtomicAdd(D.ledger, ex);
        return;
    }
    double part = ex / k;
    for (int q = 1; q < Q; ++q) {
        int n = nbr_idx(G, x, y, z, q, 1);
        if (n >= 0 && D.flags[n] == IFC) unsafeAtomicAdd(D.m + n, part);
    }
}

template <int ST>
__global__ void k_conv_excess(Geom G, Phys Ph, Dev D) {
    int nF = list_len(D, C_NF), nE = list_len(D, C_NE);
    GRID_STRIDE(i, nF) {
        int c = D.lF[i];
        double ex = D.m[c] - cell_rho<ST>(G, D, Ph, D.fB, c);
        D.m[c] = 0.0;
        share_excess<ST>(G, D, c, ex);
    }
    GRID_STRIDE(i, nE) {
        int c = D.lE[i];
        double ex = D.m[c];
        D.m[c] = 0.0;
        share_excess<ST>(G, D, c, ex);
    }
}

// root of a bubble id through the merge table; ids outside the table map to 0
__device__ __forceinline__ int bubble_root(const Dev &D, int b) {
    for (int it = 0; it < 64; ++it) {
        if (b < 0 || b >= D.maxB) return 0;
        int r = D.broot[b];
        if (r == b) return b;
        b = r;
    }
    return b < 0 || b >= D.maxB ? 0 : b;
}

template <int ST>
__global__ void k_conv_fill(Geom G, Phys Ph, Dev D) {
    int nF = list_len(D, C_NF), nE = list_len(D, C_NE);
    int nE0 = list_len(D, C_NE0), nG = list_len(D, C_NNG), nL = list_len(D, C_NNL);
    GRID_STRIDE(i, nF + nE) {
        const bool filled = i < nF;
        int c = filled ? D.lF[i] : D.lE[i - nF], x, y, z;
        cell_xyz(G, c, x, y, z);
        D.phi_nxt[c] = filled ? 1.0 : 0.0;
        for (int q = 1; q < Q; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n < 0) continue;
            uint8_t f = D.flags[n];
            if (f == IFC) {
                D.phi_nxt[n] = D.m[n] / cell_rho<ST>(G, D, Ph, D.fB, n);
            } else if (filled && f == GAS) {
                atomicOr(D.err, ERR_LG);
            } else if (!filled && f == LIQ) {
                atomicOr(D.err, ERR_LG);
            } else if (!filled && f == GAS) {
                int a = bubble_root(D, D.bub[c]), b = bubble_root(D, D.bub[n]);
                if (a != b) {
                    int s = atomicAdd(D.counters + C_NMERGE, 1);
                    if (s < D.cap) D.merges[s] = make_int2(a, b);
                    else atomicOr(D.err, ERR_CAP);
                }
            }
        }
    }
    GRID_STRIDE(i, nF) D.cv[D.lF[i]] = 0;
    // emptied cells are new gas: marked for the splitting test
    GRID_STRIDE(i, nE0) D.cv[D.lE0[i]] = (D.cv[D.lE0[i]] & CV_E) ? CV_GAD : 0;
    GRID_STRIDE(i, nG) D.cv[D.lNG[i]] = CV_GRM;  // left the gas: for the splitting test
    GRID_STRIDE(i, nL) D.cv[D.lNL[i]] = 0;
}

// serial union of merged bubbles: the lower root id survives, gas masses add
__global__ void k_bubble_merge(Dev D) {
    if (blockIdx.x || threadIdx.x) return;
    int n = list_len(D, C_NMERGE);
    for (int i = 0; i < n; ++i) {
        int a = bubble_root(D, D.merges[i].x), b = bubble_root(D, D.merges[i].y);
        if (a == b) continue;
        int lo = a < b ? a : b, hi = a < b ? b : a;
        D.broot[hi] = lo;
        D.btab[lo * B_STRIDE + B_M] += D.btab[hi * B_STRIDE + B_M];
        D.balive[hi] = 0;
        D.counters[C_MERGED] = 1;
    }
}

// after a merge every gas and interface cell carries its root id, so that the merged
// ids hold no cells and a split can take them again
__global__ void k_bubble_relabel(Geom G, Dev D) {
    if (D.counters[C_MERGED] == 0) return;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        const uint8_t f = D.flags[c];
        if (f == GAS || f == IFC) D.bub[c] = (uint16_t)bubble_root(D, D.bub[c]);
    }
}

// ---- bubble volumes: dense pass over the cell types ------------------------------
// gate: null, or a flag that must read 2 (a bubble split) for the kernel to run
__global__ void k_bubble_zero(Dev D, const int *gate) {
    if (gate && *gate != 2) return;
    GRID_STRIDE(i, D.nb * BACC_STRIDE) D.bacc[i] = 0.0;
}

// V_b = #gas cells + sum over interface cells of (1 - phi), with centroid moments;
// per-block LDS accumulation (FP64), one global atomic per block and component
__global__ __launch_bounds__(256) void k_bubble_accum(Geom G, Dev D, const double *phi, const int *gate) {
    if (gate && *gate != 2) return;
    __shared__ double acc[64 * BACC_STRIDE];
    __shared__ int root[64];
    const int nb = D.nb;
    for (int i = threadIdx.x; i < nb * BACC_STRIDE; i += blockDim.x) acc[i] = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) root[i] = bubble_root(D, i);
    __syncthreads();
    const long long N = G.N;
    const long long nchunk = (N + 15) / 16;
    // the thread's sums for the bubble of the cells it is walking; they go to the
    // block's table only when the bubble changes (the cells of one region mostly
    // belong to one bubble)
    int bc = -1;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0;
    auto flush = [&]() {
        if (bc >= 0) {
            double *a = acc + bc * BACC_STRIDE;
            atomicAdd(a + 0, a0);
            atomicAdd(a + 1, a1);
            atomicAdd(a + 2, a2);
            atomicAdd(a + 3, a3);
            atomicAdd(a + 4, a4);
            atomicAdd(a + 5, a5);
        }
        a0 = a1 = a2 = a3 = a4 = a5 = 0.0;
    };
    for (long long ch = blockIdx.x * (long long)blockDim.x + threadIdx.x; ch < nchunk;
         ch += (long long)gridDim.x * blockDim.x) {
        long long c0 = ch * 16;
        uint4 f4 = *(const uint4 *)(D.flags + c0);
        uint32_t wds[4] = {f4.x, f4.y, f4.z, f4.w};
        bool any = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t v = wds[k];
            // a byte is GAS (0) or IFC (2): test each byte
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                uint32_t f = (v >> (8 * bb)) & 0xffu;
                any |= (f == GAS || f == IFC) && (c0 + 4 * k + bb < N);
            }
        }
        if (!any) continue;
        for (int k = 0; k < 16; ++k) {
            const int c = (int)(c0 + k);
            if (c >= N) break;
            uint32_t f = (wds[k >> 2] >> (8 * (k & 3))) & 0xffu;
            if (f != GAS && f != IFC) continue;
            int id = D.bub[c];
            int b = id < nb ? root[id] : 0;
            if (b != bc) {
                flush();
                bc = b;
            }
            double w = (f == GAS) ? 1.0 : 1.0 - phi[c];
            const int x = c % G.nx, yz = c / G.nx, y = yz % G.ny, z = yz / G.ny;
            a0 += w;
            a1 += w * x;
            a2 += w * y;
            a3 += w * z;
            if (f == GAS) a4 += 1.0;
            else a5 += 1.0;
        }
    }
    flush();
    __syncthreads();
    for (int i = threadIdx.x; i < nb * BACC_STRIDE; i += blockDim.x)
        if (acc[i] != 0.0) unsafeAtomicAdd(D.bacc + i, acc[i]);
}

// rho_g = M / V for every root bubble; per-id FP32 mirror for the boundary condition
// with init set, the gas densities of the initial state are read from the
// table's density slot and the constant gas masses M = rho_g V(0) are fixed
// open: bubble 0 is a pressure outlet, held at the density in its table slot (the
// initial rho_g0) with its mass following its volume
__global__ void k_bubble_finalize(Dev D, int init, const int *gate, int open) {
    if (blockIdx.x || (gate && *gate != 2)) return;
    for (int b = threadIdx.x; b < D.nb; b += blockDim.x) {
        double *t = D.btab + b * B_STRIDE;
        const double *a = D.bacc + b * BACC_STRIDE;
        if (init) {
            t[B_M] = t[B_RHO] * a[0];
            t[B_V0] = a[0];
            D.balive[b] = a[0] > 0.0;
            D.broot[b] = b;
        }
        if (D.broot[b] != b) continue;
        t[B_V] = a[0];
        t[B_NGAS] = a[4];
        t[B_NIF] = a[5];
        if (!D.balive[b]) continue;
        const bool outlet = b == 0 && open;
        if (outlet) t[B_M] = t[B_RHO] * a[0];
        if (a[0] > 0.0) {
            if (!outlet) t[B_RHO] = t[B_M] / a[0];
            t[B_C] = a[1] / a[0];
            t[B_C + 1] = a[2] / a[0];
            t[B_C + 2] = a[3] / a[0];
        } else if (t[B_M] > 0.0) {
            // a bubble whose gas volume has vanished no longer exists; its gas mass
            // leaves (the liquid mass ledger is not involved)
            D.balive[b] = 0;
            t[B_M] = 0.0;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < D.nb; b += blockDim.x)
        D.rhog[b] = (float)D.btab[bubble_root(D, b) * B_STRIDE + B_RHO];
}


// ---- surface tension: interface curvature (end of Sec. 2.2) ----------------------
// The fill level as the curvature sees it: liquid and particle nodes 1 (perfect
// wetting), gas 0, interface cells their fill level; a position beyond a wall takes
// the nearest cell inside the box, a periodic one wraps.
__device__ __forceinline__ int st_axis(int v, int n, int per) {
    if (per) return v < 0 ? v + n : (v >= n ? v - n : v);
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}
__device__ __forceinline__ double st_fill(const Geom &G, const Dev &D, const double *phi, int i, int j, int k) {
    i = st_axis(i, G.nx, G.per[0]);
    j = st_axis(j, G.ny, G.per[1]);
    k = st_axis(k, G.nz, G.per[2]);
    const long long c = i + (long long)G.nx * (j + (long long)G.ny * k);
    const uint8_t f = D.flags[c];
    return f == GAS ? 0.0 : (f == IFC ? phi[c] : 1.0);
}
// Parker-Youngs weighted central differences over the 3x3x3 block: a cell displaced
// along the axis of the derivative counts 4, 2 or 1 for 0, 1 or 2 nonzero
// transverse offsets (sum 16, distance 2)
__device__ __forceinline__ double st_w(int a, int b) {
    return (a == 0 && b == 0) ? 4.0 : ((a == 0 || b == 0) ? 2.0 : 1.0);
}
__device__ void st_normal(const Geom &G, const Dev &D, const double *phi, int i, int j, int k, double n[3]) {
    n[0] = n[1] = n[2] = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                const double v = st_fill(G, D, phi, i + dx, j + dy, k + dz);
                if (dx) n[0] += dx * st_w(dy, dz) * v;
                if (dy) n[1] += dy * st_w(dx, dz) * v;
                if (dz) n[2] += dz * st_w(dx, dy) * v;
            }
    n[0] *= 1.0 / 32.0;
    n[1] *= 1.0 / 32.0;
    n[2] *= 1.0 / 32.0;
}
// kappa = -(1/2) div(n/|n|) at every interface cell: the mean curvature, so that
// 2 sigma kappa is the Laplace jump (a gas bubble of radius R has kappa = -1/R).
//
// Worked in tiles of KTX x KTY cells of one plane.  A marking pass lists the tiles
// that hold interface cells; the curvature pass stages the fill levels of a listed
// tile with a two-cell halo in LDS, forms the gradient of every cell of the tile
// and a one-cell halo once, and takes the divergence at the tile's interface cells
// (in the order of the per-cell definition, so the result is the same).
constexpr int KTX = 32, KTY = 8;
constexpr int KFX = KTX + 4, KFY = KTY + 4, KFZ = 5;  // staged fill levels
constexpr int KNX = KTX + 2, KNY = KTY + 2, KNZ = 3;  // gradients and their norms

// every tile with an interface cell enters the list once (tflag is zero for all
// tiles on entry; the curvature pass clears the flags of the tiles it takes)
__global__ __launch_bounds__(256) void k_curv_mark(Geom G, Dev D, unsigned *tflag, int *tlist, int *count,
                                                   int ktx, int kty) {
    const long long N = G.N;
    const long long nchunk = (N + 15) / 16;
    for (long long ch = blockIdx.x * (long long)blockDim.x + threadIdx.x; ch < nchunk;
         ch += (long long)gridDim.x * blockDim.x) {
        const long long c0 = ch * 16;
        const uint4 f4 = *(const uint4 *)(D.flags + c0);
        const uint32_t wds[4] = {f4.x, f4.y, f4.z, f4.w};
        int last = -1;
        for (int e = 0; e < 16; ++e) {
            const long long c = c0 + e;
            if (c >= N) break;
            if (((wds[e >> 2] >> (8 * (e & 3))) & 0xffu) != IFC) continue;
            const int i = (int)(c % G.nx), j = (int)((c / G.nx) % G.ny), k = (int)(c / ((long long)G.nx * G.ny));
            const int t = (k * kty + j / KTY) * ktx + i / KTX;
            if (t == last) continue;
            last = t;
            if (atomicExch(tflag + t, 1u) == 0u) tlist[atomicAdd(count, 1)] = t;
        }
    }
}

// a staged coordinate: wrapped on a periodic axis (the halo may reach past the box
// more than once in a short axis), the nearest cell inside beyond a wall
__device__ __forceinline__ int kc_wrap(int v, int n, int per) {
    if (per) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// LDS index of the point whose gradient stands for position v of the one-cell halo:
// beyond a wall the nearest cell inside (the per-cell definition clamps the
// position first); on a periodic axis v itself, since the staged fill levels are
// already wrapped
__device__ __forceinline__ int kc_pos(int v, int n, int per, int origin) {
    if (!per) v = v < 0 ? 0 : (v >= n ? n - 1 : v);
    return v - origin;
}

__global__ __launch_bounds__(256) void k_curv_tiles(Geom G, Dev D, const double *phi, unsigned *tflag,
                                                    const int *tlist, const int *count, int ktx, int kty) {
    __shared__ double F[KFZ][KFY][KFX];
    __shared__ double NG[4][KNZ][KNY][KNX];  // gradient components and norm
    const int nt = *count;
    for (int it = blockIdx.x; it < nt; it += gridDim.x) {
        const int t = tlist[it];
        const int x0 = (t % ktx) * KTX, y0 = ((t / ktx) % kty) * KTY, z = t / (ktx * kty);
        for (int e = threadIdx.x; e < KFX * KFY * KFZ; e += blockDim.x) {
            const int ex = e % KFX, ey = (e / KFX) % KFY, ez = e / (KFX * KFY);
            F[ez][ey][ex] = st_fill(G, D, phi, kc_wrap(x0 - 2 + ex, G.nx, G.per[0]),
                                    kc_wrap(y0 - 2 + ey, G.ny, G.per[1]), kc_wrap(z - 2 + ez, G.nz, G.per[2]));
        }
        __syncthreads();
        for (int e = threadIdx.x; e < KNX * KNY * KNZ; e += blockDim.x) {
            const int ex = e % KNX, ey = (e / KNX) % KNY, ez = e / (KNX * KNY);
            const int px = kc_pos(x0 - 1 + ex, G.nx, G.per[0], x0 - 2);
            const int py = kc_pos(y0 - 1 + ey, G.ny, G.per[1], y0 - 2);
            const int pz = kc_pos(z - 1 + ez, G.nz, G.per[2], z - 2);
            double n0 = 0.0, n1 = 0.0, n2 = 0.0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        const double v = F[pz + dz][py + dy][px + dx];
                        if (dx) n0 += dx * st_w(dy, dz) * v;
                        if (dy) n1 += dy * st_w(dx, dz) * v;
                        if (dz) n2 += dz * st_w(dx, dy) * v;
                    }
            n0 *= 1.0 / 32.0;
            n1 *= 1.0 / 32.0;
            n2 *= 1.0 / 32.0;
            NG[0][ez][ey][ex] = n0;
            NG[1][ez][ey][ex] = n1;
            NG[2][ez][ey][ex] = n2;
            NG[3][ez][ey][ex] = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < KTX * KTY; e += blockDim.x) {
            const int lx = e % KTX, ly = e / KTX;
            const int x = x0 + lx, y = y0 + ly;
            if (x >= G.nx || y >= G.ny) continue;
            const long long c = x + (long long)G.nx * (y + (long long)G.ny * z);
            if (D.flags[c] != IFC) continue;
            double div = 0.0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        const int a = 1 + lx + dx, b = 1 + ly + dy, d = 1 + dz;
                        const double nn = NG[3][d][b][a];
                        if (nn == 0.0) continue;
                        if (dx) div += dx * st_w(dy, dz) * NG[0][d][b][a] / nn;
                        if (dy) div += dy * st_w(dx, dz) * NG[1][d][b][a] / nn;
                        if (dz) div += dz * st_w(dx, dy) * NG[2][d][b][a] / nn;
                    }
            D.kappa[c] = (float)(-0.5 * div / 32.0);
        }
        if (threadIdx.x == 0) tflag[t] = 0u;
        __syncthreads();
    }
}

}  // namespace fsl
