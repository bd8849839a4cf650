// k_init.hpp -- initial state and host-exchange kernels.
//
// Initial state of a flat pool with spherical gas bubbles (Sec. 2.2 cell types and
// fill levels; the liquid at hydrostatic equilibrium):
//   fill level = fraction of the 8^3 sub-points at offsets (a + 1/2)/8 - 1/2 that lie
//   below the pool height and outside every gas sphere (strict comparisons), so
//   phi = k/512 exactly; phi = 1 liquid, phi = 0 gas, else interface; liquid cells
//   with a gas neighbour become interface (closure); a gas sub-point belongs to
//   bubble 0 above the pool, else to 1 + the first sphere holding it, and a cell
//   takes the lowest id among its gas sub-points; the liquid density is
//   rho_g0 (1 - 3 g_z (zs - z)) (1 for a fully liquid box), u = 0, f = equilibrium,
//   interface mass m = phi rho.
#pragma once

#include "k_free_surface.hpp"

namespace fsl {

struct InitGeo {
    double zs, rho_g0, gz;
    int ns;
    double sph[16][5];
};

__global__ void k_init_geometry(Geom G, Dev D, InitGeo I) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i = (int)(c % G.nx), j = (int)((c / G.nx) % G.ny), k = (int)(c / ((long long)G.nx * G.ny));
        const bool full = I.zs < 0.0;
        int nliq = 0, gid = 1 << 30;
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
                for (int d = 0; d < 8; ++d) {
                    double p0 = i + (2 * a - 7) / 16.0, p1 = j + (2 * b - 7) / 16.0, p2 = k + (2 * d - 7) / 16.0;
                    int id = (full || p2 < I.zs) ? -1 : 0;
                    for (int s = 0; s < I.ns && id < 0; ++s) {
                        double d0 = p0 - I.sph[s][0], d1 = p1 - I.sph[s][1], d2 = p2 - I.sph[s][2];
                        if (__dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2)) <
                            __dmul_rn(I.sph[s][3], I.sph[s][3]))
                            id = s + 1;
                    }
                    if (id < 0) ++nliq;
                    else if (id < gid) gid = id;
                }
        D.phi_cur[c] = nliq / 512.0;
        D.flags[c] = nliq == 512 ? LIQ : (nliq == 0 ? GAS : IFC);
        D.bub[c] = (uint16_t)(nliq == 512 ? 0 : gid);
        D.cv[c] = 0;
        D.pid[c] = -1;
        D.claim[c] = 0x7fffffff;
        D.m[c] = 0.0;
    }
}

__global__ void k_init_closure_mark(Geom G, Dev D) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        if (D.flags[c] != LIQ) continue;
        int x, y, z;
        cell_xyz(G, (int)c, x, y, z);
        for (int q = 1; q < Q; ++q) {
            int n = nbr_idx(G, x, y, z, q, 1);
            if (n >= 0 && D.flags[n] == GAS) {
                D.cv[c] = 1;
                D.bub[c] = D.bub[n];
                break;
            }
        }
    }
}

template <int ST>
__global__ void k_init_pdf(Geom G, Phys Ph, Dev D, InitGeo I) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        if (D.cv[c]) {
            D.flags[c] = IFC;
            D.cv[c] = 0;
        }
        uint8_t f = D.flags[c];
        if (f != LIQ && f != IFC) continue;
        int k = (int)(c / ((long long)G.nx * G.ny));
        double rho = I.zs < 0.0 ? 1.0 : I.rho_g0 * (1.0 - 3.0 * I.gz * (I.zs - k));
        store_equilibrium<ST>(G, Ph, D.fA, (int)c, rho - 1.0, 0.f, 0.f, 0.f);
        if (f == IFC) D.m[c] = D.phi_cur[c] * rho;
        else D.phi_cur[c] = 1.0;
    }
}

__global__ void k_fill_i32(int *p, long long n, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *p, long long n, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---- host exchange of populations (unshifted FP64 on the host side) ---------------
template <int ST>
__global__ void k_pop_to_f64(Geom G, Phys Ph, const void *F, int q, long long c0, long long n, double *out) {
    using SS = Store<ST>;
    const typename SS::T *p = (const typename SS::T *)F + q * G.S + c0;
    const double w = wqd(q);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = (double)SS::ld(p + i, Ph.inv) + w;
}

template <int ST>
__global__ void k_pop_from_f64(Geom G, Phys Ph, void *F, int q, long long c0, long long n, const double *in) {
    using SS = Store<ST>;
    typename SS::T *p = (typename SS::T *)F + q * G.S + c0;
    const double w = wqd(q);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        SS::st(p + i, (float)(in[i] - w), Ph.scale);
}

__global__ void k_u16_to_i32(const uint16_t *a, long long n, int *out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = a[i];
}

__global__ void k_i32_to_u16(const int *a, long long n, uint16_t *out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = (uint16_t)a[i];
}

// total mass: number of liquid cells + sum of their shifted populations + interface m
template <int ST>
__global__ __launch_bounds__(256) void k_mass(Geom G, Phys Ph, Dev D, double *out) {
    using SS = Store<ST>;
    __shared__ double red[2][256];
    const typename SS::T *p = (const typename SS::T *)D.fA;
    double s = 0.0, nl = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.N;
         c += (long long)gridDim.x * blockDim.x) {
        uint8_t f = D.flags[c];
        if (f == LIQ) {
            nl += 1.0;
            for (int q = 0; q < Q; ++q) s += (double)SS::ld(p + q * G.S + c, Ph.inv);
        } else if (f == IFC) {
            s += D.m[c];
        }
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = nl;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(out, red[0][0]);
        unsafeAtomicAdd(out + 1, red[1][0]);
    }
}

__global__ void k_zero_counters(Dev D) {
    if (threadIdx.x < C_COUNT && blockIdx.x == 0) D.counters[threadIdx.x] = 0;
}

__global__ void k_f32_to_f64(const float *in, long long n, double *out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}

}  // namespace fsl
