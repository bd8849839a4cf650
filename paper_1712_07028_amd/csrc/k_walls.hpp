// Force of the fluid on each no-slip face of the box over a step, the plate force of
// the sheared suspension (Sec. 3.1: mu_s = F_x / (A gamma)).  Every half-way
// bounce-back link exchanges momentum with its face as a particle link does (Eqs.
// netforce, momentum_transfer): Delta j = c_qbar (f*_qbar(x,t) + f_q(x,t+1)), in
// shifted storage -c_q (h*_qbar + h_q + 2 w_q), where h_q = h*_qbar + 6 w_q rho_t
// (c_q . u_w) (Eq. bbrule) with rho_t the cell's density at t from its own
// populations, as the stream-collide step takes it.  The kernel reads lattice A (the
// state at t) and the cell types at t, so it runs before the stream-collide launch.
#pragma once

#include "k_free_surface.hpp"

namespace fsl {

// the face layers to walk: layer f is (axis, side); a cell that lies on the layer of
// a lower axis in the list is left to that layer, so that each cell counts once
struct FaceSet {
    int n;
    int axis[6], side[6];
    long long start[7];  // prefix sums of the layer areas
};

template <int ST>
__global__ __launch_bounds__(256) void k_wall_forces(Geom G, Phys Ph, Dev D, FaceSet FS) {
    using SS = Store<ST>;
    const typename SS::T *A = (const typename SS::T *)D.fA;
    __shared__ double acc[18];
    if (threadIdx.x < 18) acc[threadIdx.x] = 0.0;
    __syncthreads();
    const int nn[3] = {G.nx, G.ny, G.nz};
    const long long total = FS.start[FS.n];
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += gridDim.x * 256LL) {
        int f = 0;
        while (f + 1 < FS.n && e >= FS.start[f + 1]) ++f;
        const int a = FS.axis[f];
        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;  // the other two axes
        const long long r = e - FS.start[f];
        int p[3];
        p[a] = FS.side[f] ? nn[a] - 1 : 0;
        p[b] = (int)(r % nn[b]);
        p[d] = (int)(r / nn[b]);
        bool dup = FS.side[f] && nn[a] == 1;  // one layer is both faces
        for (int k = 0; k < f; ++k) {
            const int ak = FS.axis[k];
            if (ak != a && p[ak] == (FS.side[k] ? nn[ak] - 1 : 0)) dup = true;
        }
        if (dup) continue;
        const int c = p[0] + G.nx * (p[1] + G.ny * p[2]);
        const uint8_t fl = D.flags[c];
        if (fl != LIQ && fl != IFC) continue;
        float h[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) h[q] = SS::ld(A + q * G.S + c, Ph.inv);
        const float rho_t = 1.0f + (float)cell_moments(h).drho;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const int s[3] = {p[0] - cx(q), p[1] - cy(q), p[2] - cz(q)};
            int fa = -1;
            bool crossed = false;
            for (int k = 0; k < 3; ++k) {
                if (G.per[k] || (s[k] >= 0 && s[k] < nn[k])) continue;
                crossed = true;
                if (fa < 0 && !Ph.slip[k]) fa = k;
            }
            if (!crossed || fa < 0) continue;  // no face, or free-slip faces only
            const int sd = s[fa] < 0 ? 0 : 1;
            const float *uw = D.wallu + (fa * 2 + sd) * 3;
            const float hb = h[opp(q)];
            const float hq = hb + 6.0f * wq(q) * rho_t * (cx(q) * uw[0] + cy(q) * uw[1] + cz(q) * uw[2]);
            const double m = (double)hb + (double)hq + 2.0 * wqd(q);
            double *dst = acc + 3 * (2 * fa + sd);
            if (cx(q)) atomicAdd(dst + 0, -cx(q) * m);
            if (cy(q)) atomicAdd(dst + 1, -cy(q) * m);
            if (cz(q)) atomicAdd(dst + 2, -cz(q) * m);
        }
    }
    __syncthreads();
    if (threadIdx.x < 18 && acc[threadIdx.x] != 0.0) unsafeAtomicAdd(D.wallF + threadIdx.x, acc[threadIdx.x]);
}

}  // namespace fsl
