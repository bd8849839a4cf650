// The D3Q19 pull with no arithmetic (declared in include/fsl_ceiling.h): the bandwidth
// ceiling of the stream-collide kernel's access shape.
#include <hip/hip_runtime.h>

#include "../../include/fsl_ceiling.h"
#include "fsl_device.hpp"

namespace {

// one 64 x 4 tile of a plane per block, rows of 64 consecutive cells per wave; the
// tiles of a plane run across the device's eight L2 partitions in turn
__global__ __launch_bounds__(256) void k_pull_ceiling(const float *__restrict__ A, float *__restrict__ B, int nx,
                                                      int ny, int nz, long long S, int tilesX, int tilesY) {
    const int t = blockIdx.x;
    const int x = (t % tilesX) * 64 + (threadIdx.x & 63);
    const int y = ((t / tilesX) % tilesY) * 4 + (threadIdx.x >> 6);
    const int z = t / (tilesX * tilesY);
    if (x >= nx || y >= ny) return;
    const unsigned c = (unsigned)x + (unsigned)nx * ((unsigned)y + (unsigned)ny * (unsigned)z);
    const int xm = x > 0 ? -1 : 0, xp = x < nx - 1 ? 1 : 0;
    const int ym = y > 0 ? -nx : 0, yp = y < ny - 1 ? nx : 0;
    const int zm = z > 0 ? -nx * ny : 0, zp = z < nz - 1 ? nx * ny : 0;
#pragma unroll
    for (int q = 0; q < fsl::Q; ++q) {
        // the source is the neighbour at -c_q
        const int ox = fsl::cx(q) > 0 ? xm : fsl::cx(q) < 0 ? xp : 0;
        const int oy = fsl::cy(q) > 0 ? ym : fsl::cy(q) < 0 ? yp : 0;
        const int oz = fsl::cz(q) > 0 ? zm : fsl::cz(q) < 0 ? zp : 0;
        const float v = A[q * S + (unsigned)((int)c + ox + oy + oz)];
        __builtin_nontemporal_store(v, B + q * S + c);
    }
}

}  // namespace

extern "C" int fsl_ceiling_pull(const float *A, float *B, int nx, int ny, int nz, long long S, void *hip_stream) {
    if (!A || !B || nx < 1 || ny < 1 || nz < 1 || S < (long long)nx * ny * nz || (long long)nx * ny * nz >= (1LL << 31))
        return -1;
    const int tilesX = (nx + 63) / 64, tilesY = (ny + 3) / 4;
    const long long blocks = (long long)tilesX * tilesY * nz;
    if (blocks >= (1LL << 31)) return -1;
    hipLaunchKernelGGL(k_pull_ceiling, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, A, B, nx, ny, nz,
                       S, tilesX, tilesY);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
