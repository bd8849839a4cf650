/*
 * fsl_ceiling.h -- a measurement kernel, not part of the method: the D3Q19 pull of a
 * two-lattice SoA FP32 layout with no arithmetic (every cell reads its 19
 * populations from the 19 planes at its neighbours and writes them to the 19 planes
 * of the other lattice at itself: 76 B read and 76 B written per cell).  Its
 * bandwidth is the ceiling that the stream-collide kernel's access shape allows on
 * the device, beside a plain copy.
 */
#ifndef FSL_CEILING_H
#define FSL_CEILING_H

#ifdef __cplusplus
extern "C" {
#endif

/* A, B: device arrays of 19 * S floats (plane q at q * S, cell x + nx (y + ny z));
 * S >= nx * ny * nz; the box is closed (a neighbour beyond a face is taken at the
 * face).  Enqueues one pass A -> B on hip_stream (a hipStream_t, may be 0);
 * returns 0, or -1 on bad arguments (nothing enqueued), -2 on a launch error. */
int fsl_ceiling_pull(const float *A, float *B, int nx, int ny, int nz, long long S, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
