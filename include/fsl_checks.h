/*
 * fsl_checks.h -- host entry points of libfsl_checks.so: two pure functions of the
 * library's kernels, compiled for the host from the same source, so that tests can
 * check them against exact definitions on many random inputs without a GPU.
 * Neither allocates, touches a device or keeps state; both are thread-safe.
 */
#ifndef FSL_CHECKS_H
#define FSL_CHECKS_H

#ifdef __cplusplus
extern "C" {
#endif

/* Local bubble-splitting test (bubble model, end of Sec. 2.2: a bubble is a
 * connected gas region, D3Q19 neighbours connected) on the 3x3x3 block around a
 * cell that left the gas.  gas: the block's cells still gas of the cell's root
 * bubble, rem: the block's cells of that root that also left the gas in the step,
 * both as 27-bit sets, bit (dx+1) + 3(dy+1) + 9(dz+1) (bit 13, the centre, is
 * ignored).  Returns 1 when the root's gas stays connected for certain, 0 when a
 * global labelling must decide. */
int fsl_check_split_block(unsigned gas, unsigned rem);

/* Candidate nodes of one (x, y) column for the coverage update of a sphere that
 * moved (Sec. 2.3: nodes inside a sphere are covered).  sn, so: squared in-plane
 * distances of the column from the new and old centres ((i-x)^2 + (j-y)^2, each
 * product and the sum rounded to nearest); R2 = R * R; zn, zo: the centres' z;
 * [klo, khi]: the column's node range in the box.  r (4 ints, caller-owned)
 * receives the ranges [r[0], r[1]] and [r[2], r[3]] (empty when first > last):
 * every node k of the column with (sn + (k-zn)^2 <= R2) != (so + (k-zo)^2 <= R2)
 * lies in one of them. */
void fsl_check_cov_column(double sn, double so, double R2, double zn, double zo, int klo, int khi, int r[4]);

#ifdef __cplusplus
}
#endif
#endif
