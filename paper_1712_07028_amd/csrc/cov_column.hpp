// Candidate nodes of one (x, y) column for the coverage update of a sphere that
// moved (Sec. 2.3: a node is covered while it lies inside the sphere).  Compiled
// for the device (the coverage scan) and for the host (the exactness check against
// the inside test at every node).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fsl {

// sn, so: the in-plane squared distances of the column from the new and old centres
// (formed as the inside test forms them), R2 = R * R, zn, zo: the centres' z, [klo,
// khi]: the node range of the column in the box.  Along the column the sphere holds
// one interval of nodes at each position, so the nodes whose inside test changes lie
// between the two lower ends or between the two upper ends.  The ends come from a
// square root: one node of margin on each side covers its rounding.  r receives two
// clipped ranges [r[0], r[1]] and [r[2], r[3]] (empty when lo > hi); only their
// nodes need the exact test.  A column outside both circles has none.
__host__ __device__ __forceinline__ void cov_column_ranges(double sn, double so, double R2, double zn, double zo,
                                                           int klo, int khi, int r[4]) {
    int r1lo, r1hi, r2lo, r2hi;
    if (sn > R2 && so > R2) {
        r1lo = r2lo = 1;
        r1hi = r2hi = 0;
    } else if (sn <= R2 && so <= R2) {
        const double hn = sqrt(R2 - sn), ho = sqrt(R2 - so);
        const int ln = (int)ceil(zn - hn), un = (int)floor(zn + hn);
        const int lo_ = (int)ceil(zo - ho), uo = (int)floor(zo + ho);
        r1lo = (ln < lo_ ? ln : lo_) - 1;
        r1hi = (ln > lo_ ? ln : lo_) + 1;
        r2lo = (un < uo ? un : uo) - 1;
        if (r2lo < r1hi + 1) r2lo = r1hi + 1;
        r2hi = (un > uo ? un : uo) + 1;
    } else {
        const double zc = sn <= R2 ? zn : zo, h = sqrt(R2 - (sn <= R2 ? sn : so));
        r1lo = (int)ceil(zc - h) - 1;
        r1hi = (int)floor(zc + h) + 1;
        r2lo = 1;
        r2hi = 0;
    }
    r[0] = r1lo > klo ? r1lo : klo;
    r[1] = r1hi < khi ? r1hi : khi;
    r[2] = r2lo > klo ? r2lo : klo;
    r[3] = r2hi < khi ? r2hi : khi;
}

}  // namespace fsl
