// Host builds of two pure functions of the kernels (declared in include/fsl_checks.h).
#include "../../include/fsl_checks.h"
#include "cov_column.hpp"
#include "split_block.hpp"

extern "C" {

int fsl_check_split_block(unsigned gas, unsigned rem) { return fsl::split_block_ok(gas, rem) ? 1 : 0; }

void fsl_check_cov_column(double sn, double so, double R2, double zn, double zo, int klo, int khi, int r[4]) {
    fsl::cov_column_ranges(sn, so, R2, zn, zo, klo, khi, r);
}

}  // extern "C"
