// k_adjoint.hpp -- differentiation form (frozen-flag window); not built yet.
#pragma once

#include "fsl_device.hpp"

namespace fsl {

struct AdjointState {
    char *base;
    size_t bytes;
};

inline size_t adjoint_window_bytes(int T, int k, size_t S, int maxP) {
    (void)T; (void)k; (void)S; (void)maxP;
    return 0;
}

inline void adjoint_bind(AdjointState &A, char *base, size_t bytes) {
    A.base = base;
    A.bytes = bytes;
}

template <int ST>
int adjoint_forward(AdjointState &, const Geom &, const Phys &, const Dev &, hipStream_t, int, int, double *,
                    char *err) {
    snprintf(err, 256, "differentiation window not available");
    return FSL_E_ARG;
}

template <int ST>
int adjoint_backward(AdjointState &, const Geom &, const Phys &, const Dev &, hipStream_t, const fsl_config &,
                     double, double *, double *, char *err) {
    snprintf(err, 256, "differentiation window not available");
    return FSL_E_ARG;
}

}  // namespace fsl
