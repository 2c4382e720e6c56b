// Instantiates the FP64 forms: the low-rank determinants (QMC_FP64), the
// explicit per-configuration method (QMC_FP64_EXPLICIT) and the
// finite-difference kinetic energy.

#include "qmc_kernels.h"

namespace qmc {

hipError_t launch_form_fp64(QMC_LAUNCH_ARGS) {
    QMC_NMO_SWITCH(return (launch_t<N, double, 0>(QMC_LAUNCH_PASS)))
}

hipError_t launch_form_explicit(QMC_LAUNCH_ARGS) {
    QMC_NMO_SWITCH(return (launch_t<N, double, 0, true>(QMC_LAUNCH_PASS)))
}

hipError_t launch_eval_fd(const DevSystem &S, const double *X, int64_t W, double h, double *LP, double *EL,
                          hipStream_t st) {
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    QMC_NMO_SWITCH(hipLaunchKernelGGL((k_eval_fd<N>), dim3((unsigned)blocks), dim3(kWave),
                                      (size_t)S.WPW * (walker_lds<N, false>(S)) * sizeof(double), st, S, X, W, h, LP, EL);
                   return hipGetLastError())
}

}  // namespace qmc
