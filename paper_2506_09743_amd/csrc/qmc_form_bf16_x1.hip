// Instantiates the mixed form with one BF16 matrix-core product per
// operand pair in the MO contraction (QMC_MIXED_BF16_X1).

#include "qmc_kernels.h"

namespace qmc {

hipError_t launch_form_bf16_x1(QMC_LAUNCH_ARGS) {
    QMC_NMO_SWITCH(return (launch_t<N, float, 1>(QMC_LAUNCH_PASS)))
}

}  // namespace qmc
