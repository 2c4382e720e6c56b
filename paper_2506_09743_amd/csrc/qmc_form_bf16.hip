// Instantiates the mixed forms with the MO contraction on the BF16 matrix
// cores: split operands (QMC_MIXED_BF16, split = 3) here, one product
// (QMC_MIXED_BF16_X1, split = 1) in qmc_form_bf16_x1.hip, so the two
// compile in parallel.

#include "qmc_kernels.h"

namespace qmc {

hipError_t launch_form_bf16_x1(QMC_LAUNCH_ARGS);

hipError_t launch_form_bf16(QMC_LAUNCH_ARGS, int split) {
    if (split != 3) return launch_form_bf16_x1(QMC_LAUNCH_PASS);
    QMC_NMO_SWITCH(return (launch_t<N, float, 3>(QMC_LAUNCH_PASS)))
}

}  // namespace qmc
