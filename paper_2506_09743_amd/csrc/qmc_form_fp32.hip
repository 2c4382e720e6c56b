// Instantiates the mixed form with FP32 AOs and the FP32 vector-unit MO
// contraction (QMC_MIXED_FP32).

#include "qmc_kernels.h"

namespace qmc {

hipError_t launch_form_fp32(QMC_LAUNCH_ARGS) {
    QMC_NMO_SWITCH(return (launch_t<N, float, 0>(QMC_LAUNCH_PASS)))
}

}  // namespace qmc
