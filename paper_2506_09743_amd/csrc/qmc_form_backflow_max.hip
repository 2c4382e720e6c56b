// Instantiates the inverse-backflow forms for expansions of more than
// kSmallCfgBF (up to kMaxCfgBF) configurations per spin, in a unit of their
// own so the two table sizes compile in parallel.

#include "qmc_kernels.h"

namespace qmc {

hipError_t launch_form_backflow_max(QMC_LAUNCH_ARGS, bool low_rank) {
    if (low_rank) {
        QMC_NMO_SWITCH(return (launch_t<N, double, 0, false, 2>(QMC_LAUNCH_PASS)))
    }
    QMC_NMO_SWITCH(return (launch_t<N, double, 0, true, 2>(QMC_LAUNCH_PASS)))
}

}  // namespace qmc
