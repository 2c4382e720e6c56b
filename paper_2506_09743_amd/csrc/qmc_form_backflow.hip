// Instantiates the inverse-backflow forms for expansions of up to
// kSmallCfgBF configurations per spin: the low-rank configuration update
// (QMC_FP64 with backflow) and every configuration factorised
// (QMC_FP64_EXPLICIT with backflow).

#include "qmc_kernels.h"

namespace qmc {

hipError_t launch_form_backflow_max(QMC_LAUNCH_ARGS, bool low_rank);

hipError_t launch_form_backflow(QMC_LAUNCH_ARGS, bool low_rank) {
    // BF = 1: per-lane tables for up to kSmallCfgBF configurations per spin;
    // larger expansions take the kMaxCfgBF kernels (qmc_form_backflow_max.hip)
    if (S.n_cfg_max > kSmallCfgBF) return launch_form_backflow_max(QMC_LAUNCH_PASS, low_rank);
    if (low_rank) {
        QMC_NMO_SWITCH(return (launch_t<N, double, 0, false, 1>(QMC_LAUNCH_PASS)))
    }
    QMC_NMO_SWITCH(return (launch_t<N, double, 0, true, 1>(QMC_LAUNCH_PASS)))
}

size_t backflow_lds_bytes(const DevSystem &S, bool low_rank) {
    int per = 0;
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: per = low_rank ? walker_lds_bf<N, true>(S) : walker_lds_bf<N, false>(S); break;
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return (size_t)S.WPW * per * sizeof(double);
}

}  // namespace qmc
