// Launch dispatch of libqmc's walker kernels: picks the instantiation of
// the call's arithmetic form (the kernels live in qmc_kernels.h and are
// instantiated by the qmc_form_*.hip units).

#include "qmc_walker.h"

namespace qmc {

hipError_t launch_form_fp64(bool, const DevSystem &, double *, double *, double *, double *, int64_t, int,
                            double, uint64_t, uint64_t, uint32_t, double *, const CallStreams &);
hipError_t launch_form_fp32(bool, const DevSystem &, double *, double *, double *, double *, int64_t, int,
                            double, uint64_t, uint64_t, uint32_t, double *, const CallStreams &);
hipError_t launch_form_bf16(bool, const DevSystem &, double *, double *, double *, double *, int64_t, int,
                            double, uint64_t, uint64_t, uint32_t, double *, const CallStreams &, int);
hipError_t launch_form_explicit(bool, const DevSystem &, double *, double *, double *, double *, int64_t, int,
                                double, uint64_t, uint64_t, uint32_t, double *, const CallStreams &);
hipError_t launch_form_backflow(bool, const DevSystem &, double *, double *, double *, double *, int64_t, int,
                                double, uint64_t, uint64_t, uint32_t, double *, const CallStreams &, bool);

// Sums of the [W][4] accumulators over walkers in an order fixed by W:
// thread t of the one work-group adds rows t, t + T, t + 2T, ... in turn,
// then the T partial sums meet in a binary tree (T = kReduceThreads).
constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void k_reduce_acc(const double *__restrict__ acc, int64_t W,
                                                               double *__restrict__ out) {
    __shared__ double part[5][kReduceThreads];
    const int t = threadIdx.x;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t w = t; w < W; w += kReduceThreads) {
        const double *a = acc + 4 * w;
        s[0] += a[0];
        s[1] += a[1];
        s[2] += a[2];
        s[3] += a[3];
        s[4] += a[3] != 0.0 ? 1.0 : 0.0;
    }
    for (int k = 0; k < 5; ++k) part[k][t] = s[k];
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int k = 0; k < 5; ++k) part[k][t] += part[k][t + h];
        __syncthreads();
    }
    if (t < 5) out[t] = part[t][0];
}

hipError_t launch_reduce_acc(const double *acc, int64_t W, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_acc, dim3(1), dim3(kReduceThreads), 0, st, acc, W, out);
    return hipGetLastError();
}

static int nmo_bucket(int n_mo) {
    const int b[] = {4, 8, 12, 16, 20, 24, 32};
    for (int v : b)
        if (n_mo <= v) return v;
    return -1;
}

int padded_mo(int n_mo) { return nmo_bucket(n_mo); }

size_t explicit_lds_bytes(const DevSystem &S) {
    int per = 0;
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: per = walker::walker_lds_explicit<N>(S); break;
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return (size_t)S.WPW * per * sizeof(double);
}

// form: 0 FP64, 1 mixed FP32 (VALU), 2 mixed BF16 on the matrix cores with
// split operands, 3 mixed BF16 single products, 4 FP64 with explicit
// determinants, 5 FP64 with backflow and every configuration factorised,
// 6 FP64 with backflow and the low-rank configuration update.
hipError_t launch_walkers(bool mc, int form, const DevSystem &S, double *X, double *LP, double *SG,
                          double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                          uint64_t step0, uint32_t woff, double *ACC, const CallStreams &st) {
    switch (form) {
        case 0: return launch_form_fp64(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 1: return launch_form_fp32(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 2: return launch_form_bf16(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st, 3);
        case 3: return launch_form_bf16(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st, 1);
        case 4: return launch_form_explicit(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 5: return launch_form_backflow(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st, false);
        case 6: return launch_form_backflow(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st, true);
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
