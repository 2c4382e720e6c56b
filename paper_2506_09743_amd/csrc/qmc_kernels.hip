// HIP kernels (gfx950): local energy evaluation and all-electron Metropolis
// blocks.  The per-walker stages live in qmc_walker.h.

#include "qmc_walker.h"

namespace qmc {
namespace {

using namespace walker;

struct WalkerResult {
    double logpsi, sign, eloc;
};

// Evaluates log|Psi|, sign and E_L of the lane's walker at the electron
// positions held by its lanes (x0, x1, x2 of the lane's electron).  Every
// lane of the block must call it (it contains block barriers); results are
// identical on all lanes of a walker.
template <int NMO, typename RT, int MF, bool EXPL, bool BF>
__device__ __forceinline__ WalkerResult eval_walker(const DevSystem &S, const Lane &L, double *wsm, double x0,
                                                    double x1, double x2, void *stage) {
    Core<NMO> c;
    core_stages<NMO, RT, MF, EXPL, BF>(S, L, wsm, x0, x1, x2, c, stage);

    // ---- pass 2: grad and Laplacian of Sigma at this electron ---------------
    double gS0, gS1, gS2, lapS;
    if constexpr (BF) {
        // the backflow stage returns them directly (the Laplacian in full
        // on electron 0's lane)
        gS0 = c.bgS0;
        gS1 = c.bgS1;
        gS2 = c.bgS2;
        lapS = c.blap;
    } else if constexpr (MF > 0) {
        ao_weights_mfma<NMO, MF>(S, L.lane, stage, c.av);
        sigma_derivs_t<float>(S, x0, x1, x2, make_stage(stage).out + L.lane * kRowF, gS0, gS1, gS2, lapS);
    } else {
        sigma_derivs<NMO, RT>(S, x0, x1, x2, c.av, gS0, gS1, gS2, lapS);
    }

    // ---- local energy and log|Psi| ------------------------------------------
    double part = 0.0;
    if (L.active) {
        const double kin = lapS + c.lapJ + c.gJ0 * c.gJ0 + c.gJ1 * c.gJ1 + c.gJ2 * c.gJ2 +
                           2.0 * (c.gJ0 * gS0 + c.gJ1 * gS1 + c.gJ2 * gS2);
        part = -0.5 * kin + c.vpot;
    }
    const double eloc = walker_sum(part, S.LW) + S.vnn;
    const double Jw = walker_sum(c.J, S.LW);
    WalkerResult res;
    if (c.sing_walker > 0 || c.Ssum == 0.0 || !L.wvalid) {
        res.logpsi = -INFINITY;
        res.sign = 0.0;
        res.eloc = NAN;
    } else {
        res.logpsi = Jw + c.logD_up + c.logD_dn + log(fabs(c.Ssum));
        res.sign = c.sgn_up * c.sgn_dn * (c.Ssum < 0.0 ? -1.0 : 1.0);
        res.eloc = eloc;
    }
    __syncthreads();  // LDS is reused by the next evaluation
    return res;
}

template <int NMO, bool EXPL, bool BF>
__device__ __forceinline__ int lds_per_walker(const DevSystem &S) {
    if constexpr (BF) return walker_lds_bf<NMO, !EXPL>(S);
    else if constexpr (EXPL) return walker_lds_explicit<NMO>(S);
    else return walker_lds<NMO>(S);
}

// The matrix-core forms ask for two waves per SIMD: left alone the compiler
// spends a few registers more than that allows and the kernel runs at one.
// The vector-unit forms are faster with the registers they choose.
template <int NMO, typename RT, int MF, bool EXPL, bool BF>
__global__ __launch_bounds__(kWave, (MF > 0 ? 2 : 1)) void k_eval(DevSystem S, const double *__restrict__ X, int64_t W,
                                                 double *__restrict__ LP, double *__restrict__ SG,
                                                 double *__restrict__ EL) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    double *wsm = smem + L.wloc * lds_per_walker<NMO, EXPL, BF>(S);
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (L.active) {
        const double *p = X + (w * S.ne + L.e) * 3;
        x0 = p[0];
        x1 = p[1];
        x2 = p[2];
    }
    const WalkerResult r = eval_walker<NMO, RT, MF, EXPL, BF>(S, L, wsm, x0, x1, x2, smem);
    if (L.wvalid && L.lw == 0) {
        LP[w] = r.logpsi;
        SG[w] = r.sign;
        EL[w] = r.eloc;
    }
}

template <int NMO, typename RT, int MF, bool EXPL, bool BF>
__global__ __launch_bounds__(kWave, (MF > 0 ? 2 : 1)) void k_metropolis(DevSystem S, double *__restrict__ X,
                                                      double *__restrict__ LP, double *__restrict__ SG,
                                                      double *__restrict__ EL, int64_t W, int n_steps,
                                                      double sigma, uint64_t seed, uint64_t step0,
                                                      uint32_t walker_offset, double *__restrict__ ACC) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    double *wsm = smem + L.wloc * lds_per_walker<NMO, EXPL, BF>(S);
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (L.active) {
        const double *p = X + (w * S.ne + L.e) * 3;
        x0 = p[0];
        x1 = p[1];
        x2 = p[2];
    }
    double lp = 0.0, sg = 0.0, el = 0.0;
    if (L.wvalid) {
        lp = LP[w];
        sg = SG[w];
        el = EL[w];
    }
    // running accumulators start from the caller's values, so a block split
    // at any step gives the same sums as one block
    double s_e = 0.0, s_e2 = 0.0, s_acc = 0.0;
    if (L.wvalid) {
        s_e = ACC[3 * w + 0];
        s_e2 = ACC[3 * w + 1];
        s_acc = ACC[3 * w + 2];
    }
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t wid = walker_offset + (uint32_t)w;
    const double s32 = 1.0 / 4294967296.0;
    const double two_pi = 6.283185307179586;
    // With backflow every launch takes one step (the host launches the
    // block step by step): without a loop around it the evaluation keeps
    // the registers it has on its own.
    const int steps = BF ? 1 : n_steps;
    for (int t = 0; t < steps; ++t) {
        const uint64_t step = step0 + (uint64_t)t;
        uint32_t c[4] = {wid, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)L.e};
        philox4x32_10(c, k0, k1);
        double z0, z1, z2;
        if constexpr (sizeof(RT) == sizeof(double)) {
            const double u0 = ((double)c[0] + 0.5) * s32, u1 = ((double)c[1] + 0.5) * s32;
            const double u2 = ((double)c[2] + 0.5) * s32, u3 = ((double)c[3] + 0.5) * s32;
            const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
            double s1, c1;
            sincos(two_pi * u1, &s1, &c1);
            z0 = r0 * c1;
            z1 = r0 * s1;
            z2 = r1 * cos(two_pi * u3);
        } else {
            // the mixed forms draw their normals in FP32 from the same
            // counters: 24-bit uniforms (w + 1/2) 2^-24, exact in FP32,
            // never 0 or 1, on a grid symmetric about 1/2
            const float f24 = 1.0f / 16777216.0f, tpf = 6.28318530717958648f;
            const float u0 = ((float)(c[0] >> 8) + 0.5f) * f24, u1 = ((float)(c[1] >> 8) + 0.5f) * f24;
            const float u2 = ((float)(c[2] >> 8) + 0.5f) * f24, u3 = ((float)(c[3] >> 8) + 0.5f) * f24;
            const float r0 = sqrtf(-2.0f * __logf(u0)), r1 = sqrtf(-2.0f * __logf(u2));
            float s1, c1;
            __sincosf(tpf * u1, &s1, &c1);
            z0 = double(r0 * c1);
            z1 = double(r0 * s1);
            z2 = double(r1 * __cosf(tpf * u3));
        }
        // no FMA contraction: X + sigma z rounds the product, then the sum
        const double y0 = __dadd_rn(x0, __dmul_rn(sigma, z0));
        const double y1 = __dadd_rn(x1, __dmul_rn(sigma, z1));
        const double y2 = __dadd_rn(x2, __dmul_rn(sigma, z2));
        uint32_t ca[4] = {wid, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)S.ne};
        philox4x32_10(ca, k0, k1);
        const uint64_t bits = ((((uint64_t)ca[0]) << 32) | (uint64_t)ca[1]) >> 11;
        const double u = (double)bits * (1.0 / 9007199254740992.0);

        const WalkerResult r = eval_walker<NMO, RT, MF, EXPL, BF>(S, L, wsm, y0, y1, y2, smem);
        const bool acc = isfinite(r.logpsi) && (u < exp(2.0 * (r.logpsi - lp)));
        if (acc) {
            x0 = y0;
            x1 = y1;
            x2 = y2;
            lp = r.logpsi;
            sg = r.sign;
            el = r.eloc;
        }
        s_e = __dadd_rn(s_e, el);
        s_e2 = __dadd_rn(s_e2, __dmul_rn(el, el));
        s_acc += acc ? 1.0 : 0.0;
    }
    if (L.active) {
        double *p = X + (w * S.ne + L.e) * 3;
        p[0] = x0;
        p[1] = x1;
        p[2] = x2;
    }
    if (L.wvalid && L.lw == 0) {
        LP[w] = lp;
        SG[w] = sg;
        EL[w] = el;
        ACC[3 * w + 0] = s_e;
        ACC[3 * w + 1] = s_e2;
        ACC[3 * w + 2] = s_acc;
    }
}

// Finite-difference kinetic energy, the baseline that the Jacobi-trace
// formulas replace: log|Psi| at x and at x +- h e_c for each of the 3 N_e
// coordinates (Psi only: no cofactor tables, no derivative passes), then
// lap Psi / Psi = sum_c (Psi(x + h e_c) - 2 Psi(x) + Psi(x - h e_c)) / (h^2 Psi(x)).
// The potential is taken at x.  FP64, low-rank determinants.
template <int NMO>
__global__ __launch_bounds__(kWave, 1) void k_eval_fd(DevSystem S, const double *__restrict__ X, int64_t W, double h,
                                                      double *__restrict__ LP, double *__restrict__ EL) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    double *wsm = smem + L.wloc * walker_lds<NMO>(S);
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (L.active) {
        const double *p = X + (w * S.ne + L.e) * 3;
        x0 = p[0];
        x1 = p[1];
        x2 = p[2];
    }
    double lp0, sg0, vpot;
    bool bad;
    {
        Core<NMO> c;
        double y0 = x0, y1 = x1, y2 = x2;
        core_stages<NMO, double, 0, false, false, true>(S, L, wsm, y0, y1, y2, c);
        vpot = walker_sum(L.active ? c.vpot : 0.0, S.LW) + S.vnn;
        lp0 = walker_sum(c.J, S.LW) + c.logD_up + c.logD_dn + log(fabs(c.Ssum));
        sg0 = c.sgn_up * c.sgn_dn * (c.Ssum < 0.0 ? -1.0 : 1.0);
        bad = c.sing_walker > 0 || c.Ssum == 0.0;
    }
    double lap = 0.0;
    for (int d = 0; d < 6 * S.ne; ++d) {
        const int coord = d >> 1, e = coord / 3, ax = coord % 3;
        const double step = (d & 1) ? -h : h;
        double y0 = x0, y1 = x1, y2 = x2;
        if (L.active && L.e == e) {
            if (ax == 0) y0 = x0 + step;
            else if (ax == 1) y1 = x1 + step;
            else y2 = x2 + step;
        }
        Core<NMO> c;
        core_stages<NMO, double, 0, false, false, true>(S, L, wsm, y0, y1, y2, c);
        const double lp = walker_sum(c.J, S.LW) + c.logD_up + c.logD_dn + log(fabs(c.Ssum));
        const double sg = c.sgn_up * c.sgn_dn * (c.Ssum < 0.0 ? -1.0 : 1.0);
        lap += sg * sg0 * exp(lp - lp0) - 1.0;
    }
    if (L.wvalid && L.lw == 0) {
        LP[w] = bad ? -INFINITY : lp0;
        EL[w] = bad ? NAN : -0.5 * lap / (h * h) + vpot;
    }
}

}  // namespace

// ---- launch dispatch ---------------------------------------------------------

static int nmo_bucket(int n_mo) {
    const int b[] = {4, 8, 12, 16, 20, 24, 32};
    for (int v : b)
        if (n_mo <= v) return v;
    return -1;
}

int padded_mo(int n_mo) { return nmo_bucket(n_mo); }

template <int NMO, typename RT, int MF, bool EXPL = false, bool BF = false>
static hipError_t launch_t(bool mc, const DevSystem &S, double *X, double *LP, double *SG, double *EL,
                           int64_t W, int n_steps, double sigma, uint64_t seed, uint64_t step0,
                           uint32_t woff, double *ACC, hipStream_t st) {
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    const int per = BF ? walker_lds_bf<NMO, !EXPL>(S) : (EXPL ? walker_lds_explicit<NMO>(S) : walker_lds<NMO>(S));
    size_t lds = (size_t)S.WPW * per * sizeof(double);
    if (MF > 0 && lds < (size_t)kStageBytes) lds = kStageBytes;
    if (mc && BF) {
        // one launch per step; the state and the running sums go through
        // the caller's arrays between launches, so the result is the block's
        for (int t = 0; t < n_steps; ++t) {
            hipLaunchKernelGGL((k_metropolis<NMO, RT, MF, EXPL, BF>), dim3((unsigned)blocks), dim3(kWave), lds, st,
                               S, X, LP, SG, EL, W, 1, sigma, seed, step0 + (uint64_t)t, woff, ACC);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    } else if (mc)
        hipLaunchKernelGGL((k_metropolis<NMO, RT, MF, EXPL, BF>), dim3((unsigned)blocks), dim3(kWave), lds, st,
                           S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC);
    else
        hipLaunchKernelGGL((k_eval<NMO, RT, MF, EXPL, BF>), dim3((unsigned)blocks), dim3(kWave), lds, st, S,
                           (const double *)X, W, LP, SG, EL);
    return hipGetLastError();
}

static hipError_t launch_explicit(bool mc, const DevSystem &S, double *X, double *LP, double *SG,
                                  double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                                  uint64_t step0, uint32_t woff, double *ACC, hipStream_t st) {
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: return launch_t<N, double, 0, true>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return hipErrorInvalidValue;
}

// Backflow: low-rank configurations (EXPL = false) or every configuration
// factorised (EXPL = true).
template <bool EXPL>
static hipError_t launch_backflow(bool mc, const DevSystem &S, double *X, double *LP, double *SG,
                                  double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                                  uint64_t step0, uint32_t woff, double *ACC, hipStream_t st) {
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: return launch_t<N, double, 0, EXPL, true>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return hipErrorInvalidValue;
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

hipError_t launch_eval_fd(const DevSystem &S, const double *X, int64_t W, double h, double *LP, double *EL,
                          hipStream_t st) {
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    switch (S.nmo_pad) {
#define QMC_CASE(N)                                                                                    \
    case N:                                                                                            \
        hipLaunchKernelGGL((k_eval_fd<N>), dim3((unsigned)blocks), dim3(kWave),                        \
                           (size_t)S.WPW * walker_lds<N>(S) * sizeof(double), st, S, X, W, h, LP, EL); \
        return hipGetLastError();
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return hipErrorInvalidValue;
}

size_t explicit_lds_bytes(const DevSystem &S) {
    int per = 0;
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: per = walker_lds_explicit<N>(S); break;
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return (size_t)S.WPW * per * sizeof(double);
}

template <typename RT, int MF>
static hipError_t launch_rt(bool mc, const DevSystem &S, double *X, double *LP, double *SG,
                            double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                            uint64_t step0, uint32_t woff, double *ACC, hipStream_t st) {
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: return launch_t<N, RT, MF>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return hipErrorInvalidValue;
}

// form: 0 FP64, 1 mixed FP32 (VALU), 2 mixed BF16 on the matrix cores with
// split operands, 3 mixed BF16 single products, 4 FP64 with explicit
// determinants, 5 FP64 with backflow and every configuration factorised,
// 6 FP64 with backflow and the low-rank configuration update.
hipError_t launch_walkers(bool mc, int form, const DevSystem &S, double *X, double *LP, double *SG,
                          double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                          uint64_t step0, uint32_t woff, double *ACC, hipStream_t st) {
    switch (form) {
        case 0: return launch_rt<double, 0>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 1: return launch_rt<float, 0>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 2: return launch_rt<float, 3>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 3: return launch_rt<float, 1>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 4: return launch_explicit(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 5: return launch_backflow<true>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        case 6: return launch_backflow<false>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
