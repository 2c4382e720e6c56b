// HIP kernels (gfx950): local energy evaluation and all-electron Metropolis
// blocks, and their launch.  The per-walker stages live in qmc_walker.h.
// Each qmc_form_*.hip translation unit instantiates the kernels of some
// arithmetic forms (so they compile in parallel); qmc_kernels.hip dispatches.
#pragma once

#include "qmc_walker.h"

namespace qmc {

using namespace walker;

namespace {

struct WalkerResult {
    double logpsi, sign, eloc;
};

// Mixed forms: a walker whose kinetic energy from the FP32 orbitals exceeds
// this magnitude (Ha), or is not finite, is evaluated again with FP64
// orbitals.  Such walkers have an electron inside the tightest primitives,
// where the kinetic terms are 1e4 - 1e6 Ha and cancel, so the rounding of
// FP32 orbital values (amplified by the Slater inverse) reaches ~1 Ha.
constexpr double kRefineKinetic = 3.0e4;

// One evaluation of log|Psi|, sign and E_L (hi: FP64 orbitals in a mixed
// form); kin receives the walker's kinetic energy.
template <int NMO, typename RT, int MF, bool EXPL, bool BF>
__device__ __forceinline__ WalkerResult eval_once(const DevSystem &S, const Lane &L, double *wsm, double x0,
                                                  double x1, double x2, void *stage, bool hi, double &kin_w) {
    Core<NMO> c;
    core_stages<NMO, RT, MF, EXPL, BF>(S, L, wsm, x0, x1, x2, c, stage, hi);

    // ---- pass 2: grad and Laplacian of Sigma at this electron ---------------
    double gS0, gS1, gS2, lapS;
    if constexpr (BF) {
        // the backflow stage returns them directly (the Laplacian in full
        // on electron 0's lane)
        gS0 = c.bgS0;
        gS1 = c.bgS1;
        gS2 = c.bgS2;
        lapS = c.blap;
    } else if (sizeof(RT) == sizeof(double) || hi) {
        sigma_derivs<NMO, double>(S, x0, x1, x2, c.av, gS0, gS1, gS2, lapS);
    } else {
        sigma_derivs<NMO, RT>(S, x0, x1, x2, c.av, gS0, gS1, gS2, lapS);
    }

    // ---- local energy and log|Psi| ------------------------------------------
    double part = 0.0, kin = 0.0;
    if (L.active) {
        kin = -0.5 * (lapS + c.lapJ + c.gJ0 * c.gJ0 + c.gJ1 * c.gJ1 + c.gJ2 * c.gJ2 +
                      2.0 * (c.gJ0 * gS0 + c.gJ1 * gS1 + c.gJ2 * gS2));
        part = kin + c.vpot;
    }
    const double eloc = walker_sum(part, S.LW) + S.vnn;
    const double Jw = walker_sum(c.J, S.LW);
    kin_w = walker_sum(kin, S.LW);
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

// Evaluates log|Psi|, sign and E_L of the lane's walker at the electron
// positions held by its lanes (x0, x1, x2 of the lane's electron).  Every
// lane of the block must call it (it contains block barriers); results are
// identical on all lanes of a walker.  In the mixed forms a second pass
// with FP64 orbitals runs when a walker of the wave needs it (wave-uniform
// branch); only the walkers that need it take its results, so a walker's
// result still depends on its own positions only.
template <int NMO, typename RT, int MF, bool EXPL, bool BF>
__device__ __forceinline__ WalkerResult eval_walker(const DevSystem &S, const Lane &L, double *wsm, double x0,
                                                    double x1, double x2, void *stage) {
    constexpr bool kMixed = sizeof(RT) != sizeof(double);
    WalkerResult res;
    bool need = false;
#pragma unroll 1
    for (int pass = 0; pass < (kMixed ? 2 : 1); ++pass) {
        double kin_w;
        const WalkerResult r = eval_once<NMO, RT, MF, EXPL, BF>(S, L, wsm, x0, x1, x2, stage, pass > 0, kin_w);
        if (pass == 0 || need) res = r;
        if (pass > 0) break;
        need = L.wvalid && !(fabs(kin_w) <= kRefineKinetic);
        if (!kMixed || !__any(need ? 1 : 0)) break;
    }
    return res;
}

template <int NMO, typename RT, bool EXPL, bool BF>
__host__ __device__ inline int lds_per_walker(const DevSystem &S) {
    if constexpr (BF) return walker_lds_bf<NMO, !EXPL>(S);
    else if constexpr (EXPL) return walker_lds_explicit<NMO>(S);
    else return walker_lds<NMO, (sizeof(RT) != sizeof(double))>(S);
}

// Launch shapes of the Metropolis kernel.  The FP64 low-rank form takes one
// step per launch (the host enqueues the block step by step; the arrays
// carry the state between launches): without a step loop the evaluation
// keeps the registers it has on its own instead of sharing them with values
// held across steps, and fits three waves per SIMD (168 registers), which
// its compact LDS tables (about 11.6 KB per CO wave) also allow.  The mixed
// forms carry both orbital paths and run at two waves; they keep the whole
// block in one launch (one step per launch measured 1.4x slower for them):
// the BF16 ones with a two-wave bound (left alone they take a few registers
// more and run at one), the FP32 one with the registers it chooses (252).
// The explicit kernel runs the block in one launch at one wave (its LDS and
// registers), the backflow kernels one step per launch at one wave.
template <typename RT, int MF, bool EXPL, bool BF>
constexpr bool metro_one_step() { return BF || (!EXPL && sizeof(RT) == sizeof(double)); }

template <typename RT, int MF, bool EXPL, bool BF>
constexpr int metro_waves() {
    return (EXPL || BF) ? 1 : (sizeof(RT) == sizeof(double) ? 3 : (MF == 0 ? 1 : 2));
}

template <int NMO, typename RT, int MF, bool EXPL, bool BF>
__global__ __launch_bounds__(kWave, (MF > 0 ? 2 : 1)) void k_eval(DevSystem S, const double *__restrict__ X, int64_t W,
                                                 double *__restrict__ LP, double *__restrict__ SG,
                                                 double *__restrict__ EL) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    double *wsm = smem + L.wloc * lds_per_walker<NMO, RT, EXPL, BF>(S);
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
__global__ __launch_bounds__(kWave, (metro_waves<RT, MF, EXPL, BF>())) void k_metropolis(DevSystem S, double *__restrict__ X,
                                                      double *__restrict__ LP, double *__restrict__ SG,
                                                      double *__restrict__ EL, int64_t W, int n_steps,
                                                      double sigma, uint64_t seed, uint64_t step0,
                                                      uint32_t walker_offset, double *__restrict__ ACC) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    double *wsm = smem + L.wloc * lds_per_walker<NMO, RT, EXPL, BF>(S);
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
    // (the two counts are integer-valued doubles below 2^31 in the array)
    double s_e = 0.0, s_e2 = 0.0;
    int n_acc = 0, n_bad = 0;
    if (L.wvalid) {
        s_e = ACC[4 * w + 0];
        s_e2 = ACC[4 * w + 1];
        n_acc = (int)ACC[4 * w + 2];
        n_bad = (int)ACC[4 * w + 3];
    }
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t wid = walker_offset + (uint32_t)w;
    const double s32 = 1.0 / 4294967296.0;
    const double two_pi = 6.283185307179586;
    // One step per launch where the host enqueues the block step by step:
    // without a loop around it the evaluation keeps the registers it has on
    // its own.
    const int steps = metro_one_step<RT, MF, EXPL, BF>() ? 1 : n_steps;
    for (int t = 0; t < steps; ++t) {
        const uint64_t step = step0 + (uint64_t)t;
        uint32_t c[4] = {wid, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)L.e};
        philox4x32_10(c, k0, k1);
        // Box-Muller on 32-bit uniforms (w + 1/2) 2^-32, in FP64 in every form
        const double u0 = ((double)c[0] + 0.5) * s32, u1 = ((double)c[1] + 0.5) * s32;
        const double u2 = ((double)c[2] + 0.5) * s32, u3 = ((double)c[3] + 0.5) * s32;
        const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
        double s1, c1;
        sincos(two_pi * u1, &s1, &c1);
        const double z0 = r0 * c1, z1 = r0 * s1, z2 = r1 * cos(two_pi * u3);
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
        // a state without a finite log|Psi| and E_L is counted, not summed
        if (isfinite(el) && isfinite(lp)) {
            s_e = __dadd_rn(s_e, el);
            s_e2 = __dadd_rn(s_e2, __dmul_rn(el, el));
        } else {
            ++n_bad;
        }
        n_acc += acc ? 1 : 0;
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
        ACC[4 * w + 0] = s_e;
        ACC[4 * w + 1] = s_e2;
        ACC[4 * w + 2] = (double)n_acc;
        ACC[4 * w + 3] = (double)n_bad;
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
    double *wsm = smem + L.wloc * walker_lds<NMO, false>(S);
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

// One form at one compiled MO width: eval (mc = false) or a Metropolis block.
template <int NMO, typename RT, int MF, bool EXPL = false, bool BF = false>
static hipError_t launch_t(bool mc, const DevSystem &S, double *X, double *LP, double *SG, double *EL,
                           int64_t W, int n_steps, double sigma, uint64_t seed, uint64_t step0,
                           uint32_t woff, double *ACC, hipStream_t st) {
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    const int per = lds_per_walker<NMO, RT, EXPL, BF>(S);
    size_t lds = (size_t)S.WPW * per * sizeof(double);
    if (MF > 0 && lds < (size_t)kStageBytes) lds = kStageBytes;
    if (mc && metro_one_step<RT, MF, EXPL, BF>()) {
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

// Signature shared by the per-form launchers.
#define QMC_LAUNCH_ARGS                                                                            \
    bool mc, const DevSystem &S, double *X, double *LP, double *SG, double *EL, int64_t W, int n_steps, \
        double sigma, uint64_t seed, uint64_t step0, uint32_t woff, double *ACC, hipStream_t st
#define QMC_LAUNCH_PASS mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st

// Switch over the compiled MO widths.
#define QMC_NMO_SWITCH(EXPR)                                                  \
    switch (S.nmo_pad) {                                                      \
        case 4: { constexpr int N = 4; EXPR; }                                \
        case 8: { constexpr int N = 8; EXPR; }                                \
        case 12: { constexpr int N = 12; EXPR; }                              \
        case 16: { constexpr int N = 16; EXPR; }                              \
        case 20: { constexpr int N = 20; EXPR; }                              \
        case 24: { constexpr int N = 24; EXPR; }                              \
        case 32: { constexpr int N = 32; EXPR; }                              \
    }                                                                         \
    return hipErrorInvalidValue;

hipError_t launch_form_fp64(QMC_LAUNCH_ARGS);
hipError_t launch_form_fp32(QMC_LAUNCH_ARGS);
hipError_t launch_form_bf16(QMC_LAUNCH_ARGS, int split);
hipError_t launch_form_explicit(QMC_LAUNCH_ARGS);
hipError_t launch_form_backflow(QMC_LAUNCH_ARGS, bool low_rank);

}  // namespace qmc
