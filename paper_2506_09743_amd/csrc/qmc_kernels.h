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
// orbitals (by the refinement launch that follows every mixed launch).  Such walkers have an electron inside the tightest primitives,
// where the kinetic terms are 1e4 - 1e6 Ha and cancel, so the rounding of
// FP32 orbital values (amplified by the Slater inverse) reaches ~1 Ha.
constexpr double kRefineKinetic = 3.0e4;

// Evaluates log|Psi|, sign and E_L of the lane's walker at the electron
// positions held by its lanes (x0, x1, x2 of the lane's electron).  Every
// lane of the block must call it (it contains block barriers); results are
// identical on all lanes of a walker.  need: a mixed form's result must be
// refined in FP64 (kinetic energy not finite or above kRefineKinetic).
template <int NMO, typename RT, int MF, bool EXPL, int BF>
__device__ __forceinline__ WalkerResult eval_walker(const DevSystem &S, const Lane &L, double *wsm, double x0,
                                                    double x1, double x2, void *stage, bool &need) {
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
    need = false;
    if constexpr (sizeof(RT) != sizeof(double)) need = L.wvalid && !(fabs(walker_sum(kin, S.LW)) <= kRefineKinetic);
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

template <int NMO, typename RT, bool EXPL, int BF>
__host__ __device__ inline int lds_per_walker(const DevSystem &S) {
    if constexpr (BF) return walker_lds_bf<NMO, !EXPL>(S);
    else if constexpr (EXPL) return walker_lds_explicit<NMO>(S);
    else return walker_lds<NMO, false>(S);
}

// Launch shapes of the Metropolis kernel.  The low-rank forms take one step
// per launch (the host enqueues the block step by step; the arrays carry
// the state between launches): without a step loop the evaluation keeps the
// registers it has on its own instead of sharing them with values held
// across steps, and the FP64 and FP32 kernels fit three waves per SIMD (168
// registers), which their compact LDS tables (about 11.6 KB per CO wave)
// also allow.  The BF16 kernels stage operands in about 19 KB of LDS per
// wave and run at two.  The explicit kernel runs the block in one launch at
// one wave (its LDS and registers), the backflow kernels one step per launch
// at one wave.
template <typename RT, int MF, bool EXPL, int BF>
constexpr bool metro_one_step() { return BF || !EXPL; }

template <typename RT, int MF, bool EXPL, int BF>
constexpr int metro_waves() { return (EXPL || BF) ? 1 : (MF == 0 ? 3 : 2); }

// Refinement of the mixed forms.  A walker whose FP32 result needs FP64
// orbitals is left as it was and marked in its sign entry: sign + mark, a
// sign being -1, 0 or +1 and a mark a multiple of 8 (>= 8).  The mark holds
// a kind and the step it refers to (mod 4):
//   deferred  (kind 0): step s was tried in FP32 and must be redone in FP64;
//   lagging   (kind 1): step s is still to be taken.
// An evaluation only defers (k_refine redoes the marked walkers).  In a
// Metropolis block, the step kernels skip marked walkers and k_refine, on a
// second stream one step behind, takes the marked ones: the deferred step
// in FP64, then each later step of the call in FP32 with FP64 where that
// needs it, so those walkers stay off the step kernels' critical path for
// the rest of the call and the last step leaves them unmarked.  No memory
// beyond the caller's arrays is used.
constexpr double kMarkUnit = 8.0;

__device__ __forceinline__ bool marked(double sg) { return sg >= 0.5 * kMarkUnit; }

__device__ __forceinline__ double mark_of(int kind, uint64_t step) {
    return kMarkUnit * (double)(1 + (int)(step & 3u) + 4 * kind);
}

// code of a marked entry: (step & 3) | kind << 2; its sign is what is left
__device__ __forceinline__ int mark_code(double sg) { return (int)rint(sg / kMarkUnit) - 1; }

// One evaluation of the walkers of a wave (w: this lane's walker).  A mixed
// form defers the walkers to refine (their log|Psi| and E_L are left
// unwritten); the refinement evaluates them again in FP64.
template <int NMO, typename RT, int MF, bool EXPL, int BF>
__device__ __forceinline__ void eval_wave(const DevSystem &S, const Lane &L, int64_t w, const double *__restrict__ X,
                                          double *__restrict__ LP, double *__restrict__ SG,
                                          double *__restrict__ EL, double *smem) {
    constexpr bool kMixed = sizeof(RT) != sizeof(double);
    double *wsm = smem + L.wloc * lds_per_walker<NMO, RT, EXPL, BF>(S);
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (L.active) {
        const double *p = X + (w * S.ne + L.e) * 3;
        x0 = p[0];
        x1 = p[1];
        x2 = p[2];
    }
    bool need;
    const WalkerResult r = eval_walker<NMO, RT, MF, EXPL, BF>(S, L, wsm, x0, x1, x2, smem, need);
    if (L.wvalid && L.lw == 0) {
        if (kMixed && need) {
            SG[w] = mark_of(0, 0);
        } else {
            LP[w] = r.logpsi;
            SG[w] = r.sign;
            EL[w] = r.eloc;
        }
    }
}

// Marks of one Metropolis step: in_mark is subtracted from the sign read
// (the walker's current mark, 0 when unmarked); a completed step stores
// sign + done_mark, a mixed step that needs FP64 stores sign + defer_mark
// and leaves the walker untouched.
struct StepMarks {
    double in_mark, done_mark, defer_mark;
};

// n_steps Metropolis steps of the valid walkers of a wave (w: this lane's
// walker).  Mixed forms read a caller's sign entry as its sign.  INL (mixed
// forms): a walker whose proposal needs FP64 orbitals is evaluated again
// with them right away (the wave runs the FP64 evaluation when any of its
// walkers needs it), so any number of steps can be taken; otherwise mixed
// forms take one step per call and defer such walkers.
template <int NMO, typename RT, int MF, bool EXPL, int BF, bool INL = false>
__device__ __forceinline__ void metropolis_wave(const DevSystem &S, const Lane &L, int64_t w, double *__restrict__ X,
                                                double *__restrict__ LP, double *__restrict__ SG,
                                                double *__restrict__ EL, int n_steps, double sigma, uint64_t seed,
                                                uint64_t step0, uint32_t walker_offset, double *__restrict__ ACC,
                                                double *smem, StepMarks mk) {
    constexpr bool kMixed = sizeof(RT) != sizeof(double);
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
        sg = SG[w] - mk.in_mark;
        el = EL[w];
        if constexpr (kMixed) sg = sg > 0.0 ? 1.0 : (sg < 0.0 ? -1.0 : 0.0);
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
    bool defer = false;
    for (int t = 0; t < n_steps; ++t) {
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

        bool need;
        WalkerResult r = eval_walker<NMO, RT, MF, EXPL, BF>(S, L, wsm, y0, y1, y2, smem, need);
        if constexpr (kMixed && INL) {
            if (__any(need ? 1 : 0)) {
                bool unused;
                const WalkerResult r64 =
                    eval_walker<NMO, double, 0, false, false>(S, L, wsm, y0, y1, y2, smem, unused);
                if (need) r = r64;
            }
        } else {
            defer = kMixed && need;
            if (defer) continue;  // one step per call
        }
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
    if (defer) {  // state unchanged, sign marked
        if (L.wvalid && L.lw == 0) SG[w] = sg + mk.defer_mark;
        return;
    }
    if (L.active) {
        double *p = X + (w * S.ne + L.e) * 3;
        p[0] = x0;
        p[1] = x1;
        p[2] = x2;
    }
    if (L.wvalid && L.lw == 0) {
        LP[w] = lp;
        SG[w] = sg + mk.done_mark;
        EL[w] = el;
        ACC[4 * w + 0] = s_e;
        ACC[4 * w + 1] = s_e2;
        ACC[4 * w + 2] = (double)n_acc;
        ACC[4 * w + 3] = (double)n_bad;
    }
}

template <int NMO, typename RT, int MF, bool EXPL, int BF>
__global__ __launch_bounds__(kWave, (MF > 0 ? 2 : 1)) void k_eval(DevSystem S, const double *__restrict__ X, int64_t W,
                                                 double *__restrict__ LP, double *__restrict__ SG,
                                                 double *__restrict__ EL) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    eval_wave<NMO, RT, MF, EXPL, BF>(S, L, w, X, LP, SG, EL, smem);
}

// skip_marked (mixed forms, every step of a call but its first): walkers
// already marked belong to k_refine for the rest of the call and are left
// alone, including their sign entry.
template <int NMO, typename RT, int MF, bool EXPL, int BF>
__global__ __launch_bounds__(kWave, (metro_waves<RT, MF, EXPL, BF>())) void k_metropolis(DevSystem S, double *__restrict__ X,
                                                      double *__restrict__ LP, double *__restrict__ SG,
                                                      double *__restrict__ EL, int64_t W, int n_steps,
                                                      double sigma, uint64_t seed, uint64_t step0,
                                                      uint32_t walker_offset, double *__restrict__ ACC,
                                                      int skip_marked) {
    constexpr bool kMixed = sizeof(RT) != sizeof(double);
    static_assert(!kMixed || metro_one_step<RT, MF, EXPL, BF>(), "a mixed step defers walkers one step at a time");
    extern __shared__ double smem[];
    int64_t w;
    Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    if (kMixed && skip_marked && L.wvalid && marked(SG[w])) {
        L.wvalid = false;
        L.active = false;
    }
    const int steps = metro_one_step<RT, MF, EXPL, BF>() ? 1 : n_steps;
    const StepMarks mk{0.0, 0.0, kMixed ? mark_of(0, step0) : 0.0};
    metropolis_wave<NMO, RT, MF, EXPL, BF>(S, L, w, X, LP, SG, EL, steps, sigma, seed, step0, walker_offset, ACC,
                                            smem, mk);
}

// Metropolis block in one launch (step loop) for blocks of at most
// kLoopWaves waves, the low-rank forms without backflow: with one wave per
// SIMD every wave is resident at once, so a step costs one wave's latency
// whether it is one launch or one loop trip, and the loop saves a launch
// per step (small molecules and small requests would otherwise be bound by
// launches).  Mixed forms refine inside the loop.
constexpr int64_t kLoopWaves = 1024;

template <int NMO, typename RT, int MF>
__global__ __launch_bounds__(kWave, 1) void k_metropolis_loop(DevSystem S, double *__restrict__ X,
                                                              double *__restrict__ LP, double *__restrict__ SG,
                                                              double *__restrict__ EL, int64_t W, int n_steps,
                                                              double sigma, uint64_t seed, uint64_t step0,
                                                              uint32_t walker_offset, double *__restrict__ ACC) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    metropolis_wave<NMO, RT, MF, false, false, true>(S, L, w, X, LP, SG, EL, n_steps, sigma, seed, step0,
                                                     walker_offset, ACC, smem, StepMarks{0.0, 0.0, 0.0});
}

// The refinement of a mixed evaluation (MC = false: every marked walker,
// evaluated in FP64) or of Metropolis step `step` (MC = true: the walkers
// marked for that step; last: the call's last step, which leaves them
// unmarked, else they are marked lagging for the next step).  Work-group b
// scans walkers [b span, (b + 1) span) 64 at a time and gathers the ones it
// takes into its wave's walker slots, WPW at a time, so a few hundred
// work-groups cover any W and each usually evaluates once or twice.  Every
// work-group leaves the loop once its range is scanned.  Few waves run at
// once, so the kernel takes the registers it wants (one wave per SIMD).
constexpr int kRefineGroups = 1024;

template <int NMO, typename RT, int MF, bool MC>
__global__ __launch_bounds__(kWave, 3) void k_refine(DevSystem S, double *__restrict__ X, double *__restrict__ LP,
                                                     double *__restrict__ SG, double *__restrict__ EL, int64_t W,
                                                     int64_t span, double sigma, uint64_t seed, uint64_t step,
                                                     int last, uint32_t walker_offset, double *__restrict__ ACC) {
    extern __shared__ double smem[];
    int64_t w0;
    const Lane L0 = make_lane(S, 0, W, &w0);
    const int64_t lo = (int64_t)blockIdx.x * span;
    const int64_t hi = lo + span < W ? lo + span : W;
    const int want = (int)(step & 3u);
    int64_t next = lo;  // scan cursor, the same on every lane
    while (next < hi) {
        int64_t mine = -1;  // walker of this lane's slot
        int found = 0;
        while (found < S.WPW && next < hi) {
            const int64_t q = next + L0.lane;
            bool m = false;
            if (q < hi) {
                const double v = SG[q];
                m = marked(v) && (!MC || (mark_code(v) & 3) == want);
            }
            uint64_t mask = __ballot(m ? 1 : 0);
            int64_t adv = kWave;
            while (mask != 0) {
                const int b = __ffsll((unsigned long long)mask) - 1;
                if (found == S.WPW) {
                    adv = b;  // resume at the first walker not taken
                    break;
                }
                if (L0.wloc == found) mine = next + b;
                ++found;
                mask &= mask - 1;
            }
            next += adv;
        }
        if (found == 0) break;
        Lane L = L0;
        L.wvalid = L0.wloc < found;
        L.active = L.wvalid && L0.active;
        const int64_t w = L.wvalid ? mine : 0;
        if constexpr (!MC) {
            eval_wave<NMO, double, 0, false, false>(S, L, w, X, LP, SG, EL, smem);
        } else {
            const double done = last ? 0.0 : mark_of(1, step + 1);
            // lagging walkers first take the step in FP32 (a walker that
            // needs FP64 becomes deferred), then the deferred ones in FP64
            const double sv = L.wvalid ? SG[w] : 0.0;
            Lane La = L;
            La.wvalid = L.wvalid && (mark_code(sv) >> 2) == 1;
            La.active = La.wvalid && L0.active;
            if (__any(La.wvalid ? 1 : 0)) {
                metropolis_wave<NMO, RT, MF, false, false>(S, La, w, X, LP, SG, EL, 1, sigma, seed, step,
                                                           walker_offset, ACC, smem,
                                                           StepMarks{mark_of(1, step), done, mark_of(0, step)});
                __syncthreads();  // its stores before the loads below
            }
            const double sd = L.wvalid ? SG[w] : 0.0;
            Lane Ld = L;
            Ld.wvalid = L.wvalid && marked(sd) && mark_code(sd) == want;
            Ld.active = Ld.wvalid && L0.active;
            if (__any(Ld.wvalid ? 1 : 0))
                metropolis_wave<NMO, double, 0, false, false>(S, Ld, w, X, LP, SG, EL, 1, sigma, seed, step,
                                                              walker_offset, ACC, smem,
                                                              StepMarks{mark_of(0, step), done, 0.0});
        }
        __syncthreads();  // the slots' stores before the next scan
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

// Refinement grid: ranges of whole 64-walker chunks over at most
// kRefineGroups work-groups.
struct RefineGrid {
    int64_t span;
    unsigned grid;
    explicit RefineGrid(int64_t W) {
        const int64_t chunks = (W + kWave - 1) / kWave;
        const int64_t groups = chunks < 1 ? 1 : (chunks < kRefineGroups ? chunks : kRefineGroups);
        span = ((chunks + groups - 1) / groups) * kWave;
        grid = (unsigned)((W + span - 1) / span);
    }
};

// Blocks of at least this many waves are split in two halves, one per
// stream: a one-step launch ends with a partly filled last round of waves,
// and the other stream's launch fills it.
constexpr int64_t kSplitWaves = 1536;

// Mixed blocks of more than this many waves refine on the second stream,
// one step behind (five runtime calls per step); smaller ones refine after
// each step on the caller's stream (two calls per step), where the
// refinement's latency is left to other work on the device to fill.
constexpr int64_t kLagWaves = 8192;

// One form at one compiled MO width: eval (mc = false) or a Metropolis
// block.
//  - Mixed eval: the eval launch, then k_refine on the same stream.
//  - Mixed block of more than kLagWaves waves: the step launches on st;
//    after each, k_refine of that step on the side stream (it waits for the
//    step's launch), and the step launch two steps later waits for it, so
//    the side stream runs at most one step behind; st waits for the last
//    one before the call returns.  Smaller mixed blocks: each step launch
//    followed by its k_refine on st.
//  - Other one-step blocks: the walkers in two halves of whole waves, one
//    per stream, when the block has kSplitWaves waves or more.
//  - Blocks of at most kLoopWaves waves (low-rank, no backflow, any
//    form): one k_metropolis_loop launch on st.
//  - Otherwise one launch on st.
template <int NMO, typename RT, int MF, bool EXPL = false, int BF = 0>
static hipError_t launch_t(bool mc, const DevSystem &S, double *X, double *LP, double *SG, double *EL,
                           int64_t W, int n_steps, double sigma, uint64_t seed, uint64_t step0,
                           uint32_t woff, double *ACC, const CallStreams &cs) {
    constexpr bool kMixed = sizeof(RT) != sizeof(double);
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    size_t lds = (size_t)S.WPW * lds_per_walker<NMO, RT, EXPL, BF>(S) * sizeof(double);
    if (MF > 0 && lds < (size_t)kStageBytes) lds = kStageBytes;
    const hipStream_t st = cs.st;
    hipError_t e = hipSuccess;
    if constexpr (!EXPL && !BF) {
        if (mc && blocks <= kLoopWaves) {
            size_t llds = (size_t)S.WPW * lds_per_walker<NMO, double, false, false>(S) * sizeof(double);
            if (llds < lds) llds = lds;
            hipLaunchKernelGGL((k_metropolis_loop<NMO, RT, MF>), dim3((unsigned)blocks), dim3(kWave), llds, st, S,
                               X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC);
            return hipGetLastError();
        }
    }
    auto step_launch = [&](hipStream_t s, int64_t first, int64_t n, uint64_t step, int skip) {
        const int64_t nb = (n + S.WPW - 1) / S.WPW;
        hipLaunchKernelGGL((k_metropolis<NMO, RT, MF, EXPL, BF>), dim3((unsigned)nb), dim3(kWave), lds, s, S,
                           X + first * S.ne * 3, LP + first, SG + first, EL + first, n, 1, sigma, seed, step,
                           woff + (uint32_t)first, ACC + 4 * first, skip);
    };
    if constexpr (kMixed) {
        size_t rlds = (size_t)S.WPW * lds_per_walker<NMO, double, false, false>(S) * sizeof(double);
        if (rlds < lds) rlds = lds;  // the refinement also runs the mixed step
        const RefineGrid rg(W);
        if (!mc) {
            hipLaunchKernelGGL((k_eval<NMO, RT, MF, EXPL, BF>), dim3((unsigned)blocks), dim3(kWave), lds, st, S,
                               (const double *)X, W, LP, SG, EL);
            hipLaunchKernelGGL((k_refine<NMO, RT, MF, false>), dim3(rg.grid), dim3(kWave), rlds, st, S, X, LP, SG,
                               EL, W, rg.span, 0.0, (uint64_t)0, (uint64_t)0, 0, (uint32_t)0, (double *)nullptr);
            return hipGetLastError();
        }
        if (blocks <= kLagWaves) {
            for (int t = 0; t < n_steps && e == hipSuccess; ++t) {
                const uint64_t step = step0 + (uint64_t)t;
                step_launch(st, 0, W, step, 0);
                hipLaunchKernelGGL((k_refine<NMO, RT, MF, true>), dim3(rg.grid), dim3(kWave), rlds, st, S, X, LP,
                                   SG, EL, W, rg.span, sigma, seed, step, 1, woff, ACC);
                e = hipGetLastError();
            }
            return e;
        }
        for (int t = 0; t < n_steps && e == hipSuccess; ++t) {
            const uint64_t step = step0 + (uint64_t)t;
            if (t >= 2) e = hipStreamWaitEvent(st, cs.ev[1 + (t - 2) % 3], 0);
            if (e != hipSuccess) break;
            step_launch(st, 0, W, step, t > 0 ? 1 : 0);
            if ((e = hipGetLastError()) != hipSuccess) break;
            if ((e = hipEventRecord(cs.ev[0], st)) != hipSuccess) break;
            if ((e = hipStreamWaitEvent(cs.side, cs.ev[0], 0)) != hipSuccess) break;
            hipLaunchKernelGGL((k_refine<NMO, RT, MF, true>), dim3(rg.grid), dim3(kWave), rlds, cs.side, S, X, LP,
                               SG, EL, W, rg.span, sigma, seed, step, t == n_steps - 1 ? 1 : 0, woff, ACC);
            if ((e = hipGetLastError()) != hipSuccess) break;
            e = hipEventRecord(cs.ev[1 + t % 3], cs.side);
        }
        if (e == hipSuccess) e = hipStreamWaitEvent(st, cs.ev[1 + (n_steps - 1) % 3], 0);
        return e;
    } else {
        if (mc && metro_one_step<RT, MF, EXPL, BF>()) {
            // one launch per step; the state and the running sums go
            // through the caller's arrays between launches
            const bool split = blocks >= kSplitWaves;
            const int64_t wa = split ? ((blocks + 1) / 2) * S.WPW : W;
            if (split) {
                if ((e = hipEventRecord(cs.ev[0], st)) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(cs.side, cs.ev[0], 0)) != hipSuccess) return e;
            }
            for (int t = 0; t < n_steps && e == hipSuccess; ++t) {
                step_launch(st, 0, wa, step0 + (uint64_t)t, 0);
                e = hipGetLastError();
            }
            if (split) {
                for (int t = 0; t < n_steps && e == hipSuccess; ++t) {
                    step_launch(cs.side, wa, W - wa, step0 + (uint64_t)t, 0);
                    e = hipGetLastError();
                }
                if (e == hipSuccess) e = hipEventRecord(cs.ev[1], cs.side);
                if (e == hipSuccess) e = hipStreamWaitEvent(st, cs.ev[1], 0);
            }
            return e;
        }
        if (mc) {
            hipLaunchKernelGGL((k_metropolis<NMO, RT, MF, EXPL, BF>), dim3((unsigned)blocks), dim3(kWave), lds, st,
                               S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, 0);
        } else {
            hipLaunchKernelGGL((k_eval<NMO, RT, MF, EXPL, BF>), dim3((unsigned)blocks), dim3(kWave), lds, st, S,
                               (const double *)X, W, LP, SG, EL);
        }
        return hipGetLastError();
    }
}

// Signature shared by the per-form launchers.
#define QMC_LAUNCH_ARGS                                                                            \
    bool mc, const DevSystem &S, double *X, double *LP, double *SG, double *EL, int64_t W, int n_steps, \
        double sigma, uint64_t seed, uint64_t step0, uint32_t woff, double *ACC, const CallStreams &cs
#define QMC_LAUNCH_PASS mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, cs

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
