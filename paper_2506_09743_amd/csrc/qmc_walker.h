// Device-side building blocks of the walker evaluation, shared by the
// evaluation / Metropolis kernels and the gradient kernel of libqmc.
//
// Work decomposition.  One wave of 64 lanes holds 64 / (2G) walkers; each
// walker owns 2G consecutive lanes, G per spin, and lane i of a spin group
// owns electron i of that spin.  A lane evaluates its electron's atomic
// orbitals and molecular orbitals in registers, the Slater matrices are
// factorised across the lanes of a group (row = electron), and the walker's
// scalars are reduced across its lanes with cross-lane shuffles.  Walkers
// never interact, so a walker's results do not depend on its neighbours.
//
// Kinetic energy (appendix on local energies).  With Psi = exp(J) Sigma the
// Laplacian splits into lap J + |grad J|^2 + 2 grad J . grad Sigma / Sigma +
// lap Sigma / Sigma.  Because every determinant is linear in the row of one
// electron, grad_e Sigma / Sigma = sum_m a_e[m] grad phi_m(r_e) and
// lap_e Sigma / Sigma = sum_m a_e[m] lap phi_m(r_e) with a_e[m] =
// d log Sigma / d phi_m(r_e) (this is the per-electron Jacobi trace of
// eq. claudia_trace summed over the CI expansion).  a_e follows from the
// low-rank excited-determinant algebra of eq. table: with T = A0^-1 Phi,
// every excited determinant is D0 det T[H,P] (k <= 2), Sigma = D0 S with
// S = sum_n d_n det T_up[H,P] det T_dn[H,P], and the CI-weighted cofactors
// C = dS/dT give a_e[v] = (A0^-T C)[e,v] / S on virtual orbitals and
// a_e[k] = A0^-1[k,e] - (A0^-T C T^T)[e,k] / S on reference orbitals.
// Only A0 is ever inverted, as in the paper's accelerated scheme.
#pragma once

#include "qmc_device.h"
#include "qmc_exp.h"

#include <math.h>

namespace qmc {
namespace walker {

// Determinant and cofactor records fetched per batch.
constexpr int kRecBatch = 4;


// Cross-lane exchange within a row of 16 lanes by DPP moves (no LDS round
// trip).  Walkers (LW <= 16 lanes) and spin groups (G <= 8 lanes) are
// aligned to their power-of-two size, so these steps never leave them:
// kSwap1 pairs lane ^ 1 and kSwap2 lane ^ 2 (quad permutes), kHalfMirror
// pairs lane i with 7 - i in each 8-lane half (the other quad), kMirror
// pairs lane i with 15 - i (the other half).  Applied in this order a
// reduction pairs the same partial results as an xor butterfly, and every
// lane of the span ends with the same value.  Callers run them with all
// lanes of the wave active.
constexpr int kSwap1 = 0xB1, kSwap2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    return __hiloint2double(dpp_i<CTRL>(__double2hiint(v)), dpp_i<CTRL>(__double2loint(v)));
}

// Sum over an aligned span of n = 1, 2, 4, 8 or 16 lanes.
__device__ __forceinline__ double span_sum(double v, int n) {
    if (n > 1) v += dpp_d<kSwap1>(v);
    if (n > 2) v += dpp_d<kSwap2>(v);
    if (n > 4) v += dpp_d<kHalfMirror>(v);
    if (n > 8) v += dpp_d<kMirror>(v);
    return v;
}

__device__ __forceinline__ int span_sum_i(int v, int n) {
    if (n > 1) v += dpp_i<kSwap1>(v);
    if (n > 2) v += dpp_i<kSwap2>(v);
    if (n > 4) v += dpp_i<kHalfMirror>(v);
    if (n > 8) v += dpp_i<kMirror>(v);
    return v;
}

__device__ __forceinline__ double span_max(double v, int n) {
    if (n > 1) v = fmax(v, dpp_d<kSwap1>(v));
    if (n > 2) v = fmax(v, dpp_d<kSwap2>(v));
    if (n > 4) v = fmax(v, dpp_d<kHalfMirror>(v));
    if (n > 8) v = fmax(v, dpp_d<kMirror>(v));
    return v;
}

// Largest cand over the span, ties to the lower index cl; the result is the
// same on every lane of the span.
template <int CTRL>
__device__ __forceinline__ void argmax_step(double &cand, int &cl) {
    const double oc = dpp_d<CTRL>(cand);
    const int ol = dpp_i<CTRL>(cl);
    if (oc > cand || (oc == cand && ol < cl)) {
        cand = oc;
        cl = ol;
    }
}

__device__ __forceinline__ void span_argmax(double &cand, int &cl, int n) {
    if (n > 1) argmax_step<kSwap1>(cand, cl);
    if (n > 2) argmax_step<kSwap2>(cand, cl);
    if (n > 4) argmax_step<kHalfMirror>(cand, cl);
    if (n > 8) argmax_step<kMirror>(cand, cl);
}

// Sum over the LW lanes of a walker.
__device__ __forceinline__ double walker_sum(double v, int LW) { return span_sum(v, LW); }

__device__ __forceinline__ int walker_sum_i(int v, int LW) { return span_sum_i(v, LW); }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

struct Lane {
    int lane;    // 0..63
    int wloc;    // walker slot in the wave
    int lw;      // lane within walker, 0..LW-1
    int grp;     // 0 spin up, 1 spin down
    int i;       // index within the spin group
    int e;       // electron index within the walker
    int nsig;    // electrons of this spin
    int gbase;   // first lane of the group
    bool wvalid; // walker index < W
    bool active; // owns a real electron of a valid walker
};

__device__ __forceinline__ Lane make_lane(const DevSystem &S, int64_t wave_first_walker, int64_t W,
                                          int64_t *walker) {
    Lane L;
    L.lane = threadIdx.x;
    L.wloc = L.lane / S.LW;
    L.lw = L.lane % S.LW;
    L.grp = L.lw / S.G;
    L.i = L.lw % S.G;
    L.nsig = L.grp == 0 ? S.n_up : S.n_dn;
    L.e = L.grp == 0 ? L.i : S.n_up + L.i;
    L.gbase = L.lane - L.i;
    const int64_t w = wave_first_walker + L.wloc;
    *walker = w;
    L.wvalid = (L.wloc < S.WPW) && (w < W);
    L.active = L.wvalid && (L.i < L.nsig);
    return L;
}

// Determinant ratio det T[H,P] of one spin, rank k <= 2, from the walker's
// T table (row = slot, column = MO, stride NMO).
template <int NMO>
__device__ __forceinline__ double ratio(const double *T, const int *d) {
    const int k = d[0];
    if (k == 0) return 1.0;
    const double a = T[d[1] * NMO + d[3]];
    if (k == 1) return a;
    return a * T[d[2] * NMO + d[4]] - T[d[1] * NMO + d[4]] * T[d[2] * NMO + d[3]];
}

// Determinant ratio from a packed excitation code (rank | h1 << 2 |
// h2 << 5 | p1 << 8 | p2 << 13); T rows of `ts` columns starting at column
// c0 (particles are virtual orbitals, p >= c0).
__device__ __forceinline__ double ratio_code(const double *T, uint32_t c, int ts, int c0) {
    const uint32_t k = c & 3u;
    if (k == 0) return 1.0;
    const int h1 = (c >> 2) & 7, h2 = (c >> 5) & 7, p1 = ((c >> 8) & 31) - c0, p2 = ((c >> 13) & 31) - c0;
    const double a = T[h1 * ts + p1];
    if (k == 1) return a;
    return a * T[h2 * ts + p2] - T[h1 * ts + p2] * T[h2 * ts + p1];
}

// d = a * b + c as one three-address FMA: the constant c stays in the
// register that holds it for the whole kernel instead of being copied into
// the accumulator of a two-address FMA before every use.
__device__ __forceinline__ double fma_c(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// exp(x) in FP64 (qmc_exp.h), its polynomial's multiply-adds as
// three-address FMAs.
__device__ __forceinline__ double exp_f64(double x) { return exp_cody_waite(x, fma_c); }

// 1 / x for x >= 1 (the Pade-type denominators 1 + b r): the hardware
// reciprocal estimate refined by two Newton steps, within an ulp or so of
// the quotient.
__device__ __forceinline__ double rcp_ge1(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

template <typename RT> __device__ __forceinline__ RT rt_exp(RT x);
template <> __device__ __forceinline__ double rt_exp<double>(double x) { return exp_f64(x); }
// FP32: the hardware base-2 exponential of x log2(e)
template <> __device__ __forceinline__ float rt_exp<float>(float x) {
    return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}

template <typename RT> __device__ __forceinline__ const RT *mo_table(const DevSystem &S);
template <> __device__ __forceinline__ const double *mo_table<double>(const DevSystem &S) { return S.mo; }
template <> __device__ __forceinline__ const float *mo_table<float>(const DevSystem &S) { return S.mo_f; }

// Radial part of one shell at distance r: R, and with DERIV also R'/r and
// R'' + (2l+2) R'/r.  Slater R = sum_p c_p r^kn exp(-zeta_p r), so R'/R =
// kn/r - zeta; Gaussian R = sum_p c_p exp(-alpha_p r^2), so R'/r = -2 alpha R
// and R'' + (2l+2) R'/r = (4 alpha^2 r^2 - (4l+6) alpha) R.  The primitive
// coefficients carry the radial normalisation.
template <typename RT, bool DERIV>
__device__ __forceinline__ void shell_radial(const DevSystem &S, int p, int np, int l, int kn, RT r,
                                             RT r2, RT rinv, RT &Rv, RT &Rd, RT &Rl) {
    Rv = RT(0);
    Rd = RT(0);
    Rl = RT(0);
    if (S.basis == 0) {
        const RT fl = RT(2 * l + 2);
        RT rk = RT(1);
        for (int t = 0; t < kn; ++t) rk *= r;
        for (int q = 0; q < np; ++q) {
            const double2 pe = S.prims[p + q];
            const RT ex = RT(pe.x);
            const RT f = RT(pe.y) * rk * rt_exp<RT>(-ex * r);
            Rv += f;
            if (DERIV) {
                const RT g = RT(kn) * rinv - ex;
                Rd += f * g * rinv;
                Rl += f * (g * g - RT(kn) * rinv * rinv + fl * g * rinv);
            }
        }
    } else {
        const RT fl = RT(4 * l + 6);
        for (int q = 0; q < np; ++q) {
            const double2 pe = S.prims[p + q];
            const RT ex = RT(pe.x);
            const RT f = RT(pe.y) * rt_exp<RT>(-ex * r2);
            Rv += f;
            if (DERIV) {
                Rd -= RT(2) * ex * f;
                Rl += f * (RT(4) * ex * ex * r2 - fl * ex);
            }
        }
    }
}

// Pass 1: MO values phi_m(r_e) = sum_mu C[mu][m] chi_mu(r_e) of the lane's
// electron (Methods, AO and MO layers).  AO = P(x,y,z) R(r) with P a
// Cartesian monomial; angular normalisations are folded into the rows of C.
template <int NMO, typename RT>
__device__ __forceinline__ void mo_values(const DevSystem &S, double x0, double x1, double x2,
                                          RT (&phi)[NMO]) {
#pragma unroll
    for (int m = 0; m < NMO; ++m) phi[m] = RT(0);
    const RT *C = mo_table<RT>(S);
    int p = 0;
    const RT *crow = C;
    int atom = -1;
    RT dx = RT(0), dy = RT(0), dz = RT(0), r2 = RT(0), r = RT(0);
    for (int sh = 0; sh < S.n_shells; ++sh) {
        const int4 si = S.shells[sh];
        if (si.x != atom) {  // shells of one atom share the geometry
            atom = si.x;
            const double *A = S.atoms + 4 * atom;
            // displacement in FP64, cast afterwards
            dx = RT(x0 - A[0]);
            dy = RT(x1 - A[1]);
            dz = RT(x2 - A[2]);
            r2 = dx * dx + dy * dy + dz * dz;
            r = sqrt(r2);
        }
        RT Rv, Rd, Rl;
        shell_radial<RT, false>(S, p, si.w, si.y, si.z, r, r2, RT(0), Rv, Rd, Rl);
        p += si.w;
        const int nc = (si.y + 1) * (si.y + 2) / 2;
        for (int c = 0; c < nc; ++c) {
            RT P;
            if (si.y == 0) P = RT(1);
            else if (si.y == 1) P = c == 0 ? dx : (c == 1 ? dy : dz);
            else {
                const RT u = (c < 3) ? dx : (c < 5 ? dy : dz);
                const RT v = (c == 0) ? dx : (c == 1 || c == 3) ? dy : dz;
                P = u * v;
            }
            const RT val = P * Rv;
#pragma unroll
            for (int m = 0; m < NMO; ++m) phi[m] += val * crow[m];
            crow += S.nmo_pad;
        }
    }
}

// Pass 2: grad_e Sigma / Sigma and lap_e Sigma / Sigma.  With a_e[m] =
// d log Sigma / d phi_m(r_e) and t_mu = sum_m C[mu][m] a_e[m], both are
// sum_mu t_mu (grad, lap) chi_mu(r_e); for chi = P R:
//   grad chi = R grad P + P (R'/r) d,   lap chi = R lap P + P (R'' + (2l+2) R'/r).
// This contraction is the Jacobi trace: the weights t and the products
// t (grad, lap) chi are FP64 in every form; RT is the arithmetic of the AO
// derivative factors (FP32 in the mixed forms).
template <int NMO, typename RT>
__device__ __forceinline__ void sigma_derivs(const DevSystem &S, double x0, double x1, double x2,
                                             const double (&av)[NMO], double &g0, double &g1,
                                             double &g2, double &lap) {
    const double *C = S.mo;
    int p = 0;
    const double *crow = C;
    double G0 = 0.0, G1 = 0.0, G2 = 0.0, L = 0.0;
    int atom = -1;
    RT dx = RT(0), dy = RT(0), dz = RT(0), r2 = RT(0), r = RT(0), rinv = RT(0);
    for (int sh = 0; sh < S.n_shells; ++sh) {
        const int4 si = S.shells[sh];
        if (si.x != atom) {  // shells of one atom share the geometry
            atom = si.x;
            const double *A = S.atoms + 4 * atom;
            dx = RT(x0 - A[0]);
            dy = RT(x1 - A[1]);
            dz = RT(x2 - A[2]);
            r2 = dx * dx + dy * dy + dz * dz;
            r = sqrt(r2);
            rinv = RT(1) / r;
        }
        RT Rv, Rd, Rl;
        shell_radial<RT, true>(S, p, si.w, si.y, si.z, r, r2, rinv, Rv, Rd, Rl);
        p += si.w;
        const int nc = (si.y + 1) * (si.y + 2) / 2;
        for (int c = 0; c < nc; ++c) {
            double t = 0.0;
#pragma unroll
            for (int m = 0; m < NMO; ++m) t += crow[m] * av[m];
            crow += S.nmo_pad;
            // monomial, its gradient and Laplacian
            RT P, Px, Py, Pz, PL;
            if (si.y == 0) {
                P = RT(1); Px = Py = Pz = PL = RT(0);
            } else if (si.y == 1) {
                P = c == 0 ? dx : (c == 1 ? dy : dz);
                Px = c == 0 ? RT(1) : RT(0);
                Py = c == 1 ? RT(1) : RT(0);
                Pz = c == 2 ? RT(1) : RT(0);
                PL = RT(0);
            } else {
                // xx, xy, xz, yy, yz, zz
                const int iu = (c < 3) ? 0 : (c < 5 ? 1 : 2);
                const int iv = (c == 0) ? 0 : (c == 1 || c == 3) ? 1 : 2;
                const RT u = iu == 0 ? dx : (iu == 1 ? dy : dz);
                const RT v = iv == 0 ? dx : (iv == 1 ? dy : dz);
                P = u * v;
                Px = (iu == 0 ? v : RT(0)) + (iv == 0 ? u : RT(0));
                Py = (iu == 1 ? v : RT(0)) + (iv == 1 ? u : RT(0));
                Pz = (iu == 2 ? v : RT(0)) + (iv == 2 ? u : RT(0));
                PL = iu == iv ? RT(2) : RT(0);
            }
            const RT PRd = P * Rd;
            G0 += t * double(Rv * Px + PRd * dx);
            G1 += t * double(Rv * Py + PRd * dy);
            G2 += t * double(Rv * Pz + PRd * dz);
            L += t * double(Rv * PL + P * Rl);
        }
    }
    g0 = G0;
    g1 = G1;
    g2 = G2;
    lap = L;
}

// ---- BF16 matrix-core contractions (mixed form) ------------------------------
// A wave applies the fixed 32 x 32 matrix M = C^T (MO values from AO values)
// to one 32-vector per lane with v_mfma_f32_16x16x32_bf16:
// output tile t (16 rows of M) times the vectors of lane quarter q (16 lanes)
// is one MFMA.  Vectors are staged through LDS so that lane 16 g + j supplies
// elements 8 g .. 8 g + 7 of lane 16 q + j's vector; the 16 x 16 result lands
// as rows 4 g .. 4 g + 3 in lane 16 g + j and goes back through LDS to the
// lane that owns the vector.  SPLIT = 3 writes every operand as a sum of a
// high and a low BF16 part and forms hi*hi + hi*lo + lo*hi (about 16
// significant bits); SPLIT = 1 uses the high parts only.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));
constexpr int kStageK = 32;      // padded vector length
constexpr int kRowB = 40;        // bf16 per staged row (80 B, 16-byte aligned)
constexpr int kRowF = 36;        // floats per result row (144 B)
constexpr int kStageBytes = 2 * kWave * kRowB * 2 + kWave * kRowF * 4;

struct Stage {
    __bf16 *hi, *lo;  // [64][kRowB]
    float *out;       // [64][kRowF]
};

__device__ __forceinline__ Stage make_stage(void *base) {
    Stage st;
    st.hi = (__bf16 *)base;
    st.lo = st.hi + kWave * kRowB;
    st.out = (float *)(st.lo + kWave * kRowB);
    return st;
}

__device__ __forceinline__ void stage_put(const Stage &st, int lane, int k, float v) {
    const __bf16 h = (__bf16)v;
    st.hi[lane * kRowB + k] = h;
    st.lo[lane * kRowB + k] = (__bf16)(v - (float)h);
}

// out[lane][o] = sum_k M[o][k] v_lane[k] for o < 16 NT (M = matrix mat).
template <int NT, int SPLIT>
__device__ __forceinline__ void mfma_apply(const DevSystem &S, int mat, const Stage &st, int lane) {
    const int g = lane >> 4, j = lane & 15;
    bf16x8_t ahi[NT], alo[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const uint4 h = S.mfma_tab[((mat * 2 + t) * 2 + 0) * kWave + lane];
        const uint4 l = S.mfma_tab[((mat * 2 + t) * 2 + 1) * kWave + lane];
        ahi[t] = __builtin_bit_cast(bf16x8_t, h);
        alo[t] = __builtin_bit_cast(bf16x8_t, l);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int src = (16 * q + j) * kRowB + 8 * g;
        const bf16x8_t bh = *(const bf16x8_t *)(st.hi + src);
        const bf16x8_t bl = *(const bf16x8_t *)(st.lo + src);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[t], bh, acc, 0, 0, 0);
            if (SPLIT == 3) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[t], bl, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[t], bh, acc, 0, 0, 0);
            }
            *(floatx4_t *)(st.out + (16 * q + j) * kRowF + 16 * t + 4 * g) = acc;
        }
    }
}

// Pass 1 on the matrix cores: AO values in FP32, staged as BF16 parts, MO
// values phi[m] = sum_mu C[mu][m] chi_mu with FP32 accumulation.  Every lane
// of the wave must call it.
template <int NMO, int SPLIT>
__device__ __forceinline__ void mo_values_mfma(const DevSystem &S, int lane, void *stage_base, double x0,
                                               double x1, double x2, float (&phi)[NMO]) {
    const Stage st = make_stage(stage_base);
    int p = 0, mu = 0;
    int atom = -1;
    float dx = 0.f, dy = 0.f, dz = 0.f, r2 = 0.f, r = 0.f;
    for (int sh = 0; sh < S.n_shells; ++sh) {
        const int4 si = S.shells[sh];
        if (si.x != atom) {  // shells of one atom share the geometry
            atom = si.x;
            const double *A = S.atoms + 4 * atom;
            dx = float(x0 - A[0]);
            dy = float(x1 - A[1]);
            dz = float(x2 - A[2]);
            r2 = dx * dx + dy * dy + dz * dz;
            r = sqrtf(r2);
        }
        float Rv, Rd, Rl;
        shell_radial<float, false>(S, p, si.w, si.y, si.z, r, r2, 0.f, Rv, Rd, Rl);
        p += si.w;
        const int nc = (si.y + 1) * (si.y + 2) / 2;
        for (int c = 0; c < nc; ++c, ++mu) {
            float P;
            if (si.y == 0) P = 1.f;
            else if (si.y == 1) P = c == 0 ? dx : (c == 1 ? dy : dz);
            else {
                const float u = (c < 3) ? dx : (c < 5 ? dy : dz);
                const float v = (c == 0) ? dx : (c == 1 || c == 3) ? dy : dz;
                P = u * v;
            }
            stage_put(st, lane, mu, P * Rv);
        }
    }
    for (int k = mu; k < kStageK; ++k) stage_put(st, lane, k, 0.f);
    __syncthreads();
    mfma_apply<(NMO + 15) / 16, SPLIT>(S, 0, st, lane);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NMO; ++m) phi[m] = st.out[lane * kRowF + m];
    __syncthreads();
}

// LDS of one walker (doubles): T tables [2][nmax][cols] at 0 (nmax =
// max(n_up, n_dn)) and the cofactor tables [2][nmax][cregion] after them,
// both written from the determinant stage on.  FULL layout (the adjoint's):
// cols = NMO, the T rows holding A0^-1 in their reference columns.  Compact
// layout (the evaluation and Metropolis kernels'): only the columns from
// c0 = min(n_up, n_dn) on, the ones the ratios and cofactors read; A0^-1
// passes through the cofactor region (cregion = max(cols, nmax) per row)
// before the cofactors accumulate there.  Before the determinant stage the
// same space holds the e-e-n factor table (een_table doubles at 0, when
// e-e-n terms exist) and the positions [LW][3] + pivot rows [2][NMO] at
// pos_offset.
// Doubles of e-e-n geometry per lane and nucleus: r, the unit vector from
// the nucleus, 1 / r.
constexpr int kEenGeo = 5;

__host__ __device__ inline int een_table(const DevSystem &S) {
    return S.een_n > 0 ? S.LW * S.n_atoms * (2 * S.een_n + kEenGeo) : 0;
}

template <int NMO, bool FULL = true>
__host__ __device__ inline int tab_c0(const DevSystem &S) {
    return FULL ? 0 : (S.n_up < S.n_dn ? S.n_up : S.n_dn);
}

template <int NMO, bool FULL = true>
__host__ __device__ inline int tab_cols(const DevSystem &S) {
    return NMO - tab_c0<NMO, FULL>(S);
}

template <int NMO, bool FULL = true>
__host__ __device__ inline int tab_cregion(const DevSystem &S) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn, cols = tab_cols<NMO, FULL>(S);
    return FULL ? cols : (cols > nmax ? cols : nmax);
}

template <int NMO, bool FULL = true>
__host__ __device__ inline int pos_offset(const DevSystem &S) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int t = 2 * nmax * tab_cols<NMO, FULL>(S), f = een_table(S);
    return f > t ? f : t;
}

template <int NMO, bool FULL = true>
__host__ __device__ inline int walker_lds(const DevSystem &S) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int tc = 2 * nmax * (tab_cols<NMO, FULL>(S) + tab_cregion<NMO, FULL>(S));
    const int pp = pos_offset<NMO, FULL>(S) + 3 * S.LW + 2 * NMO;
    return tc > pp ? tc : pp;
}

// ---- Jastrow stage, generic in its scalar type ------------------------------
// The evaluation runs it on doubles; the adjoint runs it on Dual numbers
// (value and one directional derivative) to differentiate J, grad_e J and
// lap_e J with respect to a Jastrow parameter or a nuclear coordinate
// (forward mode).  Parameters come through an accessor: PlainPrm returns
// the system's values, SeedPrm the same values as Duals with derivative 1 on
// one chosen entry.
struct Dual {
    double v, d;
    __device__ Dual() : v(0.0), d(0.0) {}
    __device__ explicit Dual(double x) : v(x), d(0.0) {}
    __device__ Dual(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ __forceinline__ Dual operator/(double a, Dual b) {
    const double q = a / b.v;
    return Dual(q, -q * b.d / b.v);
}
__device__ __forceinline__ Dual &operator+=(Dual &a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual &operator-=(Dual &a, Dual b) { return a = a - b; }
using ::sqrt;  // the overload below must not hide the double one
__device__ __forceinline__ Dual sqrt(Dual a) {
    const double r = ::sqrt(a.v);
    return Dual(r, 0.5 * a.d / r);
}
__device__ __forceinline__ Dual rcp_ge1(Dual x) {
    const double y = rcp_ge1(x.v);
    return Dual(y, -x.d * y * y);
}
__device__ __forceinline__ double value_of(double x) { return x; }
__device__ __forceinline__ double value_of(Dual x) { return x.v; }

struct PlainPrm {
    const DevSystem &S;
    // which terms to evaluate (all of them)
    __device__ bool use_pade() const { return true; }
    __device__ bool use_en(int) const { return true; }
    __device__ bool use_een_term(int) const { return true; }
    __device__ bool use_een(int, int) const { return true; }  // term m, nucleus a
    __device__ double b() const { return S.b; }
    __device__ double R(int a, int k) const { return S.atoms[4 * a + k]; }
    __device__ double en(int a, int k) const { return S.jas_en[3 * a + k]; }
    __device__ double een(int m, int k) const { return S.jas_een[7 * m + k]; }
};

// Seeded entry: kind 0 the Pade b, 1 the e-n parameter (i, k), 2 the e-e-n
// parameter (i, k), 3 the coordinate k of nucleus i; -1 none.
struct SeedPrm {
    const DevSystem &S;
    int kind, i, k;
    // only the terms that depend on the seeded entry (the others have zero
    // derivative)
    __device__ bool use_pade() const { return kind == 0; }
    __device__ bool use_en(int a) const { return (kind == 1 || kind == 3) && a == i; }
    __device__ bool use_een_term(int m) const { return (kind == 2 && m == i) || kind == 3; }
    __device__ bool use_een(int m, int a) const { return (kind == 2 && m == i) || (kind == 3 && a == i); }
    __device__ Dual b() const { return Dual(S.b, kind == 0 ? 1.0 : 0.0); }
    __device__ Dual R(int a, int kk) const { return Dual(S.atoms[4 * a + kk], (kind == 3 && a == i && kk == k) ? 1.0 : 0.0); }
    __device__ Dual en(int a, int kk) const { return Dual(S.jas_en[3 * a + kk], (kind == 1 && a == i && kk == k) ? 1.0 : 0.0); }
    __device__ Dual een(int m, int kk) const { return Dual(S.jas_een[7 * m + kk], (kind == 2 && m == i && kk == k) ? 1.0 : 0.0); }
};

// The lane's e-e-n factor table: per nucleus a, [een_n][2] factor values
// f(a1, b1; u) and f(a2, b2; u) of its electron at u = r_a e, then [kEenGeo] the
// geometry (u, the unit vector from the nucleus, 1 / u).  T values, LDS.
template <typename T, typename Prm>
__device__ __forceinline__ void een_table_fill(const DevSystem &S, const Lane &L, double x0, double x1, double x2,
                                               T *sF, T *sG, const Prm &prm) {
    if (S.een_n == 0 || !L.active) return;
    for (int a = 0; a < S.n_atoms; ++a) {
        const T e0 = x0 - prm.R(a, 0), e1 = x1 - prm.R(a, 1), e2 = x2 - prm.R(a, 2);
        const T u = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        const T ui = 1.0 / u;
        T *g = sG + (L.lw * S.n_atoms + a) * kEenGeo;
        g[0] = u;
        g[1] = e0 * ui;
        g[2] = e1 * ui;
        g[3] = e2 * ui;
        g[4] = ui;
        T *f = sF + (L.lw * S.n_atoms + a) * 2 * S.een_n;
        for (int m = 0; m < S.een_n; ++m) {
            f[2 * m] = prm.een(m, 1) * u * rcp_ge1(1.0 + prm.een(m, 2) * u);
            f[2 * m + 1] = prm.een(m, 3) * u * rcp_ge1(1.0 + prm.een(m, 4) * u);
        }
    }
}

template <typename T>
struct JasTerms {
    T J, g0, g1, g2, lap;
    double vpot;  // Coulomb terms of the electron (evaluated when T is double)
};

// Jastrow factor (eq. jastrow: Pade e-e kernel of eq. pade_kernel, e-n and
// e-e-n kernels of the many-body appendix) of the lane's electron: its share
// of J, grad_e J and lap_e J; with T = double also its Coulomb terms
// (eq. Hmol: half of each e-e pair, the e-n attraction).  sPos holds the
// walker's positions, sF / sG the e-e-n tables of een_table_fill.  A seeded
// accessor skips the terms that do not depend on its entry.
template <typename T, typename Prm>
__device__ __forceinline__ JasTerms<T> jastrow_terms(const DevSystem &S, const Lane &L, double x0, double x1,
                                                     double x2, const double *sPos, const T *sF, const T *sG,
                                                     const Prm &prm) {
    constexpr bool kPlain = sizeof(T) == sizeof(double);
    JasTerms<T> o;
    o.J = T(0.0);
    o.g0 = T(0.0);
    o.g1 = T(0.0);
    o.g2 = T(0.0);
    o.lap = T(0.0);
    o.vpot = 0.0;
    if (!L.active) return o;
    const T b = prm.b();
    for (int j = 0; j < S.ne && prm.use_pade(); ++j) {
        if (j == L.e) continue;
        const int lj = j < S.n_up ? j : S.G + (j - S.n_up);
        const double d0 = x0 - sPos[3 * lj], d1 = x1 - sPos[3 * lj + 1], d2 = x2 - sPos[3 * lj + 2];
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const bool same = (j < S.n_up) == (L.e < S.n_up);
        const double a = same ? S.a_par : S.a_anti;
        // one division gives both 1/r and 1/(1 + b r)
        const T den = 1.0 + b * r;
        const T q = 1.0 / (r * den);
        const T rinv = q * den, dinv = q * r;
        const T k1 = a * dinv * dinv;                 // K'(r)
        const T k2 = -2.0 * a * b * dinv * dinv * dinv;  // K''(r)
        o.J += 0.5 * a * r * dinv;
        o.g0 += k1 * d0 * rinv;
        o.g1 += k1 * d1 * rinv;
        o.g2 += k1 * d2 * rinv;
        o.lap += k2 + 2.0 * k1 * rinv;
        if constexpr (kPlain) o.vpot += 0.5 * rinv;
    }
    for (int a = 0; a < S.n_atoms; ++a) {
        const T d0 = x0 - prm.R(a, 0), d1 = x1 - prm.R(a, 1), d2 = x2 - prm.R(a, 2);
        if constexpr (kPlain) o.vpot -= S.atoms[4 * a + 3] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (S.jas_en && prm.use_en(a)) {
            // e-n kernel K = N / D, N = w0 r + w1 r^2, D = 1 + w2 r:
            // K' = (N' - K D') / D and K'' = (N'' - 2 K' D') / D
            const T r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const T w0 = prm.en(a, 0), w1 = prm.en(a, 1), w2 = prm.en(a, 2);
            const T q = 1.0 / (1.0 + w2 * r), rinv = 1.0 / r;
            const T K = (w0 + w1 * r) * r * q;
            const T K1 = (w0 + 2.0 * w1 * r - K * w2) * q;
            const T K2 = (2.0 * w1 - 2.0 * K1 * w2) * q;
            o.J += K;
            o.g0 += K1 * d0 * rinv;
            o.g1 += K1 * d1 * rinv;
            o.g2 += K1 * d2 * rinv;
            o.lap += K2 + 2.0 * K1 * rinv;
        }
    }
    // e-e-n kernel: for the ordered pair (i, j), i > j, the term is
    // c f1(r_ai) f2(r_aj) f3(r_ij).  This electron takes the role of i
    // against lower-numbered partners and of j against higher ones; its
    // own factor carries the derivatives, the partner's factor is a value
    // from the table.  The pair's value is counted at i.
    for (int j = 0; j < S.ne && S.een_n > 0; ++j) {
        if (j == L.e) continue;
        const int lj = j < S.n_up ? j : S.G + (j - S.n_up);
        const bool first = L.e > j;
        const double d0 = x0 - sPos[3 * lj], d1 = x1 - sPos[3 * lj + 1], d2 = x2 - sPos[3 * lj + 2];
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double rinv = 1.0 / r;
        const double w0 = d0 * rinv, w1 = d1 * rinv, w2 = d2 * rinv;
        for (int m = 0; m < S.een_n; ++m) {
            if (!prm.use_een_term(m)) continue;
            const T a3 = prm.een(m, 5), b3 = prm.een(m, 6);
            const T q3 = rcp_ge1(1.0 + b3 * r);
            const T f3 = a3 * r * q3, f31 = a3 * q3 * q3, f32 = -2.0 * b3 * f31 * q3;
            const T ao = first ? prm.een(m, 1) : prm.een(m, 3), bo = first ? prm.een(m, 2) : prm.een(m, 4);
            const T cm = prm.een(m, 0);
            for (int a = 0; a < S.n_atoms; ++a) {
                if (!prm.use_een(m, a)) continue;
                const T *g = sG + (L.lw * S.n_atoms + a) * kEenGeo;
                const T u = g[0];
                const T qo = rcp_ge1(1.0 + bo * u);
                const T fo = ao * u * qo, fo1 = ao * qo * qo, fo2 = -2.0 * bo * fo1 * qo;
                const T cp = cm * sF[((lj * S.n_atoms + a) * S.een_n + m) * 2 + (first ? 1 : 0)];
                const T uw = g[1] * w0 + g[2] * w1 + g[3] * w2;
                if (first) o.J += cp * fo * f3;
                o.g0 += cp * (fo1 * f3 * g[1] + fo * f31 * w0);
                o.g1 += cp * (fo1 * f3 * g[2] + fo * f31 * w1);
                o.g2 += cp * (fo1 * f3 * g[3] + fo * f31 * w2);
                o.lap += cp * ((fo2 + 2.0 * fo1 * g[4]) * f3 + 2.0 * fo1 * f31 * uw + fo * (f32 + 2.0 * f31 * rinv));
            }
        }
    }
    return o;
}

// Per-lane results of the stages every evaluation shares.
template <int NMO>
struct Core {
    double J, gJ0, gJ1, gJ2, lapJ, vpot;  // this electron's Jastrow and Coulomb terms
    int slot;                             // Gauss-Jordan slot of this electron
    double Ssum, logD_up, logD_dn, sgn_up, sgn_dn;
    int sing_walker;                      // > 0: a reference matrix is exactly singular
    double av[NMO];                       // a_e[m] = d log Sigma / d phi_m(r_e)
    double bgS0, bgS1, bgS2, blap;        // backflow: grad_e Sigma / Sigma, lap Sigma / Sigma share
};

// Jastrow and Coulomb terms, pass 1 (MO values), in-place Gauss-Jordan of
// the reference matrices, determinant ratios, S, cofactor tables and the
// adjoint vector a_e.  Every lane of the block must call it (it contains
// block barriers).  On return the walker's LDS holds the T tables
// [2][nmax][NMO] at wsm and the cofactor tables right after them.
template <int NMO>
__device__ __forceinline__ void explicit_dets(const DevSystem &S, const Lane &L, double *wsm,
                                              const double (&phi)[NMO], Core<NMO> &c);

// Backflow: grad and Laplacian of Sigma of the backflow-transformed
// determinants (eq. nabla_d), every configuration explicitly.  Every lane of
// the block must call it.  sPos holds the walker's bare positions.
template <int NMO, bool LR, int CAP>
__device__ __forceinline__ void backflow_dets(const DevSystem &S, const Lane &L, double *wsm, const double *sPos,
                                              double x0, double x1, double x2, Core<NMO> &c);

template <int NMO, bool LR>
__host__ __device__ inline int bf_pos_offset(const DevSystem &S);

// PSI: stop once log|Psi| is known (no cofactor tables, no adjoint vector):
// the values a finite-difference kinetic energy needs.  RT is the arithmetic
// of the AO evaluation and MF the MO contraction of pass 1 (FP64 when RT is
// double).  FULLT: the full table layout (walker_lds<NMO, true>), which the
// adjoint reads; otherwise the compact one.
template <int NMO, typename RT, int MF = 0, bool EXPL = false, int BF = 0, bool PSI = false,
          bool FULLT = false>
__device__ __forceinline__ void core_stages(const DevSystem &S, const Lane &L, double *wsm, double &x0,
                                            double &x1, double &x2, Core<NMO> &c, void *stage = nullptr) {
    // the compact layout serves the low-rank Metropolis and evaluation
    // kernels (fewer LDS bytes per wave, more waves per CU)
    constexpr bool kFull = FULLT || EXPL || BF;
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int c0 = tab_c0<NMO, kFull>(S), ts = tab_cols<NMO, kFull>(S);
    const int tstride = nmax * ts;                           // doubles per spin T table
    const int cstride = nmax * tab_cregion<NMO, kFull>(S);   // doubles per spin cofactor table
    double *sT = wsm;                        // [2][nmax][ts]
    double *sC = sT + 2 * tstride;           // [2][nmax][cregion / nmax] after the elimination
    // [LW][3] before the elimination (with backflow: after the backflow tables)
    double *sPos = wsm + (BF ? bf_pos_offset<NMO, !EXPL>(S) : pos_offset<NMO, kFull>(S));
    double *sPiv = sPos + 3 * S.LW;          // [2][NMO] during it
    // e-e-n table before the elimination: per lane [n_atoms][een_n][2]
    // factor values (f1, f2) of its electron, then [n_atoms][kEenGeo] geometry
    // (r, unit vector from the nucleus)
    double *sF = wsm;
    double *sG = wsm + S.LW * S.n_atoms * 2 * S.een_n;
    double *Tg = sT + L.grp * tstride;
    double *Cg = sC + L.grp * cstride;
    double *piv_row = sPiv + L.grp * NMO;

    if (!L.active) {  // a far point keeps idle lanes finite
        x0 = 100.0;
        x1 = 100.0;
        x2 = 100.0;
    }
    sPos[3 * L.lw + 0] = x0;
    sPos[3 * L.lw + 1] = x1;
    sPos[3 * L.lw + 2] = x2;
    const PlainPrm prm{S};
    een_table_fill<double>(S, L, x0, x1, x2, sF, sG, prm);
    __syncthreads();

    // ---- Jastrow and Coulomb terms of this electron (FP64) ----------------
    const JasTerms<double> jt = jastrow_terms<double>(S, L, x0, x1, x2, sPos, sF, sG, prm);
    const double J = jt.J, gJ0 = jt.g0, gJ1 = jt.g1, gJ2 = jt.g2, lapJ = jt.lap, vpot = jt.vpot;

    c.J = J;
    c.gJ0 = gJ0;
    c.gJ1 = gJ1;
    c.gJ2 = gJ2;
    c.lapJ = lapJ;
    c.vpot = vpot;

    if constexpr (BF) {
        backflow_dets<NMO, !EXPL, (BF == 1 ? kSmallCfgBF : kMaxCfgBF)>(S, L, wsm, sPos, x0, x1, x2, c);
        return;
    }

    // ---- pass 1: MO values of this electron ------------------------------
    double a[NMO];
    if constexpr (sizeof(RT) == sizeof(double)) {
        double phi[NMO];
        mo_values<NMO, double>(S, x0, x1, x2, phi);
#pragma unroll
        for (int m = 0; m < NMO; ++m) a[m] = phi[m];
    } else if constexpr (MF > 0) {
        // the staging area overlays the walkers' tables: wait for the
        // position reads of the pair loop first
        __syncthreads();
        float phi[NMO];
        mo_values_mfma<NMO, MF>(S, L.lane, stage, x0, x1, x2, phi);
#pragma unroll
        for (int m = 0; m < NMO; ++m) a[m] = double(phi[m]);
    } else {
        RT phi[NMO];
        mo_values<NMO, RT>(S, x0, x1, x2, phi);
#pragma unroll
        for (int m = 0; m < NMO; ++m) a[m] = double(phi[m]);
    }
    if constexpr (EXPL) {
        explicit_dets<NMO>(S, L, wsm, a, c);
        return;
    }

    // ---- in-place Gauss-Jordan of the reference matrix across the group --
    // Row = this electron's MO values.  Pivot column j (reference orbital j
    // after the create-time column permutation) is overwritten by the
    // inverse, so at the end the row of slot s holds A0^-1[s][slot(e)] in
    // the columns < n and T[s][v] = (A0^-1 Phi)[s][v] in the virtual columns.
    constexpr int JMAX = kMaxSpin < NMO ? kMaxSpin : NMO;
    bool done = !L.active;
    int slot = -1;
    double dprod = 1.0;
    bool singular = false;
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
        if (j >= nmax) break;
        const bool work = j < L.nsig;
        double cand = (work && !done) ? fabs(a[j]) : -1.0;
        int cl = L.i;
        span_argmax(cand, cl, S.G);
        const bool ok = work && cand > 0.0;
        if (work && !ok) singular = true;
        const bool is_piv = ok && L.active && L.i == cl;
        if (is_piv) {
            // publish the unscaled pivot row, then scale this row in place
#pragma unroll
            for (int m = 0; m < NMO; ++m) piv_row[m] = a[m];
            const double inv = 1.0 / a[j];
#pragma unroll
            for (int m = 0; m < NMO; ++m) a[m] *= inv;
            a[j] = inv;
            done = true;
            slot = j;
        }
        __syncthreads();
        // the pivot from the published row (a column without one is zero)
        const double piv = ok ? piv_row[j] : 0.0;
        if (work) dprod *= piv;
        if (ok && L.active && !is_piv) {
            // multiplier as in Doolittle elimination: equal rows cancel exactly
            const double f = a[j] / piv;
#pragma unroll
            for (int m = 0; m < NMO; ++m) a[m] -= f * piv_row[m];
            a[j] = -f;
        }
        __syncthreads();
    }
    // compact layout: the reference part of each slot's row (A0^-1) goes
    // to the cofactor region for a moment, and each lane keeps its column
    double ainv[JMAX];
    if (L.active && slot >= 0) {
#pragma unroll
        for (int m = 0; m < NMO; ++m)
            if (m >= c0) Tg[slot * ts + m - c0] = a[m];
        if constexpr (!kFull) {
#pragma unroll
            for (int k = 0; k < JMAX; ++k)
                if (k < L.nsig) Cg[slot * nmax + k] = a[k];
        }
    }
    if constexpr (!kFull) {
        __syncthreads();
        const int sl = slot < 0 ? 0 : slot;
#pragma unroll
        for (int k = 0; k < JMAX; ++k) ainv[k] = (k < nmax && k < L.nsig && L.active) ? Cg[k * nmax + sl] : 0.0;
        __syncthreads();
    }
    // Permutation parity (slot s <- electron row): inversions within the group.
    int inv_cnt = 0;
    for (int ip = 0; ip < S.G; ++ip) {
        const int so = __shfl(slot, L.gbase + ip);
        if (L.active && ip > L.i && so >= 0 && so < slot) ++inv_cnt;
    }
    inv_cnt = span_sum_i(inv_cnt, S.G);
    const double det_sign = ((inv_cnt & 1) ? -1.0 : 1.0) * (dprod < 0.0 ? -1.0 : 1.0);
    const double det_log = log(fabs(dprod));
    // the shared region now becomes the cofactor tables: zero them
    for (int q = L.lw; q < 2 * cstride; q += S.LW) sC[q] = 0.0;
    __syncthreads();

    const int wb = L.lane - L.lw;
    const double logD_up = __shfl(det_log, wb), logD_dn = __shfl(det_log, wb + S.G);
    const double sgn_up = __shfl(det_sign, wb), sgn_dn = __shfl(det_sign, wb + S.G);
    const int sing_walker = walker_sum_i(singular ? 1 : 0, S.LW);

    // ---- S = sum_n d_n det T_up[H,P] det T_dn[H,P] ----------------------
    // records are loaded kRecBatch at a time so their latencies overlap
    const double *Tup = sT, *Tdn = sT + tstride;
    double Sp = 0.0;
    for (int i0 = 0; i0 < S.det_rows; i0 += kRecBatch) {
        uint4 rb[kRecBatch];
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u)
            rb[u] = i0 + u < S.det_rows ? S.det_recs[(i0 + u) * S.LW + L.lw] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) {
            const uint4 r = rb[u];
            Sp += __hiloint2double((int)r.y, (int)r.x) * ratio_code(Tup, r.z, ts, c0) * ratio_code(Tdn, r.w, ts, c0);
        }
    }
    const double Ssum = walker_sum(Sp, S.LW);
    if constexpr (PSI) {
        c.slot = slot;
        c.Ssum = Ssum;
        c.logD_up = logD_up;
        c.logD_dn = logD_dn;
        c.sgn_up = sgn_up;
        c.sgn_dn = sgn_dn;
        c.sing_walker = sing_walker;
        __syncthreads();  // the tables are reused by the next evaluation
        return;
    }

    // ---- cofactor tables C_sigma[k][v] = dS / dT_sigma[k][v] ---------------
    // each lane runs its own list of contributions (same length on every
    // lane) and writes an entry after its last contribution
    {
        double acc = 0.0;
        for (int i0 = 0; i0 < S.cof_rows; i0 += kRecBatch) {
            uint4 rb[kRecBatch];
#pragma unroll
            for (int u = 0; u < kRecBatch; ++u)
                rb[u] = i0 + u < S.cof_rows ? S.cof_recs[(i0 + u) * S.LW + L.lw] : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < kRecBatch; ++u) {
                const uint4 r = rb[u];  // an all-zero padding record adds 0 and never flushes
                const int spin = (r.w >> 1) & 1;
                const double *Ts = spin ? Tdn : Tup, *To = spin ? Tup : Tdn;
                const uint32_t cc = r.z >> 18;
                const double tv = Ts[((cc >> 2) & 7) * ts + (cc >> 5) - c0];
                const double cof = (cc & 3) == 0 ? 1.0 : ((cc & 3) == 1 ? tv : -tv);
                acc += __hiloint2double((int)r.y, (int)r.x) * ratio_code(To, r.z & 0x3FFFFu, ts, c0) * cof;
                if (r.w & 1u) {
                    sC[spin * cstride + ((r.w >> 2) & 7) * ts + (r.w >> 5) - c0] = acc;
                    acc = 0.0;
                }
            }
        }
    }
    __syncthreads();

    // ---- a_e = d log Sigma / d phi(r_e) ------------------------------------
    // virtual orbitals: a_e[v] = (A0^-T C)[e][v] / S (C vanishes on the
    // reference columns); reference orbitals: a_e[k] = A0^-1[k][e] -
    // sum_v T[k][v] a_e[v].
    double (&av)[NMO] = c.av;
    {
        if constexpr (kFull) {
            const int sl = slot < 0 ? 0 : slot;
#pragma unroll
            for (int k = 0; k < JMAX; ++k) {
                ainv[k] = 0.0;
                if (k < nmax) {
                    const double t = Tg[k * ts + sl];
                    ainv[k] = (k < L.nsig && L.active) ? t : 0.0;
                }
            }
        }
        const double Sinv = 1.0 / Ssum;
#pragma unroll
        for (int v = 0; v < NMO; ++v) av[v] = 0.0;
#pragma unroll
        for (int k = 0; k < JMAX; ++k) {
            if (k >= nmax) break;
#pragma unroll
            for (int v = 0; v < NMO; ++v)
                if (v >= c0) av[v] += ainv[k] * Cg[k * ts + v - c0];
        }
#pragma unroll
        for (int v = 0; v < NMO; ++v) av[v] *= Sinv;
        double h[JMAX];
#pragma unroll
        for (int k = 0; k < JMAX; ++k) {
            h[k] = 0.0;
            if (k < nmax) {
#pragma unroll
                for (int v = 0; v < NMO; ++v)
                    if (v >= c0) h[k] += Tg[k * ts + v - c0] * av[v];
            }
        }
#pragma unroll
        for (int k = 0; k < JMAX; ++k) av[k] = (k < L.nsig) ? ainv[k] - h[k] : av[k];
    }

    c.slot = slot;
    c.Ssum = Ssum;
    c.logD_up = logD_up;
    c.logD_dn = logD_dn;
    c.sgn_up = sgn_up;
    c.sgn_dn = sgn_dn;
    c.sing_walker = sing_walker;
}

// ---- explicit determinants (comparison method) ---------------------------
// Every distinct spin configuration c of the CI expansion is factorised on
// its own: A_c[e][k] = phi_{occ_c[k]}(r_e) (rows = electrons of the spin,
// columns = the configuration's orbital slots) by the same in-place
// Gauss-Jordan across the spin group as the reference matrix of the
// low-rank path.  Sigma = sum_n d_n D_up D_dn, and
// a_e[m] = d log Sigma / d phi_m(r_e) = sum_c W_c (A_c^-1)[k][e] for
// m = occ_c[k], W_c = (sum over the determinants using c of d_n D_other)
// D_c / Sigma.  This is the work the low-rank scheme of eq. table avoids:
// one factorisation per configuration instead of one per spin.

// LDS of one walker for the explicit method (doubles): MO rows [LW][NMO],
// adjoint rows [LW][NMO], per configuration (log|D|, sign, weight)
// [2][n_cfg_max][3], inverse table [2][kMaxSpin][kMaxSpin], pivot rows
// [2][kMaxSpin]; the Jastrow stage's tables and positions come first and
// are dead by then.
template <int NMO>
__host__ __device__ inline int walker_lds_explicit(const DevSystem &S) {
    const int ex = 2 * S.LW * NMO + 6 * S.n_cfg_max + 2 * kMaxSpin * kMaxSpin + 2 * kMaxSpin;
    const int js = pos_offset<NMO>(S) + 3 * S.LW;
    return ex > js ? ex : js;
}

__device__ __forceinline__ double walker_max(double v, int LW) { return span_max(v, LW); }

// In-place Gauss-Jordan of the group's n x n matrix held as one row per
// lane (a[k], k < n; entries beyond n are zero).  Pivot columns are
// overwritten by the inverse exactly as for the reference matrix; slot is
// the pivot step that consumed this lane's row.  Every lane of the block
// runs the same nmax steps (block barriers inside).
__device__ __forceinline__ void group_gauss_jordan(const DevSystem &S, const Lane &L, double (&a)[kMaxSpin],
                                                   int n, int nmax, bool live, double *piv_row, int &slot,
                                                   double &dprod, bool &singular) {
    bool done = !L.active || !live;
    slot = -1;
    dprod = 1.0;
    singular = false;
#pragma unroll
    for (int j = 0; j < kMaxSpin; ++j) {
        if (j >= nmax) break;
        const bool work = live && j < n;
        double cand = (work && !done) ? fabs(a[j]) : -1.0;
        int cl = L.i;
        span_argmax(cand, cl, S.G);
        const bool ok = work && cand > 0.0;
        if (work && !ok) singular = true;
        const bool is_piv = ok && L.active && L.i == cl;
        if (is_piv) {
#pragma unroll
            for (int m = 0; m < kMaxSpin; ++m) piv_row[m] = a[m];
            const double inv = 1.0 / a[j];
#pragma unroll
            for (int m = 0; m < kMaxSpin; ++m) a[m] *= inv;
            a[j] = inv;
            done = true;
            slot = j;
        }
        __syncthreads();
        const double piv = ok ? piv_row[j] : 0.0;
        if (work) dprod *= piv;
        if (ok && L.active && !is_piv) {
            const double f = a[j] / piv;
#pragma unroll
            for (int m = 0; m < kMaxSpin; ++m) a[m] -= f * piv_row[m];
            a[j] = -f;
        }
        __syncthreads();
    }
}

// Sign of the row permutation (slot s <- electron row) within the group.
__device__ __forceinline__ double group_parity(const DevSystem &S, const Lane &L, int slot) {
    int inv_cnt = 0;
    for (int ip = 0; ip < S.G; ++ip) {
        const int so = __shfl(slot, L.gbase + ip);
        if (L.active && ip > L.i && so >= 0 && so < slot) ++inv_cnt;
    }
    inv_cnt = span_sum_i(inv_cnt, S.G);
    return (inv_cnt & 1) ? -1.0 : 1.0;
}

template <int NMO>
__device__ __forceinline__ void explicit_dets(const DevSystem &S, const Lane &L, double *wsm,
                                              const double (&phi)[NMO], Core<NMO> &c) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    double *sPhi = wsm;                                   // [LW][NMO]
    double *sA = sPhi + S.LW * NMO;                       // [LW][NMO]
    double *sCfg = sA + S.LW * NMO;                       // [2][n_cfg_max][3]
    double *sInv = sCfg + 6 * S.n_cfg_max;                // [2][kMaxSpin][kMaxSpin]
    double *sPv = sInv + 2 * kMaxSpin * kMaxSpin;         // [2][kMaxSpin]
    double *inv_g = sInv + L.grp * kMaxSpin * kMaxSpin;
    double *piv_g = sPv + L.grp * kMaxSpin;
    double *cfg_g = sCfg + L.grp * S.n_cfg_max * 3;
    const int *occ_g = S.cfg_occ + L.grp * S.n_cfg_max * kMaxSpin;
    const int ncfg_g = L.grp == 0 ? S.n_cfg_up : S.n_cfg_dn;
    const int ncmax = S.n_cfg_up > S.n_cfg_dn ? S.n_cfg_up : S.n_cfg_dn;

    __syncthreads();  // the Jastrow stage's tables are no longer read
#pragma unroll
    for (int m = 0; m < NMO; ++m) {
        sPhi[L.lw * NMO + m] = phi[m];
        sA[L.lw * NMO + m] = 0.0;
    }
    __syncthreads();

    // pass A: log|D_c| and sign of every configuration of this spin
    for (int q = 0; q < ncmax; ++q) {
        const bool live = q < ncfg_g;
        const int *occ = occ_g + (live ? q : 0) * kMaxSpin;
        double a[kMaxSpin];
#pragma unroll
        for (int k = 0; k < kMaxSpin; ++k)
            a[k] = (L.active && live && k < L.nsig) ? sPhi[L.lw * NMO + occ[k]] : 0.0;
        int slot;
        double dprod;
        bool singular;
        group_gauss_jordan(S, L, a, L.nsig, nmax, live, piv_g, slot, dprod, singular);
        const double par = group_parity(S, L, slot);
        if (live && L.i == 0) {
            cfg_g[3 * q] = singular ? -INFINITY : log(fabs(dprod));
            cfg_g[3 * q + 1] = singular ? 0.0 : par * (dprod < 0.0 ? -1.0 : 1.0);
        }
    }
    __syncthreads();

    // common shifts, Sigma / (e^mu e^md)
    double mu = -INFINITY, md = -INFINITY;
    for (int q = L.lw; q < S.n_cfg_up; q += S.LW) mu = fmax(mu, sCfg[3 * q]);
    for (int q = L.lw; q < S.n_cfg_dn; q += S.LW) md = fmax(md, sCfg[3 * (S.n_cfg_max + q)]);
    mu = walker_max(mu, S.LW);
    md = walker_max(md, S.LW);
    const bool none = mu == -INFINITY || md == -INFINITY;
    double Sp = 0.0;
    if (!none)
        for (int n = L.lw; n < S.n_det_x; n += S.LW) {
            const int2 dc = S.det_cfg[n];
            const double *u = sCfg + 3 * dc.x, *v = sCfg + 3 * (S.n_cfg_max + dc.y);
            Sp += S.ci_x[n] * u[1] * v[1] * exp((u[0] - mu) + (v[0] - md));
        }
    const double Ssum = walker_sum(Sp, S.LW);
    const bool zero = none || Ssum == 0.0 || !isfinite(Ssum);

    // weights W_c (the lanes split both spins' configurations)
    for (int q = L.lw; q < S.n_cfg_up + S.n_cfg_dn; q += S.LW) {
        const int sp = q < S.n_cfg_up ? 0 : 1;
        const int cq = sp ? q - S.n_cfg_up : q;
        double *own = sCfg + 3 * (sp * S.n_cfg_max + cq);
        const double m_own = sp ? md : mu, m_oth = sp ? mu : md;
        double acc = 0.0;
        const int *off = S.cfg_off + sp * (S.n_cfg_max + 1);
        for (int t = off[cq]; t < off[cq + 1]; ++t) {
            const int2 e = S.cfg_use[t];
            const double *o = sCfg + 3 * ((1 - sp) * S.n_cfg_max + e.y);
            acc += S.ci_x[e.x] * o[1] * exp(o[0] - m_oth);
        }
        own[2] = zero ? 0.0 : acc * own[1] * exp(own[0] - m_own) / Ssum;
    }
    __syncthreads();

    // pass B: a_e accumulated from each weighted inverse
    for (int q = 0; q < ncmax; ++q) {
        const bool in = q < ncfg_g;
        const double wq = in ? cfg_g[3 * q + 2] : 0.0;
        const bool live = in && wq != 0.0;
        const int *occ = occ_g + (in ? q : 0) * kMaxSpin;
        double a[kMaxSpin];
#pragma unroll
        for (int k = 0; k < kMaxSpin; ++k)
            a[k] = (L.active && live && k < L.nsig) ? sPhi[L.lw * NMO + occ[k]] : 0.0;
        int slot;
        double dprod;
        bool singular;
        group_gauss_jordan(S, L, a, L.nsig, nmax, live, piv_g, slot, dprod, singular);
        if (live && L.active && slot >= 0) {
#pragma unroll
            for (int k = 0; k < kMaxSpin; ++k) inv_g[slot * kMaxSpin + k] = a[k];
        }
        __syncthreads();
        if (live && L.active && slot >= 0) {
            for (int k = 0; k < L.nsig; ++k) sA[L.lw * NMO + occ[k]] += wq * inv_g[k * kMaxSpin + slot];
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < NMO; ++m) c.av[m] = sA[L.lw * NMO + m];
    c.slot = -1;
    c.Ssum = Ssum;
    c.logD_up = mu;
    c.logD_dn = md;
    c.sgn_up = 1.0;
    c.sgn_dn = 1.0;
    c.sing_walker = zero ? 1 : 0;
}

}  // namespace walker
}  // namespace qmc

#include "qmc_backflow.h"
