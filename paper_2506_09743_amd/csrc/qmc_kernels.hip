// HIP kernels (gfx950) for Slater-Jastrow VMC: local energy evaluation and
// all-electron Metropolis blocks.
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

#include "qmc_device.h"

#include <math.h>

namespace qmc {
namespace {

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m); }

// Sum over the LW lanes of a walker (LW a power of two, walkers aligned).
__device__ __forceinline__ double walker_sum(double v, int LW) {
    for (int off = 1; off < LW; off <<= 1) v += shfl_xor_d(v, off);
    return v;
}

__device__ __forceinline__ int walker_sum_i(int v, int LW) {
    for (int off = 1; off < LW; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

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

template <typename RT> __device__ __forceinline__ RT rt_exp(RT x);
template <> __device__ __forceinline__ double rt_exp<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float rt_exp<float>(float x) { return expf(x); }

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
    for (int sh = 0; sh < S.n_shells; ++sh) {
        const int4 si = S.shells[sh];
        const double *A = S.atoms + 4 * si.x;
        // displacement in FP64, cast afterwards
        const RT dx = RT(x0 - A[0]), dy = RT(x1 - A[1]), dz = RT(x2 - A[2]);
        const RT r2 = dx * dx + dy * dy + dz * dz;
        const RT r = sqrt(r2);
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
template <int NMO, typename RT>
__device__ __forceinline__ void sigma_derivs(const DevSystem &S, double x0, double x1, double x2,
                                             const double (&av)[NMO], double &g0, double &g1,
                                             double &g2, double &lap) {
    const RT *C = mo_table<RT>(S);
    RT a[NMO];
#pragma unroll
    for (int m = 0; m < NMO; ++m) a[m] = RT(av[m]);
    int p = 0;
    const RT *crow = C;
    double G0 = 0.0, G1 = 0.0, G2 = 0.0, L = 0.0;
    for (int sh = 0; sh < S.n_shells; ++sh) {
        const int4 si = S.shells[sh];
        const double *A = S.atoms + 4 * si.x;
        const RT dx = RT(x0 - A[0]), dy = RT(x1 - A[1]), dz = RT(x2 - A[2]);
        const RT r2 = dx * dx + dy * dy + dz * dz;
        const RT r = sqrt(r2);
        const RT rinv = RT(1) / r;
        RT Rv, Rd, Rl;
        shell_radial<RT, true>(S, p, si.w, si.y, si.z, r, r2, rinv, Rv, Rd, Rl);
        p += si.w;
        const int nc = (si.y + 1) * (si.y + 2) / 2;
        for (int c = 0; c < nc; ++c) {
            RT t = RT(0);
#pragma unroll
            for (int m = 0; m < NMO; ++m) t += crow[m] * a[m];
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
            G0 += double(t * (Rv * Px + PRd * dx));
            G1 += double(t * (Rv * Py + PRd * dy));
            G2 += double(t * (Rv * Pz + PRd * dz));
            L += double(t * (Rv * PL + P * Rl));
        }
    }
    g0 = G0;
    g1 = G1;
    g2 = G2;
    lap = L;
}

struct WalkerResult {
    double logpsi, sign, eloc;
};

// LDS of one walker: T tables [2][nmax][NMO] (nmax = max(n_up, n_dn)),
// then a region shared by the positions + pivot rows (before the
// determinant stage) and the cofactor tables [2][nmax][NMO] (after it).
template <int NMO>
__host__ __device__ inline int walker_lds(const DevSystem &S) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int t = 2 * nmax * NMO;
    const int a = 3 * S.LW + 2 * NMO;
    return t + (a > t ? a : t);
}

// Evaluates log|Psi|, sign and E_L of the lane's walker at the electron
// positions held by its lanes (x0, x1, x2 of the lane's electron).  Every
// lane of the block must call it (it contains block barriers); results are
// identical on all lanes of a walker.
template <int NMO, typename RT>
__device__ WalkerResult eval_walker(const DevSystem &S, const Lane &L, double *wsm, double x0,
                                    double x1, double x2) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int tstride = nmax * NMO;          // doubles per spin table
    double *sT = wsm;                        // [2][nmax][NMO]
    double *sX = sT + 2 * tstride;           // shared region
    double *sC = sX;                         // [2][nmax][NMO] after the elimination
    double *sPos = sX;                       // [LW][3] before it
    double *sPiv = sX + 3 * S.LW;            // [2][NMO] during it
    double *Tg = sT + L.grp * tstride;
    double *Cg = sC + L.grp * tstride;
    double *piv_row = sPiv + L.grp * NMO;

    if (!L.active) {  // a far point keeps idle lanes finite
        x0 = 100.0;
        x1 = 100.0;
        x2 = 100.0;
    }
    sPos[3 * L.lw + 0] = x0;
    sPos[3 * L.lw + 1] = x1;
    sPos[3 * L.lw + 2] = x2;
    __syncthreads();

    // ---- Pade e-e Jastrow and Coulomb terms of this electron -------------
    double J = 0.0, gJ0 = 0.0, gJ1 = 0.0, gJ2 = 0.0, lapJ = 0.0, vpot = 0.0;
    if (L.active) {
        for (int j = 0; j < S.ne; ++j) {
            if (j == L.e) continue;
            const int lj = j < S.n_up ? j : S.G + (j - S.n_up);
            const double d0 = x0 - sPos[3 * lj], d1 = x1 - sPos[3 * lj + 1], d2 = x2 - sPos[3 * lj + 2];
            const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const bool same = (j < S.n_up) == (L.e < S.n_up);
            const double a = same ? S.a_par : S.a_anti;
            // one division gives both 1/r and 1/(1 + b r)
            const double den = 1.0 + S.b * r;
            const double q = 1.0 / (r * den);
            const double rinv = q * den, dinv = q * r;
            const double k1 = a * dinv * dinv;                      // K'(r)
            const double k2 = -2.0 * a * S.b * dinv * dinv * dinv;  // K''(r)
            J += 0.5 * a * r * dinv;
            gJ0 += k1 * d0 * rinv;
            gJ1 += k1 * d1 * rinv;
            gJ2 += k1 * d2 * rinv;
            lapJ += k2 + 2.0 * k1 * rinv;
            vpot += 0.5 * rinv;
        }
        for (int a = 0; a < S.n_atoms; ++a) {
            const double *A = S.atoms + 4 * a;
            const double d0 = x0 - A[0], d1 = x1 - A[1], d2 = x2 - A[2];
            vpot -= A[3] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
    }

    // ---- pass 1: MO values of this electron ------------------------------
    double a[NMO];
    {
        RT phi[NMO];
        mo_values<NMO, RT>(S, x0, x1, x2, phi);
#pragma unroll
        for (int m = 0; m < NMO; ++m) a[m] = double(phi[m]);
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
        for (int off = 1; off < S.G; off <<= 1) {
            const double oc = shfl_xor_d(cand, off);
            const int ol = __shfl_xor(cl, off);
            if (oc > cand || (oc == cand && ol < cl)) {
                cand = oc;
                cl = ol;
            }
        }
        const double piv = __shfl(a[j], L.gbase + cl);
        const bool ok = work && cand > 0.0;
        if (work && !ok) singular = true;
        const bool is_piv = ok && L.active && L.i == cl;
        if (is_piv) {
            // publish the unscaled pivot row, then scale this row in place
#pragma unroll
            for (int m = 0; m < NMO; ++m) piv_row[m] = a[m];
            const double inv = 1.0 / piv;
#pragma unroll
            for (int m = 0; m < NMO; ++m) a[m] *= inv;
            a[j] = inv;
            done = true;
            slot = j;
        }
        if (work) dprod *= piv;
        __syncthreads();
        if (ok && L.active && !is_piv) {
            // multiplier as in Doolittle elimination: equal rows cancel exactly
            const double f = a[j] / piv;
#pragma unroll
            for (int m = 0; m < NMO; ++m) a[m] -= f * piv_row[m];
            a[j] = -f;
        }
        __syncthreads();
    }
    if (L.active && slot >= 0) {
#pragma unroll
        for (int m = 0; m < NMO; ++m) Tg[slot * NMO + m] = a[m];
    }
    // Permutation parity (slot s <- electron row): inversions within the group.
    int inv_cnt = 0;
    for (int ip = 0; ip < S.G; ++ip) {
        const int so = __shfl(slot, L.gbase + ip);
        if (L.active && ip > L.i && so >= 0 && so < slot) ++inv_cnt;
    }
    for (int off = 1; off < S.G; off <<= 1) inv_cnt += __shfl_xor(inv_cnt, off);
    const double det_sign = ((inv_cnt & 1) ? -1.0 : 1.0) * (dprod < 0.0 ? -1.0 : 1.0);
    const double det_log = log(fabs(dprod));
    // the shared region now becomes the cofactor tables: zero them
    for (int q = L.lw; q < 2 * tstride; q += S.LW) sC[q] = 0.0;
    __syncthreads();

    const int wb = L.lane - L.lw;
    const double logD_up = __shfl(det_log, wb), logD_dn = __shfl(det_log, wb + S.G);
    const double sgn_up = __shfl(det_sign, wb), sgn_dn = __shfl(det_sign, wb + S.G);
    const int sing_walker = walker_sum_i(singular ? 1 : 0, S.LW);

    // ---- S = sum_n d_n det T_up[H,P] det T_dn[H,P] ----------------------
    const double *Tup = sT, *Tdn = sT + tstride;
    double Sp = 0.0;
    if (L.wvalid) {
        for (int n = L.lw; n < S.n_det; n += S.LW) {
            const int *d = S.dets + n * kDetInts;
            Sp += S.ci[n] * ratio<NMO>(Tup, d) * ratio<NMO>(Tdn, d + 5);
        }
    }
    const double Ssum = walker_sum(Sp, S.LW);

    // ---- cofactor tables C_sigma[k][v] = dS / dT_sigma[k][v] ---------------
    if (L.wvalid) {
        for (int t = L.lw; t < S.n_entries; t += S.LW) {
            const int4 en = S.entries[t];
            const int end = S.entries[t + 1].w;
            const double *Ts = en.x == 0 ? Tup : Tdn;
            const double *To = en.x == 0 ? Tdn : Tup;
            const int oth = en.x == 0 ? 5 : 0;
            double val = 0.0;
            for (int c = en.w; c < end; ++c) {
                const int4 cb = S.contribs[c];
                const int *d = S.dets + cb.x * kDetInts;
                const double cof = cb.y == 0 ? 1.0 : double(cb.y) * Ts[cb.z * NMO + cb.w];
                val += S.ci[cb.x] * ratio<NMO>(To, d + oth) * cof;
            }
            sC[en.x * tstride + en.y * NMO + en.z] = val;
        }
    }
    __syncthreads();

    // ---- a_e = d log Sigma / d phi(r_e) ------------------------------------
    // virtual orbitals: a_e[v] = (A0^-T C)[e][v] / S (C vanishes on the
    // reference columns); reference orbitals: a_e[k] = A0^-1[k][e] -
    // sum_v T[k][v] a_e[v].
    double av[NMO];
    {
        const int sl = slot < 0 ? 0 : slot;
        double ainv[JMAX];
#pragma unroll
        for (int k = 0; k < JMAX; ++k) {
            ainv[k] = 0.0;
            if (k < nmax) {
                const double t = Tg[k * NMO + sl];
                ainv[k] = (k < L.nsig && L.active) ? t : 0.0;
            }
        }
        const double Sinv = 1.0 / Ssum;
#pragma unroll
        for (int v = 0; v < NMO; ++v) av[v] = 0.0;
#pragma unroll
        for (int k = 0; k < JMAX; ++k) {
            if (k >= nmax) break;
#pragma unroll
            for (int v = 0; v < NMO; ++v) av[v] += ainv[k] * Cg[k * NMO + v];
        }
#pragma unroll
        for (int v = 0; v < NMO; ++v) av[v] *= Sinv;
        double h[JMAX];
#pragma unroll
        for (int k = 0; k < JMAX; ++k) {
            h[k] = 0.0;
            if (k < nmax) {
#pragma unroll
                for (int v = 0; v < NMO; ++v) h[k] += Tg[k * NMO + v] * av[v];
            }
        }
#pragma unroll
        for (int k = 0; k < JMAX; ++k) av[k] = (k < L.nsig) ? ainv[k] - h[k] : av[k];
    }

    // ---- pass 2: grad and Laplacian of Sigma at this electron ---------------
    double gS0, gS1, gS2, lapS;
    sigma_derivs<NMO, RT>(S, x0, x1, x2, av, gS0, gS1, gS2, lapS);

    // ---- local energy and log|Psi| ------------------------------------------
    double part = 0.0;
    if (L.active) {
        const double kin = lapS + lapJ + gJ0 * gJ0 + gJ1 * gJ1 + gJ2 * gJ2 +
                           2.0 * (gJ0 * gS0 + gJ1 * gS1 + gJ2 * gS2);
        part = -0.5 * kin + vpot;
    }
    const double eloc = walker_sum(part, S.LW) + S.vnn;
    const double Jw = walker_sum(J, S.LW);
    WalkerResult res;
    if (sing_walker > 0 || Ssum == 0.0 || !L.wvalid) {
        res.logpsi = -INFINITY;
        res.sign = 0.0;
        res.eloc = NAN;
    } else {
        res.logpsi = Jw + logD_up + logD_dn + log(fabs(Ssum));
        res.sign = sgn_up * sgn_dn * (Ssum < 0.0 ? -1.0 : 1.0);
        res.eloc = eloc;
    }
    __syncthreads();  // LDS is reused by the next evaluation
    return res;
}

template <int NMO, typename RT>
__global__ __launch_bounds__(kWave) void k_eval(DevSystem S, const double *__restrict__ X, int64_t W,
                                                 double *__restrict__ LP, double *__restrict__ SG,
                                                 double *__restrict__ EL) {
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
    const WalkerResult r = eval_walker<NMO, RT>(S, L, wsm, x0, x1, x2);
    if (L.wvalid && L.lw == 0) {
        LP[w] = r.logpsi;
        SG[w] = r.sign;
        EL[w] = r.eloc;
    }
}

template <int NMO, typename RT>
__global__ __launch_bounds__(kWave) void k_metropolis(DevSystem S, double *__restrict__ X,
                                                      double *__restrict__ LP, double *__restrict__ SG,
                                                      double *__restrict__ EL, int64_t W, int n_steps,
                                                      double sigma, uint64_t seed, uint64_t step0,
                                                      uint32_t walker_offset, double *__restrict__ ACC) {
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
    for (int t = 0; t < n_steps; ++t) {
        const uint64_t step = step0 + (uint64_t)t;
        uint32_t c[4] = {wid, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)L.e};
        philox4x32_10(c, k0, k1);
        const double u0 = ((double)c[0] + 0.5) * s32, u1 = ((double)c[1] + 0.5) * s32;
        const double u2 = ((double)c[2] + 0.5) * s32, u3 = ((double)c[3] + 0.5) * s32;
        const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
        double s1, c1;
        sincos(two_pi * u1, &s1, &c1);
        const double z0 = r0 * c1, z1 = r0 * s1;
        const double z2 = r1 * cos(two_pi * u3);
        // no FMA contraction: X + sigma z rounds the product, then the sum
        const double y0 = __dadd_rn(x0, __dmul_rn(sigma, z0));
        const double y1 = __dadd_rn(x1, __dmul_rn(sigma, z1));
        const double y2 = __dadd_rn(x2, __dmul_rn(sigma, z2));
        uint32_t ca[4] = {wid, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)S.ne};
        philox4x32_10(ca, k0, k1);
        const uint64_t bits = ((((uint64_t)ca[0]) << 32) | (uint64_t)ca[1]) >> 11;
        const double u = (double)bits * (1.0 / 9007199254740992.0);

        const WalkerResult r = eval_walker<NMO, RT>(S, L, wsm, y0, y1, y2);
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

}  // namespace

// ---- launch dispatch ---------------------------------------------------------

static int nmo_bucket(int n_mo) {
    const int b[] = {4, 8, 12, 16, 20, 24, 32};
    for (int v : b)
        if (n_mo <= v) return v;
    return -1;
}

int padded_mo(int n_mo) { return nmo_bucket(n_mo); }

template <int NMO, typename RT>
static hipError_t launch_t(bool mc, const DevSystem &S, double *X, double *LP, double *SG, double *EL,
                           int64_t W, int n_steps, double sigma, uint64_t seed, uint64_t step0,
                           uint32_t woff, double *ACC, hipStream_t st) {
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    const size_t lds = (size_t)S.WPW * walker_lds<NMO>(S) * sizeof(double);
    if (mc)
        hipLaunchKernelGGL((k_metropolis<NMO, RT>), dim3((unsigned)blocks), dim3(kWave), lds, st, S, X,
                           LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC);
    else
        hipLaunchKernelGGL((k_eval<NMO, RT>), dim3((unsigned)blocks), dim3(kWave), lds, st, S,
                           (const double *)X, W, LP, SG, EL);
    return hipGetLastError();
}

template <typename RT>
static hipError_t launch_rt(bool mc, const DevSystem &S, double *X, double *LP, double *SG,
                            double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                            uint64_t step0, uint32_t woff, double *ACC, hipStream_t st) {
    switch (S.nmo_pad) {
#define QMC_CASE(N) \
    case N: return launch_t<N, RT>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
        QMC_CASE(4) QMC_CASE(8) QMC_CASE(12) QMC_CASE(16) QMC_CASE(20) QMC_CASE(24) QMC_CASE(32)
#undef QMC_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_walkers(bool mc, bool fp32, const DevSystem &S, double *X, double *LP, double *SG,
                          double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                          uint64_t step0, uint32_t woff, double *ACC, hipStream_t st) {
    if (fp32)
        return launch_rt<float>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
    return launch_rt<double>(mc, S, X, LP, SG, EL, W, n_steps, sigma, seed, step0, woff, ACC, st);
}

}  // namespace qmc
