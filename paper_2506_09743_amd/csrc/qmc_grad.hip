// Hand-written adjoint of log|Psi| and E_L (gfx950, FP64): derivatives with
// respect to the primitive exponents, the MO coefficients and the Jastrow
// parameters (Pade b; the e-n and e-e-n parameters of the many-body
// appendix when present) (Methods, eq. nabla_loss needs d log|Psi| / d theta),
// and with respect to the nuclear positions (Methods, eq. force needs
// d E_L / d R and d ln rho / d R = 2 d log|Psi| / d R).  The Jastrow part is
// differentiated in forward mode (Dual numbers through the Jastrow stage).
//
// With a_e[m] = d log Sigma / d phi_m(r_e) from the shared stages:
//   d log|Psi| / d theta = sum_e sum_mu t_mu d chi_mu(r_e) / d theta,
//   t_mu = sum_m C[mu][m] a_e[m]  (plus d J / d b for theta = b).
// The kinetic energy is E_kin = -1/2 sum_{e,m} a_e[m] B[e][m] + (Jastrow-only
// terms) with B = lap phi + 2 grad_e J . grad phi, so
//   d E_kin = -1/2 sum_{e,m} [adot_e[m] d phi[e][m] + a_e[m] d B[e][m]],
// where adot = (d^2 log Sigma / d phi d phi) B is the Hessian-vector product
// of log Sigma along B.  adot is the forward-mode derivative of the
// determinant algebra (Gauss-Jordan tables, determinant ratios, cofactors,
// a_e) in the direction phi -> phi + eps B:
//   Tdot = A0^-1 (B - B0 T),  Ainvdot = -A0^-1 B0 A0^-1,
//   rho_dot, Sdot, Cdot from the k <= 2 minors, and
//   adot_e[v] = (Ainvdot^T C + A0^-T Cdot)[e][v] / S - a_e[v] Sdot / S,
//   adot_e[k] = Ainvdot[k][e] - sum_v (Tdot[k][v] a_e[v] + T[k][v] adot_e[v]).
// Moving nucleus alpha moves its AOs: d chi(r - R) / d R = -grad chi, so the
// force terms need AO Hessians and gradients of AO Laplacians.

#include "qmc_walker.h"

namespace qmc {
namespace {

using namespace walker;

struct GradOut {
    double *dlogpsi;     // [W][P] or NULL
    double *deloc_dth;   // [W][P] or NULL
    double *dlogpsi_dR;  // [W][A][3] or NULL
    double *deloc_dR;    // [W][A][3] or NULL
    int n_param;
};

// Extra LDS doubles per walker beyond the evaluation's: three [2][nmax][NMO]
// tables (Tdot / Ainvdot, Cdot, slot-indexed B0 and Z rows), reused later
// for the per-electron rows of the MO-coefficient gradient, then positions
// and the per-atom accumulators.
// LDS of one walker in the gradient kernel (doubles).  The shared-stage
// tables (walker_lds, at 0) are followed by the forward-mode tables
// [3][2][n_max][NMO]; the Jastrow b-derivatives' positions [LW][3] come
// first in that same space (they are read before the shared stages).  Once
// a_e and its forward-mode derivative are in registers, all of it is dead
// and the per-electron rows [LW][2 n_ao + 2 NMO] (chi, beta, a, adot) take
// the block from 0.  The per-nucleus results [n_atoms][6] live past the end
// of both.
// After the MO-coefficient gradient the same block holds the walker's
// positions [LW][3] and the Dual e-e-n tables of the Jastrow directions
// (2 doubles per entry): [LW][n_atoms][2 een_n] factors, [LW][n_atoms][kEenGeo]
// geometry.
__host__ __device__ inline int grad_dual_size(const DevSystem &S) {
    return 3 * S.LW + 2 * S.LW * S.n_atoms * (2 * S.een_n + kEenGeo);
}

template <int NMO>
__host__ __device__ inline int grad_rows_end(const DevSystem &S) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int base = walker_lds<NMO>(S);
    const int fwd = base + 6 * nmax * NMO;
    const int rows = S.LW * (2 * S.n_ao + 2 * NMO);
    int e = fwd > rows ? fwd : rows;
    const int dual = grad_dual_size(S);
    return e > dual ? e : dual;
}

template <int NMO>
__host__ __device__ inline int grad_extra_lds(const DevSystem &S) {
    return grad_rows_end<NMO>(S) + 6 * S.n_atoms - walker_lds<NMO>(S);
}

// Derivative of the k <= 2 minor det T[H,P] along Tdot.
template <int NMO>
__device__ __forceinline__ double ratio_dot(const double *T, const double *Td, const int *d) {
    const int k = d[0];
    if (k == 0) return 0.0;
    const int a = d[1] * NMO + d[3];
    if (k == 1) return Td[a];
    const int b = d[2] * NMO + d[4], c = d[1] * NMO + d[4], e = d[2] * NMO + d[3];
    return Td[a] * T[b] + T[a] * Td[b] - Td[c] * T[e] - T[c] * Td[e];
}

// Monomial P of Cartesian component c of an l <= 2 shell, its gradient,
// Laplacian and Hessian (xx, yy, zz, xy, xz, yz).
struct Mono {
    double P, g[3], L, h[6];
};

__device__ __forceinline__ Mono monomial(int l, int c, double dx, double dy, double dz) {
    Mono m;
    const double d[3] = {dx, dy, dz};
    for (int k = 0; k < 3; ++k) m.g[k] = 0.0;
    for (int k = 0; k < 6; ++k) m.h[k] = 0.0;
    m.L = 0.0;
    if (l == 0) {
        m.P = 1.0;
    } else if (l == 1) {
        m.P = d[c];
        m.g[c] = 1.0;
    } else {
        const int iu = (c < 3) ? 0 : (c < 5 ? 1 : 2);
        const int iv = (c == 0) ? 0 : (c == 1 || c == 3) ? 1 : 2;
        m.P = d[iu] * d[iv];
        m.g[iu] += d[iv];
        m.g[iv] += d[iu];
        if (iu == iv) {
            m.L = 2.0;
            m.h[iu] = 2.0;
        } else {
            const int o = (iu + iv == 1) ? 3 : (iu + iv == 2 ? 4 : 5);  // xy, xz, yz
            m.h[o] = 1.0;
        }
    }
    return m;
}

// Radial sums of one shell: R, R'/r, R'' + (2l+2) R'/r, (R'' - R'/r) / r^2
// and (d/dr of the third) / r.
struct Radial {
    double v, d, l, dd, l1;
};

__device__ __forceinline__ Radial radial_full(const DevSystem &S, int p0, int np, int l, int kn, double r,
                                              double r2) {
    Radial R = {0, 0, 0, 0, 0};
    const double rinv = 1.0 / r;
    for (int q = 0; q < np; ++q) {
        const double2 pe = S.prims[p0 + q];
        const double ex = pe.x;
        if (S.basis == 0) {
            double f = pe.y * exp(-ex * r);
            for (int t = 0; t < kn; ++t) f *= r;
            const double g = kn * rinv - ex;
            const double L = g * g - kn * rinv * rinv + (2.0 * l + 2.0) * g * rinv;
            const double Lp = -2.0 * g * kn * rinv * rinv + 2.0 * kn * rinv * rinv * rinv +
                              (2.0 * l + 2.0) * (-kn * rinv * rinv * rinv - g * rinv * rinv);
            R.v += f;
            R.d += f * g * rinv;
            R.l += f * L;
            R.dd += f * (g * g - kn * rinv * rinv - g * rinv) * rinv * rinv;
            R.l1 += (f * g * L + f * Lp) * rinv;
        } else {
            const double f = pe.y * exp(-ex * r2);
            const double Q = 4.0 * ex * ex * r2 - (4.0 * l + 6.0) * ex;
            R.v += f;
            R.d += -2.0 * ex * f;
            R.l += f * Q;
            R.dd += 4.0 * ex * ex * f;
            R.l1 += f * (-2.0 * ex * Q + 8.0 * ex * ex);
        }
    }
    return R;
}

// RT: arithmetic of the forward evaluation's AO values and MO value
// contraction (double, or float for the mixed FP32 form); everything the
// adjoint adds is FP64.
template <int NMO, typename RT>
__global__ __launch_bounds__(kWave) void k_grad(DevSystem S, const double *__restrict__ X, int64_t W,
                                                GradOut G) {
    extern __shared__ double smem[];
    int64_t w;
    const Lane L = make_lane(S, (int64_t)blockIdx.x * S.WPW, W, &w);
    const int base_lds = walker_lds<NMO>(S);
    double *wsm = smem + L.wloc * (base_lds + grad_extra_lds<NMO>(S));
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int ts = nmax * NMO;                 // doubles per spin table
    double *sT = wsm;                          // T tables (shared stages)
    double *sC = wsm + 2 * ts;                 // cofactor tables (shared stages)
    double *gx = wsm + base_lds;               // gradient-only region
    double *sTD = gx, *sCD = gx + 2 * ts, *sZB = gx + 4 * ts;
    const int rows_len = 2 * S.n_ao + 2 * NMO;
    double *sRows = wsm;                       // after the forward-mode stage
    double *sAtom = wsm + grad_rows_end<NMO>(S);  // [n_atoms][6]: dlogpsi/dR, dE/dR

    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (L.active) {
        const double *p = X + (w * S.ne + L.e) * 3;
        x0 = p[0];
        x1 = p[1];
        x2 = p[2];
    }
    if (!L.active) {
        x0 = 100.0;
        x1 = 100.0;
        x2 = 100.0;
    }

    for (int q = L.lw; q < 6 * S.n_atoms; q += S.LW) sAtom[q] = 0.0;

    // ---- shared stages: MO values, Gauss-Jordan, determinants, a_e ----------
    Core<NMO> c;
    core_stages<NMO, RT, 0, false, false, false, true>(S, L, wsm, x0, x1, x2, c);
    const double gJ[3] = {c.gJ0, c.gJ1, c.gJ2};
    const double *Tg = sT + L.grp * ts;
    const double *Cg = sC + L.grp * ts;
    double *TDg = sTD + L.grp * ts;
    double *CDg = sCD + L.grp * ts;
    double *ZBg = sZB + L.grp * ts;
    const int sl = c.slot < 0 ? 0 : c.slot;

    // ---- direction B[e][m] = sum_mu C[mu][m] (lap chi + 2 grad J . grad chi) -
    double bvec[NMO];
#pragma unroll
    for (int m = 0; m < NMO; ++m) bvec[m] = 0.0;
    {
        int p = 0;
        const double *crow = S.mo;
        for (int sh = 0; sh < S.n_shells; ++sh) {
            const int4 si = S.shells[sh];
            const double *A = S.atoms + 4 * si.x;
            const double dx = x0 - A[0], dy = x1 - A[1], dz = x2 - A[2];
            const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
            const Radial R = radial_full(S, p, si.w, si.y, si.z, r, r2);
            p += si.w;
            const int nc = (si.y + 1) * (si.y + 2) / 2;
            for (int cc = 0; cc < nc; ++cc) {
                const Mono mn = monomial(si.y, cc, dx, dy, dz);
                const double gr[3] = {R.v * mn.g[0] + mn.P * R.d * dx, R.v * mn.g[1] + mn.P * R.d * dy,
                                      R.v * mn.g[2] + mn.P * R.d * dz};
                const double beta = R.v * mn.L + mn.P * R.l + 2.0 * (gJ[0] * gr[0] + gJ[1] * gr[1] + gJ[2] * gr[2]);
#pragma unroll
                for (int m = 0; m < NMO; ++m) bvec[m] += beta * crow[m];
                crow += S.nmo_pad;
            }
        }
    }

    // ---- forward mode of the determinant algebra along B -----------------
    // slot-indexed rows: reference columns hold B0 = B[e][k], virtual
    // columns hold Z[e][v] = B[e][v] - sum_k B[e][k] T[k][v]
    if (L.active && c.slot >= 0) {
#pragma unroll
        for (int v = 0; v < NMO; ++v) {
            double z = bvec[v];
            if (v >= L.nsig) {
#pragma unroll
                for (int k = 0; k < kMaxSpin; ++k)
                    if (k < L.nsig) z -= bvec[k < NMO ? k : 0] * Tg[k * NMO + v];
            }
            ZBg[c.slot * NMO + v] = z;
        }
    }
    for (int q = L.lw; q < 2 * ts; q += S.LW) sCD[q] = 0.0;
    __syncthreads();
    // row of this lane's slot: Tdot[s][v] = sum_s' Ainv[s][e(s')] Z[e(s')][v];
    // W[s][k] = (A0^-1 B0)[s][k]; Ainvdot[s][s''] = -sum_k W[s][k] Ainv[k][e(s'')]
    if (L.active && c.slot >= 0) {
        const int s = c.slot;
        double wk[kMaxSpin];
#pragma unroll
        for (int k = 0; k < kMaxSpin; ++k) {
            double acc = 0.0;
            if (k < L.nsig)
                for (int s2 = 0; s2 < L.nsig; ++s2) acc += Tg[s * NMO + s2] * ZBg[s2 * NMO + k];
            wk[k] = acc;
        }
#pragma unroll
        for (int v = 0; v < NMO; ++v) {
            double acc = 0.0;
            if (v >= L.nsig) {
                for (int s2 = 0; s2 < L.nsig; ++s2) acc += Tg[s * NMO + s2] * ZBg[s2 * NMO + v];
            } else {
#pragma unroll
                for (int k = 0; k < kMaxSpin; ++k)
                    if (k < L.nsig) acc -= wk[k] * Tg[k * NMO + v];
            }
            TDg[s * NMO + v] = acc;
        }
    }
    __syncthreads();
    const double *Tup = sT, *Tdn = sT + ts, *TDup = sTD, *TDdn = sTD + ts;
    double Sd = 0.0;
    if (L.wvalid) {
        for (int n = L.lw; n < S.n_det; n += S.LW) {
            const int *d = S.dets + n * kDetInts;
            const double ru = ratio<NMO>(Tup, d), rd = ratio<NMO>(Tdn, d + 5);
            Sd += S.ci[n] * (ratio_dot<NMO>(Tup, TDup, d) * rd + ru * ratio_dot<NMO>(Tdn, TDdn, d + 5));
        }
        for (int t = L.lw; t < S.n_entries; t += S.LW) {
            const int4 en = S.entries[t];
            const int end = S.entries[t + 1].w;
            const double *Ts = en.x == 0 ? Tup : Tdn, *TDs = en.x == 0 ? TDup : TDdn;
            const double *To = en.x == 0 ? Tdn : Tup, *TDo = en.x == 0 ? TDdn : TDup;
            const int oth = en.x == 0 ? 5 : 0;
            double val = 0.0;
            for (int q = en.w; q < end; ++q) {
                const int4 cb = S.contribs[q];
                const int *d = S.dets + cb.x * kDetInts;
                const double cof = cb.y == 0 ? 1.0 : double(cb.y) * Ts[cb.z * NMO + cb.w];
                const double cofd = cb.y == 0 ? 0.0 : double(cb.y) * TDs[cb.z * NMO + cb.w];
                val += S.ci[cb.x] * (ratio_dot<NMO>(To, TDo, d + oth) * cof + ratio<NMO>(To, d + oth) * cofd);
            }
            sCD[en.x * ts + en.y * NMO + en.z] = val;
        }
    }
    const double Sdot = walker_sum(Sd, S.LW);
    __syncthreads();

    double adot[NMO];
    {
        const double Sinv = 1.0 / c.Ssum;
        double ainv[kMaxSpin], ainvd[kMaxSpin];
#pragma unroll
        for (int k = 0; k < kMaxSpin; ++k) {
            ainv[k] = (k < L.nsig && L.active) ? Tg[k * NMO + sl] : 0.0;
            ainvd[k] = (k < L.nsig && L.active) ? TDg[k * NMO + sl] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < NMO; ++v) {
            double acc = 0.0;
            if (v >= L.nsig) {
#pragma unroll
                for (int k = 0; k < kMaxSpin; ++k)
                    if (k < L.nsig) acc += ainvd[k] * Cg[k * NMO + v] + ainv[k] * CDg[k * NMO + v];
                acc = (acc - c.av[v] * Sdot) * Sinv;
            }
            adot[v] = acc;
        }
#pragma unroll
        for (int k = 0; k < kMaxSpin; ++k) {
            if (k < L.nsig && k < NMO) {
                double h = 0.0;
#pragma unroll
                for (int v = 0; v < NMO; ++v)
                    if (v >= L.nsig) h += TDg[k * NMO + v] * c.av[v] + Tg[k * NMO + v] * adot[v];
                adot[k < NMO ? k : 0] = ainvd[k] - h;
            }
        }
    }
    __syncthreads();  // the table region becomes the per-electron rows below

    // ---- main gradient pass over the AOs ----------------------------------
    double *row = sRows + L.lw * rows_len;    // [chi | beta | a | adot]
    for (int q = 0; q < rows_len; ++q) row[q] = 0.0;
    double gS[3] = {0.0, 0.0, 0.0};
    {
        int p = 0, mu = 0;
        const double *crow = S.mo;
        for (int a = 0; a < S.n_atoms; ++a) {
            double lr[3] = {0.0, 0.0, 0.0}, er[3] = {0.0, 0.0, 0.0};
            p = 0;
            mu = 0;
            crow = S.mo;
            for (int sh = 0; sh < S.n_shells; ++sh) {
                const int4 si = S.shells[sh];
                const int nc = (si.y + 1) * (si.y + 2) / 2;
                if (si.x != a) {
                    p += si.w;
                    mu += nc;
                    crow += nc * S.nmo_pad;
                    continue;
                }
                const double *A = S.atoms + 4 * a;
                const double d[3] = {x0 - A[0], x1 - A[1], x2 - A[2]};
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], r = sqrt(r2);
                const Radial R = radial_full(S, p, si.w, si.y, si.z, r, r2);
                double A1 = 0.0, A2 = 0.0, A3 = 0.0;
                const double gd = gJ[0] * d[0] + gJ[1] * d[1] + gJ[2] * d[2];
                for (int cc = 0; cc < nc; ++cc, ++mu, crow += S.nmo_pad) {
                    const Mono mn = monomial(si.y, cc, d[0], d[1], d[2]);
                    double t = 0.0, td = 0.0;
#pragma unroll
                    for (int m = 0; m < NMO; ++m) {
                        t += crow[m] * c.av[m];
                        td += crow[m] * adot[m];
                    }
                    const double chi = mn.P * R.v;
                    double gr[3], hg[3], g3[3];
                    const double gP_gJ = mn.g[0] * gJ[0] + mn.g[1] * gJ[1] + mn.g[2] * gJ[2];
                    const double hP[3] = {mn.h[0] * gJ[0] + mn.h[3] * gJ[1] + mn.h[4] * gJ[2],
                                          mn.h[3] * gJ[0] + mn.h[1] * gJ[1] + mn.h[5] * gJ[2],
                                          mn.h[4] * gJ[0] + mn.h[5] * gJ[1] + mn.h[2] * gJ[2]};
                    for (int k = 0; k < 3; ++k) {
                        gr[k] = R.v * mn.g[k] + mn.P * R.d * d[k];
                        // (Hessian of chi) . grad J
                        hg[k] = R.v * hP[k] + mn.g[k] * R.d * gd + R.d * d[k] * gP_gJ +
                                mn.P * (R.d * gJ[k] + R.dd * d[k] * gd);
                        // gradient of lap chi
                        g3[k] = mn.L * R.d * d[k] + R.l * mn.g[k] + mn.P * R.l1 * d[k];
                    }
                    const double lap = R.v * mn.L + mn.P * R.l;
                    const double beta = lap + 2.0 * (gJ[0] * gr[0] + gJ[1] * gr[1] + gJ[2] * gr[2]);
                    if (L.active) {
                        for (int k = 0; k < 3; ++k) {
                            gS[k] += t * gr[k];
                            lr[k] -= t * gr[k];
                            er[k] += 0.5 * td * gr[k] + t * hg[k] + 0.5 * t * g3[k];
                        }
                        row[mu] = chi;
                        row[S.n_ao + mu] = beta;
                    }
                    A1 += td * mn.P;
                    A2 += t * (mn.L + 2.0 * gP_gJ);
                    A3 += t * mn.P;
                }
                // exponent derivatives of each primitive of this shell
                const double rinv = 1.0 / r;
                for (int q = 0; q < si.w; ++q) {
                    const double2 pe = S.prims[p + q];
                    const double ex = pe.x;
                    double fz, dRd, dRl;
                    if (S.basis == 0) {
                        const int nq = si.y + si.z + 1;
                        const double qn = S.normalize ? (nq + 0.5) / ex : 0.0;
                        double f = pe.y * exp(-ex * r);
                        for (int t2 = 0; t2 < si.z; ++t2) f *= r;
                        const double g = si.z * rinv - ex;
                        const double Lq = g * g - si.z * rinv * rinv + (2.0 * si.y + 2.0) * g * rinv;
                        fz = f * (qn - r);
                        dRd = (fz * g - f) * rinv;
                        dRl = fz * Lq + f * (-2.0 * g - (2.0 * si.y + 2.0) * rinv);
                    } else {
                        const double qn = S.normalize ? (0.75 + 0.5 * si.y) / ex : 0.0;
                        const double f = pe.y * exp(-ex * r2);
                        const double Q = 4.0 * ex * ex * r2 - (4.0 * si.y + 6.0) * ex;
                        fz = f * (qn - r2);
                        dRd = -2.0 * f - 2.0 * ex * fz;
                        dRl = fz * Q + f * (8.0 * ex * r2 - (4.0 * si.y + 6.0));
                    }
                    double gl = 0.0, ge = 0.0;
                    if (L.active) {
                        gl = fz * A3;
                        ge = -0.5 * (fz * (A1 + A2) + dRd * 2.0 * gd * A3 + dRl * A3);
                    }
                    gl = walker_sum(gl, S.LW);
                    ge = walker_sum(ge, S.LW);
                    if (L.wvalid && L.lw == 0) {
                        if (G.dlogpsi) G.dlogpsi[w * G.n_param + p + q] = gl;
                        if (G.deloc_dth) G.deloc_dth[w * G.n_param + p + q] = ge;
                    }
                }
                p += si.w;
            }
            // e-n attraction of this atom
            if (L.active) {
                const double *A = S.atoms + 4 * a;
                const double d[3] = {x0 - A[0], x1 - A[1], x2 - A[2]};
                const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                const double f = -A[3] / (rr * rr * rr);
                for (int k = 0; k < 3; ++k) er[k] += f * d[k];
            }
            for (int k = 0; k < 3; ++k) {
                lr[k] = walker_sum(lr[k], S.LW);
                er[k] = walker_sum(er[k], S.LW);
            }
            if (L.wvalid && L.lw == 0) {
                for (int k = 0; k < 3; ++k) {
                    sAtom[6 * a + k] = lr[k];
                    sAtom[6 * a + 3 + k] = er[k];
                }
            }
        }
    }
    // MO-coefficient gradient rows: a and adot of this electron
    if (L.active) {
#pragma unroll
        for (int m = 0; m < NMO; ++m) {
            row[2 * S.n_ao + m] = c.av[m];
            row[2 * S.n_ao + NMO + m] = adot[m];
        }
    }
    __syncthreads();

    if (L.wvalid) {
        // d/dC[mu][m]: sum over the walker's electrons (rows) of
        // chi_mu a[m] (log|Psi|) and -1/2 (adot[m] chi_mu + a[m] beta_mu) (E_L)
        const double *rows0 = sRows;
        const int nq = S.n_ao * S.n_mo;
        for (int q = L.lw; q < nq; q += S.LW) {
            const int mu = q / S.n_mo, m = q % S.n_mo;
            double gl = 0.0, ge = 0.0;
            for (int e = 0; e < S.LW; ++e) {
                const double *rw = rows0 + e * rows_len;
                gl += rw[mu] * rw[2 * S.n_ao + m];
                ge += rw[2 * S.n_ao + NMO + m] * rw[mu] + rw[2 * S.n_ao + m] * rw[S.n_ao + mu];
            }
            const int out = S.n_prim + mu * S.n_mo + S.mo_perm[m];
            const double f = S.ao_angf[mu];
            if (G.dlogpsi) G.dlogpsi[w * G.n_param + out] = f * gl;
            if (G.deloc_dth) G.deloc_dth[w * G.n_param + out] = -0.5 * f * ge;
        }
    }

    // ---- Jastrow parameters and the Jastrow part of the nuclear gradients ---
    // Forward mode over the Jastrow stage: each direction seeds one Jastrow
    // parameter (Pade b, e-n (w0, w1, w2) per nucleus, e-e-n (c, a1, b1, a2,
    // b2, a3, b3) per term) or, when the Jastrow depends on the nuclei, one
    // nuclear coordinate.  d log|Psi| = d J and
    // d E_L = -1/2 sum_e (d lap_e J + 2 grad_e J . d grad_e J + 2 d grad_e J . grad_e Sigma / Sigma).
    __syncthreads();  // the per-electron rows are no longer read
    {
        double *sP = wsm;                                   // [LW][3]
        Dual *dF = (Dual *)(wsm + 3 * S.LW);                // [LW][n_atoms][2 een_n]
        Dual *dG = dF + S.LW * S.n_atoms * 2 * S.een_n;     // [LW][n_atoms][kEenGeo]
        sP[3 * L.lw + 0] = x0;
        sP[3 * L.lw + 1] = x1;
        sP[3 * L.lw + 2] = x2;
        const int n_en = S.jas_en ? 3 * S.n_atoms : 0, n_een = 7 * S.een_n;
        const bool jas_R = (S.jas_en || S.een_n > 0) && (G.dlogpsi_dR || G.deloc_dR);
        const int n_dir = 1 + n_en + n_een + (jas_R ? 3 * S.n_atoms : 0);
        const int p_b = S.n_prim + S.n_ao * S.n_mo;        // output index of b
        for (int dir = 0; dir < n_dir; ++dir) {
            int kind, i, k, out;
            if (dir == 0) {
                kind = 0, i = 0, k = 0, out = p_b;
            } else if (dir <= n_en) {
                kind = 1, i = (dir - 1) / 3, k = (dir - 1) % 3, out = p_b + dir;
            } else if (dir <= n_en + n_een) {
                kind = 2, i = (dir - 1 - n_en) / 7, k = (dir - 1 - n_en) % 7, out = p_b + dir;
            } else {
                kind = 3, i = (dir - 1 - n_en - n_een) / 3, k = (dir - 1 - n_en - n_een) % 3, out = -1;
            }
            const SeedPrm sp{S, kind, i, k};
            een_table_fill<Dual>(S, L, x0, x1, x2, dF, dG, sp);
            __syncthreads();
            const JasTerms<Dual> jd = jastrow_terms<Dual>(S, L, x0, x1, x2, sP, dF, dG, sp);
            double dl = 0.0, de = 0.0;
            if (L.active) {
                dl = jd.J.d;
                de = -0.5 * (jd.lap.d + 2.0 * (gJ[0] * jd.g0.d + gJ[1] * jd.g1.d + gJ[2] * jd.g2.d) +
                             2.0 * (jd.g0.d * gS[0] + jd.g1.d * gS[1] + jd.g2.d * gS[2]));
            }
            dl = walker_sum(dl, S.LW);
            de = walker_sum(de, S.LW);
            if (L.wvalid && L.lw == 0) {
                if (out >= 0) {
                    if (G.dlogpsi) G.dlogpsi[w * G.n_param + out] = dl;
                    if (G.deloc_dth) G.deloc_dth[w * G.n_param + out] = de;
                } else {
                    sAtom[6 * i + k] += dl;
                    sAtom[6 * i + 3 + k] += de;
                }
            }
            __syncthreads();  // the tables are rewritten by the next direction
        }
    }
    if (L.wvalid && L.lw == 0) {
        // nuclear gradients, with the n-n repulsion
        for (int a = 0; a < S.n_atoms; ++a) {
            const double *A = S.atoms + 4 * a;
            double nn[3] = {0.0, 0.0, 0.0};
            for (int b2 = 0; b2 < S.n_atoms; ++b2) {
                if (b2 == a) continue;
                const double *B = S.atoms + 4 * b2;
                const double d[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
                const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                for (int k = 0; k < 3; ++k) nn[k] -= A[3] * B[3] * d[k] / (rr * rr * rr);
            }
            for (int k = 0; k < 3; ++k) {
                if (G.dlogpsi_dR) G.dlogpsi_dR[(w * S.n_atoms + a) * 3 + k] = sAtom[6 * a + k];
                if (G.deloc_dR) G.deloc_dR[(w * S.n_atoms + a) * 3 + k] = sAtom[6 * a + 3 + k] + nn[k];
            }
        }
    }
}

}  // namespace

template <int NMO>
static hipError_t launch_grad_t(const DevSystem &S, const double *X, int64_t W, const GradOut &G, bool mixed,
                                hipStream_t st) {
    const int64_t blocks = (W + S.WPW - 1) / S.WPW;
    const size_t lds =
        (size_t)S.WPW * (walker_lds<NMO>(S) + grad_extra_lds<NMO>(S)) * sizeof(double);
    if (mixed)
        hipLaunchKernelGGL((k_grad<NMO, float>), dim3((unsigned)blocks), dim3(kWave), lds, st, S, X, W, G);
    else
        hipLaunchKernelGGL((k_grad<NMO, double>), dim3((unsigned)blocks), dim3(kWave), lds, st, S, X, W, G);
    return hipGetLastError();
}

size_t grad_lds_bytes(const DevSystem &S) {
    int per = 0;
    switch (S.nmo_pad) {
#define QMC_LDS(N) \
    case N: per = walker_lds<N>(S) + grad_extra_lds<N>(S); break;
        QMC_LDS(4) QMC_LDS(8) QMC_LDS(12) QMC_LDS(16) QMC_LDS(20) QMC_LDS(24) QMC_LDS(32)
#undef QMC_LDS
    }
    return (size_t)S.WPW * per * sizeof(double);
}

hipError_t launch_grad(const DevSystem &S, const double *X, int64_t W, double *dlogpsi,
                       double *deloc_dth, double *dlogpsi_dR, double *deloc_dR, int n_param, bool mixed,
                       hipStream_t st) {
    GradOut G{dlogpsi, deloc_dth, dlogpsi_dR, deloc_dR, n_param};
    switch (S.nmo_pad) {
        case 4: return launch_grad_t<4>(S, X, W, G, mixed, st);
        case 8: return launch_grad_t<8>(S, X, W, G, mixed, st);
        case 12: return launch_grad_t<12>(S, X, W, G, mixed, st);
        case 16: return launch_grad_t<16>(S, X, W, G, mixed, st);
        case 20: return launch_grad_t<20>(S, X, W, G, mixed, st);
        case 24: return launch_grad_t<24>(S, X, W, G, mixed, st);
        case 32: return launch_grad_t<32>(S, X, W, G, mixed, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
