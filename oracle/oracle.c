/*
 * FP64 CPU oracle for Slater-Jastrow VMC.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg, never by the product path.  Shares no
 * code with the HIP library.
 *
 * What it computes, with the paper passage each part follows:
 *   - Hamiltonian: kinetic -1/2 sum_i lap_i, e-e repulsion, e-n attraction,
 *     n-n repulsion (Introduction, eq. Hmol), atomic units.
 *   - Wavefunction Psi = exp(J) * sum_n d_n D_n^up D_n^dn (Methods, eq. psimol).
 *     Without backflow the orbitals see the bare electron positions; with
 *     the inverse backflow (Methods, backflow transformation; kernel
 *     omega / r_ij of the Results section) they see q_i = r_i + sum_{j != i}
 *     (omega / r_ij) (r_i - r_j), every determinant depends on every
 *     electron, and its diagonal Hessian follows eq. nabla_d, evaluated
 *     coordinate by coordinate with dA and d2A from the chain rule through
 *     q(r) (AO Hessians included).  The Jastrow factor and the potential
 *     keep the bare positions.
 *   - Slater AOs N x^kx y^ky z^kz r^kn exp(-zeta r) (Methods, AO layer) and
 *     contracted Cartesian Gaussians; closed-form gradient and Laplacian.
 *   - MOs phi_k = sum_mu C[mu][k] chi_mu (Methods, MO layer; C = c*mu).
 *   - Every determinant explicitly: matrix A[i][k] = phi_{occ[k]}(r_i) (rows
 *     electrons, columns orbital slots), LU with partial pivoting, explicit
 *     inverse; grad log D from the Jacobi formula Tr(A^-1 dA) and lap D / D =
 *     Tr(A^-1 lap A) (Appendix on the single-determinant simplification,
 *     eq. claudia_trace); grad Sigma and lap Sigma from eqs. nabla_sigma and
 *     delta_sigma, whose cross term vanishes without backflow because the up
 *     and down determinants depend on disjoint electrons, and is kept with
 *     it.
 *   - Pade e-e Jastrow K = a r / (1 + b r), a = 1/4 parallel, 1/2
 *     antiparallel (Appendix on additional ansatze, eq. pade_kernel), summed
 *     over pairs i<j (eq. jastrow, e-e term); optionally the many-body
 *     terms of eq. jastrow with the kernels of the appendix's many-body
 *     Jastrow subsection: the e-n kernel (w0 r + w1 r^2) / (1 + w2 r) per
 *     nucleus and the e-e-n kernel sum_mu c_mu f1 f2 f3 over nuclei and
 *     ordered pairs i > j.
 *   - Kinetic split lap Psi / Psi = lap J + |grad J|^2 + 2 grad J . grad
 *     Sigma / Sigma + lap Sigma / Sigma (Appendix on local energies, with the
 *     Jastrow factor written as exp(J)).
 *   - Metropolis sampling with all electrons moved at once by a normal
 *     proposal (Appendix on optimisation parameters, Sampling paragraph);
 *     random numbers from Philox4x32-10 (Salmon et al., SC'11) and the
 *     Box-Muller transform (1958).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_TWO_PI 6.283185307179586

static int n_cart(int l) { return (l + 1) * (l + 2) / 2; }

int or_n_ao(const or_system *s) {
    int n = 0;
    for (int i = 0; i < s->n_shells; ++i) n += n_cart(s->shell_l[i]);
    return n;
}

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* n!! with (-1)!! = 0!! = 1 */
static double dfactorial(int n) {
    double f = 1.0;
    for (int i = n; i > 1; i -= 2) f *= i;
    return f;
}

/* x^n for integer n >= 0; 0 for n < 0 (so that n x^(n-1) vanishes at n = 0). */
static double ipow(double x, int n) {
    if (n < 0) return 0.0;
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* Radial factor of a primitive's normalisation, so that the full primitive
   x^a y^b z^c R(r) has unit norm over R^3 once multiplied by ang_norm(). */
static double rad_norm(const or_system *s, int l, int kn, double e) {
    if (!s->normalize) return 1.0;
    if (s->basis == 0) {
        int n = l + kn + 1;
        return sqrt(pow(2.0 * e, 2 * n + 1) / factorial(2 * n)) *
               sqrt(dfactorial(2 * l + 1) / (4.0 * OR_PI));
    }
    return pow(2.0 * e / OR_PI, 0.75) * pow(4.0 * e, 0.5 * l);
}

static double ang_norm(const or_system *s, int a, int b, int c) {
    if (!s->normalize) return 1.0;
    return 1.0 / sqrt(dfactorial(2 * a - 1) * dfactorial(2 * b - 1) * dfactorial(2 * c - 1));
}

/* AO value, gradient and Laplacian at point r.  For AO = f P(x,y,z) R(r) with
   P a monomial of degree l:
     grad AO = f (R grad P + P (R'/r) d)
     lap AO  = f (R lap P + P (R'' + (2l + 2) R'/r))
   using d . grad P = l P.  out[n_ao][5]. */
void or_ao(const or_system *s, const double r[3], double *out) {
    int mu = 0, p0 = 0;
    for (int sh = 0; sh < s->n_shells; ++sh) {
        const int at = s->shell_atom[sh], l = s->shell_l[sh], kn = s->shell_kn[sh];
        const int np = s->shell_nprim[sh];
        const double d[3] = {r[0] - s->R[3 * at], r[1] - s->R[3 * at + 1], r[2] - s->R[3 * at + 2]};
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double Rv = 0.0, Rd = 0.0, Rl = 0.0; /* R, R'/r, R'' + (2l+2) R'/r */
        for (int p = 0; p < np; ++p) {
            const double e = s->prim_exp[p0 + p];
            const double c = s->prim_coef[p0 + p] * rad_norm(s, l, kn, e);
            if (s->basis == 0) {
                const double f = ipow(rr, kn) * exp(-e * rr);
                const double g = kn / rr - e; /* R'/R */
                Rv += c * f;
                Rd += c * f * g / rr;
                Rl += c * f * (g * g - kn / (rr * rr) + (2.0 * l + 2.0) * g / rr);
            } else {
                const double f = exp(-e * rr * rr);
                Rv += c * f;
                Rd += c * f * (-2.0 * e);
                Rl += c * f * (4.0 * e * e * rr * rr - 2.0 * e - (2.0 * l + 2.0) * 2.0 * e);
            }
        }
        p0 += np;
        for (int a = l; a >= 0; --a) {
            for (int b = l - a; b >= 0; --b) {
                const int c = l - a - b;
                const double f = ang_norm(s, a, b, c);
                const double P = ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c);
                const double Px = a * ipow(d[0], a - 1) * ipow(d[1], b) * ipow(d[2], c);
                const double Py = b * ipow(d[0], a) * ipow(d[1], b - 1) * ipow(d[2], c);
                const double Pz = c * ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c - 1);
                const double L = a * (a - 1) * ipow(d[0], a - 2) * ipow(d[1], b) * ipow(d[2], c) +
                                 b * (b - 1) * ipow(d[0], a) * ipow(d[1], b - 2) * ipow(d[2], c) +
                                 c * (c - 1) * ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c - 2);
                double *o = out + 5 * mu;
                o[0] = f * P * Rv;
                o[1] = f * (Rv * Px + P * Rd * d[0]);
                o[2] = f * (Rv * Py + P * Rd * d[1]);
                o[3] = f * (Rv * Pz + P * Rd * d[2]);
                o[4] = f * (Rv * L + P * Rl);
                ++mu;
            }
        }
    }
}

/* x^a y^b z^c and its first and second derivatives. */
static double mono(const double d[3], int a, int b, int c) {
    return ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c);
}

/* AO Hessian by the product rule on chi = P(d) R(r):
   d_a d_b chi = R d_a d_b P + (d_a P d_b + d_b P d_a) R'/r
                 + P (delta_ab R'/r + (R'' - R'/r) d_a d_b / r^2),
   with R' and R'' summed over the primitives (Slater f = r^kn e^{-zeta r}:
   f' = (kn/r - zeta) f, f'' = ((kn/r - zeta)^2 - kn/r^2) f; Gaussian
   f = e^{-alpha r^2}: f' = -2 alpha r f, f'' = (4 alpha^2 r^2 - 2 alpha) f). */
void or_ao_hessian(const or_system *s, const double r[3], double *out) {
    int mu = 0, p0 = 0;
    static const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int sh = 0; sh < s->n_shells; ++sh) {
        const int at = s->shell_atom[sh], l = s->shell_l[sh], kn = s->shell_kn[sh];
        const int np = s->shell_nprim[sh];
        const double d[3] = {r[0] - s->R[3 * at], r[1] - s->R[3 * at + 1], r[2] - s->R[3 * at + 2]};
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double R0 = 0.0, R1 = 0.0, R2 = 0.0; /* R, R', R'' */
        for (int p = 0; p < np; ++p) {
            const double e = s->prim_exp[p0 + p];
            const double c = s->prim_coef[p0 + p] * rad_norm(s, l, kn, e);
            if (s->basis == 0) {
                const double f = ipow(rr, kn) * exp(-e * rr);
                const double g = kn / rr - e;
                R0 += c * f;
                R1 += c * f * g;
                R2 += c * f * (g * g - kn / (rr * rr));
            } else {
                const double f = exp(-e * rr * rr);
                R0 += c * f;
                R1 += c * f * (-2.0 * e * rr);
                R2 += c * f * (4.0 * e * e * rr * rr - 2.0 * e);
            }
        }
        p0 += np;
        const double q = R1 / rr, w = (R2 - q) / (rr * rr);
        for (int a = l; a >= 0; --a) {
            for (int b = l - a; b >= 0; --b) {
                const int c = l - a - b;
                const int e3[3] = {a, b, c};
                const double f = ang_norm(s, a, b, c);
                const double P = mono(d, a, b, c);
                double dP[3];
                for (int k = 0; k < 3; ++k) {
                    int ee[3] = {a, b, c};
                    dP[k] = ee[k] * mono(d, ee[0] - (k == 0), ee[1] - (k == 1), ee[2] - (k == 2));
                }
                double *o = out + 10 * mu;
                o[0] = f * P * R0;
                for (int k = 0; k < 3; ++k) o[1 + k] = f * (R0 * dP[k] + P * q * d[k]);
                for (int t = 0; t < 6; ++t) {
                    const int x1 = ia[t], x2 = ib[t];
                    int ee[3] = {e3[0], e3[1], e3[2]};
                    double ddP;
                    if (x1 == x2) {
                        ddP = ee[x1] * (ee[x1] - 1) *
                              mono(d, ee[0] - 2 * (x1 == 0), ee[1] - 2 * (x1 == 1), ee[2] - 2 * (x1 == 2));
                    } else {
                        ddP = ee[x1] * ee[x2] *
                              mono(d, ee[0] - (x1 == 0) - (x2 == 0), ee[1] - (x1 == 1) - (x2 == 1),
                                   ee[2] - (x1 == 2) - (x2 == 2));
                    }
                    const double dRR = (x1 == x2 ? q : 0.0) + w * d[x1] * d[x2];
                    o[4 + t] = f * (R0 * ddP + q * (dP[x1] * d[x2] + dP[x2] * d[x1]) + P * dRR);
                }
                ++mu;
            }
        }
    }
}

/* Inverse backflow (Methods, backflow transformation, with the kernel
   K_BF(r) = omega / r of the Results section): q_i = r_i + sum_{j != i}
   (omega / r_ij) (r_i - r_j). */
void or_backflow(const or_system *s, const double *x, double *q) {
    const int ne = s->n_up + s->n_dn;
    for (int i = 0; i < ne; ++i) {
        for (int c = 0; c < 3; ++c) q[3 * i + c] = x[3 * i + c];
        for (int j = 0; j < ne; ++j) {
            if (j == i) continue;
            double u[3];
            for (int c = 0; c < 3; ++c) u[c] = x[3 * i + c] - x[3 * j + c];
            const double r = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int c = 0; c < 3; ++c) q[3 * i + c] += s->bf_omega / r * u[c];
        }
    }
}

/* First and second derivatives of the backflow map, J[b][a] = dq_b / dx_a
   and K[b][a] = d^2 q_b / dx_a^2, b and a over the 3 N_e coordinates.  Each
   pair term T(u) = eta(|u|) u, u = r_i - r_k, eta = omega / r, has
   dT_b/du_a = eta delta_ab + eta' u_a u_b / r and
   d^2 T_b / du_a^2 = eta'' u_a^2 u_b / r^2
                      + eta' (u_b / r - u_a^2 u_b / r^3 + 2 delta_ab u_a / r);
   it enters q_i with du/dr_i = +1 and du/dr_k = -1. */
static void backflow_derivs(const or_system *s, const double *x, double *Jm, double *Km) {
    const int ne = s->n_up + s->n_dn, n3 = 3 * ne;
    const double om = s->bf_omega;
    for (int t = 0; t < n3 * n3; ++t) { Jm[t] = 0.0; Km[t] = 0.0; }
    for (int b = 0; b < n3; ++b) Jm[b * n3 + b] = 1.0;
    for (int i = 0; i < ne; ++i) {
        for (int k = 0; k < ne; ++k) {
            if (k == i) continue;
            double u[3];
            for (int c = 0; c < 3; ++c) u[c] = x[3 * i + c] - x[3 * k + c];
            const double r = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            const double eta = om / r, e1 = -om / (r * r), e2 = 2.0 * om / (r * r * r);
            for (int bb = 0; bb < 3; ++bb) {
                for (int aa = 0; aa < 3; ++aa) {
                    const double d1 = eta * (aa == bb) + e1 * u[aa] * u[bb] / r;
                    const double d2 = e2 * u[aa] * u[aa] * u[bb] / (r * r) +
                                      e1 * (u[bb] / r - u[aa] * u[aa] * u[bb] / (r * r * r) +
                                            2.0 * (aa == bb) * u[aa] / r);
                    const int row = 3 * i + bb;
                    Jm[row * n3 + 3 * i + aa] += d1;
                    Jm[row * n3 + 3 * k + aa] -= d1;
                    Km[row * n3 + 3 * i + aa] += d2;
                    Km[row * n3 + 3 * k + aa] += d2;
                }
            }
        }
    }
}

void or_mo(const or_system *s, const double *x, double *out) {
    const int ne = s->n_up + s->n_dn, nao = or_n_ao(s), nmo = s->n_mo;
    double *ao = (double *)malloc(sizeof(double) * 5 * nao);
    for (int e = 0; e < ne; ++e) {
        or_ao(s, x + 3 * e, ao);
        for (int c = 0; c < 5; ++c)
            for (int k = 0; k < nmo; ++k) {
                double acc = 0.0;
                for (int m = 0; m < nao; ++m) acc += ao[5 * m + c] * s->mo_coef[m * nmo + k];
                out[(e * 5 + c) * nmo + k] = acc;
            }
    }
    free(ao);
}

double or_nuclear_repulsion(const or_system *s) {
    double v = 0.0;
    for (int a = 0; a < s->n_atoms; ++a)
        for (int b = 0; b < a; ++b) {
            const double dx = s->R[3 * a] - s->R[3 * b], dy = s->R[3 * a + 1] - s->R[3 * b + 1],
                         dz = s->R[3 * a + 2] - s->R[3 * b + 2];
            v += s->Z[a] * s->Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return v;
}

/* LU factorisation with partial (row) pivoting, Doolittle form, in place
   (Golub & Van Loan, Gaussian elimination with partial pivoting).  a is n x n
   row-major; piv[k] is the row exchanged with row k at step k.  Returns 0 on
   an exactly zero pivot. */
static int lu_factor(int n, double *a, int *piv, double *perm_sign) {
    *perm_sign = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(a[i * n + k]) > best) { best = fabs(a[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return 0;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
            }
            *perm_sign = -*perm_sign;
        }
        for (int i = k + 1; i < n; ++i) {
            a[i * n + k] /= a[k * n + k];
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= a[i * n + k] * a[k * n + j];
        }
    }
    return 1;
}

/* Explicit inverse from the LU factors: column j solves A x = e_j. */
static void lu_inverse(int n, const double *lu, const int *piv, double *inv, double *b) {
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) b[i] = (i == j) ? 1.0 : 0.0;
        for (int k = 0; k < n; ++k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < i; ++k) b[i] -= lu[i * n + k] * b[k];
        for (int i = n - 1; i >= 0; --i) {
            for (int k = i + 1; k < n; ++k) b[i] -= lu[i * n + k] * b[k];
            b[i] /= lu[i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[i * n + j] = b[i];
    }
}

/* One spin block of one determinant.  phi = MO table [N_e][5][n_mo]; e0 =
   first electron of the spin; occ = MO per column slot.  Outputs log|D|,
   sign, grad log D for each electron of the block (g[n][3]) and lap D / D.
   Returns 0 when A is exactly singular. */
static int det_block(int n, int e0, int nmo, const double *phi, const int *occ, double *work,
                     int *piv, double *logabs, double *sgn, double *g, double *lap) {
    if (n == 0) { *logabs = 0.0; *sgn = 1.0; *lap = 0.0; return 1; }
    double *A = work, *inv = work + n * n, *b = work + 2 * n * n;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) A[i * n + k] = phi[((e0 + i) * 5 + 0) * nmo + occ[k]];
    double ps;
    if (!lu_factor(n, A, piv, &ps)) return 0;
    double la = 0.0, sg = ps;
    for (int k = 0; k < n; ++k) {
        la += log(fabs(A[k * n + k]));
        if (A[k * n + k] < 0) sg = -sg;
    }
    lu_inverse(n, A, piv, inv, b);
    double L = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double t = 0.0;
            for (int k = 0; k < n; ++k) t += inv[k * n + i] * phi[((e0 + i) * 5 + 1 + d) * nmo + occ[k]];
            g[3 * i + d] = t;
        }
        for (int k = 0; k < n; ++k) L += inv[k * n + i] * phi[((e0 + i) * 5 + 4) * nmo + occ[k]];
    }
    *logabs = la; *sgn = sg; *lap = L;
    return 1;
}

/* One spin block of one determinant with backflow.  phi = MO table at the
   transformed positions [N_e][10][n_mo] (value, gradient, Hessian).  For
   every coordinate a of every electron, dA and d2A follow from the chain
   rule through q(x), and eq. nabla_d gives d^2 D / D = Tr(A^-1 d2A) +
   Tr(A^-1 dA)^2 - Tr(A^-1 dA A^-1 dA).  Outputs log|D|, sign, g[3 N_e] =
   d log D / dx_a and lap = sum_a d^2 D / D.  Returns 0 when A is singular. */
static int det_block_bf(int n, int e0, int ne, int nmo, const double *phi, const int *occ,
                        const double *Jm, const double *Km, double *work, int *piv, double *logabs,
                        double *sgn, double *g, double *lap) {
    const int n3 = 3 * ne;
    static const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    if (n == 0) {
        *logabs = 0.0; *sgn = 1.0; *lap = 0.0;
        for (int a = 0; a < n3; ++a) g[a] = 0.0;
        return 1;
    }
    double *A = work, *inv = A + n * n, *b = inv + n * n, *dA = b + n, *d2A = dA + n * n, *M = d2A + n * n;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) A[i * n + k] = phi[((e0 + i) * 10 + 0) * nmo + occ[k]];
    double ps;
    if (!lu_factor(n, A, piv, &ps)) return 0;
    double la = 0.0, sg = ps;
    for (int k = 0; k < n; ++k) {
        la += log(fabs(A[k * n + k]));
        if (A[k * n + k] < 0) sg = -sg;
    }
    lu_inverse(n, A, piv, inv, b);
    double L = 0.0;
    for (int a = 0; a < n3; ++a) {
        for (int i = 0; i < n; ++i) {
            const double *Jr[3], *Kr[3];
            for (int bb = 0; bb < 3; ++bb) {
                Jr[bb] = Jm + (size_t)(3 * (e0 + i) + bb) * n3;
                Kr[bb] = Km + (size_t)(3 * (e0 + i) + bb) * n3;
            }
            for (int k = 0; k < n; ++k) {
                const double *ph = phi + (size_t)(e0 + i) * 10 * nmo + occ[k];
                double v1 = 0.0, v2 = 0.0;
                for (int bb = 0; bb < 3; ++bb) {
                    v1 += ph[(1 + bb) * nmo] * Jr[bb][a];
                    v2 += ph[(1 + bb) * nmo] * Kr[bb][a];
                }
                for (int t = 0; t < 6; ++t) {
                    const double h = ph[(4 + t) * nmo];
                    const double jj = Jr[ia[t]][a] * Jr[ib[t]][a];
                    v2 += (ia[t] == ib[t] ? 1.0 : 2.0) * h * jj;
                }
                dA[i * n + k] = v1;
                d2A[i * n + k] = v2;
            }
        }
        /* M = A^-1 dA; traces */
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) {
                double m = 0.0;
                for (int i = 0; i < n; ++i) m += inv[k * n + i] * dA[i * n + j];
                M[k * n + j] = m;
            }
        for (int k = 0; k < n; ++k) {
            t2 += M[k * n + k];
            double m2 = 0.0;
            for (int i = 0; i < n; ++i) m2 += inv[k * n + i] * d2A[i * n + k];
            t1 += m2;
            for (int j = 0; j < n; ++j) t3 += M[k * n + j] * M[j * n + k];
        }
        g[a] = t2;
        L += t1 + t2 * t2 - t3;
    }
    *logabs = la; *sgn = sg; *lap = L;
    return 1;
}

void or_eval_one(const or_system *s, const double *x, or_detail *out, double *grad) {
    const int nu = s->n_up, nd = s->n_dn, ne = nu + nd, nmo = s->n_mo, nd_ = s->n_det;
    const int nmax = nu > nd ? nu : nd;
    const int bf = s->bf_omega != 0.0, n3 = 3 * ne;
    double *phi = (double *)malloc(sizeof(double) * ne * (bf ? 10 : 5) * nmo);
    double *work = (double *)malloc(sizeof(double) * (5 * nmax * nmax + nmax + 1));
    int *piv = (int *)malloc(sizeof(int) * (nmax + 1));
    double *lg = (double *)malloc(sizeof(double) * nd_);       /* log|D_up D_dn| */
    double *sg = (double *)malloc(sizeof(double) * nd_);
    double *ok = (double *)malloc(sizeof(double) * nd_);
    double *gd = (double *)malloc(sizeof(double) * nd_ * (3 * ne + 1)); /* grad log D, lap */
    double *Jm = NULL, *Km = NULL, *gu = NULL, *gw = NULL;
    if (bf) {
        /* MO value, gradient and Hessian at the transformed positions. */
        const int nao = or_n_ao(s);
        double *q = (double *)malloc(sizeof(double) * n3);
        double *ao = (double *)malloc(sizeof(double) * 10 * nao);
        or_backflow(s, x, q);
        for (int e = 0; e < ne; ++e) {
            or_ao_hessian(s, q + 3 * e, ao);
            for (int c = 0; c < 10; ++c)
                for (int k = 0; k < nmo; ++k) {
                    double acc = 0.0;
                    for (int m = 0; m < nao; ++m) acc += ao[10 * m + c] * s->mo_coef[m * nmo + k];
                    phi[(e * 10 + c) * nmo + k] = acc;
                }
        }
        free(ao);
        free(q);
        Jm = (double *)malloc(sizeof(double) * n3 * n3);
        Km = (double *)malloc(sizeof(double) * n3 * n3);
        gu = (double *)malloc(sizeof(double) * n3);
        gw = (double *)malloc(sizeof(double) * n3);
        backflow_derivs(s, x, Jm, Km);
    } else {
        or_mo(s, x, phi);
    }

    int n_singular = 0;
    for (int n = 0; n < nd_; ++n) {
        double la_u, sg_u, lp_u, la_d, sg_d, lp_d;
        double *g = gd + (size_t)n * (3 * ne + 1);
        int ou, od;
        if (bf) {
            ou = det_block_bf(nu, 0, ne, nmo, phi, s->occ_up + n * nu, Jm, Km, work, piv, &la_u, &sg_u, gu, &lp_u);
            od = det_block_bf(nd, nu, ne, nmo, phi, s->occ_dn + n * nd, Jm, Km, work, piv, &la_d, &sg_d, gw, &lp_d);
        } else {
            ou = det_block(nu, 0, nmo, phi, s->occ_up + n * nu, work, piv, &la_u, &sg_u, g, &lp_u);
            od = det_block(nd, nu, nmo, phi, s->occ_dn + n * nd, work, piv, &la_d, &sg_d, g + 3 * nu, &lp_d);
        }
        ok[n] = (ou && od) ? 1.0 : 0.0;
        if (!(ou && od)) { ++n_singular; lg[n] = -INFINITY; sg[n] = 0.0; continue; }
        lg[n] = la_u + la_d;
        sg[n] = sg_u * sg_d;
        g[3 * ne] = lp_u + lp_d;
        if (bf) {
            /* eq. delta_sigma: both spin blocks depend on every electron, so
               the cross term 2 grad D_up / D_up . grad D_dn / D_dn stays. */
            for (int a = 0; a < n3; ++a) {
                g[a] = gu[a] + gw[a];
                g[3 * ne] += 2.0 * gu[a] * gw[a];
            }
        }
    }
    /* Sigma = sum_n d_n D_n^up D_n^dn, shifted by the largest |D| product. */
    double lmax = -INFINITY;
    for (int n = 0; n < nd_; ++n)
        if (ok[n] != 0.0 && s->ci[n] != 0.0 && lg[n] > lmax) lmax = lg[n];
    double S = 0.0, lapS = 0.0;
    double *gS = (double *)calloc(3 * ne, sizeof(double));
    if (lmax > -INFINITY) {
        for (int n = 0; n < nd_; ++n) {
            if (ok[n] == 0.0) continue;
            const double w = s->ci[n] * sg[n] * exp(lg[n] - lmax);
            const double *g = gd + (size_t)n * (3 * ne + 1);
            S += w;
            for (int q = 0; q < 3 * ne; ++q) gS[q] += w * g[q];
            lapS += w * g[3 * ne];
        }
    }
    double log_sigma, sign_sigma;
    if (S == 0.0) {
        log_sigma = -INFINITY; sign_sigma = 0.0;
    } else {
        log_sigma = lmax + log(fabs(S));
        sign_sigma = S > 0 ? 1.0 : -1.0;
        for (int q = 0; q < 3 * ne; ++q) gS[q] /= S;
        lapS /= S;
    }

    /* Jastrow and Coulomb pair sums. */
    double J = 0.0, lapJ = 0.0, vee = 0.0, ven = 0.0;
    double *gJ = (double *)calloc(3 * ne, sizeof(double));
    for (int i = 0; i < ne; ++i) {
        for (int j = i + 1; j < ne; ++j) {
            const double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const int same = (i < nu) == (j < nu);
            const double a = same ? s->a_par : s->a_anti, bb = s->b;
            const double den = 1.0 + bb * r;
            J += a * r / den;
            const double k1 = a / (den * den);            /* K'(r) */
            const double k2 = -2.0 * a * bb / (den * den * den); /* K''(r) */
            for (int c = 0; c < 3; ++c) {
                gJ[3 * i + c] += k1 * d[c] / r;
                gJ[3 * j + c] -= k1 * d[c] / r;
            }
            lapJ += 2.0 * (k2 + 2.0 * k1 / r);
            vee += 1.0 / r;
        }
        for (int a = 0; a < s->n_atoms; ++a) {
            const double dx = x[3 * i] - s->R[3 * a], dy = x[3 * i + 1] - s->R[3 * a + 1],
                         dz = x[3 * i + 2] - s->R[3 * a + 2];
            ven -= s->Z[a] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    /* Electron-nucleus kernel (appendix on the many-body Jastrow factor,
       Bertini form): K(r) = (w0 r + w1 r^2) / (1 + w2 r) for every
       electron-nucleus pair, so with N = w0 r + w1 r^2 and D = 1 + w2 r,
       K' = N'/D - N w2/D^2 and K'' = N''/D - 2 N' w2/D^2 + 2 N w2^2/D^3. */
    if (s->en) {
        for (int i = 0; i < ne; ++i) {
            for (int a = 0; a < s->n_atoms; ++a) {
                const double d[3] = {x[3 * i] - s->R[3 * a], x[3 * i + 1] - s->R[3 * a + 1],
                                     x[3 * i + 2] - s->R[3 * a + 2]};
                const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                const double w0 = s->en[3 * a], w1 = s->en[3 * a + 1], w2 = s->en[3 * a + 2];
                const double N = w0 * r + w1 * r * r, N1 = w0 + 2.0 * w1 * r, N2 = 2.0 * w1;
                const double D = 1.0 + w2 * r;
                const double K = N / D;
                const double K1 = N1 / D - N * w2 / (D * D);
                const double K2 = N2 / D - 2.0 * N1 * w2 / (D * D) + 2.0 * N * w2 * w2 / (D * D * D);
                J += K;
                for (int c = 0; c < 3; ++c) gJ[3 * i + c] += K1 * d[c] / r;
                lapJ += K2 + 2.0 * K1 / r;
            }
        }
    }

    /* Electron-electron-nucleus kernel (same appendix): for every nucleus and
       every ordered pair i > j, sum_mu c f(a1,b1; r_ai) f(a2,b2; r_aj)
       f(a3,b3; r_ij) with f(a,b; r) = a r / (1 + b r), f' = a / (1 + b r)^2,
       f'' = -2 a b / (1 + b r)^3.  Gradient and Laplacian by the product
       rule, with grad_i r_ai = u_i (unit vector from the nucleus),
       grad_j r_aj = v_j, grad_i r_ij = -grad_j r_ij = w (unit vector from j
       to i). */
    for (int a = 0; a < s->n_atoms && s->een_n > 0; ++a) {
        for (int i = 0; i < ne; ++i) {
            for (int j = 0; j < i; ++j) {
                double u[3], v[3], w[3];
                for (int c = 0; c < 3; ++c) {
                    u[c] = x[3 * i + c] - s->R[3 * a + c];
                    v[c] = x[3 * j + c] - s->R[3 * a + c];
                    w[c] = x[3 * i + c] - x[3 * j + c];
                }
                const double ru = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                const double rv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                const double rw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
                for (int c = 0; c < 3; ++c) { u[c] /= ru; v[c] /= rv; w[c] /= rw; }
                const double uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
                const double vw = v[0] * w[0] + v[1] * w[1] + v[2] * w[2];
                for (int m = 0; m < s->een_n; ++m) {
                    const double *q = s->een + 7 * m;
                    const double c = q[0];
                    double f1, d1, e1, f2, d2, e2, f3, d3, e3;
                    {
                        const double D = 1.0 + q[2] * ru;
                        f1 = q[1] * ru / D; d1 = q[1] / (D * D); e1 = -2.0 * q[1] * q[2] / (D * D * D);
                    }
                    {
                        const double D = 1.0 + q[4] * rv;
                        f2 = q[3] * rv / D; d2 = q[3] / (D * D); e2 = -2.0 * q[3] * q[4] / (D * D * D);
                    }
                    {
                        const double D = 1.0 + q[6] * rw;
                        f3 = q[5] * rw / D; d3 = q[5] / (D * D); e3 = -2.0 * q[5] * q[6] / (D * D * D);
                    }
                    J += c * f1 * f2 * f3;
                    for (int k = 0; k < 3; ++k) {
                        gJ[3 * i + k] += c * (d1 * u[k] * f2 * f3 + f1 * f2 * d3 * w[k]);
                        gJ[3 * j + k] += c * (f1 * d2 * v[k] * f3 - f1 * f2 * d3 * w[k]);
                    }
                    const double lap3 = e3 + 2.0 * d3 / rw;
                    lapJ += c * f2 * ((e1 + 2.0 * d1 / ru) * f3 + 2.0 * d1 * d3 * uw + f1 * lap3);
                    lapJ += c * f1 * ((e2 + 2.0 * d2 / rv) * f3 - 2.0 * d2 * d3 * vw + f2 * lap3);
                }
            }
        }
    }

    double kin = lapJ + lapS;
    for (int q = 0; q < 3 * ne; ++q) kin += gJ[q] * gJ[q] + 2.0 * gJ[q] * gS[q];
    const double e_kin = -0.5 * kin;
    const double e_pot = vee + ven + or_nuclear_repulsion(s);

    out->jastrow = J;
    out->log_sigma = log_sigma;
    out->logpsi = J + log_sigma;
    out->sign = sign_sigma;
    out->e_kin = e_kin;
    out->e_pot = e_pot;
    out->eloc = (n_singular > 0 || S == 0.0) ? NAN : e_kin + e_pot;
    if (grad)
        for (int q = 0; q < 3 * ne; ++q) grad[q] = gJ[q] + gS[q];
    free(gJ); free(gS); free(gd); free(ok); free(sg); free(lg); free(piv); free(work); free(phi);
    free(Jm); free(Km); free(gu); free(gw);
}

int or_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_eval(const or_system *s, const double *X, int64_t W, double *logpsi, double *sign,
             double *eloc, int nthreads) {
    const int ne = s->n_up + s->n_dn;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
#endif
    for (int64_t w = 0; w < W; ++w) {
        or_detail d;
        or_eval_one(s, X + (size_t)w * 3 * ne, &d, NULL);
        logpsi[w] = d.logpsi;
        sign[w] = d.sign;
        eloc[w] = d.eloc;
    }
    (void)nthreads;
}

/* ---- Philox4x32-10 -------------------------------------------------------
   Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten
   rounds of the 4x32 Philox S-box with multipliers 0xD2511F53 and
   0xCD9E8D57 and a Weyl key schedule with increments 0x9E3779B9 and
   0xBB67AE85. */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Stream layout: key = seed (low word, high word); counter = (walker id, step
   low word, step high word, call).  Call e < N_e gives electron e's normals:
   the four words become uniforms u_k = (w_k + 1/2) 2^-32 in (0,1); Box-Muller
   on (u0,u1) gives x and y, on (u2,u3) gives z.  Call N_e gives the accept
   uniform from the top 53 bits of (w0 << 32 | w1). */
void or_proposal(int n_elec, uint64_t seed, uint32_t walker_id, uint64_t step, double *z,
                 double *u_accept) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {walker_id, (uint32_t)step, (uint32_t)(step >> 32), 0};
    uint32_t w[4];
    const double s32 = 1.0 / 4294967296.0;
    for (int e = 0; e < n_elec; ++e) {
        ctr[3] = (uint32_t)e;
        or_philox4x32_10(ctr, key, w);
        const double u0 = (w[0] + 0.5) * s32, u1 = (w[1] + 0.5) * s32;
        const double u2 = (w[2] + 0.5) * s32, u3 = (w[3] + 0.5) * s32;
        const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
        z[3 * e + 0] = r0 * cos(OR_TWO_PI * u1);
        z[3 * e + 1] = r0 * sin(OR_TWO_PI * u1);
        z[3 * e + 2] = r1 * cos(OR_TWO_PI * u3);
    }
    ctr[3] = (uint32_t)n_elec;
    or_philox4x32_10(ctr, key, w);
    const uint64_t bits = (((uint64_t)w[0] << 32) | w[1]) >> 11;
    *u_accept = (double)bits * (1.0 / 9007199254740992.0);
}

void or_metropolis(const or_system *s, double *X, double *logpsi, double *sign, double *eloc,
                   int64_t W, int n_steps, double sigma, uint64_t seed, uint64_t step0,
                   uint32_t walker_offset, double *acc, uint8_t *accept_log, int nthreads) {
    const int ne = s->n_up + s->n_dn;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
    for (int64_t w = 0; w < W; ++w) {
        double *x = X + (size_t)w * 3 * ne;
        double *z = (double *)malloc(sizeof(double) * 3 * ne);
        double *xp = (double *)malloc(sizeof(double) * 3 * ne);
        for (int t = 0; t < n_steps; ++t) {
            double u;
            or_proposal(ne, seed, walker_offset + (uint32_t)w, step0 + (uint64_t)t, z, &u);
            for (int q = 0; q < 3 * ne; ++q) xp[q] = x[q] + sigma * z[q];
            or_detail d;
            or_eval_one(s, xp, &d, NULL);
            const int accept = isfinite(d.logpsi) && (u < exp(2.0 * (d.logpsi - logpsi[w])));
            if (accept) {
                memcpy(x, xp, sizeof(double) * 3 * ne);
                logpsi[w] = d.logpsi;
                sign[w] = d.sign;
                eloc[w] = d.eloc;
            }
            /* the Monte Carlo mean of eq. Ev runs over the steps whose state
               has a finite log|Psi| and E_L; the others are only counted */
            if (isfinite(eloc[w]) && isfinite(logpsi[w])) {
                acc[4 * w + 0] += eloc[w];
                acc[4 * w + 1] += eloc[w] * eloc[w];
            } else {
                acc[4 * w + 3] += 1.0;
            }
            acc[4 * w + 2] += accept ? 1.0 : 0.0;
            if (accept_log) accept_log[(size_t)t * W + w] = (uint8_t)accept;
        }
        free(xp);
        free(z);
    }
    (void)nthreads;
}
