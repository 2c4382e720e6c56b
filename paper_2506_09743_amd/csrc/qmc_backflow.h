// Inverse backflow (Methods, backflow transformation; kernel omega / r_ij of
// the Results section) with the local energy of eq. nabla_d, FP64.  Included
// at the end of qmc_walker.h; core_stages calls backflow_dets after the
// Jastrow stage, which keeps the bare positions.
//
// Notation.  q_i = r_i + sum_{j != i} s_ij u_ij, u_ij = r_i - r_j,
// s_ij = omega / r_ij.  The Jacobian of the map is made of symmetric 3 x 3
// blocks J_ij = dq_i / dr_j:
//   J_ij = -s_ij (I - h h^T)  (j != i, h = u_ij / r_ij),
//   J_ii = I + sum_{k != i} s_ik (I - h_ik h_ik^T),
// and sum over all coordinates of d^2 q_i / dr^2 is
//   k_i = -4 omega sum_{k != i} u_ik / r_ik^3.
// For one spin block with matrix A[i][k] = phi_{occ_k}(q_i) and
// Mt_{i b, i'} = sum_k d_b phi_{occ_k}(q_i) A^-1[k][i'], g_i = Mt_{i., i},
// Y_ii' = sum_j J_ij J_i'j (all electrons j), the three traces of
// eq. nabla_d summed over every coordinate are
//   sum Tr(A^-1 d2A)       = sum_i sum_k A^-1[k][i] psi_occk(i),
//                            psi_m(i) = H phi_m(q_i) : Y_ii + grad phi_m(q_i) . k_i,
//   sum Tr(A^-1 dA)^2      = sum_{i,i'} g_i^T Y_ii' g_i',
//   sum Tr((A^-1 dA)^2)    = sum_{i,i'} sum_{b,c} Mt_{i b, i'} Y_ii'[b][c] Mt_{i' c, i},
// and grad log D at electron j is sum_i J_ij g_i.  Across the CI expansion
// (eqs. nabla_sigma and delta_sigma) the determinants of the two spins no
// longer depend on disjoint electrons, so the cross term
// 2 grad D_up / D_up . grad D_dn / D_dn = 2 sum_{i up, i' dn} g_i^T Y_ii' g_i'
// stays.
//
// Work decomposition.  Lane i of a walker owns electron i as everywhere
// else.  Its MO table at q_i (value, psi, gradient for every MO) lives in a
// private array.  The pair sums above are symmetric in (i, i'), so each
// lane holds only the Y blocks of its share of the pairs (at most 9 of
// them, in registers): within a spin the partners i + d (mod n), d <= n/2,
// and of the up-down pairs the half picked by the cyclic offset between the
// two indices.  Every distinct spin configuration is factorised by the
// group's in-place Gauss-Jordan (both spins at once, one configuration each
// per step); its Mt rows and g vectors go through LDS.  Each lane keeps,
// per configuration of its spin, its g_i and, per configuration of the
// other spin, v_i = sum over its cross partners i' of Y_ii' g_i', so the
// cross term of a determinant is the sum of g_i . v_i over all lanes.
#pragma once

namespace qmc {
namespace walker {

// The system tables never change while a kernel runs: read through the
// constant address space, a load whose address is the same on every lane
// becomes a scalar load.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *const_tab(const T *p) {
    return (const __attribute__((address_space(4))) T *)p;
}

// Walker-local lane of electron j.
__device__ __forceinline__ int lane_of(const DevSystem &S, int j) {
    return j < S.n_up ? j : S.G + (j - S.n_up);
}

// LDS of one walker with backflow (doubles), from the walker's base.  A
// shared region holds in turn the diagonal Jacobian blocks [LW][6] (while
// the Y rows are built), the determinant tables of the configuration loop
// (low-rank: the reference rows [2][nmax][NMO] = A0^-1 | T and pivot rows
// [2][NMO]; explicit: inverse tables [2][G][8] and pivot rows [2][8]) and
// the weighted g [LW][3] (at the end).  Then Mt rows [2][G][3][8], published
// g [2][G][3] and per configuration (log|D|, sign, weight, L, scaled value)
// [2][n_cfg_max][5]; the positions follow at bf_pos_offset.
template <int NMO, bool LR>
__host__ __device__ inline int bf_shared_size(const DevSystem &S) {
    const int nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int dets = LR ? 2 * nmax * NMO + 2 * NMO : 2 * S.G * kMaxSpin + 2 * kMaxSpin;
    const int a = 6 * S.LW > dets ? 6 * S.LW : dets;
    return a > 3 * S.LW ? a : 3 * S.LW;
}

template <int NMO, bool LR>
__host__ __device__ inline int bf_table_size(const DevSystem &S) {
    return bf_shared_size<NMO, LR>(S) + 2 * S.G * 3 * kMaxSpin + 2 * S.G * 3 + 10 * S.n_cfg_max;
}

template <int NMO, bool LR>
__host__ __device__ inline int bf_pos_offset(const DevSystem &S) {
    const int a = pos_offset<NMO>(S), b = bf_table_size<NMO, LR>(S);
    return a > b ? a : b;
}

template <int NMO, bool LR>
__host__ __device__ inline int walker_lds_bf(const DevSystem &S) {
    return bf_pos_offset<NMO, LR>(S) + 3 * S.LW;
}

// In-place Gauss-Jordan of the spin group's reference rows [A0 | Phi]
// (NMO entries per lane, reference orbitals in columns 0..n-1): afterwards
// the row of slot s holds A0^-1[s][slot(e)] in the columns < n and
// T[s][v] = (A0^-1 Phi)[s][v] in the others.  Every lane of the block runs
// the same steps (block barriers inside).
template <int NMO>
__device__ __forceinline__ void reference_gauss_jordan(const DevSystem &S, const Lane &L, double (&a)[NMO], int nmax,
                                                       double *piv_row, int &slot, double &dprod, bool &singular) {
    constexpr int JMAX = kMaxSpin < NMO ? kMaxSpin : NMO;
    bool done = !L.active;
    slot = -1;
    dprod = 1.0;
    singular = false;
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
        const double piv = ok ? piv_row[j] : 0.0;
        if (work) dprod *= piv;
        if (ok && L.active && !is_piv) {
            const double f = a[j] / piv;
#pragma unroll
            for (int m = 0; m < NMO; ++m) a[m] -= f * piv_row[m];
            a[j] = -f;
        }
        __syncthreads();
    }
}

// Symmetric 3 x 3 block (xx, xy, xz, yy, yz, zz) of J_ij for i != j from the
// two positions.
__device__ __forceinline__ void jblock_pair(double om, const double *pi, const double *pj, double (&B)[6]) {
    const double u0 = pi[0] - pj[0], u1 = pi[1] - pj[1], u2 = pi[2] - pj[2];
    const double rinv = rsqrt(u0 * u0 + u1 * u1 + u2 * u2);
    const double s = om * rinv;
    const double h0 = u0 * rinv, h1 = u1 * rinv, h2 = u2 * rinv;
    B[0] = -s * (1.0 - h0 * h0);
    B[1] = s * h0 * h1;
    B[2] = s * h0 * h2;
    B[3] = -s * (1.0 - h1 * h1);
    B[4] = s * h1 * h2;
    B[5] = -s * (1.0 - h2 * h2);
}

// Radial factor of a shell at distance r for second derivatives: R,
// qr = R'/r and wr = (R'' - R'/r) / r^2.  Slater f = c r^kn exp(-zeta r):
// R' = f g, R'' = f (g^2 - kn/r^2), g = kn/r - zeta; Gaussian
// f = c exp(-alpha r^2): R'/r = -2 alpha f, (R'' - R'/r)/r^2 = 4 alpha^2 f.
__device__ __forceinline__ void shell_radial_h(const DevSystem &S, int p, int np, int kn, double r, double r2,
                                               double rinv, double &R, double &qr, double &wr) {
    R = 0.0;
    qr = 0.0;
    wr = 0.0;
    if (S.basis == 0) {
        double rk = 1.0;
        for (int t = 0; t < kn; ++t) rk *= r;
        const double kr = double(kn) * rinv;
        for (int q = 0; q < np; ++q) {
            const double2 pe = S.prims[p + q];
            const double f = pe.y * rk * exp_f64(-pe.x * r);
            const double g = kr - pe.x;
            R += f;
            qr += f * g * rinv;
            wr += f * (g * g - kr * rinv - g * rinv) * rinv * rinv;
        }
    } else {
        for (int q = 0; q < np; ++q) {
            const double2 pe = S.prims[p + q];
            const double f = pe.y * exp_f64(-pe.x * r2);
            R += f;
            qr -= 2.0 * pe.x * f;
            wr += 4.0 * pe.x * pe.x * f;
        }
    }
}

// Channels C0 .. C0 + NC - 1 of the lane's MO table at q in one pass over
// the shells: channel 0 value, 1 psi (Hessian contracted with Y_ii plus
// gradient dotted with k_i), 2..4 the gradient.  For chi = P(d) R(r):
//   d_a chi = R d_a P + P qr d_a,
//   H chi : Y = R (dd P : Y) + 2 qr grad P^T Y d + P (qr tr Y + wr d^T Y d).
// Returns sum_mu C[mu][m] (channel C0 + c of chi_mu) in out[c][m].
template <int NMO, int C0, int NC>
__device__ __forceinline__ void mo_channels_bf(const DevSystem &S, double q0, double q1, double q2,
                                               const double (&Y)[6], double k0, double k1, double k2,
                                               double (&out)[NC][NMO]) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < NMO; ++m) out[c][m] = 0.0;
    const double *crow = S.mo;
    int p = 0, atom = -1;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, r = 0.0, r2 = 0.0, rinv = 0.0;
    double Yd0 = 0.0, Yd1 = 0.0, Yd2 = 0.0, dYd = 0.0;
    const double trY = Y[0] + Y[3] + Y[5];
    for (int sh = 0; sh < S.n_shells; ++sh) {
        const int4 si = S.shells[sh];
        if (si.x != atom) {
            atom = si.x;
            const double *A = S.atoms + 4 * atom;
            d0 = q0 - A[0];
            d1 = q1 - A[1];
            d2 = q2 - A[2];
            r2 = d0 * d0 + d1 * d1 + d2 * d2;
            r = sqrt(r2);
            rinv = 1.0 / r;
            Yd0 = Y[0] * d0 + Y[1] * d1 + Y[2] * d2;
            Yd1 = Y[1] * d0 + Y[3] * d1 + Y[4] * d2;
            Yd2 = Y[2] * d0 + Y[4] * d1 + Y[5] * d2;
            dYd = d0 * Yd0 + d1 * Yd1 + d2 * Yd2;
        }
        double R, qr, wr;
        shell_radial_h(S, p, si.w, si.z, r, r2, rinv, R, qr, wr);
        p += si.w;
        const int nc = (si.y + 1) * (si.y + 2) / 2;
        for (int c = 0; c < nc; ++c) {
            double P, P0, P1, P2, PY;  // monomial, gradient, dd P : Y
            if (si.y == 0) {
                P = 1.0;
                P0 = P1 = P2 = PY = 0.0;
            } else if (si.y == 1) {
                P = c == 0 ? d0 : (c == 1 ? d1 : d2);
                P0 = c == 0 ? 1.0 : 0.0;
                P1 = c == 1 ? 1.0 : 0.0;
                P2 = c == 2 ? 1.0 : 0.0;
                PY = 0.0;
            } else {
                // xx, xy, xz, yy, yz, zz: d_a d_b (x_u x_v) = delta_au delta_bv + delta_av delta_bu
                const int iu = (c < 3) ? 0 : (c < 5 ? 1 : 2);
                const int iv = (c == 0) ? 0 : (c == 1 || c == 3) ? 1 : 2;
                const double u = iu == 0 ? d0 : (iu == 1 ? d1 : d2);
                const double v = iv == 0 ? d0 : (iv == 1 ? d1 : d2);
                P = u * v;
                P0 = (iu == 0 ? v : 0.0) + (iv == 0 ? u : 0.0);
                P1 = (iu == 1 ? v : 0.0) + (iv == 1 ? u : 0.0);
                P2 = (iu == 2 ? v : 0.0) + (iv == 2 ? u : 0.0);
                const int yi = iu == 0 ? iv : (iu == 1 ? 2 + iv : 5);  // packed Y index of (u, v), u <= v
                PY = 2.0 * Y[yi];
            }
            const double g0 = R * P0 + P * qr * d0, g1 = R * P1 + P * qr * d1, g2 = R * P2 + P * qr * d2;
            double val[NC];
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) {
                const int comp = C0 + ch;
                if (comp == 0) val[ch] = P * R;
                else if (comp == 1)
                    val[ch] = R * PY + 2.0 * qr * (P0 * Yd0 + P1 * Yd1 + P2 * Yd2) + P * (qr * trY + wr * dYd) +
                              g0 * k0 + g1 * k1 + g2 * k2;
                else val[ch] = comp == 2 ? g0 : (comp == 3 ? g1 : g2);
            }
#pragma unroll
            for (int m = 0; m < NMO; ++m)
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) out[ch][m] += val[ch] * crow[m];
            crow += S.nmo_pad;
        }
    }
}

// LR: configurations from the reference by the rank <= 2 update of
// eq. table (only A0 is factorised); otherwise every configuration is
// factorised on its own.
template <int NMO, bool LR, int CAP>
__device__ __forceinline__ void backflow_dets(const DevSystem &S, const Lane &L, double *wsm, const double *sPos,
                                              double x0, double x1, double x2, Core<NMO> &c) {
    const int LW = S.LW, nmax = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const double om = S.bf_omega;
    const int G = S.G;
    double *sJd = wsm;                                      // [LW][6] (shared region)
    double *sInv = wsm;                                     // [2][G][8] (shared region, explicit)
    double *sPv = sInv + 2 * G * kMaxSpin;                  // [2][8]
    double *sRef = wsm;                                     // [2][nmax][NMO] (shared region, low-rank)
    double *sPvN = sRef + 2 * nmax * NMO;                   // [2][NMO]
    double *sGb = wsm;                                      // [LW][3] (shared region, at the end)
    double *sMt = wsm + bf_shared_size<NMO, LR>(S);         // [2][G][3][8]
    double *sGp = sMt + 2 * G * 3 * kMaxSpin;               // [2][G][3]
    double *sCfg = sGp + 2 * G * 3;                         // [2][n_cfg_max][5]
    double *inv_g = sInv + L.grp * G * kMaxSpin;
    double *piv_g = sPv + L.grp * kMaxSpin;
    double *mt_g = sMt + L.grp * 3 * G * kMaxSpin;
    double *cfg_g = sCfg + L.grp * S.n_cfg_max * 5;
    const int ncfg_g = L.grp == 0 ? S.n_cfg_up : S.n_cfg_dn;
    const int ncfg_o = L.grp == 0 ? S.n_cfg_dn : S.n_cfg_up;
    const int nsig_o = L.grp == 0 ? S.n_dn : S.n_up;
    const int gb_own = L.grp * S.G, gb_oth = (1 - L.grp) * S.G;  // walker-local first lanes
    const int ncmax = S.n_cfg_up > S.n_cfg_dn ? S.n_cfg_up : S.n_cfg_dn;
    const double xs[3] = {x0, x1, x2};

    __syncthreads();  // the Jastrow stage's tables are no longer read

    // ---- transformed position, diagonal Jacobian block, k_i -------------
    double q0 = x0, q1 = x1, q2 = x2;
    double Jd[6] = {1.0, 0.0, 0.0, 1.0, 0.0, 1.0};
    double k0 = 0.0, k1 = 0.0, k2 = 0.0;
    if (L.active) {
        for (int j = 0; j < S.ne; ++j) {
            if (j == L.e) continue;
            const double *pj = sPos + 3 * lane_of(S, j);
            const double u0 = x0 - pj[0], u1 = x1 - pj[1], u2 = x2 - pj[2];
            const double rinv = rsqrt(u0 * u0 + u1 * u1 + u2 * u2);
            const double s = om * rinv;
            q0 += s * u0;
            q1 += s * u1;
            q2 += s * u2;
            const double h0 = u0 * rinv, h1 = u1 * rinv, h2 = u2 * rinv;
            Jd[0] += s * (1.0 - h0 * h0);
            Jd[1] -= s * h0 * h1;
            Jd[2] -= s * h0 * h2;
            Jd[3] += s * (1.0 - h1 * h1);
            Jd[4] -= s * h1 * h2;
            Jd[5] += s * (1.0 - h2 * h2);
            const double t = -4.0 * s * rinv * rinv;
            k0 += t * u0;
            k1 += t * u1;
            k2 += t * u2;
        }
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) sJd[6 * L.lw + t] = Jd[t];
    __syncthreads();

    // ---- Y blocks: Y_{e,j'} = sum_m J_em J_j'm over all electrons m --------
    // Both traces summed over a spin's pairs are symmetric in (i, i'), so
    // lane i takes the partners i' = i + d (mod n) for d <= n / 2 only, the
    // pairs with 0 < 2d < n at weight 2.  The pairs (i up, i' down) of the
    // cross term are split between the two groups by the cyclic offset
    // (i' - i) mod M, M = max(n_up, n_dn): below ceil(M/2) the up lane
    // takes the pair, otherwise the down lane.  Every block index is static,
    // so the blocks stay in registers.
    constexpr int kHalf = kMaxSpin / 2;
    const int mspin = S.n_up > S.n_dn ? S.n_up : S.n_dn;
    const int ncross = L.grp == 0 ? (mspin + 1) / 2 : mspin / 2;
    int own_p[kHalf + 1], oth_p[kHalf];  // partner index within its group, -1: none
#pragma unroll
    for (int d = 0; d <= kHalf; ++d) {
        int ip = L.i + d;
        if (ip >= L.nsig) ip -= L.nsig;
        own_p[d] = (L.active && 2 * d <= L.nsig) ? ip : -1;
    }
#pragma unroll
    for (int t = 0; t < kHalf; ++t) {
        int ip = L.i + t + L.grp;
        if (ip >= mspin) ip -= mspin;
        oth_p[t] = (L.active && t < ncross && ip < nsig_o) ? ip : -1;
    }
    double Yo[kHalf + 1][9], Yc[kHalf][9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
#pragma unroll
        for (int d = 0; d <= kHalf; ++d) Yo[d][t] = 0.0;
#pragma unroll
        for (int d = 0; d < kHalf; ++d) Yc[d][t] = 0.0;
    }
    if (L.active) {
        for (int m = 0; m < S.ne; ++m) {
            const int lm = lane_of(S, m);
            double A[6];
            if (m == L.e) {
#pragma unroll
                for (int t = 0; t < 6; ++t) A[t] = Jd[t];
            } else {
                jblock_pair(om, xs, sPos + 3 * lm, A);
            }
            const double a[9] = {A[0], A[1], A[2], A[1], A[3], A[4], A[2], A[4], A[5]};
#pragma unroll
            for (int d = 0; d < 2 * kHalf + 1; ++d) {
                const int ip = d <= kHalf ? own_p[d] : oth_p[d - kHalf - 1];
                if (ip < 0) continue;
                const int lp = (d <= kHalf ? gb_own : gb_oth) + ip;
                double B[6];
                if (d == 0) {
#pragma unroll
                    for (int t = 0; t < 6; ++t) B[t] = A[t];
                } else if (lp == lm) {
#pragma unroll
                    for (int t = 0; t < 6; ++t) B[t] = sJd[6 * lp + t];
                } else {
                    jblock_pair(om, sPos + 3 * lp, sPos + 3 * lm, B);
                }
                // y += A B with the full 3 x 3 forms of the two symmetric blocks
                const double b[9] = {B[0], B[1], B[2], B[1], B[3], B[4], B[2], B[4], B[5]};
                double *y = d <= kHalf ? Yo[d] : Yc[d - kHalf - 1];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        y[3 * r + cc] += a[3 * r] * b[cc] + a[3 * r + 1] * b[3 + cc] + a[3 * r + 2] * b[6 + cc];
            }
        }
    }

    // ---- MO table at q: value, psi, gradient ----------------------------
    double tab[5 * NMO];
    {
        double Yii[6] = {1.0, 0.0, 0.0, 1.0, 0.0, 1.0};
        if (L.active) {
            const double *y = Yo[0];
            Yii[0] = y[0];
            Yii[1] = y[1];
            Yii[2] = y[2];
            Yii[3] = y[4];
            Yii[4] = y[5];
            Yii[5] = y[8];
        } else {
            q0 = q1 = q2 = 100.0;  // a far point keeps idle lanes finite
        }
        // two passes over the shells: value and psi, then the gradient
        {
            double o[2][NMO];
            mo_channels_bf<NMO, 0, 2>(S, q0, q1, q2, Yii, k0, k1, k2, o);
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int m = 0; m < NMO; ++m) tab[c * NMO + m] = o[c][m];
        }
        {
            double o[3][NMO];
            mo_channels_bf<NMO, 2, 3>(S, q0, q1, q2, Yii, k0, k1, k2, o);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int m = 0; m < NMO; ++m) tab[(2 + c) * NMO + m] = o[c][m];
        }
    }

    __syncthreads();  // every lane has read the shared region's J blocks

    // ---- low-rank: the reference once --------------------------------------
    // Reference rows [A0 | Phi] by Gauss-Jordan; then per lane the reference
    // Mt row Mt0[b][i'] = sum_k d_b phi_k(q_i) A0^-1[k][i'], the first trace
    // t10 = sum_k A0^-1[k][i] psi_k(i), and the residual rows
    // Z[b][m] = d_b phi_m(q_i) - sum_k d_b phi_k(q_i) T[k][m] (b = 3: psi),
    // which vanish on the reference columns.  A configuration with holes H
    // and particles P (canonical order, sign s_c) then has
    // det A_c = s_c D0 det R, R = T[H, P], and
    // Mt_c = Mt0 + Z[:, P] R^-1 A0^-1[H, :], t1_c = t10 + sum_i Zpsi[i, P] R^-1 A0^-1[H, i].
    double Mt0[3][kMaxSpin];
    double t10 = 0.0, ref_log = 0.0, ref_sgn = 1.0;
    bool ref_sing = false;
    double zt[LR ? 4 * NMO : 1];
    int rslots[kMaxSpin];
    double *ref_g = sRef + L.grp * nmax * NMO;
    if constexpr (LR) {
        double a[NMO];
#pragma unroll
        for (int m = 0; m < NMO; ++m) a[m] = L.active ? tab[m] : 0.0;
        int slot;
        double dprod;
        reference_gauss_jordan<NMO>(S, L, a, nmax, sPvN + L.grp * NMO, slot, dprod, ref_sing);
        ref_sgn = group_parity(S, L, slot) * (dprod < 0.0 ? -1.0 : 1.0);
        ref_log = log(fabs(dprod));
        if (L.active && slot >= 0) {
#pragma unroll
            for (int m = 0; m < NMO; ++m) ref_g[slot * NMO + m] = a[m];
        }
#pragma unroll
        for (int ip = 0; ip < kMaxSpin; ++ip) rslots[ip] = ip < S.G ? __shfl(slot, L.gbase + ip) : -1;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int ip = 0; ip < kMaxSpin; ++ip) Mt0[b][ip] = 0.0;
        if (L.active && !ref_sing) {
            // the reference columns' psi and gradient, read once
            double rc[kMaxSpin][4];
#pragma unroll
            for (int k = 0; k < kMaxSpin; ++k) {
                if (k >= L.nsig) break;
#pragma unroll
                for (int b = 0; b < 4; ++b) rc[k][b] = tab[(1 + b) * NMO + k];
            }
#pragma unroll
            for (int k = 0; k < kMaxSpin; ++k) {
                if (k >= L.nsig) break;
                const double *irow = ref_g + k * NMO;
#pragma unroll
                for (int ip = 0; ip < kMaxSpin; ++ip) {
                    if (ip >= L.nsig) break;
                    const double v = irow[rslots[ip]];
                    Mt0[0][ip] += rc[k][1] * v;
                    Mt0[1][ip] += rc[k][2] * v;
                    Mt0[2][ip] += rc[k][3] * v;
                }
                t10 += irow[slot] * rc[k][0];
            }
            for (int m = 0; m < NMO; ++m) {
                double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
                if (m >= L.nsig) {
                    z0 = tab[2 * NMO + m];
                    z1 = tab[3 * NMO + m];
                    z2 = tab[4 * NMO + m];
                    z3 = tab[NMO + m];
#pragma unroll
                    for (int k = 0; k < kMaxSpin; ++k) {
                        if (k >= L.nsig) break;
                        const double t = ref_g[k * NMO + m];
                        z0 -= rc[k][1] * t;
                        z1 -= rc[k][2] * t;
                        z2 -= rc[k][3] * t;
                        z3 -= rc[k][0] * t;
                    }
                }
                zt[m] = z0;
                zt[NMO + m] = z1;
                zt[2 * NMO + m] = z2;
                zt[3 * NMO + m] = z3;
            }
        }
    }

    // ---- every configuration of each spin --------------------------------
    // per-configuration rows of this lane (CAP >= the system's configurations per spin)
    double gtab[CAP * 3], vtab[CAP * 3];
    for (int q = 0; q < ncmax; ++q) {
        const bool live = q < ncfg_g;
        double t1 = 0.0, clog = -INFINITY, csgn = 0.0;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
        bool singular, ok;
        if constexpr (LR) {
            // code: rank | h0 << 2 | h1 << 5 | p0 << 8 | p1 << 13, bit 20: odd
            // permutation to canonical order, bit 21: identically zero
            // both spins' codes by scalar loads, then this group's
            const int cu = q < S.n_cfg_up ? const_tab(S.cfg_exc)[q] : 0;
            const int cd = q < S.n_cfg_dn ? const_tab(S.cfg_exc)[S.n_cfg_max + q] : 0;
            const int code = live ? (L.grp ? cd : cu) : 0;
            const int rk = code & 3, h0 = (code >> 2) & 7, h1 = (code >> 5) & 7;
            const int p0 = (code >> 8) & 31, p1 = (code >> 13) & 31;
            double R00 = 1.0, R01 = 0.0, R10 = 0.0, R11 = 1.0;
            if (rk >= 1) R00 = ref_g[h0 * NMO + p0];
            if (rk == 2) {
                R01 = ref_g[h0 * NMO + p1];
                R10 = ref_g[h1 * NMO + p0];
                R11 = ref_g[h1 * NMO + p1];
            }
            const double detR = rk == 2 ? R00 * R11 - R01 * R10 : R00;
            singular = !live || ref_sing || ((code >> 21) & 1) || detR == 0.0;
            ok = !singular && L.active;
            if (!singular) {
                clog = ref_log + log(fabs(detR));
                csgn = ref_sgn * (((code >> 20) & 1) ? -1.0 : 1.0) * (detR < 0.0 ? -1.0 : 1.0);
            }
            if (ok) {
                // R^-1 (rows particles, columns holes)
                const double di = 1.0 / detR;
                const double Q00 = rk == 2 ? R11 * di : di, Q01 = -R01 * di, Q10 = -R10 * di, Q11 = R00 * di;
                const double za0 = zt[p0], za1 = zt[NMO + p0], za2 = zt[2 * NMO + p0], zap = zt[3 * NMO + p0];
                const double zb0 = rk == 2 ? zt[p1] : 0.0, zb1 = rk == 2 ? zt[NMO + p1] : 0.0;
                const double zb2 = rk == 2 ? zt[2 * NMO + p1] : 0.0, zbp = rk == 2 ? zt[3 * NMO + p1] : 0.0;
                const double *hr0 = ref_g + h0 * NMO, *hr1 = ref_g + h1 * NMO;
                // the updated row goes straight to LDS
                double *mrow = mt_g + L.i * 3 * kMaxSpin;
#pragma unroll
                for (int ip = 0; ip < kMaxSpin; ++ip) {
                    if (ip >= L.nsig) break;
                    double d0 = 0.0, d1 = 0.0;  // (R^-1 A0^-1[H, i'])_j
                    if (rk == 1) {
                        d0 = Q00 * hr0[rslots[ip]];
                    } else if (rk == 2) {
                        const double v0 = hr0[rslots[ip]], v1 = hr1[rslots[ip]];
                        d0 = Q00 * v0 + Q01 * v1;
                        d1 = Q10 * v0 + Q11 * v1;
                    }
                    const double m0 = Mt0[0][ip] + za0 * d0 + zb0 * d1;
                    const double m1 = Mt0[1][ip] + za1 * d0 + zb1 * d1;
                    const double m2 = Mt0[2][ip] + za2 * d0 + zb2 * d1;
                    mrow[ip] = m0;
                    mrow[kMaxSpin + ip] = m1;
                    mrow[2 * kMaxSpin + ip] = m2;
                    if (ip == L.i) {
                        g0 = m0;
                        g1 = m1;
                        g2 = m2;
                        t1 = t10 + zap * d0 + zbp * d1;
                    }
                }
            }
        } else {
            double Mt[3][kMaxSpin];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int ip = 0; ip < kMaxSpin; ++ip) Mt[b][ip] = 0.0;
            // both spins' occupations by scalar loads, then this group's
            const auto *occ_u = const_tab(S.cfg_occ) + (q < S.n_cfg_up ? q : 0) * kMaxSpin;
            const auto *occ_d = const_tab(S.cfg_occ) + (S.n_cfg_max + (q < S.n_cfg_dn ? q : 0)) * kMaxSpin;
            int occ[kMaxSpin];
#pragma unroll
            for (int k = 0; k < kMaxSpin; ++k) occ[k] = L.grp ? occ_d[k] : occ_u[k];
            double a[kMaxSpin];
#pragma unroll
            for (int k = 0; k < kMaxSpin; ++k)
                a[k] = (L.active && live && k < L.nsig) ? tab[occ[k]] : 0.0;
            int slot;
            double dprod;
            group_gauss_jordan(S, L, a, L.nsig, nmax, live, piv_g, slot, dprod, singular);
            const double par = group_parity(S, L, slot);
            if (live && !singular) {
                clog = log(fabs(dprod));
                csgn = par * (dprod < 0.0 ? -1.0 : 1.0);
            }
            if (live && L.active && slot >= 0) {
#pragma unroll
                for (int k = 0; k < kMaxSpin; ++k) inv_g[slot * kMaxSpin + k] = a[k];
            }
            int slots[kMaxSpin];
#pragma unroll
            for (int ip = 0; ip < kMaxSpin; ++ip) slots[ip] = ip < S.G ? __shfl(slot, L.gbase + ip) : -1;
            __syncthreads();

            // Mt row, g_i and the first trace; A^-1[k][i'] = inv[k][slot(i')]
            ok = live && L.active && !singular;
            if (ok) {
#pragma unroll
                for (int k = 0; k < kMaxSpin; ++k) {
                    if (k >= L.nsig) break;
                    const int mo = occ[k];
                    const double gx = tab[2 * NMO + mo], gy = tab[3 * NMO + mo], gz = tab[4 * NMO + mo];
                    const double *irow = inv_g + k * kMaxSpin;
#pragma unroll
                    for (int ip = 0; ip < kMaxSpin; ++ip) {
                        if (ip >= L.nsig) break;
                        const double v = irow[slots[ip]];
                        Mt[0][ip] += gx * v;
                        Mt[1][ip] += gy * v;
                        Mt[2][ip] += gz * v;
                    }
                    t1 += irow[slot] * tab[NMO + mo];
                }
            }
#pragma unroll
            for (int ip = 0; ip < kMaxSpin; ++ip)
                if (ip == L.i) {
                    g0 = Mt[0][ip];
                    g1 = Mt[1][ip];
                    g2 = Mt[2][ip];
                }
            if (live && L.active) {
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int ip = 0; ip < kMaxSpin; ++ip) mt_g[(L.i * 3 + b) * kMaxSpin + ip] = Mt[b][ip];
            }
        }
        if (live && L.active) {
            double *gp = sGp + (L.grp * G + L.i) * 3;
            gp[0] = g0;
            gp[1] = g1;
            gp[2] = g2;
        }
        __syncthreads();

        // third trace and |grad log D|^2 over this lane's share of the
        // spin's pairs; partial v for the other spin's configuration q
        double t3 = 0.0, gg = 0.0;
        if (ok) {
#pragma unroll
            for (int d = 0; d <= kHalf; ++d) {
                const int ip = own_p[d];
                if (ip < 0) continue;
                const double wt = (d == 0 || 2 * d == L.nsig) ? 1.0 : 2.0;
                const double *y = Yo[d];
                const double *mo_ = mt_g + ip * 3 * kMaxSpin;  // Mt_{i' c, .}
                const double m0 = mo_[L.i], m1 = mo_[kMaxSpin + L.i], m2 = mo_[2 * kMaxSpin + L.i];
                const double *gq = sGp + (L.grp * G + ip) * 3;
                const double yv0 = y[0] * m0 + y[1] * m1 + y[2] * m2;
                const double yv1 = y[3] * m0 + y[4] * m1 + y[5] * m2;
                const double yv2 = y[6] * m0 + y[7] * m1 + y[8] * m2;
                // this lane's own row Mt_{i ., i'} as published
                const double *mr = mt_g + L.i * 3 * kMaxSpin + ip;
                t3 += wt * (mr[0] * yv0 + mr[kMaxSpin] * yv1 + mr[2 * kMaxSpin] * yv2);
                const double w0 = y[0] * gq[0] + y[1] * gq[1] + y[2] * gq[2];
                const double w1 = y[3] * gq[0] + y[4] * gq[1] + y[5] * gq[2];
                const double w2 = y[6] * gq[0] + y[7] * gq[1] + y[8] * gq[2];
                gg += wt * (g0 * w0 + g1 * w1 + g2 * w2);
            }
        }
        if (live && L.active) {  // zeros for a singular configuration
            gtab[3 * q] = g0;
            gtab[3 * q + 1] = g1;
            gtab[3 * q + 2] = g2;
        }
        if (L.active && q < ncfg_o) {
            double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
            for (int t = 0; t < kHalf; ++t) {
                const int ip = oth_p[t];
                if (ip < 0) continue;
                const double *y = Yc[t];
                const double *gq = sGp + ((1 - L.grp) * G + ip) * 3;
                v0 += y[0] * gq[0] + y[1] * gq[1] + y[2] * gq[2];
                v1 += y[3] * gq[0] + y[4] * gq[1] + y[5] * gq[2];
                v2 += y[6] * gq[0] + y[7] * gq[1] + y[8] * gq[2];
            }
            vtab[3 * q] = v0;
            vtab[3 * q + 1] = v1;
            vtab[3 * q + 2] = v2;
        }
        const double Lc = span_sum(ok ? t1 + gg - t3 : 0.0, S.G);
        if (live && L.i == 0) {
            cfg_g[5 * q] = singular ? -INFINITY : clog;
            cfg_g[5 * q + 1] = singular ? 0.0 : csgn;
            cfg_g[5 * q + 3] = singular ? 0.0 : Lc;
        }
        __syncthreads();
    }

    // ---- Sigma, configuration weights ------------------------------------
    double mu = -INFINITY, md = -INFINITY;
    for (int q = L.lw; q < S.n_cfg_up; q += LW) mu = fmax(mu, sCfg[5 * q]);
    for (int q = L.lw; q < S.n_cfg_dn; q += LW) md = fmax(md, sCfg[5 * (S.n_cfg_max + q)]);
    mu = walker_max(mu, LW);
    md = walker_max(md, LW);
    const bool none = mu == -INFINITY || md == -INFINITY;
    // scaled determinant values sign * exp(log|D| - shift)
    for (int q = L.lw; q < S.n_cfg_up + S.n_cfg_dn; q += LW) {
        const int sp = q < S.n_cfg_up ? 0 : 1;
        double *own = sCfg + 5 * (sp * S.n_cfg_max + (sp ? q - S.n_cfg_up : q));
        own[4] = none ? 0.0 : own[1] * exp(own[0] - (sp ? md : mu));
    }
    __syncthreads();
    double Sp = 0.0;
    for (int n = L.lw; n < S.n_det_x; n += LW) {
        const int2 dc = S.det_cfg[n];
        Sp += S.ci_x[n] * sCfg[5 * dc.x + 4] * sCfg[5 * (S.n_cfg_max + dc.y) + 4];
    }
    const double Ssum = walker_sum(Sp, LW);
    const bool zero = none || Ssum == 0.0 || !isfinite(Ssum);
    const double Sinv = zero ? 0.0 : 1.0 / Ssum;
    for (int q = L.lw; q < S.n_cfg_up + S.n_cfg_dn; q += LW) {
        const int sp = q < S.n_cfg_up ? 0 : 1;
        const int cq = sp ? q - S.n_cfg_up : q;
        double *own = sCfg + 5 * (sp * S.n_cfg_max + cq);
        const int *off = S.cfg_off + sp * (S.n_cfg_max + 1);
        double acc = 0.0;
        for (int t = off[cq]; t < off[cq + 1]; ++t) {
            const int2 e = S.cfg_use[t];
            acc += S.ci_x[e.x] * sCfg[5 * ((1 - sp) * S.n_cfg_max + e.y) + 4];
        }
        own[2] = acc * own[4] * Sinv;
    }
    __syncthreads();

    // ---- sum_c W_c L_c, cross term, weighted g ----------------------------
    double lp = 0.0;
    for (int q = L.lw; q < S.n_cfg_up + S.n_cfg_dn; q += LW) {
        const int sp = q < S.n_cfg_up ? 0 : 1;
        const double *own = sCfg + 5 * (sp * S.n_cfg_max + (sp ? q - S.n_cfg_up : q));
        if (own[2] != 0.0) lp += own[2] * own[3];
    }
    double cr = 0.0, gb0 = 0.0, gb1 = 0.0, gb2 = 0.0;
    if (L.active && !zero) {
        // cross term: every lane adds g_i . v_i over its share of the pairs
        // for each determinant.  The loop runs over the determinants in the
        // same order on every lane, unrolled so that several determinants'
        // loads are in flight at once.
        const double *scu = sCfg + 4, *scd = sCfg + 5 * S.n_cfg_max + 4;
        const auto *det_cfg = const_tab((const int *)S.det_cfg);  // (up, down) configuration pairs
        const auto *ci_x = const_tab(S.ci_x);
#pragma unroll 4
        for (int n = 0; n < S.n_det_x; ++n) {
            const int cu = det_cfg[2 * n], cd = det_cfg[2 * n + 1];
            const double w = ci_x[n] * scu[5 * cu] * scd[5 * cd];
            const int own = L.grp ? cd : cu, oth = L.grp ? cu : cd;
            const double gv = gtab[3 * own] * vtab[3 * oth] + gtab[3 * own + 1] * vtab[3 * oth + 1] +
                              gtab[3 * own + 2] * vtab[3 * oth + 2];
            cr += w != 0.0 ? w * gv : 0.0;  // a vanishing weight drops the term whatever g is
        }
        cr *= Sinv;
#pragma unroll 4
        for (int q = 0; q < ncfg_g; ++q) {
            const double wq = cfg_g[5 * q + 2];
            if (wq != 0.0) {
                gb0 += wq * gtab[3 * q];
                gb1 += wq * gtab[3 * q + 1];
                gb2 += wq * gtab[3 * q + 2];
            }
        }
    }
    sGb[3 * L.lw] = gb0;
    sGb[3 * L.lw + 1] = gb1;
    sGb[3 * L.lw + 2] = gb2;
    const double lapS = walker_sum(lp + 2.0 * cr, LW);
    __syncthreads();

    // ---- grad Sigma / Sigma at this electron: sum_i J_ie gbar_i -----------
    double G0 = 0.0, G1 = 0.0, G2 = 0.0;
    if (L.active && !zero) {
        for (int i = 0; i < S.ne; ++i) {
            const int li = lane_of(S, i);
            double B[6];
            if (i == L.e) {
#pragma unroll
                for (int t = 0; t < 6; ++t) B[t] = Jd[t];
            } else {
                jblock_pair(om, xs, sPos + 3 * li, B);
            }
            const double *gi = sGb + 3 * li;
            G0 += B[0] * gi[0] + B[1] * gi[1] + B[2] * gi[2];
            G1 += B[1] * gi[0] + B[3] * gi[1] + B[4] * gi[2];
            G2 += B[2] * gi[0] + B[4] * gi[1] + B[5] * gi[2];
        }
    }
    c.bgS0 = G0;
    c.bgS1 = G1;
    c.bgS2 = G2;
    c.blap = (L.active && L.e == 0) ? lapS : 0.0;
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
