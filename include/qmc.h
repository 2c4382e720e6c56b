/*
 * qmc.h -- C ABI of the MI355X (gfx950) Slater-Jastrow VMC library.
 *
 * What the library computes (paper: "QMCTorch: Molecular Wavefunctions with
 * Neural Components for Energy and Force Calculations"):
 *   - the molecular Hamiltonian of the Introduction (eq. Hmol), atomic units;
 *   - the Slater-Jastrow wavefunction Psi = exp(J) sum_n d_n D_n^up D_n^dn
 *     of the Methods section (eq. psimol), with Slater or contracted
 *     Cartesian Gaussian AOs (AO layer), MOs phi = sum C chi (MO layer,
 *     C = c * mu), the e-e Pade Jastrow of eq. pade_kernel, and optionally
 *     the inverse backflow transformation (Methods; kernel omega / r_ij of
 *     the Results section) whose local energy follows eq. nabla_d;
 *   - the local energy E_L = H Psi / Psi with the kinetic split of the
 *     appendix on local energies, the Jacobi-trace derivatives of
 *     eq. claudia_trace and the excited-determinant update of eq. table;
 *   - all-electron Metropolis sampling (appendix on optimisation parameters,
 *     Sampling paragraph) whose Monte Carlo mean of E_L estimates the
 *     variational energy (eq. Ev).
 *
 * Conventions.
 *   - Electrons 0..n_up-1 are spin up, n_up..n_up+n_dn-1 spin down.
 *   - Walker positions X are [W][N_e][3] doubles, row-major, bohr.
 *   - Device pointers (prefix d_) are caller-owned device memory on the
 *     system's device; the library never frees them.  Host pointers in the
 *     descriptor are copied at create and may be freed afterwards.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call is asynchronous on that stream; results are valid once the stream
 *     has been synchronised.  Some Metropolis blocks also use a second
 *     stream owned by the handle, forked from and joined back to `stream`
 *     with events inside the call, so the ordering seen by the caller is
 *     that of `stream` alone.
 *   - Calls on one handle from several host threads are serialised while
 *     they enqueue (a mutex in the handle); their device work follows the
 *     streams they were given.
 *   - No call aborts, throws or prints.  Argument checks run before any
 *     launch and return QMC_EINVAL (QMC_ENONFINITE for a NaN or infinite
 *     value where a finite one is required); an unsupported shape returns
 *     QMC_EUNSUPPORTED; a HIP runtime failure returns QMC_EDEVICE.
 *   - Walker data are never an error: a walker whose state has no finite
 *     log|Psi| or E_L (NaN or infinite positions, coincident same-spin
 *     electrons, an exactly singular reference matrix) is reported through
 *     the Metropolis accumulators' non-finite count and left out of their
 *     sums.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMC_OK = 0,
    QMC_EINVAL = -1,        /* invalid argument or descriptor */
    QMC_ENOMEM = -2,        /* device allocation failed */
    QMC_EDEVICE = -3,       /* HIP runtime error (or no device) */
    QMC_EUNSUPPORTED = -4,  /* valid input outside the compiled limits */
    QMC_ENONFINITE = -5     /* a host argument or descriptor value that must be
                               finite is NaN or infinite (nothing launched) */
} qmc_status;

/* Arithmetic of a call.  QMC_FP64: everything in FP64.  The mixed forms
   (Methods, AO and MO layers) evaluate the AO values and derivatives in FP32
   (displacements from the nuclei formed in FP64, then rounded) and the MO
   values phi = sum C chi with FP32 accumulation; everything else is FP64:
   the proposal and accept test, the Pade Jastrow and Coulomb pair terms,
   the Slater inverse and determinant ratios, the cofactors and adjoint
   vectors, the Jacobi-trace contraction of the AO derivatives (AO weights
   t = C a_e and the products t * (grad, lap) chi) and E_L.  They differ in
   the MO value contraction:
     QMC_MIXED_FP32     FP32 vector FMAs;
     QMC_MIXED_BF16     BF16 matrix-core products with FP32 accumulation,
                        each operand split into high and low BF16 parts
                        (hi*hi + hi*lo + lo*hi, about 16 significant bits);
     QMC_MIXED_BF16_X1  one BF16 product per pair (8 significant bits).
   A walker whose kinetic energy from the reduced-precision orbitals is not
   finite or exceeds 3e4 Ha in magnitude is evaluated again with FP64
   orbitals (those are walkers with an electron inside the tightest
   primitives, where cancelling kinetic terms amplify the orbital rounding);
   its results are then the FP64 form's.  The re-evaluation runs in a later
   launch of the same call: until the call completes, the walker's sign entry
   holds a mark (a value >= 4) and the walker is otherwise left as it was,
   so a mixed-form Metropolis call reads each sign entry as its sign
   (> 0: +1, < 0: -1, else 0).  In a Metropolis block a walker re-evaluated
   at some step takes the block's later steps in that later launch (on the
   handle's second stream, one step behind): the results are those of
   single-step calls, only the order of work differs.
   The BF16 forms need n_ao <= 32.
   QMC_FP64_EXPLICIT is FP64 with a different determinant method, kept for
   comparison: every distinct spin configuration of the CI expansion is
   factorised on its own (the explicit evaluation that the low-rank
   excited-determinant scheme of eq. table accelerates).  Its results agree
   with QMC_FP64 to rounding; a walker whose reference matrix is singular but
   whose CI sum is not gets finite values here.  It returns QMC_EUNSUPPORTED
   when the per-walker tables (growing with the number of distinct
   configurations) exceed the 160 KiB of LDS of a compute unit.
   With backflow (bf_omega != 0) only FP64 exists and the mixed forms return
   QMC_EUNSUPPORTED.  QMC_FP64 factorises the reference matrices only and
   updates every configuration from them by the rank <= 2 identity of
   eq. table; QMC_FP64_EXPLICIT factorises every distinct configuration.
   Both evaluate eq. nabla_d with the cross term of eq. delta_sigma and
   agree to rounding. */
typedef enum {
    QMC_FP64 = 0,
    QMC_MIXED_FP32 = 1,
    QMC_MIXED_BF16 = 2,
    QMC_MIXED_BF16_X1 = 3,
    QMC_FP64_EXPLICIT = 4
} qmc_precision;

/* Radial form of every AO: Slater r^kn exp(-zeta r) or contracted
   Gaussians sum_p c_p exp(-alpha_p r^2) (Methods, AO layer). */
typedef enum { QMC_STO = 0, QMC_GTO = 1 } qmc_basis_kind;

typedef struct {
    int32_t n_atoms;
    const double *Z;            /* [n_atoms] nuclear charges */
    const double *R;            /* [n_atoms][3] nuclear positions (bohr) */
    int32_t n_up, n_dn;         /* 0..8 each, n_up + n_dn >= 1 */
    int32_t basis;              /* qmc_basis_kind */
    int32_t n_shells;
    const int32_t *shell_atom;  /* [n_shells] atom of each shell */
    const int32_t *shell_l;     /* [n_shells] angular momentum 0..2 (s, p, Cartesian d) */
    const int32_t *shell_kn;    /* [n_shells] Slater radial power r^kn (0 for GTO) */
    const int32_t *shell_nprim; /* [n_shells] primitives per shell (>= 1) */
    const double *prim_exp;     /* [sum nprim] zeta (STO) or alpha (GTO), > 0 */
    const double *prim_coef;    /* [sum nprim] contraction coefficients */
    int32_t normalize;          /* 1: unit-normalised primitives, 0: raw functions */
    int32_t n_mo;               /* 1..32 */
    const double *mo_coef;      /* [n_ao][n_mo] row-major, the effective c * mu */
    int32_t n_det;              /* >= 1; determinant 0 is the reference */
    const int32_t *occ_up;      /* [n_det][n_up] MO of each column slot */
    const int32_t *occ_dn;      /* [n_det][n_dn] */
    const double *ci;           /* [n_det] CI weights d_n */
    double jas_a_par;           /* Pade numerator for parallel spins (1/4) */
    double jas_a_anti;          /* Pade numerator for antiparallel spins (1/2) */
    double jas_b;               /* Pade denominator parameter (omega), >= 0 */
    /* Many-body terms of eq. jastrow (appendix, many-body Jastrow factor).
       e-n kernel per nucleus: K(r) = (w0 r + w1 r^2) / (1 + w2 r);
       e-e-n kernel: sum over nuclei a and electron pairs i > j (electron
       order as above) of sum_mu c_mu f(a1,b1; r_ai) f(a2,b2; r_aj)
       f(a3,b3; r_ij), f(a,b; r) = a r / (1 + b r).  Denominators must stay
       positive for r >= 0: w2 >= 0 and every b >= 0. */
    const double *jas_en;       /* [n_atoms][3] (w0, w1, w2), or NULL: no e-n term */
    int32_t jas_een_n;          /* e-e-n terms, 0..8 (0: none) */
    const double *jas_een;      /* [jas_een_n][7] (c, a1, b1, a2, b2, a3, b3) */
    /* Inverse backflow (Methods, backflow transformation; kernel of the
       Results section): the orbitals are evaluated at
       q_i = r_i + sum_{j != i} (bf_omega / r_ij) (r_i - r_j), the Jastrow
       factor and the potential at the bare positions.  0: no backflow.
       With backflow every determinant depends on every electron; E_L then
       uses eq. nabla_d per spin block and the cross term of eq. delta_sigma,
       per distinct spin configuration (at most 128 per spin; see
       qmc_precision for the two methods). */
    double bf_omega;
} qmc_system_desc;

typedef struct qmc_system qmc_system;

/* Builds a device-resident system on HIP device `device`.  AO order: shells
   in order; within a shell Cartesian components lexicographic with the
   x-power first (x, y, z; xx, xy, xz, yy, yz, zz).  Every determinant must
   differ from the reference by at most two orbitals per spin (single and
   double excitations, eq. table with k <= 2), and the reference occupations
   of the two spins must agree on their common slots.  *out is set only on
   QMC_OK. */
qmc_status qmc_system_create(const qmc_system_desc *desc, int32_t device, qmc_system **out);

/* Frees the system and its device tables.  NULL is ignored. */
void qmc_system_destroy(qmc_system *sys);

/* log|Psi|, sign(Psi) and E_L of W walkers.
   d_X [W][N_e][3]; d_logpsi, d_sign, d_eloc [W].  W = 0 is a no-op.  A walker
   whose reference determinant is exactly singular gets log|Psi| = -inf,
   sign = 0 and E_L = NaN. */
qmc_status qmc_eval_psi_eloc(qmc_system *sys, int32_t precision, const double *d_X, int64_t W,
                             double *d_logpsi, double *d_sign, double *d_eloc, void *stream);

/* n_steps all-electron Metropolis moves of W walkers, in place.
   Walker w at step t = step0 + s proposes X' = X + sigma z with z the
   Box-Muller normals of Philox4x32-10 (key = seed; counter = (walker_offset
   + w, t low word, t high word, electron)); it accepts when
   u < exp(2 (log|Psi'| - log|Psi|)), u from counter word 3 = N_e, and then
   takes (X', log|Psi'|, sign', E_L').  On entry d_logpsi, d_sign and d_eloc
   must describe d_X (e.g. from qmc_eval_psi_eloc).  d_acc [W][4] gains, per
   step, from the post-decision state: (E_L, E_L^2, accepted, 0) when its
   log|Psi| and E_L are finite, else (0, 0, accepted, 1): column 3 counts the
   steps left out of the sums.  The caller zeroes d_acc before a block's
   first call.  Results depend only on (seed, walker_offset + w, t), never on
   W or on how walkers are batched.  sigma must be finite (QMC_ENONFINITE)
   and >= 0 (QMC_EINVAL).  Enqueued as one kernel per step (the arrays carry
   the state between them; a mixed form adds its re-evaluation kernels, on
   the handle's second stream for blocks of more than 8192 waves of walkers,
   else on `stream`), except QMC_FP64_EXPLICIT and blocks of at most 1024
   waves without backflow: one kernel with the step loop inside.  An FP64
   block of at least 1536 waves runs its walkers in two halves, one on
   `stream` and one on the second stream.  (A wave holds 64 / (2 G) walkers,
   G the next power of two >= max(n_up, n_dn).)  The results do not depend
   on these choices. */
qmc_status qmc_metropolis_block(qmc_system *sys, int32_t precision, double *d_X, double *d_logpsi,
                                double *d_sign, double *d_eloc, int64_t W, int32_t n_steps,
                                double sigma, uint64_t seed, uint64_t step0,
                                uint32_t walker_offset, double *d_acc, void *stream);

/* log|Psi| and E_L of W walkers with the kinetic energy from central finite
   differences of Psi instead of the Jacobi-trace formulas (the baseline
   that eqs. claudia_trace / nabla_d replace; the paper's own baseline is
   automatic differentiation, Fig. kinetic_bench): Psi is evaluated at x and
   at x +- h e_c for each of the 3 N_e coordinates, and
   lap Psi / Psi = sum_c (Psi(x + h e_c) - 2 Psi(x) + Psi(x - h e_c)) / (h^2 Psi(x)).
   FP64 with the low-rank determinants; truncation error O(h^2), rounding
   error O(eps / h^2).  d_X as in qmc_eval_psi_eloc; d_logpsi, d_eloc [W].
   h must be finite and positive (QMC_EINVAL otherwise); systems with
   backflow return QMC_EUNSUPPORTED.  A walker whose reference determinant
   is exactly singular gets log|Psi| = -inf and E_L = NaN. */
qmc_status qmc_eval_eloc_fd(qmc_system *sys, const double *d_X, int64_t W, double h, double *d_logpsi,
                            double *d_eloc, void *stream);

/* Per-walker derivatives for the optimiser and for forces, FP64 (Methods:
   eq. nabla_loss needs d log|Psi| / d theta, eq. force needs d E_L / d R and
   d ln rho / d R = 2 d log|Psi| / d R).  theta is laid out as
   [primitive exponents in descriptor order | MO coefficients [n_ao][n_mo] in
   the descriptor's layout | jas_b | jas_en [n_atoms][3] when given |
   jas_een [jas_een_n][7] when given], qmc_param_count entries; the exponent
   derivatives include the normalisation's dependence when normalize = 1,
   and the nuclear derivatives include the e-n and e-e-n Jastrow terms'
   dependence on the nuclei.
     d_dlogpsi      [W][P]  d log|Psi| / d theta
     d_deloc_dtheta [W][P]  d E_L / d theta
     d_dlogpsi_dR   [W][n_atoms][3]  d log|Psi| / d R_alpha
     d_deloc_dR     [W][n_atoms][3]  d E_L / d R_alpha (includes V_nn)
   Any output may be NULL; at least one must not be.  d_X as in
   qmc_eval_psi_eloc.  precision: QMC_FP64, or QMC_MIXED_FP32 (the AO values
   and the MO value contraction of the forward evaluation in FP32, as in
   qmc_eval_psi_eloc's mixed form without its FP64 re-evaluation; every
   derivative pass FP64); the other forms return QMC_EUNSUPPORTED, a value
   outside qmc_precision QMC_EINVAL.  Returns QMC_EUNSUPPORTED when the
   walker tables do not fit the 160 KiB of LDS of a compute unit and for
   systems with backflow. */
qmc_status qmc_grad(qmc_system *sys, int32_t precision, const double *d_X, int64_t W, double *d_dlogpsi,
                    double *d_deloc_dtheta, double *d_dlogpsi_dR, double *d_deloc_dR, void *stream);

/* Number of variational parameters in the qmc_grad layout. */
int64_t qmc_param_count(const qmc_system *sys);

/* Device bytes one walker occupies across a Metropolis block (positions,
   log|Psi|, sign, E_L, the four accumulators), for admission control. */
size_t qmc_bytes_per_walker(const qmc_system *sys, int32_t precision);

/* Reduction of a block's accumulators over its walkers (the Monte Carlo
   estimate of eq. Ev): d_out[5] = (sum of column 0, sum of column 1, sum of
   column 2, sum of column 3, number of walkers with a non-zero column 3) of
   d_acc [W][4].  The summation order is fixed by W alone (a strided
   sequential pass per thread of one work-group, then a fixed binary tree),
   so the result is the same for the same accumulators wherever and however
   they were produced.  Mean energy = d_out[0] / (W n_steps - d_out[3]).
   d_out is caller-owned device memory; asynchronous on `stream`; W = 0
   writes zeros.  No workspace. */
qmc_status qmc_reduce_accumulators(const double *d_acc, int64_t W, double *d_out, void *stream);

/* Static text for a status code. */
const char *qmc_status_string(qmc_status status);

#ifdef __cplusplus
}
#endif
#endif
