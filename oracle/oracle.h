/*
 * FP64 CPU oracle for Slater-Jastrow VMC: test infrastructure only.
 *
 * This library is the slow, plain reference that the HIP path is checked
 * against.  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline may call it; the product path never does.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Every determinant of the CI expansion is evaluated explicitly (pivoted LU,
 * explicit inverse, Jacobi traces), i.e. the definition that the paper's
 * low-rank excited-determinant update reaches faster.
 */
#ifndef QMC_ORACLE_H
#define QMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n_atoms;
    const double *Z;          /* [n_atoms] */
    const double *R;          /* [n_atoms][3] bohr */
    int n_up, n_dn;           /* electrons 0..n_up-1 are spin up */
    int basis;                /* 0 = Slater (STO), 1 = contracted Gaussian (GTO) */
    int n_shells;
    const int *shell_atom, *shell_l, *shell_kn, *shell_nprim;
    const double *prim_exp, *prim_coef;   /* concatenated over shells */
    int normalize;            /* 1: unit-normalised primitives */
    int n_mo;
    const double *mo_coef;    /* [n_ao][n_mo] */
    int n_det;
    const int *occ_up;        /* [n_det][n_up] MO per column slot */
    const int *occ_dn;        /* [n_det][n_dn] */
    const double *ci;         /* [n_det] */
    double a_par, a_anti, b;  /* Pade e-e Jastrow */
    const double *en;         /* [n_atoms][3] e-n kernel (omega0, omega1, omega2)
                                 per nucleus; NULL: no e-n term */
    int een_n;                /* terms of the e-e-n kernel; 0: none */
    const double *een;        /* [een_n][7]: c, a1, b1, a2, b2, a3, b3 */
    double bf_omega;          /* inverse backflow kernel omega / r_ij; 0: none */
} or_system;

/* Per-walker detail of one evaluation. */
typedef struct {
    double logpsi, sign, eloc;
    double e_kin, e_pot;      /* eloc = e_kin + e_pot */
    double jastrow;           /* J */
    double log_sigma;         /* log|sum_n d_n D_n^up D_n^dn| */
} or_detail;

int    or_n_ao(const or_system *s);
double or_nuclear_repulsion(const or_system *s);

/* AO value, d/dx, d/dy, d/dz, Laplacian at one point: out[n_ao][5]. */
void or_ao(const or_system *s, const double r[3], double *out);

/* AO value, gradient and Hessian at one point: out[n_ao][10] = value, dx, dy,
   dz, xx, xy, xz, yy, yz, zz. */
void or_ao_hessian(const or_system *s, const double r[3], double *out);

/* Backflow-transformed positions q[N_e][3] of x[N_e][3]. */
void or_backflow(const or_system *s, const double *x, double *q);

/* MO values of every electron: out[N_e][5][n_mo] (value, dx, dy, dz, lap). */
void or_mo(const or_system *s, const double *x, double *out);

/* One walker, x[N_e][3].  grad (nullable): d log|Psi| / d x, [N_e][3]. */
void or_eval_one(const or_system *s, const double *x, or_detail *out, double *grad);

/* Batch over walkers with OpenMP; X[W][N_e][3].  nthreads <= 0: default. */
void or_eval(const or_system *s, const double *X, int64_t W, double *logpsi,
             double *sign, double *eloc, int nthreads);

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Gaussian proposal of one walker-step: z[N_e][3], and the accept uniform. */
void or_proposal(int n_elec, uint64_t seed, uint32_t walker_id, uint64_t step,
                 double *z, double *u_accept);

/* Metropolis block: n_steps all-electron moves per walker.  acc[W][4] gains
   (sum E_L, sum E_L^2, accepted count, non-finite count) of the
   post-decision state: a state whose log|Psi| or E_L is not finite adds 1 to
   the last column and nothing to the sums.
   accept_log (nullable) receives [n_steps][W] bytes. */
void or_metropolis(const or_system *s, double *X, double *logpsi, double *sign,
                   double *eloc, int64_t W, int n_steps, double sigma,
                   uint64_t seed, uint64_t step0, uint32_t walker_offset,
                   double *acc, uint8_t *accept_log, int nthreads);

int or_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
