// Device-side system tables and launch helpers shared by the HIP kernels and
// the C ABI host code of libqmc (never by the oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qmc {

// Largest spin block handled by one lane group (lanes per spin = next power
// of two >= max(n_up, n_dn) <= 8).
constexpr int kMaxSpin = 8;
constexpr int kWave = 64;
// Ints per determinant record: (rank, h1, h2, p1, p2) for spin up, then down.
constexpr int kDetInts = 10;

// Streams and events of one walker call: st is the caller's stream; side
// is a second stream and ev[0..3] events (timing off) owned by the system
// handle, used by launches that run on two streams.
struct CallStreams {
    hipStream_t st, side;
    hipEvent_t ev[4];
};

// Everything a kernel needs about one system; passed by value as a kernel
// argument.  Pointers refer to one device allocation owned by the handle.
struct DevSystem {
    int n_up, n_dn, ne, n_atoms, n_shells, n_ao, n_mo, n_det, n_entries;
    int G;    // lanes per spin group (power of two >= max(n_up, n_dn))
    int LW;   // lanes per walker = 2 G
    int WPW;  // walkers per wave = 64 / LW
    int nmo_pad;  // row stride of the MO coefficient tables
    int basis;    // 0 Slater, 1 Gaussian
    int normalize;  // 1: unit-normalised primitives (for exponent derivatives)
    int n_prim;
    double a_par, a_anti, b, vnn;
    const double *atoms;    // [n_atoms][4]: x, y, z, Z
    const int4 *shells;     // [n_shells]: atom, l, kn, nprim
    const double2 *prims;   // [n_prim]: exponent, coefficient x radial normalisation
    const double *mo;       // [n_ao][nmo_pad]: permuted columns, angular factors folded in
    const float *mo_f;      // same, FP32
    const int *dets;        // [n_det][kDetInts]
    const double *ci;       // [n_det], canonicalisation signs folded in
    const int4 *entries;    // [n_entries + 1]: spin, slot k, MO v, first contribution
    const int4 *contribs;   // [n_contrib]: det, cofactor sign (0 = unit), h', p'
    const int *mo_perm;     // [n_mo]: caller's column of each internal MO column
    const double *ao_angf;  // [n_ao]: angular normalisation folded into the MO rows
    // BF16 MFMA operand fragments [2 matrices: C^T, C][2 tiles][hi, lo][64 lanes],
    // 8 bf16 each: lane l of tile t holds M[16 t + l % 16][8 (l / 16) + e].
    const uint4 *mfma_tab;
    // Flattened determinant and cofactor work for the walker's LW lanes.
    // det_recs [det_rows][LW]: (CI weight as two words, up code, down code);
    // cof_recs [cof_rows][LW]: (CI weight, code word, target word).  An
    // excitation code packs rank | h1 << 2 | h2 << 5 | p1 << 8 | p2 << 13; the
    // code word adds the cofactor (0 unit, 1 +T, 2 -T) | h' << 2 | p' << 5
    // shifted by 18; the target word is flush | spin << 1 | k << 2 | v << 5.
    int det_rows, cof_rows;
    const uint4 *det_recs;
    const uint4 *cof_recs;
    // Many-body Jastrow: e-n kernel (w0, w1, w2) per nucleus (nullptr: none)
    // and e-e-n terms (c, a1, b1, a2, b2, a3, b3) x een_n.
    const double *jas_en;
    const double *jas_een;
    int een_n;
    // Explicit-determinant method (comparison path): distinct spin
    // configurations per spin, cfg_occ [2][n_cfg_max][kMaxSpin] internal MO
    // column per slot; det_cfg [n_det_x] (up config, down config) with the
    // caller's CI weights ci_x; per configuration the determinants that use
    // it, cfg_off [2][n_cfg_max + 1] into cfg_use [..] = (det, other-spin
    // config).
    int n_cfg_up, n_cfg_dn, n_cfg_max, n_det_x;
    const int *cfg_occ;
    const int2 *det_cfg;
    const double *ci_x;
    const int *cfg_off;
    const int2 *cfg_use;
    // Inverse backflow kernel omega / r_ij (0: none).
    double bf_omega;
    // Per distinct spin configuration [2][n_cfg_max], its excitation from the
    // reference in canonical order: rank | h0 << 2 | h1 << 5 | p0 << 8 |
    // p1 << 13, bit 20 set when the configuration's column order is an odd
    // permutation of the canonical one, bit 21 when a MO repeats (zero).
    const int *cfg_exc;
};

// Largest number of e-e-n terms.
constexpr int kMaxEen = 8;
// Largest number of distinct spin configurations per spin with backflow.
constexpr int kMaxCfgBF = 128;
// Backflow kernels are compiled for two table sizes: up to kSmallCfgBF
// configurations per spin (smaller private tables per lane) and up to
// kMaxCfgBF.
constexpr int kSmallCfgBF = 48;

}  // namespace qmc
