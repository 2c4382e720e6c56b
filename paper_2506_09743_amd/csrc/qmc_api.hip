// C ABI of libqmc: descriptor validation, host-side table construction
// (normalisation, MO column permutation, excitation canonicalisation,
// cofactor contribution lists), device residency and kernel launches.

#include "../../include/qmc.h"
#include "qmc_device.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

namespace qmc {
hipError_t launch_walkers(bool mc, int form, const DevSystem &S, double *X, double *LP, double *SG,
                          double *EL, int64_t W, int n_steps, double sigma, uint64_t seed,
                          uint64_t step0, uint32_t woff, double *ACC, const CallStreams &cs);
int padded_mo(int n_mo);
hipError_t launch_grad(const DevSystem &S, const double *X, int64_t W, double *dlogpsi,
                       double *deloc_dth, double *dlogpsi_dR, double *deloc_dR, int n_param, bool mixed,
                       hipStream_t st);
size_t grad_lds_bytes(const DevSystem &S);
size_t explicit_lds_bytes(const DevSystem &S);
size_t backflow_lds_bytes(const DevSystem &S, bool low_rank);
hipError_t launch_eval_fd(const DevSystem &S, const double *X, int64_t W, double h, double *LP, double *EL,
                          hipStream_t st);
hipError_t launch_reduce_acc(const double *acc, int64_t W, double *out, hipStream_t st);
}  // namespace qmc

using qmc::DevSystem;

struct qmc_system {
    int device;
    DevSystem S;
    void *d_mem;        // one allocation holding every table
    int n_prim;
    int64_t n_params;
    // second stream and events of the two-stream launches; the mutex keeps
    // calls from several host threads from interleaving their use
    hipStream_t side = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::mutex mu;
};

namespace {

constexpr double kPi = 3.14159265358979323846;

double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

double dfactorial(int n) {  // n!!, (-1)!! = 1
    double f = 1.0;
    for (int i = n; i > 1; i -= 2) f *= i;
    return f;
}

// Unit norm over R^3 of x^a y^b z^c R(r), split into a radial factor (per
// primitive) and an angular factor (per Cartesian component).  Slater:
// radial^2 = (2 zeta)^(2n+1) / (2n)! * (2l+1)!! / (4 pi), n = l + kn + 1.
// Gaussian: radial = (2 alpha / pi)^(3/4) (4 alpha)^(l/2).  Angular:
// 1 / sqrt((2a-1)!! (2b-1)!! (2c-1)!!).
double radial_norm(int basis, int l, int kn, double e) {
    if (basis == QMC_STO) {
        const int n = l + kn + 1;
        return sqrt(pow(2.0 * e, 2 * n + 1) / factorial(2 * n) * dfactorial(2 * l + 1) / (4.0 * kPi));
    }
    return pow(2.0 * e / kPi, 0.75) * pow(4.0 * e, 0.5 * l);
}

double angular_norm(int a, int b, int c) {
    return 1.0 / sqrt(dfactorial(2 * a - 1) * dfactorial(2 * b - 1) * dfactorial(2 * c - 1));
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool is_finite(double v) { return std::isfinite(v); }

// Canonical excitation of one spin of one determinant relative to the
// reference (after the MO permutation, reference slot k holds MO k).
struct Excitation {
    int rank = 0;
    int h[2] = {0, 0};
    int p[2] = {0, 0};
};

// Returns 0 if the determinant is identically zero (repeated MO), -1 if the
// rank exceeds 2, else 1; *sign is the parity taking the given column order
// to the canonical one (holes ascending, particles ascending in hole order).
int canonical_excitation(const std::vector<int> &occ, int n, Excitation *ex, double *sign) {
    std::vector<int> sorted(occ);
    std::sort(sorted.begin(), sorted.end());
    for (int k = 1; k < n; ++k)
        if (sorted[k] == sorted[k - 1]) return 0;
    std::vector<char> present(n, 0);
    std::vector<int> parts;
    for (int k = 0; k < n; ++k) {
        if (occ[k] < n)
            present[occ[k]] = 1;
        else
            parts.push_back(occ[k]);
    }
    std::vector<int> holes;
    for (int k = 0; k < n; ++k)
        if (!present[k]) holes.push_back(k);
    if ((int)holes.size() > 2) return -1;
    std::sort(parts.begin(), parts.end());
    std::vector<int> canon(n);
    for (int k = 0; k < n; ++k) canon[k] = k;
    for (size_t a = 0; a < holes.size(); ++a) canon[holes[a]] = parts[a];
    // parity of the permutation mapping occ -> canon (both hold distinct values)
    std::map<int, int> pos;
    for (int k = 0; k < n; ++k) pos[canon[k]] = k;
    std::vector<int> perm(n);
    for (int k = 0; k < n; ++k) perm[k] = pos[occ[k]];
    int swaps = 0;
    for (int k = 0; k < n; ++k)
        while (perm[k] != k) {
            std::swap(perm[k], perm[perm[k]]);
            ++swaps;
        }
    *sign = (swaps & 1) ? -1.0 : 1.0;
    ex->rank = (int)holes.size();
    for (size_t a = 0; a < holes.size(); ++a) {
        ex->h[a] = holes[a];
        ex->p[a] = parts[a];
    }
    return 1;
}

qmc_status validate(const qmc_system_desc *d) {
    if (!d) return QMC_EINVAL;
    if (d->n_atoms < 1 || !d->Z || !d->R) return QMC_EINVAL;
    if (d->n_up < 0 || d->n_dn < 0 || d->n_up + d->n_dn < 1) return QMC_EINVAL;
    if (d->basis != QMC_STO && d->basis != QMC_GTO) return QMC_EINVAL;
    if (d->n_shells < 1 || !d->shell_atom || !d->shell_l || !d->shell_kn || !d->shell_nprim)
        return QMC_EINVAL;
    if (!d->prim_exp || !d->prim_coef || !d->mo_coef || !d->ci) return QMC_EINVAL;
    if (d->n_up > 0 && !d->occ_up) return QMC_EINVAL;
    if (d->n_dn > 0 && !d->occ_dn) return QMC_EINVAL;
    if (d->n_mo < 1 || d->n_det < 1) return QMC_EINVAL;
    if (d->normalize != 0 && d->normalize != 1) return QMC_EINVAL;
    for (int a = 0; a < d->n_atoms; ++a) {
        if (!is_finite(d->Z[a]) || !is_finite(d->R[3 * a]) || !is_finite(d->R[3 * a + 1]) || !is_finite(d->R[3 * a + 2]))
            return QMC_ENONFINITE;
    }
    int n_prim = 0;
    for (int s = 0; s < d->n_shells; ++s) {
        if (d->shell_atom[s] < 0 || d->shell_atom[s] >= d->n_atoms) return QMC_EINVAL;
        if (d->shell_l[s] < 0 || d->shell_kn[s] < 0 || d->shell_nprim[s] < 1) return QMC_EINVAL;
        if (d->basis == QMC_GTO && d->shell_kn[s] != 0) return QMC_EINVAL;
        n_prim += d->shell_nprim[s];
    }
    for (int p = 0; p < n_prim; ++p) {
        if (!is_finite(d->prim_exp[p]) || !is_finite(d->prim_coef[p])) return QMC_ENONFINITE;
        if (!(d->prim_exp[p] > 0.0)) return QMC_EINVAL;
    }
    int n_ao = 0;
    for (int s = 0; s < d->n_shells; ++s) n_ao += (d->shell_l[s] + 1) * (d->shell_l[s] + 2) / 2;
    for (int64_t q = 0; q < (int64_t)n_ao * d->n_mo; ++q)
        if (!is_finite(d->mo_coef[q])) return QMC_ENONFINITE;
    for (int n = 0; n < d->n_det; ++n) {
        if (!is_finite(d->ci[n])) return QMC_ENONFINITE;
        for (int k = 0; k < d->n_up; ++k)
            if (d->occ_up[n * d->n_up + k] < 0 || d->occ_up[n * d->n_up + k] >= d->n_mo) return QMC_EINVAL;
        for (int k = 0; k < d->n_dn; ++k)
            if (d->occ_dn[n * d->n_dn + k] < 0 || d->occ_dn[n * d->n_dn + k] >= d->n_mo) return QMC_EINVAL;
    }
    if (!is_finite(d->jas_a_par) || !is_finite(d->jas_a_anti) || !is_finite(d->jas_b)) return QMC_ENONFINITE;
    if (d->jas_b < 0.0) return QMC_EINVAL;
    if (d->jas_en)
        for (int a = 0; a < d->n_atoms; ++a) {
            const double *w = d->jas_en + 3 * a;
            if (!is_finite(w[0]) || !is_finite(w[1]) || !is_finite(w[2])) return QMC_ENONFINITE;
            if (w[2] < 0.0) return QMC_EINVAL;
        }
    if (d->jas_een_n < 0 || d->jas_een_n > qmc::kMaxEen) return QMC_EINVAL;
    if (d->jas_een_n > 0 && !d->jas_een) return QMC_EINVAL;
    for (int m = 0; m < d->jas_een_n; ++m)
        for (int k = 0; k < 7; ++k) {
            const double v = d->jas_een[7 * m + k];
            if (!is_finite(v)) return QMC_ENONFINITE;
            if ((k == 2 || k == 4 || k == 6) && v < 0.0) return QMC_EINVAL;
        }
    if (!is_finite(d->bf_omega)) return QMC_ENONFINITE;
    return QMC_OK;
}

uint16_t to_bf16(float f) {  // round to nearest even
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float from_bf16(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// Operand fragments of the matrix-core contractions: matrix 0 = C^T (rows
// MOs, columns AOs), matrix 1 = C (rows AOs, columns MOs), both padded to
// 32 x 32; fragment (tile t, lane l) holds M[16 t + l % 16][8 (l / 16) + e],
// e = 0..7, as high and low BF16 parts.
std::vector<uint4> mfma_fragments(const std::vector<double> &mo, int n_ao, int n_mo, int stride) {
    std::vector<uint4> tab(2 * 2 * 2 * 64);
    for (int mat = 0; mat < 2; ++mat)
        for (int t = 0; t < 2; ++t)
            for (int part = 0; part < 2; ++part)
                for (int l = 0; l < 64; ++l) {
                    uint16_t h[8];
                    for (int e = 0; e < 8; ++e) {
                        const int row = 16 * t + l % 16, col = 8 * (l / 16) + e;
                        const int ao = mat == 0 ? col : row, m = mat == 0 ? row : col;
                        const double x = (ao < n_ao && m < n_mo) ? mo[(size_t)ao * stride + m] : 0.0;
                        const uint16_t hi = to_bf16((float)x);
                        h[e] = part == 0 ? hi : to_bf16((float)(x - (double)from_bf16(hi)));
                    }
                    uint4 v;
                    v.x = h[0] | ((uint32_t)h[1] << 16);
                    v.y = h[2] | ((uint32_t)h[3] << 16);
                    v.z = h[4] | ((uint32_t)h[5] << 16);
                    v.w = h[6] | ((uint32_t)h[7] << 16);
                    tab[((mat * 2 + t) * 2 + part) * 64 + l] = v;
                }
    return tab;
}

template <typename T>
size_t push_bytes(std::vector<unsigned char> &blob, const T *src, size_t count) {
    size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + sizeof(T) * count);
    if (count) memcpy(blob.data() + off, src, sizeof(T) * count);
    return off;
}

}  // namespace

extern "C" {

const char *qmc_status_string(qmc_status s) {
    switch (s) {
        case QMC_OK: return "ok";
        case QMC_EINVAL: return "invalid argument";
        case QMC_ENOMEM: return "device allocation failed";
        case QMC_EDEVICE: return "HIP device error";
        case QMC_EUNSUPPORTED: return "unsupported by this build";
        case QMC_ENONFINITE: return "non-finite argument";
    }
    return "unknown status";
}

qmc_status qmc_system_create(const qmc_system_desc *d, int32_t device, qmc_system **out) {
    if (!out) return QMC_EINVAL;
    qmc_status st = validate(d);
    if (st != QMC_OK) return st;
    const int nu = d->n_up, nd = d->n_dn, ne = nu + nd;
    if (nu > qmc::kMaxSpin || nd > qmc::kMaxSpin) return QMC_EUNSUPPORTED;
    for (int s = 0; s < d->n_shells; ++s)
        if (d->shell_l[s] > 2) return QMC_EUNSUPPORTED;
    const int nmo_pad = qmc::padded_mo(d->n_mo);
    if (nmo_pad < 0 || d->n_mo < std::max(nu, nd)) return QMC_EUNSUPPORTED;

    // --- MO permutation putting the reference orbitals first ----------------
    const int *ref_long = nu >= nd ? d->occ_up : d->occ_dn;
    const int *ref_short = nu >= nd ? d->occ_dn : d->occ_up;
    const int n_long = std::max(nu, nd), n_short = std::min(nu, nd);
    for (int k = 0; k < n_short; ++k)
        if (ref_long[k] != ref_short[k]) return QMC_EUNSUPPORTED;
    std::vector<int> new_of_old(d->n_mo, -1), old_of_new;
    for (int k = 0; k < n_long; ++k) {
        if (new_of_old[ref_long[k]] >= 0) return QMC_EUNSUPPORTED;  // reference det vanishes
        new_of_old[ref_long[k]] = k;
        old_of_new.push_back(ref_long[k]);
    }
    for (int m = 0; m < d->n_mo; ++m)
        if (new_of_old[m] < 0) {
            new_of_old[m] = (int)old_of_new.size();
            old_of_new.push_back(m);
        }

    // --- canonical excitations, folded signs ----------------------------------
    std::vector<int> dets;
    std::vector<double> ci;
    std::vector<Excitation> ex_up, ex_dn;
    for (int n = 0; n < d->n_det; ++n) {
        Excitation eu, ed;
        double su = 1.0, sd = 1.0;
        std::vector<int> ou(nu), od(nd);
        for (int k = 0; k < nu; ++k) ou[k] = new_of_old[d->occ_up[n * nu + k]];
        for (int k = 0; k < nd; ++k) od[k] = new_of_old[d->occ_dn[n * nd + k]];
        int ru = canonical_excitation(ou, nu, &eu, &su);
        int rd = canonical_excitation(od, nd, &ed, &sd);
        if (ru < 0 || rd < 0) return QMC_EUNSUPPORTED;
        if (ru == 0 || rd == 0) continue;  // identically zero determinant
        if (n == 0 && (eu.rank != 0 || ed.rank != 0)) return QMC_EUNSUPPORTED;
        ex_up.push_back(eu);
        ex_dn.push_back(ed);
        ci.push_back(d->ci[n] * su * sd);
        const Excitation *e2[2] = {&eu, &ed};
        for (int s = 0; s < 2; ++s) {
            dets.push_back(e2[s]->rank);
            dets.push_back(e2[s]->h[0]);
            dets.push_back(e2[s]->h[1]);
            dets.push_back(e2[s]->p[0]);
            dets.push_back(e2[s]->p[1]);
        }
    }
    const int n_det = (int)ci.size();

    // --- distinct spin configurations for the explicit method ----------------
    std::map<std::vector<int>, int> cfg_id[2];
    std::vector<std::vector<int>> cfgs[2];
    std::vector<int2> det_cfg;
    std::vector<double> ci_x;
    for (int n = 0; n < d->n_det; ++n) {
        int id[2];
        bool repeated = false;
        for (int s = 0; s < 2; ++s) {
            const int ns = s == 0 ? nu : nd;
            const int *occ = s == 0 ? d->occ_up + n * nu : d->occ_dn + n * nd;
            std::vector<int> c(ns);
            for (int k = 0; k < ns; ++k) c[k] = new_of_old[occ[k]];
            std::vector<int> sorted = c;
            std::sort(sorted.begin(), sorted.end());
            if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) repeated = true;
            auto it = cfg_id[s].find(c);
            if (it == cfg_id[s].end()) {
                it = cfg_id[s].emplace(c, (int)cfgs[s].size()).first;
                cfgs[s].push_back(c);
            }
            id[s] = it->second;
        }
        if (repeated) continue;  // identically zero determinant
        det_cfg.push_back(make_int2(id[0], id[1]));
        ci_x.push_back(d->ci[n]);
    }
    const int n_cfg_max = (int)std::max(cfgs[0].size(), cfgs[1].size());
    std::vector<int> cfg_occ(2 * n_cfg_max * qmc::kMaxSpin, 0);
    // canonical excitation of every configuration (low-rank backflow)
    std::vector<int> cfg_exc(2 * n_cfg_max, 0);
    for (int s = 0; s < 2; ++s)
        for (size_t q = 0; q < cfgs[s].size(); ++q) {
            Excitation ex;
            double sg = 1.0;
            const int r = canonical_excitation(cfgs[s][q], (int)cfgs[s][q].size(), &ex, &sg);
            if (r < 0) return QMC_EUNSUPPORTED;
            int code = 1 << 21;  // repeated MO: identically zero
            if (r > 0)
                code = ex.rank | ex.h[0] << 2 | ex.h[1] << 5 | ex.p[0] << 8 | ex.p[1] << 13 | (sg < 0.0 ? 1 << 20 : 0);
            cfg_exc[s * n_cfg_max + q] = code;
        }
    for (int s = 0; s < 2; ++s)
        for (size_t q = 0; q < cfgs[s].size(); ++q)
            for (size_t k = 0; k < cfgs[s][q].size(); ++k) cfg_occ[(s * n_cfg_max + q) * qmc::kMaxSpin + k] = cfgs[s][q][k];
    std::vector<int> cfg_off(2 * (n_cfg_max + 1), 0);
    std::vector<int2> cfg_use;
    for (int s = 0; s < 2; ++s) {
        std::vector<std::vector<int2>> use(n_cfg_max);
        for (size_t n = 0; n < det_cfg.size(); ++n) {
            const int own = s == 0 ? det_cfg[n].x : det_cfg[n].y, oth = s == 0 ? det_cfg[n].y : det_cfg[n].x;
            use[own].push_back(make_int2((int)n, oth));
        }
        for (int q = 0; q < n_cfg_max; ++q) {
            cfg_off[s * (n_cfg_max + 1) + q] = (int)cfg_use.size();
            cfg_use.insert(cfg_use.end(), use[q].begin(), use[q].end());
        }
        cfg_off[s * (n_cfg_max + 1) + n_cfg_max] = (int)cfg_use.size();
    }

    // --- cofactor contribution lists: C_s[k][v] = dS / dT_s[k][v] -------------
    // key (spin, k, v) -> contributions (det, sign, h', p'); sign 0 = unit cofactor
    std::map<std::tuple<int, int, int>, std::vector<int4>> ent;
    for (int n = 0; n < n_det; ++n) {
        const Excitation *e2[2] = {&ex_up[n], &ex_dn[n]};
        for (int s = 0; s < 2; ++s) {
            const Excitation &e = *e2[s];
            if (e.rank == 1) {
                ent[std::make_tuple(s, e.h[0], e.p[0])].push_back(make_int4(n, 0, 0, 0));
            } else if (e.rank == 2) {
                ent[std::make_tuple(s, e.h[0], e.p[0])].push_back(make_int4(n, 1, e.h[1], e.p[1]));
                ent[std::make_tuple(s, e.h[1], e.p[1])].push_back(make_int4(n, 1, e.h[0], e.p[0]));
                ent[std::make_tuple(s, e.h[0], e.p[1])].push_back(make_int4(n, -1, e.h[1], e.p[0]));
                ent[std::make_tuple(s, e.h[1], e.p[0])].push_back(make_int4(n, -1, e.h[0], e.p[1]));
            }
        }
    }
    // flattened records (see DevSystem): the walker's LW lanes get entries by
    // greedy longest-first packing so every lane runs the same trip count
    int G = 1;
    while (G < std::max(nu, nd)) G <<= 1;
    const int LW = 2 * G;
    auto exc_code = [](const Excitation &e) {
        return (uint32_t)e.rank | ((uint32_t)e.h[0] << 2) | ((uint32_t)e.h[1] << 5) |
               ((uint32_t)e.p[0] << 8) | ((uint32_t)e.p[1] << 13);
    };
    auto ci_words = [](double c, uint32_t *lo, uint32_t *hi) {
        uint64_t u;
        memcpy(&u, &c, 8);
        *lo = (uint32_t)u;
        *hi = (uint32_t)(u >> 32);
    };
    const int det_rows = (n_det + LW - 1) / LW;
    std::vector<uint4> det_recs((size_t)det_rows * LW, make_uint4(0, 0, 0, 0));
    for (int n = 0; n < n_det; ++n) {
        uint4 r;
        ci_words(ci[n], &r.x, &r.y);
        r.z = exc_code(ex_up[n]);
        r.w = exc_code(ex_dn[n]);
        det_recs[(size_t)(n / LW) * LW + n % LW] = r;
    }
    std::vector<std::vector<uint4>> lane_lists(LW);
    {
        std::vector<std::pair<std::tuple<int, int, int>, const std::vector<int4> *>> order;
        for (auto &kv : ent) order.push_back({kv.first, &kv.second});
        std::stable_sort(order.begin(), order.end(),
                         [](const auto &a, const auto &b) { return a.second->size() > b.second->size(); });
        for (auto &o : order) {
            int best = 0;
            for (int l = 1; l < LW; ++l)
                if (lane_lists[l].size() < lane_lists[best].size()) best = l;
            const int spin = std::get<0>(o.first), k = std::get<1>(o.first), v = std::get<2>(o.first);
            const std::vector<int4> &cl = *o.second;
            for (size_t q = 0; q < cl.size(); ++q) {
                const int4 cb = cl[q];
                const Excitation &other = spin == 0 ? ex_dn[cb.x] : ex_up[cb.x];
                uint32_t cof = 0;
                if (cb.y != 0) cof = (cb.y > 0 ? 1u : 2u) | ((uint32_t)cb.z << 2) | ((uint32_t)cb.w << 5);
                uint4 r;
                ci_words(ci[cb.x], &r.x, &r.y);
                r.z = exc_code(other) | (cof << 18);
                r.w = (q + 1 == cl.size() ? 1u : 0u) | ((uint32_t)spin << 1) | ((uint32_t)k << 2) |
                      ((uint32_t)v << 5);
                lane_lists[best].push_back(r);
            }
        }
    }
    size_t cof_rows = 0;
    for (auto &l : lane_lists) cof_rows = std::max(cof_rows, l.size());
    std::vector<uint4> cof_recs(cof_rows * LW, make_uint4(0, 0, 0, 0));
    for (int l = 0; l < LW; ++l)
        for (size_t i = 0; i < lane_lists[l].size(); ++i) cof_recs[i * LW + l] = lane_lists[l][i];

    std::vector<int4> entries, contribs;
    for (auto &kv : ent) {
        entries.push_back(make_int4(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                                    (int)contribs.size()));
        for (const int4 &c : kv.second) contribs.push_back(c);
    }
    entries.push_back(make_int4(0, 0, 0, (int)contribs.size()));
    const int n_entries = (int)entries.size() - 1;

    // --- basis tables -------------------------------------------------------
    std::vector<int4> shells;
    std::vector<double2> prims;
    std::vector<double> angf;  // per AO angular factor
    int p0 = 0;
    for (int s = 0; s < d->n_shells; ++s) {
        const int l = d->shell_l[s], kn = d->shell_kn[s], np = d->shell_nprim[s];
        shells.push_back(make_int4(d->shell_atom[s], l, kn, np));
        for (int q = 0; q < np; ++q) {
            const double e = d->prim_exp[p0 + q];
            const double c = d->prim_coef[p0 + q] * (d->normalize ? radial_norm(d->basis, l, kn, e) : 1.0);
            prims.push_back(make_double2(e, c));
        }
        p0 += np;
        for (int a = l; a >= 0; --a)
            for (int b = l - a; b >= 0; --b) angf.push_back(d->normalize ? angular_norm(a, b, l - a - b) : 1.0);
    }
    const int n_ao = (int)angf.size();
    std::vector<double> mo((size_t)n_ao * nmo_pad, 0.0);
    std::vector<float> mo_f((size_t)n_ao * nmo_pad, 0.0f);
    for (int mu = 0; mu < n_ao; ++mu)
        for (int m = 0; m < d->n_mo; ++m) {
            const double v = d->mo_coef[(size_t)mu * d->n_mo + old_of_new[m]] * angf[mu];
            mo[(size_t)mu * nmo_pad + m] = v;
            mo_f[(size_t)mu * nmo_pad + m] = (float)v;
        }
    std::vector<double> atoms;
    double vnn = 0.0;
    for (int a = 0; a < d->n_atoms; ++a) {
        atoms.push_back(d->R[3 * a]);
        atoms.push_back(d->R[3 * a + 1]);
        atoms.push_back(d->R[3 * a + 2]);
        atoms.push_back(d->Z[a]);
        for (int b = 0; b < a; ++b) {
            const double dx = d->R[3 * a] - d->R[3 * b], dy = d->R[3 * a + 1] - d->R[3 * b + 1],
                         dz = d->R[3 * a + 2] - d->R[3 * b + 2];
            vnn += d->Z[a] * d->Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }

    std::vector<unsigned char> blob;
    const size_t o_atoms = push_bytes(blob, atoms.data(), atoms.size());
    const size_t o_shells = push_bytes(blob, shells.data(), shells.size());
    const size_t o_prims = push_bytes(blob, prims.data(), prims.size());
    const size_t o_mo = push_bytes(blob, mo.data(), mo.size());
    const size_t o_mof = push_bytes(blob, mo_f.data(), mo_f.size());
    const size_t o_dets = push_bytes(blob, dets.data(), dets.size());
    const size_t o_ci = push_bytes(blob, ci.data(), ci.size());
    const size_t o_ent = push_bytes(blob, entries.data(), entries.size());
    const size_t o_con = push_bytes(blob, contribs.data(), contribs.size());
    const size_t o_perm = push_bytes(blob, old_of_new.data(), old_of_new.size());
    const size_t o_angf = push_bytes(blob, angf.data(), angf.size());
    const std::vector<uint4> frag = mfma_fragments(mo, n_ao, d->n_mo, nmo_pad);
    const size_t o_frag = push_bytes(blob, frag.data(), frag.size());
    const size_t o_drec = push_bytes(blob, det_recs.data(), det_recs.size());
    const size_t o_crec = push_bytes(blob, cof_recs.data(), cof_recs.size());
    const size_t o_jen = push_bytes(blob, d->jas_en, d->jas_en ? (size_t)3 * d->n_atoms : 0);
    const size_t o_jeen = push_bytes(blob, d->jas_een, (size_t)7 * d->jas_een_n);
    const size_t o_cocc = push_bytes(blob, cfg_occ.data(), cfg_occ.size());
    const size_t o_dcfg = push_bytes(blob, det_cfg.data(), det_cfg.size());
    const size_t o_cix = push_bytes(blob, ci_x.data(), ci_x.size());
    const size_t o_coff = push_bytes(blob, cfg_off.data(), cfg_off.size());
    const size_t o_cuse = push_bytes(blob, cfg_use.data(), cfg_use.size());
    const size_t o_cexc = push_bytes(blob, cfg_exc.data(), cfg_exc.size());

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return QMC_EDEVICE;
    if (device < 0 || device >= ndev) return QMC_EINVAL;
    DeviceGuard g(device);
    if (!g.ok) return QMC_EDEVICE;
    void *dm = nullptr;
    if (hipMalloc(&dm, blob.size()) != hipSuccess) return QMC_ENOMEM;
    if (hipMemcpy(dm, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dm);
        return QMC_EDEVICE;
    }
    qmc_system *sys = new (std::nothrow) qmc_system();
    if (!sys) {
        (void)hipFree(dm);
        return QMC_ENOMEM;
    }
    sys->device = device;
    sys->d_mem = dm;
    bool made = hipStreamCreateWithFlags(&sys->side, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < 4 && made; ++k) made = hipEventCreateWithFlags(&sys->ev[k], hipEventDisableTiming) == hipSuccess;
    if (!made) {
        qmc_system_destroy(sys);
        return QMC_EDEVICE;
    }
    unsigned char *base = (unsigned char *)dm;
    DevSystem &S = sys->S;
    S.n_up = nu;
    S.n_dn = nd;
    S.ne = ne;
    S.n_atoms = d->n_atoms;
    S.n_shells = d->n_shells;
    S.n_ao = n_ao;
    S.n_mo = d->n_mo;
    S.n_det = n_det;
    S.n_entries = n_entries;
    S.G = G;
    S.LW = 2 * G;
    S.WPW = qmc::kWave / S.LW;
    S.nmo_pad = nmo_pad;
    S.basis = d->basis;
    S.normalize = d->normalize;
    S.n_prim = (int)prims.size();
    S.a_par = d->jas_a_par;
    S.a_anti = d->jas_a_anti;
    S.b = d->jas_b;
    S.vnn = vnn;
    S.atoms = (const double *)(base + o_atoms);
    S.shells = (const int4 *)(base + o_shells);
    S.prims = (const double2 *)(base + o_prims);
    S.mo = (const double *)(base + o_mo);
    S.mo_f = (const float *)(base + o_mof);
    S.dets = (const int *)(base + o_dets);
    S.ci = (const double *)(base + o_ci);
    S.entries = (const int4 *)(base + o_ent);
    S.contribs = (const int4 *)(base + o_con);
    S.mo_perm = (const int *)(base + o_perm);
    S.ao_angf = (const double *)(base + o_angf);
    S.mfma_tab = (const uint4 *)(base + o_frag);
    S.det_rows = det_rows;
    S.cof_rows = (int)cof_rows;
    S.det_recs = (const uint4 *)(base + o_drec);
    S.cof_recs = (const uint4 *)(base + o_crec);
    S.jas_en = d->jas_en ? (const double *)(base + o_jen) : nullptr;
    S.jas_een = (const double *)(base + o_jeen);
    S.een_n = d->jas_een_n;
    S.n_cfg_up = (int)cfgs[0].size();
    S.n_cfg_dn = (int)cfgs[1].size();
    S.n_cfg_max = n_cfg_max;
    S.n_det_x = (int)det_cfg.size();
    S.cfg_occ = (const int *)(base + o_cocc);
    S.det_cfg = (const int2 *)(base + o_dcfg);
    S.ci_x = (const double *)(base + o_cix);
    S.cfg_off = (const int *)(base + o_coff);
    S.cfg_use = (const int2 *)(base + o_cuse);
    S.bf_omega = d->bf_omega;
    S.cfg_exc = (const int *)(base + o_cexc);
    sys->n_prim = (int)prims.size();
    // exponents | MO coefficients | Pade b | e-n (w0, w1, w2) per nucleus | e-e-n 7 per term
    sys->n_params = (int64_t)prims.size() + (int64_t)n_ao * d->n_mo + 1 + (d->jas_en ? 3 * (int64_t)d->n_atoms : 0) +
                    7 * (int64_t)d->jas_een_n;
    *out = sys;
    return QMC_OK;
}

void qmc_system_destroy(qmc_system *sys) {
    if (!sys) return;
    {
        DeviceGuard g(sys->device);
        for (hipEvent_t e : sys->ev)
            if (e) (void)hipEventDestroy(e);
        if (sys->side) (void)hipStreamDestroy(sys->side);
        (void)hipFree(sys->d_mem);
    }
    delete sys;
}

static qmc_status check_walk_args(qmc_system *sys, int32_t precision, int64_t W) {
    if (!sys) return QMC_EINVAL;
    if (W < 0 || W > (int64_t)0x7FFFFFFF) return QMC_EINVAL;
    if (precision < QMC_FP64 || precision > QMC_FP64_EXPLICIT) return QMC_EINVAL;
    if ((precision == QMC_MIXED_BF16 || precision == QMC_MIXED_BF16_X1) && sys->S.n_ao > 32)
        return QMC_EUNSUPPORTED;
    if (sys->S.bf_omega != 0.0) {
        // backflow: FP64 only; QMC_FP64 updates the configurations from the
        // reference, QMC_FP64_EXPLICIT factorises each
        if (precision != QMC_FP64 && precision != QMC_FP64_EXPLICIT) return QMC_EUNSUPPORTED;
        if (sys->S.n_cfg_max > qmc::kMaxCfgBF ||
            qmc::backflow_lds_bytes(sys->S, precision == QMC_FP64) > 160 * 1024)
            return QMC_EUNSUPPORTED;
        return QMC_OK;
    }
    if (precision == QMC_FP64_EXPLICIT && qmc::explicit_lds_bytes(sys->S) > 160 * 1024) return QMC_EUNSUPPORTED;
    return QMC_OK;
}

// Kernel form of a call: the precision, or with backflow 6 (low-rank) / 5
// (every configuration factorised).
static int walk_form(const qmc_system *sys, int32_t precision) {
    if (sys->S.bf_omega == 0.0) return precision;
    return precision == QMC_FP64_EXPLICIT ? 5 : 6;
}

qmc_status qmc_eval_psi_eloc(qmc_system *sys, int32_t precision, const double *d_X, int64_t W,
                             double *d_logpsi, double *d_sign, double *d_eloc, void *stream) {
    qmc_status st = check_walk_args(sys, precision, W);
    if (st != QMC_OK) return st;
    if (W == 0) return QMC_OK;
    if (!d_X || !d_logpsi || !d_sign || !d_eloc) return QMC_EINVAL;
    DeviceGuard g(sys->device);
    if (!g.ok) return QMC_EDEVICE;
    std::lock_guard<std::mutex> lock(sys->mu);
    const qmc::CallStreams cs{(hipStream_t)stream, sys->side, {sys->ev[0], sys->ev[1], sys->ev[2], sys->ev[3]}};
    hipError_t e = qmc::launch_walkers(false, walk_form(sys, precision), sys->S, (double *)d_X,
                                       d_logpsi, d_sign, d_eloc, W, 0, 0.0, 0, 0, 0, nullptr, cs);
    return e == hipSuccess ? QMC_OK : QMC_EDEVICE;
}

qmc_status qmc_metropolis_block(qmc_system *sys, int32_t precision, double *d_X, double *d_logpsi,
                                double *d_sign, double *d_eloc, int64_t W, int32_t n_steps,
                                double sigma, uint64_t seed, uint64_t step0, uint32_t walker_offset,
                                double *d_acc, void *stream) {
    qmc_status st = check_walk_args(sys, precision, W);
    if (st != QMC_OK) return st;
    if (!is_finite(sigma)) return QMC_ENONFINITE;
    if (n_steps < 0 || sigma < 0.0) return QMC_EINVAL;
    if ((uint64_t)walker_offset + (uint64_t)W > 0x100000000ull) return QMC_EINVAL;
    if (W == 0 || n_steps == 0) return QMC_OK;
    if (!d_X || !d_logpsi || !d_sign || !d_eloc || !d_acc) return QMC_EINVAL;
    DeviceGuard g(sys->device);
    if (!g.ok) return QMC_EDEVICE;
    std::lock_guard<std::mutex> lock(sys->mu);
    const qmc::CallStreams cs{(hipStream_t)stream, sys->side, {sys->ev[0], sys->ev[1], sys->ev[2], sys->ev[3]}};
    hipError_t e = qmc::launch_walkers(true, walk_form(sys, precision), sys->S, d_X, d_logpsi,
                                       d_sign, d_eloc, W, n_steps, sigma, seed, step0, walker_offset,
                                       d_acc, cs);
    return e == hipSuccess ? QMC_OK : QMC_EDEVICE;
}

qmc_status qmc_eval_eloc_fd(qmc_system *sys, const double *d_X, int64_t W, double h, double *d_logpsi,
                            double *d_eloc, void *stream) {
    if (!sys || W < 0 || W > (int64_t)0x7FFFFFFF) return QMC_EINVAL;
    if (!is_finite(h)) return QMC_ENONFINITE;
    if (!(h > 0.0)) return QMC_EINVAL;
    if (sys->S.bf_omega != 0.0) return QMC_EUNSUPPORTED;
    if (W == 0) return QMC_OK;
    if (!d_X || !d_logpsi || !d_eloc) return QMC_EINVAL;
    DeviceGuard g(sys->device);
    if (!g.ok) return QMC_EDEVICE;
    hipError_t e = qmc::launch_eval_fd(sys->S, d_X, W, h, d_logpsi, d_eloc, (hipStream_t)stream);
    return e == hipSuccess ? QMC_OK : QMC_EDEVICE;
}

qmc_status qmc_grad(qmc_system *sys, int32_t precision, const double *d_X, int64_t W, double *d_dlogpsi,
                    double *d_deloc_dtheta, double *d_dlogpsi_dR, double *d_deloc_dR, void *stream) {
    if (!sys || W < 0 || W > (int64_t)0x7FFFFFFF) return QMC_EINVAL;
    if (precision < QMC_FP64 || precision > QMC_FP64_EXPLICIT) return QMC_EINVAL;
    if (precision != QMC_FP64 && precision != QMC_MIXED_FP32) return QMC_EUNSUPPORTED;
    if (W == 0) return QMC_OK;
    if (!d_X || (!d_dlogpsi && !d_deloc_dtheta && !d_dlogpsi_dR && !d_deloc_dR)) return QMC_EINVAL;
    if (qmc::grad_lds_bytes(sys->S) > 160 * 1024) return QMC_EUNSUPPORTED;
    if (sys->S.bf_omega != 0.0) return QMC_EUNSUPPORTED;
    DeviceGuard g(sys->device);
    if (!g.ok) return QMC_EDEVICE;
    hipError_t e = qmc::launch_grad(sys->S, d_X, W, d_dlogpsi, d_deloc_dtheta, d_dlogpsi_dR, d_deloc_dR,
                                    (int)sys->n_params, precision == QMC_MIXED_FP32, (hipStream_t)stream);
    return e == hipSuccess ? QMC_OK : QMC_EDEVICE;
}

int64_t qmc_param_count(const qmc_system *sys) { return sys ? sys->n_params : -1; }

size_t qmc_bytes_per_walker(const qmc_system *sys, int32_t precision) {
    (void)precision;
    if (!sys) return 0;
    // positions + (log|Psi|, sign, E_L) + four accumulators, all FP64
    return (size_t)sys->S.ne * 3 * sizeof(double) + 7 * sizeof(double);
}

qmc_status qmc_reduce_accumulators(const double *d_acc, int64_t W, double *d_out, void *stream) {
    if (W < 0 || W > (int64_t)0x7FFFFFFF || !d_out || (W > 0 && !d_acc)) return QMC_EINVAL;
    hipError_t e = qmc::launch_reduce_acc(d_acc, W, d_out, (hipStream_t)stream);
    return e == hipSuccess ? QMC_OK : QMC_EDEVICE;
}

}  // extern "C"
