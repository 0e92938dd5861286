// C ABI: two-stage sampling (Sec. 5.4, Example 2, and Sec. 6, Example 3).
//
// Stage 1 runs RSRR on N1 points of the ellipse.  The distinct eigenvalue
// estimates inside the contour then become extra sampling points: their
// blocks T(z)^-1 U are appended to the stage-1 S, whose columns are reused,
// and the basis, projection and SS-FULL run again on all columns.  Putting
// sampling points next to the eigenvalues is what the resolvent-sampling
// approach allows and the contour-integral approach does not.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

namespace {

constexpr int MAX_TERMS = 64;
constexpr double DISTINCT_REL = 1e-6;

bool bad(rsrr_status s) { return s < 0 || s == RSRR_ENOMEM || s == RSRR_EDEVICE || s == RSRR_ENOTCONV || s == RSRR_ENAN || s == RSRR_ELIMIT; }

void keep_first(rsrr_status& acc, rsrr_status s)
{
    if (s != RSRR_OK && (acc == RSRR_OK || (!bad(acc) && bad(s)))) acc = s;
}

// Steps 3-5 on the first NL columns of S: basis, projection, SS-FULL.
rsrr_status steps_3_to_5(rsrr_ctx* c, const rsrr_nep* nep, double* S, int lds, int NL, const double gam[2], double a,
                         double b, double delta, int NQ, int KQ, double tol_gap, int max_eigs, double* lambda,
                         double* V, int ldv, double* resid, int* count, int* k_out, int* nbar)
{
    const int n = nep->n, kmax = std::min(n, NL);
    double2* Q = (double2*)ws_get(c, WS_TSQ, (size_t)n * kmax * 16);
    if (!Q) return RSRR_ENOMEM;
    int k = 0;
    rsrr_status st = RSRR_OK;
    rsrr_status e = rsrr_basis(c, n, NL, S, lds, delta, (double*)Q, n, kmax, &k, nullptr);
    keep_first(st, e);
    if (bad(e)) return e;
    *k_out = k;
    *count = 0;
    if (k < 1) return st;
    const int maxt = nep->kind == RSRR_T_HELMHOLTZ ? MAX_TERMS : nep->J;
    double2* AQ = (double2*)ws_get(c, WS_TSAQ, (size_t)maxt * k * k * 16);
    if (!AQ) return RSRR_ENOMEM;
    std::vector<rsrr_term> tout(maxt);
    int J_eff = 0;
    e = rsrr_project(c, nep, (const double*)Q, n, k, gam, std::max(a, b), (double*)AQ, maxt, &J_eff, tout.data());
    keep_first(st, e);
    if (bad(e)) return e;
    rsrr_solve_info si{};
    e = rsrr_solve(c, nep, k, (const double*)AQ, J_eff, tout.data(), (const double*)Q, n, gam, a, b, NQ, KQ, tol_gap,
                   max_eigs, lambda, V, ldv, resid, count, nullptr, &si);
    keep_first(st, e);
    if (bad(e)) return e;
    *nbar = si.nbar;
    return st;
}

}  // namespace

extern "C" rsrr_status rsrr_two_stage(rsrr_ctx* c, const rsrr_nep* nep, const double* gamma, double a, double b,
                                      int N1, const double* U, int L, int ldu, int prec, double* S, int lds,
                                      int max_new, double delta, int NQ, int KQ, double tol_gap, int max_eigs,
                                      double* lambda, double* V, int ldv, double* resid, int* count, double* z_new,
                                      rsrr_two_stage_info* tinfo)
{
    if (!c) return -1;
    if (!nep || nep->n < 1) return -2;
    if (!gamma) return -3;
    if (!(a > 0)) return -4;
    if (!(b > 0)) return -5;
    if (N1 < 1) return -6;
    if (!U) return -7;
    if (L < 1) return -8;
    if (ldu < nep->n) return -9;
    if (prec != RSRR_PREC_C128 && prec != RSRR_PREC_C64_IR) return -10;
    if (!S) return -11;
    if (lds < nep->n) return -12;
    if (max_new < 0) return -13;
    if (!(delta > 0 && delta < 1)) return -14;
    if (KQ < 1 || NQ < 2 * KQ + 1) return -15;
    if (!(tol_gap > 0)) return -17;
    if (max_eigs < 1) return -18;
    if (!lambda) return -19;
    if (!V) return -20;
    if (ldv < nep->n) return -21;
    if (!resid) return -22;
    if (!count) return -23;
    if (max_new > 0 && !z_new) return -24;
    RSRR_HIP(hipSetDevice(c->device));
    rsrr_two_stage_info ti{};
    rsrr_status st = RSRR_OK;

    // ---- stage 1: N1 contour points ----
    std::vector<double> z1(2 * (size_t)N1);
    rsrr_status e = rsrr_contour(gamma[0], gamma[1], a, b, N1, z1.data(), nullptr);
    if (e) return -6;
    e = rsrr_sample(c, nep, N1, z1.data(), U, L, ldu, prec, S, lds, nullptr);
    keep_first(st, e);
    if (bad(e)) return e;
    std::vector<double> lam1(2 * (size_t)max_eigs), res1(max_eigs);
    int cnt1 = 0;
    e = steps_3_to_5(c, nep, S, lds, N1 * L, gamma, a, b, delta, NQ, KQ, tol_gap, max_eigs, lam1.data(), V, ldv,
                     res1.data(), &cnt1, &ti.k1, &ti.nbar1);
    keep_first(st, e);
    if (bad(e)) return e;
    ti.count1 = cnt1;

    // ---- the distinct estimates inside the contour become new points ----
    std::vector<zd> znew;
    for (int i = 0; i < cnt1 && (int)znew.size() < max_new; ++i) {
        const zd l(lam1[2 * i], lam1[2 * i + 1]);
        const zd d = l - zd(gamma[0], gamma[1]);
        if ((d.real() / a) * (d.real() / a) + (d.imag() / b) * (d.imag() / b) >= 1.0) continue;
        bool dup = false;
        for (const zd& m : znew)
            if (std::abs(l - m) <= DISTINCT_REL * std::max(1.0, std::abs(l))) { dup = true; break; }
        if (!dup) znew.push_back(l);
    }
    ti.n_new = (int)znew.size();
    for (int i = 0; i < ti.n_new; ++i) {
        z_new[2 * i] = znew[i].real();
        z_new[2 * i + 1] = znew[i].imag();
    }

    // ---- stage 2: sample the new points after the stage-1 blocks, then steps 3-5 on all ----
    if (ti.n_new > 0) {
        e = rsrr_sample(c, nep, ti.n_new, z_new, U, L, ldu, prec, S + 2 * (size_t)N1 * L * lds, lds, nullptr);
        keep_first(st, e);
        if (bad(e)) return e;
    }
    int cnt = 0;
    e = steps_3_to_5(c, nep, S, lds, (N1 + ti.n_new) * L, gamma, a, b, delta, NQ, KQ, tol_gap, max_eigs, lambda, V,
                     ldv, resid, &cnt, &ti.k2, &ti.nbar2);
    keep_first(st, e);
    if (bad(e)) return e;
    *count = cnt;
    // largest stage-1 residual among the estimates inside the contour
    ti.resid1_max = 0.0;
    for (int i = 0; i < cnt1; ++i) {
        const zd d = zd(lam1[2 * i], lam1[2 * i + 1]) - zd(gamma[0], gamma[1]);
        if ((d.real() / a) * (d.real() / a) + (d.imag() / b) * (d.imag() / b) < 1.0)
            ti.resid1_max = std::max(ti.resid1_max, res1[i]);
    }
    if (tinfo) *tinfo = ti;
    return st;
}
