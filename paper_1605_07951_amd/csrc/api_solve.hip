// C ABI: SS-FULL on the projected NEP and the lift (RSRR Steps 4-5).
//
// Follows Sec. 3.3 (SS-RI with F = T_Q^-1, i.e. SS-FULL) on the RSRR
// contour: moments A_alpha = sum_m w_m zeta_m^alpha T_Q(z_m)^-1 (eq.
// Aalpha-rat with the shifted/scaled variable zeta = (z - gamma)/rho), block
// Hankel matrices H, H^< (eq. HH), SVD of H with the gap count (eq. gap),
// A = V0^H H^< W0 Sigma0^-1 (eq. A), its eigenpairs, g = M W0 Sigma0^-1 b with
// M = [A_0 ... A_{K-1}] (eq. eigens with U = I), v = Q g, lambda = gamma + rho mu.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

extern "C" rsrr_status rsrr_solve(rsrr_ctx* c, const rsrr_nep* nep, int k, const double* AQp, int J_eff,
                                  const rsrr_term* terms, const double* Qp, int ldq, const double* gamma, double a,
                                  double b, int NQ, int KQ, double tol_gap, int max_eigs, double* lambda, double* Vp,
                                  int ldv, double* resid, int* count, double* sigma_H, rsrr_solve_info* sinfo)
{
    if (!c) return -1;
    if (!nep || nep->n < 1) return -2;
    if (nep->kind == RSRR_T_SEPARABLE && (nep->J < 1 || !nep->A || nep->lda < nep->n || !nep->terms)) return -2;
    if (nep->kind == RSRR_T_HELMHOLTZ && (!nep->points || !(nep->w > 0))) return -2;
    if (nep->kind == RSRR_T_SPARSE && !csr_nep_ok(nep)) return -2;
    if (nep->kind != RSRR_T_SEPARABLE && nep->kind != RSRR_T_HELMHOLTZ && nep->kind != RSRR_T_SPARSE) return -2;
    if (k < 1 || k > nep->n) return -3;
    if (!AQp) return -4;
    if (J_eff < 1 || J_eff > 64) return -5;
    if (!terms) return -6;
    if (!Qp) return -7;
    if (ldq < nep->n) return -8;
    if (!gamma) return -9;
    if (!(a > 0)) return -10;
    if (!(b > 0)) return -11;
    if (KQ < 1) return -13;
    if (NQ < 2 * KQ + 1) return -12;
    if (!(tol_gap > 0)) return -14;
    if (max_eigs < 1) return -15;
    if (!lambda) return -16;
    if (Vp && ldv < nep->n) return -17;
    if (!count) return -18;
    RSRR_HIP(hipSetDevice(c->device));
    const int n = nep->n;
    const zd g(gamma[0], gamma[1]);
    const double rho = std::max(a, b);
    const double2* AQ = (const double2*)AQp;
    const double2* Q = (const double2*)Qp;
    *count = 0;

    // ---- moments ----
    const int twoK = 2 * KQ;
    const long kk = (long)k * k;
    double2* mom = (double2*)ws_get(c, WS_B0, (size_t)twoK * kk * 16);
    if (!mom) return RSRR_ENOMEM;
    RSRR_HIP(hipMemsetAsync(mom, 0, (size_t)twoK * kk * 16, c->stream));
    const int nb = 64;
    const int np = perm_panels(k);
    // the diagonal blocks of the FP64 LU are inverted once per panel, so the solves
    // with the k columns of I are products on the matrix cores
    const long sInv = 2L * ((k + nb - 1) / nb) * nb * nb, sTmp = (long)nb * k;
    const size_t per_pt = (size_t)kk * 16 * 2 + (size_t)k * 4 + 64 * 1024 + (size_t)(sInv + sTmp) * 16;
    // points per batched LU: 8 GiB of buffers, or the context's workspace budget when set
    const size_t mom_budget = c->ws_budget ? std::min<size_t>(c->ws_budget, (size_t)8 << 30) : (size_t)8 << 30;
    const int Mc = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::min(NQ, 256), mom_budget / per_pt));
    double2* T = (double2*)ws_get(c, WS_TLU, (size_t)Mc * kk * 16);
    double2* X = (double2*)ws_get(c, WS_TRES, (size_t)Mc * kk * 16);
    int* ipiv = (int*)ws_get(c, WS_IPIV, (size_t)Mc * k * 4);
    int2* perm = (int2*)ws_get(c, WS_PERM, (size_t)Mc * np * 2 * MAX_NB * 8);
    int* info = (int*)ws_get(c, WS_INFO, (size_t)Mc * 4);
    double2* coef = (double2*)ws_get(c, WS_COEF, (size_t)J_eff * Mc * 16);
    double2* cw = (double2*)ws_get(c, WS_B1, (size_t)Mc * twoK * 16);
    double2* I = (double2*)ws_get(c, WS_B2, (size_t)kk * 16);
    double* frob = (double*)ws_get(c, WS_FROB, (size_t)Mc * 8);
    const long nparts = (kk + 255) / 256;
    double* frobp = (double*)ws_get(c, WS_FROBP, (size_t)Mc * nparts * 8);
    double2* inv = (double2*)ws_get(c, WS_B5, (size_t)Mc * sInv * 16);
    double2* tmp = (double2*)ws_get(c, WS_B6, (size_t)Mc * sTmp * 16);
    if (!T || !X || !ipiv || !perm || !info || !coef || !cw || !I || !frob || !frobp || !inv || !tmp)
        return RSRR_ENOMEM;
    RSRR_HIP(eye(c->stream, I, k, 0, k));
    int singular = 0;
    std::vector<double2> hcoef((size_t)J_eff * Mc), hcw((size_t)Mc * twoK);
    std::vector<int> hinfo(Mc);
    for (int m0 = 0; m0 < NQ; m0 += Mc) {
        const int B = std::min(Mc, NQ - m0);
        for (int m = 0; m < B; ++m) {
            const double th = 2.0 * M_PI * (m0 + m + 0.5) / NQ;
            const zd zm = g + zd(a * std::cos(th), b * std::sin(th));
            const zd wm = zd(-a * std::sin(th), b * std::cos(th)) / (double)NQ;
            for (int j = 0; j < J_eff; ++j) {
                const zd f = term_eval(terms[j], zm);
                hcoef[(size_t)j * B + m] = make_double2(f.real(), f.imag());
            }
            const zd zeta = (zm - g) / rho;
            zd p = wm;
            for (int al = 0; al < twoK; ++al) {
                hcw[(size_t)al * B + m] = make_double2(p.real(), p.imag());
                p *= zeta;
            }
        }
        RSRR_HIP(hipMemcpyAsync(coef, hcoef.data(), (size_t)J_eff * B * 16, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(hipMemcpyAsync(cw, hcw.data(), (size_t)twoK * B * 16, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(assemble_separable(c->stream, k, J_eff, AQ, k, coef, B, nullptr, 0, 0, T, k, kk, frobp, frob));
        RSRR_HIP(hipMemsetAsync(info, 0, (size_t)B * 4, c->stream));
        LUWork w;
        w.ipiv = ipiv; w.sP = k; w.perm = perm; w.sPerm = (long)np * 2 * MAX_NB;
        w.info = info;
        w.inv = inv; w.sInv = sInv; w.tmp = tmp; w.sTmp = sTmp;
        RSRR_HIP(getrf_batched<double>(c->stream, T, kk, k, k, nb, w, B));
        RSRR_HIP(bcast_c128(c->stream, k, k, I, k, X, k, kk, B));
        RSRR_HIP(getrs_batched<double>(c->stream, T, kk, k, k, nb, w, X, kk, k, k, B));
        // mom(:, alpha) += sum_m X_m cw(m, alpha): one GEMM over the stacked vec(X_m)
        RSRR_HIP(zgemm(c->stream, 0, 0, (int)kk, twoK, B, 1.0, X, (int)kk, 0, cw, B, 0, 1.0, mom, (int)kk, 0, 1));
        RSRR_HIP(hipMemcpyAsync(hinfo.data(), info, (size_t)B * 4, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        for (int m = 0; m < B; ++m)
            if (hinfo[m] != 0) singular = 1;
    }
    if (singular) return RSRR_ESINGULAR;

    // ---- block Hankel matrices; [H; I] so that the Jacobi rotations accumulate W ----
    const int Kk = KQ * k;
    double2* Hx = (double2*)ws_get(c, WS_B3, (size_t)2 * Kk * Kk * 16);
    double2* Hs = (double2*)ws_get(c, WS_B4, (size_t)Kk * Kk * 16);
    if (!Hx || !Hs) return RSRR_ENOMEM;
    RSRR_HIP(hankel(c->stream, mom, k, KQ, 0, Hx, 2 * Kk));
    RSRR_HIP(eye(c->stream, Hx, 2 * Kk, Kk, Kk));
    RSRR_HIP(hankel(c->stream, mom, k, KQ, 1, Hs, Kk));
    rsrr_status st = RSRR_OK;
    const double eps = 2.220446049250313e-16;
    const double tol = 4.0 * std::max(1.0, std::sqrt((double)Kk)) * eps;

    // ---- SVD of H and the gap rule (eq. gap) ----
    // When the contour holds few eigenvalues, H is numerically of low rank: its
    // leading singular triplets come from a range sketch of H (one power step,
    // each product orthonormalised by BCGS2) and a one-sided Jacobi SVD of the
    // small factor.  The sketch is used only when it shows a clear gap inside
    // what it captured (g >= 10 tol_gap, and larger than any ratio the
    // uncaptured tail could show); otherwise the Jacobi SVD of the whole H runs.
    std::vector<double> s;
    std::vector<int> ord;
    int nbar = 0, nsig = 0, rS = 0;
    double gmax = 0.0;
    double2 *QY = nullptr, *XS = nullptr;
    auto gap_rule = [](const std::vector<double>& sv, int cnt, int* nb, double* g) {
        *nb = 0;
        *g = 0.0;
        for (int j = 0; j + 1 < cnt; ++j) {
            const double r = sv[j + 1] == 0.0 ? (sv[j] > 0.0 ? INFINITY : 0.0) : sv[j] / sv[j + 1];
            if (r > *g) { *g = r; *nb = j + 1; }
        }
    };
    for (int l = 64; 2 * l <= Kk; l *= 2) {
        double2* Om = (double2*)ws_get(c, WS_HS0, (size_t)Kk * l * 16);
        double2* Y = (double2*)ws_get(c, WS_HS1, (size_t)Kk * l * 16);
        double2* Z = (double2*)ws_get(c, WS_HS2, (size_t)Kk * l * 16);
        void* wb = ws_get(c, WS_HSW, bcgs2_work_bytes(Kk, l));
        double* n0 = (double*)ws_get(c, WS_HSD, (size_t)2 * l * 8);
        int* di = (int*)ws_get(c, WS_HSI, (size_t)l * 4);
        if (!Om || !Y || !Z || !wb || !n0 || !di) return RSRR_ENOMEM;
        RSRR_HIP(gaussian(c->stream, Om, Kk, l, Kk, 0x4a4b5eedull + (unsigned long long)l));
        RSRR_HIP(zgemm(c->stream, 0, 0, Kk, l, Kk, 1.0, Hx, 2 * Kk, 0, Om, Kk, 0, 0.0, Y, Kk, 0, 1));
        RSRR_HIP(bcgs2(c->stream, Y, Kk, Kk, l, wb, n0));
        RSRR_HIP(zgemm(c->stream, 1, 0, Kk, l, Kk, 1.0, Hx, 2 * Kk, 0, Y, Kk, 0, 0.0, Z, Kk, 0, 1));
        RSRR_HIP(bcgs2(c->stream, Z, Kk, Kk, l, wb, n0));
        RSRR_HIP(zgemm(c->stream, 0, 0, Kk, l, Kk, 1.0, Hx, 2 * Kk, 0, Z, Kk, 0, 0.0, Y, Kk, 0, 1));
        RSRR_HIP(bcgs2(c->stream, Y, Kk, Kk, l, wb, n0));
        RSRR_HIP(colnorms(c->stream, Kk, l, Y, Kk, 0, n0, 1));
        std::vector<double> hq(l);
        RSRR_HIP(hipMemcpyAsync(hq.data(), n0, (size_t)l * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        std::vector<int> idx;
        for (int i = 0; i < l; ++i)
            if (hq[i] > 0.5) idx.push_back(i);
        const int r = (int)idx.size();
        if (r < 2) break;
        // compacted Q_Y (into Omega's buffer), X = [H^H Q_Y; I_r]
        std::vector<double> ones(r, 1.0);
        RSRR_HIP(hipMemcpyAsync(di, idx.data(), (size_t)r * 4, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(hipMemcpyAsync(n0 + l, ones.data(), (size_t)r * 8, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(gather_scale(c->stream, Y, Kk, Kk, di, n0 + l, Om, Kk, r));
        double2* X = (double2*)ws_get(c, WS_HSX, (size_t)(Kk + r) * r * 16);
        if (!X) return RSRR_ENOMEM;
        RSRR_HIP(zgemm(c->stream, 1, 0, Kk, r, Kk, 1.0, Hx, 2 * Kk, 0, Om, Kk, 0, 0.0, X, Kk + r, 0, 1));
        RSRR_HIP(eye(c->stream, X, Kk + r, Kk, r));
        if (jacobi_svd(c, X, Kk + r, Kk, Kk + r, r, 80, tol, &st) < 0) return st;
        RSRR_HIP(colnorms(c->stream, Kk, r, X, Kk + r, 0, n0, 1));
        std::vector<double> sv(r);
        RSRR_HIP(hipMemcpyAsync(sv.data(), n0, (size_t)r * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        std::vector<int> o(r);
        std::iota(o.begin(), o.end(), 0);
        std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return sv[x] > sv[y]; });
        std::vector<double> ss(r);
        for (int i = 0; i < r; ++i) ss[i] = sv[o[i]];
        if (!(ss[0] > 0.0)) break;
        int nb1 = 0;
        double g1 = 0.0;
        bool ok;
        if (r < l) {
            // rank-deficient sketch: what it did not capture lies below the BCGS2
            // dropping level, taken as the next singular value
            std::vector<double> se(ss);
            se.push_back(4.0 * eps * std::sqrt((double)Kk * l) * ss[0]);
            gap_rule(se, r + 1, &nb1, &g1);
            ok = g1 >= 10.0 * tol_gap;
        } else {
            gap_rule(ss, r, &nb1, &g1);
            ok = g1 >= 10.0 * tol_gap && nb1 <= r - 2 && g1 >= ss[r - 1] / (eps * ss[0]);
        }
        if (ok) {
            s = ss;
            ord = o;
            nbar = nb1;
            gmax = g1;
            nsig = r;
            rS = r;
            QY = Om;
            XS = X;
            break;
        }
    }
    if (!XS) {
        if (jacobi_svd(c, Hx, 2 * Kk, Kk, 2 * Kk, Kk, 80, tol, &st) < 0) return st;
        double* nrm = (double*)ws_get(c, WS_B5, (size_t)Kk * 8);
        if (!nrm) return RSRR_ENOMEM;
        RSRR_HIP(colnorms(c->stream, Kk, Kk, Hx, 2 * Kk, 0, nrm, 1));
        std::vector<double> sv(Kk);
        RSRR_HIP(hipMemcpyAsync(sv.data(), nrm, (size_t)Kk * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        ord.resize(Kk);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sv[x] > sv[y]; });
        s.resize(Kk);
        for (int i = 0; i < Kk; ++i) s[i] = sv[ord[i]];
        nsig = Kk;
        gap_rule(s, Kk, &nbar, &gmax);
    }
    if (sigma_H)
        for (int i = 0; i < Kk; ++i) sigma_H[i] = i < nsig ? s[i] : 0.0;
    const int warn = gmax < tol_gap;
    if (sinfo) {
        sinfo->nbar = nbar;
        sinfo->warn_gap = warn;
        sinfo->gmax = gmax;
        sinfo->n_sigma = nsig;
        sinfo->truncated = 0;
    }
    if (nbar == 0 || s[0] == 0.0) return RSRR_WARN_GAP;
    // eq. A uses every retained singular triplet: the reduced matrix and its
    // eigenpairs are formed at the full count nbar; max_eigs only bounds how many
    // eigenpairs are copied out (those of lowest elliptic level first).
    if (nbar > small_eig_max()) return RSRR_ELIMIT;
    const int na = nbar;
    const int ne = std::min(na, max_eigs);
    if (sinfo) sinfo->truncated = ne < na;

    // ---- V0, W0, reduced matrix A = V0^H H^< W0 Sigma0^-1 ----
    int* dord = (int*)ws_get(c, WS_ACTIVE, (size_t)na * 4);
    double* dinv = (double*)ws_get(c, WS_NORM, (size_t)2 * na * 8);
    double2* V0 = (double2*)ws_get(c, WS_D64, (size_t)Kk * na * 16);
    double2* W0 = (double2*)ws_get(c, WS_R, (size_t)Kk * na * 16);
    double2* T1 = (double2*)ws_get(c, WS_B6, (size_t)Kk * na * 16 + (size_t)4 * na * na * 16 + (size_t)na * 16 + 64);
    double2* G = (double2*)ws_get(c, WS_B7, (size_t)k * ne * 16 + (size_t)Kk * ne * 16);
    if (!dord || !dinv || !V0 || !W0 || !T1 || !G) return RSRR_ENOMEM;
    double2* Ared = T1 + (size_t)Kk * na;
    double2* Hw = Ared + (size_t)na * na;
    double2* Zw = Hw + (size_t)na * na;
    double2* Bsel = Zw + (size_t)na * na;
    double2* mu = Bsel + (size_t)na * na;
    double2* Bv = V0;  // V0 is no longer needed once Ared is formed; reuse for the eigenvectors
    double2* Y = G + (size_t)k * ne;
    std::vector<double> hinv(2 * na);
    for (int i = 0; i < na; ++i) { hinv[i] = 1.0 / s[i]; hinv[na + i] = 1.0; }
    RSRR_HIP(hipMemcpyAsync(dord, ord.data(), (size_t)na * 4, hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(hipMemcpyAsync(dinv, hinv.data(), (size_t)2 * na * 8, hipMemcpyHostToDevice, c->stream));
    if (XS) {
        // sketch: left vectors Q_Y W (W: bottom r rows of X), right vectors (top of X) / sigma
        double2* Wsm = (double2*)ws_get(c, WS_B2, (size_t)rS * na * 16);
        if (!Wsm) return RSRR_ENOMEM;
        RSRR_HIP(gather_scale(c->stream, XS, Kk + rS, Kk, dord, dinv, W0, Kk, na));
        RSRR_HIP(gather_scale(c->stream, XS + Kk, Kk + rS, rS, dord, dinv + na, Wsm, rS, na));
        RSRR_HIP(zgemm(c->stream, 0, 0, Kk, na, rS, 1.0, QY, Kk, 0, Wsm, rS, 0, 0.0, V0, Kk, 0, 1));
    } else {
        RSRR_HIP(gather_scale(c->stream, Hx, 2 * Kk, Kk, dord, dinv, V0, Kk, na));
        RSRR_HIP(gather_scale(c->stream, Hx + Kk, 2 * Kk, Kk, dord, dinv + na, W0, Kk, na));
    }
    RSRR_HIP(zgemm(c->stream, 0, 0, Kk, na, Kk, 1.0, Hs, Kk, 0, W0, Kk, 0, 0.0, T1, Kk, 0, 1));
    RSRR_HIP(zgemm(c->stream, 1, 0, na, na, Kk, 1.0, V0, Kk, 0, T1, Kk, 0, 0.0, Ared, na, 0, 1));
    RSRR_HIP(scale_cols(c->stream, na, na, Ared, na, dinv));
    int* dstat = (int*)ws_get(c, WS_INFO, 64);
    if (!dstat) return RSRR_ENOMEM;
    RSRR_HIP(small_eig(c->stream, Ared, na, Hw, Zw, mu, Bv, dstat));
    int hstat = 0;
    std::vector<double2> hmu(na);
    RSRR_HIP(hipMemcpyAsync(&hstat, dstat, 4, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipMemcpyAsync(hmu.data(), mu, (size_t)na * 16, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    if (hstat) return RSRR_ENOTCONV;
    // ---- the ne eigenpairs of lowest elliptic level (stable: ties keep the Schur order) ----
    std::vector<zd> lall(na);
    std::vector<double> lev(na);
    for (int i = 0; i < na; ++i) {
        lall[i] = g + rho * zd(hmu[i].x, hmu[i].y);
        const zd dz = lall[i] - g;
        lev[i] = (dz.real() / a) * (dz.real() / a) + (dz.imag() / b) * (dz.imag() / b);
    }
    std::vector<int> sel(na);
    std::iota(sel.begin(), sel.end(), 0);
    std::stable_sort(sel.begin(), sel.end(), [&](int x, int y) { return lev[x] < lev[y]; });
    sel.resize(ne);
    std::vector<zd> lam(ne);
    for (int i = 0; i < ne; ++i) {
        lam[i] = lall[sel[i]];
        lambda[2 * i] = lam[i].real();
        lambda[2 * i + 1] = lam[i].imag();
    }
    RSRR_HIP(hipMemcpyAsync(dord, sel.data(), (size_t)ne * 4, hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(gather_scale(c->stream, Bv, na, na, dord, dinv + na, Bsel, na, ne));
    // ---- lift: Y = W0 Sigma0^-1 B, g = M Y, v = Q g (unit columns) ----
    RSRR_HIP(scale_cols(c->stream, Kk, na, W0, Kk, dinv));
    RSRR_HIP(zgemm(c->stream, 0, 0, Kk, ne, na, 1.0, W0, Kk, 0, Bsel, na, 0, 0.0, Y, Kk, 0, 1));
    RSRR_HIP(zgemm(c->stream, 0, 0, k, ne, Kk, 1.0, mom, k, 0, Y, Kk, 0, 0.0, G, k, 0, 1));
    *count = ne;
    if (Vp) {
        double2* V = (double2*)Vp;
        RSRR_HIP(zgemm(c->stream, 0, 0, n, ne, k, 1.0, Q, ldq, 0, G, k, 0, 0.0, V, ldv, 0, 1));
        double* vn = dinv;
        RSRR_HIP(colnorms(c->stream, n, ne, V, ldv, 0, vn, 1));
        std::vector<double> hv(ne);
        RSRR_HIP(hipMemcpyAsync(hv.data(), vn, (size_t)ne * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        for (auto& v : hv) v = v > 0 ? 1.0 / v : 0.0;
        RSRR_HIP(hipMemcpyAsync(vn, hv.data(), (size_t)ne * 8, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(scale_cols(c->stream, n, ne, V, ldv, vn));
        if (resid) {
            // ||T(lambda_i) v_i||_2 / ||T(lambda_i)||_1 in FP64 against the full T
            const size_t budget = c->ws_budget ? std::min<size_t>(c->ws_budget, (size_t)4 << 30) : (size_t)4 << 30;
            const int Bc = (int)std::max<size_t>(1, std::min<size_t>((size_t)ne, budget / ((size_t)n * n * 16)));
            double2* Tb = (double2*)ws_get(c, WS_TLU, (size_t)Bc * n * n * 16);
            double2* Rv = (double2*)ws_get(c, WS_R, (size_t)Bc * n * 16);
            double* rn = (double*)ws_get(c, WS_B5, (size_t)2 * Bc * 8);
            double* fr = (double*)ws_get(c, WS_FROB, (size_t)Bc * 8);
            double* part = (double*)ws_get(c, WS_N1, (size_t)Bc * norm1_parts(n) * 8);
            if (!Tb || !Rv || !rn || !fr || !part) return RSRR_ENOMEM;
            std::vector<double> hr(2 * Bc);
            for (int i0 = 0; i0 < ne; i0 += Bc) {
                const int B = std::min(Bc, ne - i0);
                st = assemble_c128(c, nep, lam.data() + i0, B, Tb, n, (long)n * n, fr);
                if (st) return st;
                RSRR_HIP(zgemm(c->stream, 0, 0, n, 1, n, 1.0, Tb, n, (long)n * n, V + (size_t)i0 * ldv, ldv, ldv, 0.0,
                               Rv, n, n, B));
                RSRR_HIP(colnorms(c->stream, n, 1, Rv, n, n, rn, B));
                RSRR_HIP(norm1(c->stream, Tb, n, (long)n * n, n, rn + Bc, B, part));
                RSRR_HIP(hipMemcpyAsync(hr.data(), rn, (size_t)2 * Bc * 8, hipMemcpyDeviceToHost, c->stream));
                RSRR_HIP(hipStreamSynchronize(c->stream));
                for (int i = 0; i < B; ++i) resid[i0 + i] = hr[Bc + i] > 0 ? hr[i] / hr[Bc + i] : hr[i];
            }
        }
    }
    RSRR_HIP(hipStreamSynchronize(c->stream));
    if (warn) return RSRR_WARN_GAP;
    return ne < na ? RSRR_WARN_MORE : RSRR_OK;
}
