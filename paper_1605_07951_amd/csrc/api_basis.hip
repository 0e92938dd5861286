// C ABI: basis (RSRR Step 3) and projection (RSRR Step 4, eq. Ts-NEP).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

// One-sided Jacobi SVD of A (rows 0..m-1 form the Gram; rows m..m_apply-1 are
// rotated along).  Columns whose norm is below eps*||A||_F count as zero.
// Stops when a sweep measures every pair below tol, or when the measure has
// stalled below 1e-13 for two sweeps.  Returns the number of sweeps, or -1.
int jacobi_svd(rsrr_ctx* c, double2* A, int lda, int m, int m_apply, int p, int max_sweeps, double tol,
               rsrr_status* st)
{
    const int nb = jacobi_blocks(p);
    const int rounds = nb - 1, pairs = nb / 2;
    double* off = (double*)ws_get(c, WS_B6, (size_t)rounds * pairs * 8 + (size_t)p * 8);
    if (!off) { *st = RSRR_ENOMEM; return -1; }
    double* cn = off + (size_t)rounds * pairs;
    void* work = ws_get(c, WS_JAC, jacobi_work_bytes(m, m_apply, p));
    if (!work) { *st = RSRR_ENOMEM; return -1; }
    // ||A||_F^2 (invariant under the rotations) sets the zero-column threshold
    if (colnorms(c->stream, m, p, A, lda, 0, cn, 1) != hipSuccess) { *st = RSRR_EDEVICE; return -1; }
    std::vector<double> h((size_t)rounds * pairs), hc(p);
    if (hipMemcpyAsync(hc.data(), cn, (size_t)p * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        *st = RSRR_EDEVICE;
        return -1;
    }
    double fro2 = 0.0;
    for (double v : hc) fro2 += v * v;
    const double eps = 2.220446049250313e-16;
    const double zthr2 = eps * eps * fro2;
    double prev = 1e300;
    int stall = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        for (int r = 0; r < rounds; ++r) {
            if (jacobi_round(c->stream, A, lda, m, m_apply, p, r, 1, tol, zthr2, off + (size_t)r * pairs, work) !=
                hipSuccess) {
                *st = RSRR_EDEVICE;
                return -1;
            }
        }
        if (hipMemcpyAsync(h.data(), off, h.size() * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            *st = RSRR_EDEVICE;
            return -1;
        }
        double mx = 0.0;
        for (double v : h) mx = std::max(mx, v);
        if (!(mx == mx)) { *st = RSRR_ENAN; return -1; }
        if (mx <= tol) { *st = RSRR_OK; return sw + 1; }
        stall = (mx <= 1e-13 && mx >= 0.5 * prev) ? stall + 1 : 0;
        if (stall >= 2) { *st = RSRR_OK; return sw + 1; }
        prev = mx;
    }
    *st = RSRR_ENOTCONV;
    return -1;
}

extern "C" rsrr_status rsrr_basis(rsrr_ctx* c, int n, int NL, double* S, int lds, double delta, double* Q, int ldq,
                                  int kmax, int* k, double* sigma)
{
    if (!c) return -1;
    if (n < 1) return -2;
    if (NL < 1) return -3;
    if (!S) return -4;
    if (lds < n) return -5;
    if (!(delta > 0.0 && delta < 1.0)) return -6;
    if (!Q) return -7;
    if (ldq < n) return -8;
    if (kmax < 1) return -9;
    if (!k) return -10;
    RSRR_HIP(hipSetDevice(c->device));
    double2* A = (double2*)S;
    // normalise the columns of S (Sec. 4.2); zero columns stay zero
    double* nrm = (double*)ws_get(c, WS_B5, (size_t)NL * 8);
    int* ord = (int*)ws_get(c, WS_B4, (size_t)NL * 4);
    double* inv = (double*)ws_get(c, WS_B3, (size_t)NL * 8);
    if (!nrm || !ord || !inv) return RSRR_ENOMEM;
    RSRR_HIP(colnorms(c->stream, n, NL, A, lds, 0, nrm, 1));
    std::vector<double> h(NL);
    RSRR_HIP(hipMemcpyAsync(h.data(), nrm, (size_t)NL * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    for (auto& v : h) v = v > 0.0 ? 1.0 / v : 0.0;
    RSRR_HIP(hipMemcpyAsync(inv, h.data(), (size_t)NL * 8, hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(scale_cols(c->stream, n, NL, A, lds, inv));
    RSRR_HIP(hipStreamSynchronize(c->stream));

    // Range sketch + BCGS2 + one-sided Jacobi on the small factor.
    //   Y = S Omega (Omega: NL x l seeded Gaussian), Q_Y = BCGS2(Y) with the r
    //   numerically independent columns kept, X = [S^H Q_Y; I_r]: Jacobi
    //   rotations J on the columns make the top part V Sigma (right singular
    //   vectors of B = Q_Y^H S) and the bottom part J = W, the left singular
    //   vectors of B; S's left singular vectors are Q_Y W.  When NL >= 2r the
    //   top part is replaced by R from S^H Q_Y = Q_X R (same Gram matrix, so the
    //   same rotations and singular values, on r rows instead of NL).
    // When l = min(n, NL) the sketch spans range(S) and this is the SVD of S.  A
    // smaller l is accepted when the sketch came out rank deficient (r < l) or its
    // smallest singular value is at the rounding floor (<= 1e-15 sigma_1);
    // otherwise l doubles.
    const int m = std::min(n, NL);
    int l = std::min(m, c->basis_sketch_max);
    const double tol = 4.0 * std::max(1.0, std::sqrt((double)NL)) * 2.220446049250313e-16;
    rsrr_status st = RSRR_OK;
    std::vector<int> o, idx;
    std::vector<double> sv, hq;
    double2* Yu = nullptr;
    double2* X = nullptr;
    int r = 0, xr = 0;  // X = [top (xr rows); W (r rows)] after the Jacobi sweeps
    for (;;) {
        double2* Y = (double2*)ws_get(c, WS_TLU, (size_t)n * l * 16);
        double2* Om = (double2*)ws_get(c, WS_TRES, (size_t)std::max((long)NL * l, (long)n * l) * 16);
        void* Wb = ws_get(c, WS_D64, bcgs2_work_bytes(n, l));
        double* n0 = (double*)ws_get(c, WS_B7, (size_t)l * 8);
        if (!Y || !Om || !Wb || !n0) return RSRR_ENOMEM;
        if (l >= NL) {
            // no sketch needed: orthonormalise S itself (l == NL)
            RSRR_HIP(copy_c128(c->stream, n, NL, A, lds, 0, Y, n, 0, 1));
        } else {
            RSRR_HIP(gaussian(c->stream, Om, NL, l, NL, 0x5eed5eedull + (unsigned long long)l));
            RSRR_HIP(zgemm(c->stream, 0, 0, n, l, NL, 1.0, A, lds, 0, Om, NL, 0, 0.0, Y, n, 0, 1));
        }
        RSRR_HIP(bcgs2(c->stream, Y, n, n, l, Wb, n0));
        // keep the nonzero (independent) columns of Q_Y
        RSRR_HIP(colnorms(c->stream, n, l, Y, n, 0, n0, 1));
        hq.assign(l, 0.0);
        RSRR_HIP(hipMemcpyAsync(hq.data(), n0, (size_t)l * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        idx.clear();
        for (int i = 0; i < l; ++i)
            if (hq[i] > 0.5) idx.push_back(i);
        r = (int)idx.size();
        if (r == 0) break;
        Yu = Y;
        if (r < l) {
            // Omega is dead: its buffer takes the compacted Q_Y
            std::vector<double> ones(r, 1.0);
            RSRR_HIP(hipMemcpyAsync(ord, idx.data(), (size_t)r * 4, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(hipMemcpyAsync(inv, ones.data(), (size_t)r * 8, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(gather_scale(c->stream, Y, n, n, ord, inv, Om, n, r));
            RSRR_HIP(hipStreamSynchronize(c->stream));
            Yu = Om;
        }
        if (NL >= 2 * r) {
            // QR first: B^H = S^H Q_Y = Q_X R (BCGS2), then the Jacobi rotations on
            // [R; I_r]: R has the Gram matrix of B^H, so the rotations, singular
            // values and W are those of B^H, on 2r rows instead of NL + r
            double2* Xs = (double2*)ws_get(c, WS_B0, (size_t)NL * r * 16);
            double2* Xq = (double2*)ws_get(c, WS_B1, (size_t)NL * r * 16);
            void* Wq = ws_get(c, WS_D64, bcgs2_work_bytes(NL, r));
            double* nq = (double*)ws_get(c, WS_B7, (size_t)r * 8);
            X = (double2*)ws_get(c, WS_R, (size_t)2 * r * r * 16);
            if (!Xs || !Xq || !Wq || !nq || !X) return RSRR_ENOMEM;
            RSRR_HIP(zgemm(c->stream, 1, 0, NL, r, n, 1.0, A, lds, 0, Yu, n, 0, 0.0, Xs, NL, 0, 1));
            RSRR_HIP(copy_c128(c->stream, NL, r, Xs, NL, 0, Xq, NL, 0, 1));
            RSRR_HIP(bcgs2(c->stream, Xq, NL, NL, r, Wq, nq));
            RSRR_HIP(zgemm(c->stream, 1, 0, r, r, NL, 1.0, Xq, NL, 0, Xs, NL, 0, 0.0, X, 2 * r, 0, 1));
            xr = r;
        } else {
            X = (double2*)ws_get(c, WS_R, (size_t)(NL + r) * r * 16);
            if (!X) return RSRR_ENOMEM;
            RSRR_HIP(zgemm(c->stream, 1, 0, NL, r, n, 1.0, A, lds, 0, Yu, n, 0, 0.0, X, NL + r, 0, 1));
            xr = NL;
        }
        RSRR_HIP(eye(c->stream, X, xr + r, xr, r));
        if (jacobi_svd(c, X, xr + r, xr, xr + r, r, 80, tol, &st) < 0) return st;
        double* cn = (double*)ws_get(c, WS_B5, (size_t)r * 8);
        if (!cn) return RSRR_ENOMEM;
        RSRR_HIP(colnorms(c->stream, xr, r, X, xr + r, 0, cn, 1));
        sv.assign(r, 0.0);
        RSRR_HIP(hipMemcpyAsync(sv.data(), cn, (size_t)r * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        o.resize(r);
        std::iota(o.begin(), o.end(), 0);
        std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return sv[x] > sv[y]; });
        const double s1 = sv[o[0]], sl = sv[o[r - 1]];
        if (l >= m || r < l || !(s1 > 0.0) || sl <= 1e-15 * s1) break;
        l = std::min(m, 2 * l);
    }
    const double s1 = r > 0 ? sv[o[0]] : 0.0;
    int kk = 0;
    for (int i = 0; i < r; ++i)
        if (s1 > 0.0 && sv[o[i]] > delta * s1) ++kk;
    if (sigma)
        for (int i = 0; i < m; ++i) sigma[i] = i < r ? sv[o[i]] : 0.0;
    *k = kk;
    const int kw = std::min(kk, kmax);
    if (kw > 0) {
        // W sorted by singular value (bottom r rows of X), then Q = Q_Y W
        std::vector<double> ones(kw, 1.0);
        double2* Ws = (double2*)ws_get(c, WS_B2, (size_t)r * kw * 16);
        if (!Ws) return RSRR_ENOMEM;
        RSRR_HIP(hipMemcpyAsync(ord, o.data(), (size_t)kw * 4, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(hipMemcpyAsync(inv, ones.data(), (size_t)kw * 8, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(gather_scale(c->stream, X + xr, xr + r, r, ord, inv, Ws, r, kw));
        RSRR_HIP(zgemm(c->stream, 0, 0, n, kw, r, 1.0, Yu, n, 0, Ws, r, 0, 0.0, (double2*)Q, ldq, 0, 1));
    }
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}

// Taylor degree for the Helmholtz expansion: smallest d with
// (rho r)^(d+1) / (d+1)! * e^(rho r) < 1e-17 (remainder bound of e^{i(z-gamma) r}).
static int taylor_degree(double rho, double rmax)
{
    const double x = rho * rmax;
    double term = 1.0;
    for (int d = 0; d < 200; ++d) {
        term *= x / (d + 1);
        if (term * std::exp(x) < 1e-17) return d;
    }
    return 200;
}

extern "C" rsrr_status rsrr_project(rsrr_ctx* c, const rsrr_nep* nep, const double* Qp, int ldq, int k,
                                    const double* gamma, double radius, double* AQ, int max_terms, int* J_eff,
                                    rsrr_term* terms_out)
{
    if (!c) return -1;
    if (!nep || nep->n < 1) return -2;
    if (nep->kind == RSRR_T_SEPARABLE && (nep->J < 1 || !nep->A || nep->lda < nep->n || !nep->terms)) return -2;
    if (nep->kind == RSRR_T_HELMHOLTZ && (!nep->points || !(nep->w > 0))) return -2;
    if (nep->kind == RSRR_T_SPARSE && !csr_nep_ok(nep)) return -2;
    if (nep->kind != RSRR_T_SEPARABLE && nep->kind != RSRR_T_HELMHOLTZ && nep->kind != RSRR_T_SPARSE) return -2;
    if (!Qp) return -3;
    if (ldq < nep->n) return -4;
    if (k < 1 || k > nep->n) return -5;
    if (!gamma) return -6;
    if (!(radius > 0)) return -7;
    if (!AQ) return -8;
    if (!J_eff) return -10;
    if (!terms_out) return -11;
    RSRR_HIP(hipSetDevice(c->device));
    const int n = nep->n;
    const double2* Q = (const double2*)Qp;
    double2* out = (double2*)AQ;
    if (nep->kind == RSRR_T_SEPARABLE) {
        const int J = nep->J;
        if (max_terms < J) return -9;
        double2* W = (double2*)ws_get(c, WS_B0, (size_t)J * n * k * 16);
        if (!W) return RSRR_ENOMEM;
        // W_j = A_j Q, AQ_j = Q^H W_j (all j in one batched launch each)
        RSRR_HIP(zgemm(c->stream, 0, 0, n, k, n, 1.0, (const double2*)nep->A, nep->lda, (long)nep->lda * n, Q, ldq, 0,
                       0.0, W, n, (long)n * k, J));
        RSRR_HIP(zgemm(c->stream, 1, 0, k, k, n, 1.0, Q, ldq, 0, W, n, (long)n * k, 0.0, out, k, (long)k * k, J));
        for (int j = 0; j < J; ++j) terms_out[j] = nep->terms[j];
        *J_eff = J;
    } else if (nep->kind == RSRR_T_SPARSE) {
        const int J = nep->J;
        if (max_terms < J) return -9;
        double2* W = (double2*)ws_get(c, WS_B0, (size_t)J * n * k * 16);
        double2* one = (double2*)ws_get(c, WS_COEF, 16);
        if (!W || !one) return RSRR_ENOMEM;
        const double2 h1 = make_double2(1.0, 0.0);
        RSRR_HIP(hipMemcpyAsync(one, &h1, 16, hipMemcpyHostToDevice, c->stream));
        CsrDev d;
        RSRR_TRY(csr_upload(c, nep, d));
        // W_j = A_j Q from the sparse rows, then AQ_j = Q^H W_j (one batched launch)
        for (int j = 0; j < J; ++j)
            RSRR_HIP(csr_apply(c->stream, n, 1, d.terms + j, one, 1, k, Q, ldq, W + (size_t)j * n * k, n, d.bad));
        RSRR_HIP(zgemm(c->stream, 1, 0, k, k, n, 1.0, Q, ldq, 0, W, n, (long)n * k, 0.0, out, k, (long)k * k, J));
        RSRR_TRY(csr_check(c, d));
        for (int j = 0; j < J; ++j) terms_out[j] = nep->terms[j];
        *J_eff = J;
    } else {
        // diameter bound of the point set from the host copy of the points
        std::vector<double> pts((size_t)3 * n);
        RSRR_HIP(hipMemcpyAsync(pts.data(), nep->points, pts.size() * 8, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        double cx = 0, cy = 0, cz = 0;
        for (int i = 0; i < n; ++i) { cx += pts[3 * i]; cy += pts[3 * i + 1]; cz += pts[3 * i + 2]; }
        cx /= n; cy /= n; cz /= n;
        double rr = 0;
        for (int i = 0; i < n; ++i) {
            const double dx = pts[3 * i] - cx, dy = pts[3 * i + 1] - cy, dz = pts[3 * i + 2] - cz;
            rr = std::max(rr, std::sqrt(dx * dx + dy * dy + dz * dz));
        }
        const int d = taylor_degree(radius, 2.0 * rr);
        if (max_terms < d + 1) return -9;
        // groups of G terms: generated together, then two batched products T_p Q and Q^H (T_p Q)
        const int P = d + 1;
        const size_t per = (size_t)n * n * 16 + (size_t)n * k * 16;
        size_t fr = 0, tot = 0;
        RSRR_HIP(hipMemGetInfo(&fr, &tot));
        size_t budget = std::min<size_t>(fr / 4, (size_t)8 << 30);
        if (c->ws_budget) budget = std::min(budget, c->ws_budget);
        const int G = (int)std::max<size_t>(1, std::min<size_t>((size_t)P, budget / per));
        double2* Tp = (double2*)ws_get(c, WS_B0, (size_t)G * n * n * 16);
        double2* W = (double2*)ws_get(c, WS_B1, (size_t)G * n * k * 16);
        if (!Tp || !W) return RSRR_ENOMEM;
        const long nn = (long)n * n, nk = (long)n * k;
        for (int p0 = 0; p0 < P; p0 += G) {
            const int g = std::min(G, P - p0);
            RSRR_HIP(helmholtz_taylor_range(c->stream, n, nep->points, nep->w, gamma[0], gamma[1], p0, g, Tp, n, nn));
            RSRR_HIP(zgemm(c->stream, 0, 0, n, k, n, 1.0, Tp, n, nn, Q, ldq, 0, 0.0, W, n, nk, g));
            RSRR_HIP(zgemm(c->stream, 1, 0, k, k, n, 1.0, Q, ldq, 0, W, n, nk, 0.0, out + (size_t)p0 * k * k, k,
                           (long)k * k, g));
        }
        for (int p = 0; p < P; ++p) {
            rsrr_term t = {};
            t.c_re = 1.0; t.p = p; t.z0_re = gamma[0]; t.z0_im = gamma[1];
            terms_out[p] = t;
        }
        *J_eff = P;
    }
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}
