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
            if (jacobi_round(c->stream, A, lda, m, m_apply, p, r, 2, tol, zthr2, off + (size_t)r * pairs) !=
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

    // one-sided Jacobi: S V = U Sigma
    const double tol = 4.0 * std::max(1.0, std::sqrt((double)n)) * 2.220446049250313e-16;
    rsrr_status st = RSRR_OK;
    if (jacobi_svd(c, A, lds, n, n, NL, 80, tol, &st) < 0) return st;

    // singular values = column norms, sorted descending
    RSRR_HIP(colnorms(c->stream, n, NL, A, lds, 0, nrm, 1));
    RSRR_HIP(hipMemcpyAsync(h.data(), nrm, (size_t)NL * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    std::vector<int> o(NL);
    std::iota(o.begin(), o.end(), 0);
    std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return h[a] > h[b]; });
    const int m = std::min(n, NL);
    const double s1 = h[o[0]];
    int kk = 0;
    for (int i = 0; i < m; ++i)
        if (s1 > 0.0 && h[o[i]] > delta * s1) ++kk;
    if (sigma)
        for (int i = 0; i < m; ++i) sigma[i] = h[o[i]];
    *k = kk;
    const int kw = std::min(kk, kmax);
    std::vector<double> iv(kw);
    for (int i = 0; i < kw; ++i) iv[i] = 1.0 / h[o[i]];
    RSRR_HIP(hipMemcpyAsync(ord, o.data(), (size_t)kw * 4, hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(hipMemcpyAsync(inv, iv.data(), (size_t)kw * 8, hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(gather_scale(c->stream, A, lds, n, ord, inv, (double2*)Q, ldq, kw));
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
        double2* Tp = (double2*)ws_get(c, WS_B0, (size_t)n * n * 16);
        double2* W = (double2*)ws_get(c, WS_B1, (size_t)n * k * 16);
        if (!Tp || !W) return RSRR_ENOMEM;
        for (int p = 0; p <= d; ++p) {
            RSRR_HIP(helmholtz_taylor(c->stream, n, nep->points, nep->w, gamma[0], gamma[1], p, Tp, n));
            RSRR_HIP(zgemm(c->stream, 0, 0, n, k, n, 1.0, Tp, n, 0, Q, ldq, 0, 0.0, W, n, 0, 1));
            RSRR_HIP(zgemm(c->stream, 1, 0, k, k, n, 1.0, Q, ldq, 0, W, n, 0, 0.0, out + (size_t)p * k * k, k, 0, 1));
            rsrr_term t = {};
            t.c_re = 1.0; t.p = p; t.z0_re = gamma[0]; t.z0_im = gamma[1];
            terms_out[p] = t;
        }
        *J_eff = d + 1;
    }
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}
