// C ABI: the moment matrix of the resolvent moment scheme (Sec. 4.1) from the
// sampling matrix, M = S Z (eq. MS).
//
// M_alpha = sum_i c_{alpha,i} X_i with X_i the i-th L-column block of S and
// c_{alpha,i} = omega_i zeta_i^alpha (eq. Malpha), zeta_i = (z_i - gamma)/rho,
// omega_i the barycentric weights of the zeta_i (eq. bary-wt) with every
// factor divided by the capacity C (the scaling Sec. 3.3 recommends against
// under- and overflow).  For a fixed probe column l the blocks form an
// n x N matrix (stride L lds between points) and M's columns alpha L + l an
// n x K matrix, so M is one batched FP64 MFMA GEMM over the L probe columns
// with the small N x K table c^T as the right operand.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

extern "C" rsrr_status rsrr_moments(rsrr_ctx* c, int n, int N, int L, const double* S, int lds, const double* z,
                                    const double* gamma, double rho, double capacity, int K, double* M, int ldm)
{
    if (!c) return -1;
    if (n < 1) return -2;
    if (N < 1) return -3;
    if (L < 1) return -4;
    if (!S) return -5;
    if (lds < n) return -6;
    if (!z) return -7;
    if (!gamma) return -8;
    if (!(rho > 0)) return -9;
    if (!(capacity > 0)) return -10;
    if (K < 1 || K > N) return -11;
    if (!M) return -12;
    if (ldm < n) return -13;
    RSRR_HIP(hipSetDevice(c->device));
    // weights in log form: log omega_i = -sum_{j != i} log((zeta_i - zeta_j)/C)
    std::vector<zd> zeta(N);
    for (int i = 0; i < N; ++i) zeta[i] = (zd(z[2 * i], z[2 * i + 1]) - zd(gamma[0], gamma[1])) / rho;
    std::vector<double2> cw((size_t)N * K);  // column alpha: c_{alpha, i}, ld N
    for (int i = 0; i < N; ++i) {
        zd lw(0.0, 0.0);
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            const zd d = (zeta[i] - zeta[j]) / capacity;
            if (d == zd(0.0, 0.0)) return -7;  // coincident points
            lw -= std::log(d);
        }
        zd w = std::exp(lw);
        for (int a = 0; a < K; ++a) {
            cw[(size_t)a * N + i] = make_double2(w.real(), w.imag());
            w *= zeta[i];
        }
    }
    double2* dc = (double2*)ws_get(c, WS_COEF, cw.size() * 16);
    if (!dc) return RSRR_ENOMEM;
    RSRR_HIP(hipMemcpyAsync(dc, cw.data(), cw.size() * 16, hipMemcpyHostToDevice, c->stream));
    // batch l: A = S + l lds (n x N, ld L lds), C = M + l ldm (n x K, ld L ldm)
    RSRR_HIP(zgemm(c->stream, 0, 0, n, K, N, 1.0, (const double2*)S, L * lds, lds, dc, N, 0, 0.0, (double2*)M,
                   L * ldm, ldm, L));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}
