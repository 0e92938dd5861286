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
// with the small N x K table c^T as the right operand.  The table is formed
// on the device (one thread per point) from the points copied next to it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "common.h"
#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

// Scratch of rsrr_moments_noalloc: the raw points followed by the N x K
// coefficient table, in a file-scope device array (each GPU the library runs
// on holds its own copy until the process ends).  Host code reaches it only
// through the per-device address that hipGetSymbolAddress returns.
constexpr long MOMENTS_NOALLOC_MAX = 1L << 16;   // complex entries: N + N*K <= 65536 (1 MiB)
static __device__ __align__(256) double2 scratch[MOMENTS_NOALLOC_MAX];

namespace {

std::mutex g_scratch_mu;
std::vector<double2*> g_scratch_ptr;  // by device ordinal

// c_{alpha,i} = omega_i zeta_i^alpha (column alpha, ld N), zeta_i = (z_i - gamma)/rho,
// log omega_i = -sum_{j != i} log((zeta_i - zeta_j)/C): one thread per point.
__global__ __launch_bounds__(256) void moment_weights_kernel(const double2* __restrict__ z, int N, int K, double gre,
                                                             double gim, double rho, double cap,
                                                             double2* __restrict__ cw)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double2 zi = make_double2((z[i].x - gre) / rho, (z[i].y - gim) / rho);
    double lr = 0.0, li = 0.0;
    for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        const double2 zj = make_double2((z[j].x - gre) / rho, (z[j].y - gim) / rho);
        const double dx = (zi.x - zj.x) / cap, dy = (zi.y - zj.y) / cap;
        lr -= log(hypot(dx, dy));
        li -= atan2(dy, dx);
    }
    double sn, cs;
    sincos(li, &sn, &cs);
    const double m = exp(lr);
    double2 w = make_double2(m * cs, m * sn);
    for (int a = 0; a < K; ++a) {
        cw[(long)a * N + i] = w;
        w = cmul(w, zi);
    }
}

rsrr_status check_args(rsrr_ctx* c, int n, int N, int L, const double* S, int lds, const double* z,
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
    for (int i = 0; i < N; ++i)  // coincident points have no barycentric weight
        for (int j = 0; j < i; ++j)
            if (z[2 * i] == z[2 * j] && z[2 * i + 1] == z[2 * j + 1]) return -7;
    return RSRR_OK;
}

// The points and the coefficient table in `work` (N + N*K complex), then M = S Z.
rsrr_status moments_run(rsrr_ctx* c, int n, int N, int L, const double* S, int lds, const double* z,
                        const double* gamma, double rho, double capacity, int K, double* M, int ldm, double2* work)
{
    double2* zd_ = work;
    double2* cw = work + N;
    RSRR_HIP(hipMemcpyAsync(zd_, z, (size_t)N * 16, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(moment_weights_kernel, dim3((N + 255) / 256), dim3(256), 0, c->stream, zd_, N, K, gamma[0],
                       gamma[1], rho, capacity, cw);
    RSRR_HIP(hipGetLastError());
    // batch l: A = S + l lds (n x N, ld L lds), C = M + l ldm (n x K, ld L ldm)
    RSRR_HIP(zgemm(c->stream, 0, 0, n, K, N, 1.0, (const double2*)S, L * lds, lds, cw, N, 0, 0.0, (double2*)M,
                   L * ldm, ldm, L));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}

}  // namespace

// Once per device, with that device current (rsrr_create): the device address of `scratch`.
rsrr_status noalloc_scratch_setup(int device, void** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return RSRR_EDEVICE;
        }
        g_scratch_ptr[device] = (double2*)p;
    }
    *out = g_scratch_ptr[device];
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_moments(rsrr_ctx* c, int n, int N, int L, const double* S, int lds, const double* z,
                                    const double* gamma, double rho, double capacity, int K, double* M, int ldm)
{
    const rsrr_status e = check_args(c, n, N, L, S, lds, z, gamma, rho, capacity, K, M, ldm);
    if (e) return e;
    RSRR_HIP(hipSetDevice(c->device));
    double2* work = (double2*)ws_get(c, WS_COEF, ((size_t)N + (size_t)N * K) * 16);
    if (!work) return RSRR_ENOMEM;
    return moments_run(c, n, N, L, S, lds, z, gamma, rho, capacity, K, M, ldm, work);
}

extern "C" rsrr_status rsrr_moments_noalloc(rsrr_ctx* c, int n, int N, int L, const double* S, int lds,
                                            const double* z, const double* gamma, double rho, double capacity, int K,
                                            double* M, int ldm)
{
    const rsrr_status e = check_args(c, n, N, L, S, lds, z, gamma, rho, capacity, K, M, ldm);
    if (e) return e;
    if ((long)N + (long)N * K > MOMENTS_NOALLOC_MAX) return RSRR_ELIMIT;
    if (!c->noalloc_scratch) return RSRR_EDEVICE;
    RSRR_HIP(hipSetDevice(c->device));
    return moments_run(c, n, N, L, S, lds, z, gamma, rho, capacity, K, M, ldm, (double2*)c->noalloc_scratch);
}
