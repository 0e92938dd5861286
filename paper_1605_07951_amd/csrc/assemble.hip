// Assembly of T(z_k) for a batch of sampling points (RSRR Step 2 needs
// T(z_k) at every point; it is formed once and used once, Sec. 1).
//
// Separable form T(z) = sum_j f_j(z) A_j: one pass over the A_j (FP64)
// serves PG points per thread; each entry is summed in FP64 and written as
// c64 (LU input of the mixed path) and/or c128 (LU input of the FP64 path,
// or the FP64 copy that the refinement residual uses).
//
// Helmholtz single-layer kernel (eq. nyes, kernel G): the distance r_ij is
// formed once per entry and the PG points reuse it; e^{i z r} is evaluated
// in FP64 as e^{-Im(z) r} (cos(Re(z) r) + i sin(Re(z) r)).
//
// Both kernels also write, per point and per workgroup, the partial sum of
// |T_ij|^2 (FP64); frob_finish reduces the partials in a fixed order, so
// ||T(z_k)||_F is reproducible bit for bit.
#include "common.h"
#include "kernels.h"

namespace rsrr {

constexpr int AS_NT = 256;
constexpr int AS_PG = 24;     // points per thread pass
constexpr int AS_MAXJ = 64;   // separable terms held in LDS

// element e of a column-major n x n matrix: (e % n, e / n)
template <bool O64, bool O128>
__global__ __launch_bounds__(AS_NT) void assemble_sep_kernel(
    int n, int J, const double2* __restrict__ A, int lda, long sAj,
    const double2* __restrict__ coef,   // [J][B] complex, point-fastest
    int B, int k0,                      // this launch handles points k0 .. k0+PG-1 (< B)
    float2* __restrict__ T64, int ld64, long s64,
    double2* __restrict__ T128, int ld128, long s128,
    double* __restrict__ frob_part, int nparts)
{
    __shared__ double2 f[AS_MAXJ][AS_PG];
    __shared__ double red[AS_NT / 64][AS_PG];
    const int tid = threadIdx.x;
    const int npts = min(AS_PG, B - k0);
    for (int e = tid; e < J * AS_PG; e += AS_NT) {
        const int j = e / AS_PG, p = e % AS_PG;
        f[j][p] = (p < npts) ? coef[(long)j * B + k0 + p] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const long nn = (long)n * n;
    const long e = (long)blockIdx.x * AS_NT + tid;
    double acc[AS_PG];
#pragma unroll
    for (int p = 0; p < AS_PG; ++p) acc[p] = 0.0;
    if (e < nn) {
        const int i = (int)(e % n), c = (int)(e / n);
        double2 t[AS_PG];
#pragma unroll
        for (int p = 0; p < AS_PG; ++p) t[p] = make_double2(0.0, 0.0);
        for (int j = 0; j < J; ++j) {
            const double2 a = A[(long)j * sAj + i + (long)c * lda];
#pragma unroll
            for (int p = 0; p < AS_PG; ++p) t[p] = cfma(t[p], f[j][p], a);
        }
#pragma unroll
        for (int p = 0; p < AS_PG; ++p) {
            if (p < npts) {
                const long k = k0 + p;
                if (O64) T64[k * s64 + i + (long)c * ld64] = to_c64(t[p]);
                if (O128) T128[k * s128 + i + (long)c * ld128] = t[p];
                acc[p] = t[p].x * t[p].x + t[p].y * t[p].y;
            }
        }
    }
    // workgroup partial sums of |T|^2 per point
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int p = 0; p < AS_PG; ++p) {
        double v = acc[p];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][p] = v;
    }
    __syncthreads();
    if (tid < AS_PG && tid < npts) {
        double v = 0.0;
        for (int w = 0; w < AS_NT / 64; ++w) v += red[w][tid];
        frob_part[(long)(k0 + tid) * nparts + blockIdx.x] = v;
    }
}

template <bool O64, bool O128>
__global__ __launch_bounds__(AS_NT) void assemble_helm_kernel(
    int n, const double* __restrict__ pts, double w,
    const double2* __restrict__ z, int B, int k0,
    float2* __restrict__ T64, int ld64, long s64,
    double2* __restrict__ T128, int ld128, long s128,
    double* __restrict__ frob_part, int nparts)
{
    __shared__ double red[AS_NT / 64][AS_PG];
    const int tid = threadIdx.x;
    const int npts = min(AS_PG, B - k0);
    const long nn = (long)n * n;
    const long e = (long)blockIdx.x * AS_NT + tid;
    const double inv4pi = 0.25 / M_PI;
    const double diag_re = 0.5 * sqrt(w / M_PI);
    double acc[AS_PG];
#pragma unroll
    for (int p = 0; p < AS_PG; ++p) acc[p] = 0.0;
    if (e < nn) {
        const int i = (int)(e % n), c = (int)(e / n);
        double r = 0.0;
        if (i != c) {
            const double dx = pts[3 * i] - pts[3 * c];
            const double dy = pts[3 * i + 1] - pts[3 * c + 1];
            const double dz = pts[3 * i + 2] - pts[3 * c + 2];
            r = sqrt(dx * dx + dy * dy + dz * dz);
        }
        const double scale = (i != c) ? w * inv4pi / r : 0.0;
#pragma unroll
        for (int p = 0; p < AS_PG; ++p) {
            if (p < npts) {
                const long k = k0 + p;
                const double2 zk = z[k];
                double2 t;
                if (i != c) {
                    double s, co;
                    sincos(zk.x * r, &s, &co);
                    const double m = scale * exp(-zk.y * r);
                    t = make_double2(m * co, m * s);
                } else {
                    // sqrt(w/pi)/2 + i z w/(4 pi)
                    t = make_double2(diag_re - zk.y * w * inv4pi, zk.x * w * inv4pi);
                }
                if (O64) T64[k * s64 + i + (long)c * ld64] = to_c64(t);
                if (O128) T128[k * s128 + i + (long)c * ld128] = t;
                acc[p] = t.x * t.x + t.y * t.y;
            }
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int p = 0; p < AS_PG; ++p) {
        double v = acc[p];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][p] = v;
    }
    __syncthreads();
    if (tid < AS_PG && tid < npts) {
        double v = 0.0;
        for (int ww = 0; ww < AS_NT / 64; ++ww) v += red[ww][tid];
        frob_part[(long)(k0 + tid) * nparts + blockIdx.x] = v;
    }
}

// ||T_k||_F from the partial sums, one wavefront per point, fixed order.
__global__ __launch_bounds__(64) void frob_finish_kernel(const double* __restrict__ part, int nparts,
                                                          double* __restrict__ out)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    double v = 0.0;
    for (int t = lane; t < nparts; t += 64) v += part[(long)k * nparts + t];
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) out[k] = sqrt(v);
}

// ----------------------------------------------------------------------------
// One size bucket of a ragged batch in one launch: instance q = blockIdx.y with
// its own n, terms A_j and coefficient rows (coef + coff, [J][N] point-fastest),
// point group blockIdx.z; its points are bucket matrices koff .. koff+N-1 (ld P,
// strides s64/s128), its partial sums at frob_part + k nparts_max.
// ----------------------------------------------------------------------------
template <bool O64, bool O128>
__global__ __launch_bounds__(AS_NT) void assemble_sep_group_kernel(
    const SepInstance* __restrict__ ins, const double2* __restrict__ coef, int P,
    float2* __restrict__ T64, long s64, double2* __restrict__ T128, long s128,
    double* __restrict__ frob_part, int nparts_max)
{
    __shared__ double2 f[AS_MAXJ][AS_PG];
    __shared__ double red[AS_NT / 64][AS_PG];
    const SepInstance in = ins[blockIdx.y];
    const int n = in.n, J = in.J, B = in.N;
    const int k0 = blockIdx.z * AS_PG;
    const long nn = (long)n * n;
    const int nparts = (int)((nn + AS_NT - 1) / AS_NT);
    if (k0 >= B || (int)blockIdx.x >= nparts) return;   // uniform over the workgroup
    const int tid = threadIdx.x;
    const int npts = min(AS_PG, B - k0);
    for (int e = tid; e < J * AS_PG; e += AS_NT) {
        const int j = e / AS_PG, p = e % AS_PG;
        f[j][p] = (p < npts) ? coef[in.coff + (long)j * B + k0 + p] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const long e = (long)blockIdx.x * AS_NT + tid;
    double acc[AS_PG];
#pragma unroll
    for (int p = 0; p < AS_PG; ++p) acc[p] = 0.0;
    if (e < nn) {
        const int i = (int)(e % n), c = (int)(e / n);
        double2 t[AS_PG];
#pragma unroll
        for (int p = 0; p < AS_PG; ++p) t[p] = make_double2(0.0, 0.0);
        for (int j = 0; j < J; ++j) {
            const double2 a = in.A[(long)j * in.lda * n + i + (long)c * in.lda];
#pragma unroll
            for (int p = 0; p < AS_PG; ++p) t[p] = cfma(t[p], f[j][p], a);
        }
#pragma unroll
        for (int p = 0; p < AS_PG; ++p) {
            if (p < npts) {
                const long k = in.koff + k0 + p;
                if (O64) T64[k * s64 + i + (long)c * P] = to_c64(t[p]);
                if (O128) T128[k * s128 + i + (long)c * P] = t[p];
                acc[p] = t[p].x * t[p].x + t[p].y * t[p].y;
            }
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int p = 0; p < AS_PG; ++p) {
        double v = acc[p];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][p] = v;
    }
    __syncthreads();
    if (tid < AS_PG && tid < npts)  {
        double v = 0.0;
        for (int w = 0; w < AS_NT / 64; ++w) v += red[w][tid];
        frob_part[(in.koff + k0 + tid) * (long)nparts_max + blockIdx.x] = v;
    }
}

// ||T_k||_F of every matrix of the bucket: matrix k of order nk[k] has
// ceil(nk^2 / AS_NT) partial sums at part + k nparts_max.
__global__ __launch_bounds__(64) void frob_finish_group_kernel(const double* __restrict__ part, int nparts_max,
                                                                const int* __restrict__ nk, double* __restrict__ out)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    const long nn = (long)nk[k] * nk[k];
    const int nparts = (int)((nn + AS_NT - 1) / AS_NT);
    double v = 0.0;
    for (int t = lane; t < nparts; t += 64) v += part[(long)k * nparts_max + t];
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) out[k] = sqrt(v);
}

hipError_t assemble_separable_group(hipStream_t st, const SepInstance* ins, int nins, int nmax, int Nmax,
                                    const double2* coef, int P, int M, const int* nk, float2* T64, long s64,
                                    double2* T128, long s128, double* frob_part, double* frob)
{
    const int nparts_max = (int)(((long)nmax * nmax + AS_NT - 1) / AS_NT);
    const dim3 g((unsigned)nparts_max, (unsigned)nins, (unsigned)((Nmax + AS_PG - 1) / AS_PG));
    if (T64 && T128)
        hipLaunchKernelGGL((assemble_sep_group_kernel<true, true>), g, dim3(AS_NT), 0, st, ins, coef, P, T64, s64, T128,
                           s128, frob_part, nparts_max);
    else if (T64)
        hipLaunchKernelGGL((assemble_sep_group_kernel<true, false>), g, dim3(AS_NT), 0, st, ins, coef, P, T64, s64,
                           T128, s128, frob_part, nparts_max);
    else
        hipLaunchKernelGGL((assemble_sep_group_kernel<false, true>), g, dim3(AS_NT), 0, st, ins, coef, P, T64, s64,
                           T128, s128, frob_part, nparts_max);
    hipLaunchKernelGGL(frob_finish_group_kernel, dim3(M), dim3(64), 0, st, frob_part, nparts_max, nk, frob);
    return hipGetLastError();
}

int assemble_max_terms() { return AS_MAXJ; }

hipError_t assemble_separable(hipStream_t st, int n, int J, const double2* A, int lda, const double2* coef, int B,
                              float2* T64, int ld64, long s64, double2* T128, int ld128, long s128,
                              double* frob_part, double* frob)
{
    if (J > AS_MAXJ) return hipErrorInvalidValue;
    const long nn = (long)n * n;
    const int nparts = (int)((nn + AS_NT - 1) / AS_NT);
    const long sAj = (long)lda * n;
    for (int k0 = 0; k0 < B; k0 += AS_PG) {
        if (T64 && T128)
            hipLaunchKernelGGL((assemble_sep_kernel<true, true>), dim3(nparts), dim3(AS_NT), 0, st, n, J, A, lda, sAj,
                               coef, B, k0, T64, ld64, s64, T128, ld128, s128, frob_part, nparts);
        else if (T64)
            hipLaunchKernelGGL((assemble_sep_kernel<true, false>), dim3(nparts), dim3(AS_NT), 0, st, n, J, A, lda,
                               sAj, coef, B, k0, T64, ld64, s64, T128, ld128, s128, frob_part, nparts);
        else
            hipLaunchKernelGGL((assemble_sep_kernel<false, true>), dim3(nparts), dim3(AS_NT), 0, st, n, J, A, lda,
                               sAj, coef, B, k0, T64, ld64, s64, T128, ld128, s128, frob_part, nparts);
    }
    hipLaunchKernelGGL(frob_finish_kernel, dim3(B), dim3(64), 0, st, frob_part, nparts, frob);
    return hipGetLastError();
}

// Norm partials (and the complex FP32 copy) of dense FP64 matrices formed by
// another kernel, with the partial layout of the assembly kernels above.
template <bool O64>
__global__ __launch_bounds__(AS_NT) void finish_dense_kernel(int n, const double2* __restrict__ T128, int ld128,
                                                             long s128, float2* __restrict__ T64, int ld64, long s64,
                                                             double* __restrict__ frob_part, int nparts)
{
    __shared__ double red[AS_NT / 64];
    const int tid = threadIdx.x, k = blockIdx.y;
    const long nn = (long)n * n;
    const long e = (long)blockIdx.x * AS_NT + tid;
    double v = 0.0;
    if (e < nn) {
        const int i = (int)(e % n), c = (int)(e / n);
        const double2 t = T128[(long)k * s128 + i + (long)c * ld128];
        if (O64) T64[(long)k * s64 + i + (long)c * ld64] = to_c64(t);
        v = t.x * t.x + t.y * t.y;
    }
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < AS_NT / 64; ++w) s += red[w];
        frob_part[(long)k * nparts + blockIdx.x] = s;
    }
}

hipError_t assemble_sparse(hipStream_t st, int n, int J, const CsrTerm* terms, const double2* coef, int B,
                           float2* T64, int ld64, long s64, double2* T128, int ld128, long s128,
                           double* frob_part, double* frob, int* bad)
{
    if (!T128) return hipErrorInvalidValue;
    const long nn = (long)n * n;
    const int nparts = (int)((nn + AS_NT - 1) / AS_NT);
    hipError_t e = zero_c128(st, n, n, T128, ld128, s128, B);
    if (e != hipSuccess) return e;
    e = csr_scatter(st, n, J, terms, coef, B, T128, ld128, s128, bad);
    if (e != hipSuccess) return e;
    for (int k0 = 0; k0 < B; k0 += 65535) {
        const int nb = std::min(65535, B - k0);
        if (T64)
            hipLaunchKernelGGL(finish_dense_kernel<true>, dim3(nparts, nb), dim3(AS_NT), 0, st, n,
                               T128 + (long)k0 * s128, ld128, s128, T64 + (long)k0 * s64, ld64, s64,
                               frob_part + (long)k0 * nparts, nparts);
        else
            hipLaunchKernelGGL(finish_dense_kernel<false>, dim3(nparts, nb), dim3(AS_NT), 0, st, n,
                               T128 + (long)k0 * s128, ld128, s128, T64, ld64, s64, frob_part + (long)k0 * nparts,
                               nparts);
    }
    hipLaunchKernelGGL(frob_finish_kernel, dim3(B), dim3(64), 0, st, frob_part, nparts, frob);
    return hipGetLastError();
}

hipError_t assemble_helmholtz(hipStream_t st, int n, const double* pts, double w, const double2* z, int B,
                              float2* T64, int ld64, long s64, double2* T128, int ld128, long s128,
                              double* frob_part, double* frob)
{
    const long nn = (long)n * n;
    const int nparts = (int)((nn + AS_NT - 1) / AS_NT);
    for (int k0 = 0; k0 < B; k0 += AS_PG) {
        if (T64 && T128)
            hipLaunchKernelGGL((assemble_helm_kernel<true, true>), dim3(nparts), dim3(AS_NT), 0, st, n, pts, w, z, B,
                               k0, T64, ld64, s64, T128, ld128, s128, frob_part, nparts);
        else if (T64)
            hipLaunchKernelGGL((assemble_helm_kernel<true, false>), dim3(nparts), dim3(AS_NT), 0, st, n, pts, w, z,
                               B, k0, T64, ld64, s64, T128, ld128, s128, frob_part, nparts);
        else
            hipLaunchKernelGGL((assemble_helm_kernel<false, true>), dim3(nparts), dim3(AS_NT), 0, st, n, pts, w, z,
                               B, k0, T64, ld64, s64, T128, ld128, s128, frob_part, nparts);
    }
    hipLaunchKernelGGL(frob_finish_kernel, dim3(B), dim3(64), 0, st, frob_part, nparts, frob);
    return hipGetLastError();
}

// Taylor coefficient matrix T_p of the Helmholtz kernel about gamma:
// T(z) = sum_p (z - gamma)^p T_p with (T_p)_ij = w (i r)^p e^{i gamma r} / (p! 4 pi r)
// off the diagonal; diagonal p=0: sqrt(w/pi)/2 + i gamma w/(4 pi), p=1: i w/(4 pi), p>=2: 0.
__global__ __launch_bounds__(AS_NT) void helm_taylor_kernel(int n, const double* __restrict__ pts, double w,
                                                             double2 gamma, int p, double inv_pfact,
                                                             double2* __restrict__ Tp, int ld)
{
    const long nn = (long)n * n;
    const long e = (long)blockIdx.x * AS_NT + threadIdx.x;
    if (e >= nn) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const double inv4pi = 0.25 / M_PI;
    double2 t;
    if (i != c) {
        const double dx = pts[3 * i] - pts[3 * c];
        const double dy = pts[3 * i + 1] - pts[3 * c + 1];
        const double dz = pts[3 * i + 2] - pts[3 * c + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double s, co;
        sincos(gamma.x * r, &s, &co);
        const double mag = w * inv4pi / r * exp(-gamma.y * r) * pow(r, (double)p) * inv_pfact;
        // i^p rotates by p quarter turns
        double re = mag * co, im = mag * s;
        switch (p & 3) {
            case 0: t = make_double2(re, im); break;
            case 1: t = make_double2(-im, re); break;
            case 2: t = make_double2(-re, -im); break;
            default: t = make_double2(im, -re); break;
        }
    } else {
        if (p == 0) t = make_double2(0.5 * sqrt(w / M_PI) - gamma.y * w * inv4pi, gamma.x * w * inv4pi);
        else if (p == 1) t = make_double2(0.0, w * inv4pi);
        else t = make_double2(0.0, 0.0);
    }
    Tp[i + (long)c * ld] = t;
}

// Terms p0 .. p0+G-1 at once (term p0+g at Tp + g*sT): the distance, the
// phase and the decay are evaluated once per entry and the magnitude is
// carried from one degree to the next (times r/p).
__global__ __launch_bounds__(AS_NT) void helm_taylor_range_kernel(int n, const double* __restrict__ pts, double w,
                                                                   double2 gamma, int p0, int G, double inv_p0fact,
                                                                   double2* __restrict__ Tp, int ld, long sT)
{
    const long nn = (long)n * n;
    const long e = (long)blockIdx.x * AS_NT + threadIdx.x;
    if (e >= nn) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const double inv4pi = 0.25 / M_PI;
    double2* out = Tp + i + (long)c * ld;
    if (i == c) {
        for (int g = 0; g < G; ++g) {
            const int p = p0 + g;
            double2 t = make_double2(0.0, 0.0);
            if (p == 0) t = make_double2(0.5 * sqrt(w / M_PI) - gamma.y * w * inv4pi, gamma.x * w * inv4pi);
            else if (p == 1) t = make_double2(0.0, w * inv4pi);
            out[g * sT] = t;
        }
        return;
    }
    const double dx = pts[3 * i] - pts[3 * c];
    const double dy = pts[3 * i + 1] - pts[3 * c + 1];
    const double dz = pts[3 * i + 2] - pts[3 * c + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double s, co;
    sincos(gamma.x * r, &s, &co);
    double mag = w * inv4pi / r * exp(-gamma.y * r) * pow(r, (double)p0) * inv_p0fact;
    for (int g = 0; g < G; ++g) {
        const int p = p0 + g;
        if (g > 0) mag *= r / p;
        // i^p rotates by p quarter turns
        const double re = mag * co, im = mag * s;
        double2 t;
        switch (p & 3) {
            case 0: t = make_double2(re, im); break;
            case 1: t = make_double2(-im, re); break;
            case 2: t = make_double2(-re, -im); break;
            default: t = make_double2(im, -re); break;
        }
        out[g * sT] = t;
    }
}

hipError_t helmholtz_taylor_range(hipStream_t st, int n, const double* pts, double w, double gre, double gim, int p0,
                                  int G, double2* Tp, int ld, long sT)
{
    double pf = 1.0;
    for (int q = 2; q <= p0; ++q) pf *= q;
    const long nn = (long)n * n;
    hipLaunchKernelGGL(helm_taylor_range_kernel, dim3((unsigned)((nn + AS_NT - 1) / AS_NT)), dim3(AS_NT), 0, st, n,
                       pts, w, make_double2(gre, gim), p0, G, 1.0 / pf, Tp, ld, sT);
    return hipGetLastError();
}

hipError_t helmholtz_taylor(hipStream_t st, int n, const double* pts, double w, double gre, double gim, int p,
                            double2* Tp, int ld)
{
    double pf = 1.0;
    for (int q = 2; q <= p; ++q) pf *= q;
    const long nn = (long)n * n;
    hipLaunchKernelGGL(helm_taylor_kernel, dim3((unsigned)((nn + AS_NT - 1) / AS_NT)), dim3(AS_NT), 0, st, n, pts, w,
                       make_double2(gre, gim), p, 1.0 / pf, Tp, ld);
    return hipGetLastError();
}

}  // namespace rsrr
