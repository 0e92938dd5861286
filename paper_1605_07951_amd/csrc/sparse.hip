// Sparse coefficient matrices: T(z) = sum_j f_j(z) A_j with every A_j in
// compressed sparse row storage (the storage of the finite-element models of
// Sec. 4.3 and Sec. 6, whose solvers there are sparse direct and iterative).
//
// Two kernels read the rows:
//  * csr_scatter forms dense T(z_k) for the direct path: one thread owns one
//    row of one point and adds f_j(z_k) a_e into the entries of its row, term
//    by term and entry by entry, so repeated (row, column) pairs are summed
//    and no two threads touch one entry;
//  * csr_apply forms Y = T(z_k) X for the iterative path and the projection:
//    one thread per row and SP_CPT columns walks the row's entries once for
//    all of its columns; each product is summed in FP64 in entry order.
// Both check every row range and column index before reading through it; an
// entry out of bounds is skipped and raises a device flag that the host
// turns into an error.
#include "common.h"
#include "kernels.h"

namespace rsrr {

constexpr int SP_NT = 256;
constexpr int SP_CPT = 4;   // columns of X per thread of csr_apply

// row range [e0, e1) of row i, or false (and the flag) when it lies outside [0, nnz]
RSRR_DEV bool csr_row(const CsrTerm& t, int i, int& e0, int& e1, int* bad)
{
    e0 = t.rp[i];
    e1 = t.rp[i + 1];
    if (e0 < 0 || e1 > t.nnz || e0 > e1) {
        atomicOr(bad, 1);
        return false;
    }
    return true;
}

__global__ __launch_bounds__(SP_NT) void csr_scatter_kernel(int n, int J, const CsrTerm* __restrict__ terms,
                                                            const double2* __restrict__ coef, int B,
                                                            double2* __restrict__ T, int ld, long sT,
                                                            int* __restrict__ bad)
{
    const int i = blockIdx.x * SP_NT + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n) return;
    double2* Tk = T + (long)k * sT + i;
    for (int j = 0; j < J; ++j) {
        const CsrTerm t = terms[j];
        const double2 f = coef[(long)j * B + k];
        int e0, e1;
        if (!csr_row(t, i, e0, e1, bad)) continue;
        for (int e = e0; e < e1; ++e) {
            const int col = t.ci[e];
            if ((unsigned)col >= (unsigned)n) {
                atomicOr(bad, 1);
                continue;
            }
            double2* p = Tk + (long)col * ld;
            *p = cfma(*p, f, t.v[e]);
        }
    }
}

__global__ __launch_bounds__(SP_NT) void csr_apply_kernel(int n, int J, const CsrTerm* __restrict__ terms,
                                                          const double2* __restrict__ coef, int B, int L, int C,
                                                          int cbase, const double2* __restrict__ X, int ldx,
                                                          double2* __restrict__ Y, int ldy, int* __restrict__ bad)
{
    const int i = blockIdx.x * SP_NT + threadIdx.x;
    const int c0 = cbase + blockIdx.y * SP_CPT;
    if (i >= n) return;
    double2 acc[SP_CPT];
#pragma unroll
    for (int q = 0; q < SP_CPT; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int j = 0; j < J; ++j) {
        const CsrTerm t = terms[j];
        int e0, e1;
        if (!csr_row(t, i, e0, e1, bad)) continue;
        double2 s[SP_CPT];
#pragma unroll
        for (int q = 0; q < SP_CPT; ++q) s[q] = make_double2(0.0, 0.0);
        for (int e = e0; e < e1; ++e) {
            const int col = t.ci[e];
            if ((unsigned)col >= (unsigned)n) {
                atomicOr(bad, 1);
                continue;
            }
            const double2 v = t.v[e];
#pragma unroll
            for (int q = 0; q < SP_CPT; ++q)
                if (c0 + q < C) s[q] = cfma(s[q], v, X[col + (long)(c0 + q) * ldx]);
        }
#pragma unroll
        for (int q = 0; q < SP_CPT; ++q)
            if (c0 + q < C) acc[q] = cfma(acc[q], coef[(long)j * B + (c0 + q) / L], s[q]);
    }
#pragma unroll
    for (int q = 0; q < SP_CPT; ++q)
        if (c0 + q < C) Y[i + (long)(c0 + q) * ldy] = acc[q];
}

hipError_t csr_scatter(hipStream_t st, int n, int J, const CsrTerm* terms, const double2* coef, int B, double2* T,
                       int ld, long sT, int* bad)
{
    for (int k0 = 0; k0 < B; k0 += 65535) {
        const int nb = std::min(65535, B - k0);
        hipLaunchKernelGGL(csr_scatter_kernel, dim3((unsigned)((n + SP_NT - 1) / SP_NT), (unsigned)nb), dim3(SP_NT),
                           0, st, n, J, terms, coef + k0, B, T + (long)k0 * sT, ld, sT, bad);
    }
    return hipGetLastError();
}

hipError_t csr_apply(hipStream_t st, int n, int J, const CsrTerm* terms, const double2* coef, int B, int L,
                     const double2* X, int ldx, double2* Y, int ldy, int* bad)
{
    const long C = (long)B * L;
    const long groups = (C + SP_CPT - 1) / SP_CPT;
    for (long g0 = 0; g0 < groups; g0 += 65535) {
        const int ng = (int)std::min<long>(65535, groups - g0);
        hipLaunchKernelGGL(csr_apply_kernel, dim3((unsigned)((n + SP_NT - 1) / SP_NT), (unsigned)ng), dim3(SP_NT), 0,
                           st, n, J, terms, coef, B, L, (int)C, (int)(g0 * SP_CPT), X, ldx, Y, ldy, bad);
    }
    return hipGetLastError();
}

}  // namespace rsrr
