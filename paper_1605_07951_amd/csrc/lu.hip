// Batched dense complex LU with partial pivoting and the matching solves.
//
// Factorisation (right-looking, blocked, RSRR Step 2 needs one LU per
// sampling point): for each outer panel of nb columns
//   1. the panel (all rows below the diagonal) is factored by a recursive
//      split into halves down to a register-resident base kernel;
//   2. the panel's row interchanges are composed into a permutation of at
//      most 2*nb rows (perm_build) and applied to the columns right of the
//      panel together with the unit-lower triangular solve U12 = L11^-1 A12;
//   3. the trailing matrix is updated on the matrix cores, A22 -= L21 U12.
// Columns left of the panel are never interchanged ("lazy" left swaps): the
// solve applies each panel's permutation just before that panel's forward
// elimination step, which reproduces the elimination order exactly.  Inside
// one panel the interchanges are applied to every panel column, so the
// solve can work at panel granularity.
//
// Pivot: largest |Re| + |Im| in the column, lowest row index on ties
// (LAPACK's choice).  info = first column (1-based) whose pivot is exactly
// zero; the factorisation continues past it, as getrf does.
#include <algorithm>
#include <climits>

#include "common.h"
#include "kernels.h"

namespace rsrr {

// ----------------------------------------------------------------------------
// Panel base: rows [c0, n) x columns [c0, c0+jb) of one matrix per workgroup,
// held in registers (thread t owns local rows t, t+NT, ...).
// ----------------------------------------------------------------------------
template <typename C, int NT, int RPT, int JB>
__global__ __launch_bounds__(NT) void panel_base_kernel(
    C* __restrict__ A, long sA, int lda, int n, int c0, int jb,
    int* __restrict__ ipiv, long sP, int* __restrict__ info, const int* __restrict__ active)
{
    typedef real_t<C> R;
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    C* Ab = A + (long)b * sA;
    int* pv = ipiv + (long)b * sP;
    const int m = n - c0;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int NW = NT / 64;

    __shared__ R red_v[NW];
    __shared__ int red_i[NW];
    __shared__ int s_piv;
    __shared__ C prow[JB], crow[JB];

    C v[RPT][JB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int lr = tid + NT * q;
#pragma unroll
        for (int c = 0; c < JB; ++c) {
            C e = czero<C>();
            if (lr < m && c < jb) e = Ab[(c0 + lr) + (long)(c0 + c) * lda];
            v[q][c] = e;
        }
    }

#pragma unroll
    for (int c = 0; c < JB; ++c) {
        if (c >= jb) break;
        // ---- pivot search: per-thread, wavefront shuffle, then LDS ----
        R best = (R)-1;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int lr = tid + NT * q;
            if (lr >= c && lr < m) {
                R a = cabs1(v[q][c]);
                if (a != a) a = (R)INFINITY;  // a NaN wins, so it is reported
                if (a > best) { best = a; bi = lr; }
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            R ob = __shfl_xor(best, off);
            int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { red_v[wave] = best; red_i[wave] = bi; }
        __syncthreads();
        if (wave == 0) {
            R bb = lane < NW ? red_v[lane] : (R)-1;
            int ii = lane < NW ? red_i[lane] : INT_MAX;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                R ob = __shfl_xor(bb, off);
                int oi = __shfl_xor(ii, off);
                if (ob > bb || (ob == bb && oi < ii)) { bb = ob; ii = oi; }
            }
            if (lane == 0) s_piv = (ii == INT_MAX) ? c : ii;
        }
        __syncthreads();
        const int p = s_piv;
        // ---- interchange rows c and p (panel columns only) ----
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int lr = tid + NT * q;
            if (lr == p) {
#pragma unroll
                for (int cc = 0; cc < JB; ++cc) prow[cc] = v[q][cc];
            }
            if (lr == c) {
#pragma unroll
                for (int cc = 0; cc < JB; ++cc) crow[cc] = v[q][cc];
            }
        }
        __syncthreads();
        if (p != c) {
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int lr = tid + NT * q;
                if (lr == c) {
#pragma unroll
                    for (int cc = 0; cc < JB; ++cc) v[q][cc] = prow[cc];
                }
                if (lr == p) {
#pragma unroll
                    for (int cc = 0; cc < JB; ++cc) v[q][cc] = crow[cc];
                }
            }
        }
        const C piv = prow[c];
        const bool zero = is_zero(piv);
        const bool bad = !all_finite(piv);
        if (tid == 0) {
            pv[c0 + c] = c0 + p;
            if (info[b] == 0) {
                if (bad) info[b] = -(c0 + c + 1);
                else if (zero) info[b] = c0 + c + 1;
            }
        }
        const C rp = zero ? czero<C>() : crecip(piv);
        // ---- scale the column and update the rest of the panel ----
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int lr = tid + NT * q;
            if (lr > c && lr < m) {
                if (!zero) v[q][c] = cmul(v[q][c], rp);
                const C l = v[q][c];
#pragma unroll
                for (int cc = c + 1; cc < JB; ++cc)
                    if (cc < jb) v[q][cc] = cfms(v[q][cc], l, prow[cc]);
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int lr = tid + NT * q;
        if (lr < m) {
#pragma unroll
            for (int c = 0; c < JB; ++c)
                if (c < jb) Ab[(c0 + lr) + (long)(c0 + c) * lda] = v[q][c];
        }
    }
}

// ----------------------------------------------------------------------------
// Compose the interchanges ipiv[k1 .. k1+jb) (applied in order) into a
// permutation of the affected rows: after the swaps, row dst[s] holds the
// old row src[s].  Slots 0..jb-1 are rows k1..k1+jb-1; later slots are the
// distinct rows below that were swapped in; unused slots hold (-1, -1).
// One wavefront per matrix; lane 0 replays the swaps, the wave searches.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(64) void perm_build_kernel(const int* __restrict__ ipiv, long sP, int k1, int jb,
                                                          int2* __restrict__ perm, long sPerm,
                                                          const int* __restrict__ active)
{
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const int* pv = ipiv + (long)b * sP;
    int2* pm = perm + (long)b * sPerm;
    const int lane = threadIdx.x;
    __shared__ int rowid[2 * MAX_NB], content[2 * MAX_NB];
    for (int s = lane; s < 2 * jb; s += 64) {
        rowid[s] = (s < jb) ? k1 + s : -1;
        content[s] = (s < jb) ? k1 + s : -1;
    }
    __syncthreads();
    int nout = 0;
    for (int i = 0; i < jb; ++i) {
        const int p = pv[k1 + i];
        int slot;
        if (p < k1 + jb) {
            slot = p - k1;
        } else {
            int found = INT_MAX;
            for (int base = 0; base < nout; base += 64) {
                const int s = base + lane;
                const bool hit = (s < nout) && rowid[jb + s] == p;
                const unsigned long long m = __ballot(hit);
                if (m) { found = base + __ffsll((long long)m) - 1; break; }
            }
            if (found == INT_MAX) {
                slot = jb + nout;
                if (lane == 0) { rowid[slot] = p; content[slot] = p; }
                ++nout;
            } else {
                slot = jb + found;
            }
        }
        __syncthreads();
        if (lane == 0 && slot != i) {
            const int t = content[i];
            content[i] = content[slot];
            content[slot] = t;
        }
        __syncthreads();
    }
    for (int s = lane; s < 2 * jb; s += 64) pm[s] = make_int2(rowid[s], content[s]);
}

// Wave-level ordering of LDS accesses (one wavefront, no workgroup barrier).
RSRR_DEV void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The composition of perm_build_kernel done by the first wavefront of a
// workgroup into pm (2 jb slots, LDS): after the interchanges pv[k1 .. k1+jb),
// row pm[s].x holds the old row pm[s].y.  The caller synchronises the workgroup
// afterwards.
RSRR_DEV void compose_perm_wave(const int* __restrict__ pv, int k1, int jb, int2* pm)
{
    const int lane = threadIdx.x & 63;
    for (int s = lane; s < 2 * jb; s += 64) pm[s] = s < jb ? make_int2(k1 + s, k1 + s) : make_int2(-1, -1);
    wave_sync();
    int nout = 0;
    for (int i = 0; i < jb; ++i) {
        const int p = pv[k1 + i];
        int slot;
        if (p < k1 + jb) {
            slot = p - k1;
        } else {
            int found = INT_MAX;
            for (int base = 0; base < nout; base += 64) {
                const int s = base + lane;
                const bool hit = (s < nout) && pm[jb + s].x == p;
                const unsigned long long m = __ballot(hit);
                if (m) { found = base + __ffsll((long long)m) - 1; break; }
            }
            if (found == INT_MAX) {
                slot = jb + nout;
                if (lane == 0) pm[slot] = make_int2(p, p);
                ++nout;
            } else {
                slot = jb + found;
            }
        }
        wave_sync();
        if (lane == 0 && slot != i) {
            const int t = pm[i].y;
            pm[i].y = pm[slot].y;
            pm[slot].y = t;
        }
        wave_sync();
    }
}

// ----------------------------------------------------------------------------
// Row permutation + triangular solve on a block of columns.
// X: rows indexed like the factored matrix (row r at X[r - xr0]); columns [0, ncols).
// mode 0: permute only.  mode 1: permute, then X[c0:c0+jb] = L11^-1 X[...]
// with L11 the unit-lower diagonal block of LU at (c0, c0).
// mode 2: no permutation, X[c0:c0+jb] = U11^-1 X[...] (non-unit upper).
// mode 4 / 5: X[c0:c0+jb, 0:jb] = L11^-1 / U11^-1 (the solve applied to I).
// ----------------------------------------------------------------------------
constexpr int TS_NT = 256;

// MJB: widest diagonal block staged in LDS; TC: columns per workgroup.
template <typename C, int MJB, int TC>
__global__ __launch_bounds__(TS_NT) void perm_trsm_kernel(
    const C* __restrict__ LU, long sLU, int ldl,
    const int2* __restrict__ perm, long sPerm, const int* __restrict__ ipiv, long sP,
    C* __restrict__ X, long sX, int ldx, int xr0,
    int c0, int jb, int ncols, int mode, const int* __restrict__ active)
{
    typedef real_t<C> R;
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const C* Lb = LU + (long)b * sLU;
    C* Xb = X + (long)b * sX - xr0;
    const int tid = threadIdx.x;
    const int col = tid % TC, grp = tid / TC;
    constexpr int NG = TS_NT / TC;
    const int gcol = blockIdx.x * TC + col;
    const bool colok = gcol < ncols;

    __shared__ C top[MJB][TC + 1];
    __shared__ C Ld[MJB][MJB + 1];
    __shared__ int2 pm[2 * MJB];

    const bool permute = mode == 0 || mode == 1;
    if (permute) {
        if (ipiv) {
            // composed here from the interchanges ipiv[c0 .. c0+jb) (uniform branch)
            if (tid < 64) compose_perm_wave(ipiv + (long)b * sP, c0, jb, pm);
        } else {
            const int2* pb = perm + (long)b * sPerm;
            for (int s = tid; s < 2 * jb; s += TS_NT) pm[s] = pb[s];
        }
    }
    if (mode != 0) {
        // triangle into LDS (column-major read, coalesced along rows)
        for (int e = tid; e < jb * jb; e += TS_NT) {
            const int r = e % jb, c = e / jb;
            Ld[r][c] = Lb[(c0 + r) + (long)(c0 + c) * ldl];
        }
    }
    __syncthreads();

    if (permute) {
        // gather every affected row (reads first, writes after the barrier)
        constexpr int MAXQ = (2 * MJB + NG - 1) / NG;
        C val[MAXQ];
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int s = grp + NG * q;
            C e = czero<C>();
            if (s < 2 * jb && colok) {
                const int src = pm[s].y;
                if (src >= 0) e = Xb[src + (long)gcol * ldx];
            }
            val[q] = e;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int s = grp + NG * q;
            if (s < jb) {
                top[s][col] = val[q];
            } else if (s < 2 * jb && colok) {
                const int dst = pm[s].x;
                if (dst >= 0) Xb[dst + (long)gcol * ldx] = val[q];
            }
        }
    } else if (mode >= 4) {
        for (int s = grp; s < jb; s += NG) top[s][col] = from_real<C>((R)(s == gcol ? 1 : 0));
    } else {
        for (int s = grp; s < jb; s += NG)
            top[s][col] = colok ? Xb[(c0 + s) + (long)gcol * ldx] : czero<C>();
    }
    __syncthreads();

    if (mode == 1 || mode == 4) {
        for (int l = 0; l < jb; ++l) {
            const C xl = top[l][col];
            for (int i = l + 1 + grp; i < jb; i += NG) top[i][col] = cfms(top[i][col], Ld[i][l], xl);
            __syncthreads();
        }
    } else if (mode == 2 || mode == 5) {
        for (int l = jb - 1; l >= 0; --l) {
            if (grp == 0) {
                const C d = Ld[l][l];
                top[l][col] = is_zero(d) ? top[l][col] : cmul(top[l][col], crecip(d));
            }
            __syncthreads();
            const C xl = top[l][col];
            for (int i = grp; i < l; i += NG) top[i][col] = cfms(top[i][col], Ld[i][l], xl);
            __syncthreads();
        }
    }

    if (colok)
        for (int s = grp; s < jb; s += NG) Xb[(c0 + s) + (long)gcol * ldx] = top[s][col];
}

// ----------------------------------------------------------------------------
// Row permutation of a block of columns without a solve (LDS only for the
// permutation).  A workgroup takes PR_TC columns: 2*jb threads gather the
// affected rows of all of them (the loads in flight together), then scatter
// them; rows c0..c0+jb-1 go to T (jb x ncols, ldt) when T is given, otherwise
// back into X.  perm == nullptr: identity (copy the block
// rows to T).
// ----------------------------------------------------------------------------
constexpr int PR_TC = 32;

template <typename C>
__global__ __launch_bounds__(2 * MAX_NB) void perm_rows_kernel(
    const int2* __restrict__ perm, long sPerm, C* __restrict__ X, long sX, int ldx,
    C* __restrict__ T, long sT, int ldt, int c0, int jb, int ncols, const int* __restrict__ active)
{
    typedef real_t<C> R;
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    C* Xb = X + (long)b * sX;
    C* Tb = T ? T + (long)b * sT : nullptr;
    const int s = threadIdx.x;
    int2 e = make_int2(-1, -1);
    if (s < 2 * jb) {
        if (perm) e = perm[(long)b * sPerm + s];
        else if (s < jb) e = make_int2(c0 + s, c0 + s);
    }
    // every column's source row first (all loads in flight), one barrier, then the stores
    const int cbase = blockIdx.x * PR_TC;
    C v[PR_TC];
#pragma unroll
    for (int cc = 0; cc < PR_TC; ++cc) {
        const int gcol = cbase + cc;
        v[cc] = czero<C>();
        if (gcol < ncols && e.y >= 0) v[cc] = Xb[e.y + (long)gcol * ldx];
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < PR_TC; ++cc) {
        const int gcol = cbase + cc;
        if (gcol < ncols) {
            if (s < jb) {
                if (Tb) Tb[s + (long)gcol * ldt] = v[cc];
                else Xb[(c0 + s) + (long)gcol * ldx] = v[cc];
            } else if (e.x >= 0) {
                Xb[e.x + (long)gcol * ldx] = v[cc];
            }
        }
    }
}

// ----------------------------------------------------------------------------
// host drivers
// ----------------------------------------------------------------------------

// Base width of the register-resident panel kernel for m rows.
template <typename R> static int base_width(int m);
template <> int base_width<float>(int m) { return m <= 4096 ? 8 : 4; }
template <> int base_width<double>(int m) { return m <= 2048 ? 8 : (m <= 4096 ? 4 : 2); }

template <typename C, int NT, int RPT, int JB>
static void launch_base(hipStream_t st, C* A, long sA, int lda, int n, int c0, int jb,
                        int* ipiv, long sP, int* info, const int* active, int batch)
{
    hipLaunchKernelGGL((panel_base_kernel<C, NT, RPT, JB>), dim3(batch), dim3(NT), 0, st,
                       A, sA, lda, n, c0, jb, ipiv, sP, info, active);
}

template <typename C>
static void panel_base(hipStream_t st, C* A, long sA, int lda, int n, int c0, int jb,
                       int* ipiv, long sP, int* info, const int* active, int batch)
{
    typedef real_t<C> R;
    const int m = n - c0;
#define PB(NT, RPT, JB) launch_base<C, NT, RPT, JB>(st, A, sA, lda, n, c0, jb, ipiv, sP, info, active, batch)
    if (m <= 256) {
        PB(256, 1, 8);
    } else if (m <= 512) {
        PB(256, 2, 8);
    } else if (m <= 1024) {
        PB(256, 4, 8);
    } else if (m <= 2048) {
        PB(1024, 2, 8);
    } else if (m <= 4096) {
        if (sizeof(R) == 4) PB(1024, 4, 8); else PB(1024, 4, 4);
    } else {
        if (sizeof(R) == 4) PB(1024, 8, 4); else PB(1024, 8, 2);
    }
#undef PB
}

// perm: composed interchanges of rows c0 .. c0+jb (perm_build), or nullptr with ipiv
// given: composed inside the kernel from ipiv[c0 .. c0+jb).
template <typename C>
static void perm_trsm(hipStream_t st, const C* LU, long sLU, int ldl, const int2* perm, long sPerm,
                      C* X, long sX, int ldx, int c0, int jb, int ncols, int mode,
                      const int* active, int batch, int xr0 = 0, const int* ipiv = nullptr, long sP = 0)
{
    typedef real_t<C> R;
    if (ncols <= 0 || jb <= 0) return;
    if (jb <= 64) {
        constexpr int TC = 32;
        dim3 g((ncols + TC - 1) / TC, batch);
        hipLaunchKernelGGL((perm_trsm_kernel<C, 64, TC>), g, dim3(TS_NT), 0, st, LU, sLU, ldl, perm, sPerm, ipiv, sP,
                           X, sX, ldx, xr0, c0, jb, ncols, mode, active);
    } else {
        constexpr int MJB = max_panel<R>();
        constexpr int TC = 16;
        dim3 g((ncols + TC - 1) / TC, batch);
        hipLaunchKernelGGL((perm_trsm_kernel<C, MJB, TC>), g, dim3(TS_NT), 0, st, LU, sLU, ldl, perm, sPerm, ipiv, sP,
                           X, sX, ldx, xr0, c0, jb, ncols, mode, active);
    }
}

template <typename C>
static void perm_rows(hipStream_t st, const int2* perm, long sPerm, C* X, long sX, int ldx,
                      C* T, long sT, int ldt, int c0, int jb, int ncols, const int* active, int batch)
{
    if (ncols <= 0 || jb <= 0) return;
    dim3 g((ncols + PR_TC - 1) / PR_TC, batch);
    hipLaunchKernelGGL(perm_rows_kernel<C>, g, dim3(2 * MAX_NB), 0, st, perm, sPerm, X, sX, ldx, T, sT, ldt, c0, jb,
                       ncols, active);
}

// C = beta C - alpha A B (defaults alpha = beta = 1: C -= A B).  The products
// C = A B with the diagonal-block inverses use alpha = -1, beta = 0.
template <typename C>
static hipError_t gemm_sub(hipStream_t st, int M, int N, int K, const C* A, int lda, long sA,
                           const C* B, int ldb, long sB, C* Cm, int ldc, long sC,
                           int batch, int tag = 0, double alpha = 1.0, double beta = 1.0);
template <>
hipError_t gemm_sub<float2>(hipStream_t st, int M, int N, int K, const float2* A, int lda, long sA, const float2* B,
                           int ldb, long sB, float2* Cm, int ldc, long sC, int batch, int tag, double alpha,
                           double beta)
{
    return cgemm(st, M, N, K, (float)-alpha, A, lda, sA, B, ldb, sB, (float)beta, Cm, ldc, sC, batch, tag);
}
template <>
hipError_t gemm_sub<double2>(hipStream_t st, int M, int N, int K, const double2* A, int lda, long sA,
                            const double2* B, int ldb, long sB, double2* Cm, int ldc, long sC, int batch, int tag,
                            double alpha, double beta)
{
    return zgemm(st, 0, 0, M, N, K, -alpha, A, lda, sA, B, ldb, sB, beta, Cm, ldc, sC, batch, tag);
}

template <>
hipError_t gemm_sub<float>(hipStream_t st, int M, int N, int K, const float* A, int lda, long sA, const float* B,
                           int ldb, long sB, float* Cm, int ldc, long sC, int batch, int tag, double alpha,
                           double beta)
{
    return sgemm(st, M, N, K, (float)-alpha, A, lda, sA, B, ldb, sB, (float)beta, Cm, ldc, sC, batch, tag);
}

// Recursive panel factorisation of columns [c0, c0+w) (rows c0..n-1).
template <typename C>
static void factor_panel(hipStream_t st, C* A, long sA, int lda, int n, int c0, int w,
                         int* ipiv, long sP, int* info, const int* active,
                         int batch)
{
    typedef real_t<C> R;
    const int m = n - c0;
    const int jbase = base_width<R>(m);
    if (w <= jbase) {
        panel_base<C>(st, A, sA, lda, n, c0, w, ipiv, sP, info, active, batch);
        return;
    }
    int w1 = (w / 2) / jbase * jbase;
    if (w1 < jbase) w1 = jbase;
    const int w2 = w - w1;
    factor_panel<C>(st, A, sA, lda, n, c0, w1, ipiv, sP, info, active, batch);
    // right half: interchanges of the left half (composed inside the solve kernel),
    // U12 = L11^-1 A12, A22 -= L21 U12
    C* Ar = A + (long)(c0 + w1) * lda;
    perm_trsm<C>(st, A, sA, lda, nullptr, 0, Ar, sA, lda, c0, w1, w2, 1, active, batch, 0, ipiv, sP);
    (void)gemm_sub<C>(st, m - w1, w2, w1, A + (c0 + w1) + (long)c0 * lda, lda, sA, A + c0 + (long)(c0 + w1) * lda, lda, sA,
                A + (c0 + w1) + (long)(c0 + w1) * lda, lda, sA, batch);
    factor_panel<C>(st, A, sA, lda, n, c0 + w1, w2, ipiv, sP, info, active, batch);
    // left half receives the interchanges of the right half
    perm_trsm<C>(st, A, sA, lda, nullptr, 0, A + (long)c0 * lda, sA, lda, c0 + w1, w2, w1, 0, active, batch, 0, ipiv,
                 sP);
}

// Diagonal-block inverses of panel p (complex-FP32 path): L11^-1 at
// inv + (2p) nb^2, U11^-1 at inv + (2p+1) nb^2, ld nb.
template <typename C>
static C* panel_inv(const LUWork& w, int p, int nb, int which)
{
    return (C*)w.inv + (long)(2 * p + which) * nb * nb;
}

// Inverses of the two triangles of the jb x jb diagonal block at (c0, c0):
// L11^-1 (unit lower, which = 0) at inv + (2p) nb^2 and U11^-1 (upper,
// which = 1) at inv + (2p+1) nb^2, ld nb, the other triangle zero.  By 32 x 32
// blocks: one workgroup per (block column j, triangle, matrix).  Each needed
// diagonal block is inverted by one wave, a lane per column (substitution in
// registers, the triangle read from LDS by broadcast); then block column j of
// the inverse follows by blocked substitution: for L, X_jj = L_jj^-1 and
// X_ij = -L_ii^-1 sum_{j<=k<i} L_ik X_kj; for U, upwards from X_jj = U_jj^-1.
// A zero diagonal entry of U is skipped (as in the solves).  Rows and columns
// past jb are padded with the identity.
constexpr int TI_B = 32, TI_MAXB = 4, TI_NT = 256;

template <typename C>
__global__ __launch_bounds__(TI_NT) void tri_inv_kernel(const C* __restrict__ LU, long sLU, int ldl, int c0, int jb,
                                                         C* __restrict__ inv, long sInv, int nb,
                                                         const int* __restrict__ active)
{
    const int j = blockIdx.x, b = blockIdx.y, which = blockIdx.z;
    if (active && !active[b]) return;
    const int nbk = (jb + TI_B - 1) / TI_B;
    const C* A = LU + (long)b * sLU + c0 + (long)c0 * ldl;   // the diagonal block, A(r, c) = A[r + c*ldl]
    C* X = (C*)inv + (long)b * sInv + (long)(2 * (c0 / nb) + which) * nb * nb;
    // D[i]: inverted diagonal block i until block i of column j of the inverse is
    // known, then that block (its last use as a diagonal inverse is in computing it)
    __shared__ C D[TI_MAXB][TI_B][TI_B + 1];
    __shared__ C Tt[TI_B][TI_B + 1];           // an off-diagonal block of the triangle
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto entry = [&](int r, int c) -> C {        // padded triangle entry (r, c < nbk * 32)
        if (r < jb && c < jb) return A[r + (long)c * ldl];
        return from_real<C>((real_t<C>)(r == c ? 1 : 0));
    };
    // 1. diagonal blocks i = j .. nbk-1 (L) or 0 .. j (U), staged in D[i], then inverted by
    //    wave i (TI_MAXB waves), a lane per column
    for (int e = tid; e < nbk * TI_B * TI_B; e += TI_NT) {
        const int i = e / (TI_B * TI_B), r = e % TI_B, c = (e / TI_B) % TI_B;
        D[i][r][c] = entry(i * TI_B + r, i * TI_B + c);
    }
    __syncthreads();
    C x[TI_B];
    const int i1 = wave, col = lane;
    const bool mine = i1 < nbk && (which == 0 ? i1 >= j : i1 <= j) && col < TI_B;
    if (mine) {
        if (which == 0) {
#pragma unroll
            for (int r = 0; r < TI_B; ++r) {
                C s = from_real<C>((real_t<C>)(r == col ? 1 : 0));
#pragma unroll
                for (int l = 0; l < r; ++l) s = cfms(s, D[i1][r][l], x[l]);
                x[r] = s;
            }
        } else {
#pragma unroll
            for (int r = TI_B - 1; r >= 0; --r) {
                C s = from_real<C>((real_t<C>)(r == col ? 1 : 0));
#pragma unroll
                for (int l = r + 1; l < TI_B; ++l) s = cfms(s, D[i1][r][l], x[l]);
                const C d = D[i1][r][r];
                x[r] = is_zero(d) ? s : cmul(s, crecip(d));
            }
        }
    }
    __syncthreads();
    if (mine) {
#pragma unroll
        for (int r = 0; r < TI_B; ++r) D[i1][r][col] = x[r];
    }
    __syncthreads();
    // 2. block column j: X_jj = D[j] already; X_ij replaces D[i] in order of i
    const int steps = which == 0 ? nbk - 1 - j : j;
    for (int s = 1; s <= steps; ++s) {
        const int i = which == 0 ? j + s : j - s;
        // acc = sum_k T_ik X_kj over k between i and j (exclusive of i), 4 outputs per thread
        C acc[TI_B * TI_B / TI_NT];
#pragma unroll
        for (int q = 0; q < TI_B * TI_B / TI_NT; ++q) acc[q] = czero<C>();
        const int k0 = which == 0 ? j : i + 1, k1 = which == 0 ? i - 1 : j;
        for (int k = k0; k <= k1; ++k) {
            for (int e = tid; e < TI_B * TI_B; e += TI_NT) {
                const int r = e % TI_B, c = e / TI_B;
                Tt[r][c] = entry(i * TI_B + r, k * TI_B + c);
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < TI_B * TI_B / TI_NT; ++q) {
                const int e = tid + TI_NT * q;
                const int r = e % TI_B, c = e / TI_B;
                C a = acc[q];
                for (int l = 0; l < TI_B; ++l) a = cfma(a, Tt[r][l], D[k][l][c]);
                acc[q] = a;
            }
            __syncthreads();
        }
        // X_ij = -D[i] acc (acc staged through Tt), computed in registers, then
        // written over D[i] once every thread has read it
#pragma unroll
        for (int q = 0; q < TI_B * TI_B / TI_NT; ++q) {
            const int e = tid + TI_NT * q;
            Tt[e % TI_B][e / TI_B] = acc[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TI_B * TI_B / TI_NT; ++q) {
            const int e = tid + TI_NT * q;
            const int r = e % TI_B, c = e / TI_B;
            C a = czero<C>();
            for (int l = 0; l < TI_B; ++l) a = cfms(a, D[i][r][l], Tt[l][c]);
            acc[q] = a;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TI_B * TI_B / TI_NT; ++q) {
            const int e = tid + TI_NT * q;
            D[i][e % TI_B][e / TI_B] = acc[q];
        }
        __syncthreads();
    }
    // 3. write block column j (zeros in the other triangle), rows and columns < jb
    for (int e = tid; e < nbk * TI_B * TI_B; e += TI_NT) {
        const int rr = e % (nbk * TI_B), c = e / (nbk * TI_B);
        const int gc = j * TI_B + c, i = rr / TI_B, r = rr % TI_B;
        if (rr >= jb || gc >= jb) continue;
        const bool in = which == 0 ? i >= j : i <= j;
        X[rr + (long)gc * nb] = in ? D[i][r][c] : czero<C>();
    }
}

template <typename C>
static void tri_inv(hipStream_t st, const C* LU, long sLU, int ldl, int c0, int jb, C* inv, long sInv, int nb,
                    const int* active, int batch)
{
    const int nbk = (jb + TI_B - 1) / TI_B;
    hipLaunchKernelGGL(tri_inv_kernel<C>, dim3(nbk, batch, 2), dim3(TI_NT), 0, st, LU, sLU, ldl, c0, jb, inv, sInv,
                       nb, active);
}

// D(r0.., 0..cols) = S(r0.., 0..cols): rows r0..n-1 of a column block, per matrix.
template <typename C>
__global__ __launch_bounds__(256) void copy_rows_kernel(int r0, int n, int cols, const C* __restrict__ S, int lds,
                                                         long sS, C* __restrict__ D, int ldd, long sD,
                                                         const int* __restrict__ active)
{
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const long m = n - r0;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= m * cols) return;
    const int r = r0 + (int)(e % m), c = (int)(e / m);
    D[b * sD + r + (long)c * ldd] = S[b * sS + r + (long)c * lds];
}

template <typename C>
static void copy_rows(hipStream_t st, int r0, int n, int cols, const C* S, int lds, long sS, C* D, int ldd, long sD,
                      const int* active, int batch)
{
    const long cnt = (long)(n - r0) * cols;
    if (cnt <= 0) return;
    hipLaunchKernelGGL(copy_rows_kernel<C>, dim3((unsigned)((cnt + 255) / 256), batch), dim3(256), 0, st, r0, n, cols,
                       S, lds, sS, D, ldd, sD, active);
}

template <typename C>
static hipError_t getrf_impl(hipStream_t st, C* A, long sA, int lda, int n, int nb, const LUWork& w,
                         int batch)
{
    typedef real_t<C> R;
    // diagonal-block inverses and products on the matrix cores: always in FP32, in
    // FP64 when the caller gives the inverse and scratch buffers
    const bool use_inv = sizeof(R) == 4 || (w.inv != nullptr && w.tmp != nullptr);
    if (nb > max_panel<R>()) nb = max_panel<R>();
    if (nb < MIN_NB) nb = MIN_NB;  // perm/inv storage holds perm_panels(n) panels
    UpdateRecorder* rec = w.rec;
    // trailing update C(M x N) -= Aop(M x kdepth) Bop(kdepth x N) on `st`, event-timed
    auto timed_update_on = [&](hipStream_t s, int M, int N, int kdepth, const C* Aop, int ldaop, long sAop,
                               const C* Bop, C* Cop) {
        const bool timed = rec && rec->used < rec->cap;
        if (timed) (void)hipEventRecord(rec->ev[2 * rec->used], s);
        (void)gemm_sub<C>(s, M, N, kdepth, Aop, ldaop, sAop, Bop, lda, sA, Cop, lda, sA, batch, 1);
        if (timed) {
            (void)hipEventRecord(rec->ev[2 * rec->used + 1], s);
            const double fl = (elem_traits<C>::complex ? 8.0 : 2.0) * M * (double)N * kdepth * batch;
            if (rec->lflops) rec->lflops[rec->used] = fl;
            if (rec->lmask) rec->lmask[rec->used] = (s == w.upd && s != nullptr) ? 1 : 0;
            rec->used++;
            rec->flops += fl;
            rec->bytes += (double)sizeof(C) * (2.0 * M * N + (double)M * kdepth + (double)kdepth * N) * batch;
        } else if (rec) {
            rec->dropped++;
        }
    };
    auto timed_update = [&](int M, int N, int kdepth, const C* Aop, int ldaop, long sAop, const C* Bop, C* Cop) {
        timed_update_on(st, M, N, kdepth, Aop, ldaop, sAop, Bop, Cop);
    };
    // panel p on stream s: factor, composed interchanges, diagonal-block inverses (FP32 paths)
    auto panel = [&](hipStream_t s, int c0, int jb, int p) -> int2* {
        factor_panel<C>(s, A, sA, lda, n, c0, jb, w.ipiv, w.sP, w.info, w.active, batch);
        int2* pm = w.perm + (long)p * 2 * MAX_NB;
        hipLaunchKernelGGL(perm_build_kernel, dim3(batch), dim3(64), 0, s, w.ipiv, w.sP, c0, jb, pm, w.sPerm,
                           w.active);
        if (use_inv) tri_inv<C>(s, A, sA, lda, c0, jb, (C*)w.inv, w.sInv, nb, w.active, batch);
        return pm;
    };
    // Two panels may share one trailing update of depth jb0 + jb1 (the deeper
    // product keeps the matrix cores busier per byte of A22 read and written):
    // panel p+1's columns get panel p's update first; the rows of L21_p are
    // copied and interchanged like panel p+1's rows (the stored L21_p keeps
    // panel p's row order, which the solves expect); the U rows of panel p+1
    // receive panel p's update from that copy; then A22 -= [L21_p' L21_{p+1}]
    // [U12_p; U12_{p+1}] in one product.
    const bool pairing = use_inv && w.pair != nullptr;
    int c0 = 0, p = 0;
    // Look-ahead over full pairs (two nb-wide panels with a trailing block after
    // them).  A pair's work splits into a front part that touches only its own
    // 2 nb columns (panel p, its interchanges and U rows on panel p+1's columns,
    // panel p+1's columns update, panel p+1, the interchanged copy of L21_p) and
    // a back part on the trailing columns (the interchanges and U rows of both
    // panels there, the copy of L21_{p+1}).  After the back part of pair i, the
    // trailing update is split: first the 2 nb columns of pair i+1, then, while
    // the rest of the update runs on `st`, pair i+1's front part runs on the side
    // stream (its own pair buffer); the next back part waits for both.
    if (pairing && w.side && w.pair2 && w.ev_a && w.ev_b && n > 2 * nb) {
        C* Wb[2] = {(C*)w.pair, (C*)w.pair2};
        const int ldw = w.ldpair;
        auto front = [&](hipStream_t s, int q0, int pp, C* Wp) {
            const int q1 = q0 + nb;
            C* TL = Wp + (long)ldw * 2 * nb;
            const int2* pm0 = panel(s, q0, nb, pp);
            perm_rows<C>(s, pm0, w.sPerm, A + (long)q1 * lda, sA, lda, (C*)w.tmp, w.sTmp, nb, q0, nb, nb, w.active,
                         batch);
            (void)gemm_sub<C>(s, nb, nb, nb, panel_inv<C>(w, pp, nb, 0), nb, w.sInv, (const C*)w.tmp, nb, w.sTmp,
                              A + q0 + (long)q1 * lda, lda, sA, batch, 0, -1.0, 0.0);
            (void)gemm_sub<C>(s, n - q1, nb, nb, A + q1 + (long)q0 * lda, lda, sA, A + q0 + (long)q1 * lda, lda, sA,
                              A + q1 + (long)q1 * lda, lda, sA, batch);
            const int2* pm1 = panel(s, q1, nb, pp + 1);
            copy_rows<C>(s, q1, n, nb, A + (long)q0 * lda, lda, sA, Wp, ldw, w.sPair, w.active, batch);
            perm_rows<C>(s, pm1, w.sPerm, Wp, w.sPair, ldw, TL, w.sPair, nb, q1, nb, nb, w.active, batch);
        };
        auto back = [&](int q0, int pp, C* Wp) {
            const int q1 = q0 + nb, q2 = q1 + nb, rest = n - q2;
            C* TL = Wp + (long)ldw * 2 * nb;
            const int2* pm0 = w.perm + (long)pp * 2 * MAX_NB;
            const int2* pm1 = w.perm + (long)(pp + 1) * 2 * MAX_NB;
            C* Ar2 = A + (long)q2 * lda;
            perm_rows<C>(st, pm0, w.sPerm, Ar2, sA, lda, (C*)w.tmp, w.sTmp, nb, q0, nb, rest, w.active, batch);
            (void)gemm_sub<C>(st, nb, rest, nb, panel_inv<C>(w, pp, nb, 0), nb, w.sInv, (const C*)w.tmp, nb, w.sTmp,
                              Ar2 + q0, lda, sA, batch, 0, -1.0, 0.0);
            perm_rows<C>(st, pm1, w.sPerm, Ar2, sA, lda, (C*)w.tmp, w.sTmp, nb, q1, nb, rest, w.active, batch);
            (void)gemm_sub<C>(st, nb, rest, nb, TL, nb, w.sPair, Ar2 + q0, lda, sA, (C*)w.tmp, nb, w.sTmp, batch);
            (void)gemm_sub<C>(st, nb, rest, nb, panel_inv<C>(w, pp + 1, nb, 0), nb, w.sInv, (const C*)w.tmp, nb,
                              w.sTmp, Ar2 + q1, lda, sA, batch, 0, -1.0, 0.0);
            copy_rows<C>(st, q2, n, nb, A + (long)q1 * lda, lda, sA, Wp + (long)ldw * nb, ldw, w.sPair, w.active,
                         batch);
        };
        int buf = 0;
        front(st, 0, 0, Wb[0]);
        if (w.first_panel) (void)hipEventRecord(w.first_panel, st);
        for (;;) {
            const int c2 = c0 + 2 * nb, rest = n - c2;
            back(c0, p, Wb[buf]);
            C* Aop = Wb[buf] + c2;
            const C* Bop = A + c0 + (long)c2 * lda;
            C* Cop = A + c2 + (long)c2 * lda;
            if (rest <= 2 * nb) {
                // no full pair follows: one update, the loop below finishes the tail
                timed_update(rest, rest, 2 * nb, Aop, ldw, w.sPair, Bop, Cop);
                c0 = c2;
                p += 2;
                break;
            }
            const int wn = 2 * nb;
            timed_update(rest, wn, 2 * nb, Aop, ldw, w.sPair, Bop, Cop);
            (void)hipEventRecord(w.ev_a, st);
            // the rest of the update is enqueued before the next pair's panels (a chain of
            // small launches), so the host never holds it back behind them
            if (w.upd && w.ev_c) {
                // the first la_cols columns of the update on the CUs the side stream does not
                // use (while the next panels are factored), the rest on every CU
                const int n1 = w.la_cols > 0 ? std::min(rest - wn, w.la_cols) : rest - wn;
                (void)hipStreamWaitEvent(w.upd, w.ev_a, 0);
                timed_update_on(w.upd, rest, n1, 2 * nb, Aop, ldw, w.sPair, Bop + (long)wn * lda,
                                Cop + (long)wn * lda);
                (void)hipEventRecord(w.ev_c, w.upd);
                (void)hipStreamWaitEvent(st, w.ev_c, 0);
                if (n1 < rest - wn)
                    timed_update(rest, rest - wn - n1, 2 * nb, Aop, ldw, w.sPair, Bop + (long)(wn + n1) * lda,
                                 Cop + (long)(wn + n1) * lda);
            } else {
                timed_update(rest, rest - wn, 2 * nb, Aop, ldw, w.sPair, Bop + (long)wn * lda, Cop + (long)wn * lda);
            }
            (void)hipStreamWaitEvent(w.side, w.ev_a, 0);
            front(w.side, c2, p + 2, Wb[buf ^ 1]);
            (void)hipEventRecord(w.ev_b, w.side);
            (void)hipStreamWaitEvent(st, w.ev_b, 0);
            c0 = c2;
            p += 2;
            buf ^= 1;
        }
    }
    while (c0 < n) {
        const int jb0 = (n - c0 < nb) ? n - c0 : nb;
        const int c1 = c0 + jb0;
        const int jb1 = pairing ? ((n - c1 < nb) ? n - c1 : nb) : 0;
        const int2* pm0 = panel(st, c0, jb0, p);
        const int rest0 = n - c1;
        if (rest0 > 0) {
            C* Ar = A + (long)c1 * lda;
            if (use_inv) {
                // interchanges on the right block (top rows to the scratch), then U12 = L11^-1 A12 on MFMA
                perm_rows<C>(st, pm0, w.sPerm, Ar, sA, lda, (C*)w.tmp, w.sTmp, nb, c0, jb0, rest0, w.active, batch);
                (void)gemm_sub<C>(st, jb0, rest0, jb0, panel_inv<C>(w, p, nb, 0), nb, w.sInv, (const C*)w.tmp, nb,
                                  w.sTmp, Ar + c0, lda, sA, batch, 0, -1.0, 0.0);
            } else {
                perm_trsm<C>(st, A, sA, lda, pm0, w.sPerm, Ar, sA, lda, c0, jb0, rest0, 1, w.active, batch);
            }
            if (c0 == 0 && w.first_panel) (void)hipEventRecord(w.first_panel, st);
        }
        const int c2 = c1 + jb1, rest2 = n - c2;
        if (jb1 <= 0 || rest2 <= 0) {
            if (rest0 > 0)
                timed_update(rest0, rest0, jb0, A + c1 + (long)c0 * lda, lda, sA, A + c0 + (long)c1 * lda,
                             A + c1 + (long)c1 * lda);
            c0 = c1;
            p += 1;
            continue;
        }
        C* Wp = (C*)w.pair;
        const int ldw = w.ldpair;
        C* TL = Wp + (long)ldw * 2 * nb;
        // panel p+1's columns receive panel p's update, then panel p+1
        (void)gemm_sub<C>(st, rest0, jb1, jb0, A + c1 + (long)c0 * lda, lda, sA, A + c0 + (long)c1 * lda, lda, sA,
                          A + c1 + (long)c1 * lda, lda, sA, batch);
        const int2* pm1 = panel(st, c1, jb1, p + 1);
        // L21_p rows c1.. into the pair buffer, interchanged like panel p+1 (top rows to TL)
        copy_rows<C>(st, c1, n, jb0, A + (long)c0 * lda, lda, sA, Wp, ldw, w.sPair, w.active, batch);
        perm_rows<C>(st, pm1, w.sPerm, Wp, w.sPair, ldw, TL, w.sPair, nb, c1, jb1, jb0, w.active, batch);
        // panel p+1's interchanges on the trailing columns; its U rows get panel p's update, then L11^-1
        C* Ar2 = A + (long)c2 * lda;
        perm_rows<C>(st, pm1, w.sPerm, Ar2, sA, lda, (C*)w.tmp, w.sTmp, nb, c1, jb1, rest2, w.active, batch);
        (void)gemm_sub<C>(st, jb1, rest2, jb0, TL, nb, w.sPair, A + c0 + (long)c2 * lda, lda, sA, (C*)w.tmp, nb,
                          w.sTmp, batch);
        (void)gemm_sub<C>(st, jb1, rest2, jb1, panel_inv<C>(w, p + 1, nb, 0), nb, w.sInv, (const C*)w.tmp, nb,
                          w.sTmp, Ar2 + c1, lda, sA, batch, 0, -1.0, 0.0);
        // [L21_p' L21_{p+1}] side by side, one update of depth jb0 + jb1
        copy_rows<C>(st, c2, n, jb1, A + (long)c1 * lda, lda, sA, Wp + (long)ldw * jb0, ldw, w.sPair, w.active,
                     batch);
        timed_update(rest2, rest2, jb0 + jb1, Wp + c2, ldw, w.sPair, A + c0 + (long)c2 * lda,
                     A + c2 + (long)c2 * lda);
        c0 = c2;
        p += 2;
    }
    return hipGetLastError();
}

template <typename C>
static hipError_t getrs_impl(hipStream_t st, const C* LU, long sLU, int lda, int n, int nb,
                         const LUWork& w, C* X, long sX, int ldx, int nrhs, int batch)
{
    typedef real_t<C> R;
    const bool use_inv = sizeof(R) == 4 || (w.inv != nullptr && w.tmp != nullptr);
    if (nb > max_panel<R>()) nb = max_panel<R>();
    if (nb < MIN_NB) nb = MIN_NB;
    const int np = (n + nb - 1) / nb;
    for (int p = 0; p < np; ++p) {
        const int c0 = p * nb, jb = (n - c0 < nb) ? n - c0 : nb;
        const int2* pm = w.perm + (long)p * 2 * MAX_NB;
        if (use_inv) {
            perm_rows<C>(st, pm, w.sPerm, X, sX, ldx, (C*)w.tmp, w.sTmp, nb, c0, jb, nrhs, w.active, batch);
            (void)gemm_sub<C>(st, jb, nrhs, jb, panel_inv<C>(w, p, nb, 0), nb, w.sInv, (const C*)w.tmp, nb, w.sTmp,
                              X + c0, ldx, sX, batch, 0, -1.0, 0.0);
        } else {
            perm_trsm<C>(st, LU, sLU, lda, pm, w.sPerm, X, sX, ldx, c0, jb, nrhs, 1, w.active, batch);
        }
        const int rest = n - c0 - jb;
        if (rest > 0)
            (void)gemm_sub<C>(st, rest, nrhs, jb, LU + (c0 + jb) + (long)c0 * lda, lda, sLU, X + c0, ldx, sX,
                              X + c0 + jb, ldx, sX, batch);
    }
    // Backward sweep with U11.  Panels are taken in pairs (p, p-1): after both
    // diagonal solves (the second preceded by the small coupling product with
    // U[p-1, p]) the rows above are updated once with depth jb(p-1) + jb(p);
    // the columns of U above a pair are contiguous, so no copy is needed.
    auto diag_solve = [&](int p) {
        const int c0 = p * nb, jb = (n - c0 < nb) ? n - c0 : nb;
        if (use_inv) {
            perm_rows<C>(st, nullptr, 0, X, sX, ldx, (C*)w.tmp, w.sTmp, nb, c0, jb, nrhs, w.active, batch);
            (void)gemm_sub<C>(st, jb, nrhs, jb, panel_inv<C>(w, p, nb, 1), nb, w.sInv, (const C*)w.tmp, nb, w.sTmp,
                              X + c0, ldx, sX, batch, 0, -1.0, 0.0);
        } else {
            perm_trsm<C>(st, LU, sLU, lda, nullptr, 0, X, sX, ldx, c0, jb, nrhs, 2, w.active, batch);
        }
    };
    for (int p = np - 1; p >= 0;) {
        const int c0 = p * nb, jb = (n - c0 < nb) ? n - c0 : nb;
        diag_solve(p);
        if (p >= 1) {
            const int c1 = c0 - nb;  // panel p-1 is a full panel of width nb
            (void)gemm_sub<C>(st, nb, nrhs, jb, LU + c1 + (long)c0 * lda, lda, sLU, X + c0, ldx, sX, X + c1, ldx, sX,
                              batch);
            diag_solve(p - 1);
            if (c1 > 0)
                (void)gemm_sub<C>(st, c1, nrhs, nb + jb, LU + (long)c1 * lda, lda, sLU, X + c1, ldx, sX, X, ldx, sX,
                                  batch);
            p -= 2;
        } else {
            p -= 1;
        }
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// The whole solve of getrs_impl (complex FP32, diagonal blocks by their
// inverses) for one matrix per workgroup, for right-hand-side blocks that fit
// in LDS: X (n x L, held row by row) is read once, every panel's forward step
// (interchanges, X_p = L11^-1 X_p, rows below -= L21 X_p) and backward step
// (X_p = U11^-1 X_p, rows above -= U12 X_p) runs out of LDS while the factor
// columns stream from memory once, and X is written back at the end.  The
// same operations as the launch-per-step chain, so the same result up to the
// order of the sums; a matrix with active[b] == 0 is left as it is.
//
// Work split: a product row is summed by kg adjacent lanes (lane g of the
// group takes the columns k = g, g + kg, ...) whose partial sums are combined
// by butterfly shuffles in a fixed order.  The diagonal blocks (at most 128
// rows) use kg = 4, so every lane has its share of the block's columns in
// flight at once; the off-diagonal updates use kg = 1, 2 or 4 as the number
// of rows left shrinks, so the late panels of a sweep keep every lane busy.
// The factor and the inverses are read straight from memory (no staging),
// which leaves the LDS to X alone: n = 1024 with 8 right-hand sides takes
// 64 KB, two workgroups per compute unit.
// ----------------------------------------------------------------------------
constexpr int GS_NT = 512;
constexpr int GS_KU = 16;           // factor entries of one row in flight per lane
constexpr int GS_DK = MAX_NB / 4;   // diagonal-block entries per lane (4 lanes per row)

// sum of v over the kg adjacent lanes of a group (kg a power of two <= 4; every
// lane of the wave takes part)
template <int LT>
RSRR_DEV void group_sum(float2 (&v)[LT], int kg)
{
    for (int off = 1; off < kg; off <<= 1) {
#pragma unroll
        for (int l = 0; l < LT; ++l) {
            v[l].x += __shfl_xor(v[l].x, off);
            v[l].y += __shfl_xor(v[l].y, off);
        }
    }
}

// p[off] for a uniform base p and a 32-bit element offset (the byte offset
// fits in 32 bits), so that the load takes the scalar-base form
RSRR_DEV float2 ldg_off(const float2* __restrict__ p, unsigned off)
{
    return *(const float2*)((const char*)p + (size_t)(off * 8u));
}

// rows [r0, r1) of X (in LDS, LT per row) -= A(r0:r1, c0:c0+jb) X(c0:c0+jb),
// KG lanes per row; the factor offsets fit in 32 bits (n <= 2048)
template <int LT, int KG>
RSRR_DEV void getrs_lds_update(const float2* __restrict__ A, int lda, float2* xs, int r0, int r1, int c0, int jb,
                               int tid)
{
    constexpr int ROWS = GS_NT / KG;
    const int i = tid / KG, g = tid % KG;
    for (int rb = r0; rb < r1; rb += ROWS) {
        const int r = rb + i;
        const bool on = r < r1;
        float2 acc[LT];
#pragma unroll
        for (int l = 0; l < LT; ++l) acc[l] = make_float2(0.f, 0.f);
        for (int kb = 0; kb < jb; kb += GS_KU * KG) {
            const unsigned rc = (unsigned)min(r, r1 - 1);
            float2 a[GS_KU];
#pragma unroll
            for (int u = 0; u < GS_KU; ++u) {
                const int k = kb + g + u * KG;
                const float2 v = ldg_off(A, rc + (unsigned)(c0 + min(k, jb - 1)) * (unsigned)lda);
                a[u] = (on && k < jb) ? v : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < GS_KU; ++u) {
                const int k = kb + g + u * KG;
                if (k < jb) {
#pragma unroll
                    for (int l = 0; l < LT; ++l) acc[l] = cfma(acc[l], a[u], xs[(c0 + k) * LT + l]);
                }
            }
        }
        group_sum<LT>(acc, KG);
        if (on) {
#pragma unroll
            for (int l = 0; l < LT; ++l)
                if (l % KG == g) {
                    const float2 x = xs[r * LT + l];
                    xs[r * LT + l] = make_float2(x.x - acc[l].x, x.y - acc[l].y);
                }
        }
    }
}

template <int LT>
__global__ __launch_bounds__(GS_NT) __attribute__((amdgpu_waves_per_eu(4))) void getrs_lds_kernel(const float2* __restrict__ LU, long sLU, int lda, int n,
                                                          int nb, const int2* __restrict__ perm, long sPerm,
                                                          const float2* __restrict__ inv, long sInv,
                                                          float2* __restrict__ X, long sX, int ldx, int L,
                                                          const int* __restrict__ active)
{
    extern __shared__ float2 xs[];   // n x LT, row r at xs + r LT (columns >= L stay zero)
    const int b = blockIdx.x, tid = threadIdx.x;
    if (active && !active[b]) return;
    const float2* A = LU + (long)b * sLU;
    float2* Xb = X + (long)b * sX;
    for (long e = tid; e < (long)n * LT; e += GS_NT) {
        const int r = (int)(e / LT), l = (int)(e % LT);
        xs[e] = l < L ? Xb[r + (long)l * ldx] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int np = (n + nb - 1) / nb;
    // X_p = D X_p for the jb x jb block D (ld nb) and rows c0 .. c0+jb
    auto diag = [=](const float2* D, int c0, int jb) {
        const int i = tid >> 2, g = tid & 3;
        const bool on = i < jb;
        const unsigned ic = (unsigned)min(i, jb - 1);
        float2 acc[LT];
#pragma unroll
        for (int l = 0; l < LT; ++l) acc[l] = make_float2(0.f, 0.f);
#pragma unroll
        for (int h = 0; h < GS_DK; h += GS_DK / 2) {
            float2 d[GS_DK / 2];
#pragma unroll
            for (int m = 0; m < GS_DK / 2; ++m) {
                const int k = g + 4 * (h + m);
                const unsigned kc = (unsigned)min(k, jb - 1);
                const float2 v = ldg_off(D, ic + kc * (unsigned)nb);
                d[m] = (on && k < jb) ? v : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int m = 0; m < GS_DK / 2; ++m) {
                const int k = g + 4 * (h + m);
                if (k < jb) {
#pragma unroll
                    for (int l = 0; l < LT; ++l) acc[l] = cfma(acc[l], d[m], xs[(c0 + k) * LT + l]);
                }
            }
        }
        group_sum<LT>(acc, 4);
        __syncthreads();   // every read of X_p precedes the first write
        if (on) {
#pragma unroll
            for (int l = 0; l < LT; ++l)
                if ((l & 3) == g) xs[(c0 + i) * LT + l] = acc[l];
        }
        __syncthreads();
    };
    // rows [r0, r1) -= F X_p, F the column block of the factor at (r, c0 .. c0+jb)
    auto update = [=](int r0, int r1, int c0, int jb) {
        const int R = r1 - r0;
        if (R <= GS_NT / 4) getrs_lds_update<LT, 4>(A, lda, xs, r0, r1, c0, jb, tid);
        else if (R <= GS_NT / 2) getrs_lds_update<LT, 2>(A, lda, xs, r0, r1, c0, jb, tid);
        else getrs_lds_update<LT, 1>(A, lda, xs, r0, r1, c0, jb, tid);
        __syncthreads();
    };
    for (int p = 0; p < np; ++p) {
        const int c0 = p * nb, jb = min(nb, n - c0);
        // this panel's interchanges: row pm[s].x receives old row pm[s].y
        const int2* pm = perm + (long)b * sPerm + (long)p * 2 * MAX_NB;
        constexpr int PQ = (2 * MAX_NB * LT + GS_NT - 1) / GS_NT;
        float2 v[PQ];
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int e = tid + GS_NT * q;
            v[q] = make_float2(0.f, 0.f);
            if (e < 2 * jb * LT) {
                const int src = pm[e / LT].y;
                if (src >= 0) v[q] = xs[src * LT + e % LT];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int e = tid + GS_NT * q;
            if (e < 2 * jb * LT) {
                const int2 m = pm[e / LT];
                if (m.y >= 0 && m.x >= 0) xs[m.x * LT + e % LT] = v[q];
            }
        }
        __syncthreads();
        diag(inv + (long)b * sInv + (long)(2 * p) * nb * nb, c0, jb);
        update(c0 + jb, n, c0, jb);
    }
    for (int p = np - 1; p >= 0; --p) {
        const int c0 = p * nb, jb = min(nb, n - c0);
        diag(inv + (long)b * sInv + (long)(2 * p + 1) * nb * nb, c0, jb);
        update(0, c0, c0, jb);
    }
    for (long e = tid; e < (long)n * L; e += GS_NT) {
        const int r = (int)(e % n), l = (int)(e / n);
        Xb[r + (long)l * ldx] = xs[r * LT + l];
    }
}

static int gs_width(int nrhs) { return nrhs <= 8 ? 8 : 16; }
static size_t gs_lds(int n, int nrhs) { return (size_t)n * gs_width(nrhs) * 8; }
bool getrs_lds_ok(int n, int nrhs) { return nrhs >= 1 && nrhs <= 16 && gs_lds(n, nrhs) <= (size_t)128 << 10; }

hipError_t getrs_lds_batched(hipStream_t st, const float2* LU, long sLU, int lda, int n, int nb, const LUWork& w,
                             float2* X, long sX, int ldx, int nrhs, int batch)
{
    if (!getrs_lds_ok(n, nrhs)) return hipErrorInvalidValue;
    if (nb > max_panel<float>()) nb = max_panel<float>();
    if (nb < MIN_NB) nb = MIN_NB;
    const size_t lds = gs_lds(n, nrhs);
    if (gs_width(nrhs) == 8)
        hipLaunchKernelGGL(getrs_lds_kernel<8>, dim3(batch), dim3(GS_NT), lds, st, LU, sLU, lda, n, nb, w.perm,
                           w.sPerm, (const float2*)w.inv, w.sInv, X, sX, ldx, nrhs, w.active);
    else
        hipLaunchKernelGGL(getrs_lds_kernel<16>, dim3(batch), dim3(GS_NT), lds, st, LU, sLU, lda, n, nb, w.perm,
                           w.sPerm, (const float2*)w.inv, w.sInv, X, sX, ldx, nrhs, w.active);
    return hipGetLastError();
}

template <>
hipError_t getrf_batched<float>(hipStream_t st, float2* A, long sA, int lda, int n, int nb, const LUWork& w, int batch)
{
    return getrf_impl<float2>(st, A, sA, lda, n, nb, w, batch);
}
template <>
hipError_t getrf_batched<double>(hipStream_t st, double2* A, long sA, int lda, int n, int nb, const LUWork& w,
                                 int batch)
{
    return getrf_impl<double2>(st, A, sA, lda, n, nb, w, batch);
}
template <>
hipError_t getrs_batched<float>(hipStream_t st, const float2* LU, long sLU, int lda, int n, int nb, const LUWork& w,
                                float2* X, long sX, int ldx, int nrhs, int batch)
{
    return getrs_impl<float2>(st, LU, sLU, lda, n, nb, w, X, sX, ldx, nrhs, batch);
}
template <>
hipError_t getrs_batched<double>(hipStream_t st, const double2* LU, long sLU, int lda, int n, int nb,
                                 const LUWork& w, double2* X, long sX, int ldx, int nrhs, int batch)
{
    return getrs_impl<double2>(st, LU, sLU, lda, n, nb, w, X, sX, ldx, nrhs, batch);
}
hipError_t getrf_real_batched(hipStream_t st, float* A, long sA, int lda, int n, int nb, const LUWork& w, int batch)
{
    return getrf_impl<float>(st, A, sA, lda, n, nb, w, batch);
}
hipError_t getrs_real_batched(hipStream_t st, const float* LU, long sLU, int lda, int n, int nb, const LUWork& w,
                              float* X, long sX, int ldx, int nrhs, int batch)
{
    return getrs_impl<float>(st, LU, sLU, lda, n, nb, w, X, sX, ldx, nrhs, batch);
}

}  // namespace rsrr
