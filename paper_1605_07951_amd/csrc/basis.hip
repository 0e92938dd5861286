// Truncated SVD of the normalised sampling matrix (RSRR Step 3) by block
// one-sided Jacobi in FP64.
//
// The columns of A (m x p) are split into blocks of JB_B columns.  A sweep
// pairs every block with every other once (round-robin tournament, all
// pairs of a round independent).  For a pair, one workgroup
//   1. forms the Gram matrix G = [A_I A_J]^H [A_I A_J] (2B x 2B) by
//      streaming the rows through LDS,
//   2. records max |G_pq| / sqrt(G_pp G_qq) over p != q (the convergence
//      measure of one-sided Jacobi); columns with |a|^2 <= zthr2 (rounding
//      level relative to ||A||_F) count as zero and are neither measured
//      nor rotated, so exactly rank-deficient inputs converge,
//   3. diagonalises G with cyclic two-sided Jacobi rotations (parallel
//      ordering) accumulating the unitary V,
//   4. replaces [A_I A_J] by [A_I A_J] V (rows streamed through LDS).
// When every pair's measure is below the tolerance the columns of A are
// orthogonal: A = U Sigma with the column norms as singular values.
#include "common.h"
#include "kernels.h"

namespace rsrr {

constexpr int JB_B = 16;          // columns per block
constexpr int JB_W = 2 * JB_B;    // columns per pair
constexpr int JB_NT = 256;
constexpr int JB_RC = 32;         // rows per LDS chunk

// block at tournament position pos in round r (nb even, position 0 fixed)
RSRR_DEV int rr_block(int pos, int r, int nb) { return pos == 0 ? 0 : ((pos - 1 + r) % (nb - 1)) + 1; }

// m: rows that form the Gram matrix; m_apply >= m: rows the rotations are applied
// to (rows m..m_apply-1 accumulate the right singular vectors when they start as I).
__global__ __launch_bounds__(JB_NT) void jacobi_pair_kernel(double2* __restrict__ A, int lda, int m, int m_apply,
                                                             int p, int nb, int round, int inner_sweeps, double tol,
                                                             double zthr2, double* __restrict__ offmax)
{
    __shared__ double2 tile[JB_RC][JB_W + 1];
    __shared__ double2 G[JB_W][JB_W + 1];
    __shared__ double2 V[JB_W][JB_W + 1];
    __shared__ double rc[JB_W / 2], rs[JB_W / 2];
    __shared__ double2 re[JB_W / 2];
    __shared__ int rp[JB_W / 2], rq[JB_W / 2], ron[JB_W / 2];
    __shared__ double red[JB_NT / 64];

    const int pr = blockIdx.x;  // pair index
    const int bI = rr_block(pr, round, nb), bJ = rr_block(nb - 1 - pr, round, nb);
    const int tid = threadIdx.x;
    // column of pair slot s (-1 = padding)
    auto colof = [&](int s) -> int {
        const int blk = s < JB_B ? bI : bJ;
        const int c = blk * JB_B + (s % JB_B);
        return c < p ? c : -1;
    };

    // ---- 1. Gram matrix ----
    const int gp = tid >> 3, gq0 = (tid & 7) * 4;  // each thread: G[gp][gq0..gq0+3]
    double2 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = make_double2(0.0, 0.0);
    for (int r0 = 0; r0 < m; r0 += JB_RC) {
        for (int e = tid; e < JB_RC * JB_W; e += JB_NT) {
            const int i = e % JB_RC, s = e / JB_RC;
            const int c = colof(s);
            tile[i][s] = (c >= 0 && r0 + i < m) ? A[(r0 + i) + (long)c * lda] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 4
        for (int i = 0; i < JB_RC; ++i) {
            const double2 a = tile[i][gp];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = cfma_cj(acc[u], a, tile[i][gq0 + u]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) G[gp][gq0 + u] = acc[u];
    __syncthreads();

    // ---- 2. convergence measure (before rotating) ----
    double off = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = gq0 + u;
        if (q != gp) {
            const double dp = G[gp][gp].x, dq = G[q][q].x;
            if (dp > zthr2 && dq > zthr2) {
                const double2 g = G[gp][q];
                off = fmax(off, sqrt(g.x * g.x + g.y * g.y) / sqrt(dp * dq));
            }
        }
    }
    for (int o = 32; o >= 1; o >>= 1) off = fmax(off, __shfl_xor(off, o));
    if ((tid & 63) == 0) red[tid >> 6] = off;
    for (int e = tid; e < JB_W * JB_W; e += JB_NT) {
        const int i = e / JB_W, j = e % JB_W;
        V[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    if (tid == 0) {
        double o = 0.0;
        for (int w = 0; w < JB_NT / 64; ++w) o = fmax(o, red[w]);
        offmax[pr] = o;
        red[0] = o;
    }
    __syncthreads();
    if (red[0] <= tol) return;  // pair already orthogonal: leave A unchanged

    // ---- 3. cyclic Jacobi on G (parallel ordering over JB_W indices) ----
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        for (int st = 0; st < JB_W - 1; ++st) {
            if (tid < JB_W / 2) {
                const int ip = rr_block(tid, st, JB_W), iq = rr_block(JB_W - 1 - tid, st, JB_W);
                const int a_ = ip < iq ? ip : iq, b_ = ip < iq ? iq : ip;
                const double2 g = G[a_][b_];
                const double h = sqrt(g.x * g.x + g.y * g.y);
                const double dA = G[a_][a_].x, dB = G[b_][b_].x;
                int on = 0;
                double c = 1.0, s = 0.0;
                double2 e = make_double2(1.0, 0.0);
                if (dA > zthr2 && dB > zthr2 && h > 0.25 * tol * sqrt(dA * dB)) {
                    const double zeta = (dB - dA) / (2.0 * h);
                    const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    e = make_double2(g.x / h, g.y / h);
                    on = 1;
                }
                rp[tid] = a_; rq[tid] = b_; rc[tid] = c; rs[tid] = s; re[tid] = e; ron[tid] = on;
            }
            __syncthreads();
            // columns: [x_p, x_q] <- [c x_p - s conj(e) x_q, s e x_p + c x_q] for G and V
            for (int task = tid; task < (JB_W / 2) * JB_W * 2; task += JB_NT) {
                const int which = task / ((JB_W / 2) * JB_W);  // 0: G, 1: V
                const int rem = task % ((JB_W / 2) * JB_W);
                const int k = rem / JB_W, row = rem % JB_W;
                if (!ron[k]) continue;
                const int a_ = rp[k], b_ = rq[k];
                const double c = rc[k], s = rs[k];
                const double2 e = re[k];
                double2(*M)[JB_W + 1] = which ? V : G;
                const double2 xp = M[row][a_], xq = M[row][b_];
                const double2 ecq = cmul(cconj(e), xq), exp_ = cmul(e, xp);
                M[row][a_] = make_double2(c * xp.x - s * ecq.x, c * xp.y - s * ecq.y);
                M[row][b_] = make_double2(s * exp_.x + c * xq.x, s * exp_.y + c * xq.y);
            }
            __syncthreads();
            // rows of G: row_p <- c row_p - s e row_q ; row_q <- s conj(e) row_p + c row_q
            for (int task = tid; task < (JB_W / 2) * JB_W; task += JB_NT) {
                const int k = task / JB_W, col = task % JB_W;
                if (!ron[k]) continue;
                const int a_ = rp[k], b_ = rq[k];
                const double c = rc[k], s = rs[k];
                const double2 e = re[k];
                const double2 xp = G[a_][col], xq = G[b_][col];
                const double2 eq = cmul(e, xq), cep = cmul(cconj(e), xp);
                G[a_][col] = make_double2(c * xp.x - s * eq.x, c * xp.y - s * eq.y);
                G[b_][col] = make_double2(s * cep.x + c * xq.x, s * cep.y + c * xq.y);
            }
            __syncthreads();
            if (tid < JB_W / 2 && ron[tid]) {
                const int a_ = rp[tid], b_ = rq[tid];
                G[a_][b_] = make_double2(0.0, 0.0);
                G[b_][a_] = make_double2(0.0, 0.0);
                G[a_][a_].y = 0.0;
                G[b_][b_].y = 0.0;
            }
            __syncthreads();
        }
    }

    // ---- 4. [A_I A_J] <- [A_I A_J] V ----
    for (int r0 = 0; r0 < m_apply; r0 += JB_RC) {
        for (int e = tid; e < JB_RC * JB_W; e += JB_NT) {
            const int i = e % JB_RC, s = e / JB_RC;
            const int c = colof(s);
            tile[i][s] = (c >= 0 && r0 + i < m_apply) ? A[(r0 + i) + (long)c * lda] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int e = tid; e < JB_RC * JB_W; e += JB_NT) {
            const int i = e % JB_RC, s = e / JB_RC;
            const int c = colof(s);
            if (c < 0 || r0 + i >= m_apply) continue;
            double2 v = make_double2(0.0, 0.0);
#pragma unroll 8
            for (int t = 0; t < JB_W; ++t) v = cfma(v, tile[i][t], V[t][s]);
            A[(r0 + i) + (long)c * lda] = v;
        }
        __syncthreads();
    }
}

// Q(:, i) = A(:, order[i]) * inv[i] for i < k.
__global__ __launch_bounds__(256) void gather_scale_kernel(const double2* __restrict__ A, int lda, int m,
                                                            const int* __restrict__ order,
                                                            const double* __restrict__ inv, double2* __restrict__ Q,
                                                            int ldq, int k)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)m * k) return;
    const int i = (int)(e % m), c = (int)(e / m);
    const double2 a = A[i + (long)order[c] * lda];
    const double s = inv[c];
    Q[i + (long)c * ldq] = make_double2(a.x * s, a.y * s);
}

// ----------------------------------------------------------------------------
// Seeded complex Gaussian matrix (n x m, ld n): entry e uses the counter-based
// generator splitmix64(seed, e) -> two uniforms -> Box-Muller.  Deterministic.
// ----------------------------------------------------------------------------
RSRR_DEV unsigned long long splitmix64(unsigned long long x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ __launch_bounds__(256) void gaussian_kernel(double2* __restrict__ X, int n, int m, int ld,
                                                        unsigned long long seed)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)n * m) return;
    const int i = (int)(e % n), j = (int)(e / n);
    const unsigned long long h1 = splitmix64(seed ^ splitmix64((unsigned long long)e * 2ull));
    const unsigned long long h2 = splitmix64(seed ^ splitmix64((unsigned long long)e * 2ull + 1ull));
    const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);         // [0, 1)
    const double r = sqrt(-2.0 * log(u1)) * 0.70710678118654752;
    double sn, cs;
    sincos(6.283185307179586 * u2, &sn, &cs);
    X[i + (long)j * ld] = make_double2(r * cs, r * sn);
}

// ----------------------------------------------------------------------------
// Classical Gram-Schmidt with reorthogonalisation inside one block of bw <= 32
// columns (column c against columns 0..c-1 of the block, twice, then
// normalised).  One workgroup; the block stays in global memory (L2).
// A column whose remaining norm is at most thr * ref[c] (ref = nullptr: 1) is
// numerically dependent on the columns before it and is set to zero: what
// remains of it is rounding noise, and normalising noise would break the
// orthogonality of everything after it.
// ----------------------------------------------------------------------------
constexpr int CG_BW = 32;

__global__ __launch_bounds__(256) void block_cgs2_kernel(double2* __restrict__ Y, int ld, int n, int bw,
                                                          const double* __restrict__ ref, double thr)
{
    __shared__ double2 red[4][CG_BW];
    __shared__ double2 coef[CG_BW];
    __shared__ double nred[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int c = 0; c < bw; ++c) {
        double2* y = Y + (long)c * ld;
        for (int pass = 0; pass < 2 && c > 0; ++pass) {
            double2 acc[CG_BW];
#pragma unroll
            for (int j = 0; j < CG_BW; ++j) acc[j] = make_double2(0.0, 0.0);
            for (int r = tid; r < n; r += 256) {
                const double2 v = y[r];
#pragma unroll
                for (int j = 0; j < CG_BW; ++j)
                    if (j < c) acc[j] = cfma_cj(acc[j], Y[r + (long)j * ld], v);
            }
#pragma unroll
            for (int j = 0; j < CG_BW; ++j) {
                if (j >= c) break;
                double2 a = acc[j];
                for (int o = 32; o >= 1; o >>= 1) { a.x += __shfl_xor(a.x, o); a.y += __shfl_xor(a.y, o); }
                if (lane == 0) red[wave][j] = a;
            }
            __syncthreads();
            if (tid < c) coef[tid] = cadd(cadd(red[0][tid], red[1][tid]), cadd(red[2][tid], red[3][tid]));
            __syncthreads();
            for (int r = tid; r < n; r += 256) {
                double2 v = y[r];
                for (int j = 0; j < c; ++j) v = cfms(v, Y[r + (long)j * ld], coef[j]);
                y[r] = v;
            }
            __syncthreads();
        }
        double s2 = 0.0;
        for (int r = tid; r < n; r += 256) { const double2 v = y[r]; s2 += v.x * v.x + v.y * v.y; }
        for (int o = 32; o >= 1; o >>= 1) s2 += __shfl_xor(s2, o);
        if (lane == 0) nred[wave] = s2;
        __syncthreads();
        const double nn = sqrt(nred[0] + nred[1] + nred[2] + nred[3]);
        const double inv = nn > thr * (ref ? ref[c] : 1.0) ? 1.0 / nn : 0.0;
        for (int r = tid; r < n; r += 256) { const double2 v = y[r]; y[r] = make_double2(v.x * inv, v.y * inv); }
        __syncthreads();
    }
}

hipError_t gaussian(hipStream_t st, double2* X, int n, int m, int ld, unsigned long long seed)
{
    const long e = (long)n * m;
    hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, X, n, m, ld, seed);
    return hipGetLastError();
}

// Block classical Gram-Schmidt with reorthogonalisation (BCGS2) of Y (n x m,
// ld): each block of 32 columns is projected against the finished blocks (FP64
// MFMA GEMMs) and orthonormalised inside the block, twice.  Columns found
// dependent (remaining norm <= 4 eps sqrt(n) times their original norm) come
// out as zero columns, so Q^H Q is the identity on the nonzero columns.
// W: scratch of m*32 complex; n0: scratch of m doubles.
hipError_t bcgs2(hipStream_t st, double2* Y, int ld, int n, int m, double2* W, double* n0)
{
    const double thr = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
    hipError_t e = colnorms(st, n, m, Y, ld, 0, n0, 1);
    if (e != hipSuccess) return e;
    for (int j0 = 0; j0 < m; j0 += CG_BW) {
        const int bw = (m - j0 < CG_BW) ? m - j0 : CG_BW;
        double2* Yj = Y + (long)j0 * ld;
        // two full passes (project on the finished blocks, then orthonormalise inside the
        // block): the second pass sees a block that is already well conditioned, which is
        // what makes the reorthogonalisation effective when S is nearly rank deficient
        for (int pass = 0; pass < 2; ++pass) {
            if (j0 > 0) {
                e = zgemm(st, 1, 0, j0, bw, n, 1.0, Y, ld, 0, Yj, ld, 0, 0.0, W, j0, 0, 1);
                if (e != hipSuccess) return e;
                e = zgemm(st, 0, 0, n, bw, j0, -1.0, Y, ld, 0, W, j0, 0, 1.0, Yj, ld, 0, 1);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(block_cgs2_kernel, dim3(1), dim3(256), 0, st, Yj, ld, n, bw,
                               pass == 0 ? n0 + j0 : (const double*)nullptr, thr);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            if (j0 == 0) break;
        }
    }
    return hipSuccess;
}

int jacobi_blocks(int p) { int nb = (p + JB_B - 1) / JB_B; return nb + (nb & 1); }

hipError_t jacobi_round(hipStream_t st, double2* A, int lda, int m, int m_apply, int p, int round, int inner,
                        double tol, double zthr2, double* offmax)
{
    const int nb = jacobi_blocks(p);
    hipLaunchKernelGGL(jacobi_pair_kernel, dim3(nb / 2), dim3(JB_NT), 0, st, A, lda, m, m_apply, p, nb, round, inner,
                       tol, zthr2, offmax);
    return hipGetLastError();
}

hipError_t gather_scale(hipStream_t st, const double2* A, int lda, int m, const int* order, const double* inv,
                        double2* Q, int ldq, int k)
{
    if (k <= 0) return hipSuccess;
    const long e = (long)m * k;
    hipLaunchKernelGGL(gather_scale_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, A, lda, m, order, inv,
                       Q, ldq, k);
    return hipGetLastError();
}

}  // namespace rsrr
