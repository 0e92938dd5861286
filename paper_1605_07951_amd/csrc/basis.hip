// Truncated SVD of the normalised sampling matrix (RSRR Step 3) by block
// one-sided Jacobi in FP64.
//
// The columns of A (m x p) are split into blocks of JB_B columns.  A sweep
// pairs every block with every other once (round-robin tournament, all
// pairs of a round independent).  A round is three launches:
//   1. gram:  for every pair and every slice of JR rows, one workgroup forms
//      the partial Gram matrix [A_I A_J]^H [A_I A_J] (2B x 2B) of its slice;
//   2. solve: one wave per pair sums the slices (fixed order), records
//      max |G_pq| / sqrt(G_pp G_qq) over p != q (the convergence measure of
//      one-sided Jacobi; columns with |a|^2 <= zthr2, rounding level
//      relative to ||A||_F, count as zero and are neither measured nor
//      rotated, so exactly rank-deficient inputs converge), and diagonalises
//      G by cyclic two-sided Jacobi rotations (parallel ordering),
//      accumulating the unitary V;
//   3. apply: for every pair and row slice, [A_I A_J] <- [A_I A_J] V.
// Splitting the rows keeps every CU busy although a round has only p/(2B)
// pairs.  When every pair's measure is below the tolerance the columns of A
// are orthogonal: A = U Sigma with the column norms as singular values.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rsrr {

constexpr int JB_B = 16;          // columns per block
constexpr int JB_W = 2 * JB_B;    // columns per pair
constexpr int JB_NT = 256;
constexpr int JB_RC = 32;         // rows per LDS chunk

// block at tournament position pos in round r (nb even, position 0 fixed)
RSRR_DEV int rr_block(int pos, int r, int nb) { return pos == 0 ? 0 : ((pos - 1 + r) % (nb - 1)) + 1; }

constexpr int JR = 256;           // rows per slice

RSRR_DEV int jac_col(int s, int bI, int bJ, int p)
{
    const int c = (s < JB_B ? bI : bJ) * JB_B + (s % JB_B);
    return c < p ? c : -1;
}

// 1. partial Gram matrix of rows [slice*JR, min(m, slice*JR + JR)) of pair blockIdx.x.
__global__ __launch_bounds__(JB_NT) void jacobi_gram_kernel(const double2* __restrict__ A, int lda, int m, int p,
                                                             int nb, int round, double2* __restrict__ Gp)
{
    __shared__ double2 tile[JB_RC][JB_W + 1];
    const int pr = blockIdx.x, slice = blockIdx.y, tid = threadIdx.x;
    const int bI = rr_block(pr, round, nb), bJ = rr_block(nb - 1 - pr, round, nb);
    const int gp = tid >> 3, gq0 = (tid & 7) * 4;  // each thread: G[gp][gq0..gq0+3]
    const int rlo = slice * JR, rhi = min(m, rlo + JR);
    double2 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = make_double2(0.0, 0.0);
    for (int r0 = rlo; r0 < rhi; r0 += JB_RC) {
        for (int e = tid; e < JB_RC * JB_W; e += JB_NT) {
            const int i = e % JB_RC, s = e / JB_RC;
            const int c = jac_col(s, bI, bJ, p);
            tile[i][s] = (c >= 0 && r0 + i < rhi) ? A[(r0 + i) + (long)c * lda] : make_double2(0.0, 0.0);
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
    double2* G = Gp + ((long)pr * gridDim.y + slice) * (JB_W * JB_W);
#pragma unroll
    for (int u = 0; u < 4; ++u) G[gp * JB_W + gq0 + u] = acc[u];
}

// 2. one workgroup of JS_NT threads per pair: sum the slices, measure, rotate.
// V (JB_W x JB_W, row major, entry [t][s] = V_ts) and skip[pr] go to global memory.
constexpr int JS_NT = 256;
__global__ __launch_bounds__(JS_NT) void jacobi_solve_kernel(const double2* __restrict__ Gp, int slices,
                                                              int inner_sweeps, double tol, double zthr2,
                                                              double2* __restrict__ Vout, int* __restrict__ skip,
                                                              double* __restrict__ offmax)
{
    __shared__ double2 G[JB_W][JB_W + 1];
    __shared__ double2 V[JB_W][JB_W + 1];
    __shared__ double rc[JB_W / 2], rs[JB_W / 2];
    __shared__ double2 re[JB_W / 2];
    __shared__ int rp[JB_W / 2], rq[JB_W / 2], ron[JB_W / 2];
    __shared__ double wmax[JS_NT / 64];
    const int pr = blockIdx.x, tid = threadIdx.x;
    const double2* src = Gp + (long)pr * slices * (JB_W * JB_W);
    {
        // JB_W^2 / JS_NT entries per thread, all loads of a slice in flight together; each
        // entry is summed over the slices in order
        constexpr int PER = JB_W * JB_W / JS_NT;
        double2 g[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) g[t] = make_double2(0.0, 0.0);
        for (int sl = 0; sl < slices; ++sl) {
            const double2* sp = src + (long)sl * (JB_W * JB_W) + tid;
            double2 v[PER];
#pragma unroll
            for (int t = 0; t < PER; ++t) v[t] = sp[JS_NT * t];
#pragma unroll
            for (int t = 0; t < PER; ++t) g[t] = cadd(g[t], v[t]);
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + JS_NT * t;
            G[e / JB_W][e % JB_W] = g[t];
            V[e / JB_W][e % JB_W] = make_double2(e / JB_W == e % JB_W ? 1.0 : 0.0, 0.0);
        }
    }
    __syncthreads();
    double off = 0.0;
    for (int e = tid; e < JB_W * JB_W; e += JS_NT) {
        const int i = e / JB_W, q = e % JB_W;
        if (i == q) continue;
        const double dp = G[i][i].x, dq = G[q][q].x;
        if (dp > zthr2 && dq > zthr2) {
            const double2 g = G[i][q];
            off = fmax(off, sqrt(g.x * g.x + g.y * g.y) / sqrt(dp * dq));
        }
    }
    for (int o = 32; o >= 1; o >>= 1) off = fmax(off, __shfl_xor(off, o));
    if ((tid & 63) == 0) wmax[tid >> 6] = off;
    __syncthreads();
    off = wmax[0];
    for (int w = 1; w < JS_NT / 64; ++w) off = fmax(off, wmax[w]);
    if (tid == 0) {
        offmax[pr] = off;
        skip[pr] = off <= tol ? 1 : 0;
    }
    if (off <= tol) return;  // pair already orthogonal: A stays unchanged (uniform over the workgroup)

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
            for (int task = tid; task < (JB_W / 2) * JB_W * 2; task += JS_NT) {
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
            for (int task = tid; task < (JB_W / 2) * JB_W; task += JS_NT) {
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
    double2* Vo = Vout + (long)pr * (JB_W * JB_W);
    for (int e = tid; e < JB_W * JB_W; e += JS_NT) Vo[e] = V[e / JB_W][e % JB_W];
}

// 3. [A_I A_J] <- [A_I A_J] V on rows [slice*JR, min(m_apply, slice*JR + JR)).
__global__ __launch_bounds__(JB_NT) void jacobi_apply_kernel(double2* __restrict__ A, int lda, int m_apply, int p,
                                                              int nb, int round, const double2* __restrict__ Vin,
                                                              const int* __restrict__ skip)
{
    __shared__ double2 tile[JB_RC][JB_W + 1];
    __shared__ double2 V[JB_W][JB_W + 1];
    const int pr = blockIdx.x, slice = blockIdx.y, tid = threadIdx.x;
    if (skip[pr]) return;
    const int bI = rr_block(pr, round, nb), bJ = rr_block(nb - 1 - pr, round, nb);
    const double2* Vs = Vin + (long)pr * (JB_W * JB_W);
    for (int e = tid; e < JB_W * JB_W; e += JB_NT) V[e / JB_W][e % JB_W] = Vs[e];
    const int rlo = slice * JR, rhi = min(m_apply, rlo + JR);
    for (int r0 = rlo; r0 < rhi; r0 += JB_RC) {
        for (int e = tid; e < JB_RC * JB_W; e += JB_NT) {
            const int i = e % JB_RC, s = e / JB_RC;
            const int c = jac_col(s, bI, bJ, p);
            tile[i][s] = (c >= 0 && r0 + i < rhi) ? A[(r0 + i) + (long)c * lda] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int e = tid; e < JB_RC * JB_W; e += JB_NT) {
            const int i = e % JB_RC, s = e / JB_RC;
            const int c = jac_col(s, bI, bJ, p);
            if (c < 0 || r0 + i >= rhi) continue;
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
// Classical Gram-Schmidt with reorthogonalisation inside one block of bw <= CG_BW
// columns (column c against columns 0..c-1 of the block, twice, then
// normalised).  One workgroup; the block stays in global memory (L2).
// A column whose remaining norm is at most thr * ref[c] (ref = nullptr: 1) is
// numerically dependent on the columns before it and is set to zero: what
// remains of it is rounding noise, and normalising noise would break the
// orthogonality of everything after it.
// ----------------------------------------------------------------------------
constexpr int CG_BW = 8;      // columns per block: the projections on earlier blocks are GEMMs
constexpr int CG_NT = 1024;   // one workgroup per block; many waves keep loads in flight

__global__ __launch_bounds__(CG_NT) void block_cgs2_kernel(double2* __restrict__ Y, int ld, int n, int bw,
                                                            const double* __restrict__ ref, double thr)
{
    constexpr int NW = CG_NT / 64;
    __shared__ double2 red[NW][CG_BW];
    __shared__ double2 coef[CG_BW];
    __shared__ double nred[NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int c = 0; c < bw; ++c) {
        double2* y = Y + (long)c * ld;
        for (int pass = 0; pass < 2 && c > 0; ++pass) {
            double2 acc[CG_BW];
#pragma unroll
            for (int j = 0; j < CG_BW; ++j) acc[j] = make_double2(0.0, 0.0);
            for (int r = tid; r < n; r += CG_NT) {
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
            if (tid < c) {
                double2 t = red[0][tid];
                for (int w = 1; w < NW; ++w) t = cadd(t, red[w][tid]);
                coef[tid] = t;
            }
            __syncthreads();
            for (int r = tid; r < n; r += CG_NT) {
                double2 v = y[r];
                for (int j = 0; j < c; ++j) v = cfms(v, Y[r + (long)j * ld], coef[j]);
                y[r] = v;
            }
            __syncthreads();
        }
        double s2 = 0.0;
        for (int r = tid; r < n; r += CG_NT) { const double2 v = y[r]; s2 += v.x * v.x + v.y * v.y; }
        for (int o = 32; o >= 1; o >>= 1) s2 += __shfl_xor(s2, o);
        if (lane == 0) nred[wave] = s2;
        __syncthreads();
        double tot = 0.0;
        for (int w = 0; w < NW; ++w) tot += nred[w];
        const double nn = sqrt(tot);
        const double inv = nn > thr * (ref ? ref[c] : 1.0) ? 1.0 / nn : 0.0;
        for (int r = tid; r < n; r += CG_NT) { const double2 v = y[r]; y[r] = make_double2(v.x * inv, v.y * inv); }
        __syncthreads();
    }
}

hipError_t gaussian(hipStream_t st, double2* X, int n, int m, int ld, unsigned long long seed)
{
    const long e = (long)n * m;
    hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, X, n, m, ld, seed);
    return hipGetLastError();
}

// Projection of the block Yj = Y[:, j0:j0+bw] off the finished columns
// Y[:, :j0]:  W = Y[:, :j0]^H Yj,  Yj -= Y[:, :j0] W.  Both products are
// skinny (bw columns), so each is split along its long inner dimension into
// slices that run as one batched MFMA GEMM, and the slices are summed in a
// fixed order (deterministic).
constexpr int PK_ROWS = 256;  // inner slice of W = Y^H Yj (rows of Y)
constexpr int PK_COLS = 128;  // inner slice of Yj -= Y W (columns of Y)

__global__ __launch_bounds__(256) void sum_parts_kernel(const double2* __restrict__ part, int S, int rows, int cols,
                                                         double2* __restrict__ out, int ldo, int sub)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const long cnt = (long)rows * cols;
    if (e >= cnt) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int sl = 0; sl < S; ++sl) acc = cadd(acc, part[sl * cnt + e]);
    double2* o = out + (e % rows) + (e / rows) * (long)ldo;
    *o = sub ? make_double2(o->x - acc.x, o->y - acc.y) : acc;
}

static hipError_t sum_parts(hipStream_t st, const double2* part, int S, int rows, int cols, double2* out, int ldo,
                            int sub)
{
    const long cnt = (long)rows * cols;
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, part, S, rows, cols,
                       out, ldo, sub);
    return hipGetLastError();
}

static hipError_t project_out(hipStream_t st, double2* Y, int ld, int n, int j0, int bw, double2* W, double2* part)
{
    double2* Yj = Y + (long)j0 * ld;
    const int S1 = n / PK_ROWS, r1 = n - S1 * PK_ROWS;
    hipError_t e = hipSuccess;
    if (S1 > 0)
        e = zgemm(st, 1, 0, j0, bw, PK_ROWS, 1.0, Y, ld, PK_ROWS, Yj, ld, PK_ROWS, 0.0, part, j0, (long)j0 * bw, S1);
    if (e == hipSuccess && r1 > 0)
        e = zgemm(st, 1, 0, j0, bw, r1, 1.0, Y + S1 * PK_ROWS, ld, 0, Yj + S1 * PK_ROWS, ld, 0, 0.0,
                  part + (long)S1 * j0 * bw, j0, 0, 1);
    if (e == hipSuccess) e = sum_parts(st, part, S1 + (r1 > 0), j0, bw, W, j0, 0);
    const int S2 = j0 / PK_COLS, r2 = j0 - S2 * PK_COLS;
    if (e == hipSuccess && S2 > 0)
        e = zgemm(st, 0, 0, n, bw, PK_COLS, 1.0, Y, ld, (long)PK_COLS * ld, W, j0, PK_COLS, 0.0, part, n,
                  (long)n * bw, S2);
    if (e == hipSuccess && r2 > 0)
        e = zgemm(st, 0, 0, n, bw, r2, 1.0, Y + (long)S2 * PK_COLS * ld, ld, 0, W + S2 * PK_COLS, j0, 0, 0.0,
                  part + (long)S2 * n * bw, n, 0, 1);
    if (e == hipSuccess) e = sum_parts(st, part, S2 + (r2 > 0), n, bw, Yj, ld, 1);
    return e;
}

size_t bcgs2_work_bytes(int n, int m)
{
    const size_t w = (size_t)m * CG_BW;
    const size_t p1 = (size_t)(n / PK_ROWS + 1) * m * CG_BW, p2 = (size_t)(m / PK_COLS + 1) * n * CG_BW;
    return (w + std::max(p1, p2)) * 16 + 256;
}

// Block classical Gram-Schmidt with reorthogonalisation (BCGS2) of Y (n x m,
// ld): each block of CG_BW columns is projected off the finished blocks and
// orthonormalised inside the block, twice.  Columns found dependent
// (remaining norm <= 4 eps sqrt(n) times their original norm) come out as zero
// columns, so Q^H Q is the identity on the nonzero columns.
// work: bcgs2_work_bytes(n, m) bytes; n0: scratch of m doubles.
hipError_t bcgs2(hipStream_t st, double2* Y, int ld, int n, int m, void* work, double* n0)
{
    const double thr = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
    double2* W = (double2*)work;
    double2* part = W + (size_t)m * CG_BW;
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
                e = project_out(st, Y, ld, n, j0, bw, W, part);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(block_cgs2_kernel, dim3(1), dim3(CG_NT), 0, st, Yj, ld, n, bw,
                               pass == 0 ? n0 + j0 : (const double*)nullptr, thr);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            if (j0 == 0) break;
        }
    }
    return hipSuccess;
}

int jacobi_blocks(int p) { int nb = (p + JB_B - 1) / JB_B; return nb + (nb & 1); }

size_t jacobi_work_bytes(int m, int m_apply, int p)
{
    const size_t pairs = (size_t)jacobi_blocks(p) / 2;
    const size_t slices = (size_t)(std::max(m, 1) + JR - 1) / JR;
    (void)m_apply;
    return pairs * (slices + 1) * JB_W * JB_W * 16 + pairs * 4 + 256;
}

hipError_t jacobi_round(hipStream_t st, double2* A, int lda, int m, int m_apply, int p, int round, int inner,
                        double tol, double zthr2, double* offmax, void* work)
{
    const int nb = jacobi_blocks(p), pairs = nb / 2;
    const int gs = (std::max(m, 1) + JR - 1) / JR, as = (m_apply + JR - 1) / JR;
    double2* Gp = (double2*)work;
    double2* V = Gp + (size_t)pairs * gs * JB_W * JB_W;
    int* skip = (int*)(V + (size_t)pairs * JB_W * JB_W);
    hipLaunchKernelGGL(jacobi_gram_kernel, dim3(pairs, gs), dim3(JB_NT), 0, st, A, lda, m, p, nb, round, Gp);
    hipLaunchKernelGGL(jacobi_solve_kernel, dim3(pairs), dim3(JS_NT), 0, st, Gp, gs, inner, tol, zthr2, V, skip, offmax);
    hipLaunchKernelGGL(jacobi_apply_kernel, dim3(pairs, as), dim3(JB_NT), 0, st, A, lda, m_apply, p, nb, round, V,
                       skip);
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
