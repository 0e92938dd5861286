// Truncated SVD of the normalised sampling matrix (RSRR Step 3) by block
// one-sided Jacobi in FP64.
//
// The columns of A (m x p) are split into blocks of JB_B columns.  A sweep
// pairs every block with every other once (round-robin tournament, all
// pairs of a round independent).  A round is two launches:
//   1. gram:  for every pair and every slice of JRG rows, one workgroup forms
//      the partial Gram matrix [A_I A_J]^H [A_I A_J] (2B x 2B) of its slice;
//   2. rotate: for every pair and every slice of JR rows of the m_apply rows
//      that are rotated, one workgroup sums the pair's Gram slices (fixed
//      order), measures max |G_pq| / sqrt(G_pp G_qq) over p != q (the
//      convergence measure of one-sided Jacobi; columns with |a|^2 <= zthr2,
//      rounding level relative to ||A||_F, count as zero and are neither
//      measured nor rotated, so exactly rank-deficient inputs converge),
//      diagonalises G by cyclic two-sided Jacobi rotations (parallel
//      ordering) accumulating the unitary V, and applies
//      [A_I A_J] <- [A_I A_J] V to its rows.  Every workgroup of a pair does
//      the same small diagonalisation on the same data, so they agree
//      bitwise; slice 0 records the measure.
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

// block at tournament position pos in round r (nb even, position 0 fixed)
RSRR_DEV int rr_block(int pos, int r, int nb) { return pos == 0 ? 0 : ((pos - 1 + r) % (nb - 1)) + 1; }

constexpr int JR = 256;           // rows per slice of the rotation
constexpr int JRG = 128;          // rows per slice of the Gram matrices

RSRR_DEV int jac_col(int s, int bI, int bJ, int p)
{
    const int c = (s < JB_B ? bI : bJ) * JB_B + (s % JB_B);
    return c < p ? c : -1;
}

// 1. partial Gram matrix of rows [slice*JRG, min(m, slice*JRG + JRG)) of pair blockIdx.x.
// Chunks of JG_RC rows pass through LDS; the next chunk is fetched into
// registers while the current one is multiplied.
constexpr int JG_RC = 64;
constexpr int JG_PER = JG_RC * JB_W / JB_NT;  // entries of a chunk per thread

__global__ __launch_bounds__(JB_NT) void jacobi_gram_kernel(const double2* __restrict__ A, int lda, int m, int p,
                                                             int nb, int round, double2* __restrict__ Gp)
{
    __shared__ double2 tile[JG_RC][JB_W + 1];
    const int pr = blockIdx.x, slice = blockIdx.y, tid = threadIdx.x;
    const int bI = rr_block(pr, round, nb), bJ = rr_block(nb - 1 - pr, round, nb);
    const int gp = tid >> 3, gq0 = (tid & 7) * 4;  // each thread: G[gp][gq0..gq0+3]
    const int rlo = slice * JRG, rhi = min(m, rlo + JRG);
    double2 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = make_double2(0.0, 0.0);
    double2 nx[JG_PER];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int u = 0; u < JG_PER; ++u) {
            const int e = tid + JB_NT * u, i = e % JG_RC, sc = e / JG_RC;
            const int c = jac_col(sc, bI, bJ, p);
            nx[u] = (c >= 0 && r0 + i < rhi) ? A[(r0 + i) + (long)c * lda] : make_double2(0.0, 0.0);
        }
    };
    fetch(rlo);
    for (int r0 = rlo; r0 < rhi; r0 += JG_RC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < JG_PER; ++u) {
            const int e = tid + JB_NT * u;
            tile[e % JG_RC][e / JG_RC] = nx[u];
        }
        __syncthreads();
        if (r0 + JG_RC < rhi) fetch(r0 + JG_RC);
#pragma unroll 4
        for (int i = 0; i < JG_RC; ++i) {
            const double2 a = tile[i][gp];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = cfma_cj(acc[u], a, tile[i][gq0 + u]);
        }
    }
    double2* G = Gp + ((long)pr * gridDim.y + slice) * (JB_W * JB_W);
#pragma unroll
    for (int u = 0; u < 4; ++u) G[gp * JB_W + gq0 + u] = acc[u];
}

// 2. sum the Gram slices of pair blockIdx.x, measure, diagonalise, and rotate the
// rows of slice blockIdx.y.  One step of the inner sweep applies JB_W / 2
// disjoint rotations (a_k, b_k) from both sides at once; thread (pi, pj) owns
// the 2 x 2 entries of G and of V at rows {a_pi, b_pi} x columns {a_pj, b_pj},
// so the update is done in place and a step needs two barriers.
__global__ __launch_bounds__(JB_NT) void jacobi_rotate_kernel(double2* __restrict__ A, int lda, int m_apply, int p,
                                                               int nb, int round, const double2* __restrict__ Gp,
                                                               int slices, int inner_sweeps, double tol, double zthr2,
                                                               double* __restrict__ offmax)
{
    static_assert(JB_NT == (JB_W / 2) * (JB_W / 2), "one thread per 2 x 2 block of a step");
    __shared__ double2 G[JB_W][JB_W + 1];
    __shared__ double2 V[JB_W][JB_W + 1];
    __shared__ double2 tile[JG_RC][JB_W + 1];
    __shared__ int pa[JB_W / 2], pb[JB_W / 2], pon[JB_W / 2];
    __shared__ double pc[JB_W / 2], ps[JB_W / 2];
    __shared__ double2 pe[JB_W / 2];
    __shared__ double wmax[JB_NT / 64];
    const int pr = blockIdx.x, slice = blockIdx.y, tid = threadIdx.x;
    const double2* src = Gp + (long)pr * slices * (JB_W * JB_W);
    constexpr int PER = JB_W * JB_W / JB_NT;
    {
        // JS_SL slices' loads in flight at once; each entry is summed in slice order
        constexpr int JS_SL = 8;
        double2 g[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) g[t] = make_double2(0.0, 0.0);
        for (int sl0 = 0; sl0 < slices; sl0 += JS_SL) {
            double2 v[JS_SL][PER];
#pragma unroll
            for (int q = 0; q < JS_SL; ++q) {
                const double2* sp = src + (long)(sl0 + q) * (JB_W * JB_W) + tid;
#pragma unroll
                for (int t = 0; t < PER; ++t) v[q][t] = sl0 + q < slices ? sp[JB_NT * t] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int q = 0; q < JS_SL; ++q) {
                if (sl0 + q >= slices) break;
#pragma unroll
                for (int t = 0; t < PER; ++t) g[t] = cadd(g[t], v[q][t]);
            }
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + JB_NT * t;
            G[e / JB_W][e % JB_W] = g[t];
            V[e / JB_W][e % JB_W] = make_double2(e / JB_W == e % JB_W ? 1.0 : 0.0, 0.0);
        }
    }
    __syncthreads();
    double off = 0.0;
    for (int e = tid; e < JB_W * JB_W; e += JB_NT) {
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
    for (int w = 1; w < JB_NT / 64; ++w) off = fmax(off, wmax[w]);
    if (slice == 0 && tid == 0) offmax[pr] = off;
    if (off <= tol) return;  // pair already orthogonal: A stays unchanged (uniform over the workgroup)

    const int qi = tid / (JB_W / 2), qj = tid % (JB_W / 2);
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
                pa[tid] = a_; pb[tid] = b_; pon[tid] = on; pc[tid] = c; ps[tid] = s; pe[tid] = e;
            }
            __syncthreads();
            // columns a, b (pair qj): x_a <- c x_a - s conj(e) x_b, x_b <- s e x_a + c x_b;
            // rows a, b (pair qi):    r_a <- c r_a - s e r_b,       r_b <- s conj(e) r_a + c r_b
            const int ra = pa[qi], rb = pb[qi], ca = pa[qj], cb = pb[qj];
            const bool oi = pon[qi] != 0, oj = pon[qj] != 0;
            if (oi || oj) {
                double2 g00 = G[ra][ca], g01 = G[ra][cb], g10 = G[rb][ca], g11 = G[rb][cb];
                double2 v00 = V[ra][ca], v01 = V[ra][cb], v10 = V[rb][ca], v11 = V[rb][cb];
                if (oj) {
                    const double c = pc[qj], s = ps[qj];
                    const double2 e = pe[qj], ce = cconj(e);
                    auto colop = [&](double2& xa, double2& xb) {
                        const double2 ecq = cmul(ce, xb), exp_ = cmul(e, xa);
                        const double2 na = make_double2(c * xa.x - s * ecq.x, c * xa.y - s * ecq.y);
                        xb = make_double2(s * exp_.x + c * xb.x, s * exp_.y + c * xb.y);
                        xa = na;
                    };
                    colop(g00, g01);
                    colop(g10, g11);
                    colop(v00, v01);
                    colop(v10, v11);
                    V[ra][ca] = v00; V[ra][cb] = v01; V[rb][ca] = v10; V[rb][cb] = v11;
                }
                if (oi) {
                    const double c = pc[qi], s = ps[qi];
                    const double2 e = pe[qi], ce = cconj(e);
                    auto rowop = [&](double2& xa, double2& xb) {
                        const double2 eq = cmul(e, xb), cep = cmul(ce, xa);
                        const double2 na = make_double2(c * xa.x - s * eq.x, c * xa.y - s * eq.y);
                        xb = make_double2(s * cep.x + c * xb.x, s * cep.y + c * xb.y);
                        xa = na;
                    };
                    rowop(g00, g10);
                    rowop(g01, g11);
                }
                if (qi == qj) {
                    // the rotated pair's coupling is zero, its diagonal real
                    g01 = make_double2(0.0, 0.0);
                    g10 = make_double2(0.0, 0.0);
                    g00.y = 0.0;
                    g11.y = 0.0;
                }
                G[ra][ca] = g00; G[ra][cb] = g01; G[rb][ca] = g10; G[rb][cb] = g11;
            }
            __syncthreads();
        }
    }
    // rotate the rows of this slice: [A_I A_J] <- [A_I A_J] V
    const int bI = rr_block(pr, round, nb), bJ = rr_block(nb - 1 - pr, round, nb);
    const int rlo = slice * JR, rhi = min(m_apply, rlo + JR);
    double2 nxv[JG_PER];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int u = 0; u < JG_PER; ++u) {
            const int e = tid + JB_NT * u, i = e % JG_RC, sc = e / JG_RC;
            const int c = jac_col(sc, bI, bJ, p);
            nxv[u] = (c >= 0 && r0 + i < rhi) ? A[(r0 + i) + (long)c * lda] : make_double2(0.0, 0.0);
        }
    };
    fetch(rlo);
    for (int r0 = rlo; r0 < rhi; r0 += JG_RC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < JG_PER; ++u) {
            const int e = tid + JB_NT * u;
            tile[e % JG_RC][e / JG_RC] = nxv[u];
        }
        __syncthreads();
        if (r0 + JG_RC < rhi) fetch(r0 + JG_RC);
#pragma unroll
        for (int u = 0; u < JG_PER; ++u) {
            const int e = tid + JB_NT * u, i = e % JG_RC, sc = e / JG_RC;
            const int c = jac_col(sc, bI, bJ, p);
            if (c < 0 || r0 + i >= rhi) continue;
            double2 v = make_double2(0.0, 0.0);
#pragma unroll 8
            for (int t = 0; t < JB_W; ++t) v = cfma(v, tile[i][t], V[t][sc]);
            A[(r0 + i) + (long)c * lda] = v;
        }
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

// ----------------------------------------------------------------------------
// Orthonormalisation inside a wide block from its Gram matrix.  G = Yb^H Yb
// (bw x bw) is factored G = R^H R column by column; a column is dropped (R row
// and Rinv row and column zero) when its norm after the projections on the
// earlier blocks, sqrt(G_cc), or after the earlier columns of the block,
// sqrt(d_c) with d_c the Cholesky pivot, is at most thr * ref[c] (ref =
// nullptr: thr).  The pivot carries a relative rounding error of about
// n eps G_cc / d_c, so the factorisation stops at the first column whose pivot
// falls below tau * G_cc: flag[0] = that column (bw when none), and columns
// from there on are left to the next block, which sees them projected off
// the columns kept here (the scale that made the pivot small is gone then).
// The first column that is not dropped always has d_c = G_cc, so flag[0] > 0.
// Rinv = R^-1 on the kept columns before the cut, so Yb Rinv has orthonormal
// columns up to eps cond(Yb)^2 (a second pass brings that to eps).  flag[1] =
// number of kept columns before the cut.  One workgroup; R in the upper
// triangle of the LDS array, Rinv^T in its strict lower triangle with the
// diagonal apart.
constexpr int QB = 64;        // columns per BCGS2 block
constexpr int CH_NT = 256;
constexpr int CH_EPT = (QB * (QB + 1) / 2 + CH_NT - 1) / CH_NT;   // triangle entries per thread

__global__ __launch_bounds__(CH_NT) void block_chol_kernel(const double2* __restrict__ Gin, int bw,
                                                            const double* __restrict__ ref, double thr, double tau,
                                                            double2* __restrict__ Rinv, int* __restrict__ flag)
{
    __shared__ double2 A[QB][QB + 1];
    __shared__ double gd[QB], rd[QB];
    __shared__ double2 dinv[QB];
    __shared__ int keep[QB];
    __shared__ int s_cut;
    const int tid = threadIdx.x;
    // entries of the upper triangle owned by this thread: t = j (j + 1) / 2 + i (i <= j),
    // t = tid, tid + CH_NT, ...; (-1, -1) past the end
    int2 own[CH_EPT];
#pragma unroll
    for (int q = 0; q < CH_EPT; ++q) {
        const int t = tid + CH_NT * q;
        int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > t) --j;
        while ((j + 1) * (j + 2) / 2 <= t) ++j;
        const int i = t - j * (j + 1) / 2;
        own[q] = j < bw ? make_int2(i, j) : make_int2(-1, -1);
        if (j < bw) A[i][j] = Gin[i + (long)j * bw];
    }
    if (tid < bw) gd[tid] = Gin[tid + (long)tid * bw].x;
    if (tid == 0) s_cut = bw;
    __syncthreads();
    for (int c = 0; c < bw; ++c) {
        if (tid == 0) {
            const double d = A[c][c].x, g = gd[c];
            const double lim = thr * (ref ? ref[c] : 1.0), lim2 = lim * lim;
            int k = 1;
            if (!(g > lim2) || !(d == d)) {
                k = 0;                      // dependent on the earlier blocks (or not finite)
            } else if (d < tau * g) {
                k = 0;                      // the pivot is not resolved: cut here
                s_cut = c;
            } else if (d <= lim2) {
                k = 0;                      // dependent on the earlier columns of the block
            }
            keep[c] = k;
            rd[c] = k ? sqrt(d) : 0.0;
        }
        __syncthreads();
        if (s_cut < bw) break;              // uniform: read from LDS after the barrier
        if (!keep[c]) continue;
        const double ri = 1.0 / rd[c];
        for (int j = c + 1 + tid; j < bw; j += CH_NT) A[c][j] = make_double2(A[c][j].x * ri, A[c][j].y * ri);
        if (tid == 0) A[c][c] = make_double2(rd[c], 0.0);
        __syncthreads();
        // the trailing triangle: each thread updates the entries it owns below row c
#pragma unroll
        for (int q = 0; q < CH_EPT; ++q) {
            const int i = own[q].x, j = own[q].y;
            if (i > c) {
                const double2 a = A[c][i], b = A[c][j];
                double2 t = A[i][j];
                // t -= conj(a) b
                t.x -= a.x * b.x + a.y * b.y;
                t.y -= a.x * b.y - a.y * b.x;
                A[i][j] = t;
            }
        }
        __syncthreads();
    }
    const int cut = s_cut;
    for (int c = cut + tid; c < bw; c += CH_NT) {
        keep[c] = 0;
        rd[c] = 0.0;
    }
    __syncthreads();
    // Rinv column j (thread j): Rinv_jj = 1 / R_jj, then upwards
    // Rinv_ij = -(sum_{i<k<=j} R_ik Rinv_kj) / R_ii over the kept rows
    if (tid < bw) {
        const int j = tid;
        const bool kj = keep[j] != 0;
        dinv[j] = make_double2(kj ? 1.0 / rd[j] : 0.0, 0.0);
        for (int i = j - 1; i >= 0; --i) {
            double2 v = make_double2(0.0, 0.0);
            if (kj && keep[i]) {
                double2 s = cmul(A[i][j], make_double2(1.0 / rd[j], 0.0));
                for (int k = i + 1; k < j; ++k) s = cfma(s, A[i][k], A[j][k]);
                v = make_double2(-s.x / rd[i], -s.y / rd[i]);
            }
            A[j][i] = v;
        }
    }
    __syncthreads();
    for (int e = tid; e < bw * bw; e += CH_NT) {
        const int i = e % bw, j = e / bw;
        Rinv[e] = i < j ? A[j][i] : (i == j ? dinv[j] : make_double2(0.0, 0.0));
    }
    if (tid == 0) {
        int kept = 0;
        for (int c = 0; c < bw; ++c) kept += keep[c];
        flag[0] = cut;
        flag[1] = kept;
    }
}

// G = Yb^H Yb for the bw columns of Yb, split along the rows like project_out.
static hipError_t gram_block(hipStream_t st, const double2* Yb, int ld, int n, int bw, double2* G, double2* part)
{
    const int S1 = n / PK_ROWS, r1 = n - S1 * PK_ROWS;
    const long bb = (long)bw * bw;
    hipError_t e = hipSuccess;
    if (S1 > 0) e = zgemm(st, 1, 0, bw, bw, PK_ROWS, 1.0, Yb, ld, PK_ROWS, Yb, ld, PK_ROWS, 0.0, part, bw, bb, S1);
    if (e == hipSuccess && r1 > 0)
        e = zgemm(st, 1, 0, bw, bw, r1, 1.0, Yb + S1 * PK_ROWS, ld, 0, Yb + S1 * PK_ROWS, ld, 0, 0.0,
                  part + (long)S1 * bb, bw, 0, 1);
    if (e == hipSuccess) e = sum_parts(st, part, S1 + (r1 > 0), bw, bw, G, bw, 0);
    return e;
}

size_t bcgs2_work_bytes(int n, int m)
{
    const size_t w = (size_t)m * QB;
    const size_t p1 = (size_t)(n / PK_ROWS + 1) * std::max(m, QB) * QB, p2 = (size_t)(m / PK_COLS + 1) * n * QB;
    return (w + std::max(p1, p2) + 2 * (size_t)QB * QB + (size_t)n * QB) * 16 + 512;
}

// Block classical Gram-Schmidt with reorthogonalisation (BCGS2) of Y (n x m,
// ld): each block of up to QB columns is projected off the finished blocks and
// orthonormalised inside the block from its Gram matrix, twice.  Columns found
// dependent (remaining norm <= 4 eps sqrt(n) times their original norm) come
// out as zero columns, so Q^H Q is the identity on the nonzero columns.  A
// block is cut where its Gram pivots stop being resolved in FP64 (columns of
// very different scale in one block), and the rest starts the next block.
// Once every column of a block is dependent, the range of Y is taken as
// captured and the remaining columns are set to zero: for Gaussian sketch
// columns the chance that a further column would still be independent is
// below 0.01^QB.
// work: bcgs2_work_bytes(n, m) bytes; n0: scratch of m doubles.
hipError_t bcgs2(hipStream_t st, double2* Y, int ld, int n, int m, void* work, double* n0)
{
    const double thr = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
    const double tau = 1e-6;
    const size_t p1 = (size_t)(n / PK_ROWS + 1) * std::max(m, QB) * QB, p2 = (size_t)(m / PK_COLS + 1) * n * QB;
    double2* W = (double2*)work;
    double2* part = W + (size_t)m * QB;
    double2* G = part + std::max(p1, p2);
    double2* Ri = G + (size_t)QB * QB;
    double2* T = Ri + (size_t)QB * QB;
    int* flag = (int*)(T + (size_t)n * QB);
    int hf[2] = {0, 0};
    hipError_t e = colnorms(st, n, m, Y, ld, 0, n0, 1);
    if (e != hipSuccess) return e;
    // column by column on columns [a, b) (two passes per CG_BW sub-block), for a block
    // the Gram route cannot finish; orig: the columns still carry their original scale
    auto exact = [&](int a, int b, bool orig) -> hipError_t {
        for (int s0 = a; s0 < b; s0 += CG_BW) {
            const int sbw = std::min(CG_BW, b - s0);
            for (int pass = 0; pass < 2; ++pass) {
                if (s0 > 0) {
                    hipError_t x = project_out(st, Y, ld, n, s0, sbw, W, part);
                    if (x != hipSuccess) return x;
                }
                hipLaunchKernelGGL(block_cgs2_kernel, dim3(1), dim3(CG_NT), 0, st, Y + (long)s0 * ld, ld, n, sbw,
                                   (pass == 0 && orig) ? n0 + s0 : (const double*)nullptr, thr);
                hipError_t x = hipGetLastError();
                if (x != hipSuccess) return x;
                if (s0 == 0) break;
            }
        }
        return hipSuccess;
    };
    for (int j0 = 0; j0 < m;) {
        int bw = std::min(QB, m - j0);
        double2* Yb = Y + (long)j0 * ld;
        for (int pass = 0; pass < 2; ++pass) {
            if (j0 > 0 && (e = project_out(st, Y, ld, n, j0, bw, W, part)) != hipSuccess) return e;
            if ((e = gram_block(st, Yb, ld, n, bw, G, part)) != hipSuccess) return e;
            hipLaunchKernelGGL(block_chol_kernel, dim3(1), dim3(CH_NT), 0, st, G, bw,
                               pass == 0 ? n0 + j0 : (const double*)nullptr, thr, tau, Ri, flag);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(hf, flag, sizeof(hf), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
            const int ldr = bw;
            if (hf[0] < 1 || (pass == 1 && hf[0] < bw)) {
                // not expected (see block_chol_kernel); finish these columns one by one
                if ((e = exact(j0, j0 + bw, pass == 0)) != hipSuccess) return e;
                break;
            }
            if (pass == 0) {
                if (hf[0] == bw && hf[1] == 0) return zero_c128(st, n, m - j0, Yb, ld, 0, 1);
                bw = hf[0];
            }
            if ((e = zgemm(st, 0, 0, n, bw, bw, 1.0, Yb, ld, 0, Ri, ldr, 0, 0.0, T, n, 0, 1)) != hipSuccess) return e;
            if ((e = copy_c128(st, n, bw, T, n, 0, Yb, ld, 0, 1)) != hipSuccess) return e;
        }
        j0 += bw;
    }
    return hipSuccess;
}

int jacobi_blocks(int p) { int nb = (p + JB_B - 1) / JB_B; return nb + (nb & 1); }

size_t jacobi_work_bytes(int m, int m_apply, int p)
{
    const size_t pairs = (size_t)jacobi_blocks(p) / 2;
    const size_t slices = (size_t)(std::max(m, 1) + JRG - 1) / JRG;
    (void)m_apply;
    return pairs * (slices + 1) * JB_W * JB_W * 16 + pairs * 4 + 256;
}

hipError_t jacobi_round(hipStream_t st, double2* A, int lda, int m, int m_apply, int p, int round, int inner,
                        double tol, double zthr2, double* offmax, void* work)
{
    const int nb = jacobi_blocks(p), pairs = nb / 2;
    const int gs = (std::max(m, 1) + JRG - 1) / JRG, as = (m_apply + JR - 1) / JR;
    double2* Gp = (double2*)work;
    hipLaunchKernelGGL(jacobi_gram_kernel, dim3(pairs, gs), dim3(JB_NT), 0, st, A, lda, m, p, nb, round, Gp);
    hipLaunchKernelGGL(jacobi_rotate_kernel, dim3(pairs, as), dim3(JB_NT), 0, st, A, lda, m_apply, p, nb, round, Gp,
                       gs, inner, tol, zthr2, offmax);
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
