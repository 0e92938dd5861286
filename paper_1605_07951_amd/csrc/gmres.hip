// Kernels of the flexible GMRES sampling path.
//
// C columns of an n x C block are C independent systems T(z_k) x = u (column
// c belongs to point c / L), each with its own Krylov basis.  Basis vector i
// of every column is the n x C block V + i*sV (leading dimension ldv); the
// preconditioned directions Z_i likewise.  Small per-column quantities are
// stored "index-major": entry i of column c at [i * C + c].  All arithmetic
// is FP64.
#include "common.h"
#include "kernels.h"

namespace rsrr {

constexpr int GM_NT = 256;               // threads per workgroup
constexpr int GM_RPT = 4;                // rows per thread in the column kernels
constexpr int GM_RS = GM_NT * GM_RPT;    // rows per slice
constexpr int GM_MAXM = 64;              // longest restart cycle

int gm_slices(int n) { return (n + GM_RS - 1) / GM_RS; }
int gm_max_restart() { return GM_MAXM; }

static dim3 flat_grid(long elems) { return dim3((unsigned)((elems + GM_NT - 1) / GM_NT)); }

__device__ inline double2 wave_sum(double2 v)
{
    for (int off = 32; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off);
        v.y += __shfl_xor(v.y, off);
    }
    return v;
}

// Y(:, c) = coef[c / L] * Z(:, c)
__global__ __launch_bounds__(GM_NT) void gm_point_scale_kernel(int n, int C, int L, const double2* __restrict__ Z,
                                                                int ldz, const double2* __restrict__ coef,
                                                                double2* __restrict__ Y, int ldy)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    Y[i + (long)c * ldy] = cmul(coef[c / L], Z[i + (long)c * ldz]);
}

// D = (c64) V
__global__ __launch_bounds__(GM_NT) void gm_narrow_kernel(int n, int C, const double2* __restrict__ V, int ldv,
                                                           float2* __restrict__ D, int ldd)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    D[i + (long)c * ldd] = to_c64(V[i + (long)c * ldv]);
}

// Z = (c128) D
__global__ __launch_bounds__(GM_NT) void gm_widen_kernel(int n, int C, const float2* __restrict__ D, int ldd,
                                                          double2* __restrict__ Z, int ldz)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    Z[i + (long)c * ldz] = to_c128(D[i + (long)c * ldd]);
}

// V(:, c) = U(:, c % L) - V(:, c)   (V holds T x on entry: the residual of x)
__global__ __launch_bounds__(GM_NT) void gm_resid_kernel(int n, int C, int L, const double2* __restrict__ U, int ldu,
                                                          double2* __restrict__ V, int ldv)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const double2 u = U[i + (long)(c % L) * ldu];
    double2* v = V + i + (long)c * ldv;
    *v = csub(u, *v);
}

// X(:, c) *= s[c]
__global__ __launch_bounds__(GM_NT) void gm_scale_kernel(int n, int C, const double* __restrict__ s,
                                                          double2* __restrict__ X, int ldx)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const double f = s[c];
    double2* x = X + i + (long)c * ldx;
    x->x *= f;
    x->y *= f;
}

// S(:, idx[b]*L + l) = X(:, b*L + l)
__global__ __launch_bounds__(GM_NT) void gm_scatter_kernel(int n, int C, int L, const double2* __restrict__ X,
                                                            int ldx, const int* __restrict__ idx,
                                                            double2* __restrict__ S, int lds)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const int b = c / L, l = c % L;
    S[i + ((long)idx[b] * L + l) * lds] = X[i + (long)c * ldx];
}

// part[(s * j1 + i) * C + c] = sum over the rows of slice s of conj(V_i(r, c)) W(r, c),
// i = 0 .. j1-1.  One workgroup per (column, row slice).
__global__ __launch_bounds__(GM_NT) void gm_dots_kernel(int n, int C, int j1, const double2* __restrict__ V, int ldv,
                                                         long sV, const double2* __restrict__ W, int ldw,
                                                         const int* __restrict__ done, double2* __restrict__ part)
{
    __shared__ double2 red[GM_MAXM + 1][GM_NT / 64];
    const int c = blockIdx.x, s = blockIdx.y;
    if (done[c]) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long col = (long)c * ldv;
    double2 w[GM_RPT];
#pragma unroll
    for (int q = 0; q < GM_RPT; ++q) {
        const int r = s * GM_RS + q * GM_NT + threadIdx.x;
        w[q] = r < n ? W[r + (long)c * ldw] : make_double2(0.0, 0.0);
    }
    for (int i = 0; i < j1; ++i) {
        const double2* vi = V + i * sV + col;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < GM_RPT; ++q) {
            const int r = s * GM_RS + q * GM_NT + threadIdx.x;
            if (r < n) acc = cfma(acc, cconj(vi[r]), w[q]);
        }
        acc = wave_sum(acc);
        if (lane == 0) red[i][wv] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < j1; i += GM_NT) {
        double2 t = red[i][0];
        for (int q = 1; q < GM_NT / 64; ++q) t = cadd(t, red[i][q]);
        part[((long)s * j1 + i) * C + c] = t;
    }
}

// h[i * C + c] = sum_s part[(s * j1 + i) * C + c]; Hc[i * C + c] = h (first pass) or += h.
__global__ __launch_bounds__(GM_NT) void gm_reduce_kernel(int C, int j1, int ns, const double2* __restrict__ part,
                                                           const int* __restrict__ done, double2* __restrict__ h,
                                                           double2* __restrict__ Hc, int first)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)j1 * C) return;
    const int c = (int)(e % C), i = (int)(e / C);
    double2 t = make_double2(0.0, 0.0);
    if (!done[c])
        for (int s = 0; s < ns; ++s) t = cadd(t, part[((long)s * j1 + i) * C + c]);
    h[e] = t;
    Hc[e] = first ? t : cadd(Hc[e], t);
}

// W(:, c) -= sum_{i < j1} h[i * C + c] V_i(:, c)
__global__ __launch_bounds__(GM_NT) void gm_update_kernel(int n, int C, int j1, const double2* __restrict__ V, int ldv,
                                                           long sV, const double2* __restrict__ h,
                                                           const int* __restrict__ done, double2* __restrict__ W,
                                                           int ldw)
{
    __shared__ double2 hs[GM_MAXM + 1];
    const int c = blockIdx.x, s = blockIdx.y;
    if (done[c]) return;
    for (int i = threadIdx.x; i < j1; i += GM_NT) hs[i] = h[(long)i * C + c];
    __syncthreads();
    const long col = (long)c * ldv;
#pragma unroll
    for (int q = 0; q < GM_RPT; ++q) {
        const int r = s * GM_RS + q * GM_NT + threadIdx.x;
        if (r >= n) continue;
        double2 acc = W[r + (long)c * ldw];
        for (int i = 0; i < j1; ++i) acc = cfms(acc, hs[i], V[i * sV + col + r]);
        W[r + (long)c * ldw] = acc;
    }
}

// One Arnoldi column j of every active system: apply the earlier Givens
// rotations to H(0..j, j), make the rotation that removes h_{j+1,j} = hn[c],
// store column j of the triangular factor (Rm[(j * M + i) * C + c]), update
// the right-hand side g and the residual estimate |g_{j+1}|.  A column whose
// estimate is at most thr[c] (or whose Arnoldi process broke down, hn = 0)
// is marked done with kc[c] = j + 1 and counted in *ndone.  inv[c] receives
// the factor that normalises the new basis vector (0 for done columns).
__global__ __launch_bounds__(GM_NT) void gm_givens_kernel(int C, int j, int M, const double2* __restrict__ Hc,
                                                           const double* __restrict__ hn,
                                                           const double* __restrict__ thr, double* __restrict__ cs,
                                                           double2* __restrict__ sn, double2* __restrict__ g,
                                                           double2* __restrict__ Rm, int* __restrict__ done,
                                                           int* __restrict__ kc, double* __restrict__ inv,
                                                           int* __restrict__ ndone)
{
    const int c = blockIdx.x * GM_NT + threadIdx.x;
    if (c >= C) return;
    if (done[c]) { inv[c] = 0.0; return; }
    double2 a = Hc[c];
    for (int i = 0; i < j; ++i) {
        const double ci = cs[(long)i * C + c];
        const double2 si = sn[(long)i * C + c];
        const double2 b = Hc[(long)(i + 1) * C + c];
        // [a'; b'] = [ci si; -conj(si) ci] [a; b]
        const double2 a2 = cfma(make_double2(ci * a.x, ci * a.y), si, b);
        const double2 b2 = csub(make_double2(ci * b.x, ci * b.y), cmul(cconj(si), a));
        Rm[((long)j * M + i) * C + c] = a2;
        a = b2;
    }
    const double b = hn[c];
    double cj, r;
    double2 sj;
    const double aa = sqrt(a.x * a.x + a.y * a.y);
    if (b == 0.0) {
        cj = 1.0; sj = make_double2(0.0, 0.0); r = aa;
    } else if (aa == 0.0) {
        cj = 0.0; sj = make_double2(1.0, 0.0); r = b;
    } else {
        const double t = hypot(aa, b);
        cj = aa / t;
        sj = make_double2(a.x / aa * (b / t), a.y / aa * (b / t));
        r = t;
    }
    // rotated diagonal entry: (a / |a|) t, or b when a = 0
    const double2 rjj = aa == 0.0 ? make_double2(r, 0.0) : make_double2(a.x / aa * r, a.y / aa * r);
    Rm[((long)j * M + j) * C + c] = rjj;
    cs[(long)j * C + c] = cj;
    sn[(long)j * C + c] = sj;
    const double2 gj = g[(long)j * C + c];
    const double2 g1 = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));  // -conj(s) g_j
    g[(long)j * C + c] = make_double2(cj * gj.x, cj * gj.y);
    g[(long)(j + 1) * C + c] = g1;
    const double est = sqrt(g1.x * g1.x + g1.y * g1.y);
    if (est <= thr[c] || b == 0.0) {
        done[c] = 1;
        kc[c] = j + 1;
        inv[c] = 0.0;
        atomicAdd(ndone, 1);
    } else {
        inv[c] = 1.0 / b;
    }
}

// y = R^-1 g(0..k-1) per column, k = kc[c] when the column finished in this
// cycle, jend for a column still running, 0 for a column that was done before
// the cycle (active[c] == 0).  y[i * C + c] = 0 for i >= k.
__global__ __launch_bounds__(GM_NT) void gm_solve_kernel(int C, int M, int jend, const double2* __restrict__ Rm,
                                                          const double2* __restrict__ g,
                                                          const int* __restrict__ active, const int* __restrict__ kc,
                                                          double2* __restrict__ y, int* __restrict__ steps)
{
    const int c = blockIdx.x * GM_NT + threadIdx.x;
    if (c >= C) return;
    const int k = active[c] ? (kc[c] ? kc[c] : jend) : 0;
    steps[c] = k;
    for (int i = M - 1; i >= 0; --i) {
        if (i >= k) { y[(long)i * C + c] = make_double2(0.0, 0.0); continue; }
        double2 s = g[(long)i * C + c];
        for (int l = i + 1; l < k; ++l) s = cfms(s, Rm[((long)l * M + i) * C + c], y[(long)l * C + c]);
        const double2 d = Rm[((long)i * M + i) * C + c];
        const double dd = d.x * d.x + d.y * d.y;
        y[(long)i * C + c] = dd == 0.0 ? make_double2(0.0, 0.0)
                                        : make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
    }
}

// X(:, c) += sum_{i < k} y[i * C + c] Z_i(:, c)
__global__ __launch_bounds__(GM_NT) void gm_combine_kernel(int n, int C, int k, const double2* __restrict__ Z,
                                                            int ldz, long sZ, const double2* __restrict__ y,
                                                            double2* __restrict__ X, int ldx)
{
    __shared__ double2 ys[GM_MAXM];
    const int c = blockIdx.x, s = blockIdx.y;
    for (int i = threadIdx.x; i < k; i += GM_NT) ys[i] = y[(long)i * C + c];
    __syncthreads();
    const long col = (long)c * ldz;
#pragma unroll
    for (int q = 0; q < GM_RPT; ++q) {
        const int r = s * GM_RS + q * GM_NT + threadIdx.x;
        if (r >= n) continue;
        double2 acc = X[r + (long)c * ldx];
        for (int i = 0; i < k; ++i) acc = cfma(acc, ys[i], Z[i * sZ + col + r]);
        X[r + (long)c * ldx] = acc;
    }
}

// Z = (c128) sum_{s < S} P_s (complex FP32 partial products of a split
// contraction, slice s at P + s*sP), summed in FP64.
__global__ __launch_bounds__(GM_NT) void gm_sum_widen_kernel(int n, int C, const float2* __restrict__ P, int ldp,
                                                              long sP, int S, double2* __restrict__ Z, int ldz)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const long o = i + (long)c * ldp;
    double2 acc = make_double2(0.0, 0.0);
    for (int s = 0; s < S; ++s) {
        const float2 v = P[s * sP + o];
        acc.x += (double)v.x;
        acc.y += (double)v.y;
    }
    Z[i + (long)c * ldz] = acc;
}

// W = sum_{s < S} P_s (complex FP64 partial products).
__global__ __launch_bounds__(GM_NT) void gm_sum_c128_kernel(int n, int C, const double2* __restrict__ P, int ldp,
                                                             long sP, int S, double2* __restrict__ W, int ldw)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * C) return;
    const int i = (int)(e % n), c = (int)(e / n);
    const long o = i + (long)c * ldp;
    double2 acc = P[o];
    for (int s = 1; s < S; ++s) acc = cadd(acc, P[s * sP + o]);
    W[i + (long)c * ldw] = acc;
}

// W_b = T(z_b) Z_b for the Helmholtz single-layer matrix without storing it:
// the entries are generated in FP64 as they are consumed (the same expressions
// as the assembly kernel), Z_b (n x L, L <= LC) staged through LDS in chunks
// of KC rows.  Grid: row tiles of RW x points.
template <int LC, int RW>
__global__ __launch_bounds__(RW) void helm_apply_kernel(int n, int L, const double* __restrict__ pts, double w,
                                                         const double2* __restrict__ z,
                                                         const double2* __restrict__ Z, int ldz, long sZ,
                                                         double2* __restrict__ W, int ldw, long sW)
{
    constexpr int KC = 64;
    __shared__ double2 zs[KC][LC];
    __shared__ double pc[KC][3];
    const int b = blockIdx.y;
    const int row = blockIdx.x * RW + threadIdx.x;
    const double2 zb = z[b];
    const double inv4pi = 0.25 / M_PI;
    const double diag_re = 0.5 * sqrt(w / M_PI);
    const double2* Zb = Z + b * sZ;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (row < n) { xi = pts[3 * row]; yi = pts[3 * row + 1]; zi = pts[3 * row + 2]; }
    double2 acc[LC];
#pragma unroll
    for (int c = 0; c < LC; ++c) acc[c] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < n; k0 += KC) {
        for (int e = threadIdx.x; e < KC * LC; e += RW) {
            const int kk = e % KC, c = e / KC;
            zs[kk][c] = (k0 + kk < n && c < L) ? Zb[(k0 + kk) + (long)c * ldz] : make_double2(0.0, 0.0);
        }
        for (int e = threadIdx.x; e < KC * 3; e += RW) {
            const int kk = e / 3, d = e % 3;
            pc[kk][d] = k0 + kk < n ? pts[3 * (k0 + kk) + d] : 0.0;
        }
        __syncthreads();
        if (row < n) {
            const int kend = min(KC, n - k0);
            for (int kk = 0; kk < kend; ++kk) {
                const int j = k0 + kk;
                double2 t;
                if (j != row) {
                    const double dx = xi - pc[kk][0], dy = yi - pc[kk][1], dz = zi - pc[kk][2];
                    const double r = sqrt(dx * dx + dy * dy + dz * dz);
                    const double scale = w * inv4pi / r;
                    double s, co;
                    sincos(zb.x * r, &s, &co);
                    const double m = scale * exp(-zb.y * r);
                    t = make_double2(m * co, m * s);
                } else {
                    t = make_double2(diag_re - zb.y * w * inv4pi, zb.x * w * inv4pi);
                }
#pragma unroll
                for (int c = 0; c < LC; ++c) acc[c] = cfma(acc[c], t, zs[kk][c]);
            }
        }
        __syncthreads();
    }
    if (row >= n) return;
    double2* Wb = W + b * sW;
#pragma unroll
    for (int c = 0; c < LC; ++c)
        if (c < L) Wb[row + (long)c * ldw] = acc[c];
}

hipError_t helm_apply(hipStream_t st, int n, int L, const double* pts, double w, const double2* z, const double2* Z,
                      int ldz, long sZ, double2* W, int ldw, long sW, int B)
{
    for (int c0 = 0; c0 < L; c0 += 16) {
        const int Lc = L - c0 < 16 ? L - c0 : 16;
        const double2* Zc = Z + (long)c0 * ldz;
        double2* Wc = W + (long)c0 * ldw;
#define HA_L(LC)                                                                                                   \
    hipLaunchKernelGGL((helm_apply_kernel<LC, 256>), dim3((unsigned)((n + 255) / 256), (unsigned)B), dim3(256), 0, \
                       st, n, Lc, pts, w, z, Zc, ldz, sZ, Wc, ldw, sW)
        if (Lc <= 2) HA_L(2); else if (Lc <= 4) HA_L(4); else if (Lc <= 8) HA_L(8); else HA_L(16);
#undef HA_L
    }
    return hipGetLastError();
}

// B identity matrices n x n (complex FP32, leading dimension ld, stride sA).
__global__ __launch_bounds__(GM_NT) void gm_eye_c64_kernel(int n, float2* __restrict__ A, int ld, long sA)
{
    const long e = (long)blockIdx.x * GM_NT + threadIdx.x;
    if (e >= (long)n * n) return;
    const int i = (int)(e % n), c = (int)(e / n);
    A[blockIdx.y * sA + i + (long)c * ld] = make_float2(i == c ? 1.f : 0.f, 0.f);
}

// g[c] = g0[c] (row 0 of the right-hand side), g rows 1.. untouched.
__global__ __launch_bounds__(GM_NT) void gm_g0_kernel(int C, const double* __restrict__ g0, double2* __restrict__ g)
{
    const int c = blockIdx.x * GM_NT + threadIdx.x;
    if (c < C) g[c] = make_double2(g0[c], 0.0);
}

hipError_t gm_point_scale(hipStream_t st, int n, int C, int L, const double2* Z, int ldz, const double2* coef,
                          double2* Y, int ldy)
{
    hipLaunchKernelGGL(gm_point_scale_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, L, Z, ldz, coef, Y,
                       ldy);
    return hipGetLastError();
}
hipError_t gm_narrow(hipStream_t st, int n, int C, const double2* V, int ldv, float2* D, int ldd)
{
    hipLaunchKernelGGL(gm_narrow_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, V, ldv, D, ldd);
    return hipGetLastError();
}
hipError_t gm_widen(hipStream_t st, int n, int C, const float2* D, int ldd, double2* Z, int ldz)
{
    hipLaunchKernelGGL(gm_widen_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, D, ldd, Z, ldz);
    return hipGetLastError();
}
hipError_t gm_resid(hipStream_t st, int n, int C, int L, const double2* U, int ldu, double2* V, int ldv)
{
    hipLaunchKernelGGL(gm_resid_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, L, U, ldu, V, ldv);
    return hipGetLastError();
}
hipError_t gm_scale(hipStream_t st, int n, int C, const double* s, double2* X, int ldx)
{
    hipLaunchKernelGGL(gm_scale_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, s, X, ldx);
    return hipGetLastError();
}
hipError_t gm_scatter(hipStream_t st, int n, int C, int L, const double2* X, int ldx, const int* idx, double2* S,
                      int lds)
{
    hipLaunchKernelGGL(gm_scatter_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, L, X, ldx, idx, S, lds);
    return hipGetLastError();
}
hipError_t gm_orth_pass(hipStream_t st, int n, int C, int j1, const double2* V, int ldv, long sV, double2* W, int ldw,
                        const int* done, double2* part, double2* h, double2* Hc, int first)
{
    const int ns = gm_slices(n);
    hipLaunchKernelGGL(gm_dots_kernel, dim3((unsigned)C, (unsigned)ns), dim3(GM_NT), 0, st, n, C, j1, V, ldv, sV, W,
                       ldw, done, part);
    hipLaunchKernelGGL(gm_reduce_kernel, flat_grid((long)j1 * C), dim3(GM_NT), 0, st, C, j1, ns, part, done, h, Hc,
                       first);
    hipLaunchKernelGGL(gm_update_kernel, dim3((unsigned)C, (unsigned)ns), dim3(GM_NT), 0, st, n, C, j1, V, ldv, sV, h,
                       done, W, ldw);
    return hipGetLastError();
}
hipError_t gm_givens(hipStream_t st, int C, int j, int M, const double2* Hc, const double* hn, const double* thr,
                     double* cs, double2* sn, double2* g, double2* Rm, int* done, int* kc, double* inv, int* ndone)
{
    hipLaunchKernelGGL(gm_givens_kernel, dim3((unsigned)((C + GM_NT - 1) / GM_NT)), dim3(GM_NT), 0, st, C, j, M, Hc,
                       hn, thr, cs, sn, g, Rm, done, kc, inv, ndone);
    return hipGetLastError();
}
hipError_t gm_solve(hipStream_t st, int C, int M, int jend, const double2* Rm, const double2* g, const int* active,
                    const int* kc, double2* y, int* steps)
{
    hipLaunchKernelGGL(gm_solve_kernel, dim3((unsigned)((C + GM_NT - 1) / GM_NT)), dim3(GM_NT), 0, st, C, M, jend, Rm,
                       g, active, kc, y, steps);
    return hipGetLastError();
}
hipError_t gm_combine(hipStream_t st, int n, int C, int k, const double2* Z, int ldz, long sZ, const double2* y,
                      double2* X, int ldx)
{
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(gm_combine_kernel, dim3((unsigned)C, (unsigned)gm_slices(n)), dim3(GM_NT), 0, st, n, C, k, Z,
                       ldz, sZ, y, X, ldx);
    return hipGetLastError();
}
hipError_t gm_sum_widen(hipStream_t st, int n, int C, const float2* P, int ldp, long sP, int S, double2* Z, int ldz)
{
    hipLaunchKernelGGL(gm_sum_widen_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, P, ldp, sP, S, Z, ldz);
    return hipGetLastError();
}
hipError_t gm_sum_c128(hipStream_t st, int n, int C, const double2* P, int ldp, long sP, int S, double2* W, int ldw)
{
    hipLaunchKernelGGL(gm_sum_c128_kernel, flat_grid((long)n * C), dim3(GM_NT), 0, st, n, C, P, ldp, sP, S, W, ldw);
    return hipGetLastError();
}
hipError_t gm_eye_c64(hipStream_t st, int n, float2* A, int ld, long sA, int B)
{
    hipLaunchKernelGGL(gm_eye_c64_kernel, dim3((unsigned)(((long)n * n + GM_NT - 1) / GM_NT), (unsigned)B),
                       dim3(GM_NT), 0, st, n, A, ld, sA);
    return hipGetLastError();
}
hipError_t gm_g0(hipStream_t st, int C, const double* g0, double2* g)
{
    hipLaunchKernelGGL(gm_g0_kernel, dim3((unsigned)((C + GM_NT - 1) / GM_NT)), dim3(GM_NT), 0, st, C, g0, g);
    return hipGetLastError();
}

}  // namespace rsrr
