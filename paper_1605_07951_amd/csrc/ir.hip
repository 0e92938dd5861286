// Element-wise and reduction kernels of the mixed-precision refinement
// (complex FP32 solves, FP64 residuals) and of the probe/solution copies.
// All operate on a batch of n x L column blocks (stride per point).
#include "common.h"
#include "kernels.h"

namespace rsrr {

constexpr int EW_NT = 256;

// D_k = (c64) U for every point k.
__global__ __launch_bounds__(EW_NT) void bcast_to_c64_kernel(int n, int L, const double2* __restrict__ U, int ldu,
                                                              float2* __restrict__ D, int ldd, long sD)
{
    const int k = blockIdx.y;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    D[k * sD + i + (long)c * ldd] = to_c64(U[i + (long)c * ldu]);
}

// R_k = U for every point k (FP64).
__global__ __launch_bounds__(EW_NT) void bcast_c128_kernel(int n, int L, const double2* __restrict__ U, int ldu,
                                                            double2* __restrict__ R, int ldr, long sR)
{
    const int k = blockIdx.y;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    R[k * sR + i + (long)c * ldr] = U[i + (long)c * ldu];
}

// X_k = (c128) D_k.
__global__ __launch_bounds__(EW_NT) void widen_kernel(int n, int L, const float2* __restrict__ D, int ldd, long sD,
                                                       double2* __restrict__ X, int ldx, long sX)
{
    const int k = blockIdx.y;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    X[k * sX + i + (long)c * ldx] = to_c128(D[k * sD + i + (long)c * ldd]);
}

// out[k*L + c] = ||X_k(:, c)||_2 (FP64, fixed summation order).
__global__ __launch_bounds__(EW_NT) void colnorm_kernel(int n, int L, const double2* __restrict__ X, int ldx, long sX,
                                                         double* __restrict__ out)
{
    __shared__ double red[EW_NT / 64];
    const int c = blockIdx.x, k = blockIdx.y;
    const double2* col = X + k * sX + (long)c * ldx;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += EW_NT) {
        const double2 a = col[i];
        v += a.x * a.x + a.y * a.y;
    }
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < EW_NT / 64; ++w) s += red[w];
        out[(long)k * L + c] = sqrt(s);
    }
}

// D_k(:, c) = (c64) (R_k(:, c) * inv[k*L + c]) for active points.
__global__ __launch_bounds__(EW_NT) void scale_narrow_kernel(int n, int L, const double2* __restrict__ R, int ldr,
                                                              long sR, const double* __restrict__ inv,
                                                              float2* __restrict__ D, int ldd, long sD,
                                                              const int* __restrict__ active)
{
    const int k = blockIdx.y;
    if (active && !active[k]) return;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    const double s = inv[(long)k * L + c];
    const double2 r = R[k * sR + i + (long)c * ldr];
    D[k * sD + i + (long)c * ldd] = make_float2((float)(r.x * s), (float)(r.y * s));
}

// X_k(:, c) += scale[k*L + c] * D_k(:, c) for active points.
__global__ __launch_bounds__(EW_NT) void axpy_widen_kernel(int n, int L, const float2* __restrict__ D, int ldd,
                                                            long sD, const double* __restrict__ scale,
                                                            double2* __restrict__ X, int ldx, long sX,
                                                            const int* __restrict__ active)
{
    const int k = blockIdx.y;
    if (active && !active[k]) return;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    const double s = scale[(long)k * L + c];
    const float2 d = D[k * sD + i + (long)c * ldd];
    double2* x = X + k * sX + i + (long)c * ldx;
    double2 v = *x;
    v.x += s * (double)d.x;
    v.y += s * (double)d.y;
    *x = v;
}

// ---- real FP32 correction solves (a real NEP at real points) ----
// The FP64 residual stays complex (its imaginary part is exactly zero for a
// real problem); the real FP32 LU solves with its real part.  If the problem
// is not real after all, the refinement stalls and the point is redone on the
// FP64 complex path.

// Tr_k = (float) Re T_k.
__global__ __launch_bounds__(EW_NT) void narrow_real_kernel(int n, const double2* __restrict__ T, int ldt, long sT,
                                                             float* __restrict__ Tr, int ldr, long sTr)
{
    const int k = blockIdx.y;
    const long e = (long)blockIdx.x * EW_NT + threadIdx.x;
    if (e >= (long)n * n) return;
    const int i = (int)(e % n), c = (int)(e / n);
    Tr[k * sTr + i + (long)c * ldr] = (float)T[k * sT + i + (long)c * ldt].x;
}

// D_k(:, c) = (float) (Re R_k(:, c) * inv[k*L + c]) (inv = null: 1) for active points.
__global__ __launch_bounds__(EW_NT) void scale_narrow_real_kernel(int n, int L, const double2* __restrict__ R, int ldr,
                                                                   long sR, const double* __restrict__ inv,
                                                                   float* __restrict__ D, int ldd, long sD,
                                                                   const int* __restrict__ active)
{
    const int k = blockIdx.y;
    if (active && !active[k]) return;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    const double s = inv ? inv[(long)k * L + c] : 1.0;
    D[k * sD + i + (long)c * ldd] = (float)(R[k * sR + i + (long)c * ldr].x * s);
}

// X_k(:, c) = (D_k(:, c), 0) when scale is null, else Re X_k(:, c) += scale[k*L + c] * D_k(:, c),
// for active points.
__global__ __launch_bounds__(EW_NT) void axpy_widen_real_kernel(int n, int L, const float* __restrict__ D, int ldd,
                                                                 long sD, const double* __restrict__ scale,
                                                                 double2* __restrict__ X, int ldx, long sX,
                                                                 const int* __restrict__ active)
{
    const int k = blockIdx.y;
    if (active && !active[k]) return;
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e >= n * L) return;
    const int i = e % n, c = e / n;
    const double d = (double)D[k * sD + i + (long)c * ldd];
    double2* x = X + k * sX + i + (long)c * ldx;
    if (!scale) {
        *x = make_double2(d, 0.0);
    } else {
        double2 v = *x;
        v.x += scale[(long)k * L + c] * d;
        *x = v;
    }
}

// Copy n x m (c128) blocks: Y_k = X_k.
__global__ __launch_bounds__(EW_NT) void copy_c128_kernel(int n, int m, const double2* __restrict__ X, int ldx,
                                                           long sX, double2* __restrict__ Y, int ldy, long sY)
{
    const int k = blockIdx.y;
    const long e = (long)blockIdx.x * EW_NT + threadIdx.x;
    if (e >= (long)n * m) return;
    const int i = (int)(e % n), c = (int)(e / n);
    Y[k * sY + i + (long)c * ldy] = X[k * sX + i + (long)c * ldx];
}

// Scale each column c of X (n x m) by s[c] (in place, FP64).
__global__ __launch_bounds__(EW_NT) void scale_cols_kernel(int n, int m, double2* __restrict__ X, int ldx,
                                                            const double* __restrict__ s)
{
    const long e = (long)blockIdx.x * EW_NT + threadIdx.x;
    if (e >= (long)n * m) return;
    const int i = (int)(e % n), c = (int)(e / n);
    double2* x = X + i + (long)c * ldx;
    const double f = s[c];
    x->x *= f;
    x->y *= f;
}

// ---- ragged-batch helpers ----

// Identity outside the leading nk x nk block of each P x P matrix (both copies
// may be null); the leading block is written by the assembly afterwards.  Only
// the padding is visited (grid-stride): with p = P - n, element e < n p lies in
// column e / p of the rows below the block (zero), the rest in the last p
// columns (identity).
template <typename C>
__global__ __launch_bounds__(EW_NT) void pad_identity_kernel(C* __restrict__ T, int ld, long sT, int P,
                                                              const int* __restrict__ nk)
{
    const int k = blockIdx.y;
    const int n = nk[k], p = P - n;
    const long total = p > 0 ? (long)p * (n + P) : 0;
    for (long e = (long)blockIdx.x * EW_NT + threadIdx.x; e < total; e += (long)gridDim.x * EW_NT) {
        int i, j;
        if (e < (long)n * p) {
            j = (int)(e / p);
            i = n + (int)(e % p);
        } else {
            const long f = e - (long)n * p;
            j = n + (int)(f / P);
            i = (int)(f % P);
        }
        C v;
        v.x = (i == j) ? 1 : 0;
        v.y = 0;
        T[k * sT + i + (long)j * ld] = v;
    }
}

// Fill n x m (c128) blocks with zeros (graph-safe replacement of a memset).
__global__ __launch_bounds__(EW_NT) void zero_c128_kernel(int n, int m, double2* __restrict__ X, int ldx, long sX)
{
    const int k = blockIdx.y;
    const long e = (long)blockIdx.x * EW_NT + threadIdx.x;
    if (e >= (long)n * m) return;
    X[k * sX + (e % n) + (long)(e / n) * ldx] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(EW_NT) void zero_int_kernel(int* __restrict__ p, int n)
{
    const int e = blockIdx.x * EW_NT + threadIdx.x;
    if (e < n) p[e] = 0;
}

// Per-point refinement state: active = (getrf info == 0), prev = +inf.
__global__ __launch_bounds__(EW_NT) void ir_init_kernel(int M, const int* __restrict__ info, int* __restrict__ active,
                                                         double* __restrict__ prev, double* __restrict__ resid,
                                                         int* __restrict__ iters)
{
    const int k = blockIdx.x * EW_NT + threadIdx.x;
    if (k >= M) return;
    active[k] = info[k] == 0 ? 1 : 0;
    prev[k] = INFINITY;
    resid[k] = 0.0;
    iters[k] = 0;
}

// Device-side refinement decision for iteration `it` (one thread per point):
// rn, xn: column norms of R_k and X_k (M x Lmax); un: probe column norms
// (M x Lmax, zero for padding columns); frob: ||T_k||_F.  A point stops when
// its backward error max_c ||r_c|| / (||T||_F ||x_c|| + ||u_c||) <= tol_be,
// when the residual did not halve, or at it == maxit.  Writes the scaling
// of the next correction (inv = 1/||r_c||, scl = ||r_c||).
__global__ __launch_bounds__(EW_NT) void ir_decide_kernel(int M, int Lmax, const double* __restrict__ rn,
                                                           const double* __restrict__ xn,
                                                           const double* __restrict__ un,
                                                           const double* __restrict__ frob, double tol_be, int it,
                                                           int maxit, int* __restrict__ active,
                                                           double* __restrict__ prev, double* __restrict__ resid,
                                                           int* __restrict__ iters, double* __restrict__ inv,
                                                           double* __restrict__ scl)
{
    const int k = blockIdx.x * EW_NT + threadIdx.x;
    if (k >= M) return;
    if (!active[k]) return;
    double r = 0.0, eta = 0.0;
    bool nan = false;
    for (int c = 0; c < Lmax; ++c) {
        const double u = un[(long)k * Lmax + c];
        if (!(u > 0.0)) continue;
        const double rr = rn[(long)k * Lmax + c];
        if (!(rr == rr)) nan = true;
        r = fmax(r, rr / u);
        eta = fmax(eta, rr / (frob[k] * xn[(long)k * Lmax + c] + u));
    }
    resid[k] = nan ? INFINITY : r;
    iters[k] = it;
    const bool stop = nan || eta <= tol_be || r > 0.5 * prev[k] || it >= maxit;
    prev[k] = r;
    if (stop) { active[k] = 0; return; }
    for (int c = 0; c < Lmax; ++c) {
        const double rr = rn[(long)k * Lmax + c];
        inv[(long)k * Lmax + c] = rr > 0.0 ? 1.0 / rr : 0.0;
        scl[(long)k * Lmax + c] = rr;
    }
}


// R_b = U_b - T_b X_b in FP64 for at most RS_LC right-hand sides: the product is
// skinny, so it is a stream over T (HBM bound) rather than an MFMA GEMM.  One
// workgroup per RW * RPT rows of one matrix; a chunk of 64 rows of X is staged
// in LDS and read by broadcast; each thread keeps the L sums of its RPT rows
// (rows threadIdx.x + r RW, so every load of T stays coalesced) in registers
// and walks k in order (deterministic).  With RPT rows per thread one
// broadcast read of X(k, c) serves RPT loads of T: at L = 8 and above the
// broadcast reads would otherwise use as much LDS bandwidth as the stream
// over T uses HBM.  At L <= 2 (the GMRES operator) four rows per thread keep
// more loads of T in flight.  Matrices with active[b] == 0 are skipped.  RW rows
// (= threads) per workgroup: 64 for small matrices, so that there are enough
// workgroups, 256 otherwise.
constexpr int RS_KD = 4;
template <int LC, int RW, int RPT>
__global__ __launch_bounds__(RW) void resid_skinny_kernel(int n, int L, const double2* __restrict__ T, int ldt,
                                                            long sT, const double2* __restrict__ X, int ldx, long sX,
                                                            const double2* __restrict__ U, int ldu, long sU,
                                                            double2* __restrict__ R, int ldr, long sR,
                                                            const int* __restrict__ active)
{
    constexpr int KC = 64;
    __shared__ double2 xs[KC][LC];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int row0 = blockIdx.x * RW * RPT + threadIdx.x;
    const double2* Tb = T + b * sT;
    const double2* Xb = X + b * sX;
    bool ok[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) ok[r] = row0 + r * RW < n;
    double2 acc[RPT][LC];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < LC; ++c) acc[r][c] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < n; k0 += KC) {
        for (int e = threadIdx.x; e < KC * LC; e += RW) {
            const int kk = e % KC, c = e / KC;
            xs[kk][c] = (k0 + kk < n && c < L) ? Xb[(k0 + kk) + (long)c * ldx] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (ok[0]) {
            const int kend = min(KC, n - k0);
            const double2* tp = Tb + row0 + (long)k0 * ldt;
            // RS_KD columns of T in flight per thread; past kend the last
            // column is loaded again and multiplied by the zero rows of xs
            for (int kk0 = 0; kk0 < kend; kk0 += RS_KD) {
                double2 t[RS_KD][RPT];
#pragma unroll
                for (int u = 0; u < RS_KD; ++u) {
                    const long kc = min(kk0 + u, kend - 1);
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        t[u][r] = ok[r] ? tp[r * RW + kc * ldt] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < RS_KD; ++u) {
                    if (kk0 + u < kend) {
#pragma unroll
                        for (int c = 0; c < LC; ++c) {
                            const double2 x = xs[kk0 + u][c];
#pragma unroll
                            for (int r = 0; r < RPT; ++r) acc[r][c] = cfma(acc[r][c], t[u][r], x);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    double2* Rb = R + b * sR;
    const double2* Ub = U ? U + b * sU : nullptr;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        if (!ok[r]) continue;
        const int row = row0 + r * RW;
#pragma unroll
        for (int c = 0; c < LC; ++c)
            if (c < L) {
                if (!Ub) {  // R = T X
                    Rb[row + (long)c * ldr] = acc[r][c];
                } else {
                    const double2 u = Ub[row + (long)c * ldu];
                    Rb[row + (long)c * ldr] = make_double2(u.x - acc[r][c].x, u.y - acc[r][c].y);
                }
            }
    }
}

static dim3 ew_grid(long elems, int B) { return dim3((unsigned)((elems + EW_NT - 1) / EW_NT), B); }
// Ub_k (rows < n, columns < L) = U_q for point k = koff + blockIdx.y of instance blockIdx.z.
__global__ __launch_bounds__(EW_NT) void bcast_group_kernel(const RhsInstance* __restrict__ ins,
                                                             double2* __restrict__ Ub, int ldb, long sB)
{
    const RhsInstance in = ins[blockIdx.z];
    const int k = blockIdx.y;
    const long e = (long)blockIdx.x * EW_NT + threadIdx.x;
    if (k >= in.N || e >= (long)in.n * in.L) return;
    const int i = (int)(e % in.n), c = (int)(e / in.n);
    Ub[(in.koff + k) * sB + i + (long)c * ldb] = in.U[i + (long)c * in.ldu];
}

// S_q columns k L .. k L + L - 1 (rows < n) = X_(koff + k) for point k = blockIdx.y of instance blockIdx.z.
__global__ __launch_bounds__(EW_NT) void copy_out_group_kernel(const RhsInstance* __restrict__ ins,
                                                                const double2* __restrict__ Xb, int ldb, long sB)
{
    const RhsInstance in = ins[blockIdx.z];
    const int k = blockIdx.y;
    const long e = (long)blockIdx.x * EW_NT + threadIdx.x;
    if (k >= in.N || e >= (long)in.n * in.L) return;
    const int i = (int)(e % in.n), c = (int)(e / in.n);
    in.S[i + ((long)k * in.L + c) * in.lds] = Xb[(in.koff + k) * sB + i + (long)c * ldb];
}

hipError_t bcast_group(hipStream_t st, const RhsInstance* ins, int nins, int nmax, int Lmax, int Nmax,
                       double2* Ub, int ldb, long sB)
{
    const dim3 g((unsigned)(((long)nmax * Lmax + EW_NT - 1) / EW_NT), (unsigned)Nmax, (unsigned)nins);
    hipLaunchKernelGGL(bcast_group_kernel, g, dim3(EW_NT), 0, st, ins, Ub, ldb, sB);
    return hipGetLastError();
}

hipError_t copy_out_group(hipStream_t st, const RhsInstance* ins, int nins, int nmax, int Lmax, int Nmax,
                          const double2* Xb, int ldb, long sB)
{
    const dim3 g((unsigned)(((long)nmax * Lmax + EW_NT - 1) / EW_NT), (unsigned)Nmax, (unsigned)nins);
    hipLaunchKernelGGL(copy_out_group_kernel, g, dim3(EW_NT), 0, st, ins, Xb, ldb, sB);
    return hipGetLastError();
}


hipError_t pad_identity(hipStream_t st, float2* T64, double2* T128, int ld, long sT, int P, const int* nk, int M)
{
    // one thread per padding element of a matrix of a 64-wide size bucket (P - n < 64)
    const long cover = std::min((long)P * P, 128L * P);
    if (T64) hipLaunchKernelGGL(pad_identity_kernel<float2>, ew_grid(cover, M), dim3(EW_NT), 0, st, T64, ld, sT,
                                P, nk);
    if (T128) hipLaunchKernelGGL(pad_identity_kernel<double2>, ew_grid(cover, M), dim3(EW_NT), 0, st, T128, ld,
                                 sT, P, nk);
    return hipGetLastError();
}
hipError_t zero_c128(hipStream_t st, int n, int m, double2* X, int ldx, long sX, int B)
{
    hipLaunchKernelGGL(zero_c128_kernel, ew_grid((long)n * m, B), dim3(EW_NT), 0, st, n, m, X, ldx, sX);
    return hipGetLastError();
}
hipError_t zero_int(hipStream_t st, int* p, int n)
{
    hipLaunchKernelGGL(zero_int_kernel, dim3((n + EW_NT - 1) / EW_NT), dim3(EW_NT), 0, st, p, n);
    return hipGetLastError();
}
hipError_t ir_init(hipStream_t st, int M, const int* info, int* active, double* prev, double* resid, int* iters)
{
    hipLaunchKernelGGL(ir_init_kernel, dim3((M + EW_NT - 1) / EW_NT), dim3(EW_NT), 0, st, M, info, active, prev,
                       resid, iters);
    return hipGetLastError();
}
hipError_t ir_decide(hipStream_t st, int M, int Lmax, const double* rn, const double* xn, const double* un,
                     const double* frob, double tol_be, int it, int maxit, int* active, double* prev, double* resid,
                     int* iters, double* inv, double* scl)
{
    hipLaunchKernelGGL(ir_decide_kernel, dim3((M + EW_NT - 1) / EW_NT), dim3(EW_NT), 0, st, M, Lmax, rn, xn, un, frob,
                       tol_be, it, maxit, active, prev, resid, iters, inv, scl);
    return hipGetLastError();
}

hipError_t bcast_to_c64(hipStream_t st, int n, int L, const double2* U, int ldu, float2* D, int ldd, long sD, int B)
{
    hipLaunchKernelGGL(bcast_to_c64_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, U, ldu, D, ldd, sD);
    return hipGetLastError();
}
hipError_t bcast_c128(hipStream_t st, int n, int L, const double2* U, int ldu, double2* R, int ldr, long sR, int B)
{
    hipLaunchKernelGGL(bcast_c128_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, U, ldu, R, ldr, sR);
    return hipGetLastError();
}
hipError_t widen(hipStream_t st, int n, int L, const float2* D, int ldd, long sD, double2* X, int ldx, long sX, int B)
{
    hipLaunchKernelGGL(widen_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, D, ldd, sD, X, ldx, sX);
    return hipGetLastError();
}
hipError_t colnorms(hipStream_t st, int n, int L, const double2* X, int ldx, long sX, double* out, int B)
{
    hipLaunchKernelGGL(colnorm_kernel, dim3(L, B), dim3(EW_NT), 0, st, n, L, X, ldx, sX, out);
    return hipGetLastError();
}
hipError_t scale_narrow(hipStream_t st, int n, int L, const double2* R, int ldr, long sR, const double* inv,
                        float2* D, int ldd, long sD, const int* active, int B)
{
    hipLaunchKernelGGL(scale_narrow_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, R, ldr, sR, inv, D,
                       ldd, sD, active);
    return hipGetLastError();
}
hipError_t axpy_widen(hipStream_t st, int n, int L, const float2* D, int ldd, long sD, const double* scale,
                      double2* X, int ldx, long sX, const int* active, int B)
{
    hipLaunchKernelGGL(axpy_widen_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, D, ldd, sD, scale, X,
                       ldx, sX, active);
    return hipGetLastError();
}
hipError_t copy_c128(hipStream_t st, int n, int m, const double2* X, int ldx, long sX, double2* Y, int ldy, long sY,
                     int B)
{
    hipLaunchKernelGGL(copy_c128_kernel, ew_grid((long)n * m, B), dim3(EW_NT), 0, st, n, m, X, ldx, sX, Y, ldy, sY);
    return hipGetLastError();
}
hipError_t scale_cols(hipStream_t st, int n, int m, double2* X, int ldx, const double* s)
{
    hipLaunchKernelGGL(scale_cols_kernel, ew_grid((long)n * m, 1), dim3(EW_NT), 0, st, n, m, X, ldx, s);
    return hipGetLastError();
}


bool resid_skinny_ok(int L) { return L >= 1 && L <= 16; }

hipError_t resid_skinny(hipStream_t st, int n, int L, const double2* T, int ldt, long sT, const double2* X, int ldx,
                        long sX, const double2* U, int ldu, long sU, double2* R, int ldr, long sR, const int* active,
                        int B)
{
#define RS_L(LC, RW)                                                                                             \
    do {                                                                                                         \
        constexpr int RPT = (LC >= 8) ? 2 : (LC <= 2 ? 4 : 1);                                                                  \
        hipLaunchKernelGGL((resid_skinny_kernel<LC, RW, RPT>), dim3((unsigned)((n + RW * RPT - 1) / (RW * RPT)), \
                                                                    (unsigned)B),                               \
                           dim3(RW), 0, st, n, L, T, ldt, sT, X, ldx, sX, U, ldu, sU, R, ldr, sR, active);      \
    } while (0)
    const bool small = n <= 1024;
    if (L <= 2) {
        if (small) RS_L(2, 64); else RS_L(2, 256);
    } else if (L <= 4) {
        if (small) RS_L(4, 64); else RS_L(4, 256);
    } else if (L <= 8) {
        if (small) RS_L(8, 64); else RS_L(8, 256);
    } else {
        if (small) RS_L(16, 64); else RS_L(16, 256);
    }
#undef RS_L
    return hipGetLastError();
}

hipError_t narrow_real(hipStream_t st, int n, const double2* T, int ldt, long sT, float* Tr, int ldr, long sTr,
                       int B)
{
    hipLaunchKernelGGL(narrow_real_kernel, ew_grid((long)n * n, B), dim3(EW_NT), 0, st, n, T, ldt, sT, Tr, ldr, sTr);
    return hipGetLastError();
}
hipError_t scale_narrow_real(hipStream_t st, int n, int L, const double2* R, int ldr, long sR, const double* inv,
                             float* D, int ldd, long sD, const int* active, int B)
{
    hipLaunchKernelGGL(scale_narrow_real_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, R, ldr, sR, inv,
                       D, ldd, sD, active);
    return hipGetLastError();
}
hipError_t axpy_widen_real(hipStream_t st, int n, int L, const float* D, int ldd, long sD, const double* scale,
                           double2* X, int ldx, long sX, const int* active, int B)
{
    hipLaunchKernelGGL(axpy_widen_real_kernel, ew_grid((long)n * L, B), dim3(EW_NT), 0, st, n, L, D, ldd, sD, scale,
                       X, ldx, sX, active);
    return hipGetLastError();
}

}  // namespace rsrr
