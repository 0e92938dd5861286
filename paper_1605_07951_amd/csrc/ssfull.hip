// Kernels of SS-FULL on the projected NEP (Sec. 3.3 applied in RSRR Step 4):
// block Hankel assembly (eq. HH), the eigen-decomposition of the small
// reduced matrix (eq. A) and matrix 1-norms for the residuals.
#include "common.h"
#include "kernels.h"

namespace rsrr {

// H(bi*k + i, bj*k + j) = A_{bi+bj+shift}(i, j); moments stored contiguously
// (k x k each, ld k).
__global__ __launch_bounds__(256) void hankel_kernel(const double2* __restrict__ mom, int k, int K, int shift,
                                                      double2* __restrict__ H, int ldh)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const long Kk = (long)K * k;
    if (e >= Kk * Kk) return;
    const int r = (int)(e % Kk), cidx = (int)(e / Kk);
    const int bi = r / k, i = r % k, bj = cidx / k, j = cidx % k;
    H[r + (long)cidx * ldh] = mom[(long)(bi + bj + shift) * k * k + i + (long)j * k];
}

hipError_t hankel(hipStream_t st, const double2* mom, int k, int K, int shift, double2* H, int ldh)
{
    const long e = (long)K * k * K * k;
    hipLaunchKernelGGL(hankel_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, mom, k, K, shift, H, ldh);
    return hipGetLastError();
}

// Identity into the rows m..m+p-1 of an (m+p) x p matrix (and zero elsewhere below m).
__global__ __launch_bounds__(256) void eye_kernel(double2* __restrict__ X, int ldx, int r0, int p)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)p * p) return;
    const int i = (int)(e % p), j = (int)(e / p);
    X[(r0 + i) + (long)j * ldx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

hipError_t eye(hipStream_t st, double2* X, int ldx, int r0, int p)
{
    const long e = (long)p * p;
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, X, ldx, r0, p);
    return hipGetLastError();
}

// ||T_b||_1 (largest column sum of |t_ij|) for a batch of n x n matrices.
// Pass 1: one wave per column (coalesced along the column), each workgroup of
// four waves writes the largest of its four sums.  Pass 2: one workgroup per
// matrix takes the maximum of those partial results.
constexpr int N1_COLS = 4;

__global__ __launch_bounds__(256) void norm1_cols_kernel(const double2* __restrict__ T, int ld, long sT, int n,
                                                          double* __restrict__ part)
{
    __shared__ double red[N1_COLS];
    const int b = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = blockIdx.x * N1_COLS + wave;
    double s = 0.0;
    if (j < n) {
        const double2* col = T + b * sT + (long)j * ld;
        for (int i = lane; i < n; i += 64) {
            const double2 a = col[i];
            s += sqrt(a.x * a.x + a.y * a.y);
        }
    }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(long)b * gridDim.x + blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void norm1_max_kernel(const double* __restrict__ part, int G,
                                                         double* __restrict__ out)
{
    __shared__ double red[4];
    const int b = blockIdx.x;
    double m = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) m = fmax(m, part[(long)b * G + g]);
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[b] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

hipError_t norm1(hipStream_t st, const double2* T, int ld, long sT, int n, double* out, int B, double* part)
{
    const int G = (n + N1_COLS - 1) / N1_COLS;
    hipLaunchKernelGGL(norm1_cols_kernel, dim3(G, B), dim3(256), 0, st, T, ld, sT, n, part);
    hipLaunchKernelGGL(norm1_max_kernel, dim3(B), dim3(256), 0, st, part, G, out);
    return hipGetLastError();
}

int norm1_parts(int n) { return (n + N1_COLS - 1) / N1_COLS; }

// ---------------------------------------------------------------------------
// Eigenpairs of a small general complex matrix (n x n, column-major, ld n,
// n <= SMALL_EIG_MAX): Householder reduction to Hessenberg form, single-shift
// QR with Wilkinson shifts to the Schur form T = Z^H A Z, then eigenvectors of
// T by back substitution, b = Z y (unit 2-norm).  One workgroup of one wave.
// The Householder vector is formed on lane 0; every other step is spread over
// the 64 lanes: row and column updates of the reflections, and in each QR step
// the row pair (left rotation) and column pair (right rotation) of every Givens
// rotation.  The rotations of one QR step depend on each other and are applied
// in order, one barrier apart; all lanes compute the same rotation from the
// same entries, so the control flow is uniform.
// Work arrays (device): H (n*n), Z (n*n).  Outputs: lam (n), Bv (n*n).
// Dynamic LDS: n complex (reflector) + n complex + n real (rotations).
// status[0]: 0 ok, 1 QR did not converge.
// ---------------------------------------------------------------------------
constexpr int SMALL_EIG_MAX = 1024;
int small_eig_max() { return SMALL_EIG_MAX; }

RSRR_DEV double cabs_(double2 a) { return hypot(a.x, a.y); }
RSRR_DEV double2 cdiv_(double2 a, double2 b) { return cmul(a, crecip(b)); }
RSRR_DEV double2 csqrt_(double2 a)
{
    const double r = cabs_(a);
    if (r == 0.0) return make_double2(0.0, 0.0);
    double x = sqrt(0.5 * (r + fabs(a.x)));
    double y = a.y / (2.0 * x);
    if (a.x < 0.0) { const double t = fabs(y); y = (a.y >= 0 ? x : -x); x = t; }
    return make_double2(x, y);
}

// Givens rotation [c s; -conj(s) c] (c real) that zeroes y below x.
RSRR_DEV void givens_(double2 x, double2 y, double* cc, double2* ss)
{
    const double ax = cabs_(x), ay = cabs_(y);
    const double r = hypot(ax, ay);
    if (r == 0.0) { *cc = 1.0; *ss = make_double2(0.0, 0.0); }
    else if (ax == 0.0) { *cc = 0.0; *ss = make_double2(y.x / ay, -y.y / ay); }
    else {
        *cc = ax / r;
        const double2 ph = make_double2(x.x / ax, x.y / ax);
        *ss = cmul(ph, make_double2(y.x / r, -y.y / r));
    }
}

__global__ __launch_bounds__(64) void small_eig_kernel(const double2* __restrict__ A, int n, double2* __restrict__ H,
                                                        double2* __restrict__ Z, double2* __restrict__ lam,
                                                        double2* __restrict__ Bv, int* __restrict__ status)
{
    extern __shared__ double2 s_dyn[];
    double2* s_v = s_dyn;                      // n: Householder vector
    double2* s_sn = s_dyn + n;                 // n: rotation sines of one QR step
    double* s_cs = (double*)(s_dyn + 2 * n);   // n: rotation cosines
    __shared__ double s_beta;
    const int t = threadIdx.x;
#define HH(i, j) H[(i) + (long)(j) * n]
#define ZZ(i, j) Z[(i) + (long)(j) * n]
    for (long e = t; e < (long)n * n; e += 64) {
        H[e] = A[e];
        Z[e] = make_double2((e % n) == (e / n) ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // ---- Hessenberg reduction ----
    for (int kcol = 0; kcol + 2 < n; ++kcol) {
        if (t == 0) {
            double alpha2 = 0.0;
            for (int i = kcol + 1; i < n; ++i) { const double2 x = HH(i, kcol); alpha2 += x.x * x.x + x.y * x.y; }
            const double xn = sqrt(alpha2);
            const double2 x0 = HH(kcol + 1, kcol);
            const double ax0 = cabs_(x0);
            double beta = 0.0;
            if (xn > 0.0) {
                const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
                // v = x + ph*|x| e1, H = I - beta v v^H, beta = 2 / (v^H v)
                for (int i = kcol + 1; i < n; ++i) s_v[i - kcol - 1] = HH(i, kcol);
                s_v[0] = make_double2(x0.x + ph.x * xn, x0.y + ph.y * xn);
                double vv = 0.0;
                for (int i = 0; i < n - kcol - 1; ++i) vv += s_v[i].x * s_v[i].x + s_v[i].y * s_v[i].y;
                beta = vv > 0.0 ? 2.0 / vv : 0.0;
            }
            s_beta = beta;
        }
        __syncthreads();
        const double beta = s_beta;
        const int m = n - kcol - 1;
        if (beta != 0.0) {
            // H <- P H: columns j (each lane its own column)
            for (int j = t; j < n; j += 64) {
                double2 s = make_double2(0.0, 0.0);
                for (int i = 0; i < m; ++i) s = cfma_cj(s, s_v[i], HH(kcol + 1 + i, j));
                s.x *= beta; s.y *= beta;
                for (int i = 0; i < m; ++i) HH(kcol + 1 + i, j) = cfms(HH(kcol + 1 + i, j), s_v[i], s);
            }
            __syncthreads();
            // H <- H P and Z <- Z P: rows i
            for (int i = t; i < n; i += 64) {
                double2 s = make_double2(0.0, 0.0), sz = make_double2(0.0, 0.0);
                for (int l = 0; l < m; ++l) {
                    s = cfma(s, HH(i, kcol + 1 + l), s_v[l]);
                    sz = cfma(sz, ZZ(i, kcol + 1 + l), s_v[l]);
                }
                s.x *= beta; s.y *= beta; sz.x *= beta; sz.y *= beta;
                for (int l = 0; l < m; ++l) {
                    const double2 vc = cconj(s_v[l]);
                    HH(i, kcol + 1 + l) = cfms(HH(i, kcol + 1 + l), s, vc);
                    ZZ(i, kcol + 1 + l) = cfms(ZZ(i, kcol + 1 + l), sz, vc);
                }
            }
        }
        __syncthreads();
        for (int i = kcol + 2 + t; i < n; i += 64) HH(i, kcol) = make_double2(0.0, 0.0);
        __syncthreads();
    }
    // ---- shifted QR to Schur form ----
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, iter = 0, total = 0, bad = 0;
    while (hi > 0) {
        __syncthreads();
        // deflation search (every lane, same entries, same answer)
        int lo = hi;
        while (lo > 0) {
            const double s = cabs_(HH(lo, lo)) + cabs_(HH(lo - 1, lo - 1));
            if (cabs_(HH(lo, lo - 1)) <= eps * (s > 0 ? s : 1.0)) break;
            --lo;
        }
        __syncthreads();
        if (lo > 0 && t == 0) HH(lo, lo - 1) = make_double2(0.0, 0.0);
        if (lo == hi) { --hi; iter = 0; continue; }
        if (++total > 100 * n) { bad = 1; break; }
        ++iter;
        // Wilkinson shift from the trailing 2x2 of the active block
        const double2 a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi), c = HH(hi, hi - 1), d = HH(hi, hi);
        double2 mu;
        if (iter % 11 == 10) {
            mu = make_double2(d.x + 0.75 * cabs_(c), d.y);  // exceptional shift
        } else {
            const double2 hd = make_double2(0.5 * (a.x - d.x), 0.5 * (a.y - d.y));
            const double2 disc = csqrt_(cadd(cmul(hd, hd), cmul(b, c)));
            const double2 m1 = cadd(make_double2(0.5 * (a.x + d.x), 0.5 * (a.y + d.y)), disc);
            const double2 m2 = csub(make_double2(0.5 * (a.x + d.x), 0.5 * (a.y + d.y)), disc);
            mu = cabs_(csub(m1, d)) < cabs_(csub(m2, d)) ? m1 : m2;
        }
        __syncthreads();
        // explicit shifted QR step on the active block (full rows/columns for the Schur form)
        for (int i = lo + t; i <= hi; i += 64) HH(i, i) = csub(HH(i, i), mu);
        __syncthreads();
        for (int i = lo; i < hi; ++i) {
            double cc;
            double2 ss;
            givens_(HH(i, i), HH(i + 1, i), &cc, &ss);
            if (t == 0) { s_cs[i - lo] = cc; s_sn[i - lo] = ss; }
            __syncthreads();
            // rows i, i+1: [r_i; r_{i+1}] <- [c s; -conj(s) c] [r_i; r_{i+1}]
            for (int j = i + t; j < n; j += 64) {
                const double2 u = HH(i, j), v = HH(i + 1, j);
                HH(i, j) = cadd(make_double2(cc * u.x, cc * u.y), cmul(ss, v));
                HH(i + 1, j) = csub(make_double2(cc * v.x, cc * v.y), cmul(cconj(ss), u));
            }
            __syncthreads();
        }
        for (int i = lo; i < hi; ++i) {
            const double cc = s_cs[i - lo];
            const double2 ss = s_sn[i - lo];
            // columns i, i+1 <- columns * G^H : [c_i c_{i+1}] [c -s; conj(s) c]
            const int rmax = (i + 2 <= hi) ? i + 2 : hi;
            for (int r = t; r <= rmax; r += 64) {
                const double2 u = HH(r, i), v = HH(r, i + 1);
                HH(r, i) = cadd(make_double2(cc * u.x, cc * u.y), cmul(cconj(ss), v));
                HH(r, i + 1) = csub(make_double2(cc * v.x, cc * v.y), cmul(ss, u));
            }
            for (int r = t; r < n; r += 64) {
                const double2 u = ZZ(r, i), v = ZZ(r, i + 1);
                ZZ(r, i) = cadd(make_double2(cc * u.x, cc * u.y), cmul(cconj(ss), v));
                ZZ(r, i + 1) = csub(make_double2(cc * v.x, cc * v.y), cmul(ss, u));
            }
            __syncthreads();
        }
        for (int i = lo + t; i <= hi; i += 64) HH(i, i) = cadd(HH(i, i), mu);
    }
    __syncthreads();
    if (t == 0) status[0] = bad;
    for (int i = t; i < n; i += 64) lam[i] = HH(i, i);
    // ---- eigenvectors of T (back substitution), b_i = Z y, unit norm ----
    double tn = 0.0;
    for (long e = t; e < (long)n * n; e += 64) tn = fmax(tn, cabs_(H[e]));
    for (int o = 32; o >= 1; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o));
    const double small = fmax(tn, 1e-300) * 2.220446049250313e-16;
    for (int i = t; i < n; i += 64) {
        double2* y = Bv + (long)i * n;  // use the output column as scratch for y
        for (int j = 0; j < n; ++j) y[j] = make_double2(0.0, 0.0);
        y[i] = make_double2(1.0, 0.0);
        const double2 li = HH(i, i);
        for (int j = i - 1; j >= 0; --j) {
            double2 s = make_double2(0.0, 0.0);
            for (int l = j + 1; l <= i; ++l) s = cfma(s, HH(j, l), y[l]);
            double2 den = csub(HH(j, j), li);
            if (cabs_(den) < small) den = make_double2(small, 0.0);
            const double2 q = cdiv_(s, den);
            y[j] = make_double2(-q.x, -q.y);
        }
    }
    __syncthreads();
    for (int i = t; i < n; i += 64) {
        double2* y = Bv + (long)i * n;
        // b = Z y, computed from the top (y_j = 0 for j > i), written into H's
        // column i (T is no longer needed) and copied back scaled
        double nn = 0.0;
        for (int r = 0; r < n; ++r) {
            double2 s = make_double2(0.0, 0.0);
            for (int l = 0; l <= i; ++l) s = cfma(s, ZZ(r, l), y[l]);
            HH(r, i) = s;
            nn += s.x * s.x + s.y * s.y;
        }
        nn = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int r = 0; r < n; ++r) {
            const double2 s = HH(r, i);
            y[r] = make_double2(s.x * nn, s.y * nn);
        }
    }
#undef HH
#undef ZZ
}

hipError_t small_eig(hipStream_t st, const double2* A, int n, double2* H, double2* Z, double2* lam, double2* Bv,
                     int* status)
{
    if (n < 1 || n > SMALL_EIG_MAX) return hipErrorInvalidValue;
    const size_t lds = (size_t)n * (2 * sizeof(double2) + sizeof(double));
    hipLaunchKernelGGL(small_eig_kernel, dim3(1), dim3(64), lds, st, A, n, H, Z, lam, Bv, status);
    return hipGetLastError();
}

}  // namespace rsrr
