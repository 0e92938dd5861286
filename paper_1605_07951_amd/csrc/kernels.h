// Host-side entry points of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace rsrr {

// Widest LU panel (columns): permutation slots and scratch are sized for it.
// The LDS triangle of the solve kernel holds 128 columns for complex FP32 and
// 64 for complex FP64 (panel widths are capped accordingly).
constexpr int MAX_NB = 128;
template <typename R> constexpr int max_panel() { return sizeof(R) == 4 ? 128 : 64; }
// Panel slots of the per-matrix permutation store (enough for the narrowest panel, 64).
// Panel widths of the LU are at least MIN_NB columns; storage per panel is
// sized for that many panels.
constexpr int MIN_NB = 32;
inline int perm_panels(int n) { return (n + MIN_NB - 1) / MIN_NB; }

// C = beta*C + alpha*A*B, complex single on v_mfma_f32_32x32x2f32.
// tag 1 launches a separately named instance (the LU trailing update).
hipError_t cgemm(hipStream_t st, int M, int N, int K, float alpha,
                 const float2* A, int lda, long sA, const float2* B, int ldb, long sB,
                 float beta, float2* C, int ldc, long sC, int batch, int tag = 0);

// Workgroup tiles of the complex FP32 trailing update (tag 1) that the ragged
// batch's autotuner chooses from (all 4 waves per workgroup, two LDS stages):
// 3M 128x64 (the default), 3M 64x64, 4M 128x128, 4M 64x64.  The choice holds
// for the calling host thread until changed.
enum { UPD_TILE_3M_128x64 = 0, UPD_TILE_3M_64x64 = 1, UPD_TILE_4M_128x128 = 2, UPD_TILE_4M_64x64 = 3,
       UPD_TILE_COUNT = 4 };
void set_update_tile(int t);
int get_update_tile();
const char* update_tile_name(int t);

// C = beta*C + alpha*op(A)*op(B), complex double on v_mfma_f64_16x16x4f64;
// op = conjugate transpose when the flag is set.
hipError_t zgemm(hipStream_t st, int opA, int opB, int M, int N, int K, double alpha,
                 const double2* A, int lda, long sA, const double2* B, int ldb, long sB,
                 double beta, double2* C, int ldc, long sC, int batch, int tag = 0);

// Event recorder around the LU trailing-update launches (optional).
struct UpdateRecorder {
    hipEvent_t* ev = nullptr;   // pool of 2*cap events
    int cap = 0;
    int used = 0;               // pairs recorded
    double flops = 0.0;         // algorithmic flops of the recorded launches (8 m n k)
    double bytes = 0.0;         // algorithmic bytes: C (m x n) read and written, A (m x k) and B (k x n) read once
    double* lflops = nullptr;   // per recorded launch: its algorithmic flops
    unsigned char* lmask = nullptr;  // per recorded launch: 1 when it ran on the CU-masked stream
    long dropped = 0;           // launches beyond the pool (not timed)
};

// Workspace of the batched LU (per-matrix strides in elements).
//  ipiv  : n ints                          (stride sP)
//  perm  : perm_panels(n)*2*MAX_NB int2     (stride sPerm), composed interchanges per panel
//  info  : 1 int, zero on entry            (getrf semantics; < 0: NaN/Inf pivot)
//  inv   : FP32 paths, and FP64 when given together with tmp (the diagonal blocks are
//          then solved by products with their inverses, as in FP32):
//          panels*2*nb*nb elements (stride sInv), L11^-1, U11^-1
//  tmp   : with inv: nb*max(n, nrhs) elements (stride sTmp)
//  active: optional per-matrix mask; rec: optional trailing-update event recorder
//  pair  : FP32 paths, optional: (ldpair*2*nb + nb*nb) elements per matrix (stride sPair,
//          ldpair >= n): two panels then share one trailing update of depth 2nb
struct LUWork {
    int* ipiv = nullptr; long sP = 0;
    int2* perm = nullptr; long sPerm = 0;
    int* info = nullptr;
    void* inv = nullptr; long sInv = 0;
    void* tmp = nullptr; long sTmp = 0;
    const int* active = nullptr;
    UpdateRecorder* rec = nullptr;
    hipEvent_t first_panel = nullptr;  // recorded once the first panel and its row block are done
    void* pair = nullptr; long sPair = 0; int ldpair = 0;
    // look-ahead (FP32 paths with pairs): a second pair buffer (same stride), a side
    // stream and two events; the next pair's panels are then factored on `side`
    // while the trailing update of the current pair runs on the main stream.
    void* pair2 = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    // optional: a stream whose CU mask leaves some CUs to `side`; the bulk of each
    // overlapped update runs on it (event ev_c joins it back)
    hipStream_t upd = nullptr;
    hipEvent_t ev_c = nullptr;
    int la_cols = 0;                   // columns of each overlapped update on `upd` (0: all)
};
// Elements per matrix of the pair buffer for n x n matrices and panel width nb.
inline long lu_pair_elems(int n, int nb, int ldpair) { return (long)ldpair * 2 * nb + (long)nb * nb; }

// Blocked LU with partial pivoting of `batch` n x n matrices (stride sA).
template <typename R>
hipError_t getrf_batched(hipStream_t st, typename cpx<R>::T* A, long sA, int lda, int n, int nb, const LUWork& w,
                         int batch);

// X <- T^-1 X for the factors of getrf_batched (same nb and workspace).
template <typename R>
hipError_t getrs_batched(hipStream_t st, const typename cpx<R>::T* LU, long sLU, int lda, int n, int nb,
                         const LUWork& w, typename cpx<R>::T* X, long sX, int ldx, int nrhs, int batch);

// getrs_batched<float> for right-hand-side blocks that fit in LDS (n * nrhs * 8 B
// <= 128 KB, nrhs <= 16): one workgroup per matrix runs every panel's forward and
// backward step out of LDS (the factor columns stream from memory once).  The
// factors are those of getrf_batched<float> (same nb and workspace).
bool getrs_lds_ok(int n, int nrhs);
hipError_t getrs_lds_batched(hipStream_t st, const float2* LU, long sLU, int lda, int n, int nb, const LUWork& w,
                             float2* X, long sX, int ldx, int nrhs, int batch);

// The same for real FP32 matrices (a real NEP at real points); workspace as
// for complex FP32 (inv/tmp hold real values, half the bytes used).
hipError_t getrf_real_batched(hipStream_t st, float* A, long sA, int lda, int n, int nb, const LUWork& w, int batch);
hipError_t getrs_real_batched(hipStream_t st, const float* LU, long sLU, int lda, int n, int nb, const LUWork& w,
                              float* X, long sX, int ldx, int nrhs, int batch);

// C = beta*C + alpha*A*B, real single on v_mfma_f32_32x32x2f32.
hipError_t sgemm(hipStream_t st, int M, int N, int K, float alpha, const float* A, int lda, long sA,
                 const float* B, int ldb, long sB, float beta, float* C, int ldc, long sC, int batch, int tag = 0);

// ---- assembly (assemble.hip) ----
// T64/T128 may be null (not written); batch strides s64/s128 in elements.
// frob_part: B * ceil(n*n/256) doubles of scratch; frob: B doubles (||T_k||_F).
hipError_t assemble_separable(hipStream_t st, int n, int J, const double2* A, int lda, const double2* coef, int B,
                              float2* T64, int ld64, long s64, double2* T128, int ld128, long s128,
                              double* frob_part, double* frob);
hipError_t assemble_helmholtz(hipStream_t st, int n, const double* pts, double w, const double2* z, int B,
                              float2* T64, int ld64, long s64, double2* T128, int ld128, long s128,
                              double* frob_part, double* frob);
hipError_t helmholtz_taylor(hipStream_t st, int n, const double* pts, double w, double gre, double gim, int p,
                            double2* Tp, int ld);
// Taylor terms p0 .. p0+G-1 of the Helmholtz matrix about gamma, term p0+g at Tp + g*sT.
hipError_t helmholtz_taylor_range(hipStream_t st, int n, const double* pts, double w, double gre, double gim, int p0,
                                  int G, double2* Tp, int ld, long sT);

// A sparse term matrix (compressed sparse rows, device arrays; device table
// entry): row i holds entries rp[i] .. rp[i+1]-1, entry e at column ci[e].
struct CsrTerm {
    const int* rp; const int* ci; const double2* v; int nnz; int pad;
};
// T_k = sum_j coef[j B + k] A_j for B points, A_j = terms[j] sparse (J terms):
// T128 (required) is formed in FP64 (zeroed, then each row's entries summed in
// by the thread that owns the row), then T64 (may be null) and the norms are
// taken from it.  *bad (device int) is set when a row range or column index is
// out of bounds (that entry is skipped).
hipError_t assemble_sparse(hipStream_t st, int n, int J, const CsrTerm* terms, const double2* coef, int B,
                           float2* T64, int ld64, long s64, double2* T128, int ld128, long s128,
                           double* frob_part, double* frob, int* bad);
// T_k += sum_j coef[j B + k] A_j into dense T_k (sparse.hip)
hipError_t csr_scatter(hipStream_t st, int n, int J, const CsrTerm* terms, const double2* coef, int B, double2* T,
                       int ld, long sT, int* bad);
// Y(:, c) = sum_j coef[j B + c / L] A_j X(:, c) for the C = B L columns (FP64);
// entries out of bounds are skipped and set *bad.
hipError_t csr_apply(hipStream_t st, int n, int J, const CsrTerm* terms, const double2* coef, int B, int L,
                     const double2* X, int ldx, double2* Y, int ldy, int* bad);

// One separable instance of a ragged batch's size bucket (device table entry):
// terms A (J matrices n x n, ld lda, consecutive), coefficient rows at
// coef + coff ([J][N], point-fastest), points = bucket matrices koff .. koff+N-1.
struct SepInstance {
    const double2* A; long coff; long koff; int lda, J, n, N;
};
// The whole bucket (all instances separable, J <= assemble_max_terms()) in one
// launch plus one launch for the norms; nk: per-matrix order (M matrices),
// frob_part: M * ceil(nmax^2/256) doubles.
hipError_t assemble_separable_group(hipStream_t st, const SepInstance* ins, int nins, int nmax, int Nmax,
                                    const double2* coef, int P, int M, const int* nk, float2* T64, long s64,
                                    double2* T128, long s128, double* frob_part, double* frob);
int assemble_max_terms();
// Right-hand sides and results of a bucket's instances in one launch each:
// Ub_k = [U_q; 0] for the points k of instance q, and S_q columns from X_k.
struct RhsInstance {
    const double2* U; double2* S; long koff; int ldu, lds, n, L, N;
};
hipError_t bcast_group(hipStream_t st, const RhsInstance* ins, int nins, int nmax, int Lmax, int Nmax,
                       double2* Ub, int ldb, long sB);
hipError_t copy_out_group(hipStream_t st, const RhsInstance* ins, int nins, int nmax, int Lmax, int Nmax,
                          const double2* Xb, int ldb, long sB);

// ---- element-wise helpers (ir.hip) ----
hipError_t bcast_to_c64(hipStream_t st, int n, int L, const double2* U, int ldu, float2* D, int ldd, long sD, int B);
hipError_t bcast_c128(hipStream_t st, int n, int L, const double2* U, int ldu, double2* R, int ldr, long sR, int B);
hipError_t widen(hipStream_t st, int n, int L, const float2* D, int ldd, long sD, double2* X, int ldx, long sX, int B);
hipError_t colnorms(hipStream_t st, int n, int L, const double2* X, int ldx, long sX, double* out, int B);
// R_b = U_b - T_b X_b (FP64) for L <= 16 columns, matrices with active[b] == 0
// skipped (active may be null); U null gives R_b = T_b X_b.  resid_skinny_ok(L)
// tells whether it applies.
bool resid_skinny_ok(int L);
// Real FP32 corrections for a real NEP at real points: Tr = (float) Re T;
// D = (float)(Re R * inv) (inv may be null: 1); X = (D, 0) (scale null) or
// Re X += scale * D.
hipError_t narrow_real(hipStream_t st, int n, const double2* T, int ldt, long sT, float* Tr, int ldr, long sTr,
                       int B);
hipError_t scale_narrow_real(hipStream_t st, int n, int L, const double2* R, int ldr, long sR, const double* inv,
                             float* D, int ldd, long sD, const int* active, int B);
hipError_t axpy_widen_real(hipStream_t st, int n, int L, const float* D, int ldd, long sD, const double* scale,
                           double2* X, int ldx, long sX, const int* active, int B);
hipError_t resid_skinny(hipStream_t st, int n, int L, const double2* T, int ldt, long sT, const double2* X, int ldx,
                        long sX, const double2* U, int ldu, long sU, double2* R, int ldr, long sR, const int* active,
                        int B);
hipError_t scale_narrow(hipStream_t st, int n, int L, const double2* R, int ldr, long sR, const double* inv,
                        float2* D, int ldd, long sD, const int* active, int B);
hipError_t axpy_widen(hipStream_t st, int n, int L, const float2* D, int ldd, long sD, const double* scale,
                      double2* X, int ldx, long sX, const int* active, int B);
hipError_t copy_c128(hipStream_t st, int n, int m, const double2* X, int ldx, long sX, double2* Y, int ldy, long sY,
                     int B);
hipError_t scale_cols(hipStream_t st, int n, int m, double2* X, int ldx, const double* s);
hipError_t pad_identity(hipStream_t st, float2* T64, double2* T128, int ld, long sT, int P, const int* nk, int M);
hipError_t zero_c128(hipStream_t st, int n, int m, double2* X, int ldx, long sX, int B);
hipError_t zero_int(hipStream_t st, int* p, int n);
hipError_t ir_init(hipStream_t st, int M, const int* info, int* active, double* prev, double* resid, int* iters);
hipError_t ir_decide(hipStream_t st, int M, int Lmax, const double* rn, const double* xn, const double* un,
                     const double* frob, double tol_be, int it, int maxit, int* active, double* prev, double* resid,
                     int* iters, double* inv, double* scl);

// ---- block one-sided Jacobi SVD (basis.hip) ----
int jacobi_blocks(int p);  // number of column blocks (even) for p columns
hipError_t jacobi_round(hipStream_t st, double2* A, int lda, int m, int m_apply, int p, int round, int inner,
                        double tol, double zthr2, double* offmax, void* work);
size_t jacobi_work_bytes(int m, int m_apply, int p);  // bytes of `work` for jacobi_round
hipError_t gather_scale(hipStream_t st, const double2* A, int lda, int m, const int* order, const double* inv,
                        double2* Q, int ldq, int k);
hipError_t gaussian(hipStream_t st, double2* X, int n, int m, int ld, unsigned long long seed);
hipError_t bcgs2(hipStream_t st, double2* Y, int ld, int n, int m, void* work, double* n0);
size_t bcgs2_work_bytes(int n, int m);

// ---- flexible GMRES over many columns (gmres.hip) ----
// C independent systems side by side (column c of an n x C block belongs to
// point c / L); per-column small arrays are index-major ([i * C + c]).
int gm_slices(int n);        // row slices of the column kernels (partials per column)
int gm_max_restart();        // longest restart cycle
hipError_t gm_point_scale(hipStream_t st, int n, int C, int L, const double2* Z, int ldz, const double2* coef,
                          double2* Y, int ldy);
hipError_t gm_narrow(hipStream_t st, int n, int C, const double2* V, int ldv, float2* D, int ldd);
hipError_t gm_widen(hipStream_t st, int n, int C, const float2* D, int ldd, double2* Z, int ldz);
hipError_t gm_resid(hipStream_t st, int n, int C, int L, const double2* U, int ldu, double2* V, int ldv);
hipError_t gm_scale(hipStream_t st, int n, int C, const double* s, double2* X, int ldx);
hipError_t gm_scatter(hipStream_t st, int n, int C, int L, const double2* X, int ldx, const int* idx, double2* S,
                      int lds);
// One classical Gram-Schmidt pass of W against V_0..V_{j1-1}: h = V^H W,
// W -= V h; Hc = h (first) or Hc += h.  part: gm_slices(n) * j1 * C values.
hipError_t gm_orth_pass(hipStream_t st, int n, int C, int j1, const double2* V, int ldv, long sV, double2* W, int ldw,
                        const int* done, double2* part, double2* h, double2* Hc, int first);
hipError_t gm_givens(hipStream_t st, int C, int j, int M, const double2* Hc, const double* hn, const double* thr,
                     double* cs, double2* sn, double2* g, double2* Rm, int* done, int* kc, double* inv, int* ndone);
hipError_t gm_solve(hipStream_t st, int C, int M, int jend, const double2* Rm, const double2* g, const int* active,
                    const int* kc, double2* y, int* steps);
hipError_t gm_combine(hipStream_t st, int n, int C, int k, const double2* Z, int ldz, long sZ, const double2* y,
                      double2* X, int ldx);
hipError_t gm_g0(hipStream_t st, int C, const double* g0, double2* g);
hipError_t gm_eye_c64(hipStream_t st, int n, float2* A, int ld, long sA, int B);
// W_b = T(z_b) Z_b for the Helmholtz single-layer matrix of the points, entries generated in FP64
// on the fly (matrix-free); any L (columns in groups of 16).
hipError_t helm_apply(hipStream_t st, int n, int L, const double* pts, double w, const double2* z, const double2* Z,
                      int ldz, long sZ, double2* W, int ldw, long sW, int B);
// Sums of the S slices of a split contraction (slice s at P + s*sP): Z = (c128) sum P_s, W = sum P_s.
hipError_t gm_sum_widen(hipStream_t st, int n, int C, const float2* P, int ldp, long sP, int S, double2* Z, int ldz);
hipError_t gm_sum_c128(hipStream_t st, int n, int C, const double2* P, int ldp, long sP, int S, double2* W, int ldw);

// ---- SS-FULL helpers (ssfull.hip) ----
hipError_t hankel(hipStream_t st, const double2* mom, int k, int K, int shift, double2* H, int ldh);
hipError_t eye(hipStream_t st, double2* X, int ldx, int r0, int p);
hipError_t norm1(hipStream_t st, const double2* T, int ld, long sT, int n, double* out, int B, double* part);
int norm1_parts(int n);  // doubles of `part` per matrix
// Eigenpairs of an n x n complex matrix, n <= small_eig_max().
hipError_t small_eig(hipStream_t st, const double2* A, int n, double2* H, double2* Z, double2* lam, double2* Bv,
                     int* status);
int small_eig_max();

}  // namespace rsrr
