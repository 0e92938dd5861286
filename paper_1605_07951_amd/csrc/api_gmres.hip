// C ABI: resolvent sampling with an iterative solver (RSRR Step 2, eq. hatS,
// solved by flexible GMRES with reused LU factors).
//
// Sec. 4.3 leaves the linear solver of Step 2 to the host software and notes
// that for large boundary-element or finite-element models an iterative
// solver takes the place of a factorisation per point; Sec. 6 runs GMRES with
// a preconditioner for the largest example.  Here every sampling point k and
// probe column l is one system T(z_k) x = u_l.  The systems of a chunk of
// points run side by side, column c = b*L + l of an n x (B*L) block, each
// with its own Krylov basis (restarted flexible GMRES, right preconditioning).
// The preconditioner is the complex FP32 LU of T at a reference point; one
// factorisation serves every point assigned to that reference.  The operator,
// the Krylov vectors, the Arnoldi relation and the residuals are FP64: flexible
// GMRES keeps the preconditioned directions Z_j, so the attainable accuracy
// does not depend on the factors' precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

namespace {

static int ldp(int n) { return (n + 63) / 64 * 64; }
static size_t a256(size_t b) { return (b + 255) / 256 * 256; }

// Bump allocator over one workspace slot.
struct Carve {
    char* base = nullptr;
    size_t off = 0;
    template <typename T> T* take(size_t count)
    {
        T* p = (T*)(base + off);
        off += a256(count * sizeof(T));
        return p;
    }
};

struct EvPair {
    hipEvent_t a = nullptr, b = nullptr;
    EvPair() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    ~EvPair() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    float ms() { float t = 0.f; (void)hipEventElapsedTime(&t, a, b); return t; }
};

// Length of the K slices that split a contraction of length K over about 512
// workgroups when `tiles` output tiles alone would leave the chip idle (K
// itself: no split).  Slices are multiples of 64.
static int k_slice(long tiles, int K)
{
    const long S = std::max(1L, std::min(16L, (512 + tiles - 1) / tiles));
    const int Ks = (int)((K + S - 1) / S + 63) / 64 * 64;
    return std::min(Ks, K);
}
static int n_slices(int K, int Ks) { return (K + Ks - 1) / Ks; }

struct GmChunk {
    int B, C;                      // points, columns (B * L)
    int ldy, Kop, Kso;             // separable: stacked scaled copies (J*n rows), K-slice of the operator
    double2* P;                    // split-operator partial products (n_slices(Kop, Kso) blocks)
    double2 *V, *Z, *Y, *X;        // Krylov vectors, directions, scaled copies, iterate (ld = c.ld)
    float2 *D, *D2;                // complex FP32 preconditioner input / output
    double2 *part, *h, *Hc, *Rm, *g, *sn, *y, *coef;
    double *cs, *hn, *thr, *inv, *g0;
    int *done, *act, *kc, *steps, *ndone, *pidx;
    double2* T;                    // HELMHOLTZ: per-point FP64 matrices (null: generated on the fly)
    double2* zc;                   // HELMHOLTZ: the chunk's points (device)
    const CsrTerm* csr;            // SPARSE: device table of the term matrices
    int* bad;                      // SPARSE: bounds flag of that table
    void* tmp;                     // getrs scratch
};

}  // namespace

// T(z) Z for the columns of a chunk (FP64), into W.
static rsrr_status gm_apply(rsrr_ctx* c, const rsrr_nep* nep, int L, int ld, long sT, const GmChunk& k,
                            const double2* Zin, double2* W)
{
    const int n = nep->n;
    if (nep->kind == RSRR_T_SPARSE) {
        // sum_j f_j(z_point(c)) A_j Z(:, c), straight from the sparse rows
        RSRR_HIP(csr_apply(c->stream, n, nep->J, k.csr, k.coef, k.B, L, Zin, ld, W, ld, k.bad));
        return RSRR_OK;
    }
    if (nep->kind == RSRR_T_SEPARABLE) {
        // sum_j A_j (Z diag(f_j(z_point(c)))) = [A_0 .. A_{J-1}] [Z f_0; ..; Z f_{J-1}]: the terms lie
        // back to back (matrix j at column j*n of one n x J*n matrix), so this is one GEMM of depth
        // J*n over all columns, split into K slices whose partial products are summed after
        for (int j = 0; j < nep->J; ++j)
            RSRR_HIP(gm_point_scale(c->stream, n, k.C, L, Zin, ld, k.coef + (size_t)j * k.B, k.Y + (size_t)j * n,
                                    k.ldy));
        const double2* A = (const double2*)nep->A;
        const int S1 = k.Kop / k.Kso, r1 = k.Kop - S1 * k.Kso;
        const long sP = (long)ld * k.C;
        if (S1 == 1 && r1 == 0) {
            RSRR_HIP(zgemm(c->stream, 0, 0, n, k.C, k.Kop, 1.0, A, nep->lda, 0, k.Y, k.ldy, 0, 0.0, W, ld, 0, 1));
            return RSRR_OK;
        }
        if (S1 > 0)
            RSRR_HIP(zgemm(c->stream, 0, 0, n, k.C, k.Kso, 1.0, A, nep->lda, (long)k.Kso * nep->lda, k.Y, k.ldy,
                           k.Kso, 0.0, k.P, ld, sP, S1));
        if (r1 > 0)
            RSRR_HIP(zgemm(c->stream, 0, 0, n, k.C, r1, 1.0, A + (size_t)S1 * k.Kso * nep->lda, nep->lda, 0,
                           k.Y + (size_t)S1 * k.Kso, k.ldy, 0, 0.0, k.P + (size_t)S1 * sP, ld, 0, 1));
        RSRR_HIP(gm_sum_c128(c->stream, n, k.C, k.P, ld, sP, S1 + (r1 > 0), W, ld));
    } else if (!k.T) {
        RSRR_HIP(helm_apply(c->stream, n, L, nep->points, nep->w, k.zc, Zin, ld, (long)ld * L, W, ld, (long)ld * L,
                            k.B));
    } else if (resid_skinny_ok(L)) {
        RSRR_HIP(resid_skinny(c->stream, n, L, k.T, ld, sT, Zin, ld, (long)ld * L, nullptr, 0, 0, W, ld, (long)ld * L,
                              nullptr, k.B));
    } else {
        RSRR_HIP(zgemm(c->stream, 0, 0, n, L, n, 1.0, k.T, ld, sT, Zin, ld, (long)ld * L, 0.0, W, ld, (long)ld * L,
                       k.B));
    }
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_sample_gmres(rsrr_ctx* c, const rsrr_nep* nep, int N, const double* z, int nref,
                                         const double* zref, const int* ref, const double* Up, int L, int ldu,
                                         double tol, int restart, int max_iters, int flags, double* Sp, int lds,
                                         rsrr_gmres_info* info)
{
    if (!c) return -1;
    if (!nep || nep->n < 1 || nep->n > 8192) return -2;
    if (nep->kind == RSRR_T_SEPARABLE) {
        if (nep->J < 1 || nep->J > 64 || !nep->A || nep->lda < nep->n || !nep->terms) return -2;
    } else if (nep->kind == RSRR_T_HELMHOLTZ) {
        if (!nep->points || !(nep->w > 0)) return -2;
    } else if (nep->kind == RSRR_T_SPARSE) {
        if (!csr_nep_ok(nep)) return -2;
    } else {
        return -2;
    }
    if (N < 1) return -3;
    if (!z) return -4;
    if (nref < 1) return -5;
    if (!zref) return -6;
    if (ref)
        for (int k = 0; k < N; ++k)
            if (ref[k] < 0 || ref[k] >= nref) return -7;
    if (!Up) return -8;
    if (L < 1) return -9;
    if (ldu < nep->n) return -10;
    if (!(tol > 0.0 && tol < 1.0)) return -11;
    if (restart < 1 || restart > gm_max_restart()) return -12;
    if (max_iters < 1) return -13;
    if (flags & ~RSRR_GMRES_MATRIX_FREE) return -14;
    if (!Sp) return -15;
    if (lds < nep->n) return -16;
    RSRR_HIP(hipSetDevice(c->device));
    EvPair all;
    RSRR_HIP(hipEventRecord(all.a, c->stream));
    for (double& t : c->timings) t = 0.0;

    const int n = nep->n, M = restart;
    const int ld = ldp(n);
    const long sT = (long)ld * n;
    const double2* U = (const double2*)Up;
    double2* S = (double2*)Sp;

    // ---- reference of every point, processing order grouped by reference ----
    std::vector<zd> zp(N), zr(nref);
    for (int k = 0; k < N; ++k) zp[k] = zd(z[2 * k], z[2 * k + 1]);
    for (int r = 0; r < nref; ++r) zr[r] = zd(zref[2 * r], zref[2 * r + 1]);
    std::vector<int> rk(N);
    for (int k = 0; k < N; ++k) {
        if (ref) { rk[k] = ref[k]; continue; }
        int best = 0;
        for (int r = 1; r < nref; ++r)
            if (std::abs(zp[k] - zr[r]) < std::abs(zp[k] - zr[best])) best = r;
        rk[k] = best;
    }
    std::vector<int> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rk[a] < rk[b]; });
    std::vector<int> slot(nref, -1), used;
    for (int k : order)
        if (slot[rk[k]] < 0) { slot[rk[k]] = (int)used.size(); used.push_back(rk[k]); }
    const int nf = (int)used.size();

    CsrDev csrd;  // SPARSE: the term table on the device (uploaded with the references)
    // ---- complex FP32 LU of T at the used references ----
    const int nb = std::min(std::max(c->nb_c64, MIN_NB), max_panel<float>());
    const int np = perm_panels(n);
    const long sInv = (long)((n + nb - 1) / nb) * 2 * nb * nb;
    const long sPerm = (long)np * 2 * MAX_NB;
    float2* Tf = (float2*)ws_get(c, WS_GMF, (size_t)nf * sT * 8);
    size_t fw = a256((size_t)nf * n * 4) + a256((size_t)nf * sPerm * 8) +
                a256((size_t)nf * 4) + a256((size_t)nf * sInv * 8) + a256((size_t)nf * nb * n * 8);
    Carve fc{(char*)ws_get(c, WS_GMW, fw)};
    if (!Tf || !fc.base) return RSRR_ENOMEM;
    LUWork w;
    w.ipiv = fc.take<int>((size_t)nf * n); w.sP = n;
    w.perm = fc.take<int2>((size_t)nf * sPerm); w.sPerm = sPerm;
    w.info = fc.take<int>(nf);
    w.inv = fc.take<float2>((size_t)nf * sInv); w.sInv = sInv;
    w.tmp = fc.take<float2>((size_t)nf * nb * n); w.sTmp = (long)nb * n;
    {
        EvPair ev;
        RSRR_HIP(hipEventRecord(ev.a, c->stream));
        const long nparts = ((long)n * n + 255) / 256;
        double* frobp = (double*)ws_get(c, WS_FROBP, (size_t)nf * nparts * 8);
        double* frob = (double*)ws_get(c, WS_FROB, (size_t)nf * 8);
        if (!frobp || !frob) return RSRR_ENOMEM;
        if (nep->kind == RSRR_T_SEPARABLE || nep->kind == RSRR_T_SPARSE) {
            double2* coef = (double2*)ws_get(c, WS_COEF, (size_t)nep->J * nf * 16);
            if (!coef) return RSRR_ENOMEM;
            std::vector<double2> cf((size_t)nep->J * nf);
            for (int j = 0; j < nep->J; ++j)
                for (int f = 0; f < nf; ++f) {
                    const zd v = term_eval(nep->terms[j], zr[used[f]]);
                    cf[(size_t)j * nf + f] = make_double2(v.real(), v.imag());
                }
            RSRR_HIP(hipMemcpyAsync(coef, cf.data(), cf.size() * 16, hipMemcpyHostToDevice, c->stream));
            if (nep->kind == RSRR_T_SEPARABLE) {
                RSRR_HIP(assemble_separable(c->stream, n, nep->J, (const double2*)nep->A, nep->lda, coef, nf, Tf, ld,
                                            sT, nullptr, 0, 0, frobp, frob));
            } else {
                // the references' FP64 matrices from the sparse rows (scratch), narrowed into the LU input;
                // the bounds of every row are checked here, before any operator application
                double2* T128 = (double2*)ws_get(c, WS_GMT, (size_t)nf * sT * 16);
                if (!T128) return RSRR_ENOMEM;
                RSRR_TRY(csr_upload(c, nep, csrd));
                RSRR_HIP(assemble_sparse(c->stream, n, nep->J, csrd.terms, coef, nf, Tf, ld, sT, T128, ld, sT, frobp,
                                         frob, csrd.bad));
                RSRR_TRY(csr_check(c, csrd));
            }
        } else {
            double2* zdev = (double2*)ws_get(c, WS_Z, (size_t)nf * 16);
            if (!zdev) return RSRR_ENOMEM;
            std::vector<double2> zz(nf);
            for (int f = 0; f < nf; ++f) zz[f] = make_double2(zr[used[f]].real(), zr[used[f]].imag());
            RSRR_HIP(hipMemcpyAsync(zdev, zz.data(), (size_t)nf * 16, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(assemble_helmholtz(c->stream, n, nep->points, nep->w, zdev, nf, Tf, ld, sT, nullptr, 0, 0, frobp,
                                        frob));
        }
        RSRR_HIP(hipMemsetAsync(w.info, 0, (size_t)nf * 4, c->stream));
        RSRR_HIP(getrf_batched<float>(c->stream, Tf, sT, ld, n, nb, w, nf));
        std::vector<int> hinfo(nf);
        RSRR_HIP(hipMemcpyAsync(hinfo.data(), w.info, (size_t)nf * 4, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipEventRecord(ev.b, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        c->timings[0] += ev.ms();
        for (int f = 0; f < nf; ++f) {
            if (hinfo[f] < 0) return RSRR_ENAN;
            if (hinfo[f] > 0) return RSRR_ESINGULAR;
        }
    }
    // A reference that serves several points is applied as an explicit inverse
    // (one complex FP32 GEMM per application instead of a chain of n/nb
    // triangular steps); the inverse costs about as much as 4n/(3L') solves.
    const bool use_inv = N >= 4 * nf;
    float2* Pinv = nullptr;
    if (use_inv) {
        EvPair ev;
        RSRR_HIP(hipEventRecord(ev.a, c->stream));
        Pinv = (float2*)ws_get(c, WS_GMI, (size_t)nf * sT * 8);
        if (!Pinv) return RSRR_ENOMEM;
        RSRR_HIP(gm_eye_c64(c->stream, n, Pinv, ld, sT, nf));
        RSRR_HIP(getrs_batched<float>(c->stream, Tf, sT, ld, n, nb, w, Pinv, sT, ld, n, nf));
        RSRR_HIP(hipEventRecord(ev.b, c->stream));
        RSRR_HIP(hipEventSynchronize(ev.b));
        c->timings[0] += ev.ms();
    }

    // ---- probe norms ----
    double* unrm = (double*)ws_get(c, WS_NORM, (size_t)L * 8);
    if (!unrm) return RSRR_ENOMEM;
    RSRR_HIP(colnorms(c->stream, n, L, U, ldu, 0, unrm, 1));
    std::vector<double> un(L);
    RSRR_HIP(hipMemcpyAsync(un.data(), unrm, (size_t)L * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));

    // ---- chunk size from the memory budget ----
    const int ns = gm_slices(n);
    const size_t per_col = (size_t)(2 * M + 3) * ld * 16 + (size_t)ld * 16 +
                           ((size_t)ns * (M + 1) * 16 + (size_t)(M + 1) * 16 * 3 + (size_t)M * M * 16 +
                            (size_t)M * 40 + 64) + (size_t)nb * 8 +
                           (size_t)(nep->kind == RSRR_T_SEPARABLE ? nep->J * n : 0) * 16 + (size_t)16 * ld * 24;
    size_t budget = c->ws_budget;
    if (!budget) {
        size_t fr = 0, tot = 0;
        RSRR_HIP(hipMemGetInfo(&fr, &tot));
        budget = fr / 2;
    }
    // Helmholtz operator: the points' FP64 matrices are assembled once per chunk, unless asked
    // not to or unless they would take more than half of the budget (then entries are generated
    // inside every application)
    const bool helm = nep->kind == RSRR_T_HELMHOLTZ;
    const bool mfree = helm && ((flags & RSRR_GMRES_MATRIX_FREE) || (size_t)N * sT * 16 > budget / 2);
    const size_t per_pt = (helm && !mfree ? (size_t)sT * 16 + (((size_t)n * n + 255) / 256) * 8 : 0) +
                          (size_t)nb * n * 8 + (size_t)std::max(nep->J, 1) * 16 + 64;
    int Bmax = (int)std::min<size_t>((size_t)N, std::max<size_t>(1, budget / (per_col * L + per_pt)));
    Bmax = std::max(1, std::min(Bmax, 65535));  // points per chunk ride on a grid dimension

    std::vector<int> pit(N, 0), prs(N, 0), pconv(N, 1);
    std::vector<double> pres(N, 0.0);
    bool any_nconv = false;
    float t_op = 0.f, t_pc = 0.f, t_it = 0.f;

    for (int p0 = 0; p0 < N; p0 += Bmax) {
        GmChunk k;
        k.B = std::min(Bmax, N - p0);
        k.C = k.B * L;
        const int C = k.C;
        const size_t vb = (size_t)ld * C;  // elements per n x C block
        // runs of points with the same reference (consecutive factor slots)
        std::vector<int> run0, runf;
        for (int b = 0; b < k.B; ++b) {
            const int f = slot[rk[order[p0 + b]]];
            if (run0.empty() || runf.back() != f) { run0.push_back(b); runf.push_back(f); }
        }
        const int nrun = (int)run0.size();
        run0.push_back(k.B);
        bool equal = true;
        for (int r = 1; r < nrun; ++r)
            if (run0[r + 1] - run0[r] != run0[1] - run0[0]) equal = false;
        const int maxrun = [&] { int m = 0; for (int r = 0; r < nrun; ++r) m = std::max(m, run0[r + 1] - run0[r]); return m; }();
        const long sTmp = (long)nb * std::max(n, maxrun * L);

        // Krylov workspace
        // split contractions: the separable operator (depth J*n) and the explicit-inverse
        // preconditioner (depth n per reference group)
        const bool sep = nep->kind == RSRR_T_SEPARABLE;
        k.ldy = sep ? nep->J * n : ld;
        k.Kop = sep ? nep->J * n : n;
        k.Kso = sep ? k_slice((long)((n + 63) / 64) * ((C + 63) / 64), k.Kop) : k.Kop;
        const int Sop = sep ? n_slices(k.Kop, k.Kso) : 0;
        const int bn = maxrun * L <= 32 ? 32 : (maxrun * L <= 64 ? 64 : 128);
        const int Kpc = use_inv ? k_slice((long)((n + 127) / 128) * ((maxrun * L + bn - 1) / bn), n) : n;
        const int Spc = use_inv ? n_slices(n, Kpc) : 0;
        const size_t ybytes = sep ? (size_t)k.ldy * C * 16 : vb * 16;
        const size_t kbytes = a256((size_t)(M + 1) * vb * 16) + a256((size_t)M * vb * 16) + a256(ybytes) +
                              a256(vb * 16) + a256(vb * 8) * 2 + a256((size_t)(equal ? nrun : 1) * sTmp * 8) +
                              a256((size_t)(Sop > 1 ? Sop : 0) * vb * 16) + a256((size_t)(Spc > 1 ? Spc : 0) * vb * 8);
        Carve kc{(char*)ws_get(c, WS_GMK, kbytes)};
        if (!kc.base) return RSRR_ENOMEM;
        k.V = kc.take<double2>((size_t)(M + 1) * vb);
        k.Z = kc.take<double2>((size_t)M * vb);
        k.Y = kc.take<double2>(ybytes / 16);
        k.X = kc.take<double2>(vb);
        k.D = kc.take<float2>(vb);
        k.D2 = kc.take<float2>(vb);
        k.tmp = kc.take<float2>((size_t)(equal ? nrun : 1) * sTmp);
        k.P = kc.take<double2>((size_t)(Sop > 1 ? Sop : 0) * vb);
        float2* Pp = kc.take<float2>((size_t)(Spc > 1 ? Spc : 0) * vb);
        const size_t sbytes = a256((size_t)ns * (M + 1) * C * 16) + a256((size_t)(M + 1) * C * 16) * 3 +
                              a256((size_t)M * M * C * 16) + a256((size_t)M * C * 16) * 2 + a256((size_t)M * C * 8) +
                              a256((size_t)C * 8) * 4 + a256((size_t)C * 4) * 4 + a256(64) +
                              a256((size_t)k.B * 4) + a256((size_t)std::max(nep->J, 1) * k.B * 16) +
                              a256((size_t)k.B * 16);
        Carve sc{(char*)ws_get(c, WS_GMS, sbytes)};
        if (!sc.base) return RSRR_ENOMEM;
        k.part = sc.take<double2>((size_t)ns * (M + 1) * C);
        k.h = sc.take<double2>((size_t)(M + 1) * C);
        k.Hc = sc.take<double2>((size_t)(M + 1) * C);
        k.g = sc.take<double2>((size_t)(M + 1) * C);
        k.Rm = sc.take<double2>((size_t)M * M * C);
        k.sn = sc.take<double2>((size_t)M * C);
        k.y = sc.take<double2>((size_t)M * C);
        k.cs = sc.take<double>((size_t)M * C);
        k.hn = sc.take<double>(C);
        k.thr = sc.take<double>(C);
        k.inv = sc.take<double>(C);
        k.g0 = sc.take<double>(C);
        k.done = sc.take<int>(C);
        k.act = sc.take<int>(C);
        k.kc = sc.take<int>(C);
        k.steps = sc.take<int>(C);
        k.ndone = sc.take<int>(16);
        k.pidx = sc.take<int>(k.B);
        k.coef = sc.take<double2>((size_t)std::max(nep->J, 1) * k.B);
        k.zc = sc.take<double2>(k.B);
        k.T = nullptr;
        k.csr = csrd.terms;
        k.bad = csrd.bad;

        std::vector<int> hp(k.B);
        for (int b = 0; b < k.B; ++b) hp[b] = order[p0 + b];
        RSRR_HIP(hipMemcpyAsync(k.pidx, hp.data(), (size_t)k.B * 4, hipMemcpyHostToDevice, c->stream));
        {
            EvPair ev;
            RSRR_HIP(hipEventRecord(ev.a, c->stream));
            if (nep->kind != RSRR_T_HELMHOLTZ) {
                std::vector<double2> cf((size_t)nep->J * k.B);
                for (int j = 0; j < nep->J; ++j)
                    for (int b = 0; b < k.B; ++b) {
                        const zd v = term_eval(nep->terms[j], zp[hp[b]]);
                        cf[(size_t)j * k.B + b] = make_double2(v.real(), v.imag());
                    }
                RSRR_HIP(hipMemcpyAsync(k.coef, cf.data(), cf.size() * 16, hipMemcpyHostToDevice, c->stream));
                RSRR_HIP(hipStreamSynchronize(c->stream));
            } else if (mfree) {
                std::vector<double2> zz(k.B);
                for (int b = 0; b < k.B; ++b) zz[b] = make_double2(zp[hp[b]].real(), zp[hp[b]].imag());
                RSRR_HIP(hipMemcpyAsync(k.zc, zz.data(), (size_t)k.B * 16, hipMemcpyHostToDevice, c->stream));
                RSRR_HIP(hipStreamSynchronize(c->stream));
            } else {
                k.T = (double2*)ws_get(c, WS_GMT, (size_t)k.B * sT * 16);
                if (!k.T) return RSRR_ENOMEM;
                std::vector<zd> zb(k.B);
                for (int b = 0; b < k.B; ++b) zb[b] = zp[hp[b]];
                double* frob = (double*)ws_get(c, WS_FROB, (size_t)k.B * 8);
                if (!frob) return RSRR_ENOMEM;
                const rsrr_status st = assemble_c128(c, nep, zb.data(), k.B, k.T, ld, sT, frob);
                if (st) return st;
            }
            RSRR_HIP(hipEventRecord(ev.b, c->stream));
            RSRR_HIP(hipEventSynchronize(ev.b));
            c->timings[0] += ev.ms();
        }

        // x = 0, r = u
        RSRR_HIP(zero_c128(c->stream, n, C, k.X, ld, 0, 1));
        RSRR_HIP(bcast_c128(c->stream, n, L, U, ldu, k.V, ld, (long)ld * L, k.B));
        std::vector<int> hdone(C, 0), hsteps(C), tot(C, 0), hact(C), ncyc(C, 0);
        std::vector<double> beta(C), rel(C, 0.0), hbuf(4 * (size_t)C);
        int used_steps = 0;
        for (;;) {
            // true residual norms of the current iterate
            RSRR_HIP(colnorms(c->stream, n, C, k.V, ld, 0, k.hn, 1));
            RSRR_HIP(hipMemcpyAsync(beta.data(), k.hn, (size_t)C * 8, hipMemcpyDeviceToHost, c->stream));
            RSRR_HIP(hipStreamSynchronize(c->stream));
            int nact = 0;
            for (int col = 0; col < C; ++col) {
                const double u = un[col % L];
                if (!(beta[col] == beta[col])) return RSRR_ENAN;
                rel[col] = u > 0.0 ? beta[col] / u : beta[col];
                hdone[col] = rel[col] <= tol;
                nact += !hdone[col];
            }
            if (nact == 0) break;
            if (used_steps >= max_iters) break;
            const int mc = std::min(M, max_iters - used_steps);
            for (int col = 0; col < C; ++col) {
                hact[col] = !hdone[col];
                hbuf[col] = hdone[col] ? 0.0 : 1.0 / beta[col];                       // inv0
                hbuf[(size_t)C + col] = hdone[col] ? 0.0 : beta[col];                  // g0
                hbuf[2 * (size_t)C + col] = 0.5 * tol * (un[col % L] > 0.0 ? un[col % L] : 1.0);  // thr
            }
            RSRR_HIP(hipMemcpyAsync(k.inv, hbuf.data(), (size_t)C * 8, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(hipMemcpyAsync(k.g0, hbuf.data() + C, (size_t)C * 8, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(hipMemcpyAsync(k.thr, hbuf.data() + 2 * (size_t)C, (size_t)C * 8, hipMemcpyHostToDevice,
                                    c->stream));
            RSRR_HIP(hipMemcpyAsync(k.done, hdone.data(), (size_t)C * 4, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(hipMemcpyAsync(k.act, hact.data(), (size_t)C * 4, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(zero_int(c->stream, k.kc, C));
            RSRR_HIP(zero_int(c->stream, k.ndone, 1));
            RSRR_HIP(gm_scale(c->stream, n, C, k.inv, k.V, ld));
            RSRR_HIP(gm_g0(c->stream, C, k.g0, k.g));
            const int done0 = C - nact;
            int jend = mc;
            EvPair evi;
            RSRR_HIP(hipEventRecord(evi.a, c->stream));
            for (int j = 0; j < mc; ++j) {
                double2* Vj = k.V + (size_t)j * vb;
                double2* W = k.V + (size_t)(j + 1) * vb;
                double2* Zj = k.Z + (size_t)j * vb;
                EvPair e1, e2;
                // Z_j = P^-1 V_j (complex FP32 factors of the point's reference)
                RSRR_HIP(hipEventRecord(e1.a, c->stream));
                RSRR_HIP(gm_narrow(c->stream, n, C, Vj, ld, k.D, ld));
                float2* Dz = k.D;
                bool widened = false;
                if (use_inv && Spc > 1) {
                    // Z_j = P^-1 V_j, each reference group's product split into K slices
                    const int S1 = n / Kpc, r1 = n - S1 * Kpc;
                    for (int r = 0; r < nrun; ++r) {
                        const int cols = (run0[r + 1] - run0[r]) * L;
                        const size_t o = (size_t)run0[r] * L * ld;
                        const float2* Pr = Pinv + runf[r] * sT;
                        if (S1 > 0)
                            RSRR_HIP(cgemm(c->stream, n, cols, Kpc, 1.f, Pr, ld, (long)Kpc * ld, k.D + o, ld, Kpc, 0.f,
                                           Pp + o, ld, (long)vb, S1));
                        if (r1 > 0)
                            RSRR_HIP(cgemm(c->stream, n, cols, r1, 1.f, Pr + (size_t)S1 * Kpc * ld, ld, 0,
                                           k.D + o + (size_t)S1 * Kpc, ld, 0, 0.f, Pp + (size_t)S1 * vb + o, ld, 0,
                                           1));
                    }
                    RSRR_HIP(gm_sum_widen(c->stream, n, C, Pp, ld, (long)vb, Spc, Zj, ld));
                    widened = true;
                } else if (use_inv) {
                    Dz = k.D2;
                    if (equal) {
                        const int rl = run0[1] - run0[0];
                        RSRR_HIP(cgemm(c->stream, n, rl * L, n, 1.f, Pinv + runf[0] * sT, ld, sT, k.D, ld,
                                       (long)ld * rl * L, 0.f, k.D2, ld, (long)ld * rl * L, nrun));
                    } else {
                        for (int r = 0; r < nrun; ++r) {
                            const int rl = run0[r + 1] - run0[r];
                            const size_t o = (size_t)run0[r] * L * ld;
                            RSRR_HIP(cgemm(c->stream, n, rl * L, n, 1.f, Pinv + runf[r] * sT, ld, sT, k.D + o, ld, 0,
                                           0.f, k.D2 + o, ld, 0, 1));
                        }
                    }
                } else if (equal) {
                    const int rl = run0[1] - run0[0];
                    LUWork wr = w;
                    const int f0 = runf[0];
                    wr.ipiv = w.ipiv + (long)f0 * n; wr.perm = w.perm + f0 * sPerm;
                    wr.info = w.info + f0; wr.inv = (float2*)w.inv + f0 * sInv; wr.tmp = k.tmp; wr.sTmp = sTmp;
                    RSRR_HIP(getrs_batched<float>(c->stream, Tf + f0 * sT, sT, ld, n, nb, wr, k.D, (long)ld * rl * L,
                                                  ld, rl * L, nrun));
                } else {
                    for (int r = 0; r < nrun; ++r) {
                        const int rl = run0[r + 1] - run0[r], f = runf[r];
                        LUWork wr = w;
                        wr.ipiv = w.ipiv + (long)f * n; wr.perm = w.perm + f * sPerm;
                        wr.info = w.info + f; wr.inv = (float2*)w.inv + f * sInv; wr.tmp = k.tmp; wr.sTmp = sTmp;
                        RSRR_HIP(getrs_batched<float>(c->stream, Tf + f * sT, sT, ld, n, nb, wr,
                                                      k.D + (size_t)run0[r] * L * ld, (long)ld * rl * L, ld, rl * L,
                                                      1));
                    }
                }
                if (!widened) RSRR_HIP(gm_widen(c->stream, n, C, Dz, ld, Zj, ld));
                RSRR_HIP(hipEventRecord(e1.b, c->stream));
                // W = T Z_j
                RSRR_HIP(hipEventRecord(e2.a, c->stream));
                rsrr_status st = gm_apply(c, nep, L, ld, sT, k, Zj, W);
                if (st) return st;
                RSRR_HIP(hipEventRecord(e2.b, c->stream));
                // two classical Gram-Schmidt passes, then the norm and the rotation
                RSRR_HIP(gm_orth_pass(c->stream, n, C, j + 1, k.V, ld, (long)vb, W, ld, k.done, k.part, k.h, k.Hc, 1));
                RSRR_HIP(gm_orth_pass(c->stream, n, C, j + 1, k.V, ld, (long)vb, W, ld, k.done, k.part, k.h, k.Hc, 0));
                RSRR_HIP(colnorms(c->stream, n, C, W, ld, 0, k.hn, 1));
                RSRR_HIP(gm_givens(c->stream, C, j, M, k.Hc, k.hn, k.thr, k.cs, k.sn, k.g, k.Rm, k.done, k.kc, k.inv,
                                   k.ndone));
                RSRR_HIP(gm_scale(c->stream, n, C, k.inv, W, ld));
                int nd = 0;
                RSRR_HIP(hipMemcpyAsync(&nd, k.ndone, 4, hipMemcpyDeviceToHost, c->stream));
                RSRR_HIP(hipStreamSynchronize(c->stream));
                t_pc += e1.ms();
                t_op += e2.ms();
                if (done0 + nd >= C) { jend = j + 1; break; }
            }
            // x += Z y, then the true residual r = u - T x
            RSRR_HIP(gm_solve(c->stream, C, M, jend, k.Rm, k.g, k.act, k.kc, k.y, k.steps));
            RSRR_HIP(gm_combine(c->stream, n, C, jend, k.Z, ld, (long)vb, k.y, k.X, ld));
            RSRR_HIP(hipEventRecord(evi.b, c->stream));
            RSRR_HIP(hipMemcpyAsync(hsteps.data(), k.steps, (size_t)C * 4, hipMemcpyDeviceToHost, c->stream));
            {
                EvPair e2;
                RSRR_HIP(hipEventRecord(e2.a, c->stream));
                rsrr_status st = gm_apply(c, nep, L, ld, sT, k, k.X, k.V);
                if (st) return st;
                RSRR_HIP(hipEventRecord(e2.b, c->stream));
                RSRR_HIP(gm_resid(c->stream, n, C, L, U, ldu, k.V, ld));
                RSRR_HIP(hipStreamSynchronize(c->stream));
                t_op += e2.ms();
            }
            t_it += evi.ms();
            for (int col = 0; col < C; ++col) { tot[col] += hsteps[col]; ncyc[col] += hact[col]; }
            used_steps += jend;
        }
        RSRR_HIP(gm_scatter(c->stream, n, C, L, k.X, ld, k.pidx, S, lds));
        for (int b = 0; b < k.B; ++b) {
            const int p = hp[b];
            int it = 0, ok = 1, cy = 0;
            double r = 0.0;
            for (int l = 0; l < L; ++l) {
                const int col = b * L + l;
                it = std::max(it, tot[col]);
                cy = std::max(cy, ncyc[col]);
                r = std::max(r, rel[col]);
                if (!(rel[col] <= tol)) ok = 0;
            }
            pit[p] = it;
            prs[p] = std::max(0, cy - 1);
            pconv[p] = ok;
            pres[p] = r;
            if (!ok) any_nconv = true;
        }
    }
    RSRR_HIP(hipEventRecord(all.b, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    c->timings[1] = t_op;
    c->timings[2] = t_pc;
    c->timings[3] = t_it;
    c->timings[4] = all.ms();
    if (info)
        for (int p = 0; p < N; ++p) {
            info[p].iters = pit[p];
            info[p].restarts = prs[p];
            info[p].converged = pconv[p];
            info[p].ref = rk[p];
            info[p].resid = pres[p];
            info[p].matrix_free = mfree ? 1 : 0;
            info[p].pad = 0;
        }
    return any_nconv ? RSRR_ENOTCONV : RSRR_OK;
}
