// C ABI: context, contour nodes and resolvent sampling (RSRR Steps 1-2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

void* ws_get(rsrr_ctx* c, int s, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (c->ws_size[s] >= bytes) return c->ws[s];
    if (c->ws[s]) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->ws[s]);
        c->ws[s] = nullptr;
        c->ws_size[s] = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    c->ws[s] = p;
    c->ws_size[s] = bytes;
    return p;
}

void rec_collect(rsrr_ctx* c)
{
    if (!c->rec.ev) return;
    for (int i = 0; i < c->rec.used; ++i) {
        (void)hipEventSynchronize(c->rec.ev[2 * i + 1]);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->rec.ev[2 * i], c->rec.ev[2 * i + 1]) == hipSuccess) {
            c->upd_ms += ms;
            if (c->rec.lmask && c->rec.lmask[i]) {
                c->upd_ms_masked += ms;
                c->upd_flops_masked += c->rec.lflops[i];
            }
        }
    }
    c->upd_launches += c->rec.used;
    c->upd_flops += c->rec.flops;
    c->upd_bytes += c->rec.bytes;
    c->upd_dropped += c->rec.dropped;
    c->rec.used = 0;
    c->rec.flops = 0.0;
    c->rec.bytes = 0.0;
    c->rec.dropped = 0;
}

zd term_eval(const rsrr_term& t, zd z)
{
    zd v(t.c_re, t.c_im);
    if (t.p) v *= std::pow(z - zd(t.z0_re, t.z0_im), t.p);
    if (t.tau != 0.0) v *= std::exp(-t.tau * z);
    if (t.q) v /= std::pow(z - zd(t.s_re, t.s_im), t.q);
    return v;
}

extern "C" {

const char* rsrr_version(void) { return "rsrr-mi355x 0.1 (gfx950)"; }

rsrr_status rsrr_create(rsrr_ctx** ctx, int device, void* stream)
{
    if (!ctx) return -1;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return RSRR_EDEVICE;
    if (device < 0 || device >= ndev) return -2;
    RSRR_HIP(hipSetDevice(device));
    rsrr_ctx* c = new rsrr_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (const char* e = std::getenv("RSRR_WS_BUDGET_MB")) c->ws_budget = (size_t)std::strtoull(e, nullptr, 10) << 20;
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) { delete c; return RSRR_EDEVICE; }
    if (const char* e = std::getenv("RSRR_LOOKAHEAD")) c->lookahead = std::atoi(e) != 0;
    if (const char* e = std::getenv("RSRR_LA_CUS")) c->la_cus = std::atoi(e);
    if (const char* e = std::getenv("RSRR_LA_COLS")) c->la_cols = std::atoi(e);
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->la, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->la_a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->la_b, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->la_c, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->offset, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return RSRR_EDEVICE;
    }
    if (noalloc_scratch_setup(device, &c->noalloc_scratch) != RSRR_OK) {
        rsrr_destroy(c);
        return RSRR_EDEVICE;
    }
    *ctx = c;
    return RSRR_OK;
}

rsrr_status rsrr_options_init(rsrr_options* opt)
{
    if (!opt) return -1;
    const rsrr_ctx d;
    *opt = rsrr_options{};
    opt->size = sizeof(rsrr_options);
    opt->version = RSRR_OPTIONS_VERSION;
    opt->ir_max_iters = d.ir_max_iters;
    opt->ir_max_iters_batched = d.ir_max_iters_batched;
    opt->basis_sketch_max = d.basis_sketch_max;
    opt->ir_tol = d.ir_tol;
    opt->fallback_resid = d.fallback_resid;
    opt->delta = d.delta;
    opt->tol_gap = d.tol_gap;
    return RSRR_OK;
}

// A field is read when it lies wholly inside the caller's `size` bytes.
#define RSRR_OPT_HAS(opt, f) ((opt)->size >= offsetof(rsrr_options, f) + sizeof((opt)->f))

rsrr_status rsrr_set_options(rsrr_ctx* c, const rsrr_options* opt)
{
    if (!c) return -1;
    if (!opt || !RSRR_OPT_HAS(opt, version)) return -2;
    rsrr_ctx n;  // validated copy of the option fields
    n.ir_max_iters = RSRR_OPT_HAS(opt, ir_max_iters) ? opt->ir_max_iters : c->ir_max_iters;
    n.ir_max_iters_batched = RSRR_OPT_HAS(opt, ir_max_iters_batched) ? opt->ir_max_iters_batched : c->ir_max_iters_batched;
    n.basis_sketch_max = RSRR_OPT_HAS(opt, basis_sketch_max) ? opt->basis_sketch_max : c->basis_sketch_max;
    n.ir_tol = RSRR_OPT_HAS(opt, ir_tol) ? opt->ir_tol : c->ir_tol;
    n.fallback_resid = RSRR_OPT_HAS(opt, fallback_resid) ? opt->fallback_resid : c->fallback_resid;
    n.delta = RSRR_OPT_HAS(opt, delta) ? opt->delta : c->delta;
    n.tol_gap = RSRR_OPT_HAS(opt, tol_gap) ? opt->tol_gap : c->tol_gap;
    if (n.ir_max_iters < 0 || n.ir_max_iters > 100) return -3;
    if (n.ir_max_iters_batched < 0 || n.ir_max_iters_batched > 16) return -4;
    if (n.basis_sketch_max < 8) return -5;
    if (!(n.ir_tol > 0)) return -6;
    if (!(n.fallback_resid > 0 && n.fallback_resid < 1)) return -7;
    if (!(n.delta > 0 && n.delta < 1)) return -8;
    if (!(n.tol_gap > 0)) return -9;
    c->ir_max_iters = n.ir_max_iters;
    c->ir_max_iters_batched = n.ir_max_iters_batched;
    c->basis_sketch_max = n.basis_sketch_max;
    c->ir_tol = n.ir_tol;
    c->fallback_resid = n.fallback_resid;
    c->delta = n.delta;
    c->tol_gap = n.tol_gap;
    return RSRR_OK;
}

rsrr_status rsrr_get_options(rsrr_ctx* c, rsrr_options* opt)
{
    if (!c) return -1;
    if (!opt || !RSRR_OPT_HAS(opt, version)) return -2;
    rsrr_options full;
    rsrr_options_init(&full);
    full.ir_max_iters = c->ir_max_iters;
    full.ir_max_iters_batched = c->ir_max_iters_batched;
    full.basis_sketch_max = c->basis_sketch_max;
    full.ir_tol = c->ir_tol;
    full.fallback_resid = c->fallback_resid;
    full.delta = c->delta;
    full.tol_gap = c->tol_gap;
    const size_t bytes = std::min<size_t>((size_t)opt->size, sizeof(rsrr_options));
    const unsigned long long keep = opt->size;
    std::memcpy(opt, &full, bytes);
    opt->size = keep;
    return RSRR_OK;
}

rsrr_status rsrr_destroy(rsrr_ctx* c)
{
    if (!c) return -1;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    batched_release(c);
    for (int s = 0; s < WS_COUNT; ++s)
        if (c->ws[s]) (void)hipFree(c->ws[s]);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->la) (void)hipStreamSynchronize(c->la), (void)hipStreamDestroy(c->la);
    if (c->la_a) (void)hipEventDestroy(c->la_a);
    if (c->la_b) (void)hipEventDestroy(c->la_b);
    if (c->la_c) (void)hipEventDestroy(c->la_c);
    masked_stream_release(c);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->join) (void)hipEventDestroy(c->join);
    if (c->offset) (void)hipEventDestroy(c->offset);
    if (c->rec.ev) {
        for (int i = 0; i < 2 * c->rec.cap; ++i) (void)hipEventDestroy(c->rec.ev[i]);
        delete[] c->rec.ev;
        delete[] c->rec.lflops;
        delete[] c->rec.lmask;
    }
    delete c;
    return RSRR_OK;
}

rsrr_status rsrr_contour(double gre, double gim, double a, double b, int N, double* z, double* w)
{
    if (!(a > 0)) return -3;
    if (!(b > 0)) return -4;
    if (N < 1) return -5;
    if (!z) return -6;
    for (int j = 0; j < N; ++j) {
        const double t = 2.0 * M_PI * (j + 0.5) / N;
        z[2 * j] = gre + a * std::cos(t);
        z[2 * j + 1] = gim + b * std::sin(t);
        if (w) {
            w[2 * j] = -a * std::sin(t) / N;
            w[2 * j + 1] = b * std::cos(t) / N;
        }
    }
    return RSRR_OK;
}

rsrr_status rsrr_update_stats(rsrr_ctx* c, int enable, int reset, double* out)
{
    if (!c) return -1;
    RSRR_HIP(hipSetDevice(c->device));
    if (enable && !c->rec.ev) {
        const int cap = 8192;
        c->rec.ev = new hipEvent_t[2 * cap];
        for (int i = 0; i < 2 * cap; ++i) RSRR_HIP(hipEventCreate(&c->rec.ev[i]));
        c->rec.lflops = new double[cap];
        c->rec.lmask = new unsigned char[cap];
        c->rec.cap = cap;
    }
    c->rec_on = enable != 0;
    if (reset) {
        c->upd_ms = c->upd_flops = c->upd_bytes = 0.0;
        c->upd_ms_masked = c->upd_flops_masked = 0.0;
        c->upd_launches = c->upd_dropped = 0;
    }
    if (out) {
        out[0] = (double)c->upd_launches;
        out[1] = c->upd_ms;
        out[2] = c->upd_flops;
        out[3] = (double)c->upd_dropped;
        out[4] = c->upd_bytes;
        out[5] = c->upd_ms_masked;
        out[6] = c->upd_flops_masked;
        hipDeviceProp_t prop;
        const int ncu = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.multiProcessorCount : 0;
        out[7] = ncu > 0 && c->la_cus > 0 && c->la_cus < ncu ? (double)(ncu - c->la_cus) / ncu : 1.0;
    }
    return RSRR_OK;
}

rsrr_status rsrr_last_timings(rsrr_ctx* c, double* t)
{
    if (!c) return -1;
    if (!t) return -2;
    for (int i = 0; i < 5; ++i) t[i] = c->timings[i];
    return RSRR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// sampling driver
// ---------------------------------------------------------------------------

namespace {

static int ld_pad(int n) { return (n + 63) / 64 * 64; }

struct PhaseTimer {
    rsrr_ctx* c;
    hipEvent_t a, b;
    double* acc;
    PhaseTimer(rsrr_ctx* c_, double* acc_) : c(c_), acc(acc_)
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, c->stream);
    }
    void stop()
    {
        (void)hipEventRecord(b, c->stream);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        *acc += ms;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        a = b = nullptr;
    }
    ~PhaseTimer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct SampleBufs {
    void* Tlu; double2* Tres; int* ipiv; int2* perm; int* info; double2* coef; double* frobp;
    double* frob; float2* D64; double2* R; double* norms; int* active; double2* zdev; void* inv; void* tmp;
    void* pair; void* pair2;
    hipStream_t la, upd; hipEvent_t la_a, la_b, la_c;
    int la_cols;
    int ld, np, nb; long sT, sP, sPerm, nparts, sInv, sTmp, sPair;
    LUWork lu(const int* act, UpdateRecorder* rec) const
    {
        LUWork w;
        w.ipiv = ipiv; w.sP = sP; w.perm = perm; w.sPerm = sPerm; w.info = info;
        w.inv = inv; w.sInv = sInv; w.tmp = tmp; w.sTmp = sTmp; w.active = act; w.rec = rec;
        w.pair = pair; w.sPair = sPair; w.ldpair = ld;
        w.pair2 = pair2; w.side = la; w.ev_a = la_a; w.ev_b = la_b; w.upd = upd; w.ev_c = la_c;
        w.la_cols = la_cols;
        return w;
    }
};

// Per-point bytes of the sampling buffers.
static size_t per_point_bytes(int n, int L, int prec)
{
    const size_t ld = ld_pad(n);
    const size_t np = perm_panels(n);
    size_t b = ld * n * 16;                         // FP64 copy for residuals
    b += ld * n * (prec == RSRR_PREC_C128 ? 16 : 8);  // LU input
    b += (size_t)n * 4 + np * 2 * MAX_NB * 8 + 16;
    b += ((size_t)n * n + 255) / 256 * 8 + 8;
    b += (size_t)ld * L * (8 + 16) + (size_t)L * 16;
    if (prec != RSRR_PREC_C128) {
        b += (size_t)np * 2 * 128 * 128 * 8 / 2;          // diagonal-block inverses (nb = 128: n/128 panels)
        b += (size_t)128 * std::max(n, L) * 8;            // scratch rows
        b += (size_t)lu_pair_elems(n, 128, (int)ld) * 8 * 2;  // paired trailing updates (two for the look-ahead)
    }
    return b;
}

static rsrr_status alloc_bufs(rsrr_ctx* c, int n, int L, int J, int prec, int B, SampleBufs& s)
{
    s.ld = ld_pad(n);
    s.np = perm_panels(n);
    // the real FP32 path (R32_IR) uses the complex FP32 layout with real elements (half the bytes)
    const bool fp32 = prec != RSRR_PREC_C128;
    s.nb = fp32 ? std::min(c->nb_c64, max_panel<float>()) : std::min(c->nb_c128, max_panel<double>());
    s.sInv = fp32 ? (long)((n + s.nb - 1) / s.nb) * 2 * s.nb * s.nb : 0;
    s.sTmp = fp32 ? (long)s.nb * std::max(n, L) : 0;
    s.inv = fp32 ? ws_get(c, WS_B0, (size_t)B * s.sInv * 8) : nullptr;
    s.tmp = fp32 ? ws_get(c, WS_B1, (size_t)B * s.sTmp * 8) : nullptr;
    s.sPair = fp32 ? lu_pair_elems(n, max_panel<float>(), s.ld) : 0;  // any panel width the LU clamps to
    const bool la = fp32 && c->lookahead;
    s.pair = fp32 ? ws_get(c, WS_LUP, (size_t)B * s.sPair * 8 * (la ? 2 : 1)) : nullptr;
    if (fp32 && (!s.inv || !s.tmp || !s.pair)) return RSRR_ENOMEM;
    s.pair2 = la ? (char*)s.pair + (size_t)B * s.sPair * 8 : nullptr;
    s.la = la ? c->la : nullptr;
    s.la_a = c->la_a;
    s.la_b = c->la_b;
    s.la_c = c->la_c;
    s.upd = nullptr;  // set while the factorisation runs
    s.la_cols = c->la_cols;
    s.sT = (long)s.ld * n;
    s.sP = n;
    s.sPerm = (long)s.np * 2 * MAX_NB;
    s.nparts = ((long)n * n + 255) / 256;
    const size_t esz = prec == RSRR_PREC_C128 ? 16 : 8;
    s.Tlu = ws_get(c, WS_TLU, (size_t)B * s.sT * esz);
    s.Tres = (double2*)ws_get(c, WS_TRES, (size_t)B * s.sT * 16);
    s.ipiv = (int*)ws_get(c, WS_IPIV, (size_t)B * s.sP * 4);
    s.perm = (int2*)ws_get(c, WS_PERM, (size_t)B * s.sPerm * 8);
    s.info = (int*)ws_get(c, WS_INFO, (size_t)B * 4);
    s.coef = (double2*)ws_get(c, WS_COEF, (size_t)std::max(J, 1) * B * 16);
    s.frobp = (double*)ws_get(c, WS_FROBP, (size_t)B * s.nparts * 8);
    s.frob = (double*)ws_get(c, WS_FROB, (size_t)B * 8);
    s.D64 = (float2*)ws_get(c, WS_D64, (size_t)B * s.ld * L * 8);
    s.R = (double2*)ws_get(c, WS_R, (size_t)B * s.ld * L * 16);
    s.norms = (double*)ws_get(c, WS_NORM, (size_t)3 * B * L * 8);
    s.active = (int*)ws_get(c, WS_ACTIVE, (size_t)B * 4);
    s.zdev = (double2*)ws_get(c, WS_Z, (size_t)B * 16);
    if (!s.Tlu || !s.Tres || !s.ipiv || !s.perm || !s.info || !s.coef || !s.frobp || !s.frob ||
        !s.D64 || !s.R || !s.norms || !s.active || !s.zdev)
        return RSRR_ENOMEM;
    return RSRR_OK;
}

// f_j(z_k) of a separable or sparse nep for B host points into coef (device,
// [J][B], point-fastest); the upload is complete on return.
static rsrr_status upload_coef(rsrr_ctx* c, const rsrr_nep* nep, const zd* z, int B, double2* coef)
{
    std::vector<double2> cf((size_t)nep->J * B);
    for (int j = 0; j < nep->J; ++j)
        for (int k = 0; k < B; ++k) {
            const zd f = term_eval(nep->terms[j], z[k]);
            cf[(size_t)j * B + k] = make_double2(f.real(), f.imag());
        }
    RSRR_HIP(hipMemcpyAsync(coef, cf.data(), cf.size() * 16, hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}

// Assemble T(z_k) for the batch into the LU buffer (c64 or c128) and the FP64 copy.
static rsrr_status assemble_batch(rsrr_ctx* c, const rsrr_nep* nep, const zd* z, int B, int prec, SampleBufs& s)
{
    const int n = nep->n;
    float2* T64 = prec == RSRR_PREC_C64_IR ? (float2*)s.Tlu : nullptr;
    double2* Tlu128 = prec == RSRR_PREC_C128 ? (double2*)s.Tlu : nullptr;
    if (nep->kind == RSRR_T_SEPARABLE) {
        RSRR_TRY(upload_coef(c, nep, z, B, s.coef));
        RSRR_HIP(assemble_separable(c->stream, n, nep->J, (const double2*)nep->A, nep->lda, s.coef, B, T64, s.ld,
                                    s.sT, s.Tres, s.ld, s.sT, s.frobp, s.frob));
        if (Tlu128) RSRR_HIP(copy_c128(c->stream, n, n, s.Tres, s.ld, s.sT, Tlu128, s.ld, s.sT, B));
        if (prec == RSRR_PREC_R32_IR) RSRR_HIP(narrow_real(c->stream, n, s.Tres, s.ld, s.sT, (float*)s.Tlu, s.ld, s.sT, B));
    } else if (nep->kind == RSRR_T_SPARSE) {
        // the FP64 copy is formed from the sparse rows, the LU input from it
        RSRR_TRY(upload_coef(c, nep, z, B, s.coef));
        CsrDev d;
        RSRR_TRY(csr_upload(c, nep, d));
        RSRR_HIP(assemble_sparse(c->stream, n, nep->J, d.terms, s.coef, B, T64, s.ld, s.sT, s.Tres, s.ld, s.sT,
                                 s.frobp, s.frob, d.bad));
        RSRR_TRY(csr_check(c, d));
        if (Tlu128) RSRR_HIP(copy_c128(c->stream, n, n, s.Tres, s.ld, s.sT, Tlu128, s.ld, s.sT, B));
    } else {
        std::vector<double2> zz(B);
        for (int k = 0; k < B; ++k) zz[k] = make_double2(z[k].real(), z[k].imag());
        RSRR_HIP(hipMemcpyAsync(s.zdev, zz.data(), (size_t)B * 16, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        RSRR_HIP(assemble_helmholtz(c->stream, n, nep->points, nep->w, s.zdev, B, T64, s.ld, s.sT, s.Tres, s.ld, s.sT,
                                    s.frobp, s.frob));
        if (Tlu128) RSRR_HIP(copy_c128(c->stream, n, n, s.Tres, s.ld, s.sT, Tlu128, s.ld, s.sT, B));
    }
    return RSRR_OK;
}

// R_k = U - T_k X_k (FP64) and the column norms of R_k and X_k (host copies).
static rsrr_status residual_batch(rsrr_ctx* c, int n, int L, const double2* U, int ldu, double2* X, int ldx, long sX,
                                  int B, SampleBufs& s, std::vector<double>& rn, std::vector<double>& xn)
{
    if (resid_skinny_ok(L)) {
        RSRR_HIP(resid_skinny(c->stream, n, L, s.Tres, s.ld, s.sT, X, ldx, sX, U, ldu, 0, s.R, s.ld, (long)s.ld * L,
                              nullptr, B));
    } else {
        RSRR_HIP(bcast_c128(c->stream, n, L, U, ldu, s.R, s.ld, (long)s.ld * L, B));
        RSRR_HIP(zgemm(c->stream, 0, 0, n, L, n, -1.0, s.Tres, s.ld, s.sT, X, ldx, sX, 1.0, s.R, s.ld, (long)s.ld * L,
                       B));
    }
    RSRR_HIP(colnorms(c->stream, n, L, s.R, s.ld, (long)s.ld * L, s.norms, B));
    RSRR_HIP(colnorms(c->stream, n, L, X, ldx, sX, s.norms + (size_t)B * L, B));
    rn.resize((size_t)B * L);
    xn.resize((size_t)B * L);
    RSRR_HIP(hipMemcpyAsync(rn.data(), s.norms, (size_t)B * L * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipMemcpyAsync(xn.data(), s.norms + (size_t)B * L, (size_t)B * L * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return RSRR_OK;
}

// Offset a workspace view to the matrices starting at b0.
static LUWork lu_offset(const LUWork& w, long b0, int esz = 8)
{
    LUWork o = w;
    o.ipiv = w.ipiv + b0 * w.sP;
    o.perm = w.perm + b0 * w.sPerm;
    o.info = w.info + b0;
    if (w.inv) o.inv = (char*)w.inv + b0 * w.sInv * esz;
    if (w.tmp) o.tmp = (char*)w.tmp + b0 * w.sTmp * esz;
    if (w.pair) o.pair = (char*)w.pair + b0 * w.sPair * esz;
    if (w.pair2) o.pair2 = (char*)w.pair2 + b0 * w.sPair * esz;
    if (w.active) o.active = w.active + b0;
    return o;
}

// Run f(stream, b0, count, offset_event) for the point groups, group 0 on the
// context stream and group 1 on the auxiliary stream, joined back into the
// context stream.  When group 0 records `offset_event` (the factorisation does
// after its first panel), group 1 starts only then, so the two groups' panel
// phases interleave with each other's trailing updates instead of coinciding.
template <typename F>
static rsrr_status split_groups(rsrr_ctx* c, int B, F f, bool stagger = false)
{
    const int G = (B >= 8 && c->groups > 1) ? 2 : 1;
    if (G == 1) return f(c->stream, 0, B, (hipEvent_t) nullptr);
    RSRR_HIP(hipEventRecord(c->fork, c->stream));
    RSRR_HIP(hipStreamWaitEvent(c->aux, c->fork, 0));
    const int h = B / 2;
    rsrr_status st = f(c->stream, 0, h, stagger ? c->offset : (hipEvent_t) nullptr);
    if (st) return st;
    if (stagger) RSRR_HIP(hipStreamWaitEvent(c->aux, c->offset, 0));
    st = f(c->aux, h, B - h, (hipEvent_t) nullptr);
    if (st) return st;
    RSRR_HIP(hipEventRecord(c->join, c->aux));
    RSRR_HIP(hipStreamWaitEvent(c->stream, c->join, 0));
    return RSRR_OK;
}

// The CU-masked stream of the look-ahead is created on first use and kept in the
// context (creating it per call cost about 5 ms per headline step).  While it
// exists the process's other streams lose concurrency (the ragged batch, whose
// size buckets run side by side, measured 169 -> 230 ms per step), so the
// ragged-batch path releases it (masked_stream_release) before it launches.
static void masked_stream_acquire(rsrr_ctx* c)
{
    if (!c->lookahead || c->la_cus <= 0 || c->upd) return;
    hipDeviceProp_t prop;
    const int ncu = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.multiProcessorCount : 0;
    if (c->la_cus >= ncu) return;
    // every CU but the first la_cus, which stay free for the look-ahead's panel kernels
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (int i = c->la_cus; i < ncu; ++i) mask[i / 32] |= 1u << (i % 32);
    if (hipExtStreamCreateWithCUMask(&c->upd, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        c->upd = nullptr;
    }
}

}  // namespace

void masked_stream_release(rsrr_ctx* c)
{
    if (!c->upd) return;
    (void)hipStreamSynchronize(c->upd);
    (void)hipStreamDestroy(c->upd);
    c->upd = nullptr;
}

namespace {

static rsrr_status sample_batch(rsrr_ctx* c, const rsrr_nep* nep, const zd* z, int B, const double2* U, int L, int ldu,
                                const std::vector<double>& un, int prec, double2* S, int lds,
                                rsrr_point_info* info, int* any_singular, int* any_fallback, int* any_nan)
{
    const int n = nep->n;
    SampleBufs s;
    rsrr_status st = alloc_bufs(c, n, L, nep->J, prec, B, s);
    if (st) return st;
    const long sX = (long)L * lds;
    double* tm = c->timings;

    {
        PhaseTimer t(c, &tm[0]);
        st = assemble_batch(c, nep, z, B, prec, s);
        if (st) return st;
        t.stop();
    }
    std::vector<int> hinfo(B);
    {
        PhaseTimer t(c, &tm[1]);
        RSRR_HIP(hipMemsetAsync(s.info, 0, (size_t)B * 4, c->stream));
        if (s.la != nullptr && n > 2 * s.nb) masked_stream_acquire(c);
        s.upd = s.la ? c->upd : nullptr;
        const LUWork w = s.lu(nullptr, c->rec_on ? &c->rec : nullptr);
        st = split_groups(
            c, B,
            [&](hipStream_t sm, int b0, int nbg, hipEvent_t ev) -> rsrr_status {
                LUWork wg = lu_offset(w, b0, prec == RSRR_PREC_R32_IR ? 4 : 8);
                wg.first_panel = ev;
                if (prec == RSRR_PREC_C128)
                    RSRR_HIP(getrf_batched<double>(sm, (double2*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb, wg, nbg));
                else if (prec == RSRR_PREC_R32_IR)
                    RSRR_HIP(getrf_real_batched(sm, (float*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb, wg, nbg));
                else
                    RSRR_HIP(getrf_batched<float>(sm, (float2*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb, wg, nbg));
                return RSRR_OK;
            },
            true);
        if (st) return st;
        t.stop();
        if (c->rec_on) rec_collect(c);
        RSRR_HIP(hipMemcpyAsync(hinfo.data(), s.info, (size_t)B * 4, hipMemcpyDeviceToHost, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
    }
    std::vector<int> act(B, 1);
    for (int k = 0; k < B; ++k) {
        if (info) {
            info[k].info = hinfo[k];
            info[k].ir_iters = 0;
            info[k].fallback = 0;
            info[k].resid = 0.0;
        }
        if (hinfo[k] > 0) { *any_singular = 1; act[k] = 0; }
        if (hinfo[k] < 0) { *any_nan = 1; act[k] = 0; }
    }
    RSRR_HIP(hipMemcpyAsync(s.active, act.data(), (size_t)B * 4, hipMemcpyHostToDevice, c->stream));

    std::vector<double> rn, xn, fro(B);
    RSRR_HIP(hipMemcpyAsync(fro.data(), s.frob, (size_t)B * 8, hipMemcpyDeviceToHost, c->stream));

    if (prec == RSRR_PREC_C128) {
        {
            PhaseTimer t(c, &tm[2]);
            RSRR_HIP(bcast_c128(c->stream, n, L, U, ldu, S, lds, sX, B));
            const LUWork w = s.lu(s.active, nullptr);
            st = split_groups(c, B, [&](hipStream_t sm, int b0, int nbg, hipEvent_t) -> rsrr_status {
                RSRR_HIP(getrs_batched<double>(sm, (const double2*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb,
                                               lu_offset(w, b0), S + b0 * sX, sX, lds, L, nbg));
                return RSRR_OK;
            });
            if (st) return st;
            t.stop();
        }
        {
            PhaseTimer t(c, &tm[3]);
            st = residual_batch(c, n, L, U, ldu, S, lds, sX, B, s, rn, xn);
            if (st) return st;
            t.stop();
        }
        for (int k = 0; k < B; ++k) {
            double r = 0;
            for (int cc = 0; cc < L; ++cc) r = std::max(r, rn[(size_t)k * L + cc] / un[cc]);
            if (info) info[k].resid = r;
        }
        return RSRR_OK;
    }

    // mixed path: X0 = getrs_c64(U), then refinement with FP64 residuals
    {
        PhaseTimer t(c, &tm[2]);
        const LUWork w = s.lu(s.active, nullptr);
        if (prec == RSRR_PREC_R32_IR) {
            float* D = (float*)s.D64;
            RSRR_HIP(scale_narrow_real(c->stream, n, L, U, ldu, 0, nullptr, D, s.ld, (long)s.ld * L, nullptr, B));
            st = split_groups(c, B, [&](hipStream_t sm, int b0, int nbg, hipEvent_t) -> rsrr_status {
                RSRR_HIP(getrs_real_batched(sm, (const float*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb,
                                            lu_offset(w, b0, 4), D + b0 * (long)s.ld * L, (long)s.ld * L, s.ld, L,
                                            nbg));
                return RSRR_OK;
            });
            if (st) return st;
            RSRR_HIP(axpy_widen_real(c->stream, n, L, D, s.ld, (long)s.ld * L, nullptr, S, lds, sX, nullptr, B));
        } else {
            RSRR_HIP(bcast_to_c64(c->stream, n, L, U, ldu, s.D64, s.ld, (long)s.ld * L, B));
            st = split_groups(c, B, [&](hipStream_t sm, int b0, int nbg, hipEvent_t) -> rsrr_status {
                RSRR_HIP(getrs_batched<float>(sm, (const float2*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb,
                                              lu_offset(w, b0), s.D64 + b0 * (long)s.ld * L, (long)s.ld * L, s.ld,
                                              L, nbg));
                return RSRR_OK;
            });
            if (st) return st;
            RSRR_HIP(widen(c->stream, n, L, s.D64, s.ld, (long)s.ld * L, S, lds, sX, B));
        }
        t.stop();
    }
    const double eps = 1.1102230246251565e-16;
    const double tol_be = c->ir_tol * eps * std::sqrt((double)n);
    std::vector<double> prev(B, 1e300), resid(B, 0.0), scl((size_t)B * L), inv((size_t)B * L);
    std::vector<int> done(B, 0), iters(B, 0);
    for (int k = 0; k < B; ++k) done[k] = act[k] ? 0 : 1;
    for (int it = 0;; ++it) {
        {
            PhaseTimer t(c, &tm[3]);
            st = residual_batch(c, n, L, U, ldu, S, lds, sX, B, s, rn, xn);
            if (st) return st;
            t.stop();
        }
        int live = 0;
        for (int k = 0; k < B; ++k) {
            double r = 0, eta = 0;
            for (int cc = 0; cc < L; ++cc) {
                const double rr = rn[(size_t)k * L + cc];
                r = std::max(r, rr / un[cc]);
                eta = std::max(eta, rr / (fro[k] * xn[(size_t)k * L + cc] + un[cc]));
            }
            if (!done[k]) {
                resid[k] = r;
                iters[k] = it;
                const bool conv = eta <= tol_be;
                const bool stall = r > 0.5 * prev[k];
                if (conv || stall || it >= c->ir_max_iters || !(r == r)) done[k] = 1;
                prev[k] = r;
            }
            act[k] = done[k] ? 0 : 1;
            live += act[k];
            for (int cc = 0; cc < L; ++cc) {
                const double rr = rn[(size_t)k * L + cc];
                scl[(size_t)k * L + cc] = rr;
                inv[(size_t)k * L + cc] = rr > 0 ? 1.0 / rr : 0.0;
            }
        }
        if (!live) break;
        {
            PhaseTimer t(c, &tm[2]);
            RSRR_HIP(hipMemcpyAsync(s.active, act.data(), (size_t)B * 4, hipMemcpyHostToDevice, c->stream));
            RSRR_HIP(hipMemcpyAsync(s.norms + (size_t)2 * B * L, inv.data(), (size_t)B * L * 8, hipMemcpyHostToDevice,
                                    c->stream));
            const LUWork w = s.lu(s.active, nullptr);
            double* sc = s.norms + (size_t)2 * B * L;
            if (prec == RSRR_PREC_R32_IR) {
                float* D = (float*)s.D64;
                RSRR_HIP(scale_narrow_real(c->stream, n, L, s.R, s.ld, (long)s.ld * L, sc, D, s.ld, (long)s.ld * L,
                                           s.active, B));
                st = split_groups(c, B, [&](hipStream_t sm, int b0, int nbg, hipEvent_t) -> rsrr_status {
                    RSRR_HIP(getrs_real_batched(sm, (const float*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb,
                                                lu_offset(w, b0, 4), D + b0 * (long)s.ld * L, (long)s.ld * L, s.ld,
                                                L, nbg));
                    return RSRR_OK;
                });
                if (st) return st;
                RSRR_HIP(hipMemcpyAsync(sc, scl.data(), (size_t)B * L * 8, hipMemcpyHostToDevice, c->stream));
                RSRR_HIP(axpy_widen_real(c->stream, n, L, D, s.ld, (long)s.ld * L, sc, S, lds, sX, s.active, B));
            } else {
                RSRR_HIP(scale_narrow(c->stream, n, L, s.R, s.ld, (long)s.ld * L, sc, s.D64, s.ld, (long)s.ld * L,
                                      s.active, B));
                st = split_groups(c, B, [&](hipStream_t sm, int b0, int nbg, hipEvent_t) -> rsrr_status {
                    RSRR_HIP(getrs_batched<float>(sm, (const float2*)s.Tlu + b0 * s.sT, s.sT, s.ld, n, s.nb,
                                                  lu_offset(w, b0), s.D64 + b0 * (long)s.ld * L, (long)s.ld * L,
                                                  s.ld, L, nbg));
                    return RSRR_OK;
                });
                if (st) return st;
                RSRR_HIP(hipMemcpyAsync(sc, scl.data(), (size_t)B * L * 8, hipMemcpyHostToDevice, c->stream));
                RSRR_HIP(axpy_widen(c->stream, n, L, s.D64, s.ld, (long)s.ld * L, sc, S, lds, sX, s.active, B));
            }
            t.stop();
        }
    }
    for (int k = 0; k < B; ++k) {
        if (info) {
            info[k].ir_iters = iters[k];
            info[k].resid = resid[k];
        }
    }
    // fallback: points whose refinement did not reach fallback_resid are redone in FP64
    for (int k = 0; k < B; ++k) {
        if (hinfo[k] != 0) continue;
        if (resid[k] <= c->fallback_resid) continue;
        rsrr_point_info pi;
        int sing = 0, fb = 0, nan = 0;
        st = sample_batch(c, nep, z + k, 1, U, L, ldu, un, RSRR_PREC_C128, S + (size_t)k * sX, lds, &pi, &sing, &fb,
                          &nan);
        if (st) return st;
        *any_fallback = 1;
        if (info) {
            info[k].fallback = 1;
            info[k].resid = pi.resid;
            info[k].info = pi.info;
        }
        if (sing) *any_singular = 1;
        if (nan) *any_nan = 1;
    }
    return RSRR_OK;
}

}  // namespace

bool csr_nep_ok(const rsrr_nep* nep)
{
    if (nep->J < 1 || nep->J > 64 || !nep->terms || !nep->csr) return false;
    for (int j = 0; j < nep->J; ++j) {
        const rsrr_csr& m = nep->csr[j];
        if (m.nnz < 0 || !m.rowptr || (m.nnz > 0 && (!m.col || !m.val))) return false;
    }
    return true;
}

rsrr_status csr_upload(rsrr_ctx* c, const rsrr_nep* nep, CsrDev& d)
{
    const size_t tb = ((size_t)nep->J * sizeof(CsrTerm) + 255) / 256 * 256;
    char* p = (char*)ws_get(c, WS_CSR, tb + 256);
    if (!p) return RSRR_ENOMEM;
    std::vector<CsrTerm> h(nep->J);
    for (int j = 0; j < nep->J; ++j) {
        const rsrr_csr& m = nep->csr[j];
        h[j] = CsrTerm{m.rowptr, m.col, (const double2*)m.val, m.nnz, 0};
    }
    RSRR_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(CsrTerm), hipMemcpyHostToDevice, c->stream));
    RSRR_HIP(hipMemsetAsync(p + tb, 0, 4, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    d.terms = (CsrTerm*)p;
    d.bad = (int*)(p + tb);
    return RSRR_OK;
}

rsrr_status csr_check(rsrr_ctx* c, const CsrDev& d)
{
    int h = 0;
    RSRR_HIP(hipMemcpyAsync(&h, d.bad, 4, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    return h ? -2 : RSRR_OK;
}

rsrr_status assemble_c128(rsrr_ctx* c, const rsrr_nep* nep, const zd* z, int B, double2* T, int ld, long sT,
                          double* frob)
{
    const int n = nep->n;
    const long nparts = ((long)n * n + 255) / 256;
    double* frobp = (double*)ws_get(c, WS_FROBP, (size_t)B * nparts * 8);
    if (!frobp) return RSRR_ENOMEM;
    if (nep->kind == RSRR_T_SEPARABLE || nep->kind == RSRR_T_SPARSE) {
        double2* coef = (double2*)ws_get(c, WS_COEF, (size_t)nep->J * B * 16);
        if (!coef) return RSRR_ENOMEM;
        RSRR_TRY(upload_coef(c, nep, z, B, coef));
        if (nep->kind == RSRR_T_SEPARABLE) {
            RSRR_HIP(assemble_separable(c->stream, n, nep->J, (const double2*)nep->A, nep->lda, coef, B, nullptr, 0,
                                        0, T, ld, sT, frobp, frob));
        } else {
            CsrDev d;
            RSRR_TRY(csr_upload(c, nep, d));
            RSRR_HIP(assemble_sparse(c->stream, n, nep->J, d.terms, coef, B, nullptr, 0, 0, T, ld, sT, frobp, frob,
                                     d.bad));
            RSRR_TRY(csr_check(c, d));
        }
    } else {
        double2* zdev = (double2*)ws_get(c, WS_Z, (size_t)B * 16);
        if (!zdev) return RSRR_ENOMEM;
        std::vector<double2> zz(B);
        for (int k = 0; k < B; ++k) zz[k] = make_double2(z[k].real(), z[k].imag());
        RSRR_HIP(hipMemcpyAsync(zdev, zz.data(), (size_t)B * 16, hipMemcpyHostToDevice, c->stream));
        RSRR_HIP(hipStreamSynchronize(c->stream));
        RSRR_HIP(assemble_helmholtz(c->stream, n, nep->points, nep->w, zdev, B, nullptr, 0, 0, T, ld, sT, frobp, frob));
    }
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_sample(rsrr_ctx* c, const rsrr_nep* nep, int N, const double* z, const double* U, int L,
                                   int ldu, int prec, double* S, int lds, rsrr_point_info* info)
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
    if (!U) return -5;
    if (L < 1) return -6;
    if (ldu < nep->n) return -7;
    if (prec != RSRR_PREC_C128 && prec != RSRR_PREC_C64_IR && prec != RSRR_PREC_R32_IR) return -8;
    if (prec == RSRR_PREC_R32_IR) {
        // real arithmetic needs a separable NEP and real points
        if (nep->kind != RSRR_T_SEPARABLE) return -2;
        for (int k = 0; k < N; ++k)
            if (z[2 * k + 1] != 0.0) return -4;
    }
    if (!S) return -9;
    if (lds < nep->n) return -10;
    RSRR_HIP(hipSetDevice(c->device));
    const int n = nep->n;
    for (int i = 0; i < 5; ++i) c->timings[i] = 0.0;
    RSRR_HIP(hipEventRecord(c->ev[0], c->stream));

    // probe column norms (for relative residuals)
    double* dn = (double*)ws_get(c, WS_B7, (size_t)L * 8);
    if (!dn) return RSRR_ENOMEM;
    RSRR_HIP(colnorms(c->stream, n, L, (const double2*)U, ldu, 0, dn, 1));
    std::vector<double> un(L);
    RSRR_HIP(hipMemcpyAsync(un.data(), dn, (size_t)L * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    for (auto& v : un)
        if (!(v > 0)) v = 1.0;

    // batch size from the workspace budget
    size_t budget = c->ws_budget;
    if (!budget) {
        size_t fr = 0, tot = 0;
        RSRR_HIP(hipMemGetInfo(&fr, &tot));
        budget = fr / 2;
    }
    const size_t ppb = per_point_bytes(n, L, prec);
    int Bp = (int)std::min<size_t>((size_t)N, std::max<size_t>(1, budget / ppb));

    std::vector<zd> zz(N);
    for (int k = 0; k < N; ++k) zz[k] = zd(z[2 * k], z[2 * k + 1]);
    int sing = 0, fb = 0, nan = 0;
    for (int k0 = 0; k0 < N; k0 += Bp) {
        const int B = std::min(Bp, N - k0);
        rsrr_status st = sample_batch(c, nep, zz.data() + k0, B, (const double2*)U, L, ldu, un, prec,
                                      (double2*)S + (size_t)k0 * L * lds, lds, info ? info + k0 : nullptr, &sing, &fb,
                                      &nan);
        if (st) return st;
    }
    RSRR_HIP(hipEventRecord(c->ev[1], c->stream));
    RSRR_HIP(hipEventSynchronize(c->ev[1]));
    float ms = 0.f;
    RSRR_HIP(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    c->timings[4] = ms;
    if (nan) return RSRR_ENAN;
    if (sing) return RSRR_ESINGULAR;
    if (fb) return RSRR_WARN_FALLBACK;
    return RSRR_OK;
}
