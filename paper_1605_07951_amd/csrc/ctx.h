// Library context: device, stream, grow-only workspace and phase timers.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <vector>

#include "kernels.h"
#include "rsrr.h"

typedef std::complex<double> zd;

// Workspace slots (each a grow-only device allocation owned by the context).
enum WsSlot {
    WS_TLU = 0, WS_TRES, WS_IPIV, WS_PERM, WS_INFO, WS_COEF, WS_FROBP, WS_FROB,
    WS_D64, WS_R, WS_NORM, WS_ACTIVE, WS_Z,
    WS_B0, WS_B1, WS_B2, WS_B3, WS_B4, WS_B5, WS_B6, WS_B7, WS_N1, WS_JAC, WS_TSQ, WS_TSAQ, WS_TSV,
    WS_GMF, WS_GMW, WS_GMK, WS_GMS, WS_GMT, WS_GMI,
    WS_HS0, WS_HS1, WS_HS2, WS_HSW, WS_HSX, WS_HSD, WS_HSI, WS_LUP, WS_CSR,
    WS_COUNT
};

struct rsrr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;       // second stream (default priority) for the second point group
    hipEvent_t fork = nullptr, join = nullptr, offset = nullptr;
    int groups = 1;                  // point groups factored on separate streams (1 = off; measured no overlap)
    hipStream_t la = nullptr;        // look-ahead stream of the LU (default priority): next panels beside the update
    hipEvent_t la_a = nullptr, la_b = nullptr, la_c = nullptr;
    hipStream_t upd = nullptr;       // CU-masked stream for the overlapped updates (null: no mask)
    bool lookahead = true;           // RSRR_LOOKAHEAD=0 at creation turns it off
    int la_cus = 32;                 // CUs the overlapped updates leave to the look-ahead (RSRR_LA_CUS)
    int la_cols = 0;                 // columns of each overlapped update on the masked stream (RSRR_LA_COLS)
    void* ws[WS_COUNT] = {};
    size_t ws_size[WS_COUNT] = {};
    hipEvent_t ev[2] = {};
    double timings[5] = {0, 0, 0, 0, 0};
    int nb_c64 = 128;      // outer LU panel width, complex FP32 path
    int nb_c128 = 64;      // outer LU panel width, complex FP64 path
    // options (rsrr_set_options)
    int ir_max_iters = 10;          // host refinement loop of rsrr_sample
    int ir_max_iters_batched = 3;   // device refinement of rsrr_sample_batched / the server
    int basis_sketch_max = 1024;    // first range-sketch width of rsrr_basis
    double ir_tol = 4.0;            // backward-error stop: ir_tol * u * sqrt(n)
    double fallback_resid = 1e-10;  // refined points above this are redone in FP64
    double delta = 1e-14;           // library-chosen rank truncation (server)
    double tol_gap = 1e3;           // library-chosen gap threshold (server)
    size_t ws_budget = 0;  // bytes for the per-point sampling buffers (0 = half of free memory)
    void* noalloc_scratch = nullptr;  // this device's address of the no-allocation scratch array
    // trailing-update statistics (rsrr_update_stats)
    bool rec_on = false;
    rsrr::UpdateRecorder rec;
    double upd_ms = 0.0, upd_flops = 0.0, upd_bytes = 0.0;
    double upd_ms_masked = 0.0, upd_flops_masked = 0.0;  // launches on the CU-masked stream
    long upd_launches = 0, upd_dropped = 0;
};

// Release the ragged-batch buffers and graphs of a context.
void batched_release(rsrr_ctx* c);

// Destroy the context's CU-masked look-ahead stream, if any (it is recreated on
// the next factorisation that uses it).
void masked_stream_release(rsrr_ctx* c);

// Fold the recorded update events into the running statistics (syncs the events).
void rec_collect(rsrr_ctx* c);

// Grow workspace slot `s` to at least `bytes`; returns nullptr on failure.
void* ws_get(rsrr_ctx* c, int s, size_t bytes);

// Assemble T(z_k) in complex FP64 for B host points into T (ld, stride sT);
// frob (device, B doubles) receives ||T(z_k)||_F.  Uses workspace slots
// WS_COEF, WS_Z, WS_FROBP (and WS_CSR for a SPARSE nep, whose bounds it
// checks: -2 when an entry lies out of bounds).
rsrr_status assemble_c128(rsrr_ctx* c, const rsrr_nep* nep, const zd* z, int B, double2* T, int ld, long sT,
                          double* frob);

// SPARSE nep: descriptor checks on the host (J in 1..64, terms and csr given,
// every matrix with rowptr, and col and val when nnz > 0).
bool csr_nep_ok(const rsrr_nep* nep);
// The J descriptors of a SPARSE nep as a device table in slot WS_CSR, with the
// device bounds flag (zeroed) after it; csr_check syncs the stream and returns
// -2 when a kernel found an entry out of bounds since the upload.
struct CsrDev {
    rsrr::CsrTerm* terms = nullptr;
    int* bad = nullptr;
};
rsrr_status csr_upload(rsrr_ctx* c, const rsrr_nep* nep, CsrDev& d);
rsrr_status csr_check(rsrr_ctx* c, const CsrDev& d);

// One-sided Jacobi SVD (api_basis): see jacobi_round.  Returns sweeps or -1.
int jacobi_svd(rsrr_ctx* c, double2* A, int lda, int m, int m_apply, int p, int max_sweeps, double tol,
               rsrr_status* st);

// Device address of the no-allocation scratch array on `device` (the current
// device), looked up once per device.
rsrr_status noalloc_scratch_setup(int device, void** out);

// Device-resident LU factors of one NEP's sampling points (serving: kept from
// factorisation until the request finishes, so more probe columns can be solved
// without refactoring).  Layout in one caller-provided block, each part
// 256-byte aligned: factors T (N matrices P x P, P = n rounded up to 64, stride
// sT; complex FP32 or FP64 by prec), composed row interchanges perm (stride
// sPerm) and, for complex FP32, the diagonal-block inverses inv (stride sInv),
// with the panel width nb they were made with (set by the sampling call).
struct FactorStore {
    void* T = nullptr;
    int2* perm = nullptr;
    void* inv = nullptr;
    long sT = 0, sPerm = 0, sInv = 0;
    int P = 0, N = 0, prec = 0, nb = 0;
};
size_t factor_store_bytes(int n, int N, int prec);
FactorStore factor_store_at(void* base, int n, int N, int prec);

// rsrr_sample_batched (eager launches) that also copies every instance's
// factors into keep[i] at points k0[i] .. k0[i] + N_i - 1 (keep[i] may be null).
rsrr_status sample_batched_keep(rsrr_ctx* c, int count, const rsrr_instance* inst, int prec, rsrr_point_info* info,
                                FactorStore* const* keep, const int* k0);

// X = T(z_k)^-1 U for points k0 .. k0 + in.N - 1 of a store: triangular solves with
// the kept factors and refinement against FP64 residuals (T(z_k) regenerated), no
// factorisation.  Points that do not reach fallback_resid are redone in FP64.
rsrr_status solve_from_store(rsrr_ctx* c, const rsrr_instance& in, const FactorStore& fs, int k0,
                             rsrr_point_info* info);

// Free the ragged-batch buffers (and graphs) of a context when they hold more than
// keep_bytes (after its streams have drained).
void batched_trim(rsrr_ctx* c, size_t keep_bytes);

// f(z) = c (z - z0)^p exp(-tau z) / (z - s)^q
zd term_eval(const rsrr_term& t, zd z);

#define RSRR_HIP(call)                                  \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return RSRR_EDEVICE;      \
    } while (0)
// return the status of a library step unless it is RSRR_OK
#define RSRR_TRY(call)                                  \
    do {                                                \
        rsrr_status _s = (call);                        \
        if (_s != RSRR_OK) return _s;                   \
    } while (0)
