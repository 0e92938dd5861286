// C ABI: resolvent sampling for a ragged batch of NEP instances (RSRR Step 2
// for many problems at once).
//
// Instances are grouped in size buckets P = n rounded up to 64.  Inside a
// bucket every (instance, point) pair is one P x P matrix: T(z_k) occupies the
// leading n x n block and the identity the rest, so the LU stays block
// diagonal (no pivot is ever taken from the identity part, whose entries in
// the leading columns are zero) and the solve with [U; 0] returns
// [T^-1 U; 0].  The bucket is then one uniform batch for the LU, solve and
// refinement kernels.  Refinement decisions are taken on the device (fixed
// budget of corrections, per-point masks), so a bucket's work has no host
// synchronisation and can be captured once in a hipGraph and replayed.
// The panel width of each bucket is picked by timing the factorisation with
// each candidate (autotune) and is cached per (P, precision), optionally in a
// text file (RSRR_TUNE_FILE).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

namespace {

constexpr int BUCKET = 64;

// Host tables of one bucket: per-matrix order, coefficient (separable) or point
// (Helmholtz) table of every instance in bucket order, and the instance tables of
// the bucket-wide launches (sep empty unless every instance is separable).
struct BucketHost {
    std::vector<int> nk;
    std::vector<double2> coef;
    std::vector<SepInstance> sep;
    std::vector<RhsInstance> rhs;
    int nmax = 0, Nmax = 0;
};

// One captured graph for a whole batched call: every bucket's work as an
// independent branch (forked from the capture stream onto the bucket streams and
// joined back), replayed with one launch.
struct GraphEntry {
    std::vector<unsigned long long> key;
    hipGraphExec_t exec = nullptr;
    std::vector<BucketHost> host;   // the captured buckets' host tables (uploaded before every replay)
};

constexpr int N_BUCKET_STREAMS = 8;  // replayed buckets run side by side on these (default priority)

// One autotuned configuration of a size bucket: LU panel width, workgroup tile of
// the complex FP32 trailing update, and the time of the bucket pass it won with.
struct Tuned {
    int nb = 0;
    int tile = UPD_TILE_3M_128x64;
    double ms = 0.0;
};

// Sets the update tile for the calling thread and restores the previous one.
struct TileScope {
    int prev;
    explicit TileScope(int t) : prev(get_update_tile()) { set_update_tile(t); }
    ~TileScope() { set_update_tile(prev); }
};

struct BatchedState {
    std::map<int, long> last_use;                 // bucket size P -> call counter of its last use
    long calls = 0;
    std::map<long, Tuned> tuned;                  // (P*2 + prec) -> panel width and update tile
    std::string arch;                             // device architecture the tuned entries are for
    std::unique_ptr<GraphEntry> graph;            // the last call's captured graph
    hipEvent_t cap_fork = nullptr;                // fork point inside a capture
    std::vector<void*> bufs;
    std::vector<size_t> sizes;
    bool file_loaded = false;
    hipStream_t streams[N_BUCKET_STREAMS] = {};
    hipEvent_t done[N_BUCKET_STREAMS] = {};
};

std::map<rsrr_ctx*, std::unique_ptr<BatchedState>>& states()
{
    static std::map<rsrr_ctx*, std::unique_ptr<BatchedState>> m;
    return m;
}

// contexts of different host threads (a server's sampling thread and the
// caller's) look up their state concurrently
std::mutex& states_mu()
{
    static std::mutex mu;
    return mu;
}

BatchedState& state_of(rsrr_ctx* c)
{
    std::lock_guard<std::mutex> lk(states_mu());
    auto& m = states();
    auto it = m.find(c);
    if (it == m.end()) it = m.emplace(c, std::make_unique<BatchedState>()).first;
    return *it->second;
}

void* bget(BatchedState& S, int slot, size_t bytes, hipStream_t st)
{
    if ((int)S.bufs.size() <= slot) {
        S.bufs.resize(slot + 1, nullptr);
        S.sizes.resize(slot + 1, 0);
    }
    if (bytes == 0) bytes = 256;
    if (S.sizes[slot] >= bytes) return S.bufs[slot];
    if (S.bufs[slot]) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(S.bufs[slot]);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        S.bufs[slot] = nullptr;
        S.sizes[slot] = 0;
        return nullptr;
    }
    S.bufs[slot] = p;
    S.sizes[slot] = bytes;
    return p;
}

// The autotuner's cache (RSRR_TUNE_FILE): JSON, one entry per line,
//   {"arch": "gfx950", "entries": [
//    {"P": 320, "prec": "c64", "nb": 64, "update_tile": 1, "update_tile_name": "3m_64x64_4waves", "ms": 1.23},
//    ...]}
// Entries of another architecture are ignored when read.
std::string device_arch(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { (void)hipGetLastError(); return "unknown"; }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

void load_tune_file(BatchedState& S, int device)
{
    if (S.file_loaded) return;
    S.file_loaded = true;
    S.arch = device_arch(device);
    const char* f = std::getenv("RSRR_TUNE_FILE");
    if (!f) return;
    FILE* fp = std::fopen(f, "r");
    if (!fp) return;
    char line[512];
    std::string farch;
    while (std::fgets(line, sizeof line, fp)) {
        const char* a = std::strstr(line, "\"arch\":");
        if (a) {
            char buf[64] = {0};
            if (std::sscanf(a, "\"arch\": \"%63[^\"]\"", buf) == 1) farch = buf;
        }
        const char* pp = std::strstr(line, "\"P\":");
        if (!pp || farch != S.arch) continue;
        int P = 0, nb = 0, tile = 0;
        char prec[16] = {0};
        double ms = 0.0;
        const char* q;
        if (std::sscanf(pp, "\"P\": %d", &P) != 1) continue;
        if (!(q = std::strstr(line, "\"prec\":")) || std::sscanf(q, "\"prec\": \"%15[^\"]\"", prec) != 1) continue;
        if (!(q = std::strstr(line, "\"nb\":")) || std::sscanf(q, "\"nb\": %d", &nb) != 1) continue;
        if ((q = std::strstr(line, "\"update_tile\":"))) std::sscanf(q, "\"update_tile\": %d", &tile);
        if ((q = std::strstr(line, "\"ms\":"))) std::sscanf(q, "\"ms\": %lf", &ms);
        const bool mixed = std::strcmp(prec, "c64") == 0;
        if (!mixed && std::strcmp(prec, "c128") != 0) continue;
        if (nb < MIN_NB || nb > (mixed ? max_panel<float>() : max_panel<double>())) continue;
        if (tile < 0 || tile >= UPD_TILE_COUNT) tile = UPD_TILE_3M_128x64;
        Tuned t;
        t.nb = nb;
        t.tile = tile;
        t.ms = ms;
        S.tuned[(long)P * 2 + (mixed ? 1 : 0)] = t;
    }
    std::fclose(fp);
}

void save_tune_file(const BatchedState& S)
{
    const char* f = std::getenv("RSRR_TUNE_FILE");
    if (!f) return;
    FILE* fp = std::fopen(f, "w");
    if (!fp) return;
    std::fprintf(fp, "{\"arch\": \"%s\", \"entries\": [\n", S.arch.c_str());
    size_t i = 0;
    for (auto& kv : S.tuned) {
        const int P = (int)(kv.first / 2);
        const bool mixed = (kv.first & 1) != 0;
        std::fprintf(fp, " {\"P\": %d, \"prec\": \"%s\", \"nb\": %d, \"update_tile\": %d, \"update_tile_name\": \"%s\", "
                     "\"ms\": %.4f}%s\n", P, mixed ? "c64" : "c128", kv.second.nb, kv.second.tile,
                     update_tile_name(kv.second.tile), kv.second.ms, ++i < S.tuned.size() ? "," : "");
    }
    std::fprintf(fp, "]}\n");
    std::fclose(fp);
}

struct BucketBufs {
    void* T; double2* T128; double2* Ub; double2* Xb; double2* R; float2* D64; int* ipiv; int2* perm;
    int* info; void* inv; void* tmp; int* nk; double2* coef; double* frobp; double* frob; double* un; double* rn;
    double* xn; double* inv_s; double* scl; int* active; double* prev; double* resid; int* iters; double* ones;
    void* pair; SepInstance* sep; RhsInstance* rhs;
    long sT, sU, sP, sPerm, sInv, sTmp, sPair;
};

// Strides of one point's factor data in the bucket buffers and in a FactorStore.
long bucket_sPerm(int P) { return (long)perm_panels(P) * 2 * MAX_NB; }
long bucket_sInv(int P, bool mixed) { return mixed ? 2L * max_panel<float>() * (P + max_panel<float>()) : 0; }

// The complex FP32 solves of a bucket: the whole sweep per matrix in one launch when its
// right-hand sides fit in LDS, else one launch per panel step.
hipError_t solve_c64(hipStream_t sm, const BucketBufs& b, int P, int nb, const LUWork& w, int Lmax, long M)
{
    if (getrs_lds_ok(P, Lmax))
        return getrs_lds_batched(sm, (const float2*)b.T, b.sT, P, P, nb, w, b.D64, b.sU, P, Lmax, (int)M);
    return getrs_batched<float>(sm, (const float2*)b.T, b.sT, P, P, nb, w, b.D64, b.sU, P, Lmax, (int)M);
}

// The bucket's host tables into its device buffers.
hipError_t upload_tables(hipStream_t sm, const BucketHost& h, BucketBufs& b)
{
    hipError_t e = hipMemcpyAsync(b.nk, h.nk.data(), h.nk.size() * 4, hipMemcpyHostToDevice, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(b.coef, h.coef.data(), h.coef.size() * 16, hipMemcpyHostToDevice, sm);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.rhs, h.rhs.data(), h.rhs.size() * sizeof(RhsInstance), hipMemcpyHostToDevice, sm);
    if (e == hipSuccess && !h.sep.empty())
        e = hipMemcpyAsync(b.sep, h.sep.data(), h.sep.size() * sizeof(SepInstance), hipMemcpyHostToDevice, sm);
    return e;
}

// Everything a bucket does on the device, in stream order (capturable with
// upload = false once the tables are on the device).
// keep (may be null): per entry of ids, the store that receives that instance's
// factors (null: none) at point keep_k0[q].  from (may be null): the bucket is one
// instance whose factors are already in this store from point from_k0: no
// complex FP32 assembly and no factorisation.
rsrr_status run_bucket(rsrr_ctx* c, hipStream_t sm, const rsrr_instance* inst, const std::vector<int>& ids,
                       const std::vector<long>& off, int P, int Lmax, long M, int prec, int nb, BucketBufs& b,
                       const BucketHost& h, int maxit, FactorStore* const* keep = nullptr,
                       const int* keep_k0 = nullptr, const FactorStore* from = nullptr, int from_k0 = 0,
                       bool upload = true)
{
    const bool mixed = prec == RSRR_PREC_C64_IR;
    const size_t esz = mixed ? 8 : 16;
    if (from) {
        // the kept factors stand in for the bucket's factor buffers
        b.T = (char*)from->T + (size_t)from_k0 * from->sT * esz;
        b.perm = from->perm + (size_t)from_k0 * from->sPerm;
        b.inv = mixed ? (void*)((char*)from->inv + (size_t)from_k0 * from->sInv * 8) : nullptr;
    }
    // host tables (unless the caller uploaded them: a captured graph holds kernels only),
    // then the per-matrix identity padding
    const int nins = (int)ids.size();
    if (upload) RSRR_HIP(upload_tables(sm, h, b));
    RSRR_HIP(pad_identity(sm, mixed && !from ? (float2*)b.T : nullptr, b.T128, P, b.sT, P, b.nk, (int)M));
    if (!mixed && !from) RSRR_HIP(pad_identity(sm, nullptr, (double2*)b.T, P, b.sT, P, b.nk, (int)M));
    if (!h.sep.empty()) {
        // every instance separable: the whole bucket's assembly in one launch (FP64 sums,
        // c64 and c128 copies) and one for the norms
        RSRR_HIP(assemble_separable_group(sm, b.sep, nins, h.nmax, h.Nmax, b.coef, P, (int)M, b.nk,
                                          mixed && !from ? (float2*)b.T : nullptr, b.sT, b.T128, b.sT, b.frobp,
                                          b.frob));
        if (!mixed && !from) RSRR_HIP(copy_c128(sm, P, P, b.T128, P, b.sT, (double2*)b.T, P, b.sT, (int)M));
    } else {
        // assembly of every instance's points (FP64 sums, c64 and c128 copies)
        long coff = 0;
        for (size_t q = 0; q < ids.size(); ++q) {
            const rsrr_instance& in = inst[ids[q]];
            const int n = in.nep.n;
            const long nparts = ((long)n * n + 255) / 256;
            if (in.nep.kind == RSRR_T_SEPARABLE) {
                const long cnt = (long)in.nep.J * in.N;
                RSRR_HIP(assemble_separable(sm, n, in.nep.J, (const double2*)in.nep.A, in.nep.lda, b.coef + coff,
                                            in.N, mixed && !from ? (float2*)b.T + off[q] * b.sT : nullptr, P, b.sT,
                                            b.T128 + off[q] * b.sT, P, b.sT, b.frobp + off[q] * nparts,
                                            b.frob + off[q]));
                coff += cnt;
            } else {
                const long cnt = in.N;
                RSRR_HIP(assemble_helmholtz(sm, n, in.nep.points, in.nep.w, b.coef + coff, in.N,
                                            mixed && !from ? (float2*)b.T + off[q] * b.sT : nullptr, P, b.sT,
                                            b.T128 + off[q] * b.sT, P, b.sT, b.frobp + off[q] * nparts,
                                            b.frob + off[q]));
                coff += cnt;
            }
            if (!mixed && !from)
                RSRR_HIP(copy_c128(sm, n, n, b.T128 + off[q] * b.sT, P, b.sT, (double2*)b.T + off[q] * b.sT, P,
                                   b.sT, in.N));
        }
    }
    // padded right-hand sides [U; 0], all instances in one launch
    RSRR_HIP(zero_c128(sm, P, Lmax, b.Ub, P, b.sU, (int)M));
    RSRR_HIP(bcast_group(sm, b.rhs, nins, h.nmax, Lmax, h.Nmax, b.Ub, P, b.sU));
    RSRR_HIP(colnorms(sm, P, Lmax, b.Ub, P, b.sU, b.un, (int)M));
    // factorisation
    RSRR_HIP(zero_int(sm, b.info, (int)M));
    LUWork w;
    w.ipiv = b.ipiv; w.sP = b.sP; w.perm = b.perm; w.sPerm = b.sPerm;
    w.info = b.info; w.inv = b.inv; w.sInv = b.sInv; w.tmp = b.tmp; w.sTmp = b.sTmp;
    w.pair = b.pair; w.sPair = b.sPair; w.ldpair = P;
    if (!from) {
        if (mixed) RSRR_HIP(getrf_batched<float>(sm, (float2*)b.T, b.sT, P, P, nb, w, (int)M));
        else RSRR_HIP(getrf_batched<double>(sm, (double2*)b.T, b.sT, P, P, nb, w, (int)M));
    }
    RSRR_HIP(ir_init(sm, (int)M, b.info, b.active, b.prev, b.resid, b.iters));
    w.active = b.active;
    // first solve
    if (mixed) {
        RSRR_HIP(scale_narrow(sm, P, Lmax, b.Ub, P, b.sU, b.ones, b.D64, P, b.sU, nullptr, (int)M));
        RSRR_HIP(solve_c64(sm, b, P, nb, w, Lmax, M));
        RSRR_HIP(widen(sm, P, Lmax, b.D64, P, b.sU, b.Xb, P, b.sU, (int)M));
    } else {
        RSRR_HIP(copy_c128(sm, P, Lmax, b.Ub, P, b.sU, b.Xb, P, b.sU, (int)M));
        RSRR_HIP(getrs_batched<double>(sm, (const double2*)b.T, b.sT, P, P, nb, w, b.Xb, b.sU, P, Lmax, (int)M));
    }
    // refinement with FP64 residuals, decisions on the device
    const double tol_be = c->ir_tol * 1.1102230246251565e-16 * std::sqrt((double)P);
    const int iters = mixed ? maxit : 0;
    for (int it = 0; it <= iters; ++it) {
        if (resid_skinny_ok(Lmax)) {
            // skinny: stream T once; points already decided are skipped
            RSRR_HIP(resid_skinny(sm, P, Lmax, b.T128, P, b.sT, b.Xb, P, b.sU, b.Ub, P, b.sU, b.R, P, b.sU,
                                  it == 0 ? nullptr : b.active, (int)M));
        } else {
            RSRR_HIP(copy_c128(sm, P, Lmax, b.Ub, P, b.sU, b.R, P, b.sU, (int)M));
            RSRR_HIP(zgemm(sm, 0, 0, P, Lmax, P, -1.0, b.T128, P, b.sT, b.Xb, P, b.sU, 1.0, b.R, P, b.sU, (int)M));
        }
        RSRR_HIP(colnorms(sm, P, Lmax, b.R, P, b.sU, b.rn, (int)M));
        RSRR_HIP(colnorms(sm, P, Lmax, b.Xb, P, b.sU, b.xn, (int)M));
        RSRR_HIP(ir_decide(sm, (int)M, Lmax, b.rn, b.xn, b.un, b.frob, tol_be, it, iters, b.active, b.prev, b.resid,
                           b.iters, b.inv_s, b.scl));
        if (it == iters) break;
        RSRR_HIP(scale_narrow(sm, P, Lmax, b.R, P, b.sU, b.inv_s, b.D64, P, b.sU, b.active, (int)M));
        RSRR_HIP(solve_c64(sm, b, P, nb, w, Lmax, M));
        RSRR_HIP(axpy_widen(sm, P, Lmax, b.D64, P, b.sU, b.scl, b.Xb, P, b.sU, b.active, (int)M));
    }
    // results into each instance's S, all instances in one launch
    RSRR_HIP(copy_out_group(sm, b.rhs, nins, h.nmax, Lmax, h.Nmax, b.Xb, P, b.sU));
    // factors kept on the device for later solves (same strides in the store)
    for (size_t q = 0; keep && q < ids.size(); ++q) {
        FactorStore* fs = keep[q];
        if (!fs) continue;
        const long cnt = off[q + 1] - off[q];
        const size_t k0 = (size_t)keep_k0[q];
        RSRR_HIP(hipMemcpyAsync((char*)fs->T + k0 * fs->sT * esz, (const char*)b.T + (size_t)off[q] * b.sT * esz,
                                (size_t)cnt * b.sT * esz, hipMemcpyDeviceToDevice, sm));
        RSRR_HIP(hipMemcpyAsync(fs->perm + k0 * fs->sPerm, b.perm + (size_t)off[q] * b.sPerm,
                                (size_t)cnt * b.sPerm * 8, hipMemcpyDeviceToDevice, sm));
        if (mixed)
            RSRR_HIP(hipMemcpyAsync((char*)fs->inv + k0 * fs->sInv * 8, (const char*)b.inv + (size_t)off[q] * b.sInv * 8,
                                    (size_t)cnt * b.sInv * 8, hipMemcpyDeviceToDevice, sm));
        fs->nb = nb;
    }
    return RSRR_OK;
}

}  // namespace

void batched_release(rsrr_ctx* c)
{
    std::lock_guard<std::mutex> lk(states_mu());
    auto& m = states();
    auto it = m.find(c);
    if (it == m.end()) return;
    if (it->second->graph && it->second->graph->exec) (void)hipGraphExecDestroy(it->second->graph->exec);
    if (it->second->cap_fork) (void)hipEventDestroy(it->second->cap_fork);
    for (int i = 0; i < N_BUCKET_STREAMS; ++i) {
        if (it->second->streams[i]) (void)hipStreamDestroy(it->second->streams[i]);
        if (it->second->done[i]) (void)hipEventDestroy(it->second->done[i]);
    }
    for (void* p : it->second->bufs)
        if (p) (void)hipFree(p);
    m.erase(it);
}

namespace {

// Host tables of one bucket (see BucketHost).
void bucket_tables(const rsrr_instance* inst, const std::vector<int>& ids, const std::vector<long>& off,
                   BucketHost& h)
{
    h.nk.assign(off.back(), 0);
    h.coef.clear();
    h.sep.clear();
    h.rhs.clear();
    h.nmax = h.Nmax = 0;
    bool all_sep = true;
    for (size_t q = 0; q < ids.size(); ++q) {
        const rsrr_instance& in = inst[ids[q]];
        for (long k = off[q]; k < off[q + 1]; ++k) h.nk[k] = in.nep.n;
        h.nmax = std::max(h.nmax, in.nep.n);
        h.Nmax = std::max(h.Nmax, in.N);
        RhsInstance r{};
        r.U = (const double2*)in.U; r.S = (double2*)in.S; r.koff = off[q];
        r.ldu = in.ldu; r.lds = in.lds; r.n = in.nep.n; r.L = in.L; r.N = in.N;
        h.rhs.push_back(r);
        if (in.nep.kind == RSRR_T_SEPARABLE) {
            SepInstance e{};
            e.A = (const double2*)in.nep.A; e.coff = (long)h.coef.size(); e.koff = off[q];
            e.lda = in.nep.lda; e.J = in.nep.J; e.n = in.nep.n; e.N = in.N;
            if (e.J > assemble_max_terms()) all_sep = false;
            h.sep.push_back(e);
            for (int j = 0; j < in.nep.J; ++j)
                for (int k = 0; k < in.N; ++k) {
                    const zd f = term_eval(in.nep.terms[j], zd(in.z[2 * k], in.z[2 * k + 1]));
                    h.coef.push_back(make_double2(f.real(), f.imag()));
                }
        } else {
            all_sep = false;
            for (int k = 0; k < in.N; ++k) h.coef.push_back(make_double2(in.z[2 * k], in.z[2 * k + 1]));
        }
    }
    if (!all_sep) h.sep.clear();
}

// The buffers of one bucket of M padded P x P matrices with Lmax right-hand sides,
// from the context's slots of bucket size P (with `from`, no factor buffers).
rsrr_status bucket_bufs(BatchedState& S, hipStream_t sm, int P, int Lmax, long M, int maxn, size_t ncoef, int nins,
                        bool mixed, bool from, BucketBufs& b)
{
    const int nbmax = mixed ? max_panel<float>() : max_panel<double>();
    b = BucketBufs{};
    b.sT = (long)P * P;
    b.sU = (long)P * Lmax;
    b.sP = P;
    b.sPerm = bucket_sPerm(P);
    // ceil(P/nb) panels of 2 nb^2 for any nb <= nbmax: at most 2 nbmax (P + nbmax)
    b.sInv = bucket_sInv(P, mixed);
    b.sTmp = mixed ? (long)nbmax * std::max(P, Lmax) : 0;
    b.sPair = mixed ? lu_pair_elems(P, nbmax, P) : 0;
    const size_t esz = mixed ? 8 : 16;
    const long nparts_max = ((long)maxn * maxn + 255) / 256;
    // every bucket size has its own buffers (graphs keep pointing at them, and the
    // buckets of one call run side by side)
    S.last_use[P] = S.calls;
    int s = (P / BUCKET) * 32;
    b.T = from ? (void*)(s++, nullptr) : bget(S, s++, (size_t)M * b.sT * esz, sm);
    b.T128 = (double2*)bget(S, s++, (size_t)M * b.sT * 16, sm);
    b.Ub = (double2*)bget(S, s++, (size_t)M * b.sU * 16, sm);
    b.Xb = (double2*)bget(S, s++, (size_t)M * b.sU * 16, sm);
    b.R = (double2*)bget(S, s++, (size_t)M * b.sU * 16, sm);
    b.D64 = (float2*)bget(S, s++, (size_t)M * b.sU * 8, sm);
    b.ipiv = (int*)bget(S, s++, (size_t)M * b.sP * 4, sm);
    b.perm = from ? (int2*)(s++, nullptr) : (int2*)bget(S, s++, (size_t)M * b.sPerm * 8, sm);
    b.info = (int*)bget(S, s++, (size_t)M * 4, sm);
    b.inv = mixed && !from ? bget(S, s++, (size_t)M * b.sInv * 8, sm) : (void*)(s++, nullptr);
    b.tmp = mixed ? bget(S, s++, (size_t)M * b.sTmp * 8, sm) : (void*)(s++, nullptr);
    b.nk = (int*)bget(S, s++, (size_t)M * 4, sm);
    b.coef = (double2*)bget(S, s++, ncoef * 16, sm);
    b.frobp = (double*)bget(S, s++, (size_t)M * nparts_max * 8, sm);
    b.frob = (double*)bget(S, s++, (size_t)M * 8, sm);
    b.un = (double*)bget(S, s++, (size_t)M * Lmax * 8, sm);
    b.rn = (double*)bget(S, s++, (size_t)M * Lmax * 8, sm);
    b.xn = (double*)bget(S, s++, (size_t)M * Lmax * 8, sm);
    b.inv_s = (double*)bget(S, s++, (size_t)M * Lmax * 8, sm);
    b.scl = (double*)bget(S, s++, (size_t)M * Lmax * 8, sm);
    b.active = (int*)bget(S, s++, (size_t)M * 4, sm);
    b.prev = (double*)bget(S, s++, (size_t)M * 8, sm);
    b.resid = (double*)bget(S, s++, (size_t)M * 8, sm);
    b.iters = (int*)bget(S, s++, (size_t)M * 4, sm);
    b.ones = (double*)bget(S, s++, (size_t)M * Lmax * 8, sm);
    b.pair = mixed && !from ? bget(S, s++, (size_t)M * b.sPair * 8, sm) : (void*)(s++, nullptr);
    b.sep = (SepInstance*)bget(S, s++, (size_t)nins * sizeof(SepInstance), sm);
    b.rhs = (RhsInstance*)bget(S, s++, (size_t)nins * sizeof(RhsInstance), sm);
    if ((!from && (!b.T || !b.perm || (mixed && (!b.inv || !b.pair)))) || !b.T128 || !b.Ub || !b.Xb || !b.R ||
        !b.D64 || !b.ipiv || !b.info || (mixed && !b.tmp) || !b.nk || !b.coef || !b.frobp || !b.frob ||
        !b.un || !b.rn || !b.xn || !b.inv_s || !b.scl || !b.active || !b.prev || !b.resid || !b.iters || !b.ones ||
        !b.sep || !b.rhs)
        return RSRR_ENOMEM;
    // the first solve narrows U with scale 1: ones in scl
    std::vector<double> ones((size_t)M * Lmax, 1.0);
    RSRR_HIP(hipMemcpyAsync(b.ones, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, sm));
    RSRR_HIP(hipStreamSynchronize(sm));
    return RSRR_OK;
}

struct Flags { int sing = 0, fb = 0, nan = 0; };

// Diagnostics of one bucket back to the host; points above the residual bar are
// redone in FP64.  info (may be null) is indexed by pbase[ids[q]] + k.
rsrr_status report_bucket(rsrr_ctx* c, const rsrr_instance* inst, const std::vector<int>& ids,
                          const std::vector<long>& off, long M, const int* dinfo, const int* diters,
                          const double* dres, const std::vector<long>& pbase, rsrr_point_info* info, Flags& f)
{
    std::vector<int> hinfo(M), hit(M);
    std::vector<double> hres(M);
    RSRR_HIP(hipMemcpyAsync(hinfo.data(), dinfo, (size_t)M * 4, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipMemcpyAsync(hit.data(), diters, (size_t)M * 4, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipMemcpyAsync(hres.data(), dres, (size_t)M * 8, hipMemcpyDeviceToHost, c->stream));
    RSRR_HIP(hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < ids.size(); ++q) {
        const rsrr_instance& in = inst[ids[q]];
        for (int k = 0; k < in.N; ++k) {
            const long m = off[q] + k;
            rsrr_point_info pi{};
            pi.info = hinfo[m];
            pi.ir_iters = hit[m];
            pi.resid = hres[m];
            if (hinfo[m] > 0) f.sing = 1;
            if (hinfo[m] < 0) f.nan = 1;
            if (hinfo[m] == 0 && !(hres[m] <= c->fallback_resid)) {
                // redo this point on the FP64 path
                rsrr_point_info fpi;
                const rsrr_status st = rsrr_sample(c, &in.nep, 1, in.z + 2 * k, in.U, in.L, in.ldu, RSRR_PREC_C128,
                                                   in.S + 2 * (size_t)k * in.L * in.lds, in.lds, &fpi);
                if (st < 0 || st == RSRR_EDEVICE || st == RSRR_ENOMEM) return st;
                pi.fallback = 1;
                pi.resid = fpi.resid;
                pi.info = fpi.info;
                f.fb = 1;
            }
            if (info) info[pbase[ids[q]] + k] = pi;
        }
    }
    return RSRR_OK;
}

rsrr_status validate(int count, const rsrr_instance* inst)
{
    for (int i = 0; i < count; ++i) {
        const rsrr_instance& in = inst[i];
        const rsrr_nep& e = in.nep;
        if (e.n < 1 || e.n > 8192) return -3;
        if (e.kind == RSRR_T_SEPARABLE) {
            if (e.J < 1 || e.J > 64 || !e.A || e.lda < e.n || !e.terms) return -3;
        } else if (e.kind == RSRR_T_HELMHOLTZ) {
            if (!e.points || !(e.w > 0)) return -3;
        } else {
            return -3;
        }
        if (in.N < 1 || !in.z || !in.U || in.L < 1 || in.ldu < e.n || !in.S || in.lds < e.n) return -3;
    }
    return RSRR_OK;
}

rsrr_status batched_impl(rsrr_ctx* c, int count, const rsrr_instance* inst, int prec, int flags,
                         rsrr_point_info* info, FactorStore* const* keep, const int* keep_k0)
{
    RSRR_HIP(hipSetDevice(c->device));
    masked_stream_release(c);  // a CU-masked stream would cost the buckets' streams their concurrency
    BatchedState& S = state_of(c);
    ++S.calls;
    load_tune_file(S, c->device);
    const bool use_graph = (flags & RSRR_BATCH_GRAPH) != 0 && !keep;
    const bool autotune = (flags & RSRR_BATCH_AUTOTUNE) != 0;
    const bool mixed = prec == RSRR_PREC_C64_IR;

    // point offsets of the instances in the caller's order (for info)
    std::vector<long> pbase(count + 1, 0);
    for (int i = 0; i < count; ++i) pbase[i + 1] = pbase[i] + inst[i].N;

    // buckets
    std::map<int, std::vector<int>> buckets;
    for (int i = 0; i < count; ++i) buckets[(inst[i].nep.n + BUCKET - 1) / BUCKET * BUCKET].push_back(i);

    Flags fl;
    // Every bucket has its own buffers; the buckets run side by side on a pool of
    // streams (replayed graphs or eager launches) and report after all of them.  The
    // host tables of eager launches stay alive in `pending` until then.
    struct Pending {
        std::vector<int> ids; std::vector<long> off; long M; int* info; int* iters; double* resid;
        BucketHost h; std::vector<FactorStore*> keep; std::vector<int> k0;
    };
    std::vector<Pending> pending;
    if (!S.streams[0]) {
        for (int i = 0; i < N_BUCKET_STREAMS; ++i) {
            RSRR_HIP(hipStreamCreateWithFlags(&S.streams[i], hipStreamNonBlocking));
            RSRR_HIP(hipEventCreateWithFlags(&S.done[i], hipEventDisableTiming));
        }
        RSRR_HIP(hipEventCreateWithFlags(&S.cap_fork, hipEventDisableTiming));
    }
    int nlaunched = 0;
    // on every return the launched buckets have finished before `pending` (host tables) goes away
    struct Drain {
        BatchedState& S; const int& n;
        ~Drain() { for (int i = 0; i < std::min(n, N_BUCKET_STREAMS); ++i) (void)hipStreamSynchronize(S.streams[i]); }
    } drain{S, nlaunched};
    // Longest processing time first: buckets in decreasing order of their LU work
    // (matrices x P^3), each on the stream with the least work assigned so far, so
    // the largest bucket's long chain starts first instead of running alone at the end.
    int nstreams = N_BUCKET_STREAMS;
    if (const char* e = std::getenv("RSRR_BUCKET_STREAMS")) nstreams = std::max(1, std::min(N_BUCKET_STREAMS, std::atoi(e)));
    std::vector<std::pair<double, int>> order;  // (work, P)
    for (auto& kv : buckets) {
        long pts = 0;
        for (int id : kv.second) pts += inst[id].N;
        order.push_back({(double)pts * kv.first * (double)kv.first * kv.first, kv.first});
    }
    std::stable_sort(order.begin(), order.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first > b.first;
    });
    std::vector<double> load(nstreams, 0.0);
    auto next_stream = [&](double work) {
        int s = 0;
        for (int i = 1; i < nstreams; ++i)
            if (load[i] < load[s]) s = i;
        load[s] += work;
        return s;
    };
    // graph mode: the buckets' plans, captured together after the loop
    struct Plan {
        std::vector<int> ids; std::vector<long> off; long M; int P, Lmax, nb, tile, sidx; BucketBufs b;
        BucketHost h;
    };
    std::vector<Plan> plans;
    std::vector<unsigned long long> gkey;
    const int maxit = c->ir_max_iters_batched;
    for (auto& ow : order) {
        const int P = ow.second;
        const std::vector<int>& ids = buckets[P];
        std::vector<long> off(ids.size() + 1, 0);
        int Lmax = 0, maxn = 0;
        for (size_t q = 0; q < ids.size(); ++q) {
            off[q + 1] = off[q] + inst[ids[q]].N;
            Lmax = std::max(Lmax, inst[ids[q]].L);
            maxn = std::max(maxn, inst[ids[q]].nep.n);
        }
        const long M = off.back();
        BucketHost h;
        bucket_tables(inst, ids, off, h);
        const int nbmax = mixed ? max_panel<float>() : max_panel<double>();
        BucketBufs b{};
        hipStream_t sm = c->stream;
        rsrr_status bs = bucket_bufs(S, sm, P, Lmax, M, maxn, h.coef.size(), (int)ids.size(), mixed, false, b);
        if (bs) return bs;

        // panel width and update tile: tuned (each candidate timed with one bucket pass) or default
        const long tkey = (long)P * 2 + (mixed ? 1 : 0);
        int nb = mixed ? std::min(c->nb_c64, nbmax) : std::min(c->nb_c128, nbmax);
        int tile = UPD_TILE_3M_128x64;
        auto tu = S.tuned.find(tkey);
        if (tu != S.tuned.end()) {
            nb = tu->second.nb;
            tile = tu->second.tile;
        } else if (autotune) {
            std::vector<int> nbs = mixed ? std::vector<int>{32, 64, 128} : std::vector<int>{32, 64};
            std::vector<int> tiles = mixed ? std::vector<int>{UPD_TILE_3M_128x64, UPD_TILE_3M_64x64,
                                                              UPD_TILE_4M_128x128, UPD_TILE_4M_64x64}
                                           : std::vector<int>{UPD_TILE_3M_128x64};
            float best = 1e30f;
            Tuned bt;
            bt.nb = nb;
            hipEvent_t e0, e1;
            RSRR_HIP(hipEventCreate(&e0));
            RSRR_HIP(hipEventCreate(&e1));
            for (int cb : nbs) {
                if (cb > nbmax) continue;
                for (int ct : tiles) {
                    // one full bucket pass (assembly, LU, one solve, one residual) per candidate
                    TileScope ts(ct);
                    RSRR_HIP(hipEventRecord(e0, sm));
                    rsrr_status st = run_bucket(c, sm, inst, ids, off, P, Lmax, M, prec, cb, b, h, 0);
                    if (st) return st;
                    RSRR_HIP(hipEventRecord(e1, sm));
                    RSRR_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    RSRR_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) { best = ms; bt.nb = cb; bt.tile = ct; bt.ms = ms; }
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            nb = bt.nb;
            tile = bt.tile;
            S.tuned[tkey] = bt;
            save_tune_file(S);
        }
        TileScope tile_scope(tile);

        if (use_graph) {
            // key: everything the captured work depends on
            gkey.push_back((unsigned long long)P);
            gkey.push_back((unsigned long long)prec);
            gkey.push_back((unsigned long long)nb);
            gkey.push_back((unsigned long long)tile);
            gkey.push_back((unsigned long long)M);
            gkey.push_back((unsigned long long)maxit);
            unsigned long long tolbits;
            std::memcpy(&tolbits, &c->ir_tol, 8);
            gkey.push_back(tolbits);
            for (int id : ids) {
                const rsrr_instance& in = inst[id];
                gkey.push_back((unsigned long long)(uintptr_t)in.nep.A);
                gkey.push_back((unsigned long long)(uintptr_t)in.nep.points);
                gkey.push_back((unsigned long long)(uintptr_t)in.U);
                gkey.push_back((unsigned long long)(uintptr_t)in.S);
                gkey.push_back(((unsigned long long)in.nep.n << 32) | (unsigned)in.N);
                gkey.push_back(((unsigned long long)in.L << 32) | (unsigned)in.lds);
            }
            plans.push_back(Plan{ids, off, M, P, Lmax, nb, tile, next_stream(ow.first), b, std::move(h)});
        } else {
            hipStream_t ps = S.streams[next_stream(ow.first)];
            RSRR_HIP(hipEventRecord(c->fork, c->stream));
            RSRR_HIP(hipStreamWaitEvent(ps, c->fork, 0));
            std::vector<FactorStore*> kq;
            std::vector<int> k0q;
            if (keep)
                for (int id : ids) { kq.push_back(keep[id]); k0q.push_back(keep_k0[id]); }
            pending.push_back(Pending{ids, off, M, b.info, b.iters, b.resid, std::move(h), std::move(kq),
                                      std::move(k0q)});
            Pending& pd = pending.back();
            rsrr_status st = run_bucket(c, ps, inst, ids, off, P, Lmax, M, prec, nb, b, pd.h, maxit,
                                        keep ? pd.keep.data() : nullptr, keep ? pd.k0.data() : nullptr);
            if (st) return st;
            ++nlaunched;
        }
    }
    if (use_graph && !plans.empty()) {
        auto same = [](const auto& x, const auto& y) {
            return x.size() == y.size() && std::memcmp(x.data(), y.data(), x.size() * sizeof(x[0])) == 0;
        };
        bool hit = S.graph && S.graph->key == gkey && S.graph->host.size() == plans.size();
        for (size_t i = 0; hit && i < plans.size(); ++i) {
            const BucketHost &x = S.graph->host[i], &y = plans[i].h;
            hit = same(x.coef, y.coef) && same(x.nk, y.nk) && same(x.sep, y.sep) && same(x.rhs, y.rhs);
        }
        // the tables go to the device outside the graph, before every replay (another call
        // may have used the same bucket buffers since the capture)
        for (Plan& pl : plans) RSRR_HIP(upload_tables(c->stream, pl.h, pl.b));
        if (!hit) {
            if (S.graph && S.graph->exec) (void)hipGraphExecDestroy(S.graph->exec);
            S.graph = std::make_unique<GraphEntry>();
            GraphEntry& ge = *S.graph;
            ge.key = gkey;
            for (Plan& pl : plans) ge.host.push_back(pl.h);
            // capture: fork from the capture stream onto the bucket streams, every bucket
            // on its stream, join back
            RSRR_HIP(hipEventRecord(c->fork, c->stream));
            RSRR_HIP(hipStreamWaitEvent(c->aux, c->fork, 0));
            RSRR_HIP(hipStreamBeginCapture(c->aux, hipStreamCaptureModeThreadLocal));
            rsrr_status st = RSRR_OK;
            hipError_t ce = hipEventRecord(S.cap_fork, c->aux);
            std::vector<char> used(N_BUCKET_STREAMS, 0);
            for (size_t i = 0; i < plans.size() && st == RSRR_OK && ce == hipSuccess; ++i) {
                Plan& pl = plans[i];
                hipStream_t ps = S.streams[pl.sidx];
                if (!used[pl.sidx]) {
                    ce = hipStreamWaitEvent(ps, S.cap_fork, 0);
                    used[pl.sidx] = 1;
                    if (ce != hipSuccess) break;
                }
                TileScope ts(pl.tile);
                st = run_bucket(c, ps, inst, pl.ids, pl.off, pl.P, pl.Lmax, pl.M, prec, pl.nb, pl.b, ge.host[i],
                                maxit, nullptr, nullptr, nullptr, 0, false);
            }
            for (int i = 0; i < N_BUCKET_STREAMS; ++i) {
                if (!used[i]) continue;
                // every forked stream is joined back, also after an error, so the capture ends
                (void)hipEventRecord(S.done[i], S.streams[i]);
                (void)hipStreamWaitEvent(c->aux, S.done[i], 0);
            }
            hipGraph_t g = nullptr;
            const hipError_t ee = hipStreamEndCapture(c->aux, &g);
            if (st || ce != hipSuccess || ee != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                S.graph.reset();
                return st ? st : RSRR_EDEVICE;
            }
            const hipError_t ie = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) { S.graph.reset(); return RSRR_EDEVICE; }
        }
        // one launch for the whole call, after everything enqueued on the context stream so far
        RSRR_HIP(hipEventRecord(c->fork, c->stream));
        RSRR_HIP(hipStreamWaitEvent(c->aux, c->fork, 0));
        RSRR_HIP(hipGraphLaunch(S.graph->exec, c->aux));
        RSRR_HIP(hipEventRecord(c->join, c->aux));
        RSRR_HIP(hipStreamWaitEvent(c->stream, c->join, 0));
        for (const Plan& pl : plans) {
            const rsrr_status st = report_bucket(c, inst, pl.ids, pl.off, pl.M, pl.b.info, pl.b.iters, pl.b.resid,
                                                 pbase, info, fl);
            if (st) return st;
        }
    }
    if (!pending.empty()) {
        for (int i = 0; i < std::min(nlaunched, N_BUCKET_STREAMS); ++i) {
            RSRR_HIP(hipEventRecord(S.done[i], S.streams[i]));
            RSRR_HIP(hipStreamWaitEvent(c->stream, S.done[i], 0));
        }
        for (const Pending& pd : pending) {
            const rsrr_status st = report_bucket(c, inst, pd.ids, pd.off, pd.M, pd.info, pd.iters, pd.resid, pbase,
                                                 info, fl);
            if (st) return st;
        }
    }
    if (fl.nan) return RSRR_ENAN;
    if (fl.sing) return RSRR_ESINGULAR;
    if (fl.fb) return RSRR_WARN_FALLBACK;
    return RSRR_OK;
}

}  // namespace

extern "C" rsrr_status rsrr_sample_batched(rsrr_ctx* c, int count, const rsrr_instance* inst, int prec, int flags,
                                           rsrr_point_info* info)
{
    if (!c) return -1;
    if (count < 1) return -2;
    if (!inst) return -3;
    if (prec != RSRR_PREC_C128 && prec != RSRR_PREC_C64_IR) return -4;
    const rsrr_status v = validate(count, inst);
    if (v) return v;
    return batched_impl(c, count, inst, prec, flags, info, nullptr, nullptr);
}

rsrr_status sample_batched_keep(rsrr_ctx* c, int count, const rsrr_instance* inst, int prec, rsrr_point_info* info,
                                FactorStore* const* keep, const int* k0)
{
    if (!c || count < 1 || !inst || !keep || !k0) return -1;
    const rsrr_status v = validate(count, inst);
    if (v) return v;
    for (int i = 0; i < count; ++i)
        if (keep[i] && (keep[i]->P != (inst[i].nep.n + BUCKET - 1) / BUCKET * BUCKET || keep[i]->prec != prec ||
                        k0[i] < 0 || k0[i] + inst[i].N > keep[i]->N))
            return -3;
    return batched_impl(c, count, inst, prec, 0, info, keep, k0);
}

rsrr_status solve_from_store(rsrr_ctx* c, const rsrr_instance& in, const FactorStore& fs, int k0,
                             rsrr_point_info* info)
{
    if (!c) return -1;
    if (validate(1, &in)) return -2;
    const int P = (in.nep.n + BUCKET - 1) / BUCKET * BUCKET;
    if (fs.P != P || fs.nb < MIN_NB || k0 < 0 || k0 + in.N > fs.N) return -3;
    RSRR_HIP(hipSetDevice(c->device));
    BatchedState& S = state_of(c);
    ++S.calls;
    const bool mixed = fs.prec == RSRR_PREC_C64_IR;
    std::vector<int> ids{0};
    std::vector<long> off{0, in.N};
    BucketHost h;
    bucket_tables(&in, ids, off, h);
    BucketBufs b{};
    rsrr_status st = bucket_bufs(S, c->stream, P, in.L, in.N, in.nep.n, h.coef.size(), 1, mixed, true, b);
    if (st) return st;
    st = run_bucket(c, c->stream, &in, ids, off, P, in.L, in.N, fs.prec, fs.nb, b, h, c->ir_max_iters_batched,
                    nullptr, nullptr, &fs, k0);
    if (st) return st;
    Flags fl;
    std::vector<long> pbase{0, in.N};
    st = report_bucket(c, &in, ids, off, in.N, b.info, b.iters, b.resid, pbase, info, fl);
    if (st) return st;
    if (fl.nan) return RSRR_ENAN;
    if (fl.sing) return RSRR_ESINGULAR;
    if (fl.fb) return RSRR_WARN_FALLBACK;
    return RSRR_OK;
}

size_t factor_store_bytes(int n, int N, int prec)
{
    const int P = (n + BUCKET - 1) / BUCKET * BUCKET;
    const bool mixed = prec == RSRR_PREC_C64_IR;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al((size_t)N * P * P * (mixed ? 8 : 16)) + al((size_t)N * bucket_sPerm(P) * 8) +
           al((size_t)N * bucket_sInv(P, mixed) * 8);
}

FactorStore factor_store_at(void* base, int n, int N, int prec)
{
    const int P = (n + BUCKET - 1) / BUCKET * BUCKET;
    const bool mixed = prec == RSRR_PREC_C64_IR;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    FactorStore f;
    f.P = P;
    f.N = N;
    f.prec = prec;
    f.sT = (long)P * P;
    f.sPerm = bucket_sPerm(P);
    f.sInv = bucket_sInv(P, mixed);
    char* p = (char*)base;
    f.T = p;
    p += al((size_t)N * f.sT * (mixed ? 8 : 16));
    f.perm = (int2*)p;
    p += al((size_t)N * f.sPerm * 8);
    f.inv = mixed ? (void*)p : nullptr;
    return f;
}

void batched_trim(rsrr_ctx* c, size_t keep_bytes)
{
    std::lock_guard<std::mutex> lk(states_mu());
    auto it = states().find(c);
    if (it == states().end()) return;
    BatchedState& S = *it->second;
    size_t tot = 0;
    for (size_t x : S.sizes) tot += x;
    if (tot <= keep_bytes) return;
    // free whole bucket sizes, least recently used first; the sizes of the last call stay
    // unless nothing else is left to free
    std::vector<std::pair<long, int>> order;  // (last use, P)
    for (auto& kv : S.last_use) order.push_back({kv.second, kv.first});
    std::sort(order.begin(), order.end());
    (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < N_BUCKET_STREAMS; ++i)
        if (S.streams[i]) (void)hipStreamSynchronize(S.streams[i]);
    for (int pass = 0; pass < 2 && tot > keep_bytes; ++pass) {
        for (auto& u : order) {
            if (tot <= keep_bytes) break;
            if (pass == 0 && u.first == S.calls) continue;
            const int P = u.second;
            // the captured graph points at every bucket's buffers
            if (S.graph) {
                if (S.graph->exec) (void)hipGraphExecDestroy(S.graph->exec);
                S.graph.reset();
            }
            const int s0 = (P / BUCKET) * 32;
            for (int sl = s0; sl < s0 + 32 && sl < (int)S.bufs.size(); ++sl) {
                if (S.bufs[sl]) (void)hipFree(S.bufs[sl]);
                tot -= S.sizes[sl];
                S.bufs[sl] = nullptr;
                S.sizes[sl] = 0;
            }
        }
    }
}
