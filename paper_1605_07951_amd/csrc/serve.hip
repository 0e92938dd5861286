// C ABI: a request loop that runs the whole RSRR method (Sec. 4.3) for many
// NEPs on one device, with continuous batching of their sampling points.
//
// Two host threads, each with its own rsrr_ctx on its own non-blocking
// stream:
//   sampler  admits queued requests (free slot + room for the request's whole
//            footprint in the arena: S, kept LU factors, Q, V; first come,
//            first served), then repeatedly takes sampling points from all
//            admitted requests in admission order, up to batch_bytes of LU
//            workspace, and runs them as one batched sampling call per probe
//            count L (inside it, one uniform batch per size bucket), which also
//            copies each point's factors into its request's block.  Requests
//            that arrive meanwhile join the next launch.
//   solver   runs basis, projection and SS-FULL of each request whose points
//            are all sampled; when the gap test fails or an eigenpair inside
//            has a large residual, solves the request's reserve probe columns
//            with the kept factors (no refactorisation) and runs Steps 3-5
//            again; copies the eigenpairs to the caller's host arrays and frees
//            the request's arena block (which may admit the next request).
//            Its kernels overlap the next sampling launches.
// The arena is one hipMalloc'd block sub-allocated first-fit, so admission
// decides on real HBM and the loop never calls hipMalloc/hipFree per request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace rsrr;

namespace {

constexpr int DEFAULT_NQ = 500;
constexpr int DEFAULT_KQ = 2;
constexpr int MAX_TERMS = 64;
constexpr size_t ALIGN = 256;
constexpr double REPROBE_RESID = 1e-10;   // eigen-residual bar inside the contour
constexpr size_t DEFAULT_SOLVE_BYTES = (size_t)4 << 30;

size_t al(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// The request's arena block: S | factors | Q | V.
struct Layout {
    size_t s, fac, q, v, total;
};
Layout layout_of(const rsrr_request& r, int prec)
{
    const size_t n = (size_t)r.nep.n, NL = (size_t)r.N * (r.L + r.L_extra);
    Layout l;
    l.s = al(n * NL * 16);
    l.fac = al(factor_store_bytes(r.nep.n, r.N, prec));
    l.q = al(n * std::min(n, NL) * 16);
    l.v = al(n * (size_t)r.max_eigs * 16);
    l.total = l.s + l.fac + l.q + l.v;
    return l;
}

// First-fit sub-allocator over [0, size).
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0, used = 0, peak = 0;
    void init(size_t s)
    {
        size = s;
        free_.clear();
        if (s) free_[0] = s;
    }
    long alloc(size_t bytes)
    {
        bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used += bytes;
            peak = std::max(peak, used);
            return (long)off;
        }
        return -1;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum ReqState { QUEUED, ADMITTED, SAMPLED, DONE };

struct Req {
    int id = 0;
    rsrr_request r{};
    std::vector<rsrr_term> terms;  // copy of the caller's term table
    std::vector<double> z;         // contour nodes (2N)
    Layout lay{};
    size_t s_off = 0, s_bytes = 0; // the whole arena block
    double* S = nullptr;           // n x N*(L + L_extra) in the arena: N*L initial columns, then N*L_extra
    FactorStore fs;                // kept factors of the N points
    double* Q = nullptr;           // n x min(n, N*(L + L_extra))
    double* V = nullptr;           // n x max_eigs
    int next = 0;                  // first point not yet handed to a launch
    int sampled = 0;               // points finished
    int last_launch = -1;
    ReqState state = QUEUED;
    rsrr_result res{};
};

struct Chunk {
    Req* q;
    int k0, cnt;
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool is_error(rsrr_status s) { return s < 0 || s == RSRR_ENOMEM || s == RSRR_EDEVICE || s == RSRR_ENOTCONV || s == RSRR_ENAN || s == RSRR_ESINGULAR || s == RSRR_ELIMIT; }

// Request checks shared by rsrr_server_submit and rsrr_server_footprint.
bool request_ok(const rsrr_request* r)
{
    const rsrr_nep& e = r->nep;
    if (e.n < 1 || e.n > 8192) return false;
    if (e.kind == RSRR_T_SEPARABLE) {
        if (e.J < 1 || e.J > MAX_TERMS || !e.A || e.lda < e.n || !e.terms) return false;
    } else if (e.kind == RSRR_T_HELMHOLTZ) {
        if (!e.points || !(e.w > 0)) return false;
    } else {
        return false;
    }
    return r->a > 0 && r->b > 0 && r->N >= 1 && r->L >= 1 && r->L_extra >= 0 && r->U && r->ldu >= e.n &&
           r->max_eigs >= 1 && r->lambda && r->NQ >= 0 && r->KQ >= 0 &&
           !(r->NQ > 0 && r->NQ < 2 * std::max(r->KQ, 1) + 1) && r->delta >= 0 && r->delta < 1;
}

// LU workspace of one point in a sampling launch (the bucket buffers of
// rsrr_sample_batched), bytes.
size_t point_bytes(int n, int L, bool mixed)
{
    const size_t P = (size_t)(n + 63) / 64 * 64;
    const size_t npan = (size_t)perm_panels((int)P);
    size_t b = P * P * (mixed ? 8 + 16 : 16 + 16);           // T and its FP64 copy
    b += P * (size_t)L * (3 * 16 + 8) + P * 4;               // U, X, R, narrow RHS, pivots
    b += npan * 2 * MAX_NB * 8;                               // permutations
    if (mixed) b += 2 * MAX_NB * (P + MAX_NB) * 8 + MAX_NB * std::max(P, (size_t)L) * 8;  // inverses, scratch
    b += (P * P + 255) / 256 * 8 + (size_t)L * 6 * 8 + 64;   // norms and refinement state
    return b;
}

}  // namespace

// A host thread's device context: its stream, rsrr_ctx and the post-step
// buffers it grows on demand.
struct Worker {
    hipStream_t st = nullptr;
    rsrr_ctx* c = nullptr;
    void* aq_buf = nullptr; size_t aq_cap = 0;  // projected matrices (within solve_bytes)
    std::thread th;
};

struct rsrr_server {
    rsrr_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    Worker ws;                        // sampling thread
    std::vector<std::unique_ptr<Worker>> wp;  // solve threads
    void* arena_base = nullptr;
    Arena arena;

    std::mutex mu;
    std::condition_variable cv_work;  // sampler: new request / freed slot / stop
    std::condition_variable cv_post;  // solver: sampled request / stop
    std::condition_variable cv_done;  // waiters
    std::map<int, std::unique_ptr<Req>> reqs;
    std::deque<Req*> queue;           // waiting for admission
    std::vector<Req*> admitted;       // points left to sample, admission order
    std::deque<Req*> post;            // sampled, waiting for basis/projection/solve
    int active = 0;                   // admitted and not finished
    int next_id = 1;
    bool stop = false;
    int posting = 0;                  // requests inside the solve step

    // counters
    long finished = 0, points = 0, launches = 0, max_launch = 0, repoints = 0, reprobes = 0;
    double busy_s = 0.0, busy_p = 0.0;
    size_t mem_peak = 0;

};

namespace {

void* grow(void*& p, size_t& cap, size_t bytes)
{
    if (bytes <= cap && p) return p;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return nullptr;
    }
    cap = bytes;
    return p;
}

void note_status(rsrr_result& r, rsrr_status s)
{
    if (s == RSRR_OK) return;
    if (r.status == RSRR_OK || (!is_error(r.status) && is_error(s))) r.status = s;
}

// Solve the reserve probe columns of every point from the kept factors into the
// columns N*L .. N*(L + L_extra) - 1 of S, in chunks of points sized to the
// solve thread's budget; the chunk buffers are released afterwards.
rsrr_status reprobe(rsrr_server* s, Worker* w, Req* q)
{
    const rsrr_request& r = q->r;
    const int n = r.nep.n, Lx = r.L_extra;
    const bool mixed = s->cfg.prec == RSRR_PREC_C64_IR;
    const size_t per = point_bytes(n, Lx, mixed);
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)r.N, s->cfg.solve_bytes / per));
    rsrr_status st = RSRR_OK;
    std::vector<rsrr_point_info> pi(chunk);
    for (int k0 = 0; k0 < r.N; k0 += chunk) {
        rsrr_instance in{};
        in.nep = r.nep;
        in.nep.terms = q->terms.empty() ? nullptr : q->terms.data();
        in.N = std::min(chunk, r.N - k0);
        in.z = q->z.data() + 2 * (size_t)k0;
        in.U = r.U + 2 * (size_t)r.L * r.ldu;
        in.L = Lx;
        in.ldu = r.ldu;
        in.S = q->S + 2 * ((size_t)r.N * r.L + (size_t)k0 * Lx) * n;
        in.lds = n;
        const rsrr_status e = solve_from_store(w->c, in, q->fs, k0, pi.data());
        if (e && (st == RSRR_OK || is_error(e))) st = e;
        if (is_error(e)) break;
        for (int k = 0; k < in.N; ++k) {
            q->res.fallbacks += pi[k].fallback;
            q->res.ir_iters_max = std::max(q->res.ir_iters_max, pi[k].ir_iters);
            if (pi[k].resid > q->res.sample_resid_max) q->res.sample_resid_max = pi[k].resid;
        }
    }
    batched_trim(w->c, 0);
    return st;
}

// Basis, projection, SS-FULL and the copy of the eigenpairs to the host (RSRR
// Steps 3-5) for one sampled request, on context c; a re-probe from the kept
// factors when the first pass fails its checks.
void finish_request(rsrr_server* s, Worker* w, Req* q)
{
    rsrr_ctx* c = w->c;
    hipStream_t st = w->st;
    rsrr_result& res = q->res;
    if (is_error(res.status) && res.status != RSRR_ESINGULAR) return;
    const rsrr_request& r = q->r;
    const int n = r.nep.n;
    const int kmax = (int)std::min<long>(n, (long)r.N * (r.L + r.L_extra));
    const double gam[2] = {r.gamma_re, r.gamma_im};
    const double rho = std::max(r.a, r.b);
    std::vector<double> resid(r.max_eigs, 0.0);
    double* rout = r.resid ? r.resid : resid.data();
    res.L_used = r.L;
    for (;;) {
        const int NL = r.N * res.L_used;
        int k = 0;
        rsrr_status e = rsrr_basis(c, n, NL, q->S, n, r.delta > 0 ? r.delta : c->delta, q->Q, n, kmax, &k, nullptr);
        note_status(res, e);
        if (is_error(e)) return;
        res.k = k;
        if (k < 1) return;
        const int maxt = r.nep.kind == RSRR_T_SEPARABLE ? r.nep.J : MAX_TERMS;
        const size_t aq_bytes = (size_t)maxt * k * k * 16;
        if (aq_bytes > s->cfg.solve_bytes) { note_status(res, RSRR_ENOMEM); return; }
        double2* AQ = (double2*)grow(w->aq_buf, w->aq_cap, aq_bytes);
        if (!AQ) { note_status(res, RSRR_ENOMEM); return; }
        std::vector<rsrr_term> tout(maxt);
        int J_eff = 0;
        e = rsrr_project(c, &r.nep, q->Q, n, k, gam, rho, (double*)AQ, maxt, &J_eff, tout.data());
        note_status(res, e);
        if (is_error(e)) return;
        int count = 0;
        rsrr_solve_info si{};
        e = rsrr_solve(c, &r.nep, k, (const double*)AQ, J_eff, tout.data(), q->Q, n, gam, r.a, r.b,
                       r.NQ > 0 ? r.NQ : DEFAULT_NQ, r.KQ > 0 ? r.KQ : DEFAULT_KQ, c->tol_gap, r.max_eigs, r.lambda,
                       q->V, n, rout, &count, nullptr, &si);
        if (is_error(e)) { note_status(res, e); return; }
        res.count = count;
        res.nbar = si.nbar;
        // the paper's remedy for a failed gap test or inaccurate pairs: more probe columns
        bool bad_pair = false;
        for (int i = 0; i < count; ++i) {
            const double dx = (r.lambda[2 * i] - r.gamma_re) / r.a, dy = (r.lambda[2 * i + 1] - r.gamma_im) / r.b;
            if (dx * dx + dy * dy < 1.0 && !(rout[i] <= REPROBE_RESID)) bad_pair = true;
        }
        if ((si.warn_gap || bad_pair) && r.L_extra > 0 && res.L_used == r.L) {
            const rsrr_status pe = reprobe(s, w, q);
            if (is_error(pe)) { note_status(res, pe); return; }
            if (pe == RSRR_WARN_FALLBACK) note_status(res, pe);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->repoints += r.N;
                ++s->reprobes;
            }
            res.reprobes = 1;
            res.L_used = r.L + r.L_extra;
            continue;
        }
        note_status(res, e);
        break;
    }
    if (r.V && res.count > 0) {
        if (hipMemcpyAsync(r.V, q->V, (size_t)n * res.count * 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            note_status(res, RSRR_EDEVICE);
    }
}

// Called with s->mu held: admit queued requests while a slot and arena room exist.
void admit_locked(rsrr_server* s)
{
    while (!s->queue.empty() && s->active < s->cfg.max_slots) {
        Req* q = s->queue.front();
        const long off = s->arena.alloc(q->s_bytes);
        if (off < 0) break;  // first come first served: wait for room
        s->queue.pop_front();
        q->s_off = (size_t)off;
        char* base = (char*)s->arena_base + off;
        q->S = (double*)base;
        q->fs = factor_store_at(base + q->lay.s, q->r.nep.n, q->r.N, s->cfg.prec);
        q->Q = (double*)(base + q->lay.s + q->lay.fac);
        q->V = (double*)(base + q->lay.s + q->lay.fac + q->lay.q);
        q->state = ADMITTED;
        q->res.t_admit = now_s(s->t0);
        s->admitted.push_back(q);
        ++s->active;
    }
}

// Called with s->mu held: the next launch's points.
std::vector<Chunk> pick_locked(rsrr_server* s)
{
    std::vector<Chunk> out;
    const bool mixed = s->cfg.prec == RSRR_PREC_C64_IR;
    size_t used = 0;
    for (Req* q : s->admitted) {
        if (q->next >= q->r.N) continue;
        const size_t bp = point_bytes(q->r.nep.n, q->r.L, mixed);
        long room = used < s->cfg.batch_bytes ? (long)((s->cfg.batch_bytes - used) / bp) : 0;
        if (room <= 0) {
            if (!out.empty()) break;
            room = 1;  // a point larger than the cap still runs, alone
        }
        const int cnt = (int)std::min<long>(q->r.N - q->next, room);
        out.push_back({q, q->next, cnt});
        q->next += cnt;
        used += (size_t)cnt * bp;
        if (s->cfg.flags & RSRR_SERVE_NO_BATCH) break;
    }
    return out;
}

// One sampling launch: rsrr_sample_batched per probe count L.
void run_launch(rsrr_server* s, const std::vector<Chunk>& ch, std::vector<std::vector<rsrr_point_info>>& infos,
                std::vector<rsrr_status>& codes)
{
    infos.assign(ch.size(), {});
    codes.assign(ch.size(), RSRR_OK);
    std::map<int, std::vector<int>> byL;
    for (size_t i = 0; i < ch.size(); ++i) byL[ch[i].q->r.L].push_back((int)i);
    for (auto& kv : byL) {
        std::vector<rsrr_instance> inst;
        std::vector<FactorStore*> keep;
        std::vector<int> k0;
        long tot = 0;
        for (int i : kv.second) {
            const Chunk& c = ch[i];
            const rsrr_request& r = c.q->r;
            rsrr_instance in{};
            in.nep = r.nep;
            in.nep.terms = c.q->terms.empty() ? nullptr : c.q->terms.data();
            in.N = c.cnt;
            in.z = c.q->z.data() + 2 * (size_t)c.k0;
            in.U = r.U;
            in.L = r.L;
            in.ldu = r.ldu;
            in.S = c.q->S + 2 * (size_t)c.k0 * r.L * r.nep.n;
            in.lds = r.nep.n;
            inst.push_back(in);
            keep.push_back(&c.q->fs);
            k0.push_back(c.k0);
            tot += c.cnt;
        }
        std::vector<rsrr_point_info> pi(tot);
        const rsrr_status e = sample_batched_keep(s->ws.c, (int)inst.size(), inst.data(), s->cfg.prec, pi.data(),
                                                  keep.data(), k0.data());
        long p = 0;
        for (int i : kv.second) {
            infos[i].assign(pi.begin() + p, pi.begin() + p + ch[i].cnt);
            p += ch[i].cnt;
            if (e < 0 || e == RSRR_ENOMEM || e == RSRR_EDEVICE || e == RSRR_ENAN) {
                codes[i] = e;
            } else {
                // per request: ESINGULAR only where one of its own points had a zero pivot
                for (const auto& x : infos[i]) {
                    if (x.info > 0) codes[i] = RSRR_ESINGULAR;
                    else if (x.fallback && codes[i] == RSRR_OK) codes[i] = RSRR_WARN_FALLBACK;
                }
            }
        }
    }
}

void complete_locked(rsrr_server* s, Req* q)
{
    s->arena.release(q->s_off, q->s_bytes);
    q->S = nullptr;
    q->state = DONE;
    q->res.t_done = now_s(s->t0);
    --s->active;
    ++s->finished;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

void post_one(rsrr_server* s, Worker* w, std::unique_lock<std::mutex>& lk)
{
    Req* q = s->post.front();
    s->post.pop_front();
    ++s->posting;
    lk.unlock();
    const auto t = std::chrono::steady_clock::now();
    finish_request(s, w, q);
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
    lk.lock();
    s->busy_p += dt;
    --s->posting;
    complete_locked(s, q);
}

void sampler_main(rsrr_server* s)
{
    (void)hipSetDevice(s->cfg.device);
    const bool serial = (s->cfg.flags & RSRR_SERVE_SERIAL) != 0;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (serial && !s->post.empty()) {
            post_one(s, &s->ws, lk);
            continue;
        }
        admit_locked(s);
        std::vector<Chunk> ch = pick_locked(s);
        if (ch.empty()) {
            if (s->stop && s->queue.empty() && s->admitted.empty()) break;
            s->cv_work.wait(lk);
            continue;
        }
        const int launch_id = (int)s->launches++;
        long pts = 0;
        for (auto& c : ch) pts += c.cnt;
        s->max_launch = std::max(s->max_launch, pts);
        lk.unlock();
        const auto t = std::chrono::steady_clock::now();
        std::vector<std::vector<rsrr_point_info>> infos;
        std::vector<rsrr_status> codes;
        run_launch(s, ch, infos, codes);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); fr = tot; }
        batched_trim(s->ws.c, s->cfg.batch_bytes);  // bucket buffers of earlier sizes stay within the cap
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
        lk.lock();
        s->busy_s += dt;
        s->points += pts;
        s->mem_peak = std::max(s->mem_peak, tot - fr);
        for (size_t i = 0; i < ch.size(); ++i) {
            Req* q = ch[i].q;
            rsrr_result& r = q->res;
            note_status(r, codes[i]);
            if (q->last_launch != launch_id) { ++r.launches; q->last_launch = launch_id; }
            for (const auto& x : infos[i]) {
                r.fallbacks += x.fallback;
                r.ir_iters_max = std::max(r.ir_iters_max, x.ir_iters);
                if (x.resid > r.sample_resid_max) r.sample_resid_max = x.resid;
            }
            q->sampled += ch[i].cnt;
            if (q->sampled == q->r.N) {
                q->state = SAMPLED;
                r.t_sampled = now_s(s->t0);
                s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), q));
                s->post.push_back(q);
                s->cv_post.notify_one();
            }
        }
    }
}

void solver_main(rsrr_server* s, Worker* w)
{
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (!s->post.empty()) {
            post_one(s, w, lk);
            continue;
        }
        if (s->stop && s->queue.empty() && s->admitted.empty()) break;
        s->cv_post.wait(lk);
    }
}

}  // namespace

static rsrr_status worker_init(Worker* w, int device, const rsrr_options* opt, size_t ws_budget)
{
    if (hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking) != hipSuccess) {
        w->st = nullptr;
        return RSRR_EDEVICE;
    }
    rsrr_status e = rsrr_create(&w->c, device, w->st);
    if (e) {
        w->c = nullptr;
        return e;
    }
    if (opt) e = rsrr_set_options(w->c, opt) ? -2 : RSRR_OK;
    if (ws_budget) w->c->ws_budget = ws_budget;
    return e;
}

static void worker_free(Worker* w)
{
    if (w->c) rsrr_destroy(w->c);
    if (w->aq_buf) (void)hipFree(w->aq_buf);
    if (w->st) (void)hipStreamDestroy(w->st);
    *w = Worker();
}

static void server_free(rsrr_server* s)
{
    (void)hipSetDevice(s->cfg.device);
    worker_free(&s->ws);
    for (auto& w : s->wp) worker_free(w.get());
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

extern "C" rsrr_status rsrr_server_create(rsrr_server** out, const rsrr_server_config* cfg)
{
    if (!out) return -1;
    if (!cfg || cfg->max_slots < 1 || cfg->arena_bytes == 0 || cfg->batch_bytes == 0 || cfg->solvers < 0 ||
        cfg->solvers > 8 || (cfg->prec != RSRR_PREC_C128 && cfg->prec != RSRR_PREC_C64_IR))
        return -2;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return RSRR_EDEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return -2;
    RSRR_HIP(hipSetDevice(cfg->device));
    rsrr_server* s = new rsrr_server();
    s->cfg = *cfg;
    if (s->cfg.solvers == 0) s->cfg.solvers = 2;
    s->t0 = std::chrono::steady_clock::now();
    s->cfg.options = nullptr;  // read here only
    if (s->cfg.solve_bytes == 0) s->cfg.solve_bytes = DEFAULT_SOLVE_BYTES;
    const bool serial = (cfg->flags & RSRR_SERVE_SERIAL) != 0;
    // the sampling context also runs Steps 3-5 in serial mode
    rsrr_status e = worker_init(&s->ws, cfg->device, cfg->options, serial ? s->cfg.solve_bytes : 0);
    const int nsolve = serial ? 0 : s->cfg.solvers;
    for (int i = 0; i < nsolve && !e; ++i) {
        s->wp.emplace_back(new Worker());
        e = worker_init(s->wp.back().get(), cfg->device, cfg->options, s->cfg.solve_bytes);
    }
    if (!e && hipMalloc(&s->arena_base, cfg->arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        s->arena_base = nullptr;
        e = RSRR_ENOMEM;
    }
    if (e) {
        server_free(s);
        return e;
    }
    s->arena.init(cfg->arena_bytes);
    s->ws.th = std::thread(sampler_main, s);
    for (auto& w : s->wp) w->th = std::thread(solver_main, s, w.get());
    *out = s;
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_server_footprint(const rsrr_server_config* cfg, const rsrr_request* req,
                                             unsigned long long* bytes)
{
    if (!cfg) return -1;
    if (!req || !request_ok(req)) return -2;
    if (!bytes) return -3;
    *bytes = layout_of(*req, cfg->prec).total;
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_server_submit(rsrr_server* s, const rsrr_request* r, int* id)
{
    if (!s) return -1;
    if (!r) return -2;
    if (!id) return -3;
    if (!request_ok(r)) return -2;
    const rsrr_nep& e = r->nep;
    std::unique_ptr<Req> q(new Req());
    q->r = *r;
    if (e.kind == RSRR_T_SEPARABLE) q->terms.assign(e.terms, e.terms + e.J);
    q->r.nep.terms = q->terms.empty() ? nullptr : q->terms.data();
    q->z.resize(2 * (size_t)r->N);
    const rsrr_status ce = rsrr_contour(r->gamma_re, r->gamma_im, r->a, r->b, r->N, q->z.data(), nullptr);
    if (ce) return -2;
    q->lay = layout_of(*r, s->cfg.prec);
    q->s_bytes = q->lay.total;
    q->res.footprint = q->lay.total;
    q->res.L_used = r->L;
    if (q->s_bytes > s->cfg.arena_bytes) return RSRR_ENOMEM;
    std::lock_guard<std::mutex> lk(s->mu);
    q->id = s->next_id++;
    q->res.id = q->id;
    q->res.t_submit = now_s(s->t0);
    *id = q->id;
    s->queue.push_back(q.get());
    s->reqs[q->id] = std::move(q);
    s->cv_work.notify_all();
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_server_wait(rsrr_server* s, int id, double timeout_s, rsrr_result* out)
{
    if (!s) return -1;
    if (!out) return -4;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return -2;
    Req* q = it->second.get();
    auto done = [&] { return q->state == DONE; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        return RSRR_ETIMEOUT;
    }
    *out = q->res;
    s->reqs.erase(it);
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_server_stats(rsrr_server* s, double* out)
{
    if (!s) return -1;
    if (!out) return -2;
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = (double)s->finished;
    out[1] = (double)s->points;
    out[2] = (double)s->launches;
    out[3] = (double)s->arena.peak;
    out[4] = (double)s->max_launch;
    out[5] = s->busy_s;
    out[6] = s->busy_p;
    out[7] = (double)s->mem_peak;
    out[8] = now_s(s->t0);
    out[9] = (double)s->queue.size();
    out[10] = (double)s->repoints;
    out[11] = (double)s->reprobes;
    return RSRR_OK;
}

extern "C" rsrr_status rsrr_server_destroy(rsrr_server* s)
{
    if (!s) return -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
        s->cv_post.notify_all();
    }
    // the sampler leaves once nothing is queued or admitted; the solve threads once they
    // have also drained the sampled requests
    if (s->ws.th.joinable()) s->ws.th.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_post.notify_all();
    }
    for (auto& w : s->wp)
        if (w->th.joinable()) w->th.join();
    server_free(s);
    return RSRR_OK;
}
