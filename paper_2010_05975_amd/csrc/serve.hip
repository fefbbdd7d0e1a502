// Request loop of the serving ABI (cfx_serve_*): continuous batching of
// solves on one device.
//
// Host side only.  A request is queued by cfx_serve_submit; `max_slots`
// worker threads, each with its own library handle and stream, take the
// head of the queue when it can be admitted: its device memory (factors,
// workspace, refinement vectors) is carved from the caller's arena by a
// first-fit allocator; if it does not fit, resident factors that no
// request is using are evicted, least recently used first; if it still
// does not fit, the head waits for running requests to finish (or fails
// with CFX_ENOMEM when nothing is running and it can never fit).  A head
// of order <= 512 takes the following small requests with it (up to
// batch_max) and the group is solved by one batched launch.  Requests run
// concurrently on the workers' streams; every kernel they use computes in
// a fixed order, so a request's result does not depend on its neighbours.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cfx_internal.h"

namespace cfx {
namespace {

constexpr int64_t kBatchMaxN = 512;     // orders solved by the batched launch
constexpr int64_t kBatchMaxRhs = 16;

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, cap) with neighbour coalescing.
struct Arena {
    size_t cap = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    void init(size_t bytes)
    {
        cap = bytes & ~(size_t)255;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = al(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = al(bytes ? bytes : 1);
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

// Factors on the device: F (n x n), ipiv, perm.
struct Resident {
    uint64_t id = 0;
    int64_t n = 0;
    size_t off = 0, bytes = 0;
    double *F = nullptr;
    int32_t *ipiv = nullptr, *perm = nullptr;
    int refs = 0;
    int32_t info = 0;
    int32_t prec = CFX_PREC_FP64;   // precision the factors were computed in
    bool keep = false;
    uint64_t last_use = 0;
};

size_t resident_bytes(int64_t n) { return al((size_t)n * n * 8) + 2 * al((size_t)n * 4); }

struct Job {
    uint64_t ticket = 0;
    cfx_request r{};
    cfx_result res{};
    int state = 0;            // 0 queued, 1 running, 2 done
    Resident *fac = nullptr;
    bool hit = false;
    size_t soff = 0, sbytes = 0;   // scratch of a single request
};

struct Group {
    std::vector<Job *> jobs;
    bool batched = false;
    size_t soff = 0, sbytes = 0;   // scratch of a batched group
};

}  // namespace
}  // namespace cfx

using namespace cfx;

struct cfx_server {
    cfx_serve_cfg cfg{};
    int device = 0;
    int batch_max = 256;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job *> queue;
    std::unordered_map<uint64_t, Job *> jobs;
    std::unordered_map<uint64_t, Resident *> res;
    Arena arena;
    uint64_t next_ticket = 1, next_fac = 1, clock = 0;
    int running = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    cfx_serve_stats st{};
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    char *base() const { return static_cast<char *>(cfg.arena); }
};

namespace cfx {
namespace {

size_t single_scratch(const cfx_server *S, int64_t n)
{
    const int restart = S->cfg.ir.gmres_restart;
    return al(256) + al(workspace_bytes(n, S->cfg.ir.lu.v, S->cfg.ir.lu.leaves, S->cfg.ir.lu.precision, 1,
                                                 S->cfg.ir.lu.min_leaf_rows)) +
           al(ir_vec_bytes(n, restart));
}

size_t group_scratch(size_t count)
{
    // int32 n, nrhs, info; 64-bit F, ldf, X, ldx, ipiv, A, lda, B, ldb; the
    // batched work; eta
    return al(count * 4) * 3 + al(count * 8) * 9 + al(batched_work_bytes((int32_t)count)) + al(count * 8);
}

Resident *new_resident(cfx_server *S, int64_t n, uint64_t id, size_t off)
{
    Resident *f = new Resident();
    f->id = id;
    f->n = n;
    f->off = off;
    f->bytes = resident_bytes(n);
    char *p = S->base() + off;
    f->F = reinterpret_cast<double *>(p);
    p += al((size_t)n * n * 8);
    f->ipiv = reinterpret_cast<int32_t *>(p);
    p += al((size_t)n * 4);
    f->perm = reinterpret_cast<int32_t *>(p);
    return f;
}

// Free arena bytes by evicting idle resident factors, oldest use first,
// until `need` bytes can be allocated.  Called with the lock held.
bool alloc_evicting(cfx_server *S, size_t need, size_t &off)
{
    if (S->arena.alloc(need, off)) return true;
    std::vector<Resident *> idle;
    for (auto &kv : S->res)
        if (kv.second->refs == 0) idle.push_back(kv.second);
    std::sort(idle.begin(), idle.end(), [](Resident *a, Resident *b) { return a->last_use < b->last_use; });
    for (Resident *f : idle) {
        S->arena.release(f->off, f->bytes);
        S->res.erase(f->id);
        delete f;
        ++S->st.evictions;
        if (S->arena.alloc(need, off)) return true;
    }
    return false;
}

void fail_job(cfx_server *S, Job *j, int status)
{
    j->res.status = status;
    j->res.t_admit = j->res.t_start = j->res.t_done = S->now();
    j->state = 2;
    ++S->st.failed;
}

// Admission of the queue head (and, for a small head, the small requests
// behind it).  Lock held.  Returns true when `g` holds work to run.
bool admit(cfx_server *S, Group &g)
{
    while (!S->queue.empty()) {
        Job *h = S->queue.front();
        const int64_t n = h->r.n;
        Resident *hit = nullptr;
        if (h->r.kind == CFX_RESOLVE) {
            auto it = S->res.find(h->r.factor_id);
            if (it != S->res.end() && it->second->n == n) hit = it->second;
        }
        if (!hit && n <= kBatchMaxN && h->r.nrhs <= kBatchMaxRhs) {
            // a batched group: consecutive small requests without a hit
            size_t count = 0;
            std::vector<size_t> offs;
            for (Job *j : S->queue) {
                if ((int)count >= S->batch_max || j->r.n > kBatchMaxN || j->r.nrhs > kBatchMaxRhs) break;
                if (j->r.kind == CFX_RESOLVE && S->res.count(j->r.factor_id)) break;
                ++count;
            }
            size_t soff = 0;
            // the scratch for the largest group that fits, shrinking on failure
            size_t admitted = 0;
            while (count > 0) {
                if (alloc_evicting(S, group_scratch(count), soff)) break;
                count /= 2;
            }
            if (count == 0) {
                if (S->running == 0) {
                    S->queue.pop_front();
                    fail_job(S, h, CFX_ENOMEM);
                    S->cv.notify_all();
                    continue;
                }
                return false;
            }
            for (size_t i = 0; i < count; ++i) {
                Job *j = S->queue[i];
                size_t off;
                if (!alloc_evicting(S, resident_bytes(j->r.n), off)) break;
                offs.push_back(off);
                ++admitted;
            }
            if (admitted == 0) {
                S->arena.release(soff, group_scratch(count));
                if (S->running == 0) {
                    S->queue.pop_front();
                    fail_job(S, h, CFX_ENOMEM);
                    S->cv.notify_all();
                    continue;
                }
                return false;
            }
            // keep the scratch sized for `count`; only `admitted` are used
            g.batched = true;
            g.soff = soff;
            g.sbytes = group_scratch(count);
            const double t = S->now();
            for (size_t i = 0; i < admitted; ++i) {
                Job *j = S->queue.front();
                S->queue.pop_front();
                const uint64_t id = j->r.kind == CFX_RESOLVE ? j->r.factor_id : S->next_fac++;
                if (j->r.kind == CFX_RESOLVE) ++S->st.resident_misses;
                j->fac = new_resident(S, j->r.n, id, offs[i]);
                j->fac->refs = 1;
                j->fac->keep = j->r.keep_resident != 0;
                j->res.factor_id = id;
                j->res.t_admit = t;
                j->res.batched = 1;
                j->state = 1;
                g.jobs.push_back(j);
            }
            return true;
        }
        // a single request
        const size_t sneed = single_scratch(S, n);
        size_t soff = 0, foff = 0;
        if (hit) ++hit->refs;   // protect it from eviction while allocating
        bool ok = alloc_evicting(S, sneed, soff);
        if (ok && !hit) {
            ok = alloc_evicting(S, resident_bytes(n), foff);
            if (!ok) S->arena.release(soff, sneed);
        }
        if (!ok) {
            if (hit) --hit->refs;
            if (S->running == 0) {
                S->queue.pop_front();
                fail_job(S, h, CFX_ENOMEM);
                S->cv.notify_all();
                continue;
            }
            return false;
        }
        S->queue.pop_front();
        h->soff = soff;
        h->sbytes = sneed;
        if (hit) {
            h->fac = hit;
            h->hit = true;
            ++S->st.resident_hits;
            hit->keep = hit->keep || h->r.keep_resident;
        } else {
            const uint64_t id = h->r.kind == CFX_RESOLVE ? h->r.factor_id : S->next_fac++;
            if (h->r.kind == CFX_RESOLVE) ++S->st.resident_misses;
            h->fac = new_resident(S, n, id, foff);
            h->fac->refs = 1;
            h->fac->keep = h->r.keep_resident != 0;
        }
        h->res.factor_id = h->fac->id;
        h->res.resident_hit = h->hit ? 1 : 0;
        h->res.t_admit = S->now();
        h->state = 1;
        g.jobs.push_back(h);
        g.batched = false;
        return true;
    }
    return false;
}

#define SRV_CHECK(call)                      \
    do {                                     \
        if ((rc = (call)) != 0) goto done;   \
    } while (0)
#define SRV_HIP(call)                                   \
    do {                                                \
        if ((call) != hipSuccess) {                     \
            rc = CFX_EHIP;                              \
            goto done;                                  \
        }                                               \
    } while (0)

int run_single(cfx_server *S, cfx_handle *h, hipStream_t st, Job *j)
{
    const cfx_request &r = j->r;
    const int64_t n = r.n;
    Resident *f = j->fac;
    char *sp = S->base() + j->soff;
    int32_t *dinfo = reinterpret_cast<int32_t *>(sp);
    char *wk = sp + al(256);
    const size_t wbytes = workspace_bytes(n, S->cfg.ir.lu.v, S->cfg.ir.lu.leaves, S->cfg.ir.lu.precision, 1,
                                                 S->cfg.ir.lu.min_leaf_rows);
    IrVectors v = carve_ir(wk + al(wbytes), n, S->cfg.ir.gmres_restart);
    IrParams p{S->cfg.ir.tol, S->cfg.ir.max_outer, S->cfg.ir.gmres_tol};
    p.spin_limit = solve_spin_limit(h);
    int rc = CFX_OK;
    int32_t info = 0;
    j->res.t_start = S->now();
    // factor A into f (FP64 or the configured precision)
    auto factor = [&](const cfx_lu_opts &o) -> int {
        int rc2 = CFX_OK;
        if (hipMemcpy2DAsync(f->F, (size_t)n * 8, r.A, (size_t)r.lda * 8, (size_t)n * 8, (size_t)n,
                             hipMemcpyDeviceToDevice, st) != hipSuccess)
            return CFX_EHIP;
        if ((rc2 = cfx_getrf(h, n, f->F, n, f->ipiv, dinfo, &o, wk, wbytes, st))) return rc2;
        if ((rc2 = launch_perm(n, f->ipiv, f->perm, st))) return rc2;
        if (hipMemcpyAsync(&info, dinfo, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return CFX_EHIP;
        f->info = info;
        f->prec = o.precision;
        return CFX_OK;
    };
    // the request's precision: FP64 below the low-precision threshold
    cfx_lu_opts o_req = S->cfg.ir.lu;
    if (o_req.precision != CFX_PREC_FP64 && n < S->cfg.lowp_min_n) o_req.precision = CFX_PREC_FP64;
    if (!j->hit) SRV_CHECK(factor(o_req));
    SRV_CHECK(launch_set_int(v.sync + 4, 0, st));   // give-up flag of the solves
    j->res.eta = 0.0;
    for (int64_t c = 0; c < r.nrhs; ++c) {
        IrResult ir{};
        for (;;) {
            SRV_CHECK(launch_copy_rows(n, 1, r.B + c, r.ldb, v.b, 1, st));
            SRV_CHECK(launch_gather_rows(n, 1, v.b, 1, f->perm, v.x, 1, st));
            SRV_CHECK(launch_trsv(n, 1, f->F, n, v.x, 1, v.sync, v.ys, st, p.spin_limit));
            ir = IrResult{};
            SRV_CHECK(ir_refine(r.A, r.lda, f->F, n, f->perm, v, p, &ir, st));
            if (ir.converged || f->prec == CFX_PREC_FP64) break;
            // low-precision factors that do not reach the target: refactor
            // in FP64 (the factors stay upgraded for later re-solves) and
            // solve this right-hand side again
            cfx_lu_opts o64 = S->cfg.ir.lu;
            o64.precision = CFX_PREC_FP64;
            SRV_CHECK(factor(o64));
            j->res.fallback = 1;
        }
        SRV_CHECK(launch_copy_rows(n, 1, v.x, 1, r.X + c, r.ldx, st));
        j->res.info = f->info;
        if (ir.eta > j->res.eta || ir.eta != ir.eta) j->res.eta = ir.eta;
        j->res.outer = std::max(j->res.outer, (int32_t)ir.outer);
        j->res.inner += ir.inner;
    }
    SRV_HIP(hipStreamSynchronize(st));
done:
    return rc;
}

int run_group(cfx_server *S, cfx_handle *h, hipStream_t st, Group &g)
{
    const size_t cnt = g.jobs.size();
    char *sp = S->base() + g.soff;
    // descriptor layout (matches group_scratch)
    int32_t *d_n = reinterpret_cast<int32_t *>(sp);
    int32_t *d_r = reinterpret_cast<int32_t *>(sp + al(cnt * 4));
    int32_t *d_info = reinterpret_cast<int32_t *>(sp + 2 * al(cnt * 4));
    char *q = sp + 3 * al(cnt * 4);
    double **d_F = reinterpret_cast<double **>(q);
    int64_t *d_ldf = reinterpret_cast<int64_t *>(q + al(cnt * 8));
    double **d_X = reinterpret_cast<double **>(q + 2 * al(cnt * 8));
    int64_t *d_ldx = reinterpret_cast<int64_t *>(q + 3 * al(cnt * 8));
    int32_t **d_ip = reinterpret_cast<int32_t **>(q + 4 * al(cnt * 8));
    double **d_A = reinterpret_cast<double **>(q + 5 * al(cnt * 8));
    int64_t *d_lda = reinterpret_cast<int64_t *>(q + 6 * al(cnt * 8));
    double **d_B = reinterpret_cast<double **>(q + 7 * al(cnt * 8));
    int64_t *d_ldb = reinterpret_cast<int64_t *>(q + 8 * al(cnt * 8));
    void *work = q + 9 * al(cnt * 8);
    double *d_eta = reinterpret_cast<double *>(static_cast<char *>(work) + al(batched_work_bytes((int32_t)cnt)));
    std::vector<int32_t> hn(cnt), hr(cnt), hinfo(cnt);
    std::vector<double *> hF(cnt), hX(cnt), hA(cnt), hB(cnt);
    std::vector<int64_t> hldf(cnt), hldx(cnt), hlda(cnt), hldb(cnt);
    std::vector<int32_t *> hip(cnt);
    std::vector<double> heta(cnt);
    int rc = CFX_OK;
    const double t = S->now();
    for (size_t i = 0; i < cnt; ++i) {
        Job *j = g.jobs[i];
        j->res.t_start = t;
        const cfx_request &r = j->r;
        hn[i] = (int32_t)r.n;
        hr[i] = (int32_t)r.nrhs;
        hF[i] = j->fac->F;
        hldf[i] = r.n;
        hX[i] = r.X;
        hldx[i] = r.ldx;
        hip[i] = j->fac->ipiv;
        hA[i] = const_cast<double *>(r.A);
        hlda[i] = r.lda;
        hB[i] = const_cast<double *>(r.B);
        hldb[i] = r.ldb;
        SRV_HIP(hipMemcpy2DAsync(j->fac->F, (size_t)r.n * 8, r.A, (size_t)r.lda * 8, (size_t)r.n * 8, (size_t)r.n,
                                 hipMemcpyDeviceToDevice, st));
        SRV_HIP(hipMemcpy2DAsync(r.X, (size_t)r.ldx * 8, r.B, (size_t)r.ldb * 8, (size_t)r.nrhs * 8, (size_t)r.n,
                                 hipMemcpyDeviceToDevice, st));
    }
    SRV_HIP(hipMemcpyAsync(d_n, hn.data(), cnt * 4, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_r, hr.data(), cnt * 4, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_F, hF.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_ldf, hldf.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_X, hX.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_ldx, hldx.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_ip, hip.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_A, hA.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_lda, hlda.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_B, hB.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(d_ldb, hldb.data(), cnt * 8, hipMemcpyHostToDevice, st));
    SRV_CHECK(cfx_gesv_batched(h, (int32_t)cnt, d_n, d_r, d_F, d_ldf, d_X, d_ldx, d_ip, d_info, work,
                               batched_work_bytes((int32_t)cnt), CFX_BATCHED_NO_GRAPH, st));
    {
        SRV_CHECK(launch_batched_eta((int)cnt, d_n, d_r, d_A, d_lda, d_B, d_ldb, d_X, d_ldx, d_eta, st));
        for (size_t i = 0; i < cnt; ++i)
            if (g.jobs[i]->fac->keep) SRV_CHECK(launch_perm(hn[i], hip[i], g.jobs[i]->fac->perm, st));
        SRV_HIP(hipMemcpyAsync(hinfo.data(), d_info, cnt * 4, hipMemcpyDeviceToHost, st));
        SRV_HIP(hipMemcpyAsync(heta.data(), d_eta, cnt * 8, hipMemcpyDeviceToHost, st));
        SRV_HIP(hipStreamSynchronize(st));
    }
    for (size_t i = 0; i < cnt; ++i) {
        g.jobs[i]->res.info = hinfo[i];
        g.jobs[i]->fac->info = hinfo[i];
        g.jobs[i]->res.eta = heta[i];
    }
done:
    return rc;
}

void worker_main(cfx_server *S)
{
    (void)hipSetDevice(S->device);
    cfx_handle *h = nullptr;
    hipStream_t st = nullptr;
    const bool ready = cfx_create(&h) == CFX_OK &&
                       hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        Group g;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (!S->queue.empty() && admit(S, g)) break;
                if (S->stop && S->queue.empty()) {
                    lk.unlock();
                    if (st) (void)hipStreamDestroy(st);
                    if (h) (void)cfx_destroy(h);
                    return;
                }
                S->cv.wait(lk);
            }
            ++S->running;
        }
        int rc = ready ? CFX_OK : CFX_EHIP;
        if (rc == CFX_OK) {
            if (g.batched) {
                rc = run_group(S, h, st, g);
            } else {
                rc = run_single(S, h, st, g.jobs[0]);
            }
        }
        if (st) (void)hipStreamSynchronize(st);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const double t = S->now();
            if (g.batched) {
                S->arena.release(g.soff, g.sbytes);
                ++S->st.batches;
                S->st.batched_requests += (int64_t)g.jobs.size();
            } else {
                S->arena.release(g.jobs[0]->soff, g.jobs[0]->sbytes);
            }
            for (Job *j : g.jobs) {
                Resident *f = j->fac;
                --f->refs;
                f->last_use = ++S->clock;
                auto it = S->res.find(f->id);
                bool registered = it != S->res.end() && it->second == f;
                // new factors are registered when asked for and computed
                // without error (a concurrent refactorisation of the same id
                // that registered first wins; this copy is dropped)
                if (!registered && rc == CFX_OK && f->keep && it == S->res.end()) {
                    S->res[f->id] = f;
                    registered = true;
                }
                if (!registered && f->refs == 0) {
                    S->arena.release(f->off, f->bytes);
                    delete f;
                }
                j->fac = nullptr;
                j->res.status = rc;
                j->res.t_done = t;
                j->state = 2;
                if (rc == CFX_OK) ++S->st.completed;
                else ++S->st.failed;
            }
            --S->running;
        }
        S->cv.notify_all();
    }
}

}  // namespace
}  // namespace cfx

extern "C" {

int cfx_serve_create(const cfx_serve_cfg *cfg, cfx_server **out)
{
    if (!cfg) return -1;
    if (!out) return -2;
    if (!cfg->arena || (reinterpret_cast<uintptr_t>(cfg->arena) & 255) || cfg->arena_bytes < 4096) return -1;
    if (cfg->max_slots < 1 || cfg->max_slots > 64) return -1;
    if (cfg->batch_max < 0) return -1;
    if (cfg->lowp_min_n < 0) return -1;
    {
        const cfx_ir_opts &o = cfg->ir;
        if (o.lu.v < 1 || o.lu.v > kMaxV || o.lu.leaves < 1 || o.lu.lookahead < 0 || o.lu.lookahead > 1 ||
            o.lu.min_leaf_rows < 0 || o.lu.min_leaf_rows > kMaxLeafRows)
            return -1;
        if (o.lu.precision != CFX_PREC_FP64 && o.lu.precision != CFX_PREC_BF16 && o.lu.precision != CFX_PREC_FP16 &&
            o.lu.precision != CFX_PREC_FP8)
            return CFX_ENOTSUP;
        if (!(o.tol >= 0) || o.max_outer < 0 || o.gmres_restart < 1 || o.gmres_restart > 64 ||
            !(o.gmres_tol > 0 && o.gmres_tol < 1))
            return -1;
    }
    cfx_server *S = new (std::nothrow) cfx_server();
    if (!S) return CFX_ENOMEM;
    S->cfg = *cfg;
    S->batch_max = cfg->batch_max > 0 ? cfg->batch_max : 256;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return CFX_EHIP;
    }
    S->arena.init(cfg->arena_bytes);
    S->t0 = std::chrono::steady_clock::now();
    try {
        for (int i = 0; i < cfg->max_slots; ++i) S->workers.emplace_back(worker_main, S);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv.notify_all();
        for (auto &w : S->workers) w.join();
        delete S;
        return CFX_ENOMEM;
    }
    *out = S;
    return CFX_OK;
}

int cfx_serve_submit(cfx_server *S, const cfx_request *r, uint64_t *ticket)
{
    if (!S) return -1;
    if (!r || (r->kind != CFX_SOLVE && r->kind != CFX_RESOLVE) || r->n < 1 || r->n > INT32_MAX || r->nrhs < 1 ||
        !r->A || r->lda < r->n || !r->B || r->ldb < r->nrhs || !r->X || r->ldx < r->nrhs)
        return -2;
    if (!ticket) return -3;
    Job *j = new (std::nothrow) Job();
    if (!j) return CFX_ENOMEM;
    j->r = *r;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete j;
            return CFX_EBUSY;
        }
        j->ticket = S->next_ticket++;
        j->res.t_submit = S->now();
        S->jobs[j->ticket] = j;
        S->queue.push_back(j);
        ++S->st.submitted;
        *ticket = j->ticket;
    }
    S->cv.notify_all();
    return CFX_OK;
}

int cfx_serve_poll(cfx_server *S, uint64_t ticket, cfx_result *out)
{
    if (!S) return -1;
    if (!out) return -3;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return -2;
    Job *j = it->second;
    if (j->state != 2) return CFX_PENDING;
    *out = j->res;
    S->jobs.erase(it);
    delete j;
    return CFX_OK;
}

int cfx_serve_release(cfx_server *S, uint64_t factor_id)
{
    if (!S) return -1;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->res.find(factor_id);
    if (it == S->res.end()) return -2;
    Resident *f = it->second;
    if (f->refs > 0) return CFX_EBUSY;
    S->arena.release(f->off, f->bytes);
    S->res.erase(it);
    delete f;
    S->cv.notify_all();
    return CFX_OK;
}

int cfx_serve_stats_get(cfx_server *S, cfx_serve_stats *out)
{
    if (!S) return -1;
    if (!out) return -2;
    std::lock_guard<std::mutex> lk(S->mu);
    cfx_serve_stats s = S->st;
    s.resident_factors = (int64_t)S->res.size();
    s.bytes_in_use = S->arena.used;
    s.bytes_peak = S->arena.peak;
    *out = s;
    return CFX_OK;
}

int cfx_serve_destroy(cfx_server *S)
{
    if (!S) return -1;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto &w : S->workers) w.join();
    for (auto &kv : S->jobs) delete kv.second;
    for (auto &kv : S->res) delete kv.second;
    delete S;
    return CFX_OK;
}

}  // extern "C"
