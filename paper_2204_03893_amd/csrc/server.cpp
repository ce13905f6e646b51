// Continuous-batching assembly server: arrival-order admission against
// in-flight slots and a device-memory budget, a resident plan cache (only the
// coefficients change between assemblies of one mesh, Section 5 summary),
// batched persistent launches over several streams, completion by events.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <thread>

#include "kernels.hpp"
#include "qxa_internal.hpp"

namespace qxa {

// ---- device arena ---------------------------------------------------------

DevArena::~DevArena()
{
    if (base_) hipFree(base_);
}

qxa_status DevArena::init(size_t bytes)
{
    cap_ = bytes & ~size_t(255);
    if (cap_ == 0) return fail(QXA_E_INVALID, "empty device budget");
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&base_), cap_);
    if (e != hipSuccess) {
        base_ = nullptr;
        return hip_fail(e, "hipMalloc (server budget)");
    }
    free_.clear();
    free_[0] = cap_;
    return QXA_OK;
}

void *DevArena::alloc(size_t bytes)
{
    const size_t n = granule(std::max<size_t>(bytes, 1));
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < n) continue;
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        live_[off] = n;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return base_ + off;
    }
    return nullptr;
}

void DevArena::release(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    const size_t off = size_t(static_cast<char *>(p) - base_);
    auto lv = live_.find(off);
    if (lv == live_.end()) return;
    size_t start = off, len = lv->second;
    used_ -= len;
    live_.erase(lv);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == start + len) {
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == start) {
            start = prev->first;
            len += prev->second;
            free_.erase(prev);
        }
    }
    free_[start] = len;
}

// ---- server state -----------------------------------------------------------

using Clock = std::chrono::steady_clock;

static double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// dim, n_q, points, weights of both rules: the cache and batching key part
// that fixes the reference tables.
static std::vector<double> rule_words(const qxa_quad &m, const qxa_quad &c)
{
    std::vector<double> w;
    for (const qxa_quad *q : {&m, &c}) {
        w.push_back(q->dim);
        w.push_back(q->n_q);
        w.insert(w.end(), q->points, q->points + size_t(q->n_q) * q->dim);
        w.insert(w.end(), q->weights, q->weights + q->n_q);
    }
    return w;
}

struct PlanKey {
    uint64_t mesh_serial;
    std::vector<double> rules;
    bool operator<(const PlanKey &o) const
    {
        if (mesh_serial != o.mesh_serial) return mesh_serial < o.mesh_serial;
        return rules < o.rules;
    }
};

struct CacheEntry {
    PlanKey key;
    qxa_mesh mesh = nullptr;
    std::vector<double> mr_pts, mr_w, cr_pts, cr_w;  // rules for the build
    int dim_m = 0, nq_m = 0, dim_c = 0, nq_c = 0;
    bool ready = false;
    qxa_plan plan = nullptr;
    int refs = 0;           // unreleased admitted jobs
    uint64_t last_use = 0;
    Clock::time_point t_ready;  // when the plan became resident
};

struct Job {
    uint64_t ticket = 0;
    qxa_job spec{};
    std::vector<double> mr_pts, mr_w, cr_pts, cr_w;
    double tensor[6] = {0, 0, 0, 0, 0, 0};  // copy of the conductivity tensor, if any
    PlanKey key;
    CacheEntry *entry = nullptr;
    int plan_cached = -1;  // unknown until the first cache lookup
    double plan_ms = 0.0;  // submit -> plan resident, for a job whose plan was not
    Clock::time_point t_submit, t_launch, t_done;
    void *buf = nullptr;
    double *M = nullptr, *C = nullptr;
    FusedArgs fa{};
    FixupArgs xa{};
    int status = QXA_OK;
    std::string msg;
    int batched = 0;
    double run_ms = 0.0;
    bool polled = false;
    int replans = 0;  // times its plan was rebuilt to free a contiguous range
    // copies of the result queued by qxa_server_copy_result on callers' streams:
    // release waits for them before the buffer returns to the budget
    std::vector<hipEvent_t> copies;
};

// Device and pinned host tables of one launch; held until its end event.
struct Slot {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *d_tab = nullptr, *h_tab = nullptr;  // FusedArgs[cap] | FixupArgs[cap] | int64 tile_end[cap] | fix_end[cap]
    int *d_flags = nullptr;                   // [cap] status word of each job of the launch
    int *h_flags = nullptr;                   // [cap] their copies on the host
    bool busy = false;
};

struct Launch {
    int slot;
    std::vector<Job *> jobs;
};

}  // namespace qxa

using namespace qxa;

struct qxa_server_s {
    qxa_server_opts o{};
    DevArena arena;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    std::vector<Slot> slots;
    size_t tab_bytes = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_build, cv_mem;
    bool stop = false, paused = false;
    uint64_t next_ticket = 1, use_clock = 0;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::deque<Job *> queue;
    std::vector<Job *> admitted;
    std::list<Launch> running;
    std::deque<Job *> done;
    std::map<PlanKey, std::unique_ptr<CacheEntry>> cache;
    std::deque<CacheEntry *> build_q;
    int inflight = 0;  // admitted + running
    int holders = 0;   // jobs holding job buffers
    int uploading = 0; // builders copying a plan into the budget
    int64_t n_submitted = 0, n_completed = 0, n_hits = 0, n_builds = 0, n_evictions = 0, n_launches = 0,
            n_batched = 0, max_batch = 0;
    std::thread worker;
    std::vector<std::thread> builders;
};

namespace qxa {

// Launch table of a batch: FusedArgs[cap] | FixupArgs[cap] | tile_end[cap] |
// fix_end[cap] | chain_ptr[cap * max_chains + 1] (the jobs' chains, in global
// tiles, one after the other).
static size_t tab_layout(int cap, int64_t max_chains, size_t &o_fix, size_t &o_te, size_t &o_fe, size_t &o_cp)
{
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    o_fix = al(sizeof(FusedArgs) * cap);
    o_te = o_fix + al(sizeof(FixupArgs) * cap);
    o_fe = o_te + al(sizeof(int64_t) * cap);
    o_cp = o_fe + al(sizeof(int64_t) * cap);
    return o_cp + al(sizeof(int64_t) * (size_t(cap) * size_t(max_chains) + 1));
}

static void finish_job(qxa_server s, Job *j, int status, const std::string &msg)
{
    j->status = status;
    j->msg = msg;
    j->t_done = Clock::now();
    s->done.push_back(j);
    ++s->n_completed;
}

// Evicts the least recently used resident plan that no unreleased job holds
// and (unless `force`) no waiting job needs, other than `keep`; returns false
// if there is none.
static bool evict_one(qxa_server s, bool force = false, const CacheEntry *keep = nullptr)
{
    CacheEntry *victim = nullptr;
    for (auto &kv : s->cache) {
        CacheEntry *c = kv.second.get();
        if (!c->ready || c->refs > 0 || c == keep) continue;
        if (!force && std::any_of(s->queue.begin(), s->queue.end(), [&](const Job *j) { return j->entry == c; }))
            continue;
        if (!victim || c->last_use < victim->last_use) victim = c;
    }
    if (!victim) return false;
    for (Job *j : s->queue)  // waiting jobs look the plan up again (and rebuild it)
        if (j->entry == victim) j->entry = nullptr;
    qxa_plan_destroy(victim->plan);
    s->cache.erase(victim->key);
    ++s->n_evictions;
    s->cv_mem.notify_all();
    return true;
}

// Completed launches -> completions. Lock held.
static bool reap(qxa_server s)
{
    bool progress = false;
    for (auto it = s->running.begin(); it != s->running.end();) {
        Slot &sl = s->slots[it->slot];
        const hipError_t e = hipEventQuery(sl.e1);
        if (e == hipErrorNotReady) {
            ++it;
            continue;
        }
        float ms = 0.f;
        if (e == hipSuccess) hipEventElapsedTime(&ms, sl.e0, sl.e1);
        for (size_t k = 0; k < it->jobs.size(); ++k) {
            Job *j = it->jobs[k];
            j->run_ms = ms;
            if (e != hipSuccess)
                finish_job(s, j, QXA_E_HIP, std::string("launch failed: ") + hipGetErrorString(e));
            else if (sl.h_flags[k])
                finish_job(s, j, QXA_E_NONFINITE, "non-finite coefficient value at a quadrature node");
            else
                finish_job(s, j, QXA_OK, "");
            --s->inflight;
        }
        sl.busy = false;
        it = s->running.erase(it);
        progress = true;
    }
    return progress;
}

static size_t job_bytes(const qxa_plan p)
{
    return 2 * DevArena::granule(sizeof(double) * std::max<int64_t>(p->nnz, 1)) +
           DevArena::granule(2 * sizeof(double) * std::max<int64_t>(p->n_partials, 1));
}

// Queue -> admitted, in arrival order. Lock held.
static bool admit(qxa_server s)
{
    bool progress = false;
    for (auto it = s->queue.begin(); it != s->queue.end() && s->inflight < s->o.max_inflight;) {
        Job *j = *it;
        if (!j->entry) {
            auto f = s->cache.find(j->key);
            if (f == s->cache.end()) {
                auto ce = std::make_unique<CacheEntry>();
                ce->key = j->key;
                ce->mesh = j->spec.mesh;
                ce->mr_pts = j->mr_pts;
                ce->mr_w = j->mr_w;
                ce->cr_pts = j->cr_pts;
                ce->cr_w = j->cr_w;
                ce->dim_m = j->spec.mass_rule.dim;
                ce->nq_m = j->spec.mass_rule.n_q;
                ce->dim_c = j->spec.stiff_rule.dim;
                ce->nq_c = j->spec.stiff_rule.n_q;
                j->entry = ce.get();
                s->build_q.push_back(ce.get());
                s->cache.emplace(j->key, std::move(ce));
                ++s->n_builds;
                s->cv_build.notify_one();
            } else {
                j->entry = f->second.get();
            }
            if (j->plan_cached < 0) {
                j->plan_cached = j->entry->ready ? 1 : 0;
                s->n_hits += j->plan_cached;
            }
        }
        CacheEntry *ce = j->entry;
        if (!ce->ready) {
            ++it;
            continue;
        }
        if (j->plan_cached == 0) j->plan_ms = std::max(0.0, ms_between(j->t_submit, ce->t_ready));
        qxa_plan p = ce->plan;
        const size_t need = job_bytes(p);
        void *buf = s->arena.alloc(need);
        while (!buf && evict_one(s, false, ce)) buf = s->arena.alloc(need);
        // nothing will be released: plans that other waiting jobs need go too
        while (!buf && s->holders == 0 && evict_one(s, true, ce)) buf = s->arena.alloc(need);
        if (!buf) {
            // no job holds memory and its plan is all that is left
            if (s->holders == 0 && s->arena.used() <= p->device_bytes) {
                // It would fit an empty budget, but the plan's buffers split the free space:
                // the plan goes and is rebuilt into the empty budget, where its buffers lie
                // together and leave one free range (a few times per job: another plan
                // built meanwhile can split the space again).
                if (j->replans < 4 && ce->refs == 0 && DevArena::granule(need) + p->device_bytes <= s->arena.capacity()) {
                    ++j->replans;
                    for (Job *q : s->queue)
                        if (q->entry == ce) q->entry = nullptr;
                    qxa_plan_destroy(ce->plan);
                    s->cache.erase(ce->key);
                    ++s->n_evictions;
                    s->cv_mem.notify_all();
                    progress = true;
                    continue;  // the job looks its plan up again and waits for the rebuild
                }
                finish_job(s, j, QXA_E_NOMEM, "job buffers exceed the device budget");
                it = s->queue.erase(it);
                progress = true;
                continue;
            }
            break;  // arrival order: later jobs wait behind it
        }
        char *b = static_cast<char *>(buf);
        j->buf = buf;
        j->M = reinterpret_cast<double *>(b);
        b += DevArena::granule(sizeof(double) * std::max<int64_t>(p->nnz, 1));
        j->C = reinterpret_cast<double *>(b);
        b += DevArena::granule(sizeof(double) * std::max<int64_t>(p->nnz, 1));
        double *part = reinterpret_cast<double *>(b);
        ++s->holders;
        ++ce->refs;
        ce->last_use = ++s->use_clock;
        const qxa_status st =
            make_fused_args(p, &j->spec.mass, &j->spec.stiff, j->spec.precision, j->M, j->C, part, nullptr, j->fa, j->xa);
        it = s->queue.erase(it);
        progress = true;
        if (st) {
            finish_job(s, j, st, qxa_last_error());
            continue;
        }
        s->admitted.push_back(j);
        ++s->inflight;
    }
    return progress;
}

static int free_slot(qxa_server s)
{
    for (size_t k = 0; k < s->slots.size(); ++k)
        if (!s->slots[k].busy) return int(k);
    return -1;
}

// One launch of a group of jobs sharing a kernel. Lock held.
static void launch_group(qxa_server s, std::vector<Job *> &g)
{
    const int si = free_slot(s);  // launches in flight <= jobs in flight <= slots
    if (si < 0) {
        for (Job *j : g) {
            finish_job(s, j, QXA_E_HIP, "no free launch slot");
            --s->inflight;
        }
        return;
    }
    Slot &sl = s->slots[si];
    hipStream_t st = s->streams[s->next_stream];
    s->next_stream = (s->next_stream + 1) % int(s->streams.size());
    const qxa_plan p0 = g[0]->entry->plan;
    const RefTables &R = p0->ref;
    const int prec = g[0]->spec.precision;
    (void)hipGetLastError();  // launch errors are read back with hipGetLastError
    hipError_t e = hipEventRecord(sl.e0, st);
    const auto now = Clock::now();
    for (size_t k = 0; k < g.size(); ++k) {
        g[k]->t_launch = now;
        g[k]->batched = int(g.size());
        g[k]->fa.in.flags = sl.d_flags + k;
    }
    if (e == hipSuccess) e = hipMemsetAsync(sl.d_flags, 0, sizeof(int) * g.size(), st);
    if (g.size() == 1) {
        const Job *j = g[0];
        const qxa_plan jp = j->entry->plan;
        const JobTable jt{j->fa, nullptr, nullptr, 0, jp->n_tiles, j->fa.buf_ok, jp->d_chain_ptr, jp->n_chains};
        const FixupTable ft{j->xa, nullptr, nullptr, 0, j->entry->plan->n_fix};
        if (e == hipSuccess) e = launch_fused(jt, R.dim, R.order, R.nq_m, R.nq_c, prec, st);
        if (e == hipSuccess) e = launch_fixup(ft, st);
    } else {
        size_t o_fix, o_te, o_fe, o_cp;
        tab_layout(s->o.max_inflight, s->o.batch_tile_limit, o_fix, o_te, o_fe, o_cp);
        char *h = static_cast<char *>(sl.h_tab);
        char *d = static_cast<char *>(sl.d_tab);
        auto *hfa = reinterpret_cast<FusedArgs *>(h);
        auto *hxa = reinterpret_cast<FixupArgs *>(h + o_fix);
        auto *hte = reinterpret_cast<int64_t *>(h + o_te);
        auto *hfe = reinterpret_cast<int64_t *>(h + o_fe);
        auto *hcp = reinterpret_cast<int64_t *>(h + o_cp);
        int64_t nt = 0, nf = 0, nc = 0;
        int buf = 1;
        hcp[0] = 0;
        for (size_t k = 0; k < g.size(); ++k) {
            const qxa_plan q = g[k]->entry->plan;
            buf &= g[k]->fa.buf_ok;
            hfa[k] = g[k]->fa;
            hxa[k] = g[k]->xa;
            for (int64_t c = 1; c <= q->n_chains; ++c) hcp[++nc] = nt + q->h_chain_ptr[c];
            nt += q->n_tiles;
            nf += q->n_fix;
            hte[k] = nt;
            hfe[k] = nf;
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(d, h, o_cp + sizeof(int64_t) * size_t(nc + 1), hipMemcpyHostToDevice, st);
        const JobTable jt{g[0]->fa, reinterpret_cast<const FusedArgs *>(d), reinterpret_cast<const int64_t *>(d + o_te),
                          int(g.size()), nt, buf, reinterpret_cast<const int64_t *>(d + o_cp), nc};
        const FixupTable ft{g[0]->xa, reinterpret_cast<const FixupArgs *>(d + o_fix),
                            reinterpret_cast<const int64_t *>(d + o_fe), int(g.size()), nf};
        if (e == hipSuccess) e = launch_fused(jt, R.dim, R.order, R.nq_m, R.nq_c, prec, st);
        if (e == hipSuccess) e = launch_fixup(ft, st);
        ++s->n_batched;
    }
    std::fill(sl.h_flags, sl.h_flags + g.size(), 0);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.h_flags, sl.d_flags, sizeof(int) * g.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(sl.e1, st);
    ++s->n_launches;
    s->max_batch = std::max<int64_t>(s->max_batch, int64_t(g.size()));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        for (Job *j : g) {
            finish_job(s, j, QXA_E_HIP, std::string("launch failed: ") + hipGetErrorString(e));
            --s->inflight;
        }
        return;
    }
    sl.busy = true;
    s->running.push_back(Launch{si, g});
}

// Admitted jobs -> launches: small FP64/FP32 jobs grouped by kernel, the rest
// alone. Lock held.
static bool launch_admitted(qxa_server s)
{
    if (s->admitted.empty()) return false;
    std::vector<Job *> pending;
    pending.swap(s->admitted);
    std::vector<bool> used(pending.size(), false);
    for (size_t a = 0; a < pending.size(); ++a) {
        if (used[a]) continue;
        used[a] = true;
        Job *j = pending[a];
        std::vector<Job *> g{j};
        const qxa_plan p = j->entry->plan;
        const bool small = p->n_tiles < s->o.batch_tile_limit &&
                           (j->spec.precision == QXA_FP64 || j->spec.precision == QXA_FP32);
        if (small) {
            for (size_t b = a + 1; b < pending.size(); ++b) {
                if (used[b]) continue;
                Job *k = pending[b];
                const qxa_plan q = k->entry->plan;
                if (k->spec.precision == j->spec.precision && q->n_tiles < s->o.batch_tile_limit &&
                    q->ref.dim == p->ref.dim && q->ref.order == p->ref.order && k->key.rules == j->key.rules) {
                    used[b] = true;
                    g.push_back(k);
                }
            }
        }
        launch_group(s, g);
    }
    return true;
}

static void worker_main(qxa_server s)
{
    hipSetDevice(s->o.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = reap(s);
        if (!s->stop && !s->paused) {
            progress |= admit(s);
            progress |= launch_admitted(s);
        }
        if (s->stop && s->running.empty()) break;
        if (progress) continue;
        if (!s->running.empty()) {
            // launches in flight: poll their end events
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv_work.wait(lk);
        }
    }
}

static void builder_main(qxa_server s)
{
    hipSetDevice(s->o.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_build.wait(lk, [&] { return s->stop || !s->build_q.empty(); });
        if (s->stop) break;
        CacheEntry *ce = s->build_q.front();
        s->build_q.pop_front();
        const qxa_mesh mesh = ce->mesh;
        const qxa_quad mr{ce->dim_m, ce->nq_m, ce->mr_pts.data(), ce->mr_w.data()};
        const qxa_quad cr{ce->dim_c, ce->nq_c, ce->cr_pts.data(), ce->cr_w.data()};
        lk.unlock();
        PlanStaging stg;
        qxa_status st = plan_stage(mesh, mr, cr, stg);
        std::string msg = st ? qxa_last_error() : "";
        qxa_plan p = nullptr;
        lk.lock();
        while (!st && !s->stop) {
            ++s->uploading;
            lk.unlock();
            st = plan_upload(mesh, stg, &s->arena, false, &p);  // frees what it took when it fails
            if (st) msg = qxa_last_error();
            lk.lock();
            --s->uploading;
            if (st != QXA_E_NOMEM) break;
            if (evict_one(s) || (s->holders == 0 && evict_one(s, true))) {
                st = QXA_OK;
                continue;
            }
            // nothing left to evict: wait for released results or other builders'
            // uploads, unless the plan could not fit even in an empty budget
            if ((s->holders == 0 && s->uploading == 0) || plan_bytes_lower_bound(stg) > s->arena.capacity()) {
                msg = "plan exceeds the device budget";
                break;
            }
            s->cv_mem.wait(lk);  // a release or an eviction frees memory
            st = QXA_OK;
        }
        if (s->stop) {
            if (p) qxa_plan_destroy(p);
            break;
        }
        if (st) {
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if ((*it)->entry == ce) {
                    finish_job(s, *it, st, msg);
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
            s->cache.erase(ce->key);
        } else {
            ce->plan = p;
            ce->ready = true;
            ce->t_ready = Clock::now();
            ce->last_use = ++s->use_clock;
            if (s->o.plan_cache_entries > 0)
                while (int(s->cache.size()) > s->o.plan_cache_entries && evict_one(s)) {
                }
        }
        s->cv_mem.notify_all();  // builders waiting for memory look again
        s->cv_work.notify_one();
    }
}

static void server_free(qxa_server s)
{
    hipSetDevice(s->o.device);
    for (hipStream_t st : s->streams) hipStreamSynchronize(st);
    for (auto &kv : s->jobs)
        for (hipEvent_t ev : kv.second->copies) {
            hipEventSynchronize(ev);
            hipEventDestroy(ev);
        }
    for (auto &kv : s->cache)
        if (kv.second->plan) qxa_plan_destroy(kv.second->plan);
    s->cache.clear();
    for (Slot &sl : s->slots) {
        if (sl.e0) hipEventDestroy(sl.e0);
        if (sl.e1) hipEventDestroy(sl.e1);
        if (sl.d_tab) hipFree(sl.d_tab);
        if (sl.d_flags) hipFree(sl.d_flags);
        if (sl.h_tab) hipHostFree(sl.h_tab);
        if (sl.h_flags) hipHostFree(sl.h_flags);
    }
    for (hipStream_t st : s->streams) hipStreamDestroy(st);
    delete s;
}

}  // namespace qxa

extern "C" {

qxa_status qxa_server_create(const qxa_server_opts *opts, qxa_server *out)
{
    if (!out) return fail(QXA_E_INVALID, "out is null");
    *out = nullptr;
    qxa_server_opts o{};
    if (opts) o = *opts;
    if (o.hbm_budget_bytes == 0) o.hbm_budget_bytes = size_t(4) << 30;
    if (o.max_inflight == 0) o.max_inflight = 64;
    if (o.n_streams == 0) o.n_streams = 4;
    if (o.batch_tile_limit == 0) o.batch_tile_limit = 512;
    if (o.queue_capacity == 0) o.queue_capacity = 65536;
    if (o.plan_builders == 0) o.plan_builders = 4;
    if (o.max_inflight < 1 || o.max_inflight > 4096 || o.n_streams < 1 || o.n_streams > 32 ||
        o.batch_tile_limit < 0 || o.queue_capacity < 1 || o.plan_cache_entries < 0 || o.plan_builders < 1 ||
        o.plan_builders > 64)
        return fail(QXA_E_INVALID, "server options out of range");
    QXA_HIP(hipSetDevice(o.device));
    auto *s = new qxa_server_s();
    s->o = o;
    qxa_status st = s->arena.init(o.hbm_budget_bytes);
    size_t o_fix, o_te, o_fe;
    size_t o_cp;
    s->tab_bytes = tab_layout(o.max_inflight, o.batch_tile_limit, o_fix, o_te, o_fe, o_cp);
    for (int k = 0; k < o.n_streams && !st; ++k) {
        hipStream_t h = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&h, hipStreamNonBlocking);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamCreateWithFlags");
        else s->streams.push_back(h);
    }
    s->slots.resize(size_t(o.max_inflight));
    for (Slot &sl : s->slots) {
        if (st) break;
        hipError_t e = hipEventCreate(&sl.e0);
        if (e == hipSuccess) e = hipEventCreate(&sl.e1);
        if (e == hipSuccess) e = hipMalloc(&sl.d_tab, s->tab_bytes);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sl.d_flags), sizeof(int) * o.max_inflight);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_tab, s->tab_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_flags), sizeof(int) * o.max_inflight,
                              hipHostMallocDefault);
        if (e != hipSuccess) st = hip_fail(e, "server launch tables");
    }
    if (st) {
        server_free(s);
        return st;
    }
    s->worker = std::thread(worker_main, s);
    for (int k = 0; k < o.plan_builders; ++k) s->builders.emplace_back(builder_main, s);
    *out = s;
    return QXA_OK;
}

qxa_status qxa_server_submit(qxa_server s, const qxa_job *job, uint64_t *ticket)
{
    if (!s || !job || !ticket) return fail(QXA_E_INVALID, "null argument");
    const qxa_mesh m = job->mesh;
    if (!m) return fail(QXA_E_INVALID, "job without a mesh");
    if (m->device != s->o.device) return fail(QXA_E_INVALID, "mesh lives on another device");
    for (const qxa_quad *q : {&job->mass_rule, &job->stiff_rule})
        if (q->dim != m->dim || q->n_q < 1 || q->n_q > kMaxNq || !q->points || !q->weights)
            return fail(QXA_E_INVALID, "bad quadrature rule");
    if (job->precision < QXA_FP64 || job->precision > QXA_BF16X3) return fail(QXA_E_INVALID, "unknown precision form");
    auto j = std::make_unique<Job>();
    j->spec = *job;
    j->mr_pts.assign(job->mass_rule.points, job->mass_rule.points + size_t(job->mass_rule.n_q) * m->dim);
    j->mr_w.assign(job->mass_rule.weights, job->mass_rule.weights + job->mass_rule.n_q);
    j->cr_pts.assign(job->stiff_rule.points, job->stiff_rule.points + size_t(job->stiff_rule.n_q) * m->dim);
    j->cr_w.assign(job->stiff_rule.weights, job->stiff_rule.weights + job->stiff_rule.n_q);
    j->spec.mass_rule.points = j->mr_pts.data();
    j->spec.mass_rule.weights = j->mr_w.data();
    j->spec.stiff_rule.points = j->cr_pts.data();
    j->spec.stiff_rule.weights = j->cr_w.data();
    if (job->mass.tensor) return fail(QXA_E_INVALID, "mass coefficient: a tensor applies to conductivity only");
    if (job->mass.tensor_q || job->stiff.tensor_q)
        return fail(QXA_E_UNSUPPORTED, "a tensor per quadrature node is taken by qxa_assemble_iso only");
    if (job->stiff.tensor) {
        std::copy(job->stiff.tensor, job->stiff.tensor + m->dim * (m->dim + 1) / 2, j->tensor);
        j->spec.stiff.tensor = j->tensor;
    }
    j->key = PlanKey{m->serial, rule_words(j->spec.mass_rule, j->spec.stiff_rule)};
    j->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(QXA_E_INVALID, "server is shutting down");
    if (int(s->queue.size()) >= s->o.queue_capacity) return fail(QXA_E_BUSY, "server queue full");
    j->ticket = s->next_ticket++;
    *ticket = j->ticket;
    s->queue.push_back(j.get());
    s->jobs.emplace(j->ticket, std::move(j));
    ++s->n_submitted;
    s->cv_work.notify_one();
    return QXA_OK;
}

qxa_status qxa_server_poll(qxa_server s, qxa_completion *out, int max, int *n_done)
{
    if (!s || !n_done || (max > 0 && !out)) return fail(QXA_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int n = 0;
    while (n < max && !s->done.empty()) {
        Job *j = s->done.front();
        s->done.pop_front();
        j->polled = true;
        qxa_completion &c = out[n++];
        std::memset(&c, 0, sizeof(c));
        c.ticket = j->ticket;
        c.user_tag = j->spec.user_tag;
        c.status = j->status;
        c.plan_cached = j->plan_cached > 0;
        c.plan_ms = j->plan_ms;
        c.batched = j->batched;
        c.n_nodes = j->spec.mesh->n_nodes;
        if (j->status == QXA_OK) {
            const qxa_plan p = j->entry->plan;
            c.nnz = p->nnz;
            c.M = j->M;
            c.C = j->C;
            c.row_ptr = p->d_row_ptr;
            c.col_idx = p->d_col_idx;
        }
        const Clock::time_point tl = j->batched ? j->t_launch : j->t_done;
        c.queue_ms = ms_between(j->t_submit, tl);
        c.run_ms = j->run_ms;
        c.total_ms = ms_between(j->t_submit, j->t_done);
        std::snprintf(c.message, sizeof(c.message), "%s", j->msg.c_str());
    }
    *n_done = n;
    return QXA_OK;
}

qxa_status qxa_server_copy_result(qxa_server s, uint64_t ticket, double *M_vals, double *C_vals, void *stream)
{
    if (!s) return fail(QXA_E_INVALID, "null server");
    const double *M = nullptr, *C = nullptr;
    int64_t nnz = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto f = s->jobs.find(ticket);
        if (f == s->jobs.end() || !f->second->polled) return fail(QXA_E_INVALID, "ticket not completed or unknown");
        const Job *j = f->second.get();
        if (j->status != QXA_OK) return fail(QXA_E_INVALID, "job failed; no result");
        M = j->M;
        C = j->C;
        nnz = j->entry->plan->nnz;
    }
    QXA_HIP(hipSetDevice(s->o.device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (M_vals && nnz) QXA_HIP(hipMemcpyAsync(M_vals, M, sizeof(double) * nnz, hipMemcpyDeviceToDevice, st));
    if (C_vals && nnz) QXA_HIP(hipMemcpyAsync(C_vals, C, sizeof(double) * nnz, hipMemcpyDeviceToDevice, st));
    if ((M_vals || C_vals) && nnz) {
        // the job's buffer may be reused only after these copies have read it
        hipEvent_t ev;
        QXA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ev, st);
        if (e != hipSuccess) {
            hipEventDestroy(ev);
            return hip_fail(e, "hipEventRecord");
        }
        std::lock_guard<std::mutex> lk(s->mu);
        auto f = s->jobs.find(ticket);
        if (f == s->jobs.end()) {  // released by another thread meanwhile: wait here instead
            hipEventSynchronize(ev);
            hipEventDestroy(ev);
        } else {
            f->second->copies.push_back(ev);
        }
    }
    return QXA_OK;
}

qxa_status qxa_server_release(qxa_server s, uint64_t ticket)
{
    if (!s) return fail(QXA_E_INVALID, "null server");
    std::vector<hipEvent_t> copies;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto f = s->jobs.find(ticket);
        if (f == s->jobs.end() || !f->second->polled) return fail(QXA_E_INVALID, "ticket not completed or unknown");
        copies.swap(f->second->copies);
    }
    // queued copies of the result must have read the buffer before it can serve another job
    hipError_t werr = hipSuccess;
    for (hipEvent_t ev : copies) {
        const hipError_t e = hipEventSynchronize(ev);
        if (werr == hipSuccess) werr = e;
        hipEventDestroy(ev);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto f = s->jobs.find(ticket);
    if (f == s->jobs.end()) return fail(QXA_E_INVALID, "ticket released twice");
    Job *j = f->second.get();
    for (hipEvent_t ev : j->copies) {  // copies queued while this call waited
        hipEventSynchronize(ev);
        hipEventDestroy(ev);
    }
    j->copies.clear();
    if (werr != hipSuccess) return hip_fail(werr, "hipEventSynchronize (result copy)");
    if (j->buf) {
        s->arena.release(j->buf);
        --s->holders;
        if (j->entry) --j->entry->refs;
    }
    s->jobs.erase(f);
    s->cv_mem.notify_all();
    s->cv_work.notify_one();
    return QXA_OK;
}

qxa_status qxa_server_drop_mesh(qxa_server s, qxa_mesh mesh)
{
    if (!s || !mesh) return fail(QXA_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    for (const auto &kv : s->jobs)
        if (kv.second->spec.mesh == mesh) return fail(QXA_E_BUSY, "jobs on this mesh are not released yet");
    for (const auto &kv : s->cache)
        if (kv.second->mesh == mesh && !kv.second->ready) return fail(QXA_E_BUSY, "a plan of this mesh is being built");
    for (auto it = s->cache.begin(); it != s->cache.end();) {
        if (it->second->mesh == mesh) {
            qxa_plan_destroy(it->second->plan);
            it = s->cache.erase(it);
        } else {
            ++it;
        }
    }
    s->cv_mem.notify_all();
    s->cv_work.notify_one();
    return QXA_OK;
}

qxa_status qxa_server_pause(qxa_server s, int paused)
{
    if (!s) return fail(QXA_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused != 0;
    s->cv_work.notify_one();
    return QXA_OK;
}

qxa_status qxa_server_stats(qxa_server s, int64_t *c, int n)
{
    if (!s || (n > 0 && !c)) return fail(QXA_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t v[] = {s->n_submitted,
                         s->n_completed,
                         s->n_hits,
                         s->n_builds,
                         s->n_evictions,
                         s->n_launches,
                         s->n_batched,
                         s->max_batch,
                         int64_t(s->arena.used()),
                         int64_t(s->arena.peak()),
                         int64_t(s->queue.size()),
                         int64_t(s->inflight),
                         int64_t(s->arena.capacity())};
    for (int k = 0; k < n && k < int(sizeof(v) / sizeof(v[0])); ++k) c[k] = v[k];
    return QXA_OK;
}

qxa_status qxa_server_destroy(qxa_server s)
{
    if (!s) return QXA_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_build.notify_all();
    s->cv_mem.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (std::thread &b : s->builders)
        if (b.joinable()) b.join();
    server_free(s);
    return QXA_OK;
}

}  // extern "C"
