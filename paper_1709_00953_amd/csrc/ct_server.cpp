// Serving loop over a batch (continuous batching), on the public C ABI.
//
// Jobs wait in a FIFO queue and are admitted at tick boundaries while a slot
// is free and their device footprint fits the budget (the queue head blocks
// the rest, so large jobs are not starved).  A resident job keeps its
// geometry tables, y, x, schedule tables and solver state (z^j, r) on the
// device.  Device memory is one arena of the budget, allocated when the
// server is created and sub-allocated per job (first fit); host<->device
// copies go through one pinned staging ring, so a tick neither allocates nor
// frees device memory and never waits for the device, except for the
// residual norms of the previous tick (the host runs at most one tick ahead).
// Each tick, in order:
//   1. take back staging space whose copies have completed, and hand out the
//      results of jobs whose x has arrived;
//   2. read the residual norms checked in the previous tick and retire jobs
//      at rel_tol or at their epoch cap (x copied to the staging ring, the
//      job's arena block returned: later work on the stream comes after the
//      copy);
//   3. jobs whose density table (counted on the device at admission) has
//      arrived get their schedule (host), its tables (staged) and a solver,
//      and join the batch;
//   4. admit queued jobs: arena block, geometry tables and y staged in, x
//      cleared, the density table counted and copied back (asynchronously);
//   5. one batch epoch of every resident job, and the due residual checks.
#include "ct.h"
#include "ct_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <set>
#include <vector>

using namespace ct;

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// First-fit sub-allocator over one device allocation (256-byte granules);
// adjacent free ranges are merged.
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;    // offset -> bytes

    void reset(char* b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(std::max<size_t>(bytes, 1));
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

// Pinned host staging ring.  Space is handed out in order and taken back in
// order once the event recorded after its copies has completed and, for a
// copy to the host, once its data has been consumed; the copies of one tick
// share one event.
struct Ring {
    struct Rec {
        size_t start, end;
        hipEvent_t ev;                 // nullptr until the tick's event is recorded
        bool download, consumed;
    };
    char* base = nullptr;
    size_t size = 0, head = 0;
    std::deque<Rec> recs;
    std::vector<hipEvent_t> pool;      // free events

    static bool complete(const Rec* r) { return r->ev && hipEventQuery(r->ev) == hipSuccess; }
    void reclaim() {
        while (!recs.empty()) {
            Rec& f = recs.front();
            if (!complete(&f) || (f.download && !f.consumed)) break;
            const hipEvent_t ev = f.ev;
            recs.pop_front();
            if (recs.empty() || recs.front().ev != ev) pool.push_back(ev);
        }
        if (recs.empty()) head = 0;
    }
    // a record of n bytes, or nullptr
    Rec* take(size_t n, bool download) {
        n = align256(std::max<size_t>(n, 1));
        if (n > size) return nullptr;
        size_t at;
        if (recs.empty()) {
            at = 0;
        } else {
            const size_t tail = recs.front().start;
            if (head > tail) {                                  // live data in [tail, head)
                if (head + n <= size) at = head;
                else if (n <= tail) at = 0;                 // wrap
                else return nullptr;
            } else {                                        // live data in [tail, size) and [0, head)
                if (head + n <= tail) at = head;
                else return nullptr;
            }
        }
        recs.push_back(Rec{at, at + n, nullptr, download, false});
        head = at + n;
        return &recs.back();
    }
    char* ptr(const Rec* r) const { return base + r->start; }
    // the event after this tick's copies, for every record still without one
    int seal(hipStream_t st) {
        if (recs.empty() || recs.back().ev) return CT_OK;
        if (pool.empty()) return fail(CT_EDEVICE, "no staging event free");
        const hipEvent_t ev = pool.back();
        pool.pop_back();
        if (hipEventRecord(ev, st) != hipSuccess) return fail(CT_EDEVICE, "staging event record");
        for (auto it = recs.rbegin(); it != recs.rend() && !it->ev; ++it) it->ev = ev;
        return CT_OK;
    }
};

enum State { kQueued, kCounting, kActive, kRetiring };

struct SJob {
    int32_t id = 0;
    int64_t tag = 0;
    State state = kQueued;
    ct_geom* geom = nullptr;           // created at submit (host tables only)
    ct_sched_params sched{};
    ct_solver_params sp{};
    std::vector<float> y_host;
    int64_t M = 0, N = 0;
    int m = 0, n = 0;
    // arena block: [geometry tables | workspace | y | x | schedule tables]
    size_t off = 0, bytes = 0;
    size_t b_geom = 0, b_ws = 0, b_y = 0, b_x = 0, b_sched = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    ct_schedule* sc = nullptr;
    ct_solver* sol = nullptr;
    float* y = nullptr;
    float* x = nullptr;
    Ring::Rec* r_nnz = nullptr;        // staging copy of the density table (in flight)
    std::vector<int64_t> nnz;          // the density table, once arrived
    Ring::Rec* r_x = nullptr;          // staging copy of x (retiring)
    int status = CT_OK;
    int32_t bid = -1;                  // id in the batch
    int32_t slot = -1;                 // row of the pending check
    int32_t checked = 0;               // epochs at the last enqueued check
    int32_t ran = 0;                   // epochs run
    int32_t epochs = 0;                // epochs at retirement
    bool pending = false;
    double rel = -1.0;
    std::vector<int64_t> ep_upd;       // ray-voxel updates of each epoch
    int64_t updates = 0;
};

// Upper bound of the schedule's device tables (entries, group offsets, beta,
// unions, step and epoch records), from its parameters.
size_t sched_bytes_bound(const ct_geom_desc& d, const ct_sched_params& p) {
    const size_t E = (size_t)std::max(p.epochs, 0), m = (size_t)d.n_row_blocks, n = (size_t)d.n_col_blocks;
    const size_t steps = E * n;
    return align256(std::max<size_t>(1, steps * m) * sizeof(Entry)) +
           align256(std::max<size_t>(1, steps * (m + 1)) * sizeof(int32_t)) +
           align256(std::max<size_t>(1, steps * m) * sizeof(double)) +
           align256(std::max<size_t>(1, E * m) * sizeof(Entry)) +
           align256(std::max<size_t>(1, steps) * sizeof(StepRec)) +
           align256(std::max<size_t>(1, E) * sizeof(EpochRec));
}

}  // namespace

struct ct_server {
    ct_server_params p{};
    std::chrono::steady_clock::time_point t0;
    std::deque<SJob*> queue;
    std::vector<SJob*> counting;       // admitted, density table in flight
    std::vector<SJob*> active;
    std::vector<SJob*> retiring;       // x in flight to the staging ring
    std::deque<ct_server_done> done;
    std::map<int32_t, std::vector<float>> results;
    size_t used = 0, budget = 0;
    int64_t admitted = 0, retired = 0, updates = 0;
    int32_t next_id = 0;
    ct_batch* batch = nullptr;
    void* arena_mem = nullptr;
    Arena arena;
    Ring ring;
    double* d_norms = nullptr;         // [capacity][2]
    double* h_norms = nullptr;         // pinned copy
    hipEvent_t ev = nullptr;
    bool ev_pending = false;
    hipEvent_t tick_ev = nullptr;      // after this tick's staging copies

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static void job_free(ct_server* s, SJob* j) {
    if (j->sol) ct_solver_destroy(j->sol);
    if (j->sc) ct_schedule_destroy(j->sc);
    j->sol = nullptr;
    j->sc = nullptr;
    if (j->bytes && j->state != kQueued) {
        s->arena.release(j->off, j->bytes);
        s->used -= j->bytes;
    }
}

static void job_delete(SJob* j) {
    if (j->geom) ct_geom_destroy(j->geom);
    delete j;
}

extern "C" int ct_server_create(const ct_server_params* p, ct_server** out) {
    if (!p || !out) return fail(CT_EINVAL, "NULL argument");
    *out = nullptr;
    if (p->capacity < 1 || p->capacity > kMaxBatch) return fail(CT_EINVAL, "capacity must lie in [1, %d]", kMaxBatch);
    if (p->check_every < 1) return fail(CT_EINVAL, "check_every must be >= 1");
    if (!(p->rel_tol >= 0) || !(p->tau >= 0)) return fail(CT_EINVAL, "rel_tol and tau must be >= 0");
    if (p->hbm_budget < 0) return fail(CT_EINVAL, "negative budget");
    ct_server* s = new (std::nothrow) ct_server();
    if (!s) return fail(CT_ENOMEM, "host allocation failed");
    s->p = *p;
    s->t0 = std::chrono::steady_clock::now();
    int rc = ct_batch_create(p->capacity, &s->batch);
    if (rc) {
        delete s;
        return rc;
    }
    if (p->hbm_budget > 0) {
        s->budget = (size_t)p->hbm_budget;
    } else {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            ct_server_destroy(s);
            return fail(CT_EDEVICE, "hipMemGetInfo failed");
        }
        s->budget = (size_t)(0.8 * (double)fr);
    }
    s->budget = align256(s->budget);
    // the arena, and a staging ring of a quarter of it, at most 1 GiB
    const size_t ring = std::max<size_t>(64 << 20, std::min<size_t>((size_t)1 << 30, s->budget / 4));
    const size_t nb = 2 * sizeof(double) * (size_t)p->capacity;
    bool ok = hipMalloc(&s->arena_mem, s->budget) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->ring.base, ring, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc(&s->d_norms, nb) == hipSuccess && hipHostMalloc(&s->h_norms, nb, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < 64; ++k) {
        hipEvent_t e = nullptr;
        ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) s->ring.pool.push_back(e);
    }
    if (!ok) {
        ct_server_destroy(s);
        return fail(CT_ENOMEM, "server arena (%zu bytes), staging ring or events", s->budget);
    }
    s->ring.size = ring;
    s->arena.reset((char*)s->arena_mem, s->budget);
    *out = s;
    return CT_OK;
}

extern "C" void ct_server_destroy(ct_server* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    if (s->batch) ct_batch_destroy(s->batch);
    for (auto* v : {&s->counting, &s->active, &s->retiring})
        for (SJob* j : *v) {
            if (j->sol) ct_solver_destroy(j->sol);
            if (j->sc) ct_schedule_destroy(j->sc);
            job_delete(j);
        }
    for (SJob* j : s->queue) job_delete(j);
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->ring.base) (void)hipHostFree(s->ring.base);
    std::set<hipEvent_t> evs(s->ring.pool.begin(), s->ring.pool.end());
    for (const auto& r : s->ring.recs)
        if (r.ev) evs.insert(r.ev);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (s->d_norms) (void)hipFree(s->d_norms);
    if (s->h_norms) (void)hipHostFree(s->h_norms);
    if (s->ev) (void)hipEventDestroy(s->ev);
    delete s;
}

extern "C" int ct_server_submit(ct_server* s, const ct_server_job* job, int32_t* id) {
    if (!s || !job || !job->geom || !job->y || !id) return fail(CT_EINVAL, "NULL argument");
    const ct_geom_desc& d = *job->geom;
    if (job->sched.epochs < 1) return fail(CT_EINVAL, "epoch cap must be >= 1");
    SJob* j = new (std::nothrow) SJob();
    if (!j) return fail(CT_ENOMEM, "host allocation failed");
    int rc = ct_geom_create(&d, &j->geom);         // validates; host tables only
    size_t wsb = 0;
    if (!rc) rc = ct_solver_workspace_bytes(j->geom, &job->solver, &wsb);
    if (rc) {
        job_delete(j);
        return rc;
    }
    j->tag = job->tag;
    j->sched = job->sched;
    j->sp = job->solver;
    j->m = d.n_row_blocks;
    j->n = d.n_col_blocks;
    j->M = (int64_t)d.n_views * d.nu * std::max(d.nv, 1);
    j->N = (int64_t)d.nx * d.ny * std::max(d.nz, 1);
    j->y_host.assign(job->y, job->y + j->M);
    j->b_geom = align256(geom_table_bytes(j->geom));
    j->b_ws = align256(wsb);
    j->b_y = align256((size_t)j->M * sizeof(float));
    j->b_x = align256((size_t)j->N * sizeof(float));
    j->b_sched = align256(sched_bytes_bound(d, job->sched));
    j->bytes = j->b_geom + j->b_ws + j->b_y + j->b_x + j->b_sched;
    if (j->bytes > s->budget) {
        const size_t b = j->bytes;
        job_delete(j);
        return fail(CT_EINVAL, "job needs %zu device bytes, the budget is %zu", b, s->budget);
    }
    const size_t stage = std::max(j->b_geom + j->b_y + align256((size_t)j->m * j->n * 8), j->b_sched);
    if (stage > s->ring.size || j->b_x > s->ring.size) {
        job_delete(j);
        return fail(CT_EINVAL, "job needs %zu bytes of staging, the ring has %zu", stage, s->ring.size);
    }
    j->id = s->next_id++;
    j->t_submit = s->now();
    s->queue.push_back(j);
    *id = j->id;
    return CT_OK;
}

static void push_done(ct_server* s, SJob* j) {
    ct_server_done r{};
    r.tag = j->tag;
    r.id = j->id;
    r.status = j->status;
    r.rel_residual = j->rel;
    r.t_submit = j->t_submit;
    r.t_admit = j->t_admit;
    r.t_done = s->now();
    r.bytes = (int64_t)j->bytes;
    r.updates = j->updates;
    r.epochs = j->epochs;
    s->done.push_back(r);
    ++s->retired;
}

// Begin retirement: leave the batch, copy x to the staging ring (or, when
// the ring is full, synchronously), give the arena block back (work enqueued
// later on the stream, which may reuse it, runs after the copy).
static void retire(ct_server* s, SJob* j, int status, hipStream_t st) {
    j->status = status;
    if (j->bid >= 0) {
        int32_t e = 0;
        if (ct_batch_job_epoch(s->batch, j->bid, &e) == CT_OK) j->epochs = e;
        (void)ct_batch_remove(s->batch, j->bid);
        j->bid = -1;
    }
    std::vector<float> xr;
    if (j->x) {
        const size_t xb = (size_t)j->N * sizeof(float);
        Ring::Rec* r = s->ring.take(xb, true);
        if (r && hipMemcpyAsync(s->ring.ptr(r), j->x, xb, hipMemcpyDeviceToHost, st) == hipSuccess) {
            j->r_x = r;
        } else {
            if (r) r->consumed = true;
            xr.resize((size_t)j->N);
            if (hipStreamSynchronize(st) != hipSuccess ||
                hipMemcpy(xr.data(), j->x, xb, hipMemcpyDeviceToHost) != hipSuccess) {
                if (status >= 0) j->status = CT_EDEVICE;
                xr.clear();
            }
        }
    }
    if (j->r_nnz) j->r_nnz->consumed = true;    // (a job that fails before its table arrives)
    job_free(s, j);
    j->state = kRetiring;
    if (j->r_x) {
        s->retiring.push_back(j);
    } else {
        if (!xr.empty()) s->results[j->id] = std::move(xr);
        push_done(s, j);
        job_delete(j);
    }
}

// Admission: the job's geometry tables and y staged into its arena block, x
// cleared, the density table counted and its copy back enqueued.  1: no
// staging space now.
static int admit(ct_server* s, SJob* j, hipStream_t st) {
    char* d_geom = s->arena.base + j->off;
    char* d_ws = d_geom + j->b_geom;
    j->y = (float*)(d_ws + j->b_ws);
    j->x = (float*)((char*)j->y + j->b_y);
    const size_t nb = (size_t)j->m * j->n * sizeof(int64_t);
    const size_t yb = (size_t)j->M * sizeof(float);
    Ring::Rec* up = s->ring.take(j->b_geom + yb, false);
    if (!up) return 1;
    Ring::Rec* down = s->ring.take(nb, true);
    if (!down) {
        up->consumed = true;
        // nothing was copied from `up`: let it go with this tick's event
        return 1;
    }
    char* h = s->ring.ptr(up);
    int rc = geom_table_pack(j->geom, h);
    if (!rc) std::memcpy(h + j->b_geom, j->y_host.data(), yb);
    if (!rc && (hipMemcpyAsync(d_geom, h, j->b_geom, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(j->y, h + j->b_geom, yb, hipMemcpyHostToDevice, st) != hipSuccess))
        rc = fail(CT_EDEVICE, "upload for job %d", j->id);
    if (!rc) rc = geom_table_bind(j->geom, d_geom);
    if (!rc && launch_fill(j->x, j->N, 0.f, st) != hipSuccess) rc = fail(CT_EDEVICE, "clear x of job %d", j->id);
    unsigned long long* d_cnt = nullptr;
    if (!rc) rc = geom_count_async(j->geom, s->p.tau, &d_cnt, st);
    if (!rc && hipMemcpyAsync(s->ring.ptr(down), d_cnt, nb, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = fail(CT_EDEVICE, "density read-back of job %d", j->id);
    j->r_nnz = down;
    if (rc) down->consumed = true;
    j->t_admit = s->now();
    j->y_host.clear();
    j->y_host.shrink_to_fit();
    return rc;
}

// The density table has arrived: schedule (host), its tables staged into
// the block, a solver on the workspace, reset, and the batch.  1: no staging
// space now.
static int activate(ct_server* s, SJob* j, hipStream_t st) {
    int rc = CT_OK;
    if (!j->sc) {
        rc = ct_schedule_create(j->geom, &j->sched, j->nnz.data(), &j->sc);
        if (!rc) {
            // 2 nnz(A_{I_G}^J) per group update (one back- and one forward projection)
            ct_sched_view v{};
            rc = ct_schedule_export(j->sc, &v);
            for (int e = 0; !rc && e < v.n_epochs; ++e) {
                int64_t u = 0;
                for (int c = v.epoch_col_ptr[e]; c < v.epoch_col_ptr[e + 1]; ++c)
                    for (int k = v.group_rb_ptr[v.col_group_ptr[c]]; k < v.group_rb_ptr[v.col_group_ptr[c + 1]]; ++k)
                        u += 2 * j->nnz[(size_t)v.rbs[k] * j->n + v.cols[c]];
                j->ep_upd.push_back(u);
            }
        }
        if (rc) return rc;
    }
    char* d_ws = s->arena.base + j->off + j->b_geom;
    char* d_sched = (char*)j->x + j->b_x;
    const size_t sb = sched_table_bytes(j->sc);
    if (sb > j->b_sched) return fail(CT_EINVAL, "schedule tables (%zu) beyond their bound (%zu)", sb, j->b_sched);
    Ring::Rec* r = s->ring.take(sb, false);
    if (!r) return 1;
    rc = sched_table_pack(j->sc, s->ring.ptr(r));
    if (!rc && hipMemcpyAsync(d_sched, s->ring.ptr(r), sb, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(CT_EDEVICE, "schedule upload of job %d", j->id);
    if (!rc) rc = sched_table_bind(j->sc, d_sched);
    if (!rc) rc = ct_solver_create(j->geom, &j->sp, d_ws, j->b_ws, &j->sol);
    if (!rc) rc = ct_solver_reset(j->sol, j->y, nullptr, st);
    if (!rc) {
        ct_batch_job bj{j->sol, j->sc, j->y, j->x, 0};
        rc = ct_batch_add(s->batch, &bj, &j->bid);
    }
    return rc;
}

extern "C" int ct_server_tick(ct_server* s, void* stream, ct_server_stats* stats) {
    if (!s) return fail(CT_EINVAL, "NULL server");
    hipStream_t st = (hipStream_t)stream;
    // 1. copies to the host that have arrived are consumed, then their
    //    staging space (and that of completed uploads) is taken back
    {
        std::vector<SJob*> keep;
        for (SJob* j : s->retiring) {
            if (Ring::complete(j->r_x)) {
                const float* h = (const float*)s->ring.ptr(j->r_x);
                s->results[j->id].assign(h, h + j->N);
                j->r_x->consumed = true;
                push_done(s, j);
                job_delete(j);
            } else {
                keep.push_back(j);
            }
        }
        s->retiring.swap(keep);
        for (SJob* j : s->counting) {
            if (j->r_nnz && Ring::complete(j->r_nnz)) {
                const int64_t* h = (const int64_t*)s->ring.ptr(j->r_nnz);
                j->nnz.assign(h, h + (size_t)j->m * j->n);
                j->r_nnz->consumed = true;
                j->r_nnz = nullptr;
            }
        }
        s->ring.reclaim();
    }
    // 2. results of the previous tick's checks
    if (s->ev_pending) {
        if (hipEventSynchronize(s->ev) != hipSuccess) return fail(CT_EDEVICE, "device error in a previous tick");
        s->ev_pending = false;
        std::vector<SJob*> keep;
        for (SJob* j : s->active) {
            if (j->pending) {
                j->pending = false;
                const double a = s->h_norms[2 * j->slot], b = s->h_norms[2 * j->slot + 1];
                j->rel = b > 0 ? std::sqrt(a / b) : 0.0;
                if (j->rel <= s->p.rel_tol) {
                    retire(s, j, CT_OK, st);
                    continue;
                }
                if (j->checked >= j->sched.epochs) {
                    retire(s, j, CT_NOT_CONVERGED, st);
                    continue;
                }
            }
            keep.push_back(j);
        }
        s->active.swap(keep);
    }
    // 3. admitted jobs whose density table has arrived join the batch
    {
        std::vector<SJob*> keep;
        for (SJob* j : s->counting) {
            if (j->nnz.empty()) {
                keep.push_back(j);
                continue;
            }
            const int rc = activate(s, j, st);
            if (rc == 1) {
                keep.push_back(j);
            } else if (rc) {
                retire(s, j, rc, st);
            } else {
                j->state = kActive;
                s->active.push_back(j);
            }
        }
        s->counting.swap(keep);
    }
    // 4. admission, first come first served
    while (!s->queue.empty() && (int)(s->active.size() + s->counting.size()) < s->p.capacity) {
        SJob* j = s->queue.front();
        size_t off = 0;
        if (!s->arena.alloc(j->bytes, &off)) break;
        j->off = off;
        const int rc = admit(s, j, st);
        if (rc == 1) {                                  // no staging space: the arena block waits
            s->arena.release(off, j->bytes);
            break;
        }
        s->queue.pop_front();
        s->used += j->bytes;
        j->state = kCounting;
        ++s->admitted;
        if (rc) retire(s, j, rc, st);
        else s->counting.push_back(j);
    }
    // 5. one epoch of every resident job, and the due residual checks
    if (!s->active.empty()) {
        int rc = ct_batch_epoch(s->batch, s->p.use_graph ? CT_BATCH_GRAPH : 0, nullptr, stream);
        if (rc) return rc;
        int n_checks = 0;
        for (size_t k = 0; k < s->active.size(); ++k) {
            SJob* j = s->active[k];
            int32_t e = 0;
            if ((rc = ct_batch_job_epoch(s->batch, j->bid, &e))) return rc;
            for (; j->ran < e; ++j->ran) {
                j->updates += j->ep_upd[j->ran];
                s->updates += j->ep_upd[j->ran];
            }
            if (e > j->checked && (e % s->p.check_every == 0 || e >= j->sched.epochs)) {
                j->slot = (int32_t)k;
                if ((rc = ct_residual_norms(j->sol, j->y, j->x, s->d_norms + 2 * k, stream))) return rc;
                j->checked = e;
                j->pending = true;
                ++n_checks;
            }
        }
        if (n_checks) {
            if (hipMemcpyAsync(s->h_norms, s->d_norms, 2 * sizeof(double) * s->active.size(), hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipEventRecord(s->ev, st) != hipSuccess)
                return fail(CT_EDEVICE, "residual read-back");
            s->ev_pending = true;
        }
    }
    int rc = s->ring.seal(st);
    if (rc) return rc;
    if (stats) {
        stats->active = (int32_t)(s->active.size() + s->counting.size());
        stats->queued = (int32_t)s->queue.size();
        stats->admitted = s->admitted;
        stats->retired = s->retired;
        stats->updates = s->updates;
        stats->bytes_in_use = (int64_t)s->used;
        stats->budget = (int64_t)s->budget;
        stats->now = s->now();
    }
    return CT_OK;
}

extern "C" int ct_server_poll(ct_server* s, ct_server_done* out, int32_t max, int32_t* n) {
    if (!s || !n || (max > 0 && !out)) return fail(CT_EINVAL, "NULL argument");
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return CT_OK;
}

extern "C" int ct_server_result(ct_server* s, int32_t id, float* x) {
    if (!s || !x) return fail(CT_EINVAL, "NULL argument");
    auto it = s->results.find(id);
    if (it == s->results.end()) return fail(CT_EINVAL, "no result for job %d", id);
    std::memcpy(x, it->second.data(), it->second.size() * sizeof(float));
    s->results.erase(it);
    return CT_OK;
}
