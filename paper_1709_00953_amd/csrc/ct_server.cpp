// Serving loop over a batch (continuous batching), on the public C ABI.
//
// Jobs wait in a FIFO queue and are admitted at tick boundaries while a slot
// is free and their device footprint fits the budget (the queue head blocks
// the rest, so large jobs are not starved).  A resident job keeps its
// geometry tables, y, x and solver state (z^j, r) on the device.  Each tick:
//   1. read back the residual norms checked in the previous tick and retire
//      jobs at rel_tol or at their epoch cap (x copied to the host, device
//      memory freed);
//   2. admit queued jobs (geometry tables, density table, schedule, reset);
//   3. one batch epoch of every resident job;
//   4. enqueue the true-residual norms of the jobs that are due and one copy
//      of all of them to pinned host memory, followed by an event.
// The host thus runs at most one tick ahead of the device.
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
#include <vector>

using namespace ct;

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct SJob {
    int32_t id = 0;
    int64_t tag = 0;
    // owned copy of the geometry description
    ct_geom_desc desc{};
    std::vector<double> views;
    std::vector<int32_t> rb_ptr, tiles, boxes;
    ct_sched_params sched{};
    ct_solver_params sp{};
    std::vector<float> y_host;
    int64_t M = 0, N = 0;
    size_t bytes = 0;               // charged to the budget
    double t_submit = 0, t_admit = 0;
    // resident state
    ct_geom* geom = nullptr;
    ct_schedule* sc = nullptr;
    ct_solver* sol = nullptr;
    void* ws = nullptr;
    float* y = nullptr;
    float* x = nullptr;
    int32_t bid = -1;               // id in the batch
    int32_t slot = -1;              // row of the pending check
    int32_t checked = 0;            // epochs at the last enqueued check
    int32_t ran = 0;                // epochs run
    bool pending = false;
    double rel = -1.0;
    std::vector<int64_t> ep_upd;    // ray-voxel updates of each epoch
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
    std::vector<SJob*> active;
    std::deque<ct_server_done> done;
    std::map<int32_t, std::vector<float>> results;
    size_t used = 0, budget = 0;
    int64_t admitted = 0, retired = 0, updates = 0;
    int32_t next_id = 0;
    ct_batch* batch = nullptr;
    double* d_norms = nullptr;      // [capacity][2]
    double* h_norms = nullptr;      // pinned copy
    hipEvent_t ev = nullptr;
    bool ev_pending = false;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static void job_release(SJob* j) {
    if (j->sol) ct_solver_destroy(j->sol);
    if (j->sc) ct_schedule_destroy(j->sc);
    if (j->geom) ct_geom_destroy(j->geom);
    if (j->ws) (void)hipFree(j->ws);
    if (j->y) (void)hipFree(j->y);
    if (j->x) (void)hipFree(j->x);
    j->sol = nullptr;
    j->sc = nullptr;
    j->geom = nullptr;
    j->ws = j->y = j->x = nullptr;
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
    const size_t nb = 2 * sizeof(double) * (size_t)p->capacity;
    if (hipMalloc(&s->d_norms, nb) != hipSuccess || hipHostMalloc(&s->h_norms, nb, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess) {
        ct_server_destroy(s);
        return fail(CT_ENOMEM, "server buffers");
    }
    *out = s;
    return CT_OK;
}

extern "C" void ct_server_destroy(ct_server* s) {
    if (!s) return;
    if (s->ev_pending) (void)hipEventSynchronize(s->ev);
    (void)hipDeviceSynchronize();
    if (s->batch) ct_batch_destroy(s->batch);
    for (SJob* j : s->active) {
        job_release(j);
        delete j;
    }
    for (SJob* j : s->queue) delete j;
    if (s->d_norms) (void)hipFree(s->d_norms);
    if (s->h_norms) (void)hipHostFree(s->h_norms);
    if (s->ev) (void)hipEventDestroy(s->ev);
    delete s;
}

extern "C" int ct_server_submit(ct_server* s, const ct_server_job* job, int32_t* id) {
    if (!s || !job || !job->geom || !job->y || !id) return fail(CT_EINVAL, "NULL argument");
    const ct_geom_desc& d = *job->geom;
    if (job->sched.epochs < 1) return fail(CT_EINVAL, "epoch cap must be >= 1");
    size_t fp = 0;
    int rc = ct_job_footprint(&d, &job->solver, &fp);     // validates the geometry
    if (rc) return rc;
    SJob* j = new (std::nothrow) SJob();
    if (!j) return fail(CT_ENOMEM, "host allocation failed");
    j->tag = job->tag;
    j->desc = d;
    j->views.assign(d.views, d.views + (size_t)d.n_views * 12);
    j->rb_ptr.assign(d.rb_ptr, d.rb_ptr + d.n_row_blocks + 1);
    j->tiles.assign(d.tiles, d.tiles + (size_t)j->rb_ptr.back() * 5);
    j->boxes.assign(d.boxes, d.boxes + (size_t)d.n_col_blocks * 6);
    j->desc.views = j->views.data();
    j->desc.rb_ptr = j->rb_ptr.data();
    j->desc.tiles = j->tiles.data();
    j->desc.boxes = j->boxes.data();
    j->sched = job->sched;
    j->sp = job->solver;
    j->M = (int64_t)d.n_views * d.nu * std::max(d.nv, 1);
    j->N = (int64_t)d.nx * d.ny * std::max(d.nz, 1);
    j->y_host.assign(job->y, job->y + j->M);
    j->bytes = fp + align256((size_t)j->M * sizeof(float)) + align256((size_t)j->N * sizeof(float)) +
               sched_bytes_bound(d, job->sched);
    if (j->bytes > s->budget) {
        const size_t b = j->bytes;
        delete j;
        return fail(CT_EINVAL, "job needs %zu device bytes, the budget is %zu", b, s->budget);
    }
    j->id = s->next_id++;
    j->t_submit = s->now();
    s->queue.push_back(j);
    *id = j->id;
    return CT_OK;
}

static void retire(ct_server* s, SJob* j, int status) {
    ct_server_done r{};
    r.tag = j->tag;
    r.id = j->id;
    r.status = status;
    r.rel_residual = j->rel;
    r.t_submit = j->t_submit;
    r.t_admit = j->t_admit;
    r.bytes = (int64_t)j->bytes;
    r.updates = j->updates;
    if (j->bid >= 0) {
        int32_t e = 0;
        if (ct_batch_job_epoch(s->batch, j->bid, &e) == CT_OK) r.epochs = e;
        (void)ct_batch_remove(s->batch, j->bid);
        j->bid = -1;
    }
    if (j->x) {
        std::vector<float> x((size_t)j->N);
        if (hipMemcpy(x.data(), j->x, x.size() * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess)
            s->results[j->id] = std::move(x);
        else if (status >= 0)
            r.status = CT_EDEVICE;
    }
    job_release(j);
    s->used -= j->bytes;
    r.t_done = s->now();
    s->done.push_back(r);
    ++s->retired;
    delete j;
}

// Device state of a queued job; on failure the job is retired with the error.
static int admit(ct_server* s, SJob* j, hipStream_t st) {
    int rc = ct_geom_create(&j->desc, &j->geom);
    size_t wsb = 0;
    if (!rc) rc = ct_solver_workspace_bytes(j->geom, &j->sp, &wsb);
    if (!rc && (hipMalloc(&j->ws, wsb) != hipSuccess || hipMalloc((void**)&j->y, (size_t)j->M * sizeof(float)) != hipSuccess ||
                hipMalloc((void**)&j->x, (size_t)j->N * sizeof(float)) != hipSuccess))
        rc = fail(CT_ENOMEM, "device allocation for job %d failed", j->id);
    if (!rc && (hipMemcpyAsync(j->y, j->y_host.data(), (size_t)j->M * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemsetAsync(j->x, 0, (size_t)j->N * sizeof(float), st) != hipSuccess))
        rc = fail(CT_EDEVICE, "upload for job %d failed", j->id);
    std::vector<int64_t> nnz;
    if (!rc) {
        nnz.resize((size_t)j->desc.n_row_blocks * j->desc.n_col_blocks);
        rc = ct_geom_block_nnz(j->geom, s->p.tau, nnz.data(), st);    // synchronises st
    }
    if (!rc) rc = ct_schedule_create(j->geom, &j->sched, nnz.data(), &j->sc);
    if (!rc) {
        // 2 nnz(A_{I_G}^J) per group update (one back- and one forward projection)
        ct_sched_view v{};
        rc = ct_schedule_export(j->sc, &v);
        const int n = j->desc.n_col_blocks;
        for (int e = 0; !rc && e < v.n_epochs; ++e) {
            int64_t u = 0;
            for (int c = v.epoch_col_ptr[e]; c < v.epoch_col_ptr[e + 1]; ++c)
                for (int k = v.group_rb_ptr[v.col_group_ptr[c]]; k < v.group_rb_ptr[v.col_group_ptr[c + 1]]; ++k)
                    u += 2 * nnz[(size_t)v.rbs[k] * n + v.cols[c]];
            j->ep_upd.push_back(u);
        }
    }
    if (!rc) rc = ct_solver_create(j->geom, &j->sp, j->ws, wsb, &j->sol);
    if (!rc) rc = ct_solver_reset(j->sol, j->y, nullptr, st);
    if (!rc) {
        ct_batch_job bj{j->sol, j->sc, j->y, j->x, 0};
        rc = ct_batch_add(s->batch, &bj, &j->bid);
    }
    j->t_admit = s->now();
    j->y_host.clear();
    j->y_host.shrink_to_fit();
    if (rc) {
        (void)hipStreamSynchronize(st);
        retire(s, j, rc);
    }
    return rc;
}

extern "C" int ct_server_tick(ct_server* s, void* stream, ct_server_stats* stats) {
    if (!s) return fail(CT_EINVAL, "NULL server");
    hipStream_t st = (hipStream_t)stream;
    // 1. results of the previous tick's checks
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
                    retire(s, j, CT_OK);
                    continue;
                }
                if (j->checked >= j->sched.epochs) {
                    retire(s, j, CT_NOT_CONVERGED);
                    continue;
                }
            }
            keep.push_back(j);
        }
        s->active.swap(keep);
    }
    // 2. admission, first come first served
    while (!s->queue.empty() && (int)s->active.size() < s->p.capacity && s->used + s->queue.front()->bytes <= s->budget) {
        SJob* j = s->queue.front();
        s->queue.pop_front();
        s->used += j->bytes;
        if (admit(s, j, st) == CT_OK) {
            s->active.push_back(j);
            ++s->admitted;
        }
    }
    // 3. one epoch of every resident job, 4. due residual checks
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
    if (stats) {
        stats->active = (int32_t)s->active.size();
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
