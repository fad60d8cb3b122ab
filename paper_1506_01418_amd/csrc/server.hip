// Serving loop of libpsgld: independent PSGLD runs (jobs) admitted under a
// device-memory budget and stepped together.
//
// The server is a client of the context ABI: each running job is a
// psgld_ctx on the server's stream, and a tick advances all of them with
// psgld_step_batch, which puts every coordinate-stored job of one kernel
// variant into a single launch per iteration.  Jobs are independent runs of
// Algorithm 1 (own data, factors, noise key and step sizes), so batching
// changes when their work runs, never what it computes.
//
// Admission keeps the actual device bytes of the running jobs within the
// budget: the queue head is loaded when its upper estimate fits; if its
// actual allocation then does not fit (the estimate was too low), it is
// unloaded and waits with its estimate raised to the actual figure.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"
#include "psgld.h"

using namespace psgld;

namespace {

struct Job {
    int64_t id = 0;
    psgld_job spec{};
    std::vector<int32_t> row, col, hrow, hcol;
    std::vector<float> val, dense, hval, W0, H0;
    std::vector<uint8_t> mask;
    int32_t state = PSGLD_JOB_QUEUED;
    psgld_ctx *ctx = nullptr;
    int64_t est_bytes = 0, bytes = 0;
    int64_t done = 0;
    std::vector<double> Wm, Hm, Wv, Hv;
    double rmse = std::numeric_limits<double>::quiet_NaN();
    std::string err;
};

// Upper estimate of the device bytes of a job's context (every allocation
// of the load, held-out and stepping calls, by the sizes they are made with).
int64_t estimate_bytes(const psgld_job &j)
{
    const int64_t I = j.I, J = j.J, B = j.B, Kp = padded_rank(j.K);
    // the most groups per work-group any kernel variant of this rank uses
    // (a tuned variant remembered for the shape may be applied at load)
    int64_t Q = sparse_block_threads() / sparse_threads_per_group(j.K);
    for (int q : {1, 2, 4})
        if (sparse_variant_exists(sparse_lanes_for(j.K, q), q))
            Q = std::max<int64_t>(Q, sparse_block_threads() / sparse_lanes_for(j.K, q));
    int64_t qlog = 0;
    while ((int64_t{1} << qlog) < Q) ++qlog;
    int64_t nnz = j.nnz;
    if (!j.row) {
        nnz = 0;
        for (int64_t m = 0; m < I * J; ++m) nnz += j.mask ? (j.mask[m] != 0) : 1;
    }
    int64_t b = 0;
    b += 2 * 4 * ((I + J) * Kp + 2 * kFactorPad);                 // W, H ping-pong
    b += 2 * 8 * (I + J) * Kp;                                     // FP64 sums of x and x^2
    b += 2 * 8 * (nnz + kEntryPad) + 4 * std::max<int64_t>(nnz, 1);   // entries twice, entry rows
    b += 4 * (B * I + 1) + 4 * (B * J + 1);                        // part offsets
    // schedule: tasks of every part, Q group records each, padded per XCD
    const int64_t tasks_part = (4 * nnz / B / 16 + 2 * (I + J)) / Q + 2 * B * (qlog + 2);
    b += 8 * B * tasks_part * 16 * (1 + Q);
    b += 8 * B + 4 * B;                                            // per-part tables, scales
    const int64_t splits = 2 * nnz / (Q * 16) + 1;
    b += splits * (4 * Kp + 4);
    int64_t cap = 4096;
    while (cap < 2 * j.n_iter) cap *= 2;
    b += 8 * cap;                                                  // step-size table
    b += 4 * (B * I + 1) + 32 * j.n_heldout;                       // held-out offsets, cells, sums
    if (!j.row) {
        const int64_t vb = j.precision == PSGLD_BF16_DENSE_VALUES ? 2 : 4;
        b += vb * (I * J + (kDenseRowAlign - 1) * I * B);          // dense values, rows padded
        b += (I * J + (kDenseRowAlign - 1) * I * B) / 4 + 4;        // 2-bit cell codes
        b += (J / 128 + B + 1) * int64_t{kDenseMaxRows} * Kp * 4;  // W partials
        b += (B * B + 1) * 64 + (J / 128 + B + 1) * B * 32;        // block and tile lists
    }
    return b + (1 << 20);                                          // small buffers
}

bool job_shape_ok(const psgld_job &j, std::string &why)
{
    if (j.I < 1 || j.J < 1 || j.K < 1 || j.B < 1) return why = "sizes must be >= 1", false;
    if (j.n_iter < 1) return why = "n_iter must be >= 1", false;
    if (j.row ? (!j.col || !j.val || j.nnz < 0) : !j.dense) return why = "coordinates or a dense matrix are required", false;
    if (!j.W0 || !j.H0) return why = "W0 and H0 are required", false;
    if (j.n_heldout < 0 || (j.n_heldout > 0 && (!j.hrow || !j.hcol))) return why = "held-out coordinates are required", false;
    if (j.I * j.J > (int64_t{1} << 34)) return why = "job too large", false;
    return true;
}

}  // namespace

struct psgld_server {
    psgld_server_options opt{};
    hipStream_t stream = nullptr;
    std::deque<Job *> queue;
    std::vector<Job *> running;
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    int64_t used = 0;
    int64_t next_id = 1;
    std::string err;

    psgld_status fail(psgld_status s, const std::string &m)
    {
        err = m;
        return s;
    }
};

namespace {

void unload(psgld_server *srv, Job *j)
{
    if (!j->ctx) return;
    psgld_destroy(j->ctx);
    j->ctx = nullptr;
    srv->used -= j->bytes;
    j->bytes = 0;
}

void fail_job(psgld_server *srv, Job *j, const std::string &why)
{
    j->err = why;
    unload(srv, j);
    j->state = PSGLD_JOB_FAILED;
}

// Creates and loads the job's context on the server's stream.
psgld_status load_job(psgld_server *srv, Job *j)
{
    const psgld_job &s = j->spec;
    psgld_options o;
    psgld_default_options(&o);
    o.seed = s.seed;
    o.burn_in = s.burn_in;
    o.thin = s.thin;
    o.precision = s.precision;
    o.dense_threshold = s.dense_threshold;
    if (s.dense_min_cols > 0) o.dense_min_cols = s.dense_min_cols;
    o.stream = srv->stream;
    o.device = srv->opt.device;
    o.graph_iters = -1;
    o.persistent = srv->opt.persistent ? 1 : 0;
    o.dev_alloc = srv->opt.dev_alloc;
    o.dev_free = srv->opt.dev_free;
    o.alloc_user = srv->opt.alloc_user;
    psgld_status st = psgld_create(s.I, s.J, s.K, s.B, &s.lik, &s.prior, &o, &j->ctx);
    if (st) {
        j->err = psgld_last_error(nullptr);
        return st;
    }
    if (!j->row.empty() || j->dense.empty())
        st = psgld_load_coo(j->ctx, static_cast<int64_t>(j->val.size()), j->row.data(), j->col.data(), j->val.data());
    else
        st = psgld_load_dense(j->ctx, j->dense.data(), j->mask.empty() ? nullptr : j->mask.data());
    if (!st && !j->hrow.empty())
        st = psgld_load_heldout(j->ctx, static_cast<int64_t>(j->hrow.size()), j->hrow.data(), j->hcol.data(),
                                j->hval.empty() ? nullptr : j->hval.data());
    if (!st) st = psgld_set_factors(j->ctx, j->W0.data(), j->H0.data());
    if (!st) st = psgld_memory_bytes(j->ctx, &j->bytes);
    // allocated at the first step: the step-size table and the job tables
    int64_t cap = 4096;
    while (cap < 2 * s.n_iter) cap *= 2;
    j->bytes += 8 * cap + (64 << 10);
    if (st) {
        j->err = psgld_last_error(j->ctx);
        psgld_destroy(j->ctx);
        j->ctx = nullptr;
        j->bytes = 0;
        return st;
    }
    return PSGLD_OK;
}

// Copies a finished job's results to the host and frees its context.
psgld_status retire(psgld_server *srv, Job *j)
{
    const size_t nw = static_cast<size_t>(j->spec.I) * j->spec.K, nh = static_cast<size_t>(j->spec.J) * j->spec.K;
    j->Wm.resize(nw);
    j->Hm.resize(nh);
    j->Wv.resize(nw);
    j->Hv.resize(nh);
    psgld_status st = psgld_posterior_mean(j->ctx, j->Wm.data(), j->Hm.data());
    if (!st) st = psgld_posterior_var(j->ctx, j->Wv.data(), j->Hv.data());
    if (!st && !j->hval.empty()) st = psgld_heldout_rmse(j->ctx, &j->rmse);
    if (st) {
        fail_job(srv, j, psgld_last_error(j->ctx));
        return st;
    }
    unload(srv, j);
    j->state = PSGLD_JOB_DONE;
    return PSGLD_OK;
}

Job *find(psgld_server *srv, int64_t id)
{
    auto it = srv->jobs.find(id);
    return it == srv->jobs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

psgld_status psgld_server_create(const psgld_server_options *opt, psgld_server **out)
{
    if (!opt || !out) return PSGLD_E_ARG;
    *out = nullptr;
    if (opt->hbm_budget <= 0 || opt->max_active < 1 || opt->iters_per_tick < 1 || opt->device < 0 ||
        (opt->dev_alloc == nullptr) != (opt->dev_free == nullptr))
        return PSGLD_E_ARG;
    psgld_server *srv = new (std::nothrow) psgld_server();
    if (!srv) return PSGLD_E_NOMEM;
    srv->opt = *opt;
    if (hipSetDevice(opt->device) != hipSuccess ||
        hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete srv;
        return PSGLD_E_DEVICE;
    }
    *out = srv;
    return PSGLD_OK;
}

psgld_status psgld_server_estimate_bytes(const psgld_job *job, int64_t *bytes)
{
    if (!job || !bytes) return PSGLD_E_ARG;
    std::string why;
    if (!job_shape_ok(*job, why)) return PSGLD_E_ARG;
    *bytes = estimate_bytes(*job);
    return PSGLD_OK;
}

psgld_status psgld_server_submit(psgld_server *srv, const psgld_job *job, int64_t *id)
{
    if (!srv) return PSGLD_E_ARG;
    srv->err.clear();
    if (!job || !id) return srv->fail(PSGLD_E_ARG, "job and id are required");
    std::string why;
    if (!job_shape_ok(*job, why)) return srv->fail(PSGLD_E_ARG, why);
    const int64_t est = estimate_bytes(*job);
    if (est > srv->opt.hbm_budget)
        return srv->fail(PSGLD_E_ARG, "job needs about " + std::to_string(est) + " device bytes, more than the budget");
    auto j = std::make_unique<Job>();
    j->id = srv->next_id++;
    j->spec = *job;
    j->est_bytes = est;
    const size_t K = static_cast<size_t>(job->K), I = static_cast<size_t>(job->I), J = static_cast<size_t>(job->J);
    if (job->row) {
        const size_t n = static_cast<size_t>(job->nnz);
        j->row.assign(job->row, job->row + n);
        j->col.assign(job->col, job->col + n);
        j->val.assign(job->val, job->val + n);
    } else {
        j->dense.assign(job->dense, job->dense + I * J);
        if (job->mask) j->mask.assign(job->mask, job->mask + I * J);
    }
    const size_t nh = static_cast<size_t>(job->n_heldout);
    if (nh) {
        j->hrow.assign(job->hrow, job->hrow + nh);
        j->hcol.assign(job->hcol, job->hcol + nh);
        if (job->hval) j->hval.assign(job->hval, job->hval + nh);
    }
    j->W0.assign(job->W0, job->W0 + I * K);
    j->H0.assign(job->H0, job->H0 + K * J);
    // the copies own the data from here on
    j->spec.row = j->spec.col = j->spec.hrow = j->spec.hcol = nullptr;
    j->spec.val = j->spec.dense = j->spec.hval = j->spec.W0 = j->spec.H0 = nullptr;
    j->spec.mask = nullptr;
    *id = j->id;
    srv->queue.push_back(j.get());
    srv->jobs[j->id] = std::move(j);
    return PSGLD_OK;
}

psgld_status psgld_server_tick(psgld_server *srv, int32_t *n_running, int32_t *n_queued, int32_t *n_retired)
{
    if (!srv) return PSGLD_E_ARG;
    srv->err.clear();
    if (use_device(srv->opt.device) != hipSuccess) return srv->fail(PSGLD_E_DEVICE, "cannot select the device");
    // admission, in submission order
    while (!srv->queue.empty() && static_cast<int32_t>(srv->running.size()) < srv->opt.max_active) {
        Job *j = srv->queue.front();
        if (srv->used + j->est_bytes > srv->opt.hbm_budget) break;
        if (load_job(srv, j)) {
            srv->queue.pop_front();
            j->state = PSGLD_JOB_FAILED;
            continue;
        }
        if (srv->used + j->bytes > srv->opt.hbm_budget) {
            // estimate too low: wait until the actual figure fits
            j->est_bytes = std::max(j->est_bytes, j->bytes);
            psgld_destroy(j->ctx);
            j->ctx = nullptr;
            j->bytes = 0;
            if (j->est_bytes > srv->opt.hbm_budget) {
                srv->queue.pop_front();
                j->err = "job needs more device memory than the budget";
                j->state = PSGLD_JOB_FAILED;
                continue;
            }
            break;
        }
        srv->used += j->bytes;
        srv->queue.pop_front();
        j->state = PSGLD_JOB_RUNNING;
        srv->running.push_back(j);
    }
    // one batched advance of every running job
    int32_t retired = 0;
    if (!srv->running.empty()) {
        std::vector<psgld_ctx *> ctxs;
        std::vector<int64_t> n_iter;
        std::vector<psgld_eps_schedule> sched;
        for (Job *j : srv->running) {
            ctxs.push_back(j->ctx);
            n_iter.push_back(std::min<int64_t>(srv->opt.iters_per_tick, j->spec.n_iter - j->done));
            sched.push_back(j->spec.sched);
        }
        psgld_status st = psgld_step_batch(ctxs.data(), static_cast<int32_t>(ctxs.size()), n_iter.data(), sched.data());
        if (st) {
            for (Job *j : srv->running) {
                const char *m = psgld_last_error(j->ctx);
                if (m && *m) srv->err = m;
            }
            return st == PSGLD_E_DEVICE ? st : srv->fail(st, "batched step failed: " + srv->err);
        }
        if (hipStreamSynchronize(srv->stream) != hipSuccess) {
            (void)hipGetLastError();
            return srv->fail(PSGLD_E_DEVICE, "device error while stepping the running jobs");
        }
        std::vector<Job *> still;
        for (size_t k = 0; k < srv->running.size(); ++k) {
            Job *j = srv->running[k];
            j->done += n_iter[k];
            psgld_status s = psgld_sync(j->ctx);
            if (s) {
                fail_job(srv, j, psgld_last_error(j->ctx));
                ++retired;
            } else if (j->done >= j->spec.n_iter) {
                retire(srv, j);
                ++retired;
            } else {
                still.push_back(j);
            }
        }
        srv->running.swap(still);
    }
    if (n_running) *n_running = static_cast<int32_t>(srv->running.size());
    if (n_queued) *n_queued = static_cast<int32_t>(srv->queue.size());
    if (n_retired) *n_retired = retired;
    return PSGLD_OK;
}

psgld_status psgld_server_job_info(psgld_server *srv, int64_t id, int32_t *state, int64_t *iterations,
                                   int64_t *est_bytes, int64_t *bytes)
{
    if (!srv) return PSGLD_E_ARG;
    srv->err.clear();
    Job *j = find(srv, id);
    if (!j) return srv->fail(PSGLD_E_ARG, "unknown job");
    if (state) *state = j->state;
    if (iterations) *iterations = j->done;
    if (est_bytes) *est_bytes = j->est_bytes;
    if (bytes) *bytes = j->bytes;
    return PSGLD_OK;
}

psgld_status psgld_server_job_result(psgld_server *srv, int64_t id, double *W_mean, double *H_mean,
                                     double *W_var, double *H_var, double *heldout_rmse)
{
    if (!srv) return PSGLD_E_ARG;
    srv->err.clear();
    Job *j = find(srv, id);
    if (!j) return srv->fail(PSGLD_E_ARG, "unknown job");
    if (j->state != PSGLD_JOB_DONE) return srv->fail(PSGLD_E_STATE, "job is not done");
    if (W_mean) std::copy(j->Wm.begin(), j->Wm.end(), W_mean);
    if (H_mean) std::copy(j->Hm.begin(), j->Hm.end(), H_mean);
    if (W_var) std::copy(j->Wv.begin(), j->Wv.end(), W_var);
    if (H_var) std::copy(j->Hv.begin(), j->Hv.end(), H_var);
    if (heldout_rmse) *heldout_rmse = j->rmse;
    return PSGLD_OK;
}

psgld_status psgld_server_release(psgld_server *srv, int64_t id)
{
    if (!srv) return PSGLD_E_ARG;
    srv->err.clear();
    Job *j = find(srv, id);
    if (!j) return srv->fail(PSGLD_E_ARG, "unknown job");
    if (j->state != PSGLD_JOB_DONE && j->state != PSGLD_JOB_FAILED)
        return srv->fail(PSGLD_E_STATE, "job is queued or running");
    srv->jobs.erase(id);
    return PSGLD_OK;
}

const char *psgld_server_last_error(const psgld_server *srv)
{
    return srv ? srv->err.c_str() : "server is NULL";
}

const char *psgld_server_job_error(const psgld_server *srv, int64_t id)
{
    if (!srv) return "server is NULL";
    auto it = srv->jobs.find(id);
    return it == srv->jobs.end() ? "unknown job" : it->second->err.c_str();
}

void psgld_server_destroy(psgld_server *srv)
{
    if (!srv) return;
    (void)use_device(srv->opt.device);
    (void)hipStreamSynchronize(srv->stream);
    for (auto &kv : srv->jobs)
        if (kv.second->ctx) psgld_destroy(kv.second->ctx);
    (void)hipStreamDestroy(srv->stream);
    delete srv;
}

}  // extern "C"
