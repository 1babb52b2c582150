// fgh_server.cpp -- serving loop of libfgh: homogenization solves of mixed size, rule, contrast,
// solver and tolerance submitted as they arrive, admitted by their HBM footprint into a
// caller-provided device pool, and run concurrently (one HIP stream per active slot), each with
// its fields and solver state resident in HBM from admission to retirement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/fgh.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over the caller's pool with coalescing of free neighbours.
class PoolAllocator {
public:
    void init(size_t bytes) { free_[0] = bytes; }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Job {
    int64_t id;
    fgh_request req;
    std::vector<uint8_t> phase;
    std::vector<double> table;
    size_t footprint;
    double t_submit;
};

}  // namespace

struct fgh_server_s {
    char* pool;
    size_t pool_bytes;
    int device;
    int max_active;
    PoolAllocator alloc;
    std::mutex mu;
    std::condition_variable cv_work;   // a job can be admitted / shutdown
    std::condition_variable cv_done;   // a job finished
    std::deque<Job> queue;             // submitted, not admitted (FIFO)
    std::map<int64_t, fgh_result> results;   // finished, not yet handed to the caller
    std::unordered_set<int64_t> live;        // submitted, result not yet handed to the caller
    int waiters = 0;                         // threads blocked in fgh_server_wait
    int64_t next_id = 1;
    int active = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;
    size_t peak_used = 0;
    int peak_active = 0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

size_t grid_points(const fgh_request& r)
{
    size_t n = 1;
    for (int a = 0; a < r.d; a++) n *= (size_t)(r.rule == FGH_GA ? 2 * r.N[a] - 1 : r.N[a]);
    return n;
}

size_t n_points(const fgh_request& r)
{
    size_t n = 1;
    for (int a = 0; a < r.d; a++) n *= (size_t)r.N[a];
    return n;
}

// Pool bytes a request holds while admitted: plan workspace (solver state, spectra, double-grid
// coefficients for Ga), the fluctuation field on the integration grid, the phase map.
fgh_status footprint(const fgh_request& r, size_t* bytes)
{
    size_t ws = 0;
    fgh_status s = fgh_plan_workspace(r.d, r.N, (fgh_rule)r.rule, (fgh_precision)r.precision, FGH_A_PHASE, &ws);
    if (s) return s;
    *bytes = align_up(ws) + align_up(grid_points(r) * r.d * sizeof(double)) + align_up(n_points(r));
    return FGH_OK;
}

void run_job(fgh_server_s* sv, Job& job, hipStream_t stream, size_t off, fgh_result* res)
{
    const fgh_request& r = job.req;
    char* base = sv->pool + off;
    size_t ws = 0;
    (void)fgh_plan_workspace(r.d, r.N, (fgh_rule)r.rule, (fgh_precision)r.precision, FGH_A_PHASE, &ws);
    void* workspace = base;
    double* e = reinterpret_cast<double*>(base + align_up(ws));
    uint8_t* phase = reinterpret_cast<uint8_t*>(base + align_up(ws) + align_up(grid_points(r) * r.d * sizeof(double)));
    fgh_status st = FGH_OK;
    if (hipMemcpyAsync(phase, job.phase.data(), job.phase.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        st = FGH_E_DEVICE;
    fgh_plan plan = nullptr;
    if (!st)
        st = fgh_plan_create(&plan, r.d, r.N, (fgh_rule)r.rule, (fgh_precision)r.precision, FGH_A_PHASE, nullptr, phase, job.table.data(),
                             r.n_phases, r.c_A, r.C_A, workspace, ws, stream);
    fgh_stats stats{};
    if (!st) {
        const fgh_status s2 = fgh_solve(plan, (fgh_solver)r.solver, r.E, 1, r.tol, r.max_iter, e, &stats);
        st = s2;
        double bil = 0.0, flux[3] = {0, 0, 0};
        if (s2 == FGH_OK || s2 == FGH_E_NO_CONVERGENCE) {
            if (fgh_effective(plan, r.E, 1, e, &bil, flux) != FGH_OK) st = FGH_E_DEVICE;
        }
        res->energy = bil;
        for (int c = 0; c < 3; c++) res->flux[c] = flux[c];
        res->iters = stats.iters;
        res->outer_iters = stats.outer_iters;
        res->rel_res_true = stats.rel_res_true;
        res->solve_seconds = stats.seconds;
    }
    if (plan) fgh_plan_destroy(plan);
    res->status = st;
}

void worker_main(fgh_server_s* sv)
{
    (void)hipSetDevice(sv->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        Job job;
        size_t off = 0;
        bool admitted = false;
        double t_admit = 0.0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // admit the head of the queue once its footprint fits the free pool (FIFO); when
            // nothing runs the whole pool is free, and every queued footprint fits the pool
            sv->cv_work.wait(lk, [&] {
                if (sv->stop) return true;
                if (sv->queue.empty()) return false;
                size_t o = 0;
                if (sv->alloc.alloc(sv->queue.front().footprint, &o)) {
                    off = o;
                    admitted = true;
                    return true;
                }
                return false;
            });
            if (!admitted) break;
            job = std::move(sv->queue.front());
            sv->queue.pop_front();
            sv->active++;
            sv->peak_active = std::max(sv->peak_active, sv->active);
            sv->peak_used = std::max(sv->peak_used, sv->alloc.used());
            t_admit = sv->now();
        }
        fgh_result res{};
        res.id = job.id;
        res.t_submit = job.t_submit;
        res.t_admit = t_admit;
        if (have_stream)
            run_job(sv, job, stream, off, &res);
        else
            res.status = FGH_E_DEVICE;
        res.t_done = sv->now();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->alloc.release(off, job.footprint);
            sv->active--;
            sv->results[job.id] = res;
        }
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

fgh_status fgh_request_footprint(const fgh_request* r, size_t* bytes)
{
    if (!r || !bytes) return FGH_E_INVALID;
    return footprint(*r, bytes);
}

fgh_status fgh_server_create(fgh_server* out, void* pool, size_t pool_bytes, int max_active, int device)
{
    if (!out || !pool || pool_bytes < kAlign || max_active < 1 || max_active > 16) return FGH_E_INVALID;
    if (reinterpret_cast<uintptr_t>(pool) % kAlign) return FGH_E_WORKSPACE;
    *out = nullptr;
    fgh_server_s* sv = new (std::nothrow) fgh_server_s();
    if (!sv) return FGH_E_DEVICE;
    sv->pool = static_cast<char*>(pool);
    sv->pool_bytes = pool_bytes / kAlign * kAlign;
    sv->device = device;
    sv->max_active = max_active;
    sv->alloc.init(sv->pool_bytes);
    sv->t0 = std::chrono::steady_clock::now();
    try {
        for (int i = 0; i < max_active; i++) sv->workers.emplace_back(worker_main, sv);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        for (auto& t : sv->workers) t.join();
        delete sv;
        return FGH_E_DEVICE;
    }
    *out = sv;
    return FGH_OK;
}

fgh_status fgh_server_submit(fgh_server sv, const fgh_request* r, int64_t* id)
{
    if (!sv || !r || !id) return FGH_E_INVALID;
    if (!r->phase || !r->phase_table || r->n_phases < 1 || r->n_phases > 16) return FGH_E_INVALID;
    if (r->solver == FGH_EYRE_MILTON && r->rule == FGH_GA) return FGH_E_UNSUPPORTED;
    if (!(r->tol > 0.0 && r->tol < 1.0) || r->max_iter < 1) return FGH_E_INVALID;
    Job job;
    job.req = *r;
    fgh_status s = footprint(*r, &job.footprint);
    if (s) return s;
    if (job.footprint > sv->pool_bytes) return FGH_E_WORKSPACE;
    const size_t np = n_points(*r);
    job.phase.assign(r->phase, r->phase + np);
    const int nc = r->d == 2 ? 3 : 6;
    job.table.assign(r->phase_table, r->phase_table + (size_t)r->n_phases * nc);
    job.req.phase = nullptr;
    job.req.phase_table = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        job.id = sv->next_id++;
        job.t_submit = sv->now();
        *id = job.id;
        sv->live.insert(job.id);
        sv->queue.push_back(std::move(job));
    }
    sv->cv_work.notify_all();
    return FGH_OK;
}

fgh_status fgh_server_poll(fgh_server sv, int64_t id, fgh_result* out)
{
    if (!sv || !out) return FGH_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->live.count(id)) return FGH_E_INVALID;  // never issued, or already handed out
    auto it = sv->results.find(id);
    if (it == sv->results.end()) return FGH_E_NO_CONVERGENCE;  // not finished yet
    *out = it->second;
    sv->results.erase(it);
    sv->live.erase(id);
    return FGH_OK;
}

fgh_status fgh_server_wait(fgh_server sv, int64_t id, fgh_result* out)
{
    if (!sv || !out) return FGH_E_INVALID;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (!sv->live.count(id)) return FGH_E_INVALID;
    sv->waiters++;
    // another thread may take the same result first: then the id is no longer live
    sv->cv_done.wait(lk, [&] { return sv->results.count(id) > 0 || !sv->live.count(id); });
    fgh_status st = FGH_E_INVALID;
    auto it = sv->results.find(id);
    if (it != sv->results.end()) {
        *out = it->second;
        sv->results.erase(it);
        sv->live.erase(id);
        st = FGH_OK;
    }
    sv->waiters--;
    if (sv->waiters == 0) sv->cv_done.notify_all();  // fgh_server_destroy may be waiting for this
    return st;
}

fgh_status fgh_server_drain(fgh_server sv)
{
    if (!sv) return FGH_E_INVALID;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->queue.empty() && sv->active == 0; });
    return FGH_OK;
}

fgh_status fgh_server_stats(fgh_server sv, double* now_seconds, size_t* peak_pool_bytes, int* peak_active)
{
    if (!sv) return FGH_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (now_seconds) *now_seconds = sv->now();
    if (peak_pool_bytes) *peak_pool_bytes = sv->peak_used;
    if (peak_active) *peak_active = sv->peak_active;
    return FGH_OK;
}

void fgh_server_destroy(fgh_server sv)
{
    if (!sv) return;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        // let admitted work finish; queued, not admitted requests are discarded with the status
        // FGH_E_CANCELLED, so that a thread waiting for one of them returns
        const double t = sv->now();
        for (const Job& job : sv->queue) {
            fgh_result r{};
            r.id = job.id;
            r.status = FGH_E_CANCELLED;
            r.t_submit = job.t_submit;
            r.t_admit = r.t_done = t;
            sv->results[job.id] = r;
        }
        sv->queue.clear();
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
    for (auto& t : sv->workers) t.join();
    {
        // every request has a result now: wait until the threads blocked in fgh_server_wait
        // have taken theirs and left, then free the server
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.notify_all();
        sv->cv_done.wait(lk, [&] { return sv->waiters == 0; });
    }
    delete sv;
}

}  // extern "C"
