// fgh_server.cpp -- serving loop of libfgh: homogenization solves of mixed size, rule, contrast,
// solver and tolerance submitted as they arrive, admitted by their HBM footprint into a
// caller-provided device pool, and run concurrently (one HIP stream per worker slot), each with
// its fields and solver state resident in HBM from admission to retirement.  A slot that admits a
// request whose shape can share launches also admits queued requests of the same size class and
// solves them together (fgh_solve_batch): one launch per pass for all of them; each retires, and
// frees its pool memory, as soon as its own solve has finished.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
#include "fgh_batch.hpp"

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
    double work;  // predicted loop bodies, up to a common factor (predicted_work)
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
    int peak_batch = 0;    // largest group solved together
    long long batches = 0; // groups admitted

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

constexpr int kServeBatch = 8;  // members of one shared-launch batch
// Requests are grouped only on integration grids up to this many points (45^3, 2D up to 243^2 and
// the Ga grids 81^2, 125^2): measured on MI355X with four slots, shared launches raise capacity
// 1.3-2x there, while on 81^3 and 135^3 one request's launches already fill the GPU and a group,
// which runs until its slowest member finishes, lowers capacity by about 10 %.
constexpr size_t kGroupMaxPoints = 262144;

// Loop bodies a request is expected to take, up to a factor common to its size class: the
// contrast kappa = C_A / c_A (the request's bounds, else its phase table's) gives sqrt(kappa)
// log(2 / tol) for CG, Chebyshev and Eyre-Milton and kappa log(2 / tol) for Richardson.
double predicted_work(const fgh_request& r, const std::vector<double>& table)
{
    double kappa = (r.c_A > 0.0 && r.C_A > 0.0) ? r.C_A / r.c_A : fgh::phase_table_contrast(r.d, table.data(), r.n_phases);
    if (!(kappa >= 1.0)) kappa = 1.0;
    const double steps = std::log(2.0 / r.tol);
    return (r.solver == FGH_RICHARDSON ? kappa : std::sqrt(kappa)) * steps;
}

// A group runs until its slowest member has finished and holds its worker slot until then:
// members join the head only if their predicted work is within a factor kGroupWorkRatio of the
// head's.  On a 2000-request mix with contrasts spread over three decades, unrestricted groups
// cost 5 % of capacity against no grouping at all.
constexpr double kGroupWorkRatio = 2.0;
bool similar_work(double a, double b) { return a <= kGroupWorkRatio * b && b <= kGroupWorkRatio * a; }

// Requests that can be solved together: same grid, rule, precision, solver and iteration cap.
bool same_class(const fgh_request& a, const fgh_request& b)
{
    if (a.d != b.d || a.rule != b.rule || a.precision != b.precision || a.solver != b.solver ||
        a.max_iter != b.max_iter)
        return false;
    for (int k = 0; k < a.d; k++)
        if (a.N[k] != b.N[k]) return false;
    return true;
}

struct Admitted {
    Job job;
    size_t off = 0;
    double t_admit = 0.0;
    fgh_plan plan = nullptr;
    double* e = nullptr;
    fgh_result res{};
    bool retired = false;  // fgh_solve_batch finished it (res filled)
    bool posted = false;
};

// Finished request: its result is posted and its pool memory released.
void post(fgh_server_s* sv, Admitted& a)
{
    if (a.posted) return;
    a.res.id = a.job.id;
    a.res.t_submit = a.job.t_submit;
    a.res.t_admit = a.t_admit;
    a.res.t_done = sv->now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->alloc.release(a.off, a.job.footprint);
        sv->active--;
        sv->results[a.job.id] = a.res;
    }
    a.posted = true;
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
}

// Plan of an admitted request inside its pool block: workspace, fluctuation field, phase map.
fgh_status make_plan(fgh_server_s* sv, Admitted& a, hipStream_t stream)
{
    const fgh_request& r = a.job.req;
    char* base = sv->pool + a.off;
    size_t ws = 0;
    (void)fgh_plan_workspace(r.d, r.N, (fgh_rule)r.rule, (fgh_precision)r.precision, FGH_A_PHASE, &ws);
    a.e = reinterpret_cast<double*>(base + align_up(ws));
    uint8_t* phase = reinterpret_cast<uint8_t*>(base + align_up(ws) + align_up(grid_points(r) * r.d * sizeof(double)));
    if (hipMemcpyAsync(phase, a.job.phase.data(), a.job.phase.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return FGH_E_DEVICE;
    return fgh_plan_create(&a.plan, r.d, r.N, (fgh_rule)r.rule, (fgh_precision)r.precision, FGH_A_PHASE, nullptr,
                           phase, a.job.table.data(), r.n_phases, r.c_A, r.C_A, base, ws, stream);
}

// Result of a finished solve: the effective quantities of its fluctuation.
void fill_result(Admitted& a, const fgh_stats& st)
{
    const fgh_request& r = a.job.req;
    double bil = 0.0, flux[3] = {0, 0, 0};
    int status = st.status;
    if (status == FGH_OK || status == FGH_E_NO_CONVERGENCE)
        if (fgh_effective(a.plan, r.E, 1, a.e, &bil, flux) != FGH_OK) status = FGH_E_DEVICE;
    a.res.status = status;
    a.res.energy = bil;
    for (int c = 0; c < 3; c++) a.res.flux[c] = flux[c];
    a.res.iters = st.iters;
    a.res.outer_iters = st.outer_iters;
    a.res.rel_res_true = st.rel_res_true;
    a.res.solve_seconds = st.seconds;
}

struct BatchRun {
    fgh_server_s* sv;
    std::vector<Admitted*> members;  // with a plan, in the order given to fgh_solve_batch
    std::vector<fgh_stats> stats;
};

// Called by fgh_solve_batch as member k finishes: result posted, and for k >= 1 its plan and pool
// memory released at once (member 0 hosts the batch's shared stream until the call returns).
void retire_member(void* user, int k)
{
    BatchRun* br = static_cast<BatchRun*>(user);
    Admitted& a = *br->members[k];
    fill_result(a, br->stats[k]);
    a.retired = true;
    if (k == 0) return;
    fgh_plan_destroy(a.plan);
    a.plan = nullptr;
    post(br->sv, a);
}

void run_batch(fgh_server_s* sv, std::vector<Admitted>& B, hipStream_t stream)
{
    BatchRun br{sv, {}, {}};
    for (Admitted& a : B) {
        const fgh_status st = make_plan(sv, a, stream);
        if (st) {
            if (a.plan) fgh_plan_destroy(a.plan);
            a.plan = nullptr;
            a.res.status = st;
            post(sv, a);
        } else {
            br.members.push_back(&a);
        }
    }
    const int n = (int)br.members.size();
    if (n > 0) {
        const fgh_request& r0 = br.members[0]->job.req;
        const int d = r0.d;
        std::vector<fgh_plan> plans(n);
        std::vector<double> E((size_t)n * d), tol(n);
        std::vector<double*> e(n);
        for (int k = 0; k < n; k++) {
            const Admitted& a = *br.members[k];
            plans[k] = a.plan;
            for (int c = 0; c < d; c++) E[(size_t)k * d + c] = a.job.req.E[c];
            tol[k] = a.job.req.tol;
            e[k] = a.e;
        }
        br.stats.assign(n, fgh_stats{});
        const fgh_status st = fgh_solve_batch(plans.data(), n, (fgh_solver)r0.solver, E.data(), tol.data(), r0.max_iter,
                                              e.data(), br.stats.data(), retire_member, &br);
        for (int k = 0; k < n; k++) {
            Admitted& a = *br.members[k];
            if (a.posted) continue;
            if (!a.retired) a.res.status = st != FGH_OK ? st : FGH_E_DEVICE;  // the batch failed before it finished
            if (a.plan) fgh_plan_destroy(a.plan);
            a.plan = nullptr;
            post(sv, a);
        }
    }
}

void worker_main(fgh_server_s* sv)
{
    (void)hipSetDevice(sv->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        std::vector<Admitted> batch;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // admit the head of the queue once its footprint fits the free pool (FIFO); when
            // nothing runs the whole pool is free, and every queued footprint fits the pool
            size_t off = 0;
            bool admitted = false;
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
            const double t_admit = sv->now();
            batch.reserve(kServeBatch);  // members are referenced by address while the group runs
            batch.emplace_back();
            batch.back().job = std::move(sv->queue.front());
            batch.back().off = off;
            batch.back().t_admit = t_admit;
            sv->queue.pop_front();
            // queued requests of the head's size class join it while they fit the pool
            const fgh_request h = batch.front().job.req;
            const double hw = batch.front().job.work;
            if (grid_points(h) <= kGroupMaxPoints && fgh::batch_shares_launches(h.d, h.N, h.rule, h.precision, h.solver))
                for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)batch.size() < kServeBatch;) {
                    size_t o = 0;
                    if (same_class(it->req, h) && similar_work(it->work, hw) && sv->alloc.alloc(it->footprint, &o)) {
                        batch.emplace_back();
                        batch.back().job = std::move(*it);
                        batch.back().off = o;
                        batch.back().t_admit = t_admit;
                        it = sv->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            sv->active += (int)batch.size();
            sv->peak_active = std::max(sv->peak_active, sv->active);
            sv->peak_used = std::max(sv->peak_used, sv->alloc.used());
            sv->peak_batch = std::max(sv->peak_batch, (int)batch.size());
            sv->batches++;
        }
        if (have_stream) {
            run_batch(sv, batch, stream);
        } else {
            for (Admitted& a : batch) {
                a.res.status = FGH_E_DEVICE;
                post(sv, a);
            }
        }
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
    job.work = predicted_work(job.req, job.table);
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

fgh_status fgh_server_batch_stats(fgh_server sv, int* peak_batch, int64_t* batches)
{
    if (!sv) return FGH_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (peak_batch) *peak_batch = sv->peak_batch;
    if (batches) *batches = sv->batches;
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
