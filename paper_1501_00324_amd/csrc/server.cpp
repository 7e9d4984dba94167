// Solve server with continuous batching.
//
// Requests (a matrix handle and k right-hand sides) are queued by
// server_submit and admitted in arrival order while the device-memory
// budget and the slot count allow.  One worker thread owns the device work:
// every admitted request becomes a member of the batch of its launch class
// (slot width x column-count class), which the CG engine advances with
// shared launches (one batched product and a fixed number of vector /
// reduction kernels per iteration for all members).  Membership changes
// only at chunk boundaries (every check_every iterations): finished
// requests leave and queued requests join.  A member's arithmetic does not
// depend on the other members, so every result is bitwise the result of
// solving that request alone.
//
// One step of the worker: the joiners' start (diagonal, first residual) and
// one chunk of every class are enqueued first -- the classes on separate
// streams, so their launches overlap on the device -- together with the
// copy of every class's column states to pinned host memory; then the
// worker waits once.  Descriptors are uploaded in stream order (no host
// wait); a class replays a captured graph only once its membership has
// stayed the same for a step (a graph is not worth capturing for one
// chunk).  Request state comes from a pool of device blocks kept by the
// server, so admitting and finishing requests calls neither hipMalloc nor
// hipFree (which waits for the whole device) once the pool is warm.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "internal.h"

namespace fs {
namespace {

double clock_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(
               steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    fs_csr *A = nullptr;
    int32_t k = 1;
    const double *B = nullptr;
    double *X = nullptr;
    double t_submit = 0.0, t_admit = 0.0;
    int64_t footprint = 0;         // Krylov state bytes
    CgSys sys;
    void *block = nullptr;         // pool block holding sys's state
    int64_t block_bytes = 0;
};

// Streams the launch classes are spread over (at most the hardware queues
// of a process).
constexpr int kServerStreams = 4;

// Pool block size class of a request of `bytes`: rounded up to 1/8 of its
// power of two (at most 12.5% unused), so blocks are reused across
// neighbouring sizes.
int64_t pool_class(int64_t bytes)
{
    int64_t p = 256;
    while (p < bytes) p <<= 1;
    const int64_t step = std::max<int64_t>(256, p / 8);
    return (bytes + step - 1) / step * step;
}

int64_t krylov_bytes(const fs_csr *A, int32_t k, int32_t precond)
{
    const int64_t n = A->n_rows;
    const int64_t snb = engine_spmv_blocks(A->n_groups);
    const int64_t vnb = engine_vec_blocks(A->n_rows, k);
    return 5 * n * k * 8 + (precond ? n * 8 : 0) +
           int64_t(sizeof(ColState)) * k + 4 +
           8 * 3 * int64_t(k) * std::max(snb, vnb);
}

}  // namespace
}  // namespace fs

struct fs_server {
    fs_server_opts o{};
    int device = 0;
    hipStream_t s = nullptr;                   // streams[0]
    hipStream_t streams[fs::kServerStreams] = {};
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<fs::Request *> queue;           // submitted, not admitted
    std::vector<fs::Request *> active;         // admitted, running
    std::vector<fs_server_done> done;          // finished, not polled
    int64_t used = 0;                          // budget in use
    std::map<const fs_csr *, int32_t> mat_refs;
    fs_status fatal = FS_OK;
    std::string fatal_msg;
    int64_t peak_used = 0;
    int32_t peak_active = 0;
    // running members per slot width and column-count class; joiners
    fs::Batch batch[2 * fs::kKmClasses], join[2 * fs::kKmClasses];
    int32_t stable[2 * fs::kKmClasses] = {};   // steps without a change
    // free device blocks by size class (worker thread only)
    std::multimap<int64_t, void *> pool;
    int64_t pool_bytes = 0;                    // all blocks, free or in use
    uint64_t submitted = 0, completed = 0;
};

namespace fs {
namespace {

hipStream_t class_stream(const fs_server *S, int32_t cls)
{
    return S->streams[cls % kServerStreams];
}

int32_t class_of(const Request *R)
{
    return (R->A->host.vec - 1) * kKmClasses + km_index(R->k);
}

// A block of at least `bytes` from the pool (or a new one).
fs_status pool_get(fs_server *S, int64_t bytes, void **out, int64_t *got)
{
    const int64_t c = pool_class(bytes);
    auto it = S->pool.find(c);
    if (it != S->pool.end()) {
        *out = it->second;
        *got = c;
        S->pool.erase(it);
        return FS_OK;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size_t(c));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give the free blocks back and try once more
        for (auto &f : S->pool) {
            (void)hipFree(f.second);
            S->pool_bytes -= f.first;
        }
        S->pool.clear();
        e = hipMalloc(&p, size_t(c));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FS_E_OOM, "server state block (%lld bytes): %s",
                             static_cast<long long>(c), hipGetErrorString(e));
        }
    }
    S->pool_bytes += c;
    *out = p;
    *got = c;
    return FS_OK;
}

// Return a block; free blocks beyond the budget are released.
void pool_put(fs_server *S, void *p, int64_t bytes)
{
    if (!p) return;
    S->pool.emplace(bytes, p);
    while (S->pool_bytes > S->o.hbm_budget_bytes && !S->pool.empty()) {
        auto it = std::prev(S->pool.end());
        (void)hipFree(it->second);
        S->pool_bytes -= it->first;
        S->pool.erase(it);
    }
}

// Enqueue the solution's way out (caller numbering) on the class stream.
fs_status finish_enqueue(fs_server *S, Request *R, const ColState *cols,
                         hipStream_t st)
{
    // a column with b = 0 returns x = 0
    for (int32_t c = 0; c < R->k; ++c)
        if (cols[c].bnorm2 == 0.0)
            FS_HIP_TRY(hipMemset2DAsync(static_cast<double *>(R->sys.x) + c,
                                        sizeof(double) * size_t(R->k), 0,
                                        sizeof(double), size_t(R->sys.n),
                                        st));
    FS_HIP_TRY(permute_rows(R->A->n_rows, R->k,
                            R->A->host.identity ? nullptr : R->A->d_perm,
                            static_cast<const double *>(R->sys.x), R->k, R->X,
                            R->k, false, st));
    (void)S;
    return FS_OK;
}

// After the streams have drained: the done record, memory back.
void finish_complete(fs_server *S, Request *R, const ColState *cols)
{
    fs_server_done d;
    std::memset(&d, 0, sizeof d);
    d.req_id = R->id;
    d.k = R->k;
    d.t_submit_ms = R->t_submit;
    d.t_admit_ms = R->t_admit;
    d.t_done_ms = clock_ms();
    d.info.status = FS_OK;
    for (int32_t c = 0; c < R->k; ++c) {
        const ColState &cs = cols[c];
        fs_status st = cs.status == CG_CONVERGED ? FS_OK
                     : cs.status == CG_MAXIT ? FS_E_NOT_CONVERGED
                                            : FS_E_BREAKDOWN;
        if (st != FS_OK && d.info.status == FS_OK) d.info.status = st;
        if (st == FS_E_BREAKDOWN) d.info.status = st;
        d.info.iters = std::max(d.info.iters, cs.iter);
        d.info.replacements += cs.replacements;
        const double rel = cs.bnorm2 > 0 ? std::sqrt(cs.rr_true / cs.bnorm2) : 0;
        d.info.relres = std::max(d.info.relres, rel);
    }
    d.info.ms = d.t_done_ms - d.t_submit_ms;
    sys_free(R->sys);
    pool_put(S, R->block, R->block_bytes);
    std::lock_guard<std::mutex> lk(S->mu);
    S->used -= R->footprint;
    auto it = S->mat_refs.find(R->A);
    if (it != S->mat_refs.end() && --it->second == 0) {
        S->used -= R->A->device_bytes;
        S->mat_refs.erase(it);
    }
    S->done.push_back(d);
    S->completed++;
    delete R;
}

fs_status sync_streams(fs_server *S)
{
    for (hipStream_t st : S->streams) FS_HIP_TRY(hipStreamSynchronize(st));
    return FS_OK;
}

// Admit queued requests in arrival order while they fit.
void admit(fs_server *S, std::vector<Request *> &joining)
{
    std::lock_guard<std::mutex> lk(S->mu);
    while (!S->queue.empty() &&
           int32_t(S->active.size() + joining.size()) < S->o.max_slots) {
        Request *R = S->queue.front();
        const bool mat_new = S->mat_refs.find(R->A) == S->mat_refs.end();
        const int64_t need = R->footprint + (mat_new ? R->A->device_bytes : 0);
        if (S->used + need > S->o.hbm_budget_bytes) break;
        S->used += need;
        S->mat_refs[R->A]++;
        S->peak_used = std::max(S->peak_used, S->used);
        S->queue.pop_front();
        R->t_admit = clock_ms();
        joining.push_back(R);
    }
}

fs_status step(fs_server *S)
{
    constexpr int32_t NC = 2 * kKmClasses;
    std::vector<Request *> joining;
    admit(S, joining);
    // joiners: state from the pool, b into layout order, x = 0, then their
    // start (Jacobi diagonal, first residual) per class
    for (Request *R : joining) {
        const int64_t need = sys_block_bytes(R->A, R->k, ST_F64, S->o.precond);
        FS_TRY(pool_get(S, need, &R->block, &R->block_bytes));
        sys_alloc_in(R->sys, R->A, R->k, VT_F64, ST_F64, S->o.precond,
                     R->block);
        R->sys.rtol = S->o.rtol;
        R->sys.maxit = S->o.maxit;
        const hipStream_t st = class_stream(S, class_of(R));
        FS_HIP_TRY(permute_rows(R->A->n_rows, R->k,
                                R->A->host.identity ? nullptr : R->A->d_perm,
                                R->B, R->k, static_cast<double *>(R->sys.b),
                                R->k, true, st));
        FS_HIP_TRY(fill_f64(int64_t(R->sys.n) * R->k, 0.0,
                            static_cast<double *>(R->sys.x), st));
    }
    bool joined[NC] = {};
    for (int32_t cls = 0; cls < NC && !joining.empty(); ++cls) {
        Batch &J = S->join[cls];
        J.members.clear();
        for (Request *R : joining)
            if (class_of(R) == cls) J.members.push_back(&R->sys);
        if (J.members.empty()) continue;
        joined[cls] = true;
        J.vt = VT_F64;
        J.st = ST_F64;
        J.vec = 1 + cls / kKmClasses;
        const hipStream_t st = class_stream(S, cls);
        FS_TRY(batch_build(J, st, true));
        if (S->o.precond) FS_HIP_TRY(engine_diag_inv(J.L, st));
        FS_HIP_TRY(engine_residual(J.L, 0, true, st));
    }
    if (!joining.empty()) {
        std::lock_guard<std::mutex> lk(S->mu);
        for (Request *R : joining) S->active.push_back(R);
        S->peak_active = std::max(S->peak_active, int32_t(S->active.size()));
    }
    if (S->active.empty()) return sync_streams(S);
    // members of every class (in admission order)
    std::vector<Request *> mem[NC];
    for (Request *R : S->active) mem[class_of(R)].push_back(R);
    // one chunk of every class, and the copy of its column states
    for (int32_t cls = 0; cls < NC; ++cls) {
        if (mem[cls].empty()) continue;
        Batch &B = S->batch[cls];
        const hipStream_t st = class_stream(S, cls);
        std::vector<CgSys *> syss;
        for (Request *R : mem[cls]) syss.push_back(&R->sys);
        if (syss != B.members || joined[cls]) {
            // membership changed: new descriptors (the graph goes too)
            B.members = syss;
            B.vt = VT_F64;
            B.st = ST_F64;
            B.vec = 1 + cls / kKmClasses;
            FS_TRY(batch_build(B, st, true));
            S->stable[cls] = 0;
        } else {
            S->stable[cls]++;
        }
        FS_TRY(batch_iterations(B, S->o.check_every,
                                S->o.use_graph != 0 && S->stable[cls] > 0,
                                st));
        FS_TRY(batch_stage_states(B, st));
    }
    FS_TRY(sync_streams(S));
    // columns whose recurrence residual met the tolerance: confirm against
    // the true residual (replacing it where it misses)
    bool any_met = false;
    for (int32_t cls = 0; cls < NC; ++cls) {
        if (mem[cls].empty()) continue;
        Batch &B = S->batch[cls];
        bool met = false;
        for (int32_t i = 0; i < B.L.ncols; ++i)
            met |= B.h_stage[i].status == CG_RECURRENCE_MET;
        if (!met) continue;
        any_met = true;
        const hipStream_t st = class_stream(S, cls);
        FS_HIP_TRY(engine_residual(B.L, 1, false, st));
        FS_TRY(batch_stage_states(B, st));
    }
    if (any_met) {
        FS_TRY(sync_streams(S));
        for (int32_t cls = 0; cls < NC; ++cls) {
            if (mem[cls].empty()) continue;
            Batch &B = S->batch[cls];
            bool pend = false;
            for (int32_t i = 0; i < B.L.ncols; ++i)
                pend |= B.h_stage[i].pending != 0;
            if (pend)
                FS_HIP_TRY(engine_pupdate_pending(B.L, class_stream(S, cls)));
        }
    }
    // members whose columns have all stopped
    bool any_fail = false;
    std::vector<std::vector<bool>> fin(NC);
    for (int32_t cls = 0; cls < NC; ++cls) {
        if (mem[cls].empty()) continue;
        Batch &B = S->batch[cls];
        fin[cls].assign(mem[cls].size(), false);
        int32_t j = 0;
        bool fail = false;
        for (size_t m = 0; m < mem[cls].size(); ++m) {
            bool all = true;
            for (int32_t c = 0; c < mem[cls][m]->k; ++c, ++j) {
                const int32_t st = B.h_stage[j].status;
                all &= st != CG_RUNNING;
                fail |= st == CG_MAXIT || st == CG_BREAKDOWN;
            }
            fin[cls][m] = all;
        }
        if (fail) {                    // final true residual for reports
            FS_HIP_TRY(engine_residual(B.L, 2, false, class_stream(S, cls)));
            FS_TRY(batch_stage_states(B, class_stream(S, cls)));
            any_fail = true;
        }
    }
    if (any_fail) FS_TRY(sync_streams(S));
    // finished requests leave: their solutions out, then one wait
    std::vector<std::pair<Request *, std::vector<ColState>>> out;
    for (int32_t cls = 0; cls < NC; ++cls) {
        if (mem[cls].empty()) continue;
        Batch &B = S->batch[cls];
        int32_t j = 0;
        for (size_t m = 0; m < mem[cls].size(); ++m) {
            Request *R = mem[cls][m];
            const int32_t j0 = j;
            j += R->k;
            if (!fin[cls][m]) continue;
            std::vector<ColState> cols(B.h_stage + j0, B.h_stage + j0 + R->k);
            FS_TRY(finish_enqueue(S, R, cols.data(), class_stream(S, cls)));
            out.emplace_back(R, std::move(cols));
        }
    }
    if (out.empty()) return FS_OK;
    FS_TRY(sync_streams(S));
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto &o : out)
            S->active.erase(std::find(S->active.begin(), S->active.end(),
                                      o.first));
    }
    for (auto &o : out) finish_complete(S, o.first, o.second.data());
    return FS_OK;
}

void worker_main(fs_server *S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] {
                return S->stop || !S->queue.empty() || !S->active.empty();
            });
            if (S->stop && S->queue.empty() && S->active.empty()) return;
            if (S->fatal != FS_OK) return;
        }
        fs_status st = step(S);
        if (st != FS_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->fatal = st;
            S->fatal_msg = fs_last_error();
            S->cv.notify_all();
            return;
        }
        S->cv.notify_all();
    }
}

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" {

fs_status server_opts_default(fs_server_opts *o)
{
    if (!o) return set_error(FS_E_ARG, "NULL opts");
    std::memset(o, 0, sizeof *o);
    o->hbm_budget_bytes = int64_t(16) << 30;
    o->max_slots = 64;
    o->check_every = 16;
    o->precond = FS_PC_JACOBI;
    o->rtol = 1e-8;
    o->maxit = 20000;
    o->use_graph = 1;
    return FS_OK;
}

fs_status server_create(const fs_server_opts *opts, fs_server_t *out)
{
    if (!out) return set_error(FS_E_ARG, "NULL output pointer");
    *out = nullptr;
    fs_server_opts o;
    server_opts_default(&o);
    if (opts) o = *opts;
    if (o.hbm_budget_bytes <= 0) o.hbm_budget_bytes = int64_t(16) << 30;
    if (o.max_slots <= 0) o.max_slots = 64;
    if (o.check_every <= 0) o.check_every = 16;
    if (o.rtol <= 0) o.rtol = 1e-8;
    if (o.maxit <= 0) o.maxit = 20000;
    if (o.precond != FS_PC_NONE && o.precond != FS_PC_JACOBI)
        return set_error(FS_E_ARG, "unknown preconditioner %d", o.precond);
    fs_server *S = new (std::nothrow) fs_server();
    if (!S) return set_error(FS_E_OOM, "host allocation failed");
    S->o = o;
    hipError_t e = hipGetDevice(&S->device);
    for (int i = 0; i < kServerStreams && e == hipSuccess; ++i)
        e = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
    if (e != hipSuccess) {
        for (hipStream_t st : S->streams)
            if (st) (void)hipStreamDestroy(st);
        delete S;
        return set_error(FS_E_HIP, "server stream: %s", hipGetErrorString(e));
    }
    S->s = S->streams[0];
    S->worker = std::thread(worker_main, S);
    *out = S;
    return FS_OK;
}

fs_status server_submit(fs_server_t S, fs_csr_t A, int32_t k, const double *B,
                        double *X, uint64_t *req_id)
{
    if (!S || !A) return set_error(FS_E_ARG, "NULL server or matrix");
    if (A->n_rows != A->n_cols)
        return set_error(FS_E_NOT_SQUARE, "CG needs a square matrix");
    if (k < 1 || k > 16) return set_error(FS_E_ARG, "k = %d, must be in [1, 16]", k);
    if (A->n_rows > 0 && (!B || !X)) return set_error(FS_E_ARG, "NULL block");
    if (A->device != S->device)
        return set_error(FS_E_ARG, "matrix lives on another device");
    Request *R = new (std::nothrow) Request();
    if (!R) return set_error(FS_E_OOM, "host allocation failed");
    R->A = A;
    R->k = k;
    R->B = B;
    R->X = X;
    R->t_submit = clock_ms();
    R->footprint = krylov_bytes(A, k, S->o.precond);
    if (R->footprint + A->device_bytes > S->o.hbm_budget_bytes) {
        delete R;
        return set_error(FS_E_BUDGET,
                         "request needs %lld bytes, budget is %lld",
                         (long long)(R->footprint + A->device_bytes),
                         (long long)S->o.hbm_budget_bytes);
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->fatal != FS_OK) {
            delete R;
            return set_error(S->fatal, "server stopped: %s",
                             S->fatal_msg.c_str());
        }
        R->id = S->next_id++;
        S->submitted++;
        S->queue.push_back(R);
    }
    S->cv.notify_all();
    if (req_id) *req_id = R->id;
    return FS_OK;
}

fs_status server_poll(fs_server_t S, fs_server_done *done, int32_t cap,
                      int32_t *n)
{
    if (!S || !n || (cap > 0 && !done)) return set_error(FS_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t m = std::min<int32_t>(cap, int32_t(S->done.size()));
    for (int32_t i = 0; i < m; ++i) done[i] = S->done[size_t(i)];
    S->done.erase(S->done.begin(), S->done.begin() + m);
    *n = m;
    if (S->fatal != FS_OK)
        return set_error(S->fatal, "server stopped: %s", S->fatal_msg.c_str());
    return FS_OK;
}

fs_status server_stats(fs_server_t S, fs_server_stats *st)
{
    if (!S || !st) return set_error(FS_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(st, 0, sizeof *st);
    st->queued = int32_t(S->queue.size());
    st->active = int32_t(S->active.size());
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->bytes_in_use = S->used;
    st->peak_bytes = S->peak_used;
    st->peak_active = S->peak_active;
    return FS_OK;
}

fs_status server_destroy(fs_server_t S)
{
    if (!S) return FS_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (hipStream_t st : S->streams) (void)hipStreamSynchronize(st);
    // requests left behind after a fatal error
    for (Request *R : S->active) {
        sys_free(R->sys);
        if (R->block) (void)hipFree(R->block);
        delete R;
    }
    for (Request *R : S->queue) delete R;
    for (Batch &B : S->batch) batch_free(B);
    for (Batch &B : S->join) batch_free(B);
    for (auto &f : S->pool) (void)hipFree(f.second);
    S->pool.clear();
    for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
    const fs_status f = S->fatal;
    delete S;
    return f == FS_OK ? FS_OK : set_error(f, "server had stopped on an error");
}

}  // extern "C"
