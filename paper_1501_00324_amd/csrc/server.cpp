// Solve server with continuous batching.
//
// Requests (a matrix handle and k right-hand sides) are queued by
// server_submit and admitted in arrival order while the device-memory
// budget and the slot count allow.  One worker thread owns the device work:
// every admitted request becomes a member of one batch that the CG engine
// advances with shared launches (one batched product and a fixed number of
// vector / reduction kernels per iteration for all members).  Membership
// changes only at chunk boundaries (every check_every iterations): finished
// requests leave, their memory is released, and queued requests join.  A
// member's arithmetic does not depend on the other members, so every result
// is bitwise the result of solving that request alone.
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
};

int64_t krylov_bytes(const fs_csr *A, int32_t k, int32_t precond)
{
    const int64_t n = A->n_rows;
    const int64_t snb = engine_spmv_blocks(A->n_groups);
    const int64_t vnb = engine_vec_blocks(A->n_rows);
    return 5 * n * k * 8 + (precond ? n * 8 : 0) +
           int64_t(sizeof(ColState)) * k + 4 +
           8 * 3 * int64_t(k) * std::max(snb, vnb);
}

}  // namespace
}  // namespace fs

struct fs_server {
    fs_server_opts o{};
    int device = 0;
    hipStream_t s = nullptr;
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
    fs::Batch batch[2 * fs::kKmClasses], check;
    uint64_t submitted = 0, completed = 0;
};

namespace fs {
namespace {

fs_status finish(fs_server *S, Request *R, const ColState *cols)
{
    // a column with b = 0 returns x = 0
    for (int32_t c = 0; c < R->k; ++c)
        if (cols[c].bnorm2 == 0.0)
            FS_HIP_TRY(hipMemset2DAsync(static_cast<double *>(R->sys.x) + c,
                                        sizeof(double) * size_t(R->k), 0,
                                        sizeof(double), size_t(R->sys.n),
                                        S->s));
    FS_HIP_TRY(permute_rows(R->A->n_rows, R->k,
                            R->A->host.identity ? nullptr : R->A->d_perm,
                            static_cast<const double *>(R->sys.x), R->k, R->X,
                            R->k, false, S->s));
    FS_HIP_TRY(hipStreamSynchronize(S->s));
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
    std::vector<Request *> joining;
    admit(S, joining);
    if (!joining.empty()) {
        Batch &J = S->check;
        J.members.clear();
        J.vt = VT_F64;
        J.st = ST_F64;
        for (Request *R : joining) {
            FS_TRY(sys_alloc(R->sys, R->A, R->k, VT_F64, ST_F64, S->o.precond));
            R->sys.rtol = S->o.rtol;
            R->sys.maxit = S->o.maxit;
            FS_HIP_TRY(permute_rows(R->A->n_rows, R->k,
                                    R->A->host.identity ? nullptr
                                                        : R->A->d_perm,
                                    R->B, R->k,
                                    static_cast<double *>(R->sys.b), R->k,
                                    true, S->s));
            FS_HIP_TRY(hipMemsetAsync(R->sys.x, 0,
                                      sizeof(double) * size_t(R->sys.n) * R->k,
                                      S->s));
        }
        // start the joiners (diagonal, initial residual) per launch class
        for (int32_t cls = 0; cls < 2 * kKmClasses; ++cls) {
            const int32_t vec = 1 + cls / kKmClasses, kc = cls % kKmClasses;
            J.members.clear();
            J.vec = vec;
            for (Request *R : joining)
                if (R->A->host.vec == vec && km_index(R->k) == kc)
                    J.members.push_back(&R->sys);
            if (J.members.empty()) continue;
            FS_TRY(batch_build(J, S->s));
            if (S->o.precond) FS_HIP_TRY(engine_diag_inv(J.L, S->s));
            FS_HIP_TRY(engine_residual(J.L, 0, true, S->s));
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Request *R : joining) S->active.push_back(R);
            S->peak_active = std::max(S->peak_active,
                                      int32_t(S->active.size()));
        }
    }
    if (S->active.empty()) return FS_OK;
    // one batch per slot width and column-count class; members iterate,
    // then leave when done
    for (int32_t cls = 0; cls < 2 * kKmClasses; ++cls) {
        const int32_t vec = 1 + cls / kKmClasses, kc = cls % kKmClasses;
        Batch &B = S->batch[cls];
        std::vector<Request *> mem;
        std::vector<CgSys *> syss;
        for (Request *R : S->active)
            if (R->A->host.vec == vec && km_index(R->k) == kc) {
                mem.push_back(R);
                syss.push_back(&R->sys);
            }
        if (mem.empty()) continue;
        if (syss != B.members || !joining.empty()) {
            // membership changed: new descriptors (and a new graph)
            B.members = syss;
            B.vt = VT_F64;
            B.st = ST_F64;
            B.vec = vec;
            FS_TRY(batch_build(B, S->s));
        }
        FS_TRY(batch_read_states(B, S->s));
        auto running = [&]() {
            for (int32_t i = 0; i < B.L.ncols; ++i)
                if (B.h_stage[i].status == CG_RUNNING) return true;
            return false;
        };
        if (running()) {
            FS_TRY(batch_iterations(B, S->o.check_every, S->o.use_graph != 0,
                                    S->s));
            FS_TRY(batch_read_states(B, S->s));
        }
        bool met = false;
        for (int32_t i = 0; i < B.L.ncols; ++i)
            met |= B.h_stage[i].status == CG_RECURRENCE_MET;
        if (met) {
            FS_HIP_TRY(engine_residual(B.L, 1, false, S->s));
            FS_TRY(batch_read_states(B, S->s));
            bool pend = false;
            for (int32_t i = 0; i < B.L.ncols; ++i)
                pend |= B.h_stage[i].pending != 0;
            if (pend) FS_HIP_TRY(engine_pupdate_pending(B.L, S->s));
        }
        // members whose columns have all stopped
        bool any_fail = false;
        std::vector<bool> fin(mem.size(), false);
        int32_t j = 0;
        for (size_t m = 0; m < mem.size(); ++m) {
            bool all = true;
            for (int32_t c = 0; c < mem[m]->k; ++c, ++j) {
                const int32_t st = B.h_stage[j].status;
                all &= st != CG_RUNNING;
                any_fail |= st == CG_MAXIT || st == CG_BREAKDOWN;
            }
            fin[m] = all;
        }
        if (any_fail) {                  // final true residual for reports
            FS_HIP_TRY(engine_residual(B.L, 2, false, S->s));
            FS_TRY(batch_read_states(B, S->s));
        }
        std::vector<ColState> cols(B.h_stage, B.h_stage + B.L.ncols);
        j = 0;
        for (size_t m = 0; m < mem.size(); ++m) {
            Request *R = mem[m];
            const int32_t j0 = j;
            j += R->k;
            if (!fin[m]) continue;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->active.erase(std::find(S->active.begin(),
                                          S->active.end(), R));
            }
            FS_TRY(finish(S, R, cols.data() + j0));
        }
    }
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
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete S;
        return set_error(FS_E_HIP, "server stream: %s", hipGetErrorString(e));
    }
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
    // requests left behind after a fatal error
    for (Request *R : S->active) {
        sys_free(R->sys);
        delete R;
    }
    for (Request *R : S->queue) delete R;
    (void)hipStreamSynchronize(S->s);
    for (Batch &B : S->batch) batch_free(B);
    batch_free(S->check);
    (void)hipStreamDestroy(S->s);
    const fs_status f = S->fatal;
    delete S;
    return f == FS_OK ? FS_OK : set_error(f, "server had stopped on an error");
}

}  // extern "C"
