// Host side of the CG engine: device state per system, batches of systems
// launched together, the solve loop (chunks of iterations replayed as HIP
// graphs, one small device-to-host read of the column states per chunk,
// true-residual confirmation with residual replacement), mixed-precision
// iterative refinement, and the cg_solve* entry points.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "host.h"

namespace fs {
namespace {

size_t st_size(int32_t st) { return st == ST_F64 ? 8 : 4; }

fs_status dmalloc(void **p, size_t bytes, int64_t &acct)
{
    *p = nullptr;
    if (!bytes) return FS_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? FS_E_OOM : FS_E_HIP,
                         "hipMalloc(%zu bytes): %s", bytes,
                         hipGetErrorString(e));
    }
    acct += int64_t(bytes);
    return FS_OK;
}

const void *values_of(const fs_csr *A, int32_t vt)
{
    return vt == VT_F64 ? static_cast<const void *>(A->d_val)
         : vt == VT_F32 ? static_cast<const void *>(A->d_val_f32)
                        : static_cast<const void *>(A->d_val_bf16);
}

}  // namespace

// ------------------------------------------------------------- systems
void sys_free(CgSys &S)
{
    if (S.carved) {
        // parts of a block the caller owns: only forget them
        S.x = S.r = S.p = S.q = S.b = S.dinv = nullptr;
        S.cs = nullptr;
        S.bad = nullptr;
        S.partials = nullptr;
        S.carved = false;
    } else {
        dfree(S.x); dfree(S.r); dfree(S.p); dfree(S.q); dfree(S.b);
        dfree(S.dinv); dfree(S.cs); dfree(S.bad); dfree(S.partials);
    }
    dfree(S.hist);
    S.hist_cap = 0;
    S.bytes = 0;
    S.k = 0;
}

namespace {
// sizes of the parts of a system's state, in sys_alloc order
void sys_parts(const fs_csr *A, int32_t k, int32_t st, int32_t precond,
               size_t (&sz)[9])
{
    const size_t n = size_t(A->n_rows);
    const size_t nk = n * size_t(k) * st_size(st);
    const size_t nbk = size_t(std::max(engine_spmv_blocks(A->n_groups),
                                       engine_vec_blocks(A->n_rows, k)));
    sz[0] = sz[1] = sz[2] = sz[3] = sz[4] = nk;
    sz[5] = precond ? n * st_size(st) : 0;
    sz[6] = sizeof(ColState) * size_t(k);
    sz[7] = sizeof(int32_t);
    sz[8] = sizeof(double) * 3 * size_t(k) * nbk;
}
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
}  // namespace

int64_t sys_block_bytes(const fs_csr *A, int32_t k, int32_t st,
                        int32_t precond)
{
    size_t sz[9];
    sys_parts(A, k, st, precond, sz);
    size_t t = 0;
    for (size_t v : sz) t += align256(v);
    return int64_t(t);
}

void sys_alloc_in(CgSys &S, fs_csr *A, int32_t k, int32_t vt, int32_t st,
                  int32_t precond, void *block)
{
    sys_free(S);
    S.A = A;
    S.k = k;
    S.vt = vt;
    S.st = st;
    S.precond = precond;
    S.n = A->n_rows;
    S.snb = engine_spmv_blocks(A->n_groups);
    S.vnb = engine_vec_blocks(S.n, k);
    size_t sz[9];
    sys_parts(A, k, st, precond, sz);
    char *p = static_cast<char *>(block);
    void *parts[9];
    for (int i = 0; i < 9; ++i) {
        parts[i] = sz[i] ? p : nullptr;
        p += align256(sz[i]);
    }
    S.x = parts[0]; S.r = parts[1]; S.p = parts[2]; S.q = parts[3];
    S.b = parts[4]; S.dinv = parts[5];
    S.cs = static_cast<ColState *>(parts[6]);
    S.bad = static_cast<int32_t *>(parts[7]);
    S.partials = static_cast<double *>(parts[8]);
    S.bytes = int64_t(p - static_cast<char *>(block));
    S.carved = true;
}

fs_status sys_alloc(CgSys &S, fs_csr *A, int32_t k, int32_t vt, int32_t st,
                    int32_t precond)
{
    sys_free(S);
    S.A = A;
    S.k = k;
    S.vt = vt;
    S.st = st;
    S.precond = precond;
    S.n = A->n_rows;
    S.snb = engine_spmv_blocks(A->n_groups);
    S.vnb = engine_vec_blocks(S.n, k);
    const size_t nk = size_t(S.n) * size_t(k) * st_size(st);
    fs_status r = FS_OK;
    if ((r = dmalloc(&S.x, nk, S.bytes)) || (r = dmalloc(&S.r, nk, S.bytes)) ||
        (r = dmalloc(&S.p, nk, S.bytes)) || (r = dmalloc(&S.q, nk, S.bytes)) ||
        (r = dmalloc(&S.b, nk, S.bytes)) ||
        (precond &&
         (r = dmalloc(&S.dinv, size_t(S.n) * st_size(st), S.bytes))) ||
        (r = dmalloc(reinterpret_cast<void **>(&S.cs),
                     sizeof(ColState) * size_t(k), S.bytes)) ||
        (r = dmalloc(reinterpret_cast<void **>(&S.bad), sizeof(int32_t),
                     S.bytes)) ||
        (r = dmalloc(reinterpret_cast<void **>(&S.partials),
                     sizeof(double) * 3 * size_t(k) *
                         size_t(std::max(S.snb, S.vnb)),
                     S.bytes))) {
        sys_free(S);
        return r;
    }
    return FS_OK;
}

// --------------------------------------------------------------- batches
void batch_free(Batch &B)
{
    if (B.graph) (void)hipGraphExecDestroy(B.graph);
    B.graph = nullptr;
    dfree(B.d_sys); dfree(B.d_smap); dfree(B.d_vmap); dfree(B.d_cmap);
    dfree(B.d_stage);
    if (B.h_stage) (void)hipHostFree(B.h_stage);
    B.h_stage = nullptr;
    if (B.up_ev) (void)hipEventSynchronize(B.up_ev);
    if (B.h_up) (void)hipHostFree(B.h_up);
    B.h_up = nullptr;
    B.up_cap = 0;
    if (B.up_ev) (void)hipEventDestroy(B.up_ev);
    B.up_ev = nullptr;
    B.cap_sys = B.cap_s = B.cap_v = B.cap_c = 0;
}

namespace {
template <class T>
fs_status ensure_cap(T *&p, int32_t &cap, int32_t want)
{
    if (want <= cap) return FS_OK;
    dfree(p);
    int64_t dummy = 0;
    int32_t c = std::max(want, 2 * cap);
    FS_TRY(dmalloc(reinterpret_cast<void **>(&p), sizeof(T) * size_t(c),
                   dummy));
    cap = c;
    return FS_OK;
}
}  // namespace

fs_status batch_build(Batch &B, hipStream_t s) { return batch_build(B, s, false); }

fs_status batch_build(Batch &B, hipStream_t s, bool async_upload)
{
    const int32_t m = int32_t(B.members.size());
    std::vector<SysDesc> descs(static_cast<size_t>(m));
    std::vector<int32_t> smap, vmap;
    B.cols.clear();
    int32_t kmax = 1, sb = 0, vb = 0;
    for (int32_t i = 0; i < m; ++i) {
        CgSys &S = *B.members[size_t(i)];
        const fs_csr *A = S.A;
        SysDesc &d = descs[size_t(i)];
        std::memset(&d, 0, sizeof d);
        d.groups = A->d_groups;
        d.val = S.val ? S.val : values_of(A, S.vt);
        d.col = A->d_col;
        d.cstream = A->d_col16 ? static_cast<const void *>(A->d_col16)
                               : static_cast<const void *>(A->d_col);
        d.gbase = A->d_col16 ? A->d_gbase : nullptr;
        d.n = S.n;
        d.ngroups = A->n_groups;
        d.k = S.k;
        d.maxit = S.maxit;
        d.sb0 = sb;
        d.snb = S.snb;
        d.vb0 = vb;
        d.vnb = S.vnb;
        d.x = S.x; d.r = S.r; d.p = S.p; d.q = S.q;
        d.b = S.b;
        d.dinv = S.precond ? S.dinv : nullptr;
        d.cs = S.cs;
        d.bad_diag = S.bad;
        d.partials = S.partials;
        d.rtol = S.rtol;
        d.hist = S.record && S.k == 1 ? S.hist : nullptr;
        d.hist_cap = S.hist_cap;
        smap.insert(smap.end(), size_t(S.snb), i);
        vmap.insert(vmap.end(), size_t(S.vnb), i);
        for (int32_t c = 0; c < S.k; ++c) B.cols.push_back(int2{i, c});
        sb += S.snb;
        vb += S.vnb;
        kmax = std::max(kmax, S.k);
    }
    const int32_t nc = int32_t(B.cols.size());
    FS_TRY(ensure_cap(B.d_sys, B.cap_sys, m));
    FS_TRY(ensure_cap(B.d_smap, B.cap_s, sb));
    FS_TRY(ensure_cap(B.d_vmap, B.cap_v, vb));
    if (nc > B.cap_c) {
        const int32_t cap = std::max(nc, 2 * B.cap_c);
        int64_t dummy = 0;
        dfree(B.d_cmap);
        dfree(B.d_stage);
        if (B.h_stage) (void)hipHostFree(B.h_stage);
        B.h_stage = nullptr;
        B.cap_c = 0;
        FS_TRY(dmalloc(reinterpret_cast<void **>(&B.d_cmap),
                       sizeof(int2) * size_t(cap), dummy));
        FS_TRY(dmalloc(reinterpret_cast<void **>(&B.d_stage),
                       sizeof(ColState) * size_t(cap), dummy));
        FS_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&B.h_stage),
                                 sizeof(ColState) * size_t(cap),
                                 hipHostMallocDefault));
        B.cap_c = cap;
    }
    if (async_upload) {
        // stream-ordered copies from a pinned staging area of the batch:
        // the staging area is rewritten only once the previous upload has
        // completed (its event)
        const size_t bytes = sizeof(SysDesc) * size_t(m) +
                             sizeof(int32_t) * size_t(sb + vb) +
                             sizeof(int2) * size_t(nc);
        if (B.up_ev) FS_HIP_TRY(hipEventSynchronize(B.up_ev));
        else FS_HIP_TRY(hipEventCreateWithFlags(&B.up_ev,
                                                hipEventDisableTiming));
        if (bytes > B.up_cap) {
            const size_t cap = std::max(bytes, 2 * B.up_cap);
            if (B.h_up) (void)hipHostFree(B.h_up);
            B.h_up = nullptr;
            B.up_cap = 0;
            FS_HIP_TRY(hipHostMalloc(&B.h_up, cap, hipHostMallocDefault));
            B.up_cap = cap;
        }
        char *h = static_cast<char *>(B.h_up);
        auto put = [&](void *dst, const void *src, size_t n) -> hipError_t {
            if (!n) return hipSuccess;
            std::memcpy(h, src, n);
            hipError_t e = hipMemcpyAsync(dst, h, n, hipMemcpyHostToDevice, s);
            h += n;
            return e;
        };
        FS_HIP_TRY(put(B.d_sys, descs.data(), sizeof(SysDesc) * m));
        FS_HIP_TRY(put(B.d_smap, smap.data(), sizeof(int32_t) * sb));
        FS_HIP_TRY(put(B.d_vmap, vmap.data(), sizeof(int32_t) * vb));
        FS_HIP_TRY(put(B.d_cmap, B.cols.data(), sizeof(int2) * nc));
        FS_HIP_TRY(hipEventRecord(B.up_ev, s));
    } else {
        // blocking copies: the host vectors are temporaries
        FS_HIP_TRY(hipStreamSynchronize(s));
        if (m) FS_HIP_TRY(hipMemcpy(B.d_sys, descs.data(),
                                    sizeof(SysDesc) * m,
                                    hipMemcpyHostToDevice));
        if (sb) FS_HIP_TRY(hipMemcpy(B.d_smap, smap.data(),
                                     sizeof(int32_t) * sb,
                                     hipMemcpyHostToDevice));
        if (vb) FS_HIP_TRY(hipMemcpy(B.d_vmap, vmap.data(),
                                     sizeof(int32_t) * vb,
                                     hipMemcpyHostToDevice));
        if (nc) FS_HIP_TRY(hipMemcpy(B.d_cmap, B.cols.data(),
                                     sizeof(int2) * nc,
                                     hipMemcpyHostToDevice));
    }
    B.km = km_for(kmax);
    B.L.vt = B.vt;
    B.L.st = B.st;
    B.L.vec = B.vec;
    B.L.km = B.km;
    B.L.sys = B.d_sys;
    B.L.smap = B.d_smap;
    B.L.vmap = B.d_vmap;
    B.L.cmap = B.d_cmap;
    B.L.sblocks = sb;
    B.L.vblocks = vb;
    B.L.ncols = nc;
    if (B.graph) (void)hipGraphExecDestroy(B.graph);
    B.graph = nullptr;
    B.graph_iters = 0;
    return FS_OK;
}

fs_status batch_iterations(Batch &B, int32_t iters, bool use_graph,
                           hipStream_t s)
{
    if (B.L.ncols == 0) return FS_OK;
    if (!use_graph || !s) {
        for (int32_t i = 0; i < iters; ++i)
            FS_HIP_TRY(engine_iteration(B.L, s));
        return FS_OK;
    }
    if (!B.graph || B.graph_iters != iters) {
        if (B.graph) (void)hipGraphExecDestroy(B.graph);
        B.graph = nullptr;
        hipGraph_t g = nullptr;
        FS_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int32_t i = 0; i < iters && e == hipSuccess; ++i)
            e = engine_iteration(B.L, s);
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return set_error(FS_E_HIP, "graph capture: %s",
                             hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            B.graph = nullptr;
            return set_error(FS_E_HIP, "graph instantiate: %s",
                             hipGetErrorString(e));
        }
        B.graph_iters = iters;
    }
    FS_HIP_TRY(hipGraphLaunch(B.graph, s));
    return FS_OK;
}

fs_status batch_stage_states(Batch &B, hipStream_t s)
{
    if (B.L.ncols == 0) return FS_OK;
    FS_HIP_TRY(engine_gather_states(B.L, B.d_stage, s));
    FS_HIP_TRY(hipMemcpyAsync(B.h_stage, B.d_stage,
                              sizeof(ColState) * size_t(B.L.ncols),
                              hipMemcpyDeviceToHost, s));
    return FS_OK;
}

fs_status batch_read_states(Batch &B, hipStream_t s)
{
    if (B.L.ncols == 0) return FS_OK;
    FS_TRY(batch_stage_states(B, s));
    FS_HIP_TRY(hipStreamSynchronize(s));
    return FS_OK;
}

namespace {

bool any_status(const Batch &B, int32_t st)
{
    for (int32_t i = 0; i < B.L.ncols; ++i)
        if (B.h_stage[i].status == st) return true;
    return false;
}

// Run every member of B from its current x to convergence (or failure).
// Members' b and x are set, rtol / maxit / precond are in the members.
fs_status run_batch(Batch &B, int32_t check_every, bool use_graph,
                    bool x_zero, hipStream_t s)
{
    FS_TRY(batch_build(B, s));
    bool pc = false;
    for (CgSys *S : B.members) pc |= S->precond != 0;
    if (pc) {
        for (CgSys *S : B.members)
            FS_HIP_TRY(hipMemsetAsync(S->bad, 0, sizeof(int32_t), s));
        FS_HIP_TRY(engine_diag_inv(B.L, s));
        for (CgSys *S : B.members) {
            if (!S->precond) continue;
            int32_t bad = 0;
            FS_HIP_TRY(hipMemcpyAsync(&bad, S->bad, sizeof bad,
                                      hipMemcpyDeviceToHost, s));
            FS_HIP_TRY(hipStreamSynchronize(s));
            if (bad)
                return set_error(FS_E_ARG,
                                 "Jacobi preconditioner: %d rows with a zero "
                                 "or non-finite diagonal", bad);
        }
    }
    FS_HIP_TRY(engine_residual(B.L, 0, x_zero, s));
    FS_TRY(batch_read_states(B, s));
    while (any_status(B, CG_RUNNING)) {
        FS_TRY(batch_iterations(B, check_every, use_graph, s));
        FS_TRY(batch_read_states(B, s));
        if (any_status(B, CG_RECURRENCE_MET)) {
            FS_HIP_TRY(engine_residual(B.L, 1, false, s));
            FS_TRY(batch_read_states(B, s));
            bool pending = false;
            for (int32_t i = 0; i < B.L.ncols; ++i)
                pending |= B.h_stage[i].pending != 0;
            if (pending) FS_HIP_TRY(engine_pupdate_pending(B.L, s));
        }
    }
    bool all_conv = true;
    for (int32_t i = 0; i < B.L.ncols; ++i)
        all_conv &= B.h_stage[i].status == CG_CONVERGED;
    if (!all_conv) {
        FS_HIP_TRY(engine_residual(B.L, 2, false, s));
        FS_TRY(batch_read_states(B, s));
    }
    return FS_OK;
}

fs_status status_of(const ColState &c)
{
    switch (c.status) {
    case CG_CONVERGED: return FS_OK;
    case CG_MAXIT: return FS_E_NOT_CONVERGED;
    default: return FS_E_BREAKDOWN;
    }
}

void fill_info(const ColState &c, fs_cg_info &info)
{
    info.status = status_of(c);
    info.iters = c.iter;
    info.replacements = c.replacements;
    info.relres = c.bnorm2 > 0.0 ? std::sqrt(c.rr_true / c.bnorm2) : 0.0;
}

// worst status over columns, for the return code
fs_status worst(fs_status a, fs_status b)
{
    auto rank = [](fs_status v) {
        return v == FS_OK ? 0 : v == FS_E_NOT_CONVERGED ? 1 : 2;
    };
    return rank(b) > rank(a) ? b : a;
}

fs_status normalise_opts(const fs_cg_opts *in, fs_cg_opts &o)
{
    cg_opts_default(&o);
    if (in) o = *in;
    if (o.rtol <= 0.0) o.rtol = 1e-8;
    if (o.maxit <= 0) o.maxit = 20000;
    if (o.check_every <= 0) o.check_every = 32;
    if (o.inner_rtol <= 0.0) o.inner_rtol = 1e-2;
    if (o.max_outer <= 0) o.max_outer = 50;
    if (o.precond != FS_PC_NONE && o.precond != FS_PC_JACOBI)
        return set_error(FS_E_ARG, "unknown preconditioner %d", o.precond);
    if (o.precision < FS_PREC_F64 || o.precision > FS_PREC_IR_BF16)
        return set_error(FS_E_ARG, "unknown precision %d", o.precision);
    return FS_OK;
}

fs_status ensure_stream(fs_csr *A)
{
    if (!A->stream)
        FS_HIP_TRY(hipStreamCreateWithFlags(&A->stream, hipStreamNonBlocking));
    if (!A->ev)
        FS_HIP_TRY(hipEventCreateWithFlags(&A->ev, hipEventDisableTiming));
    return FS_OK;
}

fs_status ensure_sys(CgSys *&S, fs_csr *A, int32_t k, int32_t vt, int32_t st,
                     int32_t pc)
{
    if (!S) S = new CgSys();
    if (S->k != k || S->vt != vt || S->st != st || (pc && !S->dinv) ||
        S->n != A->n_rows)
        FS_TRY(sys_alloc(*S, A, k, vt, st, pc));
    S->precond = pc;
    return FS_OK;
}

// caller block (n x k, row stride ld) -> layout block of S (ld = k)
fs_status load_block(const fs_csr *A, int32_t k, const double *src,
                     int64_t ld, void *dst, hipStream_t s)
{
    return permute_rows(A->n_rows, k, A->host.identity ? nullptr : A->d_perm,
                        src, ld, static_cast<double *>(dst), k, true, s) ==
                   hipSuccess
               ? FS_OK
               : set_error(FS_E_HIP, "permute_rows: %s",
                           hipGetErrorString(hipGetLastError()));
}

fs_status store_block(const fs_csr *A, int32_t k, const void *src,
                      double *dst, int64_t ld, hipStream_t s)
{
    return permute_rows(A->n_rows, k, A->host.identity ? nullptr : A->d_perm,
                        static_cast<const double *>(src), k, dst, ld, false,
                        s) == hipSuccess
               ? FS_OK
               : set_error(FS_E_HIP, "permute_rows: %s",
                           hipGetErrorString(hipGetLastError()));
}

// Number of eigenvalues below x of the symmetric tridiagonal (diag a,
// off-diagonal e; m entries), by the signs of the LDL^T pivots (Sturm).
int32_t sturm_count(const std::vector<double> &a, const std::vector<double> &e,
                    double x)
{
    const int32_t m = int32_t(a.size());
    int32_t cnt = 0;
    double d = 1.0;
    for (int32_t i = 0; i < m; ++i) {
        const double off = i ? e[size_t(i - 1)] * e[size_t(i - 1)] / d : 0.0;
        d = a[size_t(i)] - x - off;
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

// Condition estimate from m CG steps (ab = alpha_0, beta_0, alpha_1, ...):
// the extreme eigenvalues of the Lanczos tridiagonal T of the PCG
// coefficients, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
// T_j,j+1 = sqrt(beta_j)/alpha_j, found by bisection on the Sturm count
// inside the Gershgorin interval.  0 when nothing was recorded.
double lanczos_cond(const std::vector<double> &ab, int32_t m)
{
    if (m < 1) return 0.0;
    std::vector<double> a(static_cast<size_t>(m)), e(static_cast<size_t>(m));
    for (int32_t j = 0; j < m; ++j) {
        const double al = ab[size_t(2 * j)], be = ab[size_t(2 * j + 1)];
        a[size_t(j)] = 1.0 / al;
        if (j) {
            const double alp = ab[size_t(2 * j - 2)], bep = ab[size_t(2 * j - 1)];
            a[size_t(j)] += bep / alp;
        }
        e[size_t(j)] = be > 0.0 ? std::sqrt(be) / al : 0.0;
    }
    double lo = a[0], hi = a[0];
    for (int32_t j = 0; j < m; ++j) {
        const double r = (j ? std::fabs(e[size_t(j - 1)]) : 0.0) +
                         (j + 1 < m ? std::fabs(e[size_t(j)]) : 0.0);
        lo = std::min(lo, a[size_t(j)] - r);
        hi = std::max(hi, a[size_t(j)] + r);
    }
    if (!std::isfinite(lo) || !std::isfinite(hi)) return 0.0;
    auto kth = [&](int32_t k) {          // the k-th smallest (1-based)
        double l = lo, h = hi;
        for (int it = 0; it < 200 && h - l > 1e-15 * std::max(std::fabs(l),
                                                                std::fabs(h));
             ++it) {
            const double mid = 0.5 * (l + h);
            if (sturm_count(a, e, mid) >= k) h = mid;
            else l = mid;
        }
        return 0.5 * (l + h);
    };
    const double lmin = kth(1), lmax = kth(m);
    return lmin > 0.0 ? lmax / lmin : 0.0;
}

// FP64 CG on one handle with k right-hand sides (caller blocks B, X).
fs_status solve_f64(fs_csr *A, int32_t k, const double *Bc, int64_t ldb,
                    double *Xc, int64_t ldx, const fs_cg_opts &o,
                    fs_cg_info *infos, hipStream_t caller)
{
    FS_TRY(ensure_stream(A));
    hipStream_t s = A->stream;
    FS_HIP_TRY(hipEventRecord(A->ev, caller));
    FS_HIP_TRY(hipStreamWaitEvent(s, A->ev, 0));
    FS_TRY(ensure_sys(A->sys_f64, A, k, VT_F64, ST_F64, o.precond));
    CgSys &S = *A->sys_f64;
    S.rtol = o.rtol;
    S.maxit = o.maxit;
    S.val = nullptr;
    S.record = o.estimate_cond != 0 && k == 1;
    if (S.record && S.hist_cap < o.maxit) {
        dfree(S.hist);
        S.hist_cap = 0;
        int64_t acct = 0;
        FS_TRY(dmalloc(reinterpret_cast<void **>(&S.hist),
                       sizeof(double) * 2 * size_t(o.maxit), acct));
        S.hist_cap = o.maxit;
    }
    FS_TRY(load_block(A, k, Bc, ldb, S.b, s));
    if (o.x0_zero)
        FS_HIP_TRY(hipMemsetAsync(S.x, 0, sizeof(double) * size_t(S.n) * k, s));
    else
        FS_TRY(load_block(A, k, Xc, ldx, S.x, s));
    if (!A->batch_f64) A->batch_f64 = new Batch();
    Batch &B = *A->batch_f64;
    B.members.assign(1, &S);
    B.vt = VT_F64;
    B.st = ST_F64;
    B.vec = A->host.vec;
    FS_TRY(run_batch(B, o.check_every, o.use_graph != 0, o.x0_zero != 0, s));
    // a column with b = 0 returns x = 0
    for (int32_t c = 0; c < k; ++c)
        if (B.h_stage[c].bnorm2 == 0.0)
            FS_HIP_TRY(hipMemset2DAsync(static_cast<double *>(S.x) + c,
                                        sizeof(double) * size_t(k), 0,
                                        sizeof(double), size_t(S.n), s));
    FS_TRY(store_block(A, k, S.x, Xc, ldx, s));
    double cond = 0.0;
    if (S.record) {
        const int32_t m = std::min(B.h_stage[0].iter, S.hist_cap);
        std::vector<double> ab(2 * static_cast<size_t>(std::max(m, 1)));
        if (m > 0)
            FS_HIP_TRY(hipMemcpyAsync(ab.data(), S.hist,
                                      sizeof(double) * 2 * size_t(m),
                                      hipMemcpyDeviceToHost, s));
        FS_HIP_TRY(hipStreamSynchronize(s));
        cond = lanczos_cond(ab, m);
        S.record = false;
    }
    FS_HIP_TRY(hipStreamSynchronize(s));
    fs_status ret = FS_OK;
    const double it_bytes = 12.0 * double(A->nnz) +
                            (o.precond ? 104.0 : 88.0) * double(A->n_rows) * k;
    for (int32_t c = 0; c < k; ++c) {
        fill_info(B.h_stage[c], infos[c]);
        infos[c].outer = 0;
        infos[c].bytes = double(B.h_stage[c].iter) * it_bytes / k +
                         2.0 * (12.0 * double(A->nnz) + 16.0 * A->n_rows);
        infos[c].cond_est = cond;
        ret = worst(ret, infos[c].status);
    }
    return ret;
}

// Start a batch's CG from x = 0 without iterating: Jacobi scaling (checked)
// and the start residual r = b, p = z.
fs_status start_inner(Batch &B, bool precond, hipStream_t s)
{
    FS_TRY(batch_build(B, s));
    if (precond) {
        for (CgSys *S : B.members)
            FS_HIP_TRY(hipMemsetAsync(S->bad, 0, sizeof(int32_t), s));
        FS_HIP_TRY(engine_diag_inv(B.L, s));
        for (CgSys *S : B.members) {
            int32_t bad = 0;
            FS_HIP_TRY(hipMemcpyAsync(&bad, S->bad, sizeof bad,
                                      hipMemcpyDeviceToHost, s));
            FS_HIP_TRY(hipStreamSynchronize(s));
            if (bad)
                return set_error(FS_E_ARG,
                                 "Jacobi preconditioner: %d rows with a zero "
                                 "or non-finite diagonal", bad);
        }
    }
    FS_HIP_TRY(engine_residual(B.L, 0, true, s));
    return batch_read_states(B, s);
}

// Mixed-precision iterative refinement: FP64 residual and update, inner CG
// on the FP32 / BF16 copy of A with float vectors.
fs_status solve_ir(fs_csr *A, int32_t k, const double *Bc, int64_t ldb,
                   double *Xc, int64_t ldx, const fs_cg_opts &o,
                   fs_cg_info *infos, hipStream_t caller)
{
    const int32_t dt = o.precision == FS_PREC_IR_F32 ? FS_DT_F32 : FS_DT_BF16;
    const int32_t vt = dt == FS_DT_F32 ? VT_F32 : VT_BF16;
    const bool scaled = o.ir_scaled != 0;
    if (!scaled && !(A->dtypes & dt)) FS_TRY(csr_add_dtype(A, dt, caller));
    FS_TRY(ensure_stream(A));
    hipStream_t s = A->stream;
    FS_HIP_TRY(hipEventRecord(A->ev, caller));
    FS_HIP_TRY(hipStreamWaitEvent(s, A->ev, 0));
    if (scaled && A->lo_scaled_dt != dt) {
        // the low-precision copy of D^-1/2 A D^-1/2 (after a value update
        // or for the other precision: rebuilt)
        A->lo_scaled_dt = 0;
        dfree(A->d_val_lo_scaled);
        int64_t acct = 0;
        if (!A->d_iscale)
            FS_TRY(dmalloc(reinterpret_cast<void **>(&A->d_iscale),
                           sizeof(double) * size_t(A->n_rows), acct));
        FS_TRY(dmalloc(&A->d_val_lo_scaled,
                       size_t(A->slots) * (dt == FS_DT_F32 ? 4 : 2), acct));
        int32_t *d_bad = nullptr;
        FS_TRY(dmalloc(reinterpret_cast<void **>(&d_bad), sizeof(int32_t),
                       acct));
        int32_t bad = 0;
        hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(int32_t), s);
        if (e == hipSuccess)
            e = scaled_lowp_copy(A, dt, A->d_iscale, A->d_val_lo_scaled,
                                 d_bad, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost,
                               s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dfree(d_bad);
        FS_HIP_TRY(e);
        if (bad)
            return set_error(FS_E_ARG,
                             "scaled refinement: %d rows without a positive "
                             "diagonal", bad);
        A->lo_scaled_dt = dt;
    }
    FS_TRY(ensure_sys(A->sys_f64, A, k, VT_F64, ST_F64, o.precond));
    FS_TRY(ensure_sys(A->sys_lo, A, k, vt, ST_F32, scaled ? 0 : o.precond));
    CgSys &Out = *A->sys_f64, &In = *A->sys_lo;
    Out.rtol = o.rtol;
    Out.maxit = o.maxit;
    Out.val = nullptr;
    Out.record = false;
    In.rtol = o.inner_rtol;
    In.val = scaled ? A->d_val_lo_scaled : nullptr;
    In.record = false;
    // Jacobi scaling of the vectors around the inner solve (NULL: none)
    const double *sc = scaled ? A->d_iscale : nullptr;
    const bool in_pc = !scaled && o.precond != 0;
    FS_TRY(load_block(A, k, Bc, ldb, Out.b, s));
    if (o.x0_zero)
        FS_HIP_TRY(hipMemsetAsync(Out.x, 0, sizeof(double) * size_t(Out.n) * k,
                                  s));
    else
        FS_TRY(load_block(A, k, Xc, ldx, Out.x, s));
    if (!A->batch_f64) A->batch_f64 = new Batch();
    if (!A->batch_lo) A->batch_lo = new Batch();
    Batch &BO = *A->batch_f64, &BI = *A->batch_lo;
    BO.members.assign(1, &Out);
    BO.vt = VT_F64;
    BO.st = ST_F64;
    BO.vec = A->host.vec;
    BI.members.assign(1, &In);
    BI.vt = vt;
    BI.st = ST_F32;
    BI.vec = A->host.vec;
    FS_TRY(batch_build(BO, s));
    const int64_t nk = int64_t(Out.n) * k;
    int32_t outer = 0, inner_total = 0;
    // inner_bad: the last inner solve broke down (the low-precision copy
    // need not be positive definite when A is ill-conditioned); its partial
    // correction is still applied, and the residual test below decides
    bool x_zero = o.x0_zero != 0, inner_bad = false, stalled = false;
    // fresh: the next step starts a new inner CG (always with ir_restart;
    // otherwise at the first step, and again after a step with a kept
    // search direction failed to lower the FP64 residual)
    bool fresh = true, last_fresh = false;
    int32_t inner_base = 0;    // inner iterations before the current inner CG
    // a kept-direction step may take at most twice the iterations of the
    // last fresh step (and 64); past that it is cut and the next step is
    // fresh (the low-precision copy may be indefinite, where CG stalls)
    int32_t fresh_iters = 0;
    std::vector<ColState> last(static_cast<size_t>(k));
    double prev_rr = 0.0;
    for (;;) {
        // FP64 residual r = b - A x and its norm against rtol |b|
        FS_HIP_TRY(engine_residual(BO.L, 0, x_zero, s));
        FS_TRY(batch_read_states(BO, s));
        x_zero = false;
        bool done = true;
        double rr = 0.0;
        for (int32_t c = 0; c < k; ++c) {
            done &= BO.h_stage[c].status == CG_CONVERGED;
            rr += BO.h_stage[c].rr_true;
        }
        if (outer > 0 && !done && !(rr < prev_rr)) {
            // the last correction did not reduce the FP64 residual: undo it
            // and re-measure.  After a fresh inner solve this means the
            // low-precision matrix is too far from A for refinement to
            // converge (rounding error times condition number >= 1): stop.
            // After a step that kept the search direction, retry once with
            // a fresh inner solve.
            FS_HIP_TRY(add_f32(nk, k, -1.0, static_cast<const float *>(In.x),
                               sc, static_cast<double *>(Out.x), s));
            FS_HIP_TRY(engine_residual(BO.L, 0, false, s));
            FS_TRY(batch_read_states(BO, s));
            for (int32_t c = 0; c < k; ++c) last[size_t(c)] = BO.h_stage[c];
            if (o.ir_restart || last_fresh) {
                stalled = true;
                break;
            }
            fresh = true;
            done = false;
        } else {
            for (int32_t c = 0; c < k; ++c) last[size_t(c)] = BO.h_stage[c];
            prev_rr = rr;
        }
        if (done || outer >= o.max_outer || inner_total >= o.maxit) break;
        // inner solve A_lo d = r in single precision, d from 0; columns done
        // in FP64 get a zero inner b (their inner CG stops at once)
        for (int32_t c = 0; c < k; ++c)
            if (BO.h_stage[c].status == CG_CONVERGED)
                FS_HIP_TRY(hipMemset2DAsync(
                    static_cast<double *>(Out.r) + c,
                    sizeof(double) * size_t(k), 0, sizeof(double),
                    size_t(Out.n), s));
        FS_HIP_TRY(to_f32(nk, k, static_cast<const double *>(Out.r), sc,
                          static_cast<float *>(In.b), s));
        FS_HIP_TRY(hipMemsetAsync(In.x, 0, sizeof(float) * size_t(nk), s));
        inner_bad = false;
        if (fresh || o.ir_restart) {
            inner_base = inner_total;
            In.maxit = std::max(1, o.maxit - inner_base);
            FS_TRY(start_inner(BI, in_pc, s));
            fresh = false;
            last_fresh = true;
        } else {
            // rebase the columns that met the inner tolerance on the new
            // residual, keeping their search directions
            FS_HIP_TRY(engine_residual(BI.L, 3, true, s));
            FS_TRY(batch_read_states(BI, s));
            bool pend = false;
            for (int32_t c = 0; c < k; ++c) pend |= BI.h_stage[c].pending != 0;
            if (pend) FS_HIP_TRY(engine_pupdate_pending(BI.L, s));
            last_fresh = false;
        }
        int32_t seg0 = 0;
        for (int32_t c = 0; c < k; ++c)
            seg0 = std::max(seg0, BI.h_stage[c].iter);
        while (any_status(BI, CG_RUNNING)) {
            if (!last_fresh) {
                int32_t itn = 0;
                for (int32_t c = 0; c < k; ++c)
                    itn = std::max(itn, BI.h_stage[c].iter);
                if (itn - seg0 >= std::max(64, 2 * fresh_iters)) {
                    fresh = true;      // cut: restart the inner CG next
                    break;
                }
            }
            FS_TRY(batch_iterations(BI, o.check_every, o.use_graph != 0, s));
            FS_TRY(batch_read_states(BI, s));
            if (o.ir_restart && any_status(BI, CG_RECURRENCE_MET)) {
                // classic refinement confirms the inner solve against its own
                // true residual (with replacement) like a plain solve
                FS_HIP_TRY(engine_residual(BI.L, 1, false, s));
                FS_TRY(batch_read_states(BI, s));
                bool pend = false;
                for (int32_t c = 0; c < k; ++c)
                    pend |= BI.h_stage[c].pending != 0;
                if (pend) FS_HIP_TRY(engine_pupdate_pending(BI.L, s));
            }
        }
        int32_t it = 0;
        for (int32_t c = 0; c < k; ++c) {
            it = std::max(it, BI.h_stage[c].iter);
            if (BI.h_stage[c].status == CG_BREAKDOWN) inner_bad = true;
        }
        inner_total = inner_base + it;
        if (last_fresh) fresh_iters = it;
        // columns stopped by the iteration limit cannot be rebased
        for (int32_t c = 0; c < k; ++c)
            if (BI.h_stage[c].status == CG_MAXIT ||
                BI.h_stage[c].status == CG_BREAKDOWN)
                fresh = true;
        ++outer;
        FS_HIP_TRY(add_f32(nk, k, 1.0, static_cast<const float *>(In.x), sc,
                           static_cast<double *>(Out.x), s));
    }
    FS_TRY(store_block(A, k, Out.x, Xc, ldx, s));
    FS_HIP_TRY(hipStreamSynchronize(s));
    fs_status ret = FS_OK;
    const double sv = dt == FS_DT_F32 ? 4.0 : 2.0;
    const double in_bytes = (sv + 4.0) * double(A->nnz) +
                            (in_pc ? 52.0 : 44.0) * A->n_rows * k;
    const double out_bytes = 12.0 * double(A->nnz) + 40.0 * A->n_rows * k;
    for (int32_t c = 0; c < k; ++c) {
        const ColState &cs = last[size_t(c)];
        fs_cg_info &info = infos[c];
        info.status = cs.status == CG_CONVERGED ? FS_OK
                      : stalled && inner_bad    ? FS_E_BREAKDOWN
                                                : FS_E_NOT_CONVERGED;
        info.iters = inner_total;
        info.outer = outer;
        info.replacements = 0;
        info.relres = cs.bnorm2 > 0.0 ? std::sqrt(cs.rr_true / cs.bnorm2) : 0.0;
        info.bytes = (inner_total * in_bytes + (outer + 1) * out_bytes) / k;
        ret = worst(ret, info.status);
    }
    if (stalled && ret != FS_OK)
        set_error(ret, "mixed-precision refinement stopped after %d steps: "
                       "the FP64 residual stopped decreasing (relative "
                       "residual %.3e)%s", outer, infos[0].relres,
                  inner_bad ? "; the inner solve on the low-precision copy "
                              "broke down (that copy is not positive "
                              "definite)" : "");
    else if (ret != FS_OK)
        set_error(ret, "mixed-precision refinement: relative residual %.3e "
                       "after %d steps", infos[0].relres, outer);
    return ret;
}

fs_status check_solve_args(const fs_csr *A, int32_t k, const void *b,
                           const void *x, int64_t ldb, int64_t ldx)
{
    if (!A) return set_error(FS_E_ARG, "NULL matrix handle");
    if (A->n_rows != A->n_cols)
        return set_error(FS_E_NOT_SQUARE, "CG needs a square matrix");
    if (k < 1 || k > 16)
        return set_error(FS_E_ARG, "k = %d, must be in [1, 16]", k);
    if (ldb < k || ldx < k)
        return set_error(FS_E_ARG, "leading dimension below k");
    if (A->n_rows > 0 && (!b || !x)) return set_error(FS_E_ARG, "NULL vector");
    return FS_OK;
}

fs_status solve_any(fs_csr *A, int32_t k, const double *B, int64_t ldb,
                    double *X, int64_t ldx, const fs_cg_opts *opts,
                    fs_cg_info *infos, hipStream_t s)
{
    fs_cg_opts o;
    FS_TRY(normalise_opts(opts, o));
    FS_TRY(check_solve_args(A, k, B, X, ldb, ldx));
    if (A->n_rows == 0) {
        for (int32_t c = 0; c < k; ++c) std::memset(&infos[c], 0, sizeof(fs_cg_info));
        return FS_OK;
    }
    DeviceGuard g(A->device);
    if (o.precision == FS_PREC_F64)
        return solve_f64(A, k, B, ldb, X, ldx, o, infos, s);
    return solve_ir(A, k, B, ldb, X, ldx, o, infos, s);
}

}  // namespace

void free_solver_state(fs_csr *A)
{
    for (CgSys **S : {&A->sys_f64, &A->sys_lo}) {
        if (*S) {
            sys_free(**S);
            delete *S;
            *S = nullptr;
        }
    }
    for (Batch **B : {&A->batch_f64, &A->batch_lo}) {
        if (*B) {
            batch_free(**B);
            delete *B;
            *B = nullptr;
        }
    }
    dfree(A->d_async);
    dfree(A->d_apart);
    dfree(A->d_ainfo);
    dfree(A->d_iscale);
    dfree(A->d_val_lo_scaled);
    A->lo_scaled_dt = 0;
    if (A->ev) (void)hipEventDestroy(A->ev);
    A->ev = nullptr;
    if (A->stream) (void)hipStreamDestroy(A->stream);
    A->stream = nullptr;
}

}  // namespace fs

using namespace fs;

extern "C" fs_status cg_solve(fs_csr_t A, const double *b, double *x,
                              const fs_cg_opts *opts, fs_cg_info *info,
                              hipStream_t s)
{
    const double t0 = now_ms();
    fs_cg_info local;
    std::memset(&local, 0, sizeof local);
    fs_status st = solve_any(A, 1, b, 1, x, 1, opts, &local, s);
    local.status = st;
    local.ms = now_ms() - t0;
    if (info) *info = local;
    return st;
}

namespace fs {

fs_status async_check(fs_csr *A, const double *b, double *x,
                      const fs_cg_opts *opts, fs_cg_info *info,
                      fs_cg_opts &o)
{
    FS_TRY(normalise_opts(opts, o));
    FS_TRY(check_solve_args(A, 1, b, x, 1, 1));
    if (!info) return set_error(FS_E_ARG, "info is required");
    if (o.precision != FS_PREC_F64)
        return set_error(FS_E_UNSUPPORTED,
                         "the stream-ordered solve runs in FP64");
    if (A->n_rows == 0) return FS_OK;
    int coop = 0;
    FS_HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch,
                                     A->device));
    if (!coop)
        return set_error(FS_E_UNSUPPORTED,
                         "device without cooperative launches");
    return FS_OK;
}

fs_status async_enqueue(fs_csr *A, const double *b, double *x,
                        const fs_cg_opts &o, double *ws, double *part,
                        fs_cg_info *dinfo, fs_cg_info *info, hipStream_t s)
{
    const int64_t n = A->n_rows;
    double *B = ws, *X = B + n, *R = X + n, *P = R + n, *Q = P + n,
           *Dv = Q + n, *Z = Dv + n;
    FS_TRY(load_block(A, 1, b, 1, B, s));
    if (o.x0_zero)
        FS_HIP_TRY(fill_f64(n, 0.0, X, s));
    else
        FS_TRY(load_block(A, 1, x, 1, X, s));
    FS_HIP_TRY(launch_cg_persistent(A, persistent_blocks(A), B, X, R, P, Q,
                                    Z, o.precond ? Dv : nullptr, part, dinfo,
                                    o.rtol, o.maxit, o.x0_zero != 0, s));
    FS_TRY(store_block(A, 1, X, x, 1, s));
    FS_HIP_TRY(hipMemcpyAsync(info, dinfo, sizeof(fs_cg_info),
                              hipMemcpyDeviceToHost, s));
    return FS_OK;
}

}  // namespace fs

extern "C" fs_status cg_solve_async(fs_csr_t A, const double *b, double *x,
                                    const fs_cg_opts *opts, fs_cg_info *info,
                                    hipStream_t s)
{
    fs_cg_opts o;
    FS_TRY(async_check(A, b, x, opts, info, o));
    if (A->n_rows == 0) {
        std::memset(info, 0, sizeof(fs_cg_info));
        return FS_OK;
    }
    DeviceGuard g(A->device);
    const int64_t n = A->n_rows;
    if (!A->d_async) {
        // first use: workspace of the handle (allocation synchronises)
        int64_t acct = 0;
        FS_TRY(dmalloc(reinterpret_cast<void **>(&A->d_async),
                       sizeof(double) * size_t(7 * n), acct));
        FS_TRY(dmalloc(reinterpret_cast<void **>(&A->d_apart),
                       sizeof(double) * kPersistPartials, acct));
        FS_TRY(dmalloc(reinterpret_cast<void **>(&A->d_ainfo),
                       sizeof(fs_cg_info), acct));
        A->device_bytes += acct;
    }
    return async_enqueue(A, b, x, o, A->d_async, A->d_apart, A->d_ainfo, info,
                         s);
}

extern "C" fs_status cg_solve_multi(fs_csr_t A, int32_t k, const double *B,
                                    int64_t ldb, double *X, int64_t ldx,
                                    const fs_cg_opts *opts, fs_cg_info *info,
                                    hipStream_t s)
{
    const double t0 = now_ms();
    if (k < 1 || k > 16)
        return set_error(FS_E_ARG, "k = %d, must be in [1, 16]", k);
    std::vector<fs_cg_info> local(static_cast<size_t>(k));
    std::memset(local.data(), 0, sizeof(fs_cg_info) * size_t(k));
    fs_status st = solve_any(A, k, B, ldb, X, ldx, opts, local.data(), s);
    const double ms = now_ms() - t0;
    for (auto &i : local) {
        if (st != FS_OK && i.status == FS_OK && i.iters == 0 && i.relres == 0)
            i.status = st;
        i.ms = ms;
    }
    if (info) std::memcpy(info, local.data(), sizeof(fs_cg_info) * size_t(k));
    return st;
}

extern "C" fs_status cg_solve_batch(int32_t m, const fs_csr_t *A,
                                    const int32_t *k, const double *const *B,
                                    double *const *X, const fs_cg_opts *opts,
                                    fs_cg_info *info, hipStream_t caller)
{
    const double t0 = now_ms();
    fs_cg_opts o;
    FS_TRY(normalise_opts(opts, o));
    if (m < 0 || (m > 0 && (!A || !k || !B || !X)))
        return set_error(FS_E_ARG, "NULL batch array or negative count");
    if (o.precision != FS_PREC_F64)
        return set_error(FS_E_UNSUPPORTED,
                         "batched solves run in FP64 (mixed precision is "
                         "available per system through cg_solve)");
    int32_t ncols = 0, dev = -1;
    for (int32_t i = 0; i < m; ++i) {
        FS_TRY(check_solve_args(A[i], k[i], B[i], X[i], k[i], k[i]));
        if (dev >= 0 && A[i]->device != dev)
            return set_error(FS_E_ARG, "batch members on different devices");
        dev = A[i]->device;
        ncols += k[i];
    }
    std::vector<fs_cg_info> local(static_cast<size_t>(ncols));
    std::memset(local.data(), 0, sizeof(fs_cg_info) * size_t(ncols));
    if (m == 0) return FS_OK;
    DeviceGuard g(dev);
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    FS_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    std::vector<CgSys> sys(static_cast<size_t>(m));
    fs_status st = FS_OK;
    auto run = [&]() -> fs_status {
        FS_HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        FS_HIP_TRY(hipEventRecord(ev, caller));
        FS_HIP_TRY(hipStreamWaitEvent(s, ev, 0));
        for (int32_t i = 0; i < m; ++i) {
            CgSys &S = sys[size_t(i)];
            if (A[i]->n_rows == 0) continue;
            FS_TRY(sys_alloc(S, A[i], k[i], VT_F64, ST_F64, o.precond));
            S.rtol = o.rtol;
            S.maxit = o.maxit;
            FS_TRY(load_block(A[i], k[i], B[i], k[i], S.b, s));
            if (o.x0_zero)
                FS_HIP_TRY(hipMemsetAsync(S.x, 0, sizeof(double) * size_t(S.n) *
                                                      size_t(k[i]), s));
            else
                FS_TRY(load_block(A[i], k[i], X[i], k[i], S.x, s));
        }
        // one batch per slot vector width and column-count class (both
        // are template parameters of the kernels)
        for (int32_t cls = 0; cls < 2 * kKmClasses; ++cls) {
            const int32_t vec = 1 + cls / kKmClasses, kc = cls % kKmClasses;
            Batch Bt;
            Bt.vt = VT_F64;
            Bt.st = ST_F64;
            Bt.vec = vec;
            std::vector<int32_t> idx;
            for (int32_t i = 0; i < m; ++i)
                if (A[i]->n_rows > 0 && A[i]->host.vec == vec &&
                    km_index(k[i]) == kc) {
                    Bt.members.push_back(&sys[size_t(i)]);
                    idx.push_back(i);
                }
            if (Bt.members.empty()) continue;
            fs_status r = run_batch(Bt, o.check_every, o.use_graph != 0,
                                    o.x0_zero != 0, s);
            if (r == FS_OK) {
                int32_t j = 0;
                for (int32_t i : idx) {
                    CgSys &S = sys[size_t(i)];
                    int32_t off = 0;
                    for (int32_t q = 0; q < i; ++q) off += k[q];
                    for (int32_t c = 0; c < S.k; ++c, ++j) {
                        const ColState &cs = Bt.h_stage[j];
                        fill_info(cs, local[size_t(off + c)]);
                        local[size_t(off + c)].bytes =
                            cs.iter * (12.0 * double(A[i]->nnz) / S.k +
                                       (o.precond ? 104.0 : 88.0) * S.n);
                        if (cs.bnorm2 == 0.0)
                            FS_HIP_TRY(hipMemset2DAsync(
                                static_cast<double *>(S.x) + c,
                                sizeof(double) * size_t(S.k), 0,
                                sizeof(double), size_t(S.n), s));
                    }
                    FS_TRY(store_block(A[i], S.k, S.x, X[i], S.k, s));
                }
            }
            batch_free(Bt);
            FS_TRY(r);
        }
        FS_HIP_TRY(hipStreamSynchronize(s));
        return FS_OK;
    };
    st = run();
    (void)hipStreamSynchronize(s);
    for (CgSys &S : sys) sys_free(S);
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(s);
    if (st != FS_OK) return st;
    const double ms = now_ms() - t0;
    for (auto &i : local) {
        i.ms = ms;
        st = worst(st, i.status);
    }
    if (info) std::memcpy(info, local.data(), sizeof(fs_cg_info) * size_t(ncols));
    if (st != FS_OK)
        set_error(st, "batched CG: at least one right-hand side did not "
                      "converge");
    return st;
}

namespace fs {
namespace {

// Workgroup size of cg_solve_batch_wg per batch shape, chosen by timing the
// candidates on the first call for that shape (results do not depend on
// it, so the timed runs also produce the answer).
constexpr int32_t kWgCandidates[] = {256, 512, 1024};
// tuned choice: threads * 4 + the cap on the LDS mode (2: z, x, r, p, q in
// LDS where they fit; 1: z alone, which leaves room for more workgroups
// per compute unit)
std::mutex g_wg_mu;
std::map<std::array<int64_t, 6>, int32_t> g_wg_tuned;

// Work space of cg_solve_batch_wg per device, kept between calls and grown
// to the largest batch (held until the process ends: freeing it from a
// static destructor could run after the HIP runtime has shut down).  A
// call holds its device's lock from the first use of the space to the
// end, so calls on one device run one at a time.
struct WgSpace {
    std::mutex mu;
    char *mem = nullptr;
    size_t cap = 0;
};
constexpr int kWgDevices = 64;
WgSpace g_wg_space[kWgDevices];

}  // namespace
}  // namespace fs

extern "C" fs_status cg_solve_batch_wg(int32_t m, const fs_csr_t *A,
                                       const double *const *b,
                                       double *const *x,
                                       const fs_cg_opts *opts,
                                       fs_cg_info *info, hipStream_t s)
{
    fs_cg_opts o;
    FS_TRY(normalise_opts(opts, o));
    if (m < 0 || (m > 0 && (!A || !b || !x)))
        return set_error(FS_E_ARG, "NULL batch array or negative count");
    if (o.precision != FS_PREC_F64)
        return set_error(FS_E_UNSUPPORTED,
                         "one-workgroup solves run in FP64");
    if (o.wg_threads != 0 && o.wg_threads != 256 && o.wg_threads != 512 &&
        o.wg_threads != 1024)
        return set_error(FS_E_ARG,
                         "wg_threads = %d, must be 0, 256, 512 or 1024",
                         o.wg_threads);
    int dev = -1;
    int32_t parts = 1;
    int64_t ws = 0, rows = 0, nnz = 0;
    uint64_t kinds = 0;   // the members' slot widths and column streams
    for (int32_t i = 0; i < m; ++i) {
        FS_TRY(check_solve_args(A[i], 1, b[i], x[i], 1, 1));
        const fs_csr *Ai = A[i];
        if (Ai->n_rows > kWgMaxRows || Ai->n_groups > kWgMaxParts)
            return set_error(FS_E_ARG,
                             "system %d: %d rows, %d row groups; one "
                             "workgroup takes at most %d rows and %d groups",
                             i, Ai->n_rows, Ai->n_groups, kWgMaxRows,
                             kWgMaxParts);
        if (dev >= 0 && Ai->device != dev)
            return set_error(FS_E_ARG, "batch members on different devices");
        dev = Ai->device;
        const int32_t nc = (Ai->n_rows + kWave - 1) / kWave;
        parts = std::max({parts,
                          (Ai->n_groups + kWgGroupsPerUnit - 1) /
                              kWgGroupsPerUnit,
                          (nc + kWgChunksPerUnit - 1) / kWgChunksPerUnit});
        ws += 7 * int64_t(Ai->n_rows);
        rows += Ai->n_rows;
        nnz += Ai->nnz;
        kinds = kinds * 1000003u + uint64_t(Ai->host.vec * 2 + (Ai->d_col16 ? 1 : 0));
    }
    std::vector<fs_cg_info> local(static_cast<size_t>(std::max(m, 1)));
    std::memset(local.data(), 0, sizeof(fs_cg_info) * local.size());
    if (m == 0) return FS_OK;
    DeviceGuard g(dev);
    // LDS per workgroup: the part regions, then the vectors a system keeps
    // there -- z, x, r, p and q when they fit beside the parts, else z
    // alone when it fits, else none
    int lds_max = 0;
    FS_HIP_TRY(hipDeviceGetAttribute(
        &lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t vcap =
        (int64_t(lds_max) - int64_t(sizeof(double)) * 6 * parts) /
        int64_t(sizeof(double));
    auto lds_mode = [&](int64_t n, int cap) {
        return std::min(cap, 5 * n <= vcap ? 2 : n <= vcap ? 1 : 0);
    };
    auto lds_doubles = [&](int cap) {
        int64_t v = 0;
        for (int32_t i = 0; i < m; ++i) {
            const int64_t n = A[i]->n_rows, md = lds_mode(n, cap);
            v = std::max<int64_t>(v, md == 2 ? 5 * n : md == 1 ? n : 0);
        }
        return int32_t(v);
    };
    const bool two_modes = lds_doubles(2) != lds_doubles(1);
    // one allocation: descriptors, result records, then the systems'
    // vectors (b, x, r, p, q, z, D^-1; layout numbering)
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t o_info = up(sizeof(WgSys) * size_t(m));
    const size_t o_vec = o_info + up(sizeof(fs_cg_info) * size_t(m));
    if (dev < 0 || dev >= kWgDevices)
        return set_error(FS_E_ARG, "device %d out of range", dev);
    WgSpace &W = g_wg_space[dev];
    std::lock_guard<std::mutex> space_lock(W.mu);
    const size_t need = o_vec + sizeof(double) * size_t(ws);
    if (need > W.cap) {
        // the old space is idle: every call synchronises before it returns
        dfree(W.mem);
        W.cap = 0;
        int64_t acct = 0;
        FS_TRY(dmalloc(reinterpret_cast<void **>(&W.mem), need, acct));
        W.cap = need;
    }
    char *mem = W.mem;
    WgSys *dsys = reinterpret_cast<WgSys *>(mem);
    fs_cg_info *dinfo = reinterpret_cast<fs_cg_info *>(mem + o_info);
    double *vec = reinterpret_cast<double *>(mem + o_vec);
    std::vector<WgSys> hs(static_cast<size_t>(m));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    auto run = [&]() -> fs_status {
        double *cur = vec;
        for (int32_t i = 0; i < m; ++i) {
            const fs_csr *Ai = A[i];
            WgSys &S = hs[size_t(i)];
            std::memset(&S, 0, sizeof S);
            S.info = dinfo + i;
            const int64_t n = Ai->n_rows;
            if (n == 0) continue;
            double *B = cur;
            S.groups = Ai->d_groups;
            S.val = Ai->d_val;
            S.col = Ai->d_col;
            S.cstream = Ai->d_col16 ? static_cast<const void *>(Ai->d_col16)
                                    : static_cast<const void *>(Ai->d_col);
            S.gbase = Ai->d_col16 ? Ai->d_gbase : nullptr;
            S.n = Ai->n_rows;
            S.ngroups = Ai->n_groups;
            S.vec = Ai->host.vec;
            S.narrow = Ai->d_col16 ? 1 : 0;
            S.zl = lds_mode(Ai->n_rows, 2);
            S.perm = Ai->host.identity ? nullptr : Ai->d_perm;
            S.b_in = b[i];
            S.x_in = x[i];
            S.x_out = x[i];
            S.b = B;
            S.x = B + n;
            S.r = B + 2 * n;
            S.p = B + 3 * n;
            S.q = B + 4 * n;
            S.z = B + 5 * n;
            S.dinv = o.precond ? B + 6 * n : nullptr;
            S.nnz = double(Ai->nnz);
            cur += 7 * n;
        }
        FS_HIP_TRY(hipMemsetAsync(dinfo, 0, sizeof(fs_cg_info) * size_t(m), s));
        // the descriptors with the LDS modes under a cap (uploaded when the
        // stream is idle: before the first launch, and between timed runs)
        int cur_cap = -1;
        auto modes = [&](int cap) -> fs_status {
            if (cap == cur_cap) return FS_OK;
            for (int32_t i = 0; i < m; ++i)
                if (A[i]->n_rows > 0)
                    hs[size_t(i)].zl = lds_mode(A[i]->n_rows, cap);
            FS_HIP_TRY(hipMemcpyAsync(dsys, hs.data(),
                                      sizeof(WgSys) * size_t(m),
                                      hipMemcpyHostToDevice, s));
            cur_cap = cap;
            return FS_OK;
        };
        auto launch = [&](int32_t threads, int cap, bool write_out)
            -> fs_status {
            FS_TRY(modes(cap));
            FS_HIP_TRY(launch_cg_wg(dsys, m, threads, parts, lds_doubles(cap),
                                    o.rtol, o.maxit, o.x0_zero != 0,
                                    write_out, dev, s));
            return FS_OK;
        };
        int32_t choice = o.wg_threads ? o.wg_threads * 4 + 2 : 0;
        const std::array<int64_t, 6> key = {dev, m, rows, nnz, parts,
                                            int64_t(kinds)};
        if (!choice) {
            std::lock_guard<std::mutex> lk(g_wg_mu);
            auto it = g_wg_tuned.find(key);
            if (it != g_wg_tuned.end()) choice = it->second;
        }
        if (choice) {
            FS_TRY(launch(choice / 4, choice % 4, true));
        } else {
            FS_HIP_TRY(hipEventCreate(&ev0));
            FS_HIP_TRY(hipEventCreate(&ev1));
            std::vector<int32_t> cand;
            for (int cap : {1, 2})
                if (cap == 2 || two_modes)
                    for (int32_t c : kWgCandidates) cand.push_back(c * 4 + cap);
            float best = 0.0f;
            for (size_t j = 0; j < cand.size(); ++j) {
                // every run starts from the caller's x; only the last writes
                // it back (all give bitwise the same x)
                FS_HIP_TRY(hipEventRecord(ev0, s));
                FS_TRY(launch(cand[j] / 4, cand[j] % 4, j + 1 == cand.size()));
                FS_HIP_TRY(hipEventRecord(ev1, s));
                FS_HIP_TRY(hipEventSynchronize(ev1));
                float t = 0.0f;
                FS_HIP_TRY(hipEventElapsedTime(&t, ev0, ev1));
                if (!choice || t < best) {
                    best = t;
                    choice = cand[j];
                }
            }
            std::lock_guard<std::mutex> lk(g_wg_mu);
            g_wg_tuned[key] = choice;
        }
        FS_HIP_TRY(hipMemcpyAsync(local.data(), dinfo,
                                  sizeof(fs_cg_info) * size_t(m),
                                  hipMemcpyDeviceToHost, s));
        FS_HIP_TRY(hipStreamSynchronize(s));
        return FS_OK;
    };
    fs_status st = run();
    (void)hipStreamSynchronize(s);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (st != FS_OK) return st;
    for (int32_t i = 0; i < m; ++i) st = worst(st, local[size_t(i)].status);
    if (info) std::memcpy(info, local.data(), sizeof(fs_cg_info) * size_t(m));
    if (st != FS_OK)
        set_error(st, "one-workgroup CG: at least one system did not "
                      "converge");
    return st;
}
