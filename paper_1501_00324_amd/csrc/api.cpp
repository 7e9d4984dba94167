// The C ABI: handle lifetime, products and the CG driver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "host.h"

namespace fs {

namespace {
thread_local std::string g_last_error;

void free_handle(fs_csr *A)
{
    free_solver_state(A);
    dfree(A->d_groups); dfree(A->d_val); dfree(A->d_val_f32);
    dfree(A->d_val_bf16); dfree(A->d_col); dfree(A->d_map); dfree(A->d_imap);
    dfree(A->d_jpos); dfree(A->d_rstart);
    dfree(A->d_col16); dfree(A->d_gbase);
    dfree(A->d_perm); dfree(A->d_iperm); dfree(A->d_xtmp); dfree(A->d_Xtmp);
}

fs_status check_handle(const fs_csr *A)
{
    if (!A) return set_error(FS_E_ARG, "NULL matrix handle");
    return FS_OK;
}

}  // namespace

fs_status set_error(fs_status code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

}  // namespace fs

using namespace fs;

extern "C" {

const char *fs_last_error(void) { return g_last_error.c_str(); }

fs_status csr_opts_default(fs_csr_opts *o)
{
    if (!o) return set_error(FS_E_ARG, "NULL opts");
    std::memset(o, 0, sizeof *o);
    o->reorder = FS_REORDER_AUTO;
    o->sort_window = 0;
    o->threshold = 48;
    o->lanes_min = 1;
    o->lanes_max = 64;
    return FS_OK;
}

fs_status cg_opts_default(fs_cg_opts *o)
{
    if (!o) return set_error(FS_E_ARG, "NULL opts");
    std::memset(o, 0, sizeof *o);
    o->rtol = 1e-8;
    o->maxit = 20000;
    o->precond = FS_PC_JACOBI;
    o->precision = FS_PREC_F64;
    o->inner_rtol = 1e-2;
    o->check_every = 32;
    o->use_graph = 1;
    o->max_outer = 50;
    return FS_OK;
}

}  // extern "C"

namespace fs {
namespace {

// Row starts and byte-wide in-row positions of the slots (the value
// refresh reads one byte per slot instead of the 4-byte inverse map), for
// matrices whose rows hold at most 255 entries and whose positions fit 32
// bits; otherwise the refresh keeps the inverse map.  After the inverse map
// is built, on the same stream.
fs_status build_refresh_rows(fs_csr *A, const int32_t *h_rp, int64_t &acct,
                             hipStream_t s)
{
    if (A->slots == 0 || A->nnz > INT32_MAX) return FS_OK;
    int32_t maxlen = 0;
    for (int32_t i = 0; i < A->n_rows; ++i)
        maxlen = std::max(maxlen, h_rp[size_t(i) + 1] - h_rp[size_t(i)]);
    if (maxlen > 255) return FS_OK;
    FS_TRY(dalloc(&A->d_jpos, A->slots, acct));
    FS_TRY(dalloc(&A->d_rstart, A->n_rows, acct));
    FS_HIP_TRY(launch_refresh_rows(A->d_groups, A->n_groups, A->host.vec,
                                   A->d_imap, A->d_jpos, A->d_rstart, s));
    return FS_OK;
}

// Device handle from host structure arrays (layout built here) and device
// values.  Synchronises s.
fs_status create_from_host(int32_t n_rows, int32_t n_cols, int64_t nnz,
                           const int32_t *h_rp, const int32_t *h_col,
                           const double *vals, const fs_csr_opts &o,
                           hipStream_t s, int dev, fs_csr **out)
{
    fs_csr *A = new (std::nothrow) fs_csr();
    if (!A) return set_error(FS_E_OOM, "host allocation failed");
    A->n_rows = n_rows;
    A->n_cols = n_cols;
    A->nnz = nnz;
    A->device = dev;
    A->build = FS_BUILD_HOST;
    fs_status st = build_layout(n_rows, n_cols, nnz, h_rp, h_col, o, A->host);
    if (st != FS_OK) {
        delete A;
        return st;
    }
    HostLayout &L = A->host;
    A->n_groups = int32_t(L.groups.size());
    A->slots = L.slots;
    A->pipe_product = A->n_groups > 0 &&
                      L.slots >= 32 * int64_t(kWave) * A->n_groups;

    auto fail = [&](fs_status code) {
        (void)hipStreamSynchronize(s);
        free_handle(A);
        delete A;
        return code;
    };
    int64_t &acct = A->device_bytes;
    if ((st = dalloc(&A->d_groups, A->n_groups, acct)) ||
        (st = dalloc(&A->d_val, A->slots, acct)) ||
        (st = dalloc(&A->d_col, A->slots, acct)) ||
        (st = dalloc(&A->d_map, nnz, acct)) ||
        (st = dalloc(&A->d_imap, A->slots, acct)) ||
        (st = dalloc(&A->d_perm, n_rows, acct)) ||
        (st = dalloc(&A->d_iperm, n_rows, acct)) ||
        (st = dalloc(&A->d_xtmp, n_cols, acct)))
        return fail(st);
    if (L.index_bits == 16)
        if ((st = dalloc(&A->d_col16, A->slots, acct)) ||
            (st = dalloc(&A->d_gbase, A->n_groups, acct)))
            return fail(st);
    if (o.dtypes & FS_DT_F32)
        if ((st = dalloc(&A->d_val_f32, A->slots, acct))) return fail(st);
    if (o.dtypes & FS_DT_BF16)
        if ((st = dalloc(&A->d_val_bf16, A->slots, acct))) return fail(st);

    hipError_t e = hipSuccess;
#define FS_CREATE_HIP(expr)                                                 \
    if ((e = (expr)) != hipSuccess)                                         \
        return fail(set_error(FS_E_HIP, "%s: %s", #expr, hipGetErrorString(e)))
    if (A->n_groups)
        FS_CREATE_HIP(hipMemcpyAsync(A->d_groups, L.groups.data(),
                                     sizeof(Group) * L.groups.size(),
                                     hipMemcpyHostToDevice, s));
    if (A->slots) {
        FS_CREATE_HIP(hipMemcpyAsync(A->d_col, L.slot_col.data(),
                                     sizeof(int32_t) * size_t(A->slots),
                                     hipMemcpyHostToDevice, s));
        FS_CREATE_HIP(hipMemsetAsync(A->d_val, 0,
                                     sizeof(double) * size_t(A->slots), s));
        if (A->d_col16) {
            FS_CREATE_HIP(hipMemcpyAsync(A->d_col16, L.slot_c16.data(),
                                         sizeof(uint16_t) * size_t(A->slots),
                                         hipMemcpyHostToDevice, s));
            FS_CREATE_HIP(hipMemcpyAsync(A->d_gbase, L.gbase.data(),
                                         sizeof(int32_t) * L.gbase.size(),
                                         hipMemcpyHostToDevice, s));
        }
        if (A->d_val_f32)
            FS_CREATE_HIP(hipMemsetAsync(A->d_val_f32, 0,
                                         sizeof(float) * size_t(A->slots), s));
        if (A->d_val_bf16)
            FS_CREATE_HIP(hipMemsetAsync(A->d_val_bf16, 0,
                                         sizeof(uint16_t) * size_t(A->slots),
                                         s));
    }
    if (nnz)
        FS_CREATE_HIP(hipMemcpyAsync(A->d_map, L.map.data(),
                                     sizeof(int32_t) * size_t(nnz),
                                     hipMemcpyHostToDevice, s));
    if (A->slots)
        FS_CREATE_HIP(hipMemsetAsync(A->d_imap, 0xff,
                                     sizeof(int32_t) * size_t(A->slots), s));
    FS_CREATE_HIP(launch_inverse_map(A->d_map, nnz, A->d_imap, s));
    if ((st = build_refresh_rows(A, h_rp, acct, s))) return fail(st);
    if (n_rows) {
        FS_CREATE_HIP(hipMemcpyAsync(A->d_perm, L.perm.data(),
                                     sizeof(int32_t) * size_t(n_rows),
                                     hipMemcpyHostToDevice, s));
        FS_CREATE_HIP(hipMemcpyAsync(A->d_iperm, L.iperm.data(),
                                     sizeof(int32_t) * size_t(n_rows),
                                     hipMemcpyHostToDevice, s));
    }
    FS_CREATE_HIP(launch_value_scatter(vals, A->d_map, nnz, A->d_val,
                                       A->d_val_f32, A->d_val_bf16, s));
    FS_CREATE_HIP(hipStreamSynchronize(s));
#undef FS_CREATE_HIP
    A->dtypes = FS_DT_F64 | (A->d_val_f32 ? FS_DT_F32 : 0) |
                (A->d_val_bf16 ? FS_DT_BF16 : 0);
    // the slot columns and map are on the device now; keep only what the
    // info / permutation queries need on the host
    std::vector<int32_t>().swap(L.slot_col);
    std::vector<int32_t>().swap(L.map);
    std::vector<uint16_t>().swap(L.slot_c16);
    *out = A;
    return FS_OK;
}

// Device array -> host array (allocated here, not zero-filled).  The copy
// lands in a pinned buffer at full link speed and is then copied out by
// several threads, which also spreads the first-touch page faults of the
// destination (a direct copy into fresh pageable memory, or a zero-filled
// std::vector, costs several times the transfer; reading the pinned buffer
// itself from the host is slower than reading ordinary memory).
// Synchronises s.
template <class T>
fs_status fetch_to_host(std::unique_ptr<T[]> &dst, const T *src, int64_t n,
                        hipStream_t s)
{
    dst.reset();
    if (n <= 0) return FS_OK;
    dst.reset(new (std::nothrow) T[size_t(n)]);
    if (!dst) return set_error(FS_E_OOM, "host allocation failed");
    PinnedBuf<T> pin;
    FS_TRY(pin.alloc(n));
    FS_HIP_TRY(hipMemcpyAsync(pin.data(), src, sizeof(T) * size_t(n),
                              hipMemcpyDeviceToHost, s));
    FS_HIP_TRY(hipStreamSynchronize(s));
    constexpr int64_t kPiece = int64_t(1) << 20;     // elements per task
    const int64_t np = (n + kPiece - 1) / kPiece;
    T *d = dst.get();
    const T *h = pin.data();
    parallel_chunks(np, [&](int64_t c) {
        const int64_t a = c * kPiece, len = std::min(kPiece, n - a);
        std::memcpy(d + a, h + a, sizeof(T) * size_t(len));
    });
    return FS_OK;
}

// Device handle with the per-non-zero phases of the layout build on the
// device: the host reads only the row offsets (and the columns when the row
// order needs the graph), computes the row order and the row groups
// (layout_order, layout_groups, the same code as the host builder), and the
// kernels validate the columns, assign slots, write the CSR -> slot map and
// the 16-bit offsets, and sum the bandwidth statistics.  Falls back to the
// host builder when a row exceeds FS_BUILD_DEVICE_MAX_ROW entries (the
// per-row ranking costs L * ceil(L / 64) steps for a row of length L).
// Synchronises s.
fs_status create_on_device(int32_t n_rows, int32_t n_cols, int64_t nnz,
                           const int32_t *rowptr, const int32_t *colind,
                           const double *vals, const fs_csr_opts &o,
                           hipStream_t s, int dev, fs_csr **out)
{
    std::vector<int32_t> h_rp(static_cast<size_t>(n_rows) + 1);
    FS_HIP_TRY(hipMemcpyAsync(h_rp.data(), rowptr,
                              sizeof(int32_t) * (size_t(n_rows) + 1),
                              hipMemcpyDeviceToHost, s));
    FS_HIP_TRY(hipStreamSynchronize(s));
    FS_TRY(layout_check_rowptr(n_rows, nnz, h_rp.data()));
    int32_t maxlen = 0;
    for (int32_t i = 0; i < n_rows; ++i)
        maxlen = std::max(maxlen, h_rp[size_t(i) + 1] - h_rp[size_t(i)]);
    std::unique_ptr<int32_t[]> h_col;
    auto host_cols = [&]() -> fs_status {
        return fetch_to_host(h_col, colind, nnz, s);
    };
    if (maxlen > FS_BUILD_DEVICE_MAX_ROW) {
        FS_TRY(host_cols());
        return create_from_host(n_rows, n_cols, nnz, h_rp.data(),
                                h_col.get(), vals, o, s, dev, out);
    }

    // flags: [0] first bad column, [1] first duplicate, [2..3] band sums
    unsigned long long *d_flags = nullptr;
    int2 *d_lohi = nullptr;
    int64_t scratch_bytes = 0;
    FS_TRY(dalloc(&d_flags, 4, scratch_bytes));
    struct Scratch {
        unsigned long long *&f;
        int2 *&l;
        ~Scratch() { dfree(f); dfree(l); }
    } scratch{d_flags, d_lohi};
    unsigned long long flags[4];
    const unsigned long long kNone = ~0ull;
    FS_HIP_TRY(hipMemsetAsync(d_flags, 0xff, 2 * sizeof(flags[0]), s));
    FS_HIP_TRY(hipMemsetAsync(d_flags + 2, 0, 2 * sizeof(flags[0]), s));
    FS_HIP_TRY(launch_check_cols(colind, nnz, n_cols, d_flags, s));
    FS_HIP_TRY(hipMemcpyAsync(flags, d_flags, sizeof(flags[0]),
                              hipMemcpyDeviceToHost, s));
    FS_HIP_TRY(hipStreamSynchronize(s));
    if (flags[0] != kNone) {
        int32_t c = 0;
        FS_HIP_TRY(hipMemcpy(&c, colind + flags[0], sizeof c,
                             hipMemcpyDeviceToHost));
        return set_error(FS_E_BAD_CSR, "column %d out of range at %lld", c,
                         (long long)flags[0]);
    }
    LayoutParams prm;
    FS_TRY(layout_params(o, prm));
    if (layout_order_reads_columns(n_rows, n_cols, o)) FS_TRY(host_cols());

    fs_csr *A = new (std::nothrow) fs_csr();
    if (!A) return set_error(FS_E_OOM, "host allocation failed");
    A->n_rows = n_rows;
    A->n_cols = n_cols;
    A->nnz = nnz;
    A->device = dev;
    A->build = FS_BUILD_DEVICE;
    HostLayout &L = A->host;
    auto fail = [&](fs_status code) {
        (void)hipStreamSynchronize(s);
        free_handle(A);
        delete A;
        return code;
    };
    fs_status st = layout_order(n_rows, n_cols, h_rp.data(), h_col.get(), o,
                                L);
    if (st == FS_OK)
        st = layout_groups(n_rows, n_cols, h_rp.data(), o, prm, L);
    if (st != FS_OK) return fail(st);
    h_col.reset();
    A->n_groups = int32_t(L.groups.size());
    A->slots = L.slots;
    A->pipe_product = A->n_groups > 0 &&
                      L.slots >= 32 * int64_t(kWave) * A->n_groups;
    const bool square = n_rows == n_cols;

    int64_t &acct = A->device_bytes;
    if ((st = dalloc(&A->d_groups, A->n_groups, acct)) ||
        (st = dalloc(&A->d_val, A->slots, acct)) ||
        (st = dalloc(&A->d_col, A->slots, acct)) ||
        (st = dalloc(&A->d_map, nnz, acct)) ||
        (st = dalloc(&A->d_imap, A->slots, acct)) ||
        (st = dalloc(&A->d_perm, n_rows, acct)) ||
        (st = dalloc(&A->d_iperm, n_rows, acct)) ||
        (st = dalloc(&A->d_xtmp, n_cols, acct)) ||
        (st = dalloc(&d_lohi, A->n_groups, scratch_bytes)))
        return fail(st);
    if (o.dtypes & FS_DT_F32)
        if ((st = dalloc(&A->d_val_f32, A->slots, acct))) return fail(st);
    if (o.dtypes & FS_DT_BF16)
        if ((st = dalloc(&A->d_val_bf16, A->slots, acct))) return fail(st);

    hipError_t e = hipSuccess;
#define FS_DEV_HIP(expr)                                                    \
    if ((e = (expr)) != hipSuccess)                                         \
        return fail(set_error(FS_E_HIP, "%s: %s", #expr, hipGetErrorString(e)))
    if (A->n_groups)
        FS_DEV_HIP(hipMemcpyAsync(A->d_groups, L.groups.data(),
                                  sizeof(Group) * L.groups.size(),
                                  hipMemcpyHostToDevice, s));
    if (n_rows) {
        FS_DEV_HIP(hipMemcpyAsync(A->d_perm, L.perm.data(),
                                  sizeof(int32_t) * size_t(n_rows),
                                  hipMemcpyHostToDevice, s));
        FS_DEV_HIP(hipMemcpyAsync(A->d_iperm, L.iperm.data(),
                                  sizeof(int32_t) * size_t(n_rows),
                                  hipMemcpyHostToDevice, s));
    }
    if (A->slots) {
        FS_DEV_HIP(hipMemsetAsync(A->d_col, 0xff,
                                  sizeof(int32_t) * size_t(A->slots), s));
        FS_DEV_HIP(hipMemsetAsync(A->d_val, 0,
                                  sizeof(double) * size_t(A->slots), s));
        if (A->d_val_f32)
            FS_DEV_HIP(hipMemsetAsync(A->d_val_f32, 0,
                                      sizeof(float) * size_t(A->slots), s));
        if (A->d_val_bf16)
            FS_DEV_HIP(hipMemsetAsync(A->d_val_bf16, 0,
                                      sizeof(uint16_t) * size_t(A->slots), s));
    }
    FS_DEV_HIP(launch_assign_slots(A->d_groups, A->n_groups, L.vec, A->d_perm,
                                   L.symmetric_relabel ? A->d_iperm : nullptr,
                                   rowptr, colind, A->d_col, A->d_map, d_lohi,
                                   d_flags + 1, s));
    if (square)
        FS_DEV_HIP(launch_band(n_rows, rowptr, colind, A->d_iperm,
                               d_flags + 2, s));
    std::vector<int2> lohi(size_t(A->n_groups));
    if (A->n_groups)
        FS_DEV_HIP(hipMemcpyAsync(lohi.data(), d_lohi,
                                  sizeof(int2) * lohi.size(),
                                  hipMemcpyDeviceToHost, s));
    FS_DEV_HIP(hipMemcpyAsync(flags + 1, d_flags + 1, 3 * sizeof(flags[0]),
                              hipMemcpyDeviceToHost, s));
    FS_DEV_HIP(hipStreamSynchronize(s));
    if (flags[1] != kNone) {
        const int64_t k = int64_t(flags[1]);
        const int32_t row = int32_t(std::upper_bound(h_rp.begin(), h_rp.end(),
                                                     int32_t(k)) -
                                    h_rp.begin()) - 1;
        int32_t c = 0;
        FS_DEV_HIP(hipMemcpy(&c, colind + k, sizeof c, hipMemcpyDeviceToHost));
        return fail(set_error(FS_E_BAD_CSR, "duplicate column %d in row %d",
                              c, row));
    }
    if (square && nnz > 0) {
        // integer sums: the same values the host builder's chunked sums give
        L.band_before = double(flags[2]) / double(nnz);
        L.band_after = double(flags[3]) / double(nnz);
    }
    // 16-bit offsets when every group's columns span fewer than 65535
    L.index_bits = 32;
    bool fits = o.index_bits == 0 && A->n_groups > 0;
    for (size_t g = 0; g < lohi.size() && fits; ++g)
        fits = lohi[g].y - lohi[g].x < 0xffff;
    if (fits) {
        if ((st = dalloc(&A->d_col16, A->slots, acct)) ||
            (st = dalloc(&A->d_gbase, A->n_groups, acct)))
            return fail(st);
        FS_DEV_HIP(launch_offsets16(A->d_groups, A->n_groups, A->d_col, d_lohi,
                                    A->d_col16, A->d_gbase, s));
        L.index_bits = 16;
    }
    if (A->slots)
        FS_DEV_HIP(hipMemsetAsync(A->d_imap, 0xff,
                                  sizeof(int32_t) * size_t(A->slots), s));
    FS_DEV_HIP(launch_inverse_map(A->d_map, nnz, A->d_imap, s));
    if ((st = build_refresh_rows(A, h_rp.data(), acct, s))) return fail(st);
    FS_DEV_HIP(launch_value_scatter(vals, A->d_map, nnz, A->d_val,
                                    A->d_val_f32, A->d_val_bf16, s));
    FS_DEV_HIP(hipStreamSynchronize(s));
#undef FS_DEV_HIP
    A->dtypes = FS_DT_F64 | (A->d_val_f32 ? FS_DT_F32 : 0) |
                (A->d_val_bf16 ? FS_DT_BF16 : 0);
    *out = A;
    return FS_OK;
}

// Mean time of one layout-numbering product, from HIP events around
// `reps` launches on s.
fs_status time_product(fs_csr *A, const double *x, double *y, int reps,
                       hipStream_t s, double &us)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FS_HIP_TRY(hipEventCreate(&e0));
    FS_HIP_TRY(hipEventCreate(&e1));
    for (int i = 0; i < 3; ++i) FS_HIP_TRY(launch_spmv_f64(A, x, y, nullptr, s));
    FS_HIP_TRY(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) FS_HIP_TRY(launch_spmv_f64(A, x, y, nullptr, s));
    FS_HIP_TRY(hipEventRecord(e1, s));
    FS_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    FS_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    us = 1e3 * double(ms) / reps;
    return FS_OK;
}

// Tuned layout choices, by matrix signature (sizes and a hash of the row
// length sequence), for the life of the process.
struct TuneKey {
    int32_t n_rows, n_cols;
    int64_t nnz;
    uint64_t hash;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(n_rows, n_cols, nnz, hash) <
               std::tie(o.n_rows, o.n_cols, o.nnz, o.hash);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int32_t, int32_t>> g_tune;  // -> (lanes, vec)

uint64_t row_hash(int32_t n, const int32_t *rp)
{
    uint64_t h = 1469598103934665603ull;                   // FNV-1a
    for (int32_t i = 0; i < n; ++i) {
        h ^= uint64_t(uint32_t(rp[i + 1] - rp[i]));
        h *= 1099511628211ull;
    }
    return h;
}

// Project autotuner: time the product for a small set of row-group shapes
// (lanes per row T and slots per load V) on the real matrix and keep the
// fastest.  The locality permutation is computed once and reused.
fs_status create_tuned(int32_t n_rows, int32_t n_cols, int64_t nnz,
                       const int32_t *h_rp, const int32_t *h_col,
                       const double *vals, fs_csr_opts o, hipStream_t s,
                       int dev, fs_csr **out)
{
    const TuneKey key{n_rows, n_cols, nnz, row_hash(n_rows, h_rp)};
    std::pair<int32_t, int32_t> chosen{0, 0};   // {0, 0}: default shape
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            chosen = it->second;
            cached = true;
        }
    }
    // the first candidate is the default shape; it fixes the permutation
    fs_csr *best = nullptr;
    FS_TRY(create_from_host(n_rows, n_cols, nnz, h_rp, h_col, vals, o, s,
                            dev, &best));
    if (cached && chosen.first > 0) {
        // rebuild the cached shape exactly as the tuning run built it: the
        // default build's permutation, no further window sort
        const std::vector<int32_t> perm = best->host.perm;
        const int32_t reorder0 = best->host.reorder;
        fs_csr_opts oc = o;
        oc.reorder = FS_REORDER_USER;
        oc.perm = perm.data();
        oc.sort_window = 1;
        oc.lanes_min = oc.lanes_max = chosen.first;
        oc.vec = chosen.second;
        fs_csr *A = nullptr;
        const fs_status st = create_from_host(n_rows, n_cols, nnz, h_rp,
                                              h_col, vals, oc, s, dev, &A);
        free_handle(best);
        delete best;
        if (st != FS_OK) return st;
        best = A;
        best->host.reorder = reorder0;
    }
    if (cached || n_rows != n_cols || n_rows == 0) {
        best->tuned = cached ? 2 : 0;
        *out = best;
        return FS_OK;
    }
    double *x = nullptr, *y = nullptr;
    int64_t dummy = 0;
    fs_status st = FS_OK;
    if ((st = dalloc(&x, n_cols, dummy)) || (st = dalloc(&y, n_rows, dummy))) {
        dfree(x);
        free_handle(best);
        delete best;
        return st;
    }
    (void)hipMemsetAsync(x, 0, sizeof(double) * size_t(n_cols), s);
    double best_us = 0.0;
    st = time_product(best, x, y, 20, s, best_us);
    const std::vector<int32_t> perm = best->host.perm;
    const int32_t reorder0 = best->host.reorder;
    const int32_t cand[][2] = {{1, 2}, {1, 1}, {2, 2}, {2, 1}, {4, 2}, {8, 1}};
    int32_t ntried = 1;
    for (const auto &c : cand) {
        if (st != FS_OK) break;
        fs_csr_opts oc = o;
        oc.reorder = FS_REORDER_USER;
        oc.perm = perm.data();
        oc.sort_window = 1;
        oc.lanes_min = oc.lanes_max = c[0];
        oc.vec = c[1];
        fs_csr *A = nullptr;
        st = create_from_host(n_rows, n_cols, nnz, h_rp, h_col, vals, oc, s,
                              dev, &A);
        if (st != FS_OK) break;
        double us = 0.0;
        st = time_product(A, x, y, 20, s, us);
        ++ntried;
        if (st == FS_OK && us < best_us) {
            std::swap(A, best);
            best_us = us;
            chosen = {c[0], c[1]};
        }
        free_handle(A);
        delete A;
    }
    dfree(x);
    dfree(y);
    if (st != FS_OK) {
        free_handle(best);
        delete best;
        return st;
    }
    // candidates reuse the first build's permutation: report its origin
    best->host.reorder = reorder0;
    best->tuned = 1;
    best->tune_candidates = ntried;
    best->tune_best_us = best_us;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = chosen;
    }
    *out = best;
    return FS_OK;
}

}  // namespace
}  // namespace fs

extern "C" {

fs_status csr_create(int32_t n_rows, int32_t n_cols, int64_t nnz,
                     const int32_t *rowptr, const int32_t *colind,
                     const double *vals, const fs_csr_opts *opts,
                     hipStream_t s, fs_csr_t *out)
{
    const double t0 = now_ms();
    if (!out) return set_error(FS_E_ARG, "NULL output handle pointer");
    *out = nullptr;
    if (n_rows < 0 || n_cols < 0 || nnz < 0)
        return set_error(FS_E_ARG, "negative size (%d x %d, nnz %lld)",
                         n_rows, n_cols, (long long)nnz);
    if (nnz >= INT32_MAX)
        return set_error(FS_E_UNSUPPORTED, "nnz must be below 2^31");
    if (!rowptr || (nnz > 0 && (!colind || !vals)))
        return set_error(FS_E_ARG, "NULL CSR array");
    fs_csr_opts o;
    csr_opts_default(&o);
    if (opts) o = *opts;
    if (o.dtypes & ~(FS_DT_F64 | FS_DT_F32 | FS_DT_BF16))
        return set_error(FS_E_ARG, "unknown dtype bits 0x%x", o.dtypes);

    if (o.build != FS_BUILD_HOST && o.build != FS_BUILD_DEVICE)
        return set_error(FS_E_ARG, "unknown build option %d", o.build);

    int dev = 0;
    FS_HIP_TRY(hipGetDevice(&dev));
    if (o.build == FS_BUILD_DEVICE && !o.autotune) {
        fs_csr *A = nullptr;
        FS_TRY(create_on_device(n_rows, n_cols, nnz, rowptr, colind, vals, o,
                                s, dev, &A));
        A->t_build_ms = now_ms() - t0;
        *out = A;
        return FS_OK;
    }
    std::unique_ptr<int32_t[]> h_rp, h_col;
    FS_TRY(fetch_to_host(h_rp, rowptr, int64_t(n_rows) + 1, s));
    FS_TRY(fetch_to_host(h_col, colind, nnz, s));
    fs_csr *A = nullptr;
    if (o.autotune)
        FS_TRY(create_tuned(n_rows, n_cols, nnz, h_rp.get(), h_col.get(),
                            vals, o, s, dev, &A));
    else
        FS_TRY(create_from_host(n_rows, n_cols, nnz, h_rp.get(),
                                h_col.get(), vals, o, s, dev, &A));
    A->t_build_ms = now_ms() - t0;
    *out = A;
    return FS_OK;
}

fs_status csr_layout_host(int32_t n_rows, int32_t n_cols, int64_t nnz,
                          const int32_t *rowptr, const int32_t *colind,
                          const fs_csr_opts *opts, int32_t *n_groups,
                          int64_t *slots, int32_t *vec, int32_t *groups,
                          int32_t *slot_col, int32_t *map, int32_t *perm)
{
    if (n_rows < 0 || n_cols < 0 || nnz < 0)
        return set_error(FS_E_ARG, "negative size");
    if (nnz >= INT32_MAX)
        return set_error(FS_E_UNSUPPORTED, "nnz must be below 2^31");
    if (!rowptr || (nnz > 0 && !colind))
        return set_error(FS_E_ARG, "NULL CSR array");
    fs_csr_opts o;
    csr_opts_default(&o);
    if (opts) o = *opts;
    HostLayout L;
    FS_TRY(build_layout(n_rows, n_cols, nnz, rowptr, colind, o, L));
    if (n_groups) *n_groups = int32_t(L.groups.size());
    if (slots) *slots = L.slots;
    if (vec) *vec = L.vec;
    if (groups && !L.groups.empty())
        std::memcpy(groups, L.groups.data(), sizeof(Group) * L.groups.size());
    if (slot_col && L.slots)
        std::memcpy(slot_col, L.slot_col.data(),
                    sizeof(int32_t) * size_t(L.slots));
    if (map && nnz) std::memcpy(map, L.map.data(), sizeof(int32_t) * size_t(nnz));
    if (perm && n_rows)
        std::memcpy(perm, L.perm.data(), sizeof(int32_t) * size_t(n_rows));
    return FS_OK;
}

fs_status csr_update_values(fs_csr_t A, const double *vals, hipStream_t s)
{
    FS_TRY(check_handle(A));
    if (!vals && A->nnz > 0) return set_error(FS_E_ARG, "NULL values");
    DeviceGuard g(A->device);
    if (A->d_jpos)
        FS_HIP_TRY(launch_value_refresh_rows(
            A->d_groups, A->n_groups, A->host.vec, A->d_jpos, A->d_rstart,
            vals, A->d_val, A->d_val_f32, A->d_val_bf16, s));
    else
        FS_HIP_TRY(launch_value_refresh(A->d_groups, A->n_groups, A->d_imap,
                                        vals, A->d_val, A->d_val_f32,
                                        A->d_val_bf16, s));
    A->lo_scaled_dt = 0;   // the scaled copy is rebuilt by the next solve
    return FS_OK;
}

fs_status csr_get_values(fs_csr_t A, double *vals, hipStream_t s)
{
    FS_TRY(check_handle(A));
    if (!vals && A->nnz > 0) return set_error(FS_E_ARG, "NULL values");
    DeviceGuard g(A->device);
    FS_HIP_TRY(launch_value_gather(A->d_val, A->d_map, A->nnz, vals, s));
    return FS_OK;
}

fs_status csr_info(fs_csr_t A, fs_csr_stats *st)
{
    FS_TRY(check_handle(A));
    if (!st) return set_error(FS_E_ARG, "NULL stats");
    std::memset(st, 0, sizeof *st);
    st->n_rows = A->n_rows;
    st->n_cols = A->n_cols;
    st->nnz = A->nnz;
    st->slots = A->slots;
    st->n_groups = A->n_groups;
    st->reorder = A->host.reorder;
    st->padding = A->slots ? double(A->slots - A->nnz) / double(A->slots) : 0.0;
    st->bytes_algorithmic = 12 * A->nnz + 8 * int64_t(A->n_cols) +
                            8 * int64_t(A->n_rows);
    const bool narrow = A->d_col16 != nullptr;
    st->bytes_layout = (narrow ? 10 : 12) * A->slots +
                       int64_t(sizeof(Group) + (narrow ? 4 : 0)) * A->n_groups +
                       8 * int64_t(A->n_cols) + 8 * int64_t(A->n_rows);
    st->index_bits = narrow ? 16 : 32;
    for (int i = 0; i < 7; ++i) st->groups_by_lanes[i] = A->host.groups_by_lanes[i];
    st->dtypes = A->dtypes;
    st->vec = A->host.vec;
    st->mean_band_before = A->host.band_before;
    st->mean_band_after = A->host.band_after;
    st->t_build_ms = A->t_build_ms;
    st->tuned = A->tuned;
    st->tune_candidates = A->tune_candidates;
    st->tune_best_us = A->tune_best_us;
    st->device_bytes = A->device_bytes;
    st->build = A->build;
    return FS_OK;
}

fs_status csr_get_perm(fs_csr_t A, int32_t *perm_host)
{
    FS_TRY(check_handle(A));
    if (!perm_host && A->n_rows > 0) return set_error(FS_E_ARG, "NULL perm");
    if (A->n_rows)
        std::memcpy(perm_host, A->host.perm.data(),
                    sizeof(int32_t) * size_t(A->n_rows));
    return FS_OK;
}

fs_status csr_get_layout(fs_csr_t A, int32_t *groups, int32_t *slot_col,
                         int32_t *map, uint16_t *col16, int32_t *gbase)
{
    FS_TRY(check_handle(A));
    if ((col16 || gbase) && !A->d_col16)
        return set_error(FS_E_ARG, "the layout has 32-bit column indices");
    DeviceGuard g(A->device);
    if (groups && A->n_groups)
        FS_HIP_TRY(hipMemcpy(groups, A->d_groups,
                             sizeof(Group) * size_t(A->n_groups),
                             hipMemcpyDeviceToHost));
    if (slot_col && A->slots)
        FS_HIP_TRY(hipMemcpy(slot_col, A->d_col,
                             sizeof(int32_t) * size_t(A->slots),
                             hipMemcpyDeviceToHost));
    if (map && A->nnz)
        FS_HIP_TRY(hipMemcpy(map, A->d_map, sizeof(int32_t) * size_t(A->nnz),
                             hipMemcpyDeviceToHost));
    if (col16 && A->slots)
        FS_HIP_TRY(hipMemcpy(col16, A->d_col16,
                             sizeof(uint16_t) * size_t(A->slots),
                             hipMemcpyDeviceToHost));
    if (gbase && A->n_groups)
        FS_HIP_TRY(hipMemcpy(gbase, A->d_gbase,
                             sizeof(int32_t) * size_t(A->n_groups),
                             hipMemcpyDeviceToHost));
    return FS_OK;
}

fs_status csr_destroy(fs_csr_t A)
{
    if (!A) return FS_OK;
    DeviceGuard g(A->device);
    (void)hipDeviceSynchronize();
    free_handle(A);
    delete A;
    return FS_OK;
}

fs_status spmv(fs_csr_t A, const double *x, double *y, hipStream_t s)
{
    FS_TRY(check_handle(A));
    if ((!x && A->n_cols) || (!y && A->n_rows))
        return set_error(FS_E_ARG, "NULL vector");
    if (x == y && x) return set_error(FS_E_ARG, "x and y must not alias");
    DeviceGuard g(A->device);
    const HostLayout &L = A->host;
    if (L.identity) {
        FS_HIP_TRY(launch_spmv_f64(A, x, y, nullptr, s));
    } else if (L.symmetric_relabel) {
        // x' = x(perm), then y(perm[row]) = (A' x')[row] in the epilogue
        FS_HIP_TRY(launch_gather(A->n_cols, A->d_perm, x, A->d_xtmp, s));
        FS_HIP_TRY(launch_spmv_f64(A, A->d_xtmp, y, A->d_perm, s));
    } else {
        FS_HIP_TRY(launch_spmv_f64(A, x, y, A->d_perm, s));
    }
    return FS_OK;
}

fs_status spmv_csr(int32_t n_rows, int32_t n_cols, int64_t nnz,
                   const int32_t *rowptr, const int32_t *colind,
                   const double *vals, const double *x, double *y,
                   hipStream_t s)
{
    if (n_rows < 0 || n_cols < 0 || nnz < 0)
        return set_error(FS_E_ARG, "negative size");
    if (n_rows == 0) return FS_OK;
    if (!rowptr || !y || (nnz > 0 && (!colind || !vals)) ||
        (n_cols > 0 && !x))
        return set_error(FS_E_ARG, "NULL array");
    if (x == y) return set_error(FS_E_ARG, "x and y must not alias");
    FS_HIP_TRY(launch_spmv_csr(n_rows, n_cols, nnz, rowptr, colind, vals, x,
                               y, s));
    return FS_OK;
}

fs_status probe_read_bandwidth(const double *buf, int64_t n, double *sink,
                               int32_t blocks, hipStream_t s)
{
    if (n < 0 || blocks < 1 || blocks > (1 << 20))
        return set_error(FS_E_ARG, "n must be >= 0 and blocks in [1, 2^20]");
    if (n >= 2 && (!buf || !sink))
        return set_error(FS_E_ARG, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0)
        return set_error(FS_E_ARG, "buffer must be 16-byte aligned");
    FS_HIP_TRY(launch_read_probe(buf, n, sink, blocks, s));
    return FS_OK;
}

fs_status spmv_batch(int32_t m, const fs_csr_t *A, const double *const *x,
                     double *const *y, hipStream_t s)
{
    if (m < 0) return set_error(FS_E_ARG, "negative batch size %d", m);
    if (m == 0) return FS_OK;
    if (!A || !x || !y) return set_error(FS_E_ARG, "NULL batch array");
    int dev = -1;
    for (int32_t i = 0; i < m; ++i) {
        FS_TRY(check_handle(A[i]));
        if ((!x[i] && A[i]->n_cols) || (!y[i] && A[i]->n_rows))
            return set_error(FS_E_ARG, "NULL vector in batch entry %d", i);
        if (dev >= 0 && A[i]->device != dev)
            return set_error(FS_E_ARG, "batch members on different devices");
        dev = A[i]->device;
    }
    // no x_i may alias any y_j (the products run concurrently)
    std::vector<const void *> ys;
    for (int32_t i = 0; i < m; ++i)
        if (A[i]->n_rows) ys.push_back(y[i]);
    std::sort(ys.begin(), ys.end());
    if (std::adjacent_find(ys.begin(), ys.end()) != ys.end())
        return set_error(FS_E_ARG, "two batch entries share one y");
    for (int32_t i = 0; i < m; ++i)
        if (A[i]->n_cols && std::binary_search(ys.begin(), ys.end(),
                                               static_cast<const void *>(x[i])))
            return set_error(FS_E_ARG, "x of batch entry %d is some y", i);
    DeviceGuard g(dev);
    FS_HIP_TRY(launch_spmv_batch(m, A, x, y, s));
    return FS_OK;
}

fs_status spmv_perm(fs_csr_t A, const double *xp, double *yp, hipStream_t s)
{
    FS_TRY(check_handle(A));
    if (A->n_rows != A->n_cols)
        return set_error(FS_E_NOT_SQUARE, "spmv_perm needs a square matrix");
    if ((!xp || !yp) && A->n_rows) return set_error(FS_E_ARG, "NULL vector");
    if (xp == yp && xp) return set_error(FS_E_ARG, "x and y must not alias");
    DeviceGuard g(A->device);
    FS_HIP_TRY(launch_spmv_f64(A, xp, yp, nullptr, s));
    return FS_OK;
}

fs_status csr_permute(fs_csr_t A, int32_t dir, const double *in, double *out,
                      hipStream_t s)
{
    FS_TRY(check_handle(A));
    if ((!in || !out) && A->n_rows) return set_error(FS_E_ARG, "NULL vector");
    if (in == out && in) return set_error(FS_E_ARG, "in and out must not alias");
    DeviceGuard g(A->device);
    if (dir == FS_TO_LAYOUT)
        FS_HIP_TRY(launch_gather(A->n_rows, A->d_perm, in, out, s));
    else if (dir == FS_FROM_LAYOUT)
        FS_HIP_TRY(launch_scatter(A->n_rows, A->d_perm, in, out, s));
    else
        return set_error(FS_E_ARG, "unknown direction %d", dir);
    return FS_OK;
}

fs_status spmm(fs_csr_t A, int32_t k, const double *X, int64_t ldx,
               double *Y, int64_t ldy, hipStream_t s)
{
    FS_TRY(check_handle(A));
    if (k < 1 || k > 16) return set_error(FS_E_ARG, "k = %d, must be in [1, 16]", k);
    if (ldx < k || ldy < k) return set_error(FS_E_ARG, "leading dimension below k");
    if ((!X && A->n_cols) || (!Y && A->n_rows))
        return set_error(FS_E_ARG, "NULL block");
    if (X == Y && X) return set_error(FS_E_ARG, "X and Y must not alias");
    DeviceGuard g(A->device);
    const HostLayout &L = A->host;
    if (L.identity) {
        FS_HIP_TRY(launch_spmm_f64(A, k, X, ldx, Y, ldy, nullptr, s));
    } else if (L.symmetric_relabel) {
        // X' = X(perm, :) in a k-wide buffer, then Y(perm[row], :) = (A' X')
        const int64_t need = int64_t(A->n_cols) * k;
        if (need > A->xtmp_cap) {
            FS_HIP_TRY(hipStreamSynchronize(s));
            dfree(A->d_Xtmp);
            A->xtmp_cap = 0;
            FS_TRY(dalloc(&A->d_Xtmp, int64_t(A->n_cols) * 16, A->device_bytes));
            A->xtmp_cap = int64_t(A->n_cols) * 16;
        }
        FS_HIP_TRY(permute_rows(A->n_cols, k, A->d_perm, X, ldx, A->d_Xtmp, k,
                                true, s));
        FS_HIP_TRY(launch_spmm_f64(A, k, A->d_Xtmp, k, Y, ldy, A->d_perm, s));
    } else {
        FS_HIP_TRY(launch_spmm_f64(A, k, X, ldx, Y, ldy, A->d_perm, s));
    }
    return FS_OK;
}

fs_status spmv_lowp(fs_csr_t A, int32_t dtype, const float *xp, float *yp,
                    hipStream_t s)
{
    FS_TRY(check_handle(A));
    if (A->n_rows != A->n_cols)
        return set_error(FS_E_NOT_SQUARE, "spmv_lowp needs a square matrix");
    if (dtype != FS_DT_F32 && dtype != FS_DT_BF16)
        return set_error(FS_E_ARG, "dtype must be FS_DT_F32 or FS_DT_BF16");
    if (!(A->dtypes & dtype))
        return set_error(FS_E_ARG, "no %s copy: call csr_add_dtype first",
                         dtype == FS_DT_F32 ? "FP32" : "BF16");
    if ((!xp || !yp) && A->n_rows) return set_error(FS_E_ARG, "NULL vector");
    if (xp == yp && xp) return set_error(FS_E_ARG, "x and y must not alias");
    DeviceGuard g(A->device);
    FS_HIP_TRY(launch_spmv_lowp(A, dtype, xp, yp, s));
    return FS_OK;
}

fs_status csr_add_dtype(fs_csr_t A, int32_t dtype, hipStream_t s)
{
    FS_TRY(check_handle(A));
    if (dtype != FS_DT_F32 && dtype != FS_DT_BF16)
        return set_error(FS_E_ARG, "dtype must be FS_DT_F32 or FS_DT_BF16");
    if (A->dtypes & dtype) return FS_OK;
    DeviceGuard g(A->device);
    if (dtype == FS_DT_F32)
        FS_TRY(dalloc(&A->d_val_f32, A->slots, A->device_bytes));
    else
        FS_TRY(dalloc(&A->d_val_bf16, A->slots, A->device_bytes));
    FS_HIP_TRY(cast_slots(A->slots, A->d_val,
                          dtype == FS_DT_F32 ? A->d_val_f32 : nullptr,
                          dtype == FS_DT_BF16 ? A->d_val_bf16 : nullptr, s));
    FS_HIP_TRY(hipStreamSynchronize(s));
    A->dtypes |= dtype;
    return FS_OK;
}

}  // extern "C"

