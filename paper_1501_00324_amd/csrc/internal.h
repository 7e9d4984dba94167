// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fespmv.h"

namespace fs {

// ----------------------------------------------------------------- errors
fs_status set_error(fs_status code, const char *fmt, ...);
void clear_error();

#define FS_HIP_TRY(expr)                                                    \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess)                                               \
            return ::fs::set_error(FS_E_HIP, "%s: %s (%s:%d)", #expr,       \
                                   hipGetErrorString(e_), __FILE__,         \
                                   __LINE__);                               \
    } while (0)

#define FS_TRY(expr)                                                        \
    do {                                                                    \
        fs_status s_ = (expr);                                              \
        if (s_ != FS_OK) return s_;                                         \
    } while (0)

// ----------------------------------------------------------------- layout
// One row group is processed by one 64-lane wavefront.  A group holds
// 64 / T consecutive layout rows, T lanes per row (T a power of two); entry
// e of a row (columns ascending) goes to lane (row_in_group * T + e % T),
// slot e / T of that lane.  Slots are interleaved so that one wave-wide
// load of V consecutive slots per lane (V = 1 or 2, per matrix) is one
// contiguous 64*V element block:
//     element index = base + (s / V) * 64 * V + lane * V + s % V.
constexpr int kWave = 64;
constexpr int kBlock = 256;        // threads per workgroup (4 waves)

struct Group {                     // 16 bytes, read once per wave
    int32_t base64;                // first element index / 64
    int32_t row0;                  // first layout row
    int32_t nrows;                 // rows in the group (1..64/T)
    int32_t width_lt;              // slots per lane | log2(T) << 24
};

struct HostLayout {
    std::vector<int32_t> perm;     // layout row i <- caller row perm[i]
    std::vector<int32_t> iperm;
    std::vector<Group> groups;
    std::vector<int32_t> slot_col; // layout column per slot, -1 = padding
    std::vector<int32_t> map;      // CSR position k -> slot index
    int64_t slots = 0;
    int32_t vec = 2;                 // slots per lane per load (1 or 2)
    int32_t reorder = FS_REORDER_NONE;
    int32_t groups_by_lanes[7] = {0, 0, 0, 0, 0, 0, 0};
    double band_before = 0.0, band_after = 0.0;
    bool symmetric_relabel = false;  // columns relabelled by iperm
    bool identity = true;            // perm is the identity
};

fs_status build_layout(int32_t n_rows, int32_t n_cols, int64_t nnz,
                       const int32_t *rowptr, const int32_t *col,
                       const fs_csr_opts &o, HostLayout &L);

// ------------------------------------------------------------ CG scalars
struct CgScalars {
    double rho, gamma, alpha, beta;
    double rr;          // |r|^2 of the recurrence residual
    double rr_true;     // |b - A x|^2 from the last true-residual check
    double bnorm2, tol2;
    int32_t iter, done, status, maxit;
    uint32_t counter;   // last-block-done ticket, reset by the last block
    int32_t replacements;
    int32_t pad[2];
};
enum { CG_RUNNING = 0, CG_CONVERGED = 1, CG_RECURRENCE_MET = 2,
       CG_BREAKDOWN = 3, CG_MAXIT = 4 };

// Per-handle Krylov workspace (layout numbering), allocated on first solve.
struct CgWork {
    int32_t n = 0;
    double *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr,
           *b = nullptr, *dinv = nullptr, *partials = nullptr;
    CgScalars *sc = nullptr;       // device
    CgScalars *sc_host = nullptr;  // pinned host mirror
    int32_t nparts = 0;
    hipStream_t stream = nullptr;  // solves run here, ordered after the
                                   // caller's stream by an event
    hipEvent_t done_ev = nullptr;
    hipGraphExec_t graph = nullptr;
    int32_t graph_k = 0, graph_pc = -1;
};

}  // namespace fs

struct fs_csr {
    int32_t n_rows, n_cols;
    int64_t nnz;
    int device;
    fs::HostLayout host;           // kept for info / perm queries
    int32_t n_groups = 0;
    int64_t slots = 0;
    fs::Group *d_groups = nullptr;
    double *d_val = nullptr;
    float *d_val_f32 = nullptr;
    uint16_t *d_val_bf16 = nullptr;
    int32_t *d_col = nullptr;
    int32_t *d_map = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_iperm = nullptr;
    double *d_xtmp = nullptr;      // gathered x for caller-numbering spmv
    int32_t dtypes = FS_DT_F64;
    double t_build_ms = 0.0;
    int64_t device_bytes = 0;
    fs::CgWork cg;
};

namespace fs {
// ---------------------------------------------------------------- launchers
// All launchers are asynchronous on stream s and return hipError_t.
hipError_t launch_value_scatter(const double *vals, const int32_t *map,
                                int64_t nnz, double *slot_val, float *f32,
                                uint16_t *bf16, hipStream_t s);
hipError_t launch_gather(int32_t n, const int32_t *perm, const double *in,
                         double *out, hipStream_t s);
hipError_t launch_scatter(int32_t n, const int32_t *perm, const double *in,
                          double *out, hipStream_t s);
// y[row or yperm[row]] = (A x)[row] over all groups.
hipError_t launch_spmv_f64(const fs_csr *A, const double *x, double *y,
                           const int32_t *yperm, hipStream_t s);

// CG (layout numbering)
int32_t cg_partials_needed(const fs_csr *A);
hipError_t launch_cg_spmv_dot(const fs_csr *A, CgWork &w, hipStream_t s);
hipError_t launch_cg_update(CgWork &w, int32_t precond, hipStream_t s);
hipError_t launch_cg_pupdate(CgWork &w, int32_t precond, hipStream_t s);
// r = b - A x, with partial sums for |r|^2 and r.z; mode 0: initial residual
// (sets rho, rr, bnorm2, tol2 and p = z); mode 1: convergence check with
// residual replacement; mode 2: measurement only (rr_true).
hipError_t launch_cg_residual(const fs_csr *A, CgWork &w, int32_t precond,
                              int32_t mode, double rtol, int32_t maxit,
                              int32_t x_is_zero, hipStream_t s);
// dinv = 1 / diag(A) in layout numbering; rows with a zero or non-finite
// diagonal are counted in sc->pad[0].
hipError_t launch_diag_inv(const fs_csr *A, double *dinv, CgScalars *sc,
                           hipStream_t s);
}  // namespace fs
