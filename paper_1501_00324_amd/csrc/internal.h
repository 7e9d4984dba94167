// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fespmv.h"
#include "layout.h"

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
// Group, kWave and kBlock (the device data layout) are in layout.h.
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
    // 16-bit column indices: slot_c16[s] = column - gbase[group], 0xffff
    // for padding; empty when index_bits == 32
    int32_t index_bits = 32;
    std::vector<uint16_t> slot_c16;
    std::vector<int32_t> gbase;
};

fs_status build_layout(int32_t n_rows, int32_t n_cols, int64_t nnz,
                       const int32_t *rowptr, const int32_t *col,
                       const fs_csr_opts &o, HostLayout &L);

// Phases of build_layout, shared with the device builder (which runs the
// per-non-zero phases -- column checks, bandwidth, slot assignment, 16-bit
// offsets -- on the GPU and these on the host).
struct LayoutParams { int32_t threshold, tmin, tmax; };
fs_status layout_check_rowptr(int32_t n_rows, int64_t nnz,
                              const int32_t *rowptr);
fs_status layout_params(const fs_csr_opts &o, LayoutParams &p);
// true when layout_order needs the column indices (graph reordering)
bool layout_order_reads_columns(int32_t n_rows, int32_t n_cols,
                                const fs_csr_opts &o);
// initial row order (identity, caller's, or reverse Cuthill-McKee): L.perm,
// L.reorder.  col may be NULL when layout_order_reads_columns is false.
fs_status layout_order(int32_t n_rows, int32_t n_cols, const int32_t *rowptr,
                       const int32_t *col, const fs_csr_opts &o,
                       HostLayout &L);
// window sort and row groups from the row lengths: L.perm (final), iperm,
// identity, symmetric_relabel, vec, groups, groups_by_lanes, slots
fs_status layout_groups(int32_t n_rows, int32_t n_cols, const int32_t *rowptr,
                        const fs_csr_opts &o, const LayoutParams &prm,
                        HostLayout &L);

// ------------------------------------------------- batched CG engine state
// Status of one right-hand side.
enum { CG_RUNNING = 0, CG_CONVERGED = 1, CG_RECURRENCE_MET = 2,
       CG_BREAKDOWN = 3, CG_MAXIT = 4 };

struct ColState {                // one right-hand side, device resident
    double rho, gamma, alpha, beta;
    double rr;                   // |r|^2 of the recurrence residual
    double rr_true;              // |b - A x|^2 at the last true check
    double bnorm2, tol2;
    double rho_prev;             // rho of the previous iteration (fused path)
    int32_t iter, status, pending, maxit;
    int32_t replacements, pad[3];
};

// One linear system of a batched launch, in layout numbering.  Vectors are
// n x k, row-major (leading dimension k), of the launch's vector type.
struct SysDesc {
    const Group *groups;
    const void *val;             // slot values: double, float or bf16 bits
    const int32_t *col;          // 32-bit slot columns
    const void *cstream;         // column stream of the products: col, or
    const int32_t *gbase;        //   16-bit offsets from gbase[group]
    int32_t n, ngroups, k, maxit;
    int32_t sb0, snb;            // blocks in the group-shaped grid
    int32_t vb0, vnb;            // blocks in the row-shaped grid
    void *x, *r, *p, *q;
    const void *b, *dinv;        // dinv NULL: no preconditioner
    ColState *cs;                // k entries
    int32_t *bad_diag;           // rows with a zero / non-finite diagonal
    double *partials;            // 3 * k * max(snb, vnb) entries
    double rtol;
    double *hist;                // alpha_j, beta_j per iteration (one
    int32_t hist_cap, pad2;      //   column), or NULL: not recorded
};

// Column-count class of a system with k right-hand sides: the launch's
// compile-time column count (1, 2, 4, 8 or 16) and its index 0..4.  Systems
// share a launch only with systems of the same class, so the arithmetic of
// a system never depends on the other members of its batch.
constexpr int kKmClasses = 5;
inline int32_t km_for(int32_t k)
{
    return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
}
inline int32_t km_index(int32_t k)
{
    return k <= 1 ? 0 : k <= 2 ? 1 : k <= 4 ? 2 : k <= 8 ? 3 : 4;
}

// Value / vector type classes of a launch.
enum { VT_F64 = 0, VT_F32 = 1, VT_BF16 = 2 };
enum { ST_F64 = 0, ST_F32 = 1 };

struct EngineLaunch {            // one batched launch shape
    int32_t vt, st, vec, km;     // value type, vector type, slots/load, max k
    const SysDesc *sys;          // device array of systems
    const int32_t *smap;         // group-shaped grid block -> system
    const int32_t *vmap;         // row-shaped grid block -> system
    const int2 *cmap;            // finalize block -> (system, column)
    int32_t sblocks, vblocks, ncols;  // grid sizes
};

int32_t engine_spmv_blocks(int32_t ngroups);
int32_t engine_vec_blocks(int32_t n, int32_t k);
// One CG iteration for every running right-hand side of every system:
// Q = A P with p.q, then x/r update with r.z and r.r, then the p update.
hipError_t engine_iteration(const EngineLaunch &L, hipStream_t s);
// mode 0 (start: r = b - A x, p = z, sets the per-column state), 1 (true
// residual check with replacement), 2 (measure |b - A x| only), 3 (rebase
// the columns that met their tolerance on a new b, keeping p).
hipError_t engine_residual(const EngineLaunch &L, int32_t mode,
                           bool x_zero, hipStream_t s);
// p = z + beta p for the columns whose residual was just replaced.
hipError_t engine_pupdate_pending(const EngineLaunch &L, hipStream_t s);
// dinv = 1 / diag(A) (vector type of the launch); counts bad diagonals.
hipError_t engine_diag_inv(const EngineLaunch &L, hipStream_t s);
// staging[i] = the ColState of finalize column i (cmap order).
hipError_t engine_gather_states(const EngineLaunch &L, ColState *staging,
                                hipStream_t s);
// n x k row blocks between caller (stride ld*) and layout order; perm NULL
// is the identity.
hipError_t permute_rows(int32_t n, int32_t k, const int32_t *perm,
                        const double *src, int64_t lds, double *dst,
                        int64_t ldd, bool to_layout, hipStream_t s);
// b = float(a) (sc NULL) or float(sc[row] a), n entries, k per row
hipError_t to_f32(int64_t n, int32_t k, const double *a, const double *sc,
                  float *b, hipStream_t s);
// x += alpha * d (d widened exactly), or x += alpha * (sc[row] d)
hipError_t add_f32(int64_t n, int32_t k, double alpha, const float *d,
                   const double *sc, double *x, hipStream_t s);
// sc = diag(A)^-1/2 (FP64, layout rows; non-positive diagonals counted in
// *bad) and out = the FP32 / BF16 copy of D^-1/2 A D^-1/2 in slot order
hipError_t scaled_lowp_copy(const struct ::fs_csr *A, int32_t dtype,
                            double *sc, void *out, int32_t *bad,
                            hipStream_t s);
hipError_t cast_slots(int64_t n, const double *v, float *f32, uint16_t *bf16,
                      hipStream_t s);
// p[0 .. n) = v (a kernel, not a memset: safe inside captured work)
hipError_t fill_f64(int64_t n, double v, double *p, hipStream_t s);

// ------------------------------------------------------------ host engine
// Device state of one system (matrix + k right-hand sides) in one vector
// precision, in layout numbering.
struct CgSys {
    struct ::fs_csr *A = nullptr;
    int32_t k = 0, vt = VT_F64, st = ST_F64, precond = 1;
    int32_t n = 0, snb = 0, vnb = 0;
    void *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr,
         *b = nullptr, *dinv = nullptr;
    ColState *cs = nullptr;
    int32_t *bad = nullptr;
    double *partials = nullptr;
    double rtol = 1e-8;
    int32_t maxit = 20000;
    int64_t bytes = 0;
    const void *val = nullptr;   // values used instead of A's (scaled copy)
    double *hist = nullptr;      // coefficient record (2 per iteration)
    int32_t hist_cap = 0;
    bool record = false;         // record the coefficients in this solve
    bool carved = false;         // parts of a caller-owned block
};

// A set of systems launched together (same value/vector types and slot
// vector width).  Device copies of the descriptors and block maps.
struct Batch {
    std::vector<CgSys *> members;
    int32_t vt = VT_F64, st = ST_F64, vec = 2, km = 1;
    SysDesc *d_sys = nullptr;
    int32_t *d_smap = nullptr, *d_vmap = nullptr;
    int2 *d_cmap = nullptr;
    ColState *d_stage = nullptr, *h_stage = nullptr;
    int32_t cap_sys = 0, cap_s = 0, cap_v = 0, cap_c = 0;
    EngineLaunch L{};
    hipGraphExec_t graph = nullptr;
    int32_t graph_iters = 0;
    std::vector<int2> cols;           // (member, column) per finalize block
    // pinned staging of stream-ordered descriptor uploads, and the event
    // of the last upload
    void *h_up = nullptr;
    size_t up_cap = 0;
    hipEvent_t up_ev = nullptr;
};

fs_status sys_alloc(CgSys &S, struct ::fs_csr *A, int32_t k, int32_t vt,
                    int32_t st, int32_t precond);
// One device block for all of a system's state (sys_alloc_in carves it;
// the block stays the caller's: sys_free only forgets the parts).
int64_t sys_block_bytes(const struct ::fs_csr *A, int32_t k, int32_t st,
                        int32_t precond);
void sys_alloc_in(CgSys &S, struct ::fs_csr *A, int32_t k, int32_t vt,
                  int32_t st, int32_t precond, void *block);
void sys_free(CgSys &S);
fs_status batch_build(Batch &B, hipStream_t s);   // upload descs and maps
// async_upload: stream-ordered upload from pinned staging, no host wait
fs_status batch_build(Batch &B, hipStream_t s, bool async_upload);
// gather the column states and copy them to h_stage, without waiting
fs_status batch_stage_states(Batch &B, hipStream_t s);
void batch_free(Batch &B);
fs_status batch_iterations(Batch &B, int32_t iters, bool use_graph,
                           hipStream_t s);
fs_status batch_read_states(Batch &B, hipStream_t s);  // -> h_stage
void free_solver_state(struct ::fs_csr *A);
// Stream-ordered solve (cg_solve_async and its no-allocation variant):
// argument checks (o receives the normalised options), then the enqueue
// with workspace ws (7 n doubles), part (kPersistPartials doubles) and the
// device result dinfo, copied to the host record info on s.
fs_status async_check(struct ::fs_csr *A, const double *b, double *x,
                      const fs_cg_opts *opts, fs_cg_info *info,
                      fs_cg_opts &o);
fs_status async_enqueue(struct ::fs_csr *A, const double *b, double *x,
                        const fs_cg_opts &o, double *ws, double *part,
                        fs_cg_info *dinfo, fs_cg_info *info, hipStream_t s);

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
    uint16_t *d_col16 = nullptr;   // 16-bit offsets (index_bits 16), or NULL
    int32_t *d_gbase = nullptr;    // per-group column base for d_col16
    int32_t *d_map = nullptr;
    int32_t *d_imap = nullptr;     // slot -> CSR position, -1 = padding
    // the product runs the pipelined lane sum: lanes own 32 or more slots
    // on average (at least four 8-slot batches)
    bool pipe_product = false;
    // per-Newton-step refresh through row starts (rows of <= 255 entries):
    // d_rstart[row] = CSR position of the row's first entry, d_jpos[slot] =
    // position within the row, 255 = padding; NULL: refresh through d_imap
    uint8_t *d_jpos = nullptr;
    int32_t *d_rstart = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_iperm = nullptr;
    double *d_xtmp = nullptr;      // gathered x for caller-numbering spmv
    double *d_Xtmp = nullptr;      // gathered X for caller-numbering spmm
    int64_t xtmp_cap = 0;
    int32_t dtypes = FS_DT_F64;
    double t_build_ms = 0.0;
    int64_t device_bytes = 0;
    int32_t tuned = 0, tune_candidates = 0;
    double tune_best_us = 0.0;
    int32_t build = FS_BUILD_HOST; // the builder that ran (FS_BUILD_*)
    // solver state, created on the first solve and kept for reuse
    hipStream_t stream = nullptr;  // solves run here, ordered after the
    hipEvent_t ev = nullptr;       // caller's stream by an event
    fs::CgSys *sys_f64 = nullptr;  // one right-hand side, FP64
    fs::CgSys *sys_lo = nullptr;   // inner system of mixed precision
    fs::Batch *batch_f64 = nullptr, *batch_lo = nullptr;
    // stream-ordered solves (cg_solve_async): b, x, r, p, q, dinv in layout
    // numbering, block partials, the device result
    double *d_async = nullptr, *d_apart = nullptr;
    fs_cg_info *d_ainfo = nullptr;
    // scaled refinement: D^-1/2 per layout row and the low-precision copy
    // of D^-1/2 A D^-1/2 (dtype lo_scaled_dt; 0 = none or stale after a
    // value update)
    double *d_iscale = nullptr;
    void *d_val_lo_scaled = nullptr;
    int32_t lo_scaled_dt = 0;
};

namespace fs {
// ---------------------------------------------------------------- launchers
// All launchers are asynchronous on stream s and return hipError_t.
hipError_t launch_value_scatter(const double *vals, const int32_t *map,
                                int64_t nnz, double *slot_val, float *f32,
                                uint16_t *bf16, hipStream_t s);
// device layout build (build.hip)
hipError_t launch_inverse_map(const int32_t *map, int64_t nnz, int32_t *imap,
                              hipStream_t s);
hipError_t launch_value_refresh(const Group *groups, int32_t ngroups,
                                const int32_t *imap, const double *vals,
                                double *val, float *f32, uint16_t *bf16,
                                hipStream_t s);
// d_jpos / d_rstart from the inverse map (one wavefront per row group)
hipError_t launch_refresh_rows(const Group *groups, int32_t ngroups,
                               int32_t vec, const int32_t *imap,
                               uint8_t *jpos, int32_t *rstart, hipStream_t s);
// the refresh through them
hipError_t launch_value_refresh_rows(const Group *groups, int32_t ngroups,
                                     int32_t vec, const uint8_t *jpos,
                                     const int32_t *rstart,
                                     const double *vals, double *val,
                                     float *f32, uint16_t *bf16,
                                     hipStream_t s);
hipError_t launch_check_cols(const int32_t *col, int64_t nnz, int32_t n_cols,
                             unsigned long long *first, hipStream_t s);
hipError_t launch_band(int32_t n, const int32_t *rowptr, const int32_t *col,
                       const int32_t *iperm, unsigned long long *sums,
                       hipStream_t s);
hipError_t launch_assign_slots(const Group *groups, int32_t ngroups,
                               int32_t vec, const int32_t *perm,
                               const int32_t *iperm, const int32_t *rowptr,
                               const int32_t *col, int32_t *slot_col,
                               int32_t *map, int2 *lohi,
                               unsigned long long *dup, hipStream_t s);
hipError_t launch_offsets16(const Group *groups, int32_t ngroups,
                            const int32_t *slot_col, const int2 *lohi,
                            uint16_t *col16, int32_t *gbase, hipStream_t s);
hipError_t launch_gather(int32_t n, const int32_t *perm, const double *in,
                         double *out, hipStream_t s);
hipError_t launch_scatter(int32_t n, const int32_t *perm, const double *in,
                          double *out, hipStream_t s);
// y[row or yperm[row]] = (A x)[row] over all groups.
hipError_t launch_spmv_f64(const fs_csr *A, const double *x, double *y,
                           const int32_t *yperm, hipStream_t s);
// Y[row or yperm[row], :] = (A X)[row, :] for k <= 16 columns.
hipError_t launch_spmm_f64(const fs_csr *A, int32_t k, const double *X,
                           int64_t ldx, double *Y, int64_t ldy,
                           const int32_t *yperm, hipStream_t s);
// m products y_i = A_i x_i in caller numbering, descriptors passed as
// kernel arguments (kBatchPerLaunch matrices per launch).
constexpr int kBatchPerLaunch = 56;
hipError_t launch_spmv_batch(int32_t m, const fs_csr *const *A,
                             const double *const *x, double *const *y,
                             hipStream_t s);
// Whole-solve persistent CG (one cooperative launch, one right-hand side,
// FP64, layout numbering): grid size for the handle, and the launch.  info
// is a device struct written at the end.
constexpr int kPersistMaxBlocks = 1024;
// block partials of the persistent kernel (two regions of 3 per block),
// then its grid barrier counter (at double index kPersistBarrierAt)
constexpr int kPersistBarrierAt = 2 * 3 * kPersistMaxBlocks;
constexpr int kPersistPartials = kPersistBarrierAt + 32;
int32_t persistent_blocks(const fs_csr *A);
hipError_t launch_cg_persistent(const fs_csr *A, int32_t nblocks,
                                const double *b, double *x, double *r,
                                double *p, double *q, double *z, double *dinv,
                                double *part, fs_cg_info *info, double rtol,
                                int32_t maxit, bool x_zero, hipStream_t s);
// One-workgroup solves (FP64, one right-hand side per system, layout
// numbering): the whole Jacobi-PCG solve of a system in one workgroup, one
// launch for a batch.  A system's per-group and per-64-row sums live in LDS,
// which bounds it to kWgMaxParts row groups and kWgMaxRows rows.
constexpr int32_t kWgMaxParts = 1024;
constexpr int32_t kWgMaxRows = 64 * kWgMaxParts;
struct WgSys {
    const Group *groups;
    const double *val;
    const int32_t *col;        // 32-bit layout columns (diagonal search)
    const void *cstream;       // column stream of the product
    const int32_t *gbase;      // group bases of 16-bit offsets, or NULL
    int32_t n, ngroups, vec, narrow;
    int32_t zl, pad;           // vectors in LDS: 0 none, 1 z = D^-1 r,
                               // 2 z, x, r, p, q
    const int32_t *perm;       // layout row i is caller row perm[i] (NULL:
                               // the same numbering)
    const double *b_in, *x_in; // caller's b and initial guess
    double *x_out;             // caller's x (written at the end)
    double *b;                 // work space, layout numbering
    double *x, *r, *p, *q, *z, *dinv;  // dinv NULL: no preconditioner
    fs_cg_info *info;          // device record of the result
    double nnz;
};
// Units of one wavefront's work: row groups per unit (product steps) and
// 64-row chunks per unit (vector step).
constexpr int32_t kWgGroupsPerUnit = 2;
constexpr int32_t kWgChunksPerUnit = 4;
// threads: 256, 512 or 1024; parts >= every system's group and chunk
// units (LDS: 48 bytes per part, then vec_doubles for the vectors that the
// systems keep in LDS: n per system with zl = 1, 5 n with zl = 2).
// write_out false: x_out is left alone (timed runs of the same inputs).
hipError_t launch_cg_wg(const WgSys *d_sys, int32_t m, int32_t threads,
                        int32_t parts, int32_t vec_doubles, double rtol,
                        int32_t maxit, bool x_zero, bool write_out,
                        int device, hipStream_t s);
// Plain CSR product (no layout), lanes per row from the mean row length.
int32_t csr_lanes_log2(int32_t n_rows, int64_t nnz);
hipError_t launch_spmv_csr(int32_t n_rows, int32_t n_cols, int64_t nnz,
                           const int32_t *rowptr, const int32_t *col,
                           const double *val, const double *x, double *y,
                           hipStream_t s);
// Streaming read of n doubles (n even, 16-byte aligned) by `blocks`
// workgroups; one partial sum per block into sink.
hipError_t launch_read_probe(const double *buf, int64_t n, double *sink,
                             int32_t blocks, hipStream_t s);
// Low-precision product in layout numbering: y = A_lo x (float vectors,
// float accumulation), A_lo the FP32 or BF16 copy.
hipError_t launch_spmv_lowp(const fs_csr *A, int32_t dtype, const float *x,
                            float *y, hipStream_t s);
// vals[k] = slot_val[map[k]]: the FP64 values back in CSR order.
hipError_t launch_value_gather(const double *slot_val, const int32_t *map,
                               int64_t nnz, double *vals, hipStream_t s);

// ------------------------------------------------------------- assembly
// Device plan of one sum-only product out[tpos[t]] = sum_j in[idx_t(j)]
// (tpos[t] = -1: a filler task, nothing written): tasks t are cut into
// waves of 64; wave w stores its tasks' index lists
// column-interleaved, idx_t(j) = aidx[(base64 + j) * 64 + t % 64] for
// j < width (-1 after a task's last entry), base64 and width = waves[w].
struct AsmPlan {
    int64_t ntasks = 0;
    int32_t nwaves = 0;
    int64_t stored = 0;          // aidx entries, padding included
    int64_t contrib = 0;         // entries that are not padding
    int32_t *d_waves = nullptr;  // 2 per wave: base64, width
    int32_t *d_tpos = nullptr;
    int32_t *d_aidx = nullptr;
};
// f32 / bf16 (may be NULL) receive the rounded result at the same place.
hipError_t launch_assemble(const AsmPlan &P, const double *in, double *out,
                           float *f32, uint16_t *bf16, hipStream_t s);
// Row-group plan of the matrix assembly (accumulation in LDS): one
// workgroup per row group of the layout zeroes the group's slot region in
// LDS, adds the element values of its rows into it and writes the region
// out.  The rows of a group are taken `rows` (= 64 / nde) at a time by one
// wavefront (a batch); step k of a batch gives every row of the batch its
// k-th element row e*nde + a (ascending) and lane q*nde + b adds element
// value (e*nde + a)*nde + b at its LDS offset.
constexpr int kAsmLdsMax = 6144;  // doubles of LDS per group region (48 KiB)
struct AsmLdsPlan {
    int32_t ngroups = 0, nde = 0, rows = 0;
    int32_t region_max = 0;      // doubles of the widest group region
    int64_t nbatch = 0, nrec = 0, contrib = 0;
    int32_t *d_gdesc = nullptr;  // 4 per group: base64, width, batch0, nbatch
    int32_t *d_bdesc = nullptr;  // 2 per batch: first record, steps
    int32_t *d_ea = nullptr;     // `rows` per record: e*nde + a, -1 = none
    uint16_t *d_off = nullptr;   // 64 per record: LDS offset, 0xffff = none
};
// With re != NULL the element vectors are summed in the same launch into
// r (caller numbering: r[perm[layout row]]); groups / perm are the matrix's.
// With ordered, ke is the plan-ordered element buffer (row rec * rows + q
// holds the element row that batch row q adds at record rec) and re is
// ignored.
hipError_t launch_assemble_lds(const AsmLdsPlan &P, const double *ke,
                               double *val, float *f32, uint16_t *bf16,
                               const Group *groups, const int32_t *perm,
                               const double *re, double *r, bool ordered,
                               hipStream_t s);
}  // namespace fs

struct fs_asm {
    fs_csr *A = nullptr;
    int device = 0;
    int32_t n_elem = 0, nde = 0;
    bool lds = false;            // matrix by the row-group plan kl
    fs::AsmPlan km, rv;          // matrix (into A's slots), vector (rows)
    fs::AsmLdsPlan kl;
    double t_build_ms = 0.0;
    int64_t device_bytes = 0;
};
