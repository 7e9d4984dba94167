// gfx950 kernels for the FEM SpMV / CG path.
//
// SpMV (paper: statement y = A x, section "Description of Current GPU
// Methods"; row-grouped column-interleaved kernels, section "Development of
// Novel GPU Algorithms") is bandwidth bound (2 flops per 12-byte slot), so
// nothing here uses MFMA.  What matters on CDNA4:
//  * one 64-lane wavefront per row group, 16-byte (two-slot) loads per lane
//    so each wave-wide access is one contiguous 1 KiB (values) / 512 B
//    (columns) block; the matrix stream is loaded non-temporally so that the
//    gathered vector keeps its place in L2 / MALL;
//  * rows with T > 1 lanes are reduced with cross-lane shuffles (no LDS
//    traffic, no barrier), replacing the paper's shared-memory tree;
//  * workgroups are renumbered so that each of the 8 XCDs (own 4 MB L2)
//    walks a contiguous range of row groups and therefore a narrow window
//    of x in the locality (RCM) order;
//  * padded slots carry column -1 and are skipped, so padding never
//    multiplies an Inf/NaN of x.
// CG (paper: Jacobi-preconditioned CG, at least one SpMV per iteration) runs
// as three fused kernels per iteration with device-resident scalars and a
// deterministic two-stage reduction (per-block partials in a fixed order,
// summed by the last block to finish).
#include <cmath>

#include "internal.h"

namespace fs {
namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef int iv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));

constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kVecBlocks = 1024;   // max workgroups of the vector kernels

// Workgroups are dispatched round-robin over the 8 XCDs; renumber so XCD k
// owns one contiguous range of logical blocks.  A bijection for any grid.
__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    constexpr int NX = 8;
    const int xcd = bid % NX, idx = bid / NX;
    const int base = nblk / NX, rem = nblk % NX;
    return xcd * base + (xcd < rem ? xcd : rem) + idx;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int V> struct Slots;
template <> struct Slots<1> { typedef double D; typedef int I; };
template <> struct Slots<2> { typedef dv2 D; typedef iv2 I; };

// Padded slots (column -1) read x[0] (always in bounds: a matrix with
// slots has at least one column) and the select drops the product, so an
// Inf/NaN there never reaches the sum.
__device__ __forceinline__ void slot_fma(int c, double a, const double *x,
                                         double &acc)
{
    const double xv = x[c < 0 ? 0 : c];
    acc = fma(a, c >= 0 ? xv : 0.0, acc);
}

// This lane's share of its row: sum over its slots of a * x[col].  The
// matrix stream is loaded in batches of 8 slots (all column and value
// loads of a batch issued before any gather) so that each wavefront keeps
// ~12 KiB of the stream plus 512 gathers in flight.
template <int V>
__device__ __forceinline__ double group_lane_sum(const Group &g, int lane,
                                                 const double *__restrict__ val,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ x)
{
    typedef typename Slots<V>::D D;
    typedef typename Slots<V>::I I;
    constexpr int U = 8 / V;
    const int width = g.width_lt & 0xffffff;
    const long base = long(g.base64) * kWave;
    const D *pv = reinterpret_cast<const D *>(val + base) + lane;
    const I *pc = reinterpret_cast<const I *>(col + base) + lane;
    const int nch = width / V;
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
    for (; j + U <= nch; j += U) {
        I c[U];
        D a[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            c[u] = __builtin_nontemporal_load(pc + (j + u) * kWave);
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = __builtin_nontemporal_load(pv + (j + u) * kWave);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (V == 1) {
                slot_fma(c[u], a[u], x, (u & 1) ? acc1 : acc0);
            } else {
                slot_fma(c[u].x, a[u].x, x, acc0);
                slot_fma(c[u].y, a[u].y, x, acc1);
            }
        }
    }
    for (; j < nch; ++j) {
        const I c = __builtin_nontemporal_load(pc + j * kWave);
        const D a = __builtin_nontemporal_load(pv + j * kWave);
        if constexpr (V == 1) {
            slot_fma(c, a, x, acc0);
        } else {
            slot_fma(c.x, a.x, x, acc0);
            slot_fma(c.y, a.y, x, acc1);
        }
    }
    return acc0 + acc1;
}

__device__ __forceinline__ double row_reduce(double acc, int lt)
{
    for (int o = 1; o < (1 << lt); o <<= 1) acc += __shfl_xor(acc, o, kWave);
    return acc;
}

__device__ __forceinline__ Group load_group(const Group *groups, int g)
{
    Group d = groups[g];
    d.base64 = __builtin_amdgcn_readfirstlane(d.base64);
    d.row0 = __builtin_amdgcn_readfirstlane(d.row0);
    d.nrows = __builtin_amdgcn_readfirstlane(d.nrows);
    d.width_lt = __builtin_amdgcn_readfirstlane(d.width_lt);
    return d;
}

// ---------------------------------------------------------------- SpMV
// SCATTER: write y(yperm[row]) (caller numbering, the final re-mapping of
// the paper's K1), else y(row) in layout numbering (K1r).
template <int V, bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_spmv_f64(
    const Group *__restrict__ groups, int ngroups,
    const double *__restrict__ val, const int *__restrict__ col,
    const double *__restrict__ x, double *__restrict__ y,
    const int *__restrict__ yperm)
{
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int g = __builtin_amdgcn_readfirstlane(
        b * kWavesPerBlock + int(threadIdx.x >> 6));
    if (g >= ngroups) return;
    const int lane = threadIdx.x & (kWave - 1);
    const Group gd = load_group(groups, g);
    const int lt = gd.width_lt >> 24;
    double acc = row_reduce(group_lane_sum<V>(gd, lane, val, col, x), lt);
    const int r = lane >> lt;
    if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
        const int row = gd.row0 + r;
        y[SCATTER ? yperm[row] : row] = acc;
    }
}

// ------------------------------------------------- deterministic reductions
// Each block folds its NV values (wave butterflies, then the 4 waves in a
// fixed order), stores them at its logical index, and the last block to
// arrive sums all partials in index order.  Returns true in the last block,
// with the totals in `tot` (valid in every thread of that block).
template <int NV>
__device__ bool two_stage_sum(double (&v)[NV], double *partials, int nblk,
                              int b, uint32_t *counter, double (&tot)[NV])
{
    __shared__ double sh[NV][kWavesPerBlock];
    __shared__ int last;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int i = 0; i < kWavesPerBlock; ++i) s += sh[k][i];
            partials[k * nblk + b] = s;
        }
        __threadfence();
        const uint32_t t = atomicAdd(counter, 1u);
        last = (t == uint32_t(nblk - 1));
    }
    __syncthreads();
    if (!last) return false;
    // acquire: every other block's partial is visible after this fence;
    // plain loads so the whole column of partials is in flight at once
    __threadfence();
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        s[k] = 0.0;
        const double *pk = partials + k * nblk;
#pragma unroll 8
        for (int i = threadIdx.x; i < nblk; i += kBlock) s[k] += pk[i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double ws = wave_sum(s[k]);
        if (lane == 0) sh[k][w] = ws;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i) t += sh[k][i];
        tot[k] = t;
    }
    if (threadIdx.x == 0) atomicExch(counter, 0u);
    return true;
}

// ------------------------------------------------------------------- CG
// q = A p and gamma = p.q; the last block sets alpha = rho / gamma or flags
// a breakdown (gamma <= 0 or non-finite).
template <int V>
__global__ __launch_bounds__(kBlock) void k_cg_spmv_dot(
    const Group *__restrict__ groups, int ngroups,
    const double *__restrict__ val, const int *__restrict__ col,
    const double *__restrict__ p, double *__restrict__ q, CgScalars *sc,
    double *partials)
{
    if (sc->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int g = __builtin_amdgcn_readfirstlane(
        b * kWavesPerBlock + int(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    double v[1] = {0.0};
    if (g < ngroups) {
        const Group gd = load_group(groups, g);
        const int lt = gd.width_lt >> 24;
        const double acc =
            row_reduce(group_lane_sum<V>(gd, lane, val, col, p), lt);
        const int r = lane >> lt;
        if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
            const int row = gd.row0 + r;
            q[row] = acc;
            v[0] = p[row] * acc;
        }
    }
    double tot[1];
    if (two_stage_sum<1>(v, partials, gridDim.x, b, &sc->counter, tot) &&
        threadIdx.x == 0) {
        const double gamma = tot[0];
        sc->gamma = gamma;
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            sc->status = CG_BREAKDOWN;
            sc->done = 1;
        } else {
            sc->alpha = sc->rho / gamma;
        }
    }
}

// x += alpha p; r -= alpha q; z = D^-1 r; partial sums r.z and r.r.  The
// last block counts the iteration and either stops (recurrence residual
// met, breakdown, iteration limit) or sets beta and rho for the p update.
__global__ __launch_bounds__(kBlock) void k_cg_update(
    int n, double *__restrict__ x, double *__restrict__ r,
    const double *__restrict__ p, const double *__restrict__ q,
    const double *__restrict__ dinv, CgScalars *sc, double *partials)
{
    if (sc->done) return;
    const double alpha = sc->alpha;
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
         i += gridDim.x * kBlock) {
        const double ri = r[i] - alpha * q[i];
        x[i] += alpha * p[i];
        r[i] = ri;
        const double zi = dinv ? dinv[i] * ri : ri;
        v[0] += ri * zi;
        v[1] += ri * ri;
    }
    double tot[2];
    if (two_stage_sum<2>(v, partials, gridDim.x, blockIdx.x, &sc->counter,
                         tot) &&
        threadIdx.x == 0) {
        const double rz = tot[0], rr = tot[1];
        sc->iter += 1;
        sc->rr = rr;
        if (rr <= sc->tol2) {
            sc->status = CG_RECURRENCE_MET;
            sc->done = 1;
            return;
        }
        const double beta = rz / sc->rho;
        if (!isfinite(beta) || !isfinite(rr)) {
            sc->status = CG_BREAKDOWN;
            sc->done = 1;
            return;
        }
        sc->beta = beta;
        sc->rho = rz;
        if (sc->iter >= sc->maxit) {
            sc->status = CG_MAXIT;
            sc->done = 1;
        }
    }
}

// p = D^-1 r + beta p
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(
    int n, double *__restrict__ p, const double *__restrict__ r,
    const double *__restrict__ dinv, const CgScalars *sc)
{
    if (sc->done) return;
    const double beta = sc->beta;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
         i += gridDim.x * kBlock) {
        const double zi = dinv ? dinv[i] * r[i] : r[i];
        p[i] = zi + beta * p[i];
    }
}

// r = b - A x (x = 0: r = b) with z = D^-1 r; partials r.r, r.z, b.b.
// mode 0: start of a solve (sets rho, bnorm2, tol2, p = z, done when b = 0
//         or the initial guess already meets the tolerance);
// mode 1: convergence check -- stop when the true residual meets the
//         tolerance, else keep it (residual replacement) and set beta/rho;
// mode 2: measurement only (rr_true).
template <int V, bool X_ZERO>
__global__ __launch_bounds__(kBlock) void k_cg_residual(
    const Group *__restrict__ groups, int ngroups,
    const double *__restrict__ val, const int *__restrict__ col,
    const double *__restrict__ x, const double *__restrict__ bvec,
    double *__restrict__ r, double *__restrict__ p,
    const double *__restrict__ dinv, CgScalars *sc, double *partials,
    int mode, double rtol, int maxit)
{
    const int bl = xcd_remap(blockIdx.x, gridDim.x);
    const int g = __builtin_amdgcn_readfirstlane(
        bl * kWavesPerBlock + int(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    double v[3] = {0.0, 0.0, 0.0};
    if (g < ngroups) {
        const Group gd = load_group(groups, g);
        const int lt = gd.width_lt >> 24;
        double acc = 0.0;
        if (!X_ZERO)
            acc = row_reduce(group_lane_sum<V>(gd, lane, val, col, x), lt);
        const int rr = lane >> lt;
        if ((lane & ((1 << lt) - 1)) == 0 && rr < gd.nrows) {
            const int row = gd.row0 + rr;
            const double bi = bvec[row];
            const double ri = bi - acc;
            const double zi = dinv ? dinv[row] * ri : ri;
            r[row] = ri;
            if (mode == 0) p[row] = zi;
            v[0] = ri * ri;
            v[1] = ri * zi;
            v[2] = bi * bi;
        }
    }
    double tot[3];
    if (two_stage_sum<3>(v, partials, gridDim.x, bl, &sc->counter, tot) &&
        threadIdx.x == 0) {
        const double rr = tot[0], rz = tot[1], bb = tot[2];
        sc->rr_true = rr;
        if (mode == 0) {
            sc->bnorm2 = bb;
            sc->tol2 = rtol * rtol * bb;
            sc->rho = rz;
            sc->rr = rr;
            sc->iter = 0;
            sc->maxit = maxit;
            sc->replacements = 0;
            sc->status = CG_RUNNING;
            sc->done = 0;
            if (bb == 0.0 || rr <= sc->tol2) {
                sc->status = CG_CONVERGED;
                sc->done = 1;
            } else if (!isfinite(rr) || !isfinite(rz)) {
                sc->status = CG_BREAKDOWN;
                sc->done = 1;
            }
        } else if (mode == 1) {
            if (rr <= sc->tol2) {
                sc->status = CG_CONVERGED;
                sc->done = 1;
            } else {
                const double beta = rz / sc->rho;
                sc->replacements += 1;
                sc->rr = rr;
                if (!isfinite(beta)) {
                    sc->status = CG_BREAKDOWN;
                    sc->done = 1;
                } else {
                    sc->beta = beta;
                    sc->rho = rz;
                    sc->status = sc->iter >= sc->maxit ? CG_MAXIT : CG_RUNNING;
                    sc->done = sc->iter >= sc->maxit ? 1 : 0;
                }
            }
        }
    }
}

// Jacobi: dinv[row] = 1 / A(row,row) in layout numbering; counts rows whose
// diagonal is zero or non-finite in sc->pad[0].
template <int V>
__global__ __launch_bounds__(kBlock) void k_diag_inv(
    const Group *__restrict__ groups, int ngroups,
    const double *__restrict__ val, const int *__restrict__ col,
    double *__restrict__ dinv, CgScalars *sc)
{
    const int g = blockIdx.x * kWavesPerBlock + int(threadIdx.x >> 6);
    if (g >= ngroups) return;
    const int lane = threadIdx.x & (kWave - 1);
    const Group gd = load_group(groups, g);
    const int lt = gd.width_lt >> 24, width = gd.width_lt & 0xffffff;
    const int r = lane >> lt;
    const int row = gd.row0 + r;
    const long base = long(gd.base64) * kWave;
    double d = 0.0;
    for (int s = 0; s < width; ++s) {
        const long idx = base + long(s / V) * kWave * V + lane * V + s % V;
        if (col[idx] == row) d += val[idx];
    }
    d = row_reduce(d, lt);
    if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
        if (d == 0.0 || !isfinite(d)) atomicAdd(&sc->pad[0], 1);
        dinv[row] = 1.0 / d;
    }
}

// ---------------------------------------------------------- data movement
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return uint16_t((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__global__ __launch_bounds__(kBlock) void k_value_scatter(
    const double *__restrict__ vals, const int *__restrict__ map, long nnz,
    double *__restrict__ out, float *__restrict__ f32,
    uint16_t *__restrict__ bf16)
{
    for (long k = long(blockIdx.x) * kBlock + threadIdx.x; k < nnz;
         k += long(gridDim.x) * kBlock) {
        const double v = vals[k];
        const int s = map[k];
        out[s] = v;
        const float f = float(v);
        if (f32) f32[s] = f;
        if (bf16) bf16[s] = f32_to_bf16_rne(f);
    }
}

__global__ __launch_bounds__(kBlock) void k_gather(
    int n, const int *__restrict__ perm, const double *__restrict__ in,
    double *__restrict__ out)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
         i += gridDim.x * kBlock)
        out[i] = in[perm[i]];
}

__global__ __launch_bounds__(kBlock) void k_scatter(
    int n, const int *__restrict__ perm, const double *__restrict__ in,
    double *__restrict__ out)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
         i += gridDim.x * kBlock)
        out[perm[i]] = in[i];
}

int vec_blocks(long n)
{
    long b = (n + kBlock - 1) / kBlock;
    if (b > kVecBlocks) b = kVecBlocks;
    return b < 1 ? 1 : int(b);
}

int spmv_blocks(int ngroups)
{
    return (ngroups + kWavesPerBlock - 1) / kWavesPerBlock;
}

}  // namespace

// --------------------------------------------------------------- launchers
hipError_t launch_value_scatter(const double *vals, const int32_t *map,
                                int64_t nnz, double *slot_val, float *f32,
                                uint16_t *bf16, hipStream_t s)
{
    if (nnz == 0) return hipSuccess;
    long blocks = (nnz + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_value_scatter, dim3(unsigned(blocks)), dim3(kBlock),
                       0, s, vals, map, long(nnz), slot_val, f32, bf16);
    return hipGetLastError();
}

hipError_t launch_gather(int32_t n, const int32_t *perm, const double *in,
                         double *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n,
                       perm, in, out);
    return hipGetLastError();
}

hipError_t launch_scatter(int32_t n, const int32_t *perm, const double *in,
                          double *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n,
                       perm, in, out);
    return hipGetLastError();
}

// Instantiate F<V> for the matrix's slot vector width.
#define FS_LAUNCH_V(A, KERNEL, grid, ...)                                     \
    do {                                                                    \
        if ((A)->host.vec == 1)                                             \
            hipLaunchKernelGGL(KERNEL<1>, grid, dim3(kBlock), 0, __VA_ARGS__); \
        else                                                                \
            hipLaunchKernelGGL(KERNEL<2>, grid, dim3(kBlock), 0, __VA_ARGS__); \
    } while (0)

template <int V> struct SpmvScatter {
    template <bool S> static void go(const fs_csr *A, const double *x,
                                     double *y, const int32_t *yperm,
                                     hipStream_t s)
    {
        hipLaunchKernelGGL((k_spmv_f64<V, S>), dim3(spmv_blocks(A->n_groups)),
                           dim3(kBlock), 0, s, A->d_groups, A->n_groups,
                           A->d_val, A->d_col, x, y, yperm);
    }
};

hipError_t launch_spmv_f64(const fs_csr *A, const double *x, double *y,
                           const int32_t *yperm, hipStream_t s)
{
    if (A->n_groups == 0) return hipSuccess;
    if (A->host.vec == 1) {
        if (yperm) SpmvScatter<1>::go<true>(A, x, y, yperm, s);
        else SpmvScatter<1>::go<false>(A, x, y, yperm, s);
    } else {
        if (yperm) SpmvScatter<2>::go<true>(A, x, y, yperm, s);
        else SpmvScatter<2>::go<false>(A, x, y, yperm, s);
    }
    return hipGetLastError();
}

int32_t cg_partials_needed(const fs_csr *A)
{
    int32_t a = 3 * spmv_blocks(A->n_groups);
    int32_t b = 2 * vec_blocks(A->n_rows);
    return a > b ? a : b;
}

hipError_t launch_cg_spmv_dot(const fs_csr *A, CgWork &w, hipStream_t s)
{
    FS_LAUNCH_V(A, k_cg_spmv_dot, dim3(spmv_blocks(A->n_groups)), s,
                A->d_groups, A->n_groups, A->d_val, A->d_col, w.p, w.q, w.sc,
                w.partials);
    return hipGetLastError();
}

hipError_t launch_cg_update(CgWork &w, int32_t precond, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update, dim3(vec_blocks(w.n)), dim3(kBlock), 0,
                       s, w.n, w.x, w.r, w.p, w.q,
                       precond ? w.dinv : nullptr, w.sc, w.partials);
    return hipGetLastError();
}

hipError_t launch_cg_pupdate(CgWork &w, int32_t precond, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_pupdate, dim3(vec_blocks(w.n)), dim3(kBlock), 0,
                       s, w.n, w.p, w.r, precond ? w.dinv : nullptr, w.sc);
    return hipGetLastError();
}

template <int V> struct Residual {
    template <bool XZ> static void go(const fs_csr *A, CgWork &w,
                                      const double *dinv, int32_t mode,
                                      double rtol, int32_t maxit,
                                      hipStream_t s)
    {
        hipLaunchKernelGGL((k_cg_residual<V, XZ>),
                           dim3(spmv_blocks(A->n_groups)), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, A->d_col, w.x,
                           w.b, w.r, w.p, dinv, w.sc, w.partials, mode, rtol,
                           maxit);
    }
};

hipError_t launch_cg_residual(const fs_csr *A, CgWork &w, int32_t precond,
                              int32_t mode, double rtol, int32_t maxit,
                              int32_t x_is_zero, hipStream_t s)
{
    const double *dinv = precond ? w.dinv : nullptr;
    if (A->host.vec == 1) {
        if (x_is_zero) Residual<1>::go<true>(A, w, dinv, mode, rtol, maxit, s);
        else Residual<1>::go<false>(A, w, dinv, mode, rtol, maxit, s);
    } else {
        if (x_is_zero) Residual<2>::go<true>(A, w, dinv, mode, rtol, maxit, s);
        else Residual<2>::go<false>(A, w, dinv, mode, rtol, maxit, s);
    }
    return hipGetLastError();
}

hipError_t launch_diag_inv(const fs_csr *A, double *dinv, CgScalars *sc,
                           hipStream_t s)
{
    if (A->n_groups == 0) return hipSuccess;
    FS_LAUNCH_V(A, k_diag_inv, dim3(spmv_blocks(A->n_groups)), s,
                A->d_groups, A->n_groups, A->d_val, A->d_col, dinv, sc);
    return hipGetLastError();
}

}  // namespace fs
