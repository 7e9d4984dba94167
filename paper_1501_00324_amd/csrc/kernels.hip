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
//    multiplies an Inf/NaN of x;
//  * when every group's columns span fewer than 65535, column indices are
//    stored as 16-bit offsets from a per-group base (NARROW): 10 instead of
//    12 bytes of matrix stream per slot.
// The CG iteration, multi-right-hand-side products and the low-precision
// products live in engine.hip.
#include <cmath>

#include "device.h"

namespace fs {
namespace {

// ---------------------------------------------------------------- SpMV
// SCATTER: write y(yperm[row]) (caller numbering, the final re-mapping of
// the paper's K1), else y(row) in layout numbering (K1r).  PIPE: the
// software-pipelined lane sum (two register sets, 4 wavefronts per SIMD),
// which pays when lanes own several 8-slot batches; matrices with short
// rows (a lane owning one or two batches) run the plain loop at 8
// wavefronts per SIMD -- measured: 3-D P1 Laplacian (15 entries per row)
// 27% and graded 2-D triangles (7 per row) 34% slower pipelined, the
// elasticity matrices (44-81 per row) 2-5% faster.
template <int V, bool SCATTER, bool NARROW, bool PIPE>
__global__ __launch_bounds__(kBlock) void k_spmv_f64(
    const Group *__restrict__ groups, int ngroups,
    const double *__restrict__ val, const void *__restrict__ col,
    const int *__restrict__ gbase, const double *__restrict__ x,
    double *__restrict__ y, const int *__restrict__ yperm)
{
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int g = __builtin_amdgcn_readfirstlane(
        b * kWavesPerBlock + int(threadIdx.x >> 6));
    if (g >= ngroups) return;
    const int lane = threadIdx.x & (kWave - 1);
    const Group gd = load_group(gbl(groups), g);
    const int lt = gd.width_lt >> 24;
    const int gb = NARROW ? load_gbase(gbl(gbase), g) : 0;
    double acc;
    if constexpr (PIPE)
        acc = group_lane_sum<V, NARROW>(gd, lane, gbl(val), gbl(col), gb,
                                        gbl(x));
    else
        acc = group_lane_sum_plain<V, NARROW>(gd, lane, gbl(val), gbl(col),
                                              gb, gbl(x));
    acc = row_reduce(acc, lt);
    const int r = lane >> lt;
    if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
        const int row = gd.row0 + r;
        y[SCATTER ? yperm[row] : row] = acc;
    }
}

// ---------------------------------------------------------- data movement
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

__global__ __launch_bounds__(kBlock) void k_value_gather(
    const double *__restrict__ slot_val, const int *__restrict__ map,
    long nnz, double *__restrict__ vals)
{
    for (long k = long(blockIdx.x) * kBlock + threadIdx.x; k < nnz;
         k += long(gridDim.x) * kBlock)
        vals[k] = slot_val[map[k]];
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

hipError_t launch_value_gather(const double *slot_val, const int32_t *map,
                               int64_t nnz, double *vals, hipStream_t s)
{
    if (nnz == 0) return hipSuccess;
    long blocks = (nnz + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_value_gather, dim3(unsigned(blocks)), dim3(kBlock),
                       0, s, slot_val, map, long(nnz), vals);
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

namespace {

template <int V, bool S, bool N>
void spmv_go(const fs_csr *A, const double *x, double *y,
             const int32_t *yperm, hipStream_t s)
{
    const void *col = N ? static_cast<const void *>(A->d_col16)
                        : static_cast<const void *>(A->d_col);
    if (A->pipe_product)
        hipLaunchKernelGGL((k_spmv_f64<V, S, N, true>),
                           dim3(spmv_blocks(A->n_groups)), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, col,
                           A->d_gbase, x, y, yperm);
    else
        hipLaunchKernelGGL((k_spmv_f64<V, S, N, false>),
                           dim3(spmv_blocks(A->n_groups)), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, col,
                           A->d_gbase, x, y, yperm);
}

template <int V>
void spmv_v(const fs_csr *A, const double *x, double *y, const int32_t *yperm,
            hipStream_t s)
{
    const bool n = A->d_col16 != nullptr;
    if (yperm) {
        if (n) spmv_go<V, true, true>(A, x, y, yperm, s);
        else spmv_go<V, true, false>(A, x, y, yperm, s);
    } else {
        if (n) spmv_go<V, false, true>(A, x, y, yperm, s);
        else spmv_go<V, false, false>(A, x, y, yperm, s);
    }
}

}  // namespace

hipError_t launch_spmv_f64(const fs_csr *A, const double *x, double *y,
                           const int32_t *yperm, hipStream_t s)
{
    if (A->n_groups == 0) return hipSuccess;
    if (A->host.vec == 1) spmv_v<1>(A, x, y, yperm, s);
    else spmv_v<2>(A, x, y, yperm, s);
    return hipGetLastError();
}

}  // namespace fs
