// Batched FP64 products: m independent y_i = A_i x_i (caller numbering),
// a gather launch and a product launch per 56 matrices.  Small FEM
// matrices cannot fill 256 CUs on their own and pay the launch latency once
// per product; here every matrix owns a contiguous range of workgroups of
// one launch.  The per-matrix
// descriptors travel as kernel arguments, so a call allocates nothing,
// copies nothing to the device and can be captured in a graph.
//
//   k_gather_batch : x'_i = x_i(perm_i) for matrices whose columns were
//                    relabelled by the locality order (the K1r renumbering)
//   k_spmv_batch   : y_i(yperm_i[row]) = (A'_i x'_i)[row], one row group per
//                    wavefront, the same lane arithmetic as the single
//                    product (bitwise equal results)
#include "device.h"

namespace fs {
namespace {

struct GatherDesc {
    const int32_t *perm;
    const double *in;
    double *out;
    int32_t n, b0;                     // rows, first block of this matrix
};

struct ProdDesc {
    const Group *groups;
    const double *val;
    const void *col;                   // 32-bit columns or 16-bit offsets
    const int32_t *gbase;              // group bases of 16-bit offsets, or NULL
    const double *x;
    double *y;
    const int32_t *yperm;              // NULL: y in layout order
    int32_t ngroups, b0;
};

template <typename D> struct DescArgs {
    int32_t m, nblocks;
    D d[kBatchPerLaunch];
};

// Index of the member that owns block b (members sorted by b0, d[0].b0 = 0).
template <typename D>
__device__ __forceinline__ int owner_of(const DescArgs<D> &a, int b)
{
    int lo = 0, hi = a.m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.d[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_gather_batch(
    const DescArgs<GatherDesc> a)
{
    const int i = owner_of(a, int(blockIdx.x));
    const GatherDesc &g = a.d[i];
    const int r = (int(blockIdx.x) - g.b0) * kBlock + int(threadIdx.x);
    if (r < g.n) g.out[r] = g.in[g.perm[r]];
}

template <int V>
__global__ __launch_bounds__(kBlock) void k_spmv_batch(
    const DescArgs<ProdDesc> a)
{
    const int b = xcd_remap(int(blockIdx.x), int(gridDim.x));
    const int i = owner_of(a, b);
    const ProdDesc &p = a.d[i];
    const int g = __builtin_amdgcn_readfirstlane(
        (b - p.b0) * kWavesPerBlock + int(threadIdx.x >> 6));
    if (g >= p.ngroups) return;
    const int lane = threadIdx.x & (kWave - 1);
    const Group gd = load_group(gbl(p.groups), g);
    const int lt = gd.width_lt >> 24;
    const double acc =
        p.gbase ? row_reduce(group_lane_sum_plain<V, true>(
                                 gd, lane, gbl(p.val), gbl(p.col),
                                 load_gbase(gbl(p.gbase), g), gbl(p.x)),
                             lt)
                : row_reduce(group_lane_sum_plain<V, false>(
                                 gd, lane, gbl(p.val), gbl(p.col), 0,
                                 gbl(p.x)),
                             lt);
    const int r = lane >> lt;
    if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
        const int row = gd.row0 + r;
        p.y[p.yperm ? p.yperm[row] : row] = acc;
    }
}

}  // namespace

hipError_t launch_spmv_batch(int32_t m, const fs_csr *const *A,
                             const double *const *x, double *const *y,
                             hipStream_t s)
{
    auto gathered = [](const fs_csr *M) {
        return M->n_groups > 0 && !M->host.identity &&
               M->host.symmetric_relabel;
    };
    // Rounds of at most kBatchPerLaunch members in which no handle is
    // gathered twice (the gather target is the handle's own x buffer):
    // one gather launch, then one product launch per slot width.
    for (int32_t i0 = 0; i0 < m;) {
        int32_t i1 = i0;
        for (; i1 < m && i1 - i0 < kBatchPerLaunch; ++i1) {
            if (!gathered(A[i1])) continue;
            bool dup = false;
            for (int32_t j = i0; j < i1; ++j) dup |= A[j] == A[i1];
            if (dup) break;
        }
        DescArgs<GatherDesc> ga{};
        int32_t nb = 0;
        for (int32_t i = i0; i < i1; ++i) {
            const fs_csr *M = A[i];
            if (!gathered(M)) continue;
            GatherDesc &d = ga.d[ga.m++];
            d.perm = M->d_perm;
            d.in = x[i];
            d.out = M->d_xtmp;
            d.n = M->n_cols;
            d.b0 = nb;
            nb += (M->n_cols + kBlock - 1) / kBlock;
        }
        if (ga.m > 0) {
            ga.nblocks = nb;
            hipLaunchKernelGGL(k_gather_batch, dim3(nb), dim3(kBlock), 0, s,
                               ga);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        for (int32_t vec = 1; vec <= 2; ++vec) {
            DescArgs<ProdDesc> pa{};
            nb = 0;
            for (int32_t i = i0; i < i1; ++i) {
                const fs_csr *M = A[i];
                if (M->n_groups == 0 || M->host.vec != vec) continue;
                ProdDesc &d = pa.d[pa.m++];
                d.groups = M->d_groups;
                d.val = M->d_val;
                d.col = M->d_col16 ? static_cast<const void *>(M->d_col16)
                                   : static_cast<const void *>(M->d_col);
                d.gbase = M->d_col16 ? M->d_gbase : nullptr;
                d.x = gathered(M) ? M->d_xtmp : x[i];
                d.y = y[i];
                d.yperm = M->host.identity ? nullptr : M->d_perm;
                d.ngroups = M->n_groups;
                d.b0 = nb;
                nb += spmv_blocks(M->n_groups);
            }
            if (pa.m == 0) continue;
            pa.nblocks = nb;
            if (vec == 1)
                hipLaunchKernelGGL(k_spmv_batch<1>, dim3(nb), dim3(kBlock), 0,
                                   s, pa);
            else
                hipLaunchKernelGGL(k_spmv_batch<2>, dim3(nb), dim3(kBlock), 0,
                                   s, pa);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        i0 = i1;
    }
    return hipSuccess;
}

}  // namespace fs
