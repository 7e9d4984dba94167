// Plain CSR product without a layout (CSR-vector: T lanes per row stride
// over the row's entries, shuffle reduction) -- the product a caller gets
// before any layout is built, and the reference point for the layout build's
// break-even count (section "Cost of Reordering Matrix Values": a reorder
// pays off after enough products).  Memory safe for any input: row bounds
// and column indices are clamped, so a malformed CSR gives wrong numbers,
// never an out-of-bounds access.
#include <type_traits>

#include "device.h"

namespace fs {
namespace {

template <int LT>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(
    int n, int ncols, long nnz, const int *__restrict__ rowptr,
    const int *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ x, double *__restrict__ y)
{
    constexpr int T = 1 << LT;
    const long t = long(blockIdx.x) * kBlock + threadIdx.x;
    const long row = t >> LT;
    const int l = int(t & (T - 1));
    double acc = 0.0;
    if (row < n && ncols > 0) {
        long b = rowptr[row], e = rowptr[row + 1];
        b = b < 0 ? 0 : (b > nnz ? nnz : b);
        e = e < b ? b : (e > nnz ? nnz : e);
        for (long k = b + l; k < e; k += T) {
            int c = col[k];
            c = c < 0 ? 0 : (c >= ncols ? ncols - 1 : c);
            acc = fma(val[k], x[c], acc);
        }
    }
    acc = row_reduce(acc, LT);
    if (row < n && l == 0) y[row] = acc;
}

}  // namespace

// Lanes per row: the largest power of two not above half the mean row
// length (two or more entries per lane on average), at most 64.
int32_t csr_lanes_log2(int32_t n_rows, int64_t nnz)
{
    const double mean = n_rows > 0 ? double(nnz) / n_rows : 0.0;
    int lt = 0;
    while (lt < 6 && double(4 << lt) <= mean) ++lt;
    return lt;
}

hipError_t launch_spmv_csr(int32_t n_rows, int32_t n_cols, int64_t nnz,
                           const int32_t *rowptr, const int32_t *col,
                           const double *val, const double *x, double *y,
                           hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    const int lt = csr_lanes_log2(n_rows, nnz);
    const long threads = long(n_rows) << lt;
    const dim3 g(unsigned((threads + kBlock - 1) / kBlock)), b(kBlock);
    auto go = [&](auto tag) {
        constexpr int L = decltype(tag)::value;
        hipLaunchKernelGGL(k_spmv_csr<L>, g, b, 0, s, n_rows, n_cols,
                           long(nnz), rowptr, col, val, x, y);
    };
    switch (lt) {
    case 0: go(std::integral_constant<int, 0>()); break;
    case 1: go(std::integral_constant<int, 1>()); break;
    case 2: go(std::integral_constant<int, 2>()); break;
    case 3: go(std::integral_constant<int, 3>()); break;
    case 4: go(std::integral_constant<int, 4>()); break;
    case 5: go(std::integral_constant<int, 5>()); break;
    default: go(std::integral_constant<int, 6>()); break;
    }
    return hipGetLastError();
}

}  // namespace fs

// ---------------------------------------------------------------------
// Read-bandwidth probe: every lane streams 16-byte non-temporal loads
// over the buffer and folds them into one value per block (written to
// sink, so the loads cannot be dropped).  The achievable streaming rate
// against which the products' rates can be read.
namespace fs {
namespace {

__global__ __launch_bounds__(kBlock) void k_read_probe(
    const dv2 *__restrict__ p, long n2, double *__restrict__ sink)
{
    double s = 0.0;
    for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < n2;
         i += long(gridDim.x) * kBlock) {
        const dv2 v = __builtin_nontemporal_load(p + i);
        s += v.x + v.y;
    }
    s = wave_sum(s);
    __shared__ double sh[kWavesPerBlock];
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += sh[w];
        sink[blockIdx.x] = t;
    }
}

}  // namespace

hipError_t launch_read_probe(const double *buf, int64_t n, double *sink,
                             int32_t blocks, hipStream_t s)
{
    if (n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<const dv2 *>(buf), long(n / 2), sink);
    return hipGetLastError();
}

}  // namespace fs
