// Device side of the layout build: the phases that touch every non-zero
// (column range check, bandwidth sums, slot assignment with the
// CSR-position -> slot map, 16-bit column offsets).  The row order and the
// row groups come from the host (they need only the row lengths, or the
// graph for reverse Cuthill-McKee); the results are the same arrays the
// host builder writes, bit for bit.
//
// Paper: section "Cost of Reordering Matrix Values" -- the layout's value
// map comes from one scan of the pattern, after which every value refresh is
// a device scatter; here that scan runs on the device as well.
#include "device.h"

namespace fs {
namespace {

// Smallest CSR position whose column lies outside [0, n_cols).
__global__ __launch_bounds__(kBlock) void k_check_cols(
    const int *__restrict__ col, long nnz, int n_cols,
    unsigned long long *__restrict__ first)
{
    const long stride = long(gridDim.x) * kBlock;
    for (long k = long(blockIdx.x) * kBlock + threadIdx.x; k < nnz;
         k += stride) {
        const int c = col[k];
        if (c < 0 || c >= n_cols) atomicMin(first, (unsigned long long)k);
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sums of |i - c| and |iperm[i] - iperm[c]| over the entries (i, c): 16
// lanes per row (four rows per wave in flight), the lanes striding over the
// row's entries; the block's sums meet in LDS and go out as one pair of
// atomics (atomics on one address serialise, so a grid of at most
// kBandBlocks keeps them few).  Integer sums, so the order of the additions
// does not matter.
constexpr int kBandLanes = 16;
constexpr int kBandBlocks = 2048;

__global__ __launch_bounds__(kBlock) void k_band(
    int n, const int *__restrict__ rowptr, const int *__restrict__ col,
    const int *__restrict__ iperm, unsigned long long *__restrict__ sums)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane & (kBandLanes - 1);
    const long first = (long(blockIdx.x) * kBlock + threadIdx.x) / kBandLanes;
    const long stride = long(gridDim.x) * kBlock / kBandLanes;
    unsigned long long s0 = 0, s1 = 0;
    for (long i = first; i < n; i += stride) {
        const int k0 = rowptr[i], k1 = rowptr[i + 1];
        const long ri = iperm[i];
        for (int k = k0 + sub; k < k1; k += kBandLanes) {
            const int c = col[k];
            const long d0 = i - c, d1 = ri - iperm[c];
            s0 += (unsigned long long)(d0 < 0 ? -d0 : d0);
            s1 += (unsigned long long)(d1 < 0 ? -d1 : d1);
        }
    }
    __shared__ unsigned long long part[2][kWavesPerBlock];
    s0 = wave_sum_u64(s0);
    s1 = wave_sum_u64(s1);
    const int w = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][w] = s0;
        part[1][w] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long t = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) t += part[threadIdx.x][i];
        atomicAdd(sums + threadIdx.x, t);
    }
}

__device__ __forceinline__ int layout_col(const int *__restrict__ col,
                                          const int *__restrict__ iperm,
                                          int k)
{
    const int c = col[k];
    return iperm ? iperm[c] : c;
}

// Slot assignment, one wave per row group.  A row's entries are ranked by
// their (relabelled) column: entry e of rank m goes to lane
// row_in_group * T + m % T, slot m / T of that lane, i.e. element
// base + (s / V) * 64 * V + lane * V + s % V (the column-interleaved order
// of sections "ELL-WARP" and "ELL-WARP v2 (K2)", with the columns sorted
// as in "K1rs").  Lanes hold up to 64 entries of the row; each counts the
// smaller columns over the whole row through cross-lane reads, so a row of
// length L costs L * ceil(L / 64) steps.  An entry whose column repeats an
// earlier entry of its row is a duplicate: the smallest such CSR position
// is reported through *dup.  The group's smallest and largest column go to
// lohi (0, -1 for a group without entries).
__global__ __launch_bounds__(kBlock) void k_assign_slots(
    const Group *__restrict__ groups, int ngroups, int V,
    const int *__restrict__ perm, const int *__restrict__ iperm,
    const int *__restrict__ rowptr, const int *__restrict__ col,
    int *__restrict__ slot_col, int *__restrict__ map,
    int2 *__restrict__ lohi, unsigned long long *__restrict__ dup)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w0 = __builtin_amdgcn_readfirstlane(
        int(blockIdx.x) * kWavesPerBlock + int(threadIdx.x >> 6));
    const int nw = gridDim.x * kWavesPerBlock;
    for (int g = w0; g < ngroups; g += nw) {
        const Group G = load_group(gbl(groups), g);
        const int lt = G.width_lt >> 24, T = 1 << lt;
        const long base = long(G.base64) * kWave;
        int mn = INT_MAX, mx = -1;
        for (int rr = 0; rr < G.nrows; ++rr) {
            const int orow = perm[G.row0 + rr];
            const int k0 = __builtin_amdgcn_readfirstlane(rowptr[orow]);
            const int len =
                __builtin_amdgcn_readfirstlane(rowptr[orow + 1]) - k0;
            for (int e0 = 0; e0 < len; e0 += kWave) {
                const int e = e0 + lane;
                const int c = e < len ? layout_col(col, iperm, k0 + e) : INT_MAX;
                int rank = 0;
                bool rep = false;
                for (int f0 = 0; f0 < len; f0 += kWave) {
                    int cf_lane = c;
                    if (f0 != e0) {
                        const int f = f0 + lane;
                        cf_lane = f < len ? layout_col(col, iperm, k0 + f)
                                          : INT_MAX;
                    }
                    const int nf = min(kWave, len - f0);
                    for (int t = 0; t < nf; ++t) {
                        const int cf = __builtin_amdgcn_readlane(cf_lane, t);
                        rank += cf < c ? 1 : 0;
                        rep = rep || (cf == c && f0 + t < e);
                    }
                }
                if (e < len) {
                    const int ln = rr * T + (rank & (T - 1));
                    const int s = rank >> lt;
                    const long idx = base + long(s / V) * kWave * V +
                                     long(ln) * V + s % V;
                    slot_col[idx] = c;
                    map[k0 + e] = int(idx);
                    mn = min(mn, c);
                    mx = max(mx, c);
                    if (rep) atomicMin(dup, (unsigned long long)(k0 + e));
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, __shfl_xor(mn, o, kWave));
            mx = max(mx, __shfl_xor(mx, o, kWave));
        }
        if (lane == 0) lohi[g] = make_int2(mx < 0 ? 0 : mn, mx);
    }
}

// 16-bit column offsets from each group's smallest column (0xffff marks
// padding), one wave per group over its whole slot region.
__global__ __launch_bounds__(kBlock) void k_offsets16(
    const Group *__restrict__ groups, int ngroups,
    const int *__restrict__ slot_col, const int2 *__restrict__ lohi,
    uint16_t *__restrict__ col16, int *__restrict__ gbase)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w0 = __builtin_amdgcn_readfirstlane(
        int(blockIdx.x) * kWavesPerBlock + int(threadIdx.x >> 6));
    const int nw = gridDim.x * kWavesPerBlock;
    for (int g = w0; g < ngroups; g += nw) {
        const Group G = load_group(gbl(groups), g);
        const long base = long(G.base64) * kWave;
        const long region = long(G.width_lt & 0xffffff) * kWave;
        const int lo = lohi[g].x;
        for (long t = lane; t < region; t += kWave) {
            const int c = slot_col[base + t];
            col16[base + t] = c < 0 ? uint16_t(0xffff) : uint16_t(c - lo);
        }
        if (lane == 0) gbase[g] = lo;
    }
}

// Inverse of the CSR-position -> slot map: imap[map[k]] = k (padding slots
// keep the -1 they were filled with).
__global__ __launch_bounds__(kBlock) void k_inverse_map(
    const int *__restrict__ map, long nnz, int *__restrict__ imap)
{
    const long stride = long(gridDim.x) * kBlock;
    for (long k = long(blockIdx.x) * kBlock + threadIdx.x; k < nnz;
         k += stride)
        imap[map[k]] = int(k);
}

// Value refresh in slot order (paper: section "Cost of Reordering Matrix
// Values", the per-Newton-step reorder of the values into the layout): one
// workgroup per row group walks the group's slot region, slot s taking
// vals[imap[s]] (0 for padding).  The slot arrays are written in full
// coalesced lines; the CSR values are gathered, but a group's region only
// touches the CSR ranges of its own rows, which stay in the CU's cache
// while the workgroup walks it.  The FP32 / BF16 copies round as the
// scatter at creation does.
__global__ __launch_bounds__(kBlock) void k_value_refresh(
    const Group *__restrict__ groups, const int *__restrict__ imap,
    const double *__restrict__ vals, double *__restrict__ val,
    float *__restrict__ f32, uint16_t *__restrict__ bf16)
{
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const Group G = load_group(gbl(groups), g);
    const long base = long(G.base64) * kWave;
    const long end = base + long(G.width_lt & 0xffffff) * kWave;
    // U slots per thread at a time: all their positions are loaded, then
    // all their values gathered, then all stored, so each thread keeps U
    // independent gathers in flight instead of one dependent pair (config
    // 1: U = 4 / 8 / 16 take 195 / 178 / 160 us; with 16 a whole row group
    // of up to 4096 slots is one batch)
    constexpr int U = 16;
    for (long t0 = base + threadIdx.x; t0 < end; t0 += U * kBlock) {
        int k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long t = t0 + long(u) * kBlock;
            k[u] = t < end ? __builtin_nontemporal_load(imap + t) : -1;
        }
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = k[u] < 0 ? 0.0 : vals[k[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long t = t0 + long(u) * kBlock;
            if (t >= end) continue;
            const double v = a[u];
            // streamed out, so the slot arrays do not evict the rows' values
            __builtin_nontemporal_store(v, val + t);
            if (f32 || bf16) {
                const float f = float(v);
                if (f32) __builtin_nontemporal_store(f, f32 + t);
                if (bf16)
                    __builtin_nontemporal_store(f32_to_bf16_rne(f), bf16 + t);
            }
        }
    }
}

// Row starts and byte-wide positions for the refresh (one wavefront per row
// group): a row's entries fill exactly its lanes' non-padding slots, so
// the smallest CSR position among them is the row's start, and every slot
// stores its entry's offset from that start.  Rows hold at most 255
// entries (checked by the caller); 255 marks padding.
__global__ __launch_bounds__(kBlock) void k_refresh_rows(
    const Group *__restrict__ groups, int ngroups, int vec,
    const int *__restrict__ imap, uint8_t *__restrict__ jpos,
    int *__restrict__ rstart)
{
    const int g = int(blockIdx.x) * kWavesPerBlock + int(threadIdx.x >> 6);
    if (g >= ngroups) return;
    const int lane = threadIdx.x & (kWave - 1);
    const Group G = load_group(gbl(groups), g);
    const long base = long(G.base64) * kWave;
    const int nch = (G.width_lt & 0xffffff) / vec, lt = G.width_lt >> 24;
    int mn = 0x7fffffff;
    for (int j = 0; j < nch; ++j)
        for (int t = 0; t < vec; ++t) {
            const int k = imap[base + (long(j) * kWave + lane) * vec + t];
            if (k >= 0 && k < mn) mn = k;
        }
    for (int o = 1; o < (1 << lt); o <<= 1)
        mn = min(mn, __shfl_xor(mn, o, kWave));
    const int r = lane >> lt;
    if ((lane & ((1 << lt) - 1)) == 0 && r < G.nrows)
        rstart[G.row0 + r] = mn == 0x7fffffff ? 0 : mn;
    for (int j = 0; j < nch; ++j)
        for (int t = 0; t < vec; ++t) {
            const long i = base + (long(j) * kWave + lane) * vec + t;
            const int k = imap[i];
            jpos[i] = k < 0 ? uint8_t(255) : uint8_t(k - mn);
        }
}

// The refresh through row starts: the map read is one byte per slot
// instead of four.  Thread x of a group's workgroup takes the group's slots
// x, x + 256, ... -- always the same lane (256 is a multiple of 64 vec
// slots), so one row and one row start per thread.
__global__ __launch_bounds__(kBlock) void k_value_refresh_rows(
    const Group *__restrict__ groups, int vec,
    const uint8_t *__restrict__ jpos, const int *__restrict__ rstart,
    const double *__restrict__ vals, double *__restrict__ val,
    float *__restrict__ f32, uint16_t *__restrict__ bf16)
{
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const Group G = load_group(gbl(groups), g);
    const long base = long(G.base64) * kWave;
    const long end = base + long(G.width_lt & 0xffffff) * kWave;
    const int lt = G.width_lt >> 24;
    const int r = ((int(threadIdx.x) / vec) & (kWave - 1)) >> lt;
    const long rs = r < G.nrows ? long(rstart[G.row0 + r]) : 0;
    constexpr int U = 16;
    for (long t0 = base + threadIdx.x; t0 < end; t0 += U * kBlock) {
        int jp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long t = t0 + long(u) * kBlock;
            jp[u] = t < end ? int(__builtin_nontemporal_load(jpos + t)) : 255;
        }
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = jp[u] == 255 ? 0.0 : vals[rs + jp[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long t = t0 + long(u) * kBlock;
            if (t >= end) continue;
            const double v = a[u];
            __builtin_nontemporal_store(v, val + t);
            if (f32 || bf16) {
                const float f = float(v);
                if (f32) __builtin_nontemporal_store(f, f32 + t);
                if (bf16)
                    __builtin_nontemporal_store(f32_to_bf16_rne(f), bf16 + t);
            }
        }
    }
}

int wave_grid(long waves)
{
    const long b = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return int(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t launch_inverse_map(const int32_t *map, int64_t nnz, int32_t *imap,
                              hipStream_t s)
{
    if (nnz == 0) return hipSuccess;
    const long b = (nnz + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_inverse_map, dim3(unsigned(b > 8192 ? 8192 : b)),
                       dim3(kBlock), 0, s, map, long(nnz), imap);
    return hipGetLastError();
}

hipError_t launch_value_refresh(const Group *groups, int32_t ngroups,
                                const int32_t *imap, const double *vals,
                                double *val, float *f32, uint16_t *bf16,
                                hipStream_t s)
{
    if (ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_value_refresh, dim3(ngroups), dim3(kBlock), 0, s,
                       groups, imap, vals, val, f32, bf16);
    return hipGetLastError();
}

hipError_t launch_refresh_rows(const Group *groups, int32_t ngroups,
                               int32_t vec, const int32_t *imap,
                               uint8_t *jpos, int32_t *rstart, hipStream_t s)
{
    if (ngroups == 0) return hipSuccess;
    const int b = (ngroups + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_refresh_rows, dim3(b), dim3(kBlock), 0, s, groups,
                       ngroups, vec, imap, jpos, rstart);
    return hipGetLastError();
}

hipError_t launch_value_refresh_rows(const Group *groups, int32_t ngroups,
                                     int32_t vec, const uint8_t *jpos,
                                     const int32_t *rstart,
                                     const double *vals, double *val,
                                     float *f32, uint16_t *bf16,
                                     hipStream_t s)
{
    if (ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_value_refresh_rows, dim3(ngroups), dim3(kBlock), 0,
                       s, groups, vec, jpos, rstart, vals, val, f32, bf16);
    return hipGetLastError();
}

hipError_t launch_check_cols(const int32_t *col, int64_t nnz, int32_t n_cols,
                             unsigned long long *first, hipStream_t s)
{
    if (nnz == 0) return hipSuccess;
    const long b = (nnz + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_check_cols, dim3(unsigned(b > 8192 ? 8192 : b)),
                       dim3(kBlock), 0, s, col, long(nnz), n_cols, first);
    return hipGetLastError();
}

hipError_t launch_band(int32_t n, const int32_t *rowptr, const int32_t *col,
                       const int32_t *iperm, unsigned long long *sums,
                       hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const long b = (long(n) * kBandLanes + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_band, dim3(unsigned(b > kBandBlocks ? kBandBlocks : b)),
                       dim3(kBlock), 0, s, n, rowptr, col, iperm, sums);
    return hipGetLastError();
}

hipError_t launch_assign_slots(const Group *groups, int32_t ngroups,
                               int32_t vec, const int32_t *perm,
                               const int32_t *iperm, const int32_t *rowptr,
                               const int32_t *col, int32_t *slot_col,
                               int32_t *map, int2 *lohi,
                               unsigned long long *dup, hipStream_t s)
{
    if (ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_assign_slots, dim3(wave_grid(ngroups)), dim3(kBlock),
                       0, s, groups, ngroups, vec, perm, iperm, rowptr, col,
                       slot_col, map, lohi, dup);
    return hipGetLastError();
}

hipError_t launch_offsets16(const Group *groups, int32_t ngroups,
                            const int32_t *slot_col, const int2 *lohi,
                            uint16_t *col16, int32_t *gbase, hipStream_t s)
{
    if (ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_offsets16, dim3(wave_grid(ngroups)), dim3(kBlock), 0,
                       s, groups, ngroups, slot_col, lohi, col16, gbase);
    return hipGetLastError();
}

}  // namespace fs
