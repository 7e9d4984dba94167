// Finite-element assembly as a sum-only product (paper: section
// "Description of Current GPU Methods", assembly of the global tangent
// matrix and residual as an SpMV with a vector of ones whose
// multiplications are dropped).  One lane owns one output entry and adds its
// element contributions in ascending order, so the result is bitwise the
// sequential element-by-element sum.  The index lists of a wavefront's 64
// entries are stored column-interleaved (one coalesced 256-byte load per
// step), tasks inside a window of output positions are ordered by
// contribution count so the lists of one wavefront have nearly equal length,
// and the element values are gathered through the cache hierarchy (a line
// of an element matrix serves neighbouring rows of the same node).
#include "device.h"

namespace fs {
namespace {

__global__ __launch_bounds__(kBlock) void k_assemble(
    const int2 *__restrict__ waves, int nwaves, long ntasks,
    const int *__restrict__ tpos, const int *__restrict__ aidx,
    const double *__restrict__ in, double *__restrict__ out,
    float *__restrict__ f32, uint16_t *__restrict__ bf16)
{
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int w = __builtin_amdgcn_readfirstlane(
        b * kWavesPerBlock + int(threadIdx.x >> 6));
    if (w >= nwaves) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int2 wd = waves[w];
    const int base64 = __builtin_amdgcn_readfirstlane(wd.x);
    const int width = __builtin_amdgcn_readfirstlane(wd.y);
    const int *p = aidx + long(base64) * kWave + lane;
    // padding entries (-1) come after a lane's real ones; they read in[0]
    // (present whenever width > 0) and add +0.0, which leaves a sum that
    // started from +0.0 unchanged
    constexpr int U = 8;
    double acc = 0.0;
    int j = 0;
    for (; j + U <= width; j += U) {
        int c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            c[u] = __builtin_nontemporal_load(p + long(j + u) * kWave);
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = in[c[u] < 0 ? 0 : c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = c[u] >= 0 ? v[u] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    for (; j < width; ++j) {
        const int c = __builtin_nontemporal_load(p + long(j) * kWave);
        const double v = in[c < 0 ? 0 : c];
        acc += c >= 0 ? v : 0.0;
    }
    const long t = long(w) * kWave + lane;
    const int q = t < ntasks ? tpos[t] : -1;    // -1: filler task
    if (q >= 0) {
        out[q] = acc;
        if (f32 || bf16) {
            const float f = float(acc);
            if (f32) f32[q] = f;
            if (bf16) bf16[q] = f32_to_bf16_rne(f);
        }
    }
}

// U consecutive steps of one batch: lane q*nde + b adds element value
// (ea_q * nde + b) into LDS slot off.  Every load is unconditional (indices
// clamped) and lanes without work add 0.0 into a private dummy slot past
// the group region, so the loop has no divergent branches.  With WR the
// first lane of row q also adds element vector entry ea_q into racc.  With
// ORD the element rows come from a buffer stored in the plan's own order
// (row rec * rows + q), so they are read contiguously and ea is not needed.
template <int U, bool WR, bool ORD>
__device__ __forceinline__ void lds_steps(long rec, int lane, int qc,
                                          bool act, int b, int nde, int rows,
                                          int dummy,
                                          const int *__restrict__ ea,
                                          const uint16_t *__restrict__ off,
                                          const double *__restrict__ ke,
                                          const double *__restrict__ re,
                                          double *acc, double &racc)
{
    int o[U], e[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        o[u] = int(__builtin_nontemporal_load(off + (rec + u) * kWave + lane));
    if constexpr (!ORD) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            e[u] = __builtin_nontemporal_load(ea + (rec + u) * rows + qc);
    }
    double w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if constexpr (ORD) {
            // rows of dropped element rows carry offsets 0xffff only
            const bool use = act && o[u] != 0xffff;
            v[u] = __builtin_nontemporal_load(
                ke + ((rec + u) * rows + qc) * nde + b);
            v[u] = use ? v[u] : 0.0;
            o[u] = use ? o[u] : dummy;
            continue;
        }
        const bool use = act && e[u] >= 0 && o[u] != 0xffff;
        v[u] = ke[long(use ? e[u] : 0) * nde + b];
        v[u] = use ? v[u] : 0.0;
        o[u] = use ? o[u] : dummy;
        if constexpr (WR) {
            const bool ur = act && b == 0 && e[u] >= 0;
            w[u] = re[ur ? e[u] : 0];
            w[u] = ur ? w[u] : 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[o[u]] += v[u];
    if constexpr (WR) {
#pragma unroll
        for (int u = 0; u < U; ++u) racc += w[u];
    }
}

// Row-group assembly: the block's row group accumulates in LDS.  A wave
// takes `rows` rows at a time; at step k lane q*nde + b adds element value
// (ea_q * nde + b) of row q's k-th element row ea_q, so the nde lanes of a
// row read nde consecutive doubles and every element row is read once.
// The adds into one slot come from steps of one row in ascending order
// (a slot belongs to one row and an element touches it once), and one
// wave's LDS accesses complete in program order, so each slot receives its
// contributions in ascending element order.  With WR the element vectors
// are assembled in the same pass: row q of a batch adds re[ea_q] at every
// step (again element order) and writes r at its caller row perm[row].
template <int U, bool WR, bool ORD>
__global__ __launch_bounds__(kBlock) void k_assemble_lds(
    const int4 *__restrict__ gdesc, const int2 *__restrict__ bdesc,
    const int *__restrict__ ea, const uint16_t *__restrict__ off, int nde,
    int rows, const double *__restrict__ ke, double *__restrict__ val,
    float *__restrict__ f32, uint16_t *__restrict__ bf16,
    const Group *__restrict__ groups, const int *__restrict__ perm,
    const double *__restrict__ re, double *__restrict__ r)
{
    extern __shared__ double acc[];   // group region + 64 dummy slots
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int4 gd = gdesc[g];
    const int region = gd.y * kWave;
    for (int t = threadIdx.x; t < region; t += kBlock) acc[t] = 0.0;
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane / nde, b = lane - q * nde;
    const bool act = q < rows;
    const int qc = act ? q : rows - 1;
    const int dummy = region + lane;
    for (int j = wave; j < gd.w; j += kWavesPerBlock) {
        const int2 bd = bdesc[gd.z + j];
        const long r0 = __builtin_amdgcn_readfirstlane(bd.x);
        const int K = __builtin_amdgcn_readfirstlane(bd.y);
        double racc = 0.0;
        int k = 0;
        for (; k + U <= K; k += U)
            lds_steps<U, WR, ORD>(r0 + k, lane, qc, act, b, nde, rows, dummy,
                                  ea, off, ke, re, acc, racc);
        for (; k < K; ++k)
            lds_steps<1, WR, ORD>(r0 + k, lane, qc, act, b, nde, rows, dummy,
                                  ea, off, ke, re, acc, racc);
        if constexpr (WR) {
            const int rr = j * rows + q;
            const Group lg = load_group(gbl(groups), g);
            if (act && b == 0 && rr < lg.nrows) r[perm[lg.row0 + rr]] = racc;
        }
    }
    __syncthreads();
    const long base = long(gd.x) * kWave;
    for (int t = threadIdx.x; t < region; t += kBlock) {
        const double a = acc[t];
        val[base + t] = a;
        if (f32 || bf16) {
            const float f = float(a);
            if (f32) f32[base + t] = f;
            if (bf16) bf16[base + t] = f32_to_bf16_rne(f);
        }
    }
}

}  // namespace

hipError_t launch_assemble_lds(const AsmLdsPlan &P, const double *ke,
                               double *val, float *f32, uint16_t *bf16,
                               const Group *groups, const int32_t *perm,
                               const double *re, double *r, bool ordered,
                               hipStream_t s)
{
    if (P.ngroups == 0) return hipSuccess;
    const size_t lds = size_t(P.region_max + kWave) * sizeof(double);
    const auto gd = reinterpret_cast<const int4 *>(P.d_gdesc);
    const auto bd = reinterpret_cast<const int2 *>(P.d_bdesc);
    if (ordered)
        hipLaunchKernelGGL((k_assemble_lds<8, false, true>), dim3(P.ngroups),
                           dim3(kBlock), lds, s, gd, bd, P.d_ea, P.d_off,
                           P.nde, P.rows, ke, val, f32, bf16, groups, perm,
                           nullptr, nullptr);
    else if (re)
        hipLaunchKernelGGL((k_assemble_lds<8, true, false>), dim3(P.ngroups),
                           dim3(kBlock), lds, s, gd, bd, P.d_ea, P.d_off,
                           P.nde, P.rows, ke, val, f32, bf16, groups, perm,
                           re, r);
    else
        hipLaunchKernelGGL((k_assemble_lds<8, false, false>),
                           dim3(P.ngroups), dim3(kBlock), lds, s, gd, bd,
                           P.d_ea, P.d_off, P.nde, P.rows, ke, val, f32, bf16,
                           groups, perm, re, r);
    return hipGetLastError();
}

hipError_t launch_assemble(const AsmPlan &P, const double *in, double *out,
                           float *f32, uint16_t *bf16, hipStream_t s)
{
    if (P.nwaves == 0) return hipSuccess;
    hipLaunchKernelGGL(k_assemble, dim3(spmv_blocks(P.nwaves)), dim3(kBlock),
                       0, s, reinterpret_cast<const int2 *>(P.d_waves),
                       P.nwaves, long(P.ntasks), P.d_tpos, P.d_aidx, in, out,
                       f32, bf16);
    return hipGetLastError();
}

}  // namespace fs
