// Device helpers shared by the kernel translation units: slot loads, row
// reductions and XCD-aware block numbering.  Everything has internal
// linkage.
#pragma once

#include <cmath>
#include <type_traits>

#include "internal.h"

namespace fs {
namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef int iv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef unsigned short us2 __attribute__((ext_vector_type(2)));

constexpr int kWavesPerBlock = kBlock / kWave;

// Pointers into global memory.  Most kernels find their pointers inside
// descriptor structs, where the compiler cannot tell that they address
// global memory and emits flat accesses (which also count against the LDS
// counter, so they serialise with cross-lane shuffles, and rule out scalar
// loads of uniform data); casting them to the global address space gives
// plain global and scalar loads.
#define FS_GLOBAL __attribute__((address_space(1)))
template <class T> using gptr = const FS_GLOBAL T *;
template <class T> using gmut = FS_GLOBAL T *;
template <class T> __device__ __forceinline__ gptr<T> gbl(const T *p)
{
    return (gptr<T>)p;
}
template <class T> __device__ __forceinline__ gmut<T> gblw(T *p)
{
    return (gmut<T>)p;
}
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

// Slot element types for V slots per load: values, 32-bit columns, 16-bit
// column offsets.
template <int V> struct Slots;
template <> struct Slots<1> { typedef double D; typedef int I; typedef uint16_t H; };
template <> struct Slots<2> { typedef dv2 D; typedef iv2 I; typedef us2 H; };

// Column index stream of a group: 32-bit layout columns (NARROW = false)
// or 16-bit offsets from the group's base column gb, 0xffff marking
// padding (NARROW = true).  Both decode to a layout column, -1 = padding.
template <int V, bool NARROW> struct ColStream {
    typedef typename std::conditional<NARROW, typename Slots<V>::H,
                                      typename Slots<V>::I>::type P;
    typedef typename std::conditional<NARROW, uint16_t, int32_t>::type E;
    gptr<P> p;
    int gb;
    __device__ __forceinline__ ColStream(gptr<void> col, long base, int lane,
                                         int gbase)
        : p(reinterpret_cast<gptr<P>>(static_cast<gptr<E>>(col) + base) +
            lane),
          gb(gbase)
    {
    }
    __device__ __forceinline__ P load(int j) const
    {
        return __builtin_nontemporal_load(p + long(j) * kWave);
    }
    __device__ __forceinline__ int get(const P &c, int t) const
    {
        int v;
        if constexpr (V == 1) v = int(c);
        else v = t ? int(c.y) : int(c.x);
        if constexpr (NARROW) return v == 0xffff ? -1 : gb + v;
        else return v;
    }
};

// Padded slots (column -1) read x[0] (always in bounds: a matrix with
// slots has at least one column) and the select drops the product, so an
// Inf/NaN there never reaches the sum.
__device__ __forceinline__ void slot_fma(int c, double a, gptr<double> x,
                                         double &acc)
{
    const double xv = x[c < 0 ? 0 : c];
    acc = fma(a, c >= 0 ? xv : 0.0, acc);
}

// This lane's share of its row: sum over its slots of a * x[col].  The
// matrix stream is read in batches of 8 slots (a batch's column and value
// loads are issued together) and software-pipelined over two register sets:
// the gathers of batch b are issued first, then the stream loads of batch
// b + 1, then batch b's products consume the gathers.  Loads complete in
// issue order, so waiting for batch b's gathers leaves batch b + 1's values
// in flight, and a wavefront always has matrix stream outstanding (the
// plain order -- stream, gathers, products -- leaves the stream idle during
// every gather round).  The scheduling barriers keep the compiler from
// hoisting the next batch's loads above the gathers, which would make the
// gather wait cover them too.  The batches are taken in pairs (the two
// register sets alternate without copies, which would wait for the loads);
// an odd last batch and the slots past the last full batch follow.  The
// sums are formed in the same order as the unpipelined loop.  Costs
// registers: 4 wavefronts per SIMD instead of 8, measured 2.3-2.5% faster
// on the 0.42 GB and 1.9 GB elasticity matrices than the unpipelined loop at
// 8 wavefronts, and faster than this loop held to 6 wavefronts.
template <int V, bool NARROW>
__device__ __forceinline__ double group_lane_sum(const Group &g, int lane,
                                                 gptr<double> val,
                                                 gptr<void> col, int gb,
                                                 gptr<double> x)
{
    typedef typename Slots<V>::D D;
    typedef ColStream<V, NARROW> CS;
    typedef typename CS::P PI;
    constexpr int U = 8 / V;
    const int width = g.width_lt & 0xffffff;
    const long base = long(g.base64) * kWave;
    gptr<D> pv = reinterpret_cast<gptr<D>>(val + base) + lane;
    const CS cs(col, base, lane, gb);
    const int nch = width / V;
    const int nb = nch / U;              // full batches
    double acc0 = 0.0, acc1 = 0.0;
    auto load = [&](PI (&c)[U], D (&a)[U], int b) {
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cs.load(b * U + u);
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = __builtin_nontemporal_load(pv + (b * U + u) * kWave);
    };
    // padded slots (column -1) gather x[0] and the select drops them
    auto gather = [&](const PI (&c)[U], int (&cc)[U * V],
                      double (&xv)[U * V]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < V; ++t) cc[u * V + t] = cs.get(c[u], t);
#pragma unroll
        for (int i = 0; i < U * V; ++i) xv[i] = x[cc[i] < 0 ? 0 : cc[i]];
    };
    auto products = [&](const D (&a)[U], const int (&cc)[U * V],
                        const double (&xv)[U * V]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (V == 1) {
                double &acc = (u & 1) ? acc1 : acc0;
                acc = fma(a[u], cc[u] >= 0 ? xv[u] : 0.0, acc);
            } else {
                acc0 = fma(a[u].x, cc[2 * u] >= 0 ? xv[2 * u] : 0.0, acc0);
                acc1 = fma(a[u].y, cc[2 * u + 1] >= 0 ? xv[2 * u + 1] : 0.0,
                           acc1);
            }
        }
    };
    if (nb > 0) {
        PI c0[U], c1[U];
        D a0[U], a1[U];
        load(c0, a0, 0);
        int b = 0;
        for (; b + 2 <= nb; b += 2) {
            int cc[U * V];
            double xv[U * V];
            gather(c0, cc, xv);
            __builtin_amdgcn_sched_barrier(0);
            load(c1, a1, b + 1);
            __builtin_amdgcn_sched_barrier(0);
            products(a0, cc, xv);
            gather(c1, cc, xv);
            __builtin_amdgcn_sched_barrier(0);
            // the last pair reloads batch b + 1 (no branch in the loop)
            load(c0, a0, b + 2 < nb ? b + 2 : b + 1);
            __builtin_amdgcn_sched_barrier(0);
            products(a1, cc, xv);
        }
        if (b < nb) {                    // odd last batch, already loaded
            int cc[U * V];
            double xv[U * V];
            gather(c0, cc, xv);
            products(a0, cc, xv);
        }
    }
    for (int j = nb * U; j < nch; ++j) {
        const PI c = cs.load(j);
        const D a = __builtin_nontemporal_load(pv + j * kWave);
        if constexpr (V == 1) {
            slot_fma(cs.get(c, 0), a, x, (j & 1) ? acc1 : acc0);
        } else {
            slot_fma(cs.get(c, 0), a.x, x, acc0);
            slot_fma(cs.get(c, 1), a.y, x, acc1);
        }
    }
    return acc0 + acc1;
}

// The same sum without pipelining, in batches of B slots (one register
// set): for kernels whose register budget is already spent, such as the
// 1024-thread blocks of the persistent solve (128 registers per lane, where
// 16-slot batches fit and keep more loads in flight).  The order of the
// sums does not depend on B.
template <int V, bool NARROW, int B = 8>
__device__ __forceinline__ double group_lane_sum_plain(const Group &g,
                                                       int lane,
                                                       gptr<double> val,
                                                       gptr<void> col, int gb,
                                                       gptr<double> x)
{
    typedef typename Slots<V>::D D;
    typedef ColStream<V, NARROW> CS;
    constexpr int U = B / V;
    const int width = g.width_lt & 0xffffff;
    const long base = long(g.base64) * kWave;
    gptr<D> pv = reinterpret_cast<gptr<D>>(val + base) + lane;
    const CS cs(col, base, lane, gb);
    const int nch = width / V;
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
    for (; j + U <= nch; j += U) {
        typename CS::P c[U];
        D a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cs.load(j + u);
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = __builtin_nontemporal_load(pv + (j + u) * kWave);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (V == 1) {
                slot_fma(cs.get(c[u], 0), a[u], x, (u & 1) ? acc1 : acc0);
            } else {
                slot_fma(cs.get(c[u], 0), a[u].x, x, acc0);
                slot_fma(cs.get(c[u], 1), a[u].y, x, acc1);
            }
        }
    }
    for (; j < nch; ++j) {
        const typename CS::P c = cs.load(j);
        const D a = __builtin_nontemporal_load(pv + j * kWave);
        if constexpr (V == 1) {
            slot_fma(cs.get(c, 0), a, x, (j & 1) ? acc1 : acc0);
        } else {
            slot_fma(cs.get(c, 0), a.x, x, acc0);
            slot_fma(cs.get(c, 1), a.y, x, acc1);
        }
    }
    return acc0 + acc1;
}

// Sum over the T = 2^lt lanes of each row (lanes of a row are adjacent).
template <typename T>
__device__ __forceinline__ T row_reduce(T acc, int lt)
{
    for (int o = 1; o < (1 << lt); o <<= 1) acc += __shfl_xor(acc, o, kWave);
    return acc;
}

__device__ __forceinline__ Group load_group(gptr<Group> groups, int g)
{
    Group d;
    d.base64 = __builtin_amdgcn_readfirstlane(groups[g].base64);
    d.row0 = __builtin_amdgcn_readfirstlane(groups[g].row0);
    d.nrows = __builtin_amdgcn_readfirstlane(groups[g].nrows);
    d.width_lt = __builtin_amdgcn_readfirstlane(groups[g].width_lt);
    return d;
}

// Column base of group g for 16-bit column offsets (0 when there are none).
__device__ __forceinline__ int load_gbase(gptr<int32_t> gbase, int g)
{
    return gbase ? __builtin_amdgcn_readfirstlane(gbase[g]) : 0;
}

// float -> bfloat16, round to nearest even; NaN stays a (quiet) NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return uint16_t((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

inline int vec_blocks(long n)
{
    long b = (n + kBlock - 1) / kBlock;
    if (b > kVecBlocks) b = kVecBlocks;
    return b < 1 ? 1 : int(b);
}

inline int spmv_blocks(int ngroups)
{
    return (ngroups + kWavesPerBlock - 1) / kWavesPerBlock;
}


}  // namespace
}  // namespace fs
