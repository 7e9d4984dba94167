// Device helpers shared by the kernel translation units: slot loads, row
// reductions and XCD-aware block numbering.  Everything has internal
// linkage.
#pragma once

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
            slot_fma(c, a, x, (j & 1) ? acc1 : acc0);
        } else {
            slot_fma(c.x, a.x, x, acc0);
            slot_fma(c.y, a.y, x, acc1);
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

__device__ __forceinline__ Group load_group(const Group *groups, int g)
{
    Group d = groups[g];
    d.base64 = __builtin_amdgcn_readfirstlane(d.base64);
    d.row0 = __builtin_amdgcn_readfirstlane(d.row0);
    d.nrows = __builtin_amdgcn_readfirstlane(d.nrows);
    d.width_lt = __builtin_amdgcn_readfirstlane(d.width_lt);
    return d;
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
