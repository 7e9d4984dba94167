// Batched, multi-right-hand-side conjugate-gradient engine.
//
// One launch advances every running right-hand side of every system in a
// batch: systems own contiguous block ranges of the grid (a block -> system
// map), so a batch of many small systems costs the same three launches per
// iteration as one large system, and each system's arithmetic -- including
// its reduction trees, which depend only on its own size -- is identical
// whether it runs alone or in a batch.  A single solve is a batch of one
// system with one column.
//
// Per iteration (textbook preconditioned CG, the solver the paper runs
// around its SpMV; M = diag(A) or I; with one column the two finalize
// kernels are folded into the vector kernels, see k_update_fused):
//   k_spmm_dot   : Q = A P, per-block partials of p_c . q_c
//   k_fin_dot    : gamma_c, alpha_c = rho_c / gamma_c (breakdown check)
//   k_update     : x += alpha p, r -= alpha q, z = M^-1 r; partials of r.z
//                  and r.r
//   k_fin_update : stop a column when |r| <= rtol |b| (confirmed by the host
//                  against the true residual), else beta and rho
//   k_pupdate    : p = z + beta p
// Reductions are two kernels: per-block partials in a fixed order, then one
// block per (system, column) sums them in index order.  No atomics and no
// fences: kernel boundaries order everything, and the sums depend only on
// the system's own grid.
// Vectors are n x k row-major.  Systems share a launch only with systems of
// the same column-count class (k rounded up to 1, 2, 4, 8, 16), and the
// order of every sum is fixed by the class and the system's own shape, so a
// system's results do not depend on the other members of its batch.  With
// one column a lane gathers x for its own slots; with KM > 1 columns the
// lanes of a wavefront gather rows of X cooperatively (coop_group).
// The vector type ST is double for FP64 solves and float for the inner
// solve of mixed-precision refinement; values VT are double, float or bf16;
// every dot product is accumulated in double.
#include <algorithm>
#include <type_traits>

#include "device.h"

namespace fs {
namespace {

// Group-shaped grids give each wavefront one row group (as the plain
// product does) up to this many blocks; larger matrices give a block a
// contiguous run of groups.  A static split with several groups per
// wavefront loses ~20% to tail imbalance (measured on config 1).
constexpr int kMaxSpmvBlocks = 16384;

template <typename VT, int V> struct Pack;
template <> struct Pack<double, 1> { typedef double T; };
template <> struct Pack<double, 2> { typedef dv2 T; };
template <> struct Pack<float, 1> { typedef float T; };
template <> struct Pack<float, 2> { typedef fv2 T; };
template <> struct Pack<uint16_t, 1> { typedef uint16_t T; };
template <> struct Pack<uint16_t, 2> { typedef us2 T; };

template <typename ST> __device__ __forceinline__ ST widen(double v) { return ST(v); }
template <typename ST> __device__ __forceinline__ ST widen(float v) { return ST(v); }
template <typename ST> __device__ __forceinline__ ST widen(uint16_t h)
{
    return ST(__uint_as_float(uint32_t(h) << 16));
}

template <typename VT, typename ST, int V>
__device__ __forceinline__ void unpack(typename Pack<VT, V>::T a, ST (&o)[V])
{
    if constexpr (V == 1) {
        o[0] = widen<ST>(a);
    } else {
        o[0] = widen<ST>(a.x);
        o[1] = widen<ST>(a.y);
    }
}

// acc{0,1}[c] += a * X[col, c] over this lane's slots, even slots into
// acc0, odd slots into acc1.  Padded slots (col -1) read row 0 of X and
// drop the product through a select.
template <typename VT, typename ST, int V, int KM, bool N>
__device__ __forceinline__ void lane_sums(const Group &g, int lane,
                                          gptr<VT> val, gptr<void> col,
                                          int gb, gptr<ST> X, int k, long ldx,
                                          ST (&acc0)[KM], ST (&acc1)[KM])
{
    typedef typename Pack<VT, V>::T PV;
    typedef ColStream<V, N> CS;
    typedef typename CS::P PI;
    constexpr int U0 = KM == 1 ? 8 : (KM == 2 ? 4 : 2);
    constexpr int U = U0 / V > 0 ? U0 / V : 1;
    const int width = g.width_lt & 0xffffff;
    const long base = long(g.base64) * kWave;
    gptr<PV> pv = reinterpret_cast<gptr<PV>>(val + base) + lane;
    const CS cs(col, base, lane, gb);
    const int nch = width / V;
    auto slot = [&](int c, ST a, bool odd) {
        gptr<ST> xr = X + long(c < 0 ? 0 : c) * ldx;
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            if (KM == 1 || q < k) {
                const ST xv = xr[q];
                ST &acc = odd ? acc1[q] : acc0[q];
                acc = fma(a, c >= 0 ? xv : ST(0), acc);
            }
        }
    };
    int j = 0;
    for (; j + U <= nch; j += U) {
        PI c[U];
        PV a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cs.load(j + u);
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = __builtin_nontemporal_load(pv + (j + u) * kWave);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ST aa[V];
            unpack<VT, ST, V>(a[u], aa);
#pragma unroll
            for (int t = 0; t < V; ++t)
                slot(cs.get(c[u], t), aa[t], ((j + u) * V + t) & 1);
        }
    }
    for (; j < nch; ++j) {
        ST aa[V];
        const PI c = cs.load(j);
        unpack<VT, ST, V>(__builtin_nontemporal_load(pv + j * kWave), aa);
#pragma unroll
        for (int t = 0; t < V; ++t) slot(cs.get(c, t), aa[t], (j * V + t) & 1);
    }
}

// f(std::true_type) for 16-bit column offsets, else f(std::false_type);
// the flag is uniform over a system, so the branch is too.
template <class F>
__device__ __forceinline__ void with_narrow(bool narrow, F &&f)
{
    if (narrow) f(std::true_type());
    else f(std::false_type());
}

__device__ __forceinline__ bool any_running(const SysDesc &S)
{
    for (int c = 0; c < S.k; ++c)
        if (S.cs[c].status == CG_RUNNING) return true;
    return false;
}

// Fold NV per-thread values over the block (wave butterflies, then the
// waves in order) and store them as this block's partials.
template <int NV>
__device__ __forceinline__ void store_partials(double (&v)[NV], int nact,
                                               double *partials, int nblk,
                                               int b)
{
    __shared__ double sh[NV][kWavesPerBlock];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        if (j >= nact) continue;
        const double s = wave_sum(v[j]);
        if (lane == 0) sh[j][w] = s;
    }
    __syncthreads();
    if (int(threadIdx.x) < nact) {
        double s = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i) s += sh[threadIdx.x][i];
        partials[long(threadIdx.x) * nblk + b] = s;
    }
}

// Sum of partials[j * nblk + 0 .. nblk-1] for j < NJ, in index order
// (thread t takes t, t + 256, ...; then the block folds).  Valid in thread 0.
template <int NJ>
__device__ __forceinline__ void sum_partials(const double *partials, int nblk,
                                             int j0, double (&out)[NJ])
{
    __shared__ double sh[NJ][kWavesPerBlock];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    // loads are issued eight at a time (the sum keeps its index order; the
    // padding adds +0.0, which leaves a sum started at +0.0 unchanged)
    constexpr int U = 8;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const auto pj = gbl(partials + long(j0 + j) * nblk);
        double s = 0.0;
        for (int i0 = threadIdx.x; i0 < nblk; i0 += U * kBlock) {
            double a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * kBlock;
                a[u] = pj[i < nblk ? i : 0];
                a[u] = i < nblk ? a[u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s += a[u];
        }
        s = wave_sum(s);
        if (lane == 0) sh[j][w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        double t = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i) t += sh[j][i];
        out[j] = t;
    }
}

// Per-column block partials for column-split thread mappings: thread t
// carries column t % KM.  Lanes of equal column are folded with butterflies
// over the lane bits above log2(KM), the waves in order, and partial
// NVPC*c + j of this block is stored at partials[(NVPC*c + j) * nblk + b].
// With KM = 1 this is exactly store_partials.
template <int NVPC, int KM>
__device__ __forceinline__ void store_col_partials(double (&v)[NVPC], int k,
                                                   double *partials, int nblk,
                                                   int b)
{
    __shared__ double sh[NVPC][KM][kWavesPerBlock];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int j = 0; j < NVPC; ++j) {
        double s = v[j];
#pragma unroll
        for (int o = 32; o >= KM; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (lane < KM) sh[j][lane][w] = s;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NVPC * k) {
        const int c = t / NVPC, j = t % NVPC;
        double s = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i) s += sh[j][c][i];
        partials[long(t) * nblk + b] = s;
    }
}

// A slot's (value, column) pair as the wavefront shares it through LDS.
template <typename ST> struct SlotRec;
template <> struct SlotRec<double> { double a; int c, pad; };   // 16 bytes
template <> struct SlotRec<float> { float a; int c; };          // 8 bytes

// The block's broadcast buffers: two per wavefront of V * 64 records (one
// array per element type and slot width, shared by every caller in a
// kernel).
template <typename ST, int V> __device__ __forceinline__ SlotRec<ST> *coop_buffer()
{
    __shared__ SlotRec<ST> recs[kWavesPerBlock * 2 * V * kWave];
    return recs;
}

// Order this wavefront's LDS writes before its later LDS reads (and its
// reads before later writes): LDS operations of one wavefront execute in
// order, so only the compiler has to be kept from moving them.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Multi-column product of one row group with cooperative gathers (KM > 1).
// Lane L works on column q = L % KM for the slot pairs held by lanes
// p = r * (64/KM) + L / KM, rounds r = 0..KM-1: the matrix entry (column,
// value) of lane p is broadcast -- each lane writes its entries to a
// per-wavefront LDS buffer once, and every round is one LDS read that the
// KM lanes of a row share -- and 64/KM rows of X are read per instruction,
// each a contiguous run of KM values.  (A lane gathering its own row of X
// would touch 64 cache lines per instruction; broadcasting by cross-lane
// shuffles costs three permutes per round.)  Two buffers alternate, so the
// writes for the next slot load never wait for this one's reads.
// emit(row_in_group, q, value) is called once per (row, column < k).
template <typename VT, typename ST, int V, int KM, bool N, class Emit>
__device__ __forceinline__ void coop_group(const Group &g, int lane,
                                           gptr<VT> val, gptr<void> col,
                                           int gb, gptr<ST> X, int k,
                                           long ldx, Emit emit)
{
    static_assert(KM > 1, "single-column products use lane_sums");
    typedef typename Pack<VT, V>::T PV;
    typedef ColStream<V, N> CS;
    constexpr int R = kWave / KM;
    const int q = lane % KM, m = lane / KM;
    const int width = g.width_lt & 0xffffff;
    const long base = long(g.base64) * kWave;
    gptr<PV> pv = reinterpret_cast<gptr<PV>>(val + base) + lane;
    const CS cs(col, base, lane, gb);
    ST acc[KM];
#pragma unroll
    for (int r = 0; r < KM; ++r) acc[r] = ST(0);
    // columns q >= k read column 0 and drop it, so no load sits behind a
    // branch and a round's gathers are all in flight together
    const bool qok = q < k;
    const int qc = qok ? q : 0;
    constexpr int RB = KM < 8 ? KM : 8;      // rounds per batch of gathers
    const int nch = width / V;
    SlotRec<ST> *const recs = coop_buffer<ST, V>() +
                              int(threadIdx.x >> 6) * 2 * V * kWave;
    int buf = 0;
    // with few columns the next chunk's (column, value) loads are issued
    // before this chunk's gathers (k = 2: 23% faster); with 8 or 16 columns
    // the gathers dominate and the extra registers would spill
    constexpr bool PF = KM <= 4;
    typename CS::P cvn{};
    PV avn{};
    if (PF && nch > 0) {
        cvn = cs.load(0);
        avn = __builtin_nontemporal_load(pv);
    }
    for (int j = 0; j < nch; ++j) {
        int cc[V];
        ST aa[V];
        typename CS::P cv;
        PV av;
        if constexpr (PF) {
            cv = cvn;
            av = avn;
            if (j + 1 < nch) {
                cvn = cs.load(j + 1);
                avn = __builtin_nontemporal_load(pv + (j + 1) * kWave);
            }
        } else {
            cv = cs.load(j);
            av = __builtin_nontemporal_load(pv + j * kWave);
        }
#pragma unroll
        for (int t = 0; t < V; ++t) cc[t] = cs.get(cv, t);
        unpack<VT, ST, V>(av, aa);
        SlotRec<ST> *rb = recs + buf * V * kWave;
        buf ^= 1;
#pragma unroll
        for (int t = 0; t < V; ++t) {
            rb[t * kWave + lane].a = aa[t];
            rb[t * kWave + lane].c = cc[t];
        }
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < V; ++t) {
#pragma unroll
            for (int r0 = 0; r0 < KM; r0 += RB) {
                int sc[RB];
                ST sa[RB], xv[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const SlotRec<ST> &e = rb[t * kWave + (r0 + u) * R + m];
                    sc[u] = e.c;
                    sa[u] = e.a;
                }
#pragma unroll
                for (int u = 0; u < RB; ++u)
                    xv[u] = X[long(sc[u] < 0 ? 0 : sc[u]) * ldx + qc];
#pragma unroll
                for (int u = 0; u < RB; ++u)
                    acc[r0 + u] = fma(sa[u], (qok && sc[u] >= 0) ? xv[u] : ST(0),
                                      acc[r0 + u]);
                // keep the scheduler from hoisting the next batch's gathers
                // above this one (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    const int lt = g.width_lt >> 24, T = 1 << lt;
    if (T <= R) {
        // the T lanes of a row sit at consecutive m within one round
#pragma unroll
        for (int r = 0; r < KM; ++r)
            for (int o = KM; o < KM * T; o <<= 1)
                acc[r] += __shfl_xor(acc[r], o, kWave);
#pragma unroll
        for (int r = 0; r < KM; ++r) {
            const int rg = (r * R + m) >> lt;
            if ((m & (T - 1)) == 0 && rg < g.nrows && q < k) emit(rg, q, acc[r]);
        }
    } else {
        // a row spans T / R whole rounds
        const int rounds = T / R;
#pragma unroll
        for (int r = 0; r < KM; ++r)
#pragma unroll
            for (int o = KM; o < kWave; o <<= 1)
                acc[r] += __shfl_xor(acc[r], o, kWave);
#pragma unroll
        for (int s = 1; s < KM; s <<= 1)
            if (s < rounds) {
#pragma unroll
                for (int r = 0; r + s < KM; r += 2 * s) acc[r] += acc[r + s];
            }
#pragma unroll
        for (int r = 0; r < KM; ++r) {
            const int rg = (r * R) >> lt;
            if (r % rounds == 0 && m == 0 && rg < g.nrows && q < k)
                emit(rg, q, acc[r]);
        }
    }
}

// coop_group with two adjacent columns per lane: KM/2 lanes per gathered
// row, 128/KM rows per round, KM/2 rounds per slot, and 16-byte X loads.
// The texture address unit processes a gather instruction at a fixed rate of
// lanes per cycle whatever each lane loads, and the KM = 16 product is bound
// by it (counters: address unit busy 88% of the kernel); two columns per
// lane halve its gather instructions.  Every (row, column) sum is formed
// exactly as in coop_group (each slot lane's entries in order, then the same
// tree over a row's lanes), and the values are handed to the lanes that
// emit them in coop_group, so stores and p.q partials are bitwise
// coop_group's.  Needs k even (16-byte aligned X rows); used for KM >= 8
// (with fewer columns coop_group's early loads of the next slot win).
template <typename VT, int V, int KM, bool N, class Emit>
__device__ __forceinline__ void coop_group_pair(const Group &g, int lane,
                                                gptr<VT> val, gptr<void> col,
                                                int gb, gptr<double> X, int k,
                                                long ldx, Emit emit)
{
    static_assert(KM >= 4, "pairs need at least four columns");
    typedef typename Pack<VT, V>::T PV;
    typedef ColStream<V, N> CS;
    constexpr int H = KM / 2;
    constexpr int R = kWave / H;
    const int h = lane % H, m = lane / H;
    const int width = g.width_lt & 0xffffff;
    const long base = long(g.base64) * kWave;
    gptr<PV> pv = reinterpret_cast<gptr<PV>>(val + base) + lane;
    const CS cs(col, base, lane, gb);
    double acc0[H], acc1[H];
#pragma unroll
    for (int r = 0; r < H; ++r) acc0[r] = acc1[r] = 0.0;
    const bool hok = 2 * h < k;
    const int hc = hok ? 2 * h : 0;
    constexpr int RB = H < 8 ? H : 8;
    const int nch = width / V;
    SlotRec<double> *const recs = coop_buffer<double, V>() +
                                  int(threadIdx.x >> 6) * 2 * V * kWave;
    int buf = 0;
    for (int j = 0; j < nch; ++j) {
        int cc[V];
        double aa[V];
        const typename CS::P cv = cs.load(j);
        const PV av = __builtin_nontemporal_load(pv + j * kWave);
#pragma unroll
        for (int t = 0; t < V; ++t) cc[t] = cs.get(cv, t);
        unpack<VT, double, V>(av, aa);
        SlotRec<double> *rb = recs + buf * V * kWave;
        buf ^= 1;
#pragma unroll
        for (int t = 0; t < V; ++t) {
            rb[t * kWave + lane].a = aa[t];
            rb[t * kWave + lane].c = cc[t];
        }
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < V; ++t) {
#pragma unroll
            for (int r0 = 0; r0 < H; r0 += RB) {
                int sc[RB];
                double sa[RB];
                dv2 xv[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const SlotRec<double> &e = rb[t * kWave + (r0 + u) * R + m];
                    sc[u] = e.c;
                    sa[u] = e.a;
                }
#pragma unroll
                for (int u = 0; u < RB; ++u)
                    xv[u] = *reinterpret_cast<gptr<dv2>>(
                        X + long(sc[u] < 0 ? 0 : sc[u]) * ldx + hc);
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const bool ok = hok && sc[u] >= 0;
                    acc0[r0 + u] = fma(sa[u], ok ? xv[u].x : 0.0, acc0[r0 + u]);
                    acc1[r0 + u] = fma(sa[u], ok ? xv[u].y : 0.0, acc1[r0 + u]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    const int lt = g.width_lt >> 24, T = 1 << lt;
    // the tree over a row's lanes, as in coop_group
    if (T <= R) {
#pragma unroll
        for (int r = 0; r < H; ++r)
            for (int o = H; o < H * T; o <<= 1) {
                acc0[r] += __shfl_xor(acc0[r], o, kWave);
                acc1[r] += __shfl_xor(acc1[r], o, kWave);
            }
    } else {
        const int rounds = T / R;
#pragma unroll
        for (int r = 0; r < H; ++r)
#pragma unroll
            for (int o = H; o < kWave; o <<= 1) {
                acc0[r] += __shfl_xor(acc0[r], o, kWave);
                acc1[r] += __shfl_xor(acc1[r], o, kWave);
            }
#pragma unroll
        for (int s = 1; s < H; s <<= 1)
            if (s < rounds) {
#pragma unroll
                for (int r = 0; r + s < H; r += 2 * s) {
                    acc0[r] += acc0[r + s];
                    acc1[r] += acc1[r + s];
                }
            }
    }
    // hand every row's value to the lane that emits it in coop_group (lane
    // q + KM mo, round r holds rows r * RO + mo), so the stores and the
    // order of the p.q partials are exactly coop_group's: the value of
    // round r sits in round r / 2 here, in lane ((r % 2) RO + mo) H + q / 2
    constexpr int RO = kWave / KM;
    const int q = lane % KM, mo = lane / KM;
    double fin[KM];
#pragma unroll
    for (int r = 0; r < KM; ++r) {
        const int src = ((r & 1) * RO + mo) * H + (q >> 1);
        const double v0 = __shfl(acc0[r >> 1], src, kWave);
        const double v1 = __shfl(acc1[r >> 1], src, kWave);
        fin[r] = (q & 1) ? v1 : v0;
    }
    if (T <= RO) {
#pragma unroll
        for (int r = 0; r < KM; ++r) {
            const int rg = (r * RO + mo) >> lt;
            if ((mo & (T - 1)) == 0 && rg < g.nrows && q < k) emit(rg, q, fin[r]);
        }
    } else {
        const int rounds = T / RO;
#pragma unroll
        for (int r = 0; r < KM; ++r) {
            const int rg = (r * RO) >> lt;
            if (r % rounds == 0 && mo == 0 && rg < g.nrows && q < k)
                emit(rg, q, fin[r]);
        }
    }
}

// Occupancy floor (waves per SIMD) of the products in the CG iteration:
// the gathers are latency bound; KM = 1 holds 7 waves (at 8 the FP64
// product spills a register and the solve slows by 13%), KM = 8 and 16
// hold 4 (128 registers), except the float KM = 16 product, which needs
// more registers and keeps 3.
constexpr int spmm_dot_min_waves(int km, int st_bytes)
{
    return km == 16 && st_bytes == 4 ? 3 : km >= 8 ? 4 : km == 1 ? 7 : 1;
}

// Q = A P for every column with per-block partials of p_c . q_c.
template <typename VT, typename ST, int V, int KM>
__global__ __launch_bounds__(kBlock, spmm_dot_min_waves(KM, int(sizeof(ST)))) void k_spmm_dot(
    const SysDesc *__restrict__ sys, const int *__restrict__ smap)
{
    const int gb = xcd_remap(blockIdx.x, gridDim.x);
    const SysDesc &S = sys[smap[gb]];
    if (!any_running(S)) return;
    const int lb = gb - S.sb0, nb = S.snb, k = S.k;
    const auto val = gbl(static_cast<const VT *>(S.val));
    const auto P = gbl(static_cast<const ST *>(S.p));
    const auto Q = gblw(static_cast<ST *>(S.q));
    const auto cst = gbl(S.cstream);
    const int g0 = int(long(lb) * S.ngroups / nb);
    const int g1 = int(long(lb + 1) * S.ngroups / nb);
    const int lane = threadIdx.x & (kWave - 1);
    double dot[1] = {0.0};
    with_narrow(S.gbase != nullptr, [&](auto nt) {
        constexpr bool N = decltype(nt)::value;
        for (int g = g0 + int(threadIdx.x >> 6); g < g1; g += kWavesPerBlock) {
            const Group gd =
                load_group(gbl(S.groups), __builtin_amdgcn_readfirstlane(g));
            const int gb = N ? load_gbase(gbl(S.gbase), g) : 0;
            if constexpr (KM == 1) {
                const int lt = gd.width_lt >> 24, r = lane >> lt;
                const bool own = (lane & ((1 << lt) - 1)) == 0 && r < gd.nrows;
                const long row = gd.row0 + (r < gd.nrows ? r : 0);
                const ST pr = P[row];          // early, off the tail
                ST a0[1] = {ST(0)}, a1[1] = {ST(0)};
                lane_sums<VT, ST, V, 1, N>(gd, lane, val, cst, gb, P, 1, 1,
                                           a0, a1);
                const ST v = row_reduce(a0[0] + a1[0], lt);
                if (own) {
                    Q[row] = v;
                    dot[0] += double(pr) * double(v);
                }
            } else {
                auto emit = [&](int rg, int q, ST v) {
                    const long e = long(gd.row0 + rg) * k + q;
                    Q[e] = v;
                    dot[0] += double(P[e]) * double(v);
                };
                // engine vectors are n x k with rows of k values: 16-byte
                // aligned when k is even
                if constexpr (KM >= 8 && std::is_same<ST, double>::value) {
                    if ((k & 1) == 0)
                        coop_group_pair<VT, V, KM, N>(gd, lane, val, cst, gb,
                                                      P, k, k, emit);
                    else
                        coop_group<VT, ST, V, KM, N>(gd, lane, val, cst, gb,
                                                     P, k, k, emit);
                } else {
                    coop_group<VT, ST, V, KM, N>(gd, lane, val, cst, gb, P, k,
                                                 k, emit);
                }
            }
        }
    });
    store_col_partials<1, KM>(dot, k, S.partials, nb, lb);
}

// One block per (system, column): gamma = p.q, alpha = rho / gamma.
__global__ __launch_bounds__(kBlock) void k_fin_dot(
    const SysDesc *__restrict__ sys, const int2 *__restrict__ cmap)
{
    const int2 sc = cmap[blockIdx.x];
    const SysDesc &S = sys[sc.x];
    ColState &cs = S.cs[sc.y];
    if (cs.status != CG_RUNNING) return;
    double t[1];
    sum_partials<1>(S.partials, S.snb, sc.y, t);
    if (threadIdx.x == 0) {
        cs.gamma = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) cs.status = CG_BREAKDOWN;
        else cs.alpha = cs.rho / t[0];
    }
}

template <typename ST, int KM>
__global__ __launch_bounds__(kBlock) void k_update(
    const SysDesc *__restrict__ sys, const int *__restrict__ vmap)
{
    const SysDesc &S = sys[vmap[blockIdx.x]];
    const int lb = blockIdx.x - S.vb0, nb = S.vnb, k = S.k, n = S.n;
    ST *X = static_cast<ST *>(S.x);
    ST *R = static_cast<ST *>(S.r);
    const ST *P = static_cast<const ST *>(S.p);
    const ST *Q = static_cast<const ST *>(S.q);
    const ST *D = static_cast<const ST *>(S.dinv);
    if (!any_running(S)) return;
    // thread t: column c = t % KM of rows lb*RPB + t/KM, + nb*RPB, ...: a
    // wavefront covers 64/KM consecutive rows x KM columns, contiguous
    constexpr int RPB = kBlock / KM;
    const int c = int(threadIdx.x) % KM;
    const bool run = c < k && S.cs[c].status == CG_RUNNING;
    const ST alpha = run ? ST(S.cs[c].alpha) : ST(0);
    double v[2] = {0.0, 0.0};
    if (run)
        for (long i = long(lb) * RPB + threadIdx.x / KM; i < n;
             i += long(nb) * RPB) {
            const long e = i * k + c;
            const ST ri = R[e] - alpha * Q[e];
            X[e] += alpha * P[e];
            R[e] = ri;
            const ST zi = D ? D[i] * ri : ri;
            v[0] += double(ri) * double(zi);
            v[1] += double(ri) * double(ri);
        }
    store_col_partials<2, KM>(v, k, S.partials, nb, lb);
}

// Single-column fused forms (KM = 1): the finalize kernels disappear.  Every
// block sums the system's partials itself, in the same order, so all
// blocks hold bitwise the same scalars; the system's first block alone
// writes the column state.  Fields that other blocks of the same kernel
// read are never written by it: k_update_fused reads rho and writes
// rho_prev, gamma, alpha (and a breakdown status, which every block
// derives itself); k_pupdate_fused reads rho_prev and writes rho, beta,
// rr, iter, status.  The p.q partials stay at partials[0 .. snb), the
// r.z / r.r partials go to partials[snb .. snb + 2 vnb).
// The first kPrefetchRows rows of each thread are loaded before the partial
// sums, so the loads and the reduction's latency overlap (the kernels are
// short: ~6 rows per thread on a 774k-row system).
constexpr int kPrefetchRows = 6;

// alpha_j and beta_j of iteration j = cs.iter into the system's coefficient
// record (condition estimate), when it asks for one; beta = 0 where the
// recurrence stopped (the record then splits there).
__device__ __forceinline__ void record_coeffs(const SysDesc &S,
                                              const ColState &cs, double beta)
{
    if (S.hist && cs.iter < S.hist_cap) {
        S.hist[2 * long(cs.iter)] = cs.alpha;
        S.hist[2 * long(cs.iter) + 1] = beta;
    }
}

template <typename ST>
__global__ __launch_bounds__(kBlock) void k_update_fused(
    const SysDesc *__restrict__ sys, const int *__restrict__ vmap)
{
    const SysDesc &S = sys[vmap[blockIdx.x]];
    const int lb = blockIdx.x - S.vb0, nb = S.vnb, n = S.n;
    ColState &cs = S.cs[0];
    if (cs.status != CG_RUNNING) return;
    const auto X = gblw(static_cast<ST *>(S.x));
    const auto R = gblw(static_cast<ST *>(S.r));
    const auto P = gbl(static_cast<const ST *>(S.p));
    const auto Q = gbl(static_cast<const ST *>(S.q));
    const auto D = gbl(static_cast<const ST *>(S.dinv));
    constexpr int PF = kPrefetchRows;
    const long i0 = long(lb) * kBlock + threadIdx.x, st = long(nb) * kBlock;
    ST xf[PF], pf[PF], rf[PF], qf[PF], df[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
        const long i = i0 + t * st, ic = i < n ? i : 0;
        xf[t] = X[ic];
        pf[t] = P[ic];
        rf[t] = R[ic];
        qf[t] = Q[ic];
        df[t] = D ? D[ic] : ST(1);
    }
    double g1[1];
    sum_partials<1>(S.partials, S.snb, 0, g1);
    const double gamma = g1[0], rho = cs.rho;
    const bool bad = !(gamma > 0.0) || !isfinite(gamma);
    const double alpha_d = bad ? 0.0 : rho / gamma;
    if (lb == 0 && threadIdx.x == 0) {
        cs.gamma = gamma;
        cs.alpha = alpha_d;
        cs.rho_prev = rho;
        if (bad) cs.status = CG_BREAKDOWN;
    }
    if (bad) return;
    const ST alpha = ST(alpha_d);
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int t = 0; t < PF; ++t) {
        const long i = i0 + t * st;
        if (i < n) {
            const ST ri = rf[t] - alpha * qf[t];
            X[i] = xf[t] + alpha * pf[t];
            R[i] = ri;
            const ST zi = D ? df[t] * ri : ri;
            v[0] += double(ri) * double(zi);
            v[1] += double(ri) * double(ri);
        }
    }
    for (long i = i0 + PF * st; i < n; i += st) {
        const ST ri = R[i] - alpha * Q[i];
        X[i] += alpha * P[i];
        R[i] = ri;
        const ST zi = D ? D[i] * ri : ri;
        v[0] += double(ri) * double(zi);
        v[1] += double(ri) * double(ri);
    }
    store_col_partials<2, 1>(v, 1, S.partials + S.snb, nb, lb);
}

template <typename ST>
__global__ __launch_bounds__(kBlock) void k_pupdate_fused(
    const SysDesc *__restrict__ sys, const int *__restrict__ vmap)
{
    const SysDesc &S = sys[vmap[blockIdx.x]];
    const int lb = blockIdx.x - S.vb0, nb = S.vnb, n = S.n;
    ColState &cs = S.cs[0];
    if (cs.status != CG_RUNNING) return;
    const auto P = gblw(static_cast<ST *>(S.p));
    const auto R = gbl(static_cast<const ST *>(S.r));
    const auto D = gbl(static_cast<const ST *>(S.dinv));
    constexpr int PF = kPrefetchRows;
    const long i0 = long(lb) * kBlock + threadIdx.x, st = long(nb) * kBlock;
    ST pf[PF], zf[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
        const long i = i0 + t * st, ic = i < n ? i : 0;
        pf[t] = P[ic];
        zf[t] = D ? D[ic] * R[ic] : R[ic];
    }
    double t[2];
    sum_partials<2>(S.partials + S.snb, nb, 0, t);
    const double rz = t[0], rr = t[1];
    const bool lead = lb == 0 && threadIdx.x == 0;
    if (rr <= cs.tol2) {
        if (lead) {
            record_coeffs(S, cs, 0.0);
            cs.iter += 1;
            cs.rr = rr;
            cs.status = CG_RECURRENCE_MET;
        }
        return;
    }
    const double beta = rz / cs.rho_prev;
    if (!isfinite(beta) || !isfinite(rr)) {
        if (lead) {
            cs.iter += 1;
            cs.rr = rr;
            cs.status = CG_BREAKDOWN;
        }
        return;
    }
    if (lead) {
        record_coeffs(S, cs, beta);
        cs.iter += 1;
        cs.rr = rr;
        cs.beta = beta;
        cs.rho = rz;
        if (cs.iter >= cs.maxit) cs.status = CG_MAXIT;
    }
    const ST b = ST(beta);
#pragma unroll
    for (int t = 0; t < PF; ++t) {
        const long i = i0 + t * st;
        if (i < n) P[i] = zf[t] + b * pf[t];
    }
    for (long i = i0 + PF * st; i < n; i += st) {
        const ST zi = D ? D[i] * R[i] : R[i];
        P[i] = zi + b * P[i];
    }
}

// One block per (system, column): count the iteration; stop when the
// recurrence residual meets the tolerance, else beta = rz / rho.
__global__ __launch_bounds__(kBlock) void k_fin_update(
    const SysDesc *__restrict__ sys, const int2 *__restrict__ cmap)
{
    const int2 sc = cmap[blockIdx.x];
    const SysDesc &S = sys[sc.x];
    ColState &cs = S.cs[sc.y];
    if (cs.status != CG_RUNNING) return;
    double t[2];
    sum_partials<2>(S.partials, S.vnb, 2 * sc.y, t);
    if (threadIdx.x != 0) return;
    const double rz = t[0], rr = t[1];
    cs.iter += 1;
    cs.rr = rr;
    if (rr <= cs.tol2) {
        cs.status = CG_RECURRENCE_MET;
        return;
    }
    const double beta = rz / cs.rho;
    if (!isfinite(beta) || !isfinite(rr)) {
        cs.status = CG_BREAKDOWN;
        return;
    }
    cs.beta = beta;
    cs.rho = rz;
    if (cs.iter >= cs.maxit) cs.status = CG_MAXIT;
}

// p = z + beta p for running columns (PENDING = false) or for the columns
// whose residual was just replaced (PENDING = true).
template <typename ST, int KM, bool PENDING>
__global__ __launch_bounds__(kBlock) void k_pupdate(
    const SysDesc *__restrict__ sys, const int *__restrict__ vmap)
{
    const SysDesc &S = sys[vmap[blockIdx.x]];
    const int lb = blockIdx.x - S.vb0, nb = S.vnb, k = S.k, n = S.n;
    ST *P = static_cast<ST *>(S.p);
    const ST *R = static_cast<const ST *>(S.r);
    const ST *D = static_cast<const ST *>(S.dinv);
    constexpr int RPB = kBlock / KM;
    const int c = int(threadIdx.x) % KM;
    const bool upd = c < k && (PENDING ? S.cs[c].pending != 0
                                       : S.cs[c].status == CG_RUNNING);
    if (!upd) return;
    const ST beta = ST(S.cs[c].beta);
    for (long i = long(lb) * RPB + threadIdx.x / KM; i < n;
         i += long(nb) * RPB) {
        const long e = i * k + c;
        const ST zi = D ? D[i] * R[e] : R[e];
        P[e] = zi + beta * P[e];
    }
}

// r = b - A x (x = 0: r = b) for every column, z = M^-1 r, with r.r, r.z
// and b.b.  MODE 0 starts a solve (writes r and p = z, sets the column
// state); MODE 1 checks the columns whose recurrence residual met the
// tolerance against the true residual (writes r only for them; residual
// replacement when the true residual is too large); MODE 2 only measures;
// MODE 3 rebases the columns whose recurrence residual met the tolerance
// on a new right-hand side b (as MODE 1, and the tolerance becomes
// rtol |b_new|): the search direction is kept, so a refinement step
// continues the Krylov iteration instead of restarting it.
template <typename VT, typename ST, int V, int KM, bool XZ, int MODE>
__global__ __launch_bounds__(kBlock) void k_residual(
    const SysDesc *__restrict__ sys, const int *__restrict__ smap)
{
    const int gb = xcd_remap(blockIdx.x, gridDim.x);
    const SysDesc &S = sys[smap[gb]];
    const int lb = gb - S.sb0, nb = S.snb, k = S.k;
    const auto val = gbl(static_cast<const VT *>(S.val));
    const auto X = gbl(static_cast<const ST *>(S.x));
    const auto B = gbl(static_cast<const ST *>(S.b));
    const auto D = gbl(static_cast<const ST *>(S.dinv));
    const auto R = gblw(static_cast<ST *>(S.r));
    const auto P = gblw(static_cast<ST *>(S.p));
    const auto cst = gbl(S.cstream);
    bool wr[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c)
        wr[c] = c < k && (MODE == 0 ||
                          ((MODE == 1 || MODE == 3) &&
                           S.cs[c].status == CG_RECURRENCE_MET));
    const int g0 = int(long(lb) * S.ngroups / nb);
    const int g1 = int(long(lb + 1) * S.ngroups / nb);
    const int lane = threadIdx.x & (kWave - 1);
    double v[3 * KM];
#pragma unroll
    for (int c = 0; c < 3 * KM; ++c) v[c] = 0.0;
    for (int g = g0 + int(threadIdx.x >> 6); g < g1; g += kWavesPerBlock) {
        const Group gd =
            load_group(gbl(S.groups), __builtin_amdgcn_readfirstlane(g));
        ST a0[KM], a1[KM];
#pragma unroll
        for (int c = 0; c < KM; ++c) a0[c] = a1[c] = ST(0);
        if (!XZ) {
            if (S.gbase)
                lane_sums<VT, ST, V, KM, true>(gd, lane, val, cst,
                                               load_gbase(gbl(S.gbase), g), X,
                                               k, k, a0, a1);
            else
                lane_sums<VT, ST, V, KM, false>(gd, lane, val, cst, 0, X, k,
                                                k, a0, a1);
        }
        const int lt = gd.width_lt >> 24, r = lane >> lt;
        const bool owner = (lane & ((1 << lt) - 1)) == 0 && r < gd.nrows;
        const long row = gd.row0 + r;
        const ST di = (owner && D) ? D[row] : ST(1);
#pragma unroll
        for (int c = 0; c < KM; ++c) {
            if (KM > 1 && c >= k) continue;
            const ST ax = XZ ? ST(0) : row_reduce(a0[c] + a1[c], lt);
            if (owner) {
                const ST bi = B[row * k + c];
                const ST ri = bi - ax;
                const ST zi = D ? di * ri : ri;
                if (wr[c]) R[row * k + c] = ri;
                if (MODE == 0) P[row * k + c] = zi;
                v[3 * c] += double(ri) * double(ri);
                v[3 * c + 1] += double(ri) * double(zi);
                v[3 * c + 2] += double(bi) * double(bi);
            }
        }
    }
    store_partials<3 * KM>(v, 3 * (KM == 1 ? 1 : k), S.partials, nb, lb);
}

// One block per (system, column) after k_residual.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_fin_residual(
    const SysDesc *__restrict__ sys, const int2 *__restrict__ cmap)
{
    const int2 sc = cmap[blockIdx.x];
    const SysDesc &S = sys[sc.x];
    ColState &cs = S.cs[sc.y];
    if ((MODE == 1 || MODE == 3) && cs.status != CG_RECURRENCE_MET) {
        if (threadIdx.x == 0) cs.pending = 0;
        return;
    }
    double t[3];
    sum_partials<3>(S.partials, S.snb, 3 * sc.y, t);
    if (threadIdx.x != 0) return;
    const double rr = t[0], rz = t[1], bb = t[2];
    cs.rr_true = rr;
    if (MODE == 0) {
        cs.bnorm2 = bb;
        cs.tol2 = S.rtol * S.rtol * bb;
        cs.rho = rz;
        cs.rr = rr;
        cs.iter = 0;
        cs.maxit = S.maxit;
        cs.replacements = 0;
        cs.pending = 0;
        cs.alpha = cs.beta = cs.gamma = 0.0;
        if (bb == 0.0 || rr <= cs.tol2) cs.status = CG_CONVERGED;
        else if (!isfinite(rr) || !isfinite(rz)) cs.status = CG_BREAKDOWN;
        else cs.status = CG_RUNNING;
    } else if (MODE == 1 || MODE == 3) {
        cs.pending = 0;
        if (MODE == 3) {
            cs.bnorm2 = bb;
            cs.tol2 = S.rtol * S.rtol * bb;
        }
        if (rr <= cs.tol2) {
            cs.status = CG_CONVERGED;
            return;
        }
        cs.replacements += 1;
        cs.rr = rr;
        const double beta = rz / cs.rho;
        if (!isfinite(beta)) {
            cs.status = CG_BREAKDOWN;
            return;
        }
        cs.beta = beta;
        cs.rho = rz;
        if (cs.iter >= cs.maxit) {
            cs.status = CG_MAXIT;
        } else {
            cs.status = CG_RUNNING;
            cs.pending = 1;
        }
    }
}

// dinv = 1 / diag(A) in the launch's vector type; zero or non-finite
// diagonals are counted in ctr->bad_diag.
template <typename VT, typename ST, int V>
__global__ __launch_bounds__(kBlock) void k_diag(
    const SysDesc *__restrict__ sys, const int *__restrict__ smap)
{
    const int gb = blockIdx.x;
    const SysDesc &S = sys[smap[gb]];
    if (!S.dinv) return;                  // system without preconditioner
    const int lb = gb - S.sb0, nb = S.snb;
    const VT *val = static_cast<const VT *>(S.val);
    ST *D = const_cast<ST *>(static_cast<const ST *>(S.dinv));
    const int g0 = int(long(lb) * S.ngroups / nb);
    const int g1 = int(long(lb + 1) * S.ngroups / nb);
    const int lane = threadIdx.x & (kWave - 1);
    for (int g = g0 + int(threadIdx.x >> 6); g < g1; g += kWavesPerBlock) {
        const Group gd =
            load_group(gbl(S.groups), __builtin_amdgcn_readfirstlane(g));
        const int lt = gd.width_lt >> 24, width = gd.width_lt & 0xffffff;
        const int r = lane >> lt;
        const int row = gd.row0 + r;
        const long base = long(gd.base64) * kWave;
        double d = 0.0;
        for (int s = 0; s < width; ++s) {
            const long idx = base + long(s / V) * kWave * V + lane * V + s % V;
            if (S.col[idx] == row) d += double(widen<ST>(val[idx]));
        }
        d = row_reduce(d, lt);
        if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
            if (d == 0.0 || !isfinite(d)) atomicAdd(S.bad_diag, 1);
            D[row] = ST(1.0 / d);
        }
    }
}

// ------------------------------------------------------------- products
// Y[row or yperm[row], :] = (A X)[row, :] for k <= KM columns; one group per
// wavefront, XCD-aware block order.  With KM = 1 and a float / bf16 value
// array this is the low-precision product (float vectors and sums).
template <typename VT, typename ST, int V, int KM, bool SCATTER, bool N>
__global__ __launch_bounds__(kBlock) void k_spmm(
    const Group *__restrict__ groups, int ngroups, const VT *__restrict__ val,
    const void *__restrict__ col, const int *__restrict__ gbase,
    const ST *__restrict__ X, long ldx, ST *__restrict__ Y, long ldy, int k,
    const int *__restrict__ yperm)
{
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int g = __builtin_amdgcn_readfirstlane(
        b * kWavesPerBlock + int(threadIdx.x >> 6));
    if (g >= ngroups) return;
    const int lane = threadIdx.x & (kWave - 1);
    const Group gd = load_group(gbl(groups), g);
    const int gb = N ? load_gbase(gbl(gbase), g) : 0;
    if constexpr (KM == 1) {
        ST a0[1] = {ST(0)}, a1[1] = {ST(0)};
        lane_sums<VT, ST, V, 1, N>(gd, lane, gbl(val), gbl(col), gb, gbl(X),
                                   1, ldx, a0, a1);
        const int lt = gd.width_lt >> 24, r = lane >> lt;
        const ST v = row_reduce(a0[0] + a1[0], lt);
        if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
            const int row = gd.row0 + r;
            Y[(SCATTER ? long(yperm[row]) : long(row)) * ldy] = v;
        }
    } else {
        coop_group<VT, ST, V, KM, N>(
            gd, lane, gbl(val), gbl(col), gb, gbl(X), k, ldx,
            [&](int rg, int q, ST v) {
                const int row = gd.row0 + rg;
                Y[(SCATTER ? long(yperm[row]) : long(row)) * ldy + q] = v;
            });
    }
}

// ------------------------------------------------------------ dispatch
template <int KM> struct KmTag { static constexpr int value = KM; };

template <class F> void with_km(int km, F &&f)
{
    switch (km) {
    case 1: f(KmTag<1>()); break;
    case 2: f(KmTag<2>()); break;
    case 4: f(KmTag<4>()); break;
    case 8: f(KmTag<8>()); break;
    default: f(KmTag<16>()); break;
    }
}

template <typename VT, typename ST> struct TypeTag {
    typedef VT V;
    typedef ST S;
};

template <class F> void with_types(int vt, int st, F &&f)
{
    if (st == ST_F64) f(TypeTag<double, double>());
    else if (vt == VT_F32) f(TypeTag<float, float>());
    else f(TypeTag<uint16_t, float>());
}

}  // namespace

int32_t engine_spmv_blocks(int32_t ngroups)
{
    int32_t b = (ngroups + kWavesPerBlock - 1) / kWavesPerBlock;
    if (b > kMaxSpmvBlocks) b = kMaxSpmvBlocks;
    return b < 1 ? 1 : b;
}

// Row-shaped grids: at most 1024 workgroups, 512 for single-column systems.
// Every block of the single-column vector kernels sums the whole set of
// partials of the launch before it (the product's, one per group-shaped
// block, and then the update's), so fewer blocks read fewer partials; with
// six rows prefetched per thread, 512 blocks take 87.6 us per config-1
// iteration against 89.5 us with 1024 and four rows (and 97.6 us with
// 2048).
int32_t engine_vec_blocks(int32_t n, int32_t k)
{
    const int32_t b = vec_blocks(n);
    return k == 1 ? std::min(b, 512) : b;
}

hipError_t engine_iteration(const EngineLaunch &L, hipStream_t s)
{
    with_types(L.vt, L.st, [&](auto tt) {
        typedef typename decltype(tt)::V VT;
        typedef typename decltype(tt)::S ST;
        with_km(L.km, [&](auto kt) {
            constexpr int KM = decltype(kt)::value;
            if (L.vec == 1)
                hipLaunchKernelGGL((k_spmm_dot<VT, ST, 1, KM>), dim3(L.sblocks),
                                   dim3(kBlock), 0, s, L.sys, L.smap);
            else
                hipLaunchKernelGGL((k_spmm_dot<VT, ST, 2, KM>), dim3(L.sblocks),
                                   dim3(kBlock), 0, s, L.sys, L.smap);
            if constexpr (KM == 1) {
                hipLaunchKernelGGL((k_update_fused<ST>), dim3(L.vblocks),
                                   dim3(kBlock), 0, s, L.sys, L.vmap);
                hipLaunchKernelGGL((k_pupdate_fused<ST>), dim3(L.vblocks),
                                   dim3(kBlock), 0, s, L.sys, L.vmap);
            } else {
                hipLaunchKernelGGL(k_fin_dot, dim3(L.ncols), dim3(kBlock), 0,
                                   s, L.sys, L.cmap);
                hipLaunchKernelGGL((k_update<ST, KM>), dim3(L.vblocks),
                                   dim3(kBlock), 0, s, L.sys, L.vmap);
                hipLaunchKernelGGL(k_fin_update, dim3(L.ncols), dim3(kBlock),
                                   0, s, L.sys, L.cmap);
                hipLaunchKernelGGL((k_pupdate<ST, KM, false>), dim3(L.vblocks),
                                   dim3(kBlock), 0, s, L.sys, L.vmap);
            }
        });
    });
    return hipGetLastError();
}

template <typename VT, typename ST, int V, int KM, bool XZ>
static void residual_mode(const EngineLaunch &L, int mode, hipStream_t s)
{
    const dim3 g(L.sblocks), b(kBlock), f(L.ncols);
    if (mode == 0) {
        hipLaunchKernelGGL((k_residual<VT, ST, V, KM, XZ, 0>), g, b, 0, s,
                           L.sys, L.smap);
        hipLaunchKernelGGL(k_fin_residual<0>, f, b, 0, s, L.sys, L.cmap);
    } else if (mode == 1) {
        hipLaunchKernelGGL((k_residual<VT, ST, V, KM, XZ, 1>), g, b, 0, s,
                           L.sys, L.smap);
        hipLaunchKernelGGL(k_fin_residual<1>, f, b, 0, s, L.sys, L.cmap);
    } else if (mode == 2) {
        hipLaunchKernelGGL((k_residual<VT, ST, V, KM, XZ, 2>), g, b, 0, s,
                           L.sys, L.smap);
        hipLaunchKernelGGL(k_fin_residual<2>, f, b, 0, s, L.sys, L.cmap);
    } else {
        hipLaunchKernelGGL((k_residual<VT, ST, V, KM, XZ, 3>), g, b, 0, s,
                           L.sys, L.smap);
        hipLaunchKernelGGL(k_fin_residual<3>, f, b, 0, s, L.sys, L.cmap);
    }
}

hipError_t engine_residual(const EngineLaunch &L, int32_t mode, bool x_zero,
                           hipStream_t s)
{
    with_types(L.vt, L.st, [&](auto tt) {
        typedef typename decltype(tt)::V VT;
        typedef typename decltype(tt)::S ST;
        with_km(L.km, [&](auto kt) {
            constexpr int KM = decltype(kt)::value;
            if (L.vec == 1) {
                if (x_zero) residual_mode<VT, ST, 1, KM, true>(L, mode, s);
                else residual_mode<VT, ST, 1, KM, false>(L, mode, s);
            } else {
                if (x_zero) residual_mode<VT, ST, 2, KM, true>(L, mode, s);
                else residual_mode<VT, ST, 2, KM, false>(L, mode, s);
            }
        });
    });
    return hipGetLastError();
}

hipError_t engine_pupdate_pending(const EngineLaunch &L, hipStream_t s)
{
    with_types(L.vt, L.st, [&](auto tt) {
        typedef typename decltype(tt)::S ST;
        with_km(L.km, [&](auto kt) {
            constexpr int KM = decltype(kt)::value;
            hipLaunchKernelGGL((k_pupdate<ST, KM, true>), dim3(L.vblocks),
                               dim3(kBlock), 0, s, L.sys, L.vmap);
        });
    });
    return hipGetLastError();
}

hipError_t engine_diag_inv(const EngineLaunch &L, hipStream_t s)
{
    with_types(L.vt, L.st, [&](auto tt) {
        typedef typename decltype(tt)::V VT;
        typedef typename decltype(tt)::S ST;
        if (L.vec == 1)
            hipLaunchKernelGGL((k_diag<VT, ST, 1>), dim3(L.sblocks),
                               dim3(kBlock), 0, s, L.sys, L.smap);
        else
            hipLaunchKernelGGL((k_diag<VT, ST, 2>), dim3(L.sblocks),
                               dim3(kBlock), 0, s, L.sys, L.smap);
    });
    return hipGetLastError();
}

// ------------------------------------------------------- auxiliary kernels
namespace {

// staging[b] = state of column cmap[b].y of system cmap[b].x
__global__ void k_gather_states(const SysDesc *__restrict__ sys,
                                const int2 *__restrict__ cmap, int ncols,
                                ColState *__restrict__ staging)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= ncols) return;
    const int2 sc = cmap[b];
    staging[b] = sys[sc.x].cs[sc.y];
}

// Row permutation of an n x k block: TO_LAYOUT dst[i, :] = src[perm[i], :],
// else dst[perm[i], :] = src[i, :].  ld of the caller side is ldc, of the
// layout side k.
template <bool TO_LAYOUT>
__global__ __launch_bounds__(kBlock) void k_permute_rows(
    int n, int k, const int *__restrict__ perm, const double *__restrict__ src,
    long lds, double *__restrict__ dst, long ldd)
{
    const long total = long(n) * k;
    for (long e = long(blockIdx.x) * kBlock + threadIdx.x; e < total;
         e += long(gridDim.x) * kBlock) {
        const int i = int(e / k), c = int(e % k);
        const long pi = perm ? perm[i] : i;
        if (TO_LAYOUT) dst[i * ldd + c] = src[pi * lds + c];
        else dst[pi * ldd + c] = src[i * lds + c];
    }
}

// b = float(a), or float(sc[row] * a) with sc != NULL (k entries per row)
__global__ __launch_bounds__(kBlock) void k_to_f32(long n, int k,
                                                   const double *__restrict__ a,
                                                   const double *__restrict__ sc,
                                                   float *__restrict__ b)
{
    for (long e = long(blockIdx.x) * kBlock + threadIdx.x; e < n;
         e += long(gridDim.x) * kBlock)
        b[e] = float(sc ? sc[e / k] * a[e] : a[e]);
}

// x += alpha d, or x += alpha (sc[row] d) with sc != NULL
__global__ __launch_bounds__(kBlock) void k_add_f32(long n, int k, double alpha,
                                                    const float *__restrict__ d,
                                                    const double *__restrict__ sc,
                                                    double *__restrict__ x)
{
    for (long e = long(blockIdx.x) * kBlock + threadIdx.x; e < n;
         e += long(gridDim.x) * kBlock) {
        const double de = sc ? sc[e / k] * double(d[e]) : double(d[e]);
        x[e] += alpha * de;
    }
}

// Jacobi scaling of the layout: sc[row] = 1 / sqrt(a_row,row); rows whose
// diagonal is not positive and finite get 0 and are counted in *bad.  One
// wavefront per row group (grid-stride).
template <int V>
__global__ __launch_bounds__(kBlock) void k_diag_rsqrt(
    const Group *__restrict__ groups, int ngroups, const double *__restrict__ val,
    const int32_t *__restrict__ col, double *__restrict__ sc,
    int32_t *__restrict__ bad)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int g = blockIdx.x * kWavesPerBlock + int(threadIdx.x >> 6);
         g < ngroups; g += gridDim.x * kWavesPerBlock) {
        const Group gd = load_group(gbl(groups), __builtin_amdgcn_readfirstlane(g));
        const int lt = gd.width_lt >> 24, width = gd.width_lt & 0xffffff;
        const int r = lane >> lt, row = gd.row0 + r;
        const long base = long(gd.base64) * kWave;
        double d = 0.0;
        for (int s = 0; s < width; ++s) {
            const long idx = base + long(s / V) * kWave * V + lane * V + s % V;
            if (col[idx] == row) d += val[idx];
        }
        d = row_reduce(d, lt);
        if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
            const bool ok = d > 0.0 && isfinite(d);
            if (!ok) atomicAdd(bad, 1);
            sc[row] = ok ? 1.0 / sqrt(d) : 0.0;
        }
    }
}

// Low-precision copy of the Jacobi-scaled values: slot (row, col) holds
// round((a * sc[row]) * sc[col]) (FP64 products, then float nearest, then
// bf16 nearest-even); padding stays 0.
template <int V>
__global__ __launch_bounds__(kBlock) void k_cast_scaled(
    const Group *__restrict__ groups, int ngroups, const double *__restrict__ val,
    const int32_t *__restrict__ col, const double *__restrict__ sc,
    float *__restrict__ f32, uint16_t *__restrict__ bf16)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int g = blockIdx.x * kWavesPerBlock + int(threadIdx.x >> 6);
         g < ngroups; g += gridDim.x * kWavesPerBlock) {
        const Group gd = load_group(gbl(groups), __builtin_amdgcn_readfirstlane(g));
        const int lt = gd.width_lt >> 24, width = gd.width_lt & 0xffffff;
        const int row = gd.row0 + (lane >> lt);
        const long base = long(gd.base64) * kWave;
        for (int s = 0; s < width; ++s) {
            const long idx = base + long(s / V) * kWave * V + lane * V + s % V;
            const int c = col[idx];
            const float f = c >= 0 ? float((val[idx] * sc[row]) * sc[c]) : 0.0f;
            if (f32) f32[idx] = f;
            if (bf16) bf16[idx] = f32_to_bf16_rne(f);
        }
    }
}

// Low-precision copies of the slot values (padding stays 0).
__global__ __launch_bounds__(kBlock) void k_cast_slots(
    long n, const double *__restrict__ v, float *__restrict__ f32,
    uint16_t *__restrict__ bf16)
{
    for (long e = long(blockIdx.x) * kBlock + threadIdx.x; e < n;
         e += long(gridDim.x) * kBlock) {
        const float f = float(v[e]);
        if (f32) f32[e] = f;
        if (bf16) bf16[e] = f32_to_bf16_rne(f);
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(long n, double v,
                                                     double *__restrict__ p)
{
    for (long e = long(blockIdx.x) * kBlock + threadIdx.x; e < n;
         e += long(gridDim.x) * kBlock)
        p[e] = v;
}

int flat_blocks(long n)
{
    long b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    return b < 1 ? 1 : int(b);
}

}  // namespace

hipError_t engine_gather_states(const EngineLaunch &L, ColState *staging,
                                hipStream_t s)
{
    if (L.ncols == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_states, dim3((L.ncols + 63) / 64), dim3(64), 0,
                       s, L.sys, L.cmap, L.ncols, staging);
    return hipGetLastError();
}

hipError_t permute_rows(int32_t n, int32_t k, const int32_t *perm,
                        const double *src, int64_t lds, double *dst,
                        int64_t ldd, bool to_layout, hipStream_t s)
{
    const long total = long(n) * k;
    if (total == 0) return hipSuccess;
    if (to_layout)
        hipLaunchKernelGGL(k_permute_rows<true>, dim3(flat_blocks(total)),
                           dim3(kBlock), 0, s, n, k, perm, src, long(lds), dst,
                           long(ldd));
    else
        hipLaunchKernelGGL(k_permute_rows<false>, dim3(flat_blocks(total)),
                           dim3(kBlock), 0, s, n, k, perm, src, long(lds), dst,
                           long(ldd));
    return hipGetLastError();
}

hipError_t to_f32(int64_t n, int32_t k, const double *a, const double *sc,
                  float *b, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3(flat_blocks(n)), dim3(kBlock), 0, s,
                       long(n), int(k), a, sc, b);
    return hipGetLastError();
}

hipError_t add_f32(int64_t n, int32_t k, double alpha, const float *d,
                   const double *sc, double *x, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_f32, dim3(flat_blocks(n)), dim3(kBlock), 0, s,
                       long(n), int(k), alpha, d, sc, x);
    return hipGetLastError();
}

hipError_t scaled_lowp_copy(const fs_csr *A, int32_t dtype, double *sc,
                            void *out, int32_t *bad, hipStream_t s)
{
    if (A->n_groups == 0) return hipSuccess;
    const int nb = std::min((A->n_groups + kWavesPerBlock - 1) / kWavesPerBlock,
                            8192);
    float *f32 = dtype == FS_DT_F32 ? static_cast<float *>(out) : nullptr;
    uint16_t *bf = dtype == FS_DT_BF16 ? static_cast<uint16_t *>(out) : nullptr;
    if (A->host.vec == 1) {
        hipLaunchKernelGGL(k_diag_rsqrt<1>, dim3(nb), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, A->d_col, sc,
                           bad);
        hipLaunchKernelGGL(k_cast_scaled<1>, dim3(nb), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, A->d_col, sc,
                           f32, bf);
    } else {
        hipLaunchKernelGGL(k_diag_rsqrt<2>, dim3(nb), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, A->d_col, sc,
                           bad);
        hipLaunchKernelGGL(k_cast_scaled<2>, dim3(nb), dim3(kBlock), 0, s,
                           A->d_groups, A->n_groups, A->d_val, A->d_col, sc,
                           f32, bf);
    }
    return hipGetLastError();
}

hipError_t fill_f64(int64_t n, double v, double *p, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(flat_blocks(n)), dim3(kBlock), 0, s,
                       long(n), v, p);
    return hipGetLastError();
}

hipError_t cast_slots(int64_t n, const double *v, float *f32, uint16_t *bf16,
                      hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast_slots, dim3(flat_blocks(n)), dim3(kBlock), 0, s,
                       long(n), v, f32, bf16);
    return hipGetLastError();
}


hipError_t launch_spmm_f64(const fs_csr *A, int32_t k, const double *X,
                           int64_t ldx, double *Y, int64_t ldy,
                           const int32_t *yperm, hipStream_t s)
{
    if (A->n_groups == 0) return hipSuccess;
    const dim3 grid((A->n_groups + kWavesPerBlock - 1) / kWavesPerBlock);
    const int km = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
    with_km(km, [&](auto kt) {
        constexpr int KM = decltype(kt)::value;
        auto go = [&](auto vtag, auto stag) {
            constexpr int V = decltype(vtag)::value;
            constexpr bool SC = decltype(stag)::value;
            if (A->d_col16)
                hipLaunchKernelGGL((k_spmm<double, double, V, KM, SC, true>),
                                   grid, dim3(kBlock), 0, s, A->d_groups,
                                   A->n_groups, A->d_val, A->d_col16,
                                   A->d_gbase, X, long(ldx), Y, long(ldy), k,
                                   yperm);
            else
                hipLaunchKernelGGL((k_spmm<double, double, V, KM, SC, false>),
                                   grid, dim3(kBlock), 0, s, A->d_groups,
                                   A->n_groups, A->d_val, A->d_col, nullptr,
                                   X, long(ldx), Y, long(ldy), k, yperm);
        };
        if (A->host.vec == 1) {
            if (yperm) go(KmTag<1>(), std::true_type());
            else go(KmTag<1>(), std::false_type());
        } else {
            if (yperm) go(KmTag<2>(), std::true_type());
            else go(KmTag<2>(), std::false_type());
        }
    });
    return hipGetLastError();
}

hipError_t launch_spmv_lowp(const fs_csr *A, int32_t dtype, const float *x,
                            float *y, hipStream_t s)
{
    if (A->n_groups == 0) return hipSuccess;
    const dim3 grid((A->n_groups + kWavesPerBlock - 1) / kWavesPerBlock);
    auto go = [&](auto vt, auto vtag) {
        typedef typename decltype(vt)::V VT;
        constexpr int V = decltype(vtag)::value;
        const VT *val = dtype == FS_DT_F32
                            ? reinterpret_cast<const VT *>(A->d_val_f32)
                            : reinterpret_cast<const VT *>(A->d_val_bf16);
        if (A->d_col16)
            hipLaunchKernelGGL((k_spmm<VT, float, V, 1, false, true>), grid,
                               dim3(kBlock), 0, s, A->d_groups, A->n_groups,
                               val, A->d_col16, A->d_gbase, x, 1L, y, 1L, 1,
                               nullptr);
        else
            hipLaunchKernelGGL((k_spmm<VT, float, V, 1, false, false>), grid,
                               dim3(kBlock), 0, s, A->d_groups, A->n_groups,
                               val, A->d_col, nullptr, x, 1L, y, 1L, 1,
                               nullptr);
    };
    if (dtype == FS_DT_F32) {
        if (A->host.vec == 1) go(TypeTag<float, float>(), KmTag<1>());
        else go(TypeTag<float, float>(), KmTag<2>());
    } else {
        if (A->host.vec == 1) go(TypeTag<uint16_t, float>(), KmTag<1>());
        else go(TypeTag<uint16_t, float>(), KmTag<2>());
    }
    return hipGetLastError();
}

}  // namespace fs
