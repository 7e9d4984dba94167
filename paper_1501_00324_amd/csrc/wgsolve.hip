// One-workgroup solves: each system of a batch runs its whole Jacobi-PCG
// solve (the solver the paper runs around its SpMV, sections "Computational
// Cost of the Finite Element Method" and "Description of Current GPU
// Methods") inside one workgroup of a single launch.  For small systems a
// solve is bound by launch and synchronisation latency, not by bandwidth:
// here an iteration costs two workgroup barriers instead of three kernel
// launches and a host round trip per chunk; the matrix, re-read every
// iteration, stays in the L2 of the XCD that runs its workgroup (plain
// cached loads, unlike the streaming loads of the large products), and
// the Krylov vectors stay in LDS when they fit: z, x, r, p, q (then only
// the slot stream, D^-1 and b are read from L2), else z = D^-1 r alone,
// which the product gathers.
//
// Reductions do not depend on the workgroup size: the work is cut into
// fixed units (two row groups in the product steps, four 64-row chunks in
// the vector step); the one wavefront that takes a unit adds each lane's
// share over the unit in a fixed order, reduces across the wavefront and
// stores the result in LDS at the unit's index, and every wavefront then
// adds the stored values in index order.  So x, the iteration count and
// the residuals are bitwise the same for 256, 512 or 1024 threads, alone
// or in any batch, and the workgroup size can be chosen by timing alone.
// Two LDS regions alternate between successive reductions: a region is
// rewritten two reductions later, after a barrier that every wavefront
// reaches only once it has read the region's sums.
//
// Iteration (as in the persistent solve: the product gathers z, and p and
// q = A p follow the same recurrence, so the direction update needs no
// phase of its own; the first iteration takes p = z, q = A z):
//   w = A z; p = z + beta p; q = w + beta q; p.q  | barrier | alpha
//   x += alpha p; r -= alpha q; z = D^-1 r; r.z, r.r | barrier | beta
// When |r| meets the tolerance, b - A x is recomputed; if it misses, it
// replaces r and the iteration continues.
#include <algorithm>

#include "device.h"

namespace fs {
namespace {

enum { W_RUNNING = 0, W_CONVERGED = 1, W_BREAKDOWN = 2, W_MAXIT = 3 };

constexpr int kGU = kWgGroupsPerUnit;
constexpr int kCU = kWgChunksPerUnit;
static_assert(kGU == 2, "the product pairs the two groups of a unit");

struct WgArgs {
    double rtol, clock_khz;
    int32_t maxit, x_zero, write_out;
    int32_t parts;                  // LDS entries per value
};

// This lane's share of its row in each of G row groups of equal width,
// sum over its slots of a * x[col], with plain (cached) loads of the slot
// stream; the G groups' loads are issued together, U slots of each per
// batch.  A group's sum is formed in the same order for any G and U (two
// accumulators by slot parity, each in slot order).
template <int V, bool N, int G, int U, class XP>
__device__ __forceinline__ void wg_lane_sums(const Group (&g)[G],
                                             const int (&gb)[G], int lane,
                                             gptr<double> val, gptr<void> col,
                                             XP x, double (&out)[G])
{
    static_assert(U % 2 == 0, "slot parity must match the batch position");
    typedef typename Slots<V>::D D;
    typedef typename std::conditional<N, typename Slots<V>::H,
                                      typename Slots<V>::I>::type P;
    typedef typename std::conditional<N, uint16_t, int32_t>::type E;
    const int nch = (g[0].width_lt & 0xffffff) / V;
    gptr<D> pv[G];
    gptr<P> pc[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const long base = long(g[k].base64) * kWave;
        pv[k] = reinterpret_cast<gptr<D>>(val + base) + lane;
        pc[k] = reinterpret_cast<gptr<P>>(static_cast<gptr<E>>(col) + base) +
                lane;
    }
    auto colof = [&](const P &c, int t, int k) {
        int v;
        if constexpr (V == 1) v = int(c);
        else v = t ? int(c.y) : int(c.x);
        if constexpr (N) return v == 0xffff ? -1 : gb[k] + v;
        else return v;
    };
    double acc0[G], acc1[G];
#pragma unroll
    for (int k = 0; k < G; ++k) acc0[k] = acc1[k] = 0.0;
    // padded slots (column -1) read x[0] and add nothing
    auto fma1 = [&](int c, double av, double &acc) {
        const double xv = x[c < 0 ? 0 : c];
        acc = fma(av, c >= 0 ? xv : 0.0, acc);
    };
    auto use = [&](const P &c, const D &a, int k, int j) {
        if constexpr (V == 1) {
            fma1(colof(c, 0, k), a, (j & 1) ? acc1[k] : acc0[k]);
        } else {
            fma1(colof(c, 0, k), a.x, acc0[k]);
            fma1(colof(c, 1, k), a.y, acc1[k]);
        }
    };
    int j = 0;
    for (; j + U <= nch; j += U) {
        P c[G][U];
        D a[G][U];
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) c[k][u] = pc[k][long(j + u) * kWave];
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) a[k][u] = pv[k][long(j + u) * kWave];
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) use(c[k][u], a[k][u], k, u);
    }
    for (; j < nch; ++j) {
        P c[G];
        D a[G];
#pragma unroll
        for (int k = 0; k < G; ++k) c[k] = pc[k][long(j) * kWave];
#pragma unroll
        for (int k = 0; k < G; ++k) a[k] = pv[k][long(j) * kWave];
#pragma unroll
        for (int k = 0; k < G; ++k) use(c[k], a[k], k, j);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) out[k] = acc0[k] + acc1[k];
}

// Sums of NJ values over the stored parts (one per unit), added in index
// order; every wavefront forms them itself, bitwise alike.
template <int NJ>
__device__ __forceinline__ void part_totals(const double *buf, int np,
                                            int stride, double (&out)[NJ])
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        double s = 0.0;
        for (int i = lane; i < np; i += kWave) s += buf[j * stride + i];
        out[j] = wave_sum(s);
    }
}

// Where the vectors live (MODE): 0 all in global memory; 1 z in LDS; 2 z,
// x, r, p and q in LDS (x copied in at the start and out at the end; b and
// D^-1, which the iterations only read, stay in global memory and L2).
template <int V, bool N, int MODE>
__device__ __forceinline__ void wg_solve(const WgSys &S, const WgArgs &a,
                                         double *lds)
{
    const long t_start = wall_clock64();
    const int lane = threadIdx.x & (kWave - 1);
    const int w = int(threadIdx.x >> 6), nw = int(blockDim.x >> 6);
    const int n = S.n, ng = S.ngroups, nc = (n + kWave - 1) / kWave;
    // units: kGU row groups (product steps), kCU 64-row chunks (vector
    // step); one wavefront takes a unit, sums each lane's share over it in
    // a fixed order, and stores one part per value
    const int nug = (ng + kGU - 1) / kGU, nuc = (nc + kCU - 1) / kCU;
    const int P = a.parts;
    const gptr<Group> G = gbl(S.groups);
    const gptr<double> val = gbl(S.val);
    const gptr<void> cstream = gbl(S.cstream);
    const gptr<int32_t> col = gbl(S.col);
    const bool pc = S.dinv != nullptr;   // Jacobi preconditioner
    // the vectors: LDS after the two part regions (z first), or global
    double *const zl = lds + 6 * P;
    auto vec = [&](double *g, int k) {
        if constexpr (MODE == 2) return zl + long(k) * n;
        else return gblw(g);
    };
    auto zv = [&]() {
        if constexpr (MODE >= 1) return zl;
        else return gblw(S.z);
    }();
    const auto X = vec(S.x, 1), R = vec(S.r, 2), Pv = vec(S.p, 3),
               Q = vec(S.q, 4);
    const auto D = gblw(S.dinv);   // read-only after the scaling pass
    const auto Bv = gblw(S.b);
    const auto perm = gbl(S.perm);
    auto zget = [&](int i) -> double { return zv[i]; };
    auto zput = [&](int i, double v) { zv[i] = v; };
    auto zsrc = [&]() {
        if constexpr (MODE >= 1) return static_cast<const double *>(zl);
        else return gbl(static_cast<const double *>(S.z));
    };
    auto xsrc = [&]() {
        if constexpr (MODE == 2) return static_cast<const double *>(X);
        else return gbl(static_cast<const double *>(S.x));
    };
    int red = 0;   // reductions so far: region (red & 1) is next
    auto region = [&]() {
        double *r = lds + (red & 1) * 3 * P;
        ++red;
        return r;
    };
    auto group = [&](int g) {
        return load_group(G, __builtin_amdgcn_readfirstlane(g));
    };
    auto gbase = [&](int g) { return N ? load_gbase(gbl(S.gbase), g) : 0; };
    // product of group g with x, reduced over the T lanes of each row
    auto gsum = [&](const Group &gd, int g, auto x) {
        const Group gg[1] = {gd};
        const int gb[1] = {gbase(g)};
        double o[1];
        wg_lane_sums<V, N, 1, 8 / V>(gg, gb, lane, val, cstream, x, o);
        return row_reduce(o[0], gd.width_lt >> 24);
    };
    // row of lane in group gd (clamped to the group), and whether the lane
    // owns it
    auto owner = [&](const Group &gd, int &row) {
        const int lt = gd.width_lt >> 24, r = lane >> lt;
        row = gd.row0 + (r < gd.nrows ? r : 0);
        return (lane & ((1 << lt) - 1)) == 0 && r < gd.nrows;
    };
    // a reduction over group units: f(g, gd, v) adds group g's share of
    // NJ values to this lane's v[]
    auto group_pass = [&](double *buf, auto f, auto nj) {
        constexpr int NJ = decltype(nj)::value;
        for (int u = w; u < nug; u += nw) {
            double v[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) v[j] = 0.0;
            for (int g = u * kGU; g < std::min(ng, (u + 1) * kGU); ++g)
                f(g, group(g), v);
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const double t = wave_sum(v[j]);
                if (lane == 0) buf[j * P + u] = t;
            }
        }
    };

    // b (and the guess) into the layout numbering
    for (int i = int(threadIdx.x); i < n; i += int(blockDim.x)) {
        const int pi = S.perm ? perm[i] : i;
        Bv[i] = gbl(S.b_in)[pi];
        if (!a.x_zero) X[i] = gbl(S.x_in)[pi];
    }
    __syncthreads();
    // Jacobi scaling: 1 / a_ii from the row's slots
    if (pc) {
        for (int g = w; g < ng; g += nw) {
            const Group gd = group(g);
            const int width = gd.width_lt & 0xffffff, lt = gd.width_lt >> 24;
            int row;
            const bool own = owner(gd, row);
            const long base = long(gd.base64) * kWave;
            double d = 0.0;
            for (int s = 0; s < width; ++s) {
                const long idx =
                    base + long(s / V) * kWave * V + lane * V + s % V;
                if (col[idx] == row) d += val[idx];
            }
            d = row_reduce(d, lt);
            if (own) D[row] = 1.0 / d;
        }
    }
    __syncthreads();
    // start: r = b - A x (x = 0 written when the guess is zero), z = D^-1 r;
    // |r|^2, r.z, |b|^2
    double s3[3];
    {
        double *buf = region();
        group_pass(buf, [&](int g, const Group &gd, double (&v)[3]) {
            const double ax = a.x_zero ? 0.0 : gsum(gd, g, xsrc());
            int row;
            if (owner(gd, row)) {
                const double bi = Bv[row], ri = bi - ax;
                const double zi = pc ? D[row] * ri : ri;
                if (a.x_zero) X[row] = 0.0;
                R[row] = ri;
                zput(row, zi);
                v[0] += ri * ri;
                v[1] += ri * zi;
                v[2] += bi * bi;
            }
        }, std::integral_constant<int, 3>());
        __syncthreads();
        part_totals<3>(buf, nug, P, s3);
    }
    const double bb = s3[2], tol2 = a.rtol * a.rtol * bb;
    double rho = s3[1], rr = s3[0], rr_true = s3[0];
    int status = W_RUNNING, it = 0, repl = 0;
    if (bb == 0.0) {
        for (int i = int(threadIdx.x); i < n; i += int(blockDim.x)) X[i] = 0.0;
        status = W_CONVERGED;
        rr_true = 0.0;
    } else if (rr <= tol2) {
        status = W_CONVERGED;
    } else if (!isfinite(rr) || !isfinite(rho)) {
        status = W_BREAKDOWN;
    }
    bool first = true;
    double beta = 0.0;
    while (status == W_RUNNING) {
        // w = A z; p = z + beta p, q = w + beta q; p.q.  The two groups of
        // a unit are multiplied together when their widths agree, and each
        // row's own z, p, q are loaded before the gathers.
        double *buf = region();
        for (int u = w; u < nug; u += nw) {
            const int g0 = u * kGU, g1 = g0 + 1;
            const bool two = g1 < ng;
            const Group gd0 = group(g0), gd1 = two ? group(g1) : gd0;
            int row0, row1;
            const bool own0 = owner(gd0, row0), own1 = two && owner(gd1, row1);
            if (!two) row1 = row0;
            const double z0 = zget(row0), z1 = zget(row1);
            const double p0 = first ? 0.0 : Pv[row0];
            const double q0 = first ? 0.0 : Q[row0];
            const double p1 = first ? 0.0 : Pv[row1];
            const double q1 = first ? 0.0 : Q[row1];
            double w0, w1 = 0.0;
            if (two && gd0.width_lt == gd1.width_lt) {
                const Group gg[2] = {gd0, gd1};
                const int gb[2] = {gbase(g0), gbase(g1)};
                double o[2];
                wg_lane_sums<V, N, 2, 4 / V>(gg, gb, lane, val, cstream,
                                             zsrc(), o);
                w0 = row_reduce(o[0], gd0.width_lt >> 24);
                w1 = row_reduce(o[1], gd1.width_lt >> 24);
            } else {
                w0 = gsum(gd0, g0, zsrc());
                if (two) w1 = gsum(gd1, g1, zsrc());
            }
            double v = 0.0;
            if (own0) {
                const double pi = first ? z0 : z0 + beta * p0;
                const double qi = first ? w0 : w0 + beta * q0;
                Pv[row0] = pi;
                Q[row0] = qi;
                v += pi * qi;
            }
            if (own1) {
                const double pi = first ? z1 : z1 + beta * p1;
                const double qi = first ? w1 : w1 + beta * q1;
                Pv[row1] = pi;
                Q[row1] = qi;
                v += pi * qi;
            }
            v = wave_sum(v);
            if (lane == 0) buf[u] = v;
        }
        __syncthreads();
        double s1[1];
        part_totals<1>(buf, nug, P, s1);
        const double gamma = s1[0];
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            status = W_BREAKDOWN;
            break;
        }
        const double alpha = rho / gamma;
        first = false;
        // x += alpha p, r -= alpha q, z = D^-1 r; r.z, r.r (a unit's chunks
        // loaded together, summed per lane in chunk order)
        buf = region();
        for (int u = w; u < nuc; u += nw) {
            double rv[kCU], qv[kCU], xv[kCU], pv[kCU], dv[kCU];
#pragma unroll
            for (int k = 0; k < kCU; ++k) {
                const int i = (u * kCU + k) * kWave + lane;
                const int ic = i < n ? i : 0;
                rv[k] = R[ic];
                qv[k] = Q[ic];
                xv[k] = X[ic];
                pv[k] = Pv[ic];
                dv[k] = pc ? D[ic] : 1.0;
            }
            double v0 = 0.0, v1 = 0.0;
#pragma unroll
            for (int k = 0; k < kCU; ++k) {
                const int i = (u * kCU + k) * kWave + lane;
                if (i < n) {
                    const double ri = rv[k] - alpha * qv[k];
                    X[i] = xv[k] + alpha * pv[k];
                    R[i] = ri;
                    const double zi = pc ? dv[k] * ri : ri;
                    zput(i, zi);
                    v0 += ri * zi;
                    v1 += ri * ri;
                }
            }
            v0 = wave_sum(v0);
            v1 = wave_sum(v1);
            if (lane == 0) {
                buf[u] = v0;
                buf[P + u] = v1;
            }
        }
        __syncthreads();
        double s2[2];
        part_totals<2>(buf, nuc, P, s2);
        ++it;
        double rz = s2[0];
        rr = s2[1];
        if (rr <= tol2) {
            // confirm against the true residual; replace r if it misses
            buf = region();
            group_pass(buf, [&](int g, const Group &gd, double (&v)[2]) {
                const double ax = gsum(gd, g, xsrc());
                int row;
                if (owner(gd, row)) {
                    const double ri = Bv[row] - ax;
                    const double zi = pc ? D[row] * ri : ri;
                    R[row] = ri;
                    zput(row, zi);
                    v[0] += ri * zi;
                    v[1] += ri * ri;
                }
            }, std::integral_constant<int, 2>());
            __syncthreads();
            part_totals<2>(buf, nug, P, s2);
            rr_true = s2[1];
            if (rr_true <= tol2) {
                status = W_CONVERGED;
                break;
            }
            ++repl;
            rz = s2[0];
            rr = rr_true;
        } else if (!isfinite(rr)) {
            status = W_BREAKDOWN;
            break;
        }
        beta = rz / rho;
        if (!isfinite(beta)) {
            status = W_BREAKDOWN;
            break;
        }
        rho = rz;
        if (it >= a.maxit) {
            status = W_MAXIT;
            break;
        }
    }
    if (status != W_CONVERGED) {
        // the true residual of the returned x (x was last written before
        // the barrier that preceded the exit)
        double *buf = region();
        group_pass(buf, [&](int g, const Group &gd, double (&v)[1]) {
            const double ax = gsum(gd, g, xsrc());
            int row;
            if (owner(gd, row)) {
                const double ri = Bv[row] - ax;
                v[0] += ri * ri;
            }
        }, std::integral_constant<int, 1>());
        __syncthreads();
        double s1[1];
        part_totals<1>(buf, nug, P, s1);
        rr_true = s1[0];
    }
    if (a.write_out) {
        // x back into the caller's numbering (every wavefront's last
        // writes of x precede the barrier of the last reduction)
        for (int i = int(threadIdx.x); i < n; i += int(blockDim.x))
            gblw(S.x_out)[S.perm ? perm[i] : i] = X[i];
    }
    if (threadIdx.x == 0) {
        fs_cg_info o;
        o.status = status == W_CONVERGED ? FS_OK
                   : status == W_MAXIT   ? FS_E_NOT_CONVERGED
                                         : FS_E_BREAKDOWN;
        o.iters = it;
        o.outer = 0;
        o.replacements = repl;
        o.cond_est = 0.0;
        o.relres = bb > 0.0 ? sqrt(rr_true / bb) : 0.0;
        o.ms = double(wall_clock64() - t_start) / a.clock_khz;
        o.bytes = double(it) * (12.0 * S.nnz + (pc ? 104.0 : 88.0) * n) +
                  2.0 * (12.0 * S.nnz + 16.0 * n);
        *S.info = o;
    }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_cg_wg(const WgSys *__restrict__ sys,
                                              const WgArgs a)
{
    extern __shared__ double lds[];
    const WgSys S = sys[blockIdx.x];
    if (S.n == 0) return;
    auto go = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        if (S.vec == 2) {
            if (S.narrow) wg_solve<2, true, M>(S, a, lds);
            else wg_solve<2, false, M>(S, a, lds);
        } else {
            if (S.narrow) wg_solve<1, true, M>(S, a, lds);
            else wg_solve<1, false, M>(S, a, lds);
        }
    };
    if (S.zl == 2) go(std::integral_constant<int, 2>());
    else if (S.zl == 1) go(std::integral_constant<int, 1>());
    else go(std::integral_constant<int, 0>());
}

}  // namespace

hipError_t launch_cg_wg(const WgSys *d_sys, int32_t m, int32_t threads,
                        int32_t parts, int32_t vec_doubles, double rtol,
                        int32_t maxit, bool x_zero, bool write_out,
                        int device, hipStream_t s)
{
    int khz = 0;
    hipError_t e =
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
    if (e != hipSuccess) return e;
    WgArgs a;
    a.rtol = rtol;
    a.clock_khz = double(khz > 0 ? khz : 100000);
    a.maxit = maxit;
    a.x_zero = x_zero ? 1 : 0;
    a.write_out = write_out ? 1 : 0;
    a.parts = parts;
    const size_t lds = sizeof(double) * size_t(2 * 3 * parts + vec_doubles);
    const void *fn = threads == 256   ? reinterpret_cast<const void *>(k_cg_wg<256>)
                     : threads == 512 ? reinterpret_cast<const void *>(k_cg_wg<512>)
                     : threads == 1024
                         ? reinterpret_cast<const void *>(k_cg_wg<1024>)
                         : nullptr;
    if (!fn) return hipErrorInvalidValue;
    if (lds > 65536) {
        // above the default limit of dynamic LDS per workgroup
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds));
        if (e != hipSuccess) return e;
    }
    switch (threads) {
    case 256:
        hipLaunchKernelGGL(k_cg_wg<256>, dim3(m), dim3(256), lds, s, d_sys, a);
        break;
    case 512:
        hipLaunchKernelGGL(k_cg_wg<512>, dim3(m), dim3(512), lds, s, d_sys, a);
        break;
    default:
        hipLaunchKernelGGL(k_cg_wg<1024>, dim3(m), dim3(1024), lds, s, d_sys,
                           a);
        break;
    }
    return hipGetLastError();
}

}  // namespace fs
