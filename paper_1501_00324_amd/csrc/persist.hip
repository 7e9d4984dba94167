// Whole-solve persistent CG: one cooperative launch runs the Jacobi-PCG
// iteration of one system (the solver the paper runs around its SpMV) to
// the end, so the solve is ordered on the caller's stream like any kernel
// and needs no host round trip per chunk of iterations.
//
// Every block owns a contiguous range of row groups (products) and of rows
// (vector steps).  Grid-wide barriers separate the phases; after each
// barrier every block sums the per-block partials itself, in one fixed
// order, so all blocks hold bitwise the same scalars (alpha, beta, the
// residual norms) and take the same branch at every decision: the number
// of barriers is the same in every block.
//
// The barrier is a counter that only grows: barrier number k is passed
// once the counter has reached (k + 1) * gridDim.x.  One thread per block
// arrives with a device-scope release (the block's writes, ordered before
// it by __syncthreads, become visible to every XCD) and waits with
// device-scope acquire loads; the cooperative launch keeps every block
// resident, so the wait ends.  On MI355X this costs 7-12 us per barrier
// with one block per CU, against 27 us for the cooperative-groups grid
// barrier at that size and 50-58 us at two blocks per CU (measured in
// isolation), so the grid has one block per CU.
//
// Partials live in two regions used in turn by successive reductions.
// Every write of partials is followed by a grid barrier, and a block
// reaches that barrier only after it has read the previous reduction's
// sums; so when reduction k+2 writes region (k mod 2), every block has
// left get_sums of reduction k (it has passed the barrier of reduction
// k+1).  With one region a fast block could overwrite partials that a slow
// block is still summing.  Per iteration:
//   w = A z; p = z + beta p,        |
//   q = w + beta q (= A p); p.q     | barrier | gamma, alpha
//   x += alpha p, r -= alpha q,     |
//   z = D^-1 r, partials r.z, r.r   | barrier | rz, rr, beta
// (the product gathers z rather than p, so the direction update needs no
// phase of its own: q follows the same recurrence as p; the first
// iteration takes p = z, q = A z)
// When |r| meets the tolerance, b - A x is recomputed (one more product);
// if it misses, it replaces r and the iteration continues.
#include <algorithm>

#include "device.h"

namespace fs {
namespace {

// 1024-thread blocks (16 wavefronts, one block per CU at this kernel's
// register use): a grid barrier costs roughly a fixed time per arriving
// block, so fewer, larger blocks make each barrier cheaper.
constexpr int kPB = 1024;
constexpr int kPW = kPB / kWave;

struct PcgArgs {
    const Group *groups;
    const double *val;
    const int32_t *col;            // 32-bit columns (diagonal search)
    const void *cstream;           // column stream of the products
    const int32_t *gbase;          // group bases of 16-bit offsets, or NULL
    int32_t n, ngroups;
    const double *b;               // layout numbering
    double *x, *r, *p, *q, *dinv;  // dinv NULL: no preconditioner
    double *z;                     // D^-1 r
    double *part;                  // 2 regions of 3 * kPersistMaxBlocks
    unsigned *bar;                 // barrier counter, 0 at launch
    fs_cg_info *info;              // device copy of the result
    double rtol, nnz, clock_khz;
    int32_t maxit, x_zero;
};

// Block partial sums of NJ values -> part[j * nb + b].
template <int NJ>
__device__ __forceinline__ void put_partials(const double (&v)[NJ],
                                             double *part, int nb, int b)
{
    __shared__ double sh[3][kPW];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const double s = wave_sum(v[j]);
        if (lane == 0) sh[j][w] = s;
    }
    __syncthreads();
    if (int(threadIdx.x) < NJ) {
        double t = 0.0;
        for (int i = 0; i < kPW; ++i) t += sh[threadIdx.x][i];
        part[long(threadIdx.x) * nb + b] = t;
    }
    __syncthreads();
}

// After a grid barrier: the NJ grid-wide sums, identical in every block.
// The partials are read with device-scope loads (never a stale line of
// this CU's vector cache), so every block sees the same values and takes
// the same branches -- the barrier count cannot diverge between blocks.
template <int NJ>
__device__ __forceinline__ void get_sums(double *part, int nb,
                                         double (&out)[NJ])
{
    __shared__ double res[3];
    if (threadIdx.x < kWave) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            double s = 0.0;
            for (int i = threadIdx.x; i < nb; i += kWave)
                s += __hip_atomic_load(part + j * nb + i, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            s = wave_sum(s);
            if (threadIdx.x == 0) res[j] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) out[j] = res[j];
    __syncthreads();
}

// b - A x for the rows of this block's groups (A x skipped when XZ); calls
// f(row, r_row) on the owner lane of every row.
template <int V, bool N, bool XZ, class F>
__device__ __forceinline__ void residual_rows(const PcgArgs &a, int g0, int g1,
                                              F f)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int g = g0 + int(threadIdx.x >> 6); g < g1; g += kPW) {
        const Group gd = load_group(gbl(a.groups), __builtin_amdgcn_readfirstlane(g));
        const int lt = gd.width_lt >> 24;
        double ax = 0.0;
        if (!XZ)
            ax = row_reduce(group_lane_sum_plain<V, N, 16>(
                                gd, lane, gbl(a.val), gbl(a.cstream),
                                N ? load_gbase(gbl(a.gbase), g) : 0,
                                gbl(a.x)),
                            lt);
        const int r = lane >> lt;
        if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
            const int row = gd.row0 + r;
            f(row, a.b[row] - ax);
        }
    }
}

enum { P_RUNNING = 0, P_CONVERGED = 1, P_BREAKDOWN = 2, P_MAXIT = 3 };

// Barrier number k of the grid (k counts this block's barriers; every block
// passes the same sequence).
__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned &k)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = (k + 1) * gridDim.x;
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE,
                                 __HIP_MEMORY_SCOPE_AGENT) < target)
            __builtin_amdgcn_s_sleep(1);
    }
    ++k;
    __syncthreads();
}

// Region of the partials for the next reduction (alternates; see the top).
__device__ __forceinline__ double *next_region(double *part, int &k)
{
    double *p = part + (k & 1) * (3 * kPersistMaxBlocks);
    ++k;
    return p;
}

template <int V, bool N>
__global__ __launch_bounds__(kPB) void k_cg_persistent(const PcgArgs a)
{
    unsigned nbar = 0;             // barriers passed
    const long t_start = wall_clock64();
    const int nb = int(gridDim.x);
    const int lb = xcd_remap(int(blockIdx.x), nb);
    const int g0 = int(long(lb) * a.ngroups / nb);
    const int g1 = int(long(lb + 1) * a.ngroups / nb);
    const int r0 = int(long(lb) * a.n / nb), r1 = int(long(lb + 1) * a.n / nb);
    const int lane = threadIdx.x & (kWave - 1);
    double *D = a.dinv;

    // Jacobi scaling for this block's groups (the same rows the start pass
    // below writes, so no barrier is needed in between)
    if (D) {
        for (int g = g0 + int(threadIdx.x >> 6); g < g1; g += kPW) {
            const Group gd =
                load_group(gbl(a.groups), __builtin_amdgcn_readfirstlane(g));
            const int lt = gd.width_lt >> 24, width = gd.width_lt & 0xffffff;
            const int r = lane >> lt, row = gd.row0 + r;
            const long base = long(gd.base64) * kWave;
            double d = 0.0;
            for (int s = 0; s < width; ++s) {
                const long idx = base + long(s / V) * kWave * V + lane * V + s % V;
                if (a.col[idx] == row) d += a.val[idx];
            }
            d = row_reduce(d, lt);
            if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows)
                D[row] = 1.0 / d;
        }
    }
    // start: r = b - A x, z = D^-1 r; |r|^2, r.z, |b|^2
    double v3[3] = {0.0, 0.0, 0.0};
    auto start = [&](int row, double ri) {
        const double zi = D ? D[row] * ri : ri;
        const double bi = a.b[row];
        a.r[row] = ri;
        a.z[row] = zi;
        v3[0] += ri * ri;
        v3[1] += ri * zi;
        v3[2] += bi * bi;
    };
    if (a.x_zero) residual_rows<V, N, true>(a, g0, g1, start);
    else residual_rows<V, N, false>(a, g0, g1, start);
    int red = 0;  // reductions so far (selects the partials region)
    double *pr = next_region(a.part, red);
    put_partials<3>(v3, pr, nb, lb);
    grid_barrier(a.bar, nbar);
    double s3[3];
    get_sums<3>(pr, nb, s3);
    const double bb = s3[2], tol2 = a.rtol * a.rtol * bb;
    double rho = s3[1], rr = s3[0], rr_true = s3[0];
    int status = P_RUNNING, it = 0, repl = 0;
    if (bb == 0.0) {
        // b = 0: x = 0 is the solution
        for (int i = r0 + int(threadIdx.x); i < r1; i += kPB) a.x[i] = 0.0;
        status = P_CONVERGED;
        rr_true = 0.0;
    } else if (rr <= tol2) {
        status = P_CONVERGED;
    } else if (!isfinite(rr) || !isfinite(rho)) {
        status = P_BREAKDOWN;
    }
    bool first = true;             // no previous search direction yet
    double beta = 0.0;
    while (status == P_RUNNING) {
        // the product gathers z: w = A z, and for this block's rows
        // p = z + beta p, q = w + beta q (= A p); p.q
        double v1[1] = {0.0};
        for (int g = g0 + int(threadIdx.x >> 6); g < g1; g += kPW) {
            const Group gd =
                load_group(gbl(a.groups), __builtin_amdgcn_readfirstlane(g));
            const int lt = gd.width_lt >> 24;
            const double wv =
                row_reduce(group_lane_sum_plain<V, N, 16>(
                               gd, lane, gbl(a.val), gbl(a.cstream),
                               N ? load_gbase(gbl(a.gbase), g) : 0,
                               gbl(a.z)),
                           lt);
            const int r = lane >> lt;
            if ((lane & ((1 << lt) - 1)) == 0 && r < gd.nrows) {
                const int row = gd.row0 + r;
                const double zi = a.z[row];
                const double pi = first ? zi : zi + beta * a.p[row];
                const double qi = first ? wv : wv + beta * a.q[row];
                a.p[row] = pi;
                a.q[row] = qi;
                v1[0] += pi * qi;
            }
        }
        pr = next_region(a.part, red);
        put_partials<1>(v1, pr, nb, lb);
        grid_barrier(a.bar, nbar);
        double s1[1];
        get_sums<1>(pr, nb, s1);
        const double gamma = s1[0];
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            status = P_BREAKDOWN;
            break;
        }
        const double alpha = rho / gamma;
        first = false;
        // x, r update; z = D^-1 r; r.z, r.r
        double v2[2] = {0.0, 0.0};
        for (int i = r0 + int(threadIdx.x); i < r1; i += kPB) {
            const double ri = a.r[i] - alpha * a.q[i];
            a.x[i] += alpha * a.p[i];
            a.r[i] = ri;
            const double zi = D ? D[i] * ri : ri;
            a.z[i] = zi;
            v2[0] += ri * zi;
            v2[1] += ri * ri;
        }
        pr = next_region(a.part, red);
        put_partials<2>(v2, pr, nb, lb);
        grid_barrier(a.bar, nbar);
        double s2[2];
        get_sums<2>(pr, nb, s2);
        ++it;
        double rz = s2[0];
        rr = s2[1];
        if (rr <= tol2) {
            // confirm against the true residual; replace r if it misses
            double w2[2] = {0.0, 0.0};
            residual_rows<V, N, false>(a, g0, g1, [&](int row, double ri) {
                a.r[row] = ri;
                const double zi = D ? D[row] * ri : ri;
                a.z[row] = zi;
                w2[0] += ri * zi;
                w2[1] += ri * ri;
            });
            pr = next_region(a.part, red);
            put_partials<2>(w2, pr, nb, lb);
            grid_barrier(a.bar, nbar);
            get_sums<2>(pr, nb, s2);
            rr_true = s2[1];
            if (rr_true <= tol2) {
                status = P_CONVERGED;
                break;
            }
            ++repl;
            rz = s2[0];
            rr = rr_true;
        } else if (!isfinite(rr)) {
            status = P_BREAKDOWN;
            break;
        }
        beta = rz / rho;
        if (!isfinite(beta)) {
            status = P_BREAKDOWN;
            break;
        }
        rho = rz;
        if (it >= a.maxit) {
            status = P_MAXIT;
            break;
        }
        // the next product gathers z, written before the last barrier; the
        // direction update p = z + beta p happens in it
    }
    if (status != P_CONVERGED) {
        // report the true residual of the returned x
        grid_barrier(a.bar, nbar);
        double w1[1] = {0.0};
        residual_rows<V, N, false>(a, g0, g1,
                                [&](int, double ri) { w1[0] += ri * ri; });
        pr = next_region(a.part, red);
        put_partials<1>(w1, pr, nb, lb);
        grid_barrier(a.bar, nbar);
        double s1[1];
        get_sums<1>(pr, nb, s1);
        rr_true = s1[0];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        fs_cg_info o;
        o.status = status == P_CONVERGED ? FS_OK
                   : status == P_MAXIT   ? FS_E_NOT_CONVERGED
                                         : FS_E_BREAKDOWN;
        o.iters = it;
        o.outer = 0;
        o.replacements = repl;
        o.cond_est = 0.0;
        o.relres = bb > 0.0 ? sqrt(rr_true / bb) : 0.0;
        o.ms = double(wall_clock64() - t_start) / a.clock_khz;
        o.bytes = double(it) * (12.0 * a.nnz + (D ? 104.0 : 88.0) * a.n) +
                  2.0 * (12.0 * a.nnz + 16.0 * a.n);
        *a.info = o;
    }
}

// Blocks of the grid: one per CU (the barrier's cost grows with the number
// of arriving blocks), provided one block fits on a CU at all.
template <int V, bool N> int max_coresident(int device)
{
    static int cached[64];
    if (device < 0 || device >= 64) return 0;
    if (cached[device] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, k_cg_persistent<V, N>, kPB, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                  device) != hipSuccess)
            return 0;
        cached[device] = per_cu >= 1 ? cus : 0;
    }
    return cached[device];
}

__global__ void k_zero_counter(unsigned *c) { *c = 0u; }

}  // namespace

int32_t persistent_blocks(const fs_csr *A)
{
    const int want = std::max((A->n_groups + kPW - 1) / kPW,
                              (A->n_rows + kPB - 1) / kPB);
    const bool n = A->d_col16 != nullptr;
    const int cap = A->host.vec == 1
                        ? (n ? max_coresident<1, true>(A->device)
                             : max_coresident<1, false>(A->device))
                        : (n ? max_coresident<2, true>(A->device)
                             : max_coresident<2, false>(A->device));
    return std::max(1, std::min({want, cap, kPersistMaxBlocks}));
}

hipError_t launch_cg_persistent(const fs_csr *A, int32_t nblocks,
                                const double *b, double *x, double *r,
                                double *p, double *q, double *z, double *dinv,
                                double *part, fs_cg_info *info, double rtol,
                                int32_t maxit, bool x_zero, hipStream_t s)
{
    int khz = 0;
    hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate,
                                         A->device);
    if (e != hipSuccess) return e;
    PcgArgs a;
    a.groups = A->d_groups;
    a.val = A->d_val;
    a.col = A->d_col;
    a.cstream = A->d_col16 ? static_cast<const void *>(A->d_col16)
                           : static_cast<const void *>(A->d_col);
    a.gbase = A->d_col16 ? A->d_gbase : nullptr;
    a.n = A->n_rows;
    a.ngroups = A->n_groups;
    a.b = b;
    a.x = x;
    a.r = r;
    a.p = p;
    a.q = q;
    a.z = z;
    a.dinv = dinv;
    a.part = part;
    a.bar = reinterpret_cast<unsigned *>(part + kPersistBarrierAt);
    a.info = info;
    a.rtol = rtol;
    a.nnz = double(A->nnz);
    a.clock_khz = double(khz > 0 ? khz : 100000);
    a.maxit = maxit;
    a.x_zero = x_zero ? 1 : 0;
    void *args[] = {&a};
    const bool n = A->d_col16 != nullptr;
    const void *fn =
        A->host.vec == 1
            ? (n ? reinterpret_cast<const void *>(k_cg_persistent<1, true>)
                 : reinterpret_cast<const void *>(k_cg_persistent<1, false>))
            : (n ? reinterpret_cast<const void *>(k_cg_persistent<2, true>)
                 : reinterpret_cast<const void *>(k_cg_persistent<2, false>));
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, a.bar);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(kPB), args, 0,
                                      s);
}

}  // namespace fs
