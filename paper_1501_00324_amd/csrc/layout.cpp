// Host-side layout builder: CSR validation, locality reordering, row
// grouping and the CSR-position -> slot map.
//
// The layout follows the row-grouped, column-interleaved idea of the paper
// (section "Development of Novel GPU Algorithms": rows sorted by length,
// grouped per warp, padded to the group's longest row, stored column-major;
// several lanes per row when a row is long, ELL-WARP v2 (K2); columns
// relabelled and sorted, K1r/K1rs).  Differences for gfx950: a group is one
// 64-lane wavefront, rows are only sorted inside windows (the locality
// order from reverse Cuthill-McKee is kept between windows because there is
// no texture cache to hide a scrambled x), and each lane loads two adjacent
// slots per access.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "host.h"

namespace fs {
namespace {

constexpr int64_t kRowChunk = 16384;

// Pattern of A + A^T without the diagonal, rows sorted.  Only used for the
// reordering, never for arithmetic.
struct Graph {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    int32_t n = 0;
    int32_t deg(int32_t v) const { return int32_t(rp[v + 1] - rp[v]); }
};

// True when every row is sorted and the pattern looks symmetric: equal row
// and column counts, and equal fingerprints sum h(i) g(c) and sum h(c) g(i)
// over the entries (i, c) (wrap-around 64-bit sums of a mixing hash; equal
// for every symmetric pattern, unequal for a non-symmetric one except with
// negligible probability).  Only the ordering uses the graph, and any
// permutation is a valid layout, so a false positive could cost locality,
// never correctness.
uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

bool sorted_symmetric_pattern(int32_t n, const int32_t *rowptr,
                              const int32_t *col)
{
    const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
    std::vector<uint64_t> s1(size_t(nch), 0), s2(size_t(nch), 0);
    std::vector<char> sorted(size_t(nch), 1);
    // column counts, in parallel over row chunks (relaxed atomic adds: the
    // counts do not depend on the order of the additions)
    std::vector<int64_t> colcount(size_t(n), 0);
    parallel_chunks(nch, [&](int64_t c) {
        const int64_t k1 =
            rowptr[std::min<int64_t>(n, (c + 1) * kRowChunk)];
        for (int64_t k = rowptr[c * kRowChunk]; k < k1; ++k)
            __atomic_fetch_add(&colcount[size_t(col[k])], int64_t(1),
                               __ATOMIC_RELAXED);
    });
    parallel_chunks(nch, [&](int64_t c) {
        uint64_t a = 0, b = 0;
        const int32_t i1 = int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
        for (int32_t i = int32_t(c * kRowChunk); i < i1; ++i) {
            if (colcount[size_t(i)] != rowptr[i + 1] - rowptr[i])
                sorted[size_t(c)] = 0;
            const uint64_t hi = mix64(uint64_t(i)), gi = mix64(~uint64_t(i));
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int32_t cc = col[k];
                if (k > rowptr[i] && col[k - 1] >= cc) sorted[size_t(c)] = 0;
                a += hi * mix64(~uint64_t(cc));
                b += mix64(uint64_t(cc)) * gi;
            }
        }
        s1[size_t(c)] = a;
        s2[size_t(c)] = b;
    });
    uint64_t a = 0, b = 0;
    for (int64_t c = 0; c < nch; ++c) {
        if (!sorted[size_t(c)]) return false;
        a += s1[size_t(c)];
        b += s2[size_t(c)];
    }
    return a == b;
}

Graph symmetric_graph(int32_t n, const int32_t *rowptr, const int32_t *col)
{
    if (sorted_symmetric_pattern(n, rowptr, col)) {
        // the pattern of A without the diagonal
        Graph g;
        g.n = n;
        g.rp.assign(size_t(n) + 1, 0);
        const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
        parallel_chunks(nch, [&](int64_t c) {
            const int32_t i1 =
                int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
            for (int32_t i = int32_t(c * kRowChunk); i < i1; ++i) {
                int64_t m = 0;
                for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                    m += col[k] != i;
                g.rp[size_t(i) + 1] = m;
            }
        });
        for (int32_t i = 0; i < n; ++i) g.rp[i + 1] += g.rp[i];
        g.ci.resize(size_t(g.rp[n]));
        parallel_chunks(nch, [&](int64_t c) {
            const int32_t i1 =
                int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
            for (int32_t i = int32_t(c * kRowChunk); i < i1; ++i) {
                int64_t o = g.rp[i];
                for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                    if (col[k] != i) g.ci[size_t(o++)] = col[k];
            }
        });
        return g;
    }
    // transpose pattern by counting sort: rows of T come out sorted
    std::vector<int64_t> tp(size_t(n) + 1, 0);
    int64_t nnz = rowptr[n];
    for (int64_t k = 0; k < nnz; ++k) tp[size_t(col[k]) + 1]++;
    for (int32_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
    std::vector<int32_t> ti(static_cast<size_t>(nnz));
    {
        std::vector<int64_t> pos(tp.begin(), tp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                ti[size_t(pos[col[k]]++)] = i;
    }
    // merge row i of A (sorted copy) with row i of T, dropping i itself:
    // sizes first, then the rows, both in parallel over row chunks
    Graph g;
    g.n = n;
    g.rp.assign(size_t(n) + 1, 0);
    const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
    auto merge_row = [&](int32_t i, std::vector<int32_t> &row, int32_t *out) {
        row.assign(col + rowptr[i], col + rowptr[i + 1]);
        if (!std::is_sorted(row.begin(), row.end()))
            std::sort(row.begin(), row.end());
        size_t a = 0, b = size_t(tp[i]), be = size_t(tp[i + 1]);
        int32_t last = -1;
        int64_t m = 0;
        while (a < row.size() || b < be) {
            int32_t v;
            if (b >= be || (a < row.size() && row[a] <= ti[b])) v = row[a++];
            else v = ti[b++];
            if (v != last && v != i) {
                if (out) out[m] = v;
                ++m;
            }
            last = v;
        }
        return m;
    };
    parallel_chunks(nch, [&](int64_t c) {
        std::vector<int32_t> row;
        const int32_t i1 = int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
        for (int32_t i = int32_t(c * kRowChunk); i < i1; ++i)
            g.rp[size_t(i) + 1] = merge_row(i, row, nullptr);
    });
    for (int32_t i = 0; i < n; ++i) g.rp[i + 1] += g.rp[i];
    g.ci.resize(size_t(g.rp[n]));
    parallel_chunks(nch, [&](int64_t c) {
        std::vector<int32_t> row;
        const int32_t i1 = int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
        for (int32_t i = int32_t(c * kRowChunk); i < i1; ++i)
            merge_row(i, row, g.ci.data() + g.rp[i]);
    });
    return g;
}

// Breadth-first levels from r over the component; returns eccentricity and
// fills `last` with the last level.
int32_t bfs_levels(const Graph &g, int32_t r, std::vector<int32_t> &stamp,
                   int32_t tag, std::vector<int32_t> &queue,
                   std::vector<int32_t> &last)
{
    queue.clear();
    queue.push_back(r);
    stamp[r] = tag;
    size_t head = 0, level_start = 0;
    int32_t ecc = 0;
    while (true) {
        size_t level_end = queue.size();
        while (head < level_end) {
            int32_t u = queue[head++];
            for (int64_t k = g.rp[u]; k < g.rp[u + 1]; ++k) {
                int32_t v = g.ci[size_t(k)];
                if (stamp[v] != tag) {
                    stamp[v] = tag;
                    queue.push_back(v);
                }
            }
        }
        if (queue.size() == level_end) {
            last.assign(queue.begin() + long(level_start),
                        queue.begin() + long(level_end));
            return ecc;
        }
        level_start = level_end;
        ++ecc;
    }
}

// Reverse Cuthill-McKee (Cuthill & McKee 1969; George & Liu's
// pseudo-peripheral start).  order[i] = old index of new index i.
std::vector<int32_t> rcm_order(const Graph &g)
{
    const int32_t n = g.n;
    std::vector<int32_t> order;
    order.reserve(size_t(n));
    std::vector<char> visited(size_t(n), 0);
    std::vector<int32_t> stamp(size_t(n), -1), queue, last, nb;
    int32_t tag = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (visited[s]) continue;
        // pseudo-peripheral node of s's component
        int32_t r = s;
        int32_t ecc = bfs_levels(g, r, stamp, tag++, queue, last);
        for (int it = 0; it < 8; ++it) {
            int32_t best = last[0];
            for (int32_t v : last)
                if (g.deg(v) < g.deg(best)) best = v;
            int32_t e2 = bfs_levels(g, best, stamp, tag++, queue, last);
            if (e2 <= ecc) break;
            r = best;
            ecc = e2;
        }
        // Cuthill-McKee from r: neighbours in increasing degree
        size_t head = order.size();
        order.push_back(r);
        visited[r] = 1;
        while (head < order.size()) {
            int32_t u = order[head++];
            nb.clear();
            for (int64_t k = g.rp[u]; k < g.rp[u + 1]; ++k) {
                int32_t v = g.ci[size_t(k)];
                if (!visited[v]) {
                    visited[v] = 1;
                    nb.push_back(v);
                }
            }
            std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return g.deg(a) < g.deg(b);
            });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Reverse Cuthill-McKee on the graph compressed by supervariables:
// consecutive vertices with identical closed neighbourhoods (the DOFs of
// one mesh node in an elasticity matrix) become one vertex, ordered as a
// unit with its members kept in ascending order.  The search then visits
// nine times fewer edges for three DOFs per node; without such vertices the
// graph is used as it is.
std::vector<int32_t> rcm_order_compressed(const Graph &g)
{
    const int32_t n = g.n;
    if (n == 0) return {};
    // same[i]: N[i-1] + {i-1} == N[i] + {i}, i.e. i-1 and i are adjacent
    // and their other neighbours agree
    std::vector<char> same(size_t(n), 0);
    const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
    parallel_chunks(nch, [&](int64_t c) {
        const int32_t i1 = int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
        for (int32_t i = std::max<int32_t>(1, int32_t(c * kRowChunk)); i < i1;
             ++i) {
            const int32_t a = i - 1, b = i;
            if (g.deg(a) != g.deg(b)) continue;
            int64_t pa = g.rp[a], ea = g.rp[a + 1];
            int64_t pb = g.rp[b], eb = g.rp[b + 1];
            bool has_b = false, has_a = false, eq = true;
            while (eq) {
                while (pa < ea && g.ci[size_t(pa)] == b) { has_b = true; ++pa; }
                while (pb < eb && g.ci[size_t(pb)] == a) { has_a = true; ++pb; }
                if (pa >= ea || pb >= eb) {
                    eq = pa >= ea && pb >= eb;
                    break;
                }
                eq = g.ci[size_t(pa)] == g.ci[size_t(pb)];
                ++pa;
                ++pb;
            }
            same[size_t(i)] = eq && has_a && has_b;
        }
    });
    std::vector<int32_t> sv(static_cast<size_t>(n));
    std::vector<int32_t> first;
    first.reserve(size_t(n) + 1);
    for (int32_t i = 0; i < n; ++i) {
        if (i == 0 || !same[size_t(i)]) first.push_back(i);
        sv[size_t(i)] = int32_t(first.size()) - 1;
    }
    const int32_t m = int32_t(first.size());
    first.push_back(n);
    if (m == n) return rcm_order(g);
    // quotient graph from each supervariable's first member (sv is
    // monotone, so mapped rows stay sorted and duplicates are adjacent)
    Graph q;
    q.n = m;
    q.rp.assign(size_t(m) + 1, 0);
    auto qrow = [&](int32_t s, int32_t *out) {
        const int32_t r = first[size_t(s)];
        int32_t last = -1;
        int64_t k = 0;
        for (int64_t e = g.rp[r]; e < g.rp[r + 1]; ++e) {
            const int32_t t = sv[size_t(g.ci[size_t(e)])];
            if (t == s || t == last) continue;
            if (out) out[k] = t;
            ++k;
            last = t;
        }
        return k;
    };
    const int64_t qch = (m + kRowChunk - 1) / kRowChunk;
    parallel_chunks(qch, [&](int64_t c) {
        const int32_t s1 = int32_t(std::min<int64_t>(m, (c + 1) * kRowChunk));
        for (int32_t s = int32_t(c * kRowChunk); s < s1; ++s)
            q.rp[size_t(s) + 1] = qrow(s, nullptr);
    });
    for (int32_t s = 0; s < m; ++s) q.rp[s + 1] += q.rp[s];
    q.ci.resize(size_t(q.rp[m]));
    parallel_chunks(qch, [&](int64_t c) {
        const int32_t s1 = int32_t(std::min<int64_t>(m, (c + 1) * kRowChunk));
        for (int32_t s = int32_t(c * kRowChunk); s < s1; ++s)
            qrow(s, q.ci.data() + q.rp[s]);
    });
    const std::vector<int32_t> qo = rcm_order(q);
    std::vector<int32_t> order;
    order.reserve(size_t(n));
    for (int32_t s : qo)
        for (int32_t v = first[size_t(s)]; v < first[size_t(s) + 1]; ++v)
            order.push_back(v);
    return order;
}

// Mean |row - col| over the entries; partial sums per fixed row chunk added
// in chunk order, so the value does not depend on the thread count.
double mean_band(int32_t n, const int32_t *rowptr, const int32_t *col,
                 const int32_t *iperm)
{
    int64_t nnz = rowptr[n];
    if (nnz == 0) return 0.0;
    const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
    std::vector<double> part(size_t(nch), 0.0);
    parallel_chunks(nch, [&](int64_t c) {
        double s = 0.0;
        const int32_t i1 = int32_t(std::min<int64_t>(n, (c + 1) * kRowChunk));
        for (int32_t i = int32_t(c * kRowChunk); i < i1; ++i) {
            int64_t ri = iperm ? iperm[i] : i;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                int64_t cc = iperm ? iperm[col[k]] : col[k];
                s += double(ri > cc ? ri - cc : cc - ri);
            }
        }
        part[size_t(c)] = s;
    });
    double s = 0.0;
    for (double v : part) s += v;
    return s / double(nnz);
}

bool is_pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

fs_status layout_check_rowptr(int32_t n_rows, int64_t nnz,
                              const int32_t *rowptr)
{
    // CSR arrays of values, column indices and row offsets (paper: section
    // "Description of Current GPU Methods")
    if (rowptr[0] != 0)
        return set_error(FS_E_BAD_CSR, "rowptr[0] = %d, expected 0", rowptr[0]);
    for (int32_t i = 0; i < n_rows; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return set_error(FS_E_BAD_CSR, "rowptr decreases at row %d", i);
    if (int64_t(rowptr[n_rows]) != nnz)
        return set_error(FS_E_BAD_CSR, "rowptr[n] = %d but nnz = %lld",
                         rowptr[n_rows], (long long)nnz);
    return FS_OK;
}

fs_status layout_params(const fs_csr_opts &o, LayoutParams &p)
{
    p.threshold = o.threshold > 0 ? o.threshold : 48;
    p.tmin = o.lanes_min > 0 ? o.lanes_min : 1;
    p.tmax = o.lanes_max > 0 ? o.lanes_max : 64;
    if (!is_pow2(p.tmin) || !is_pow2(p.tmax) || p.tmin > p.tmax ||
        p.tmax > kWave)
        return set_error(FS_E_ARG, "lanes_min/lanes_max must be powers of "
                         "two with 1 <= min <= max <= 64");
    if (o.vec < 0 || o.vec > 2)
        return set_error(FS_E_ARG, "vec must be 0 (auto), 1 or 2");
    if (o.index_bits != 0 && o.index_bits != 32)
        return set_error(FS_E_ARG, "index_bits must be 0 (auto) or 32");
    return FS_OK;
}

bool layout_order_reads_columns(int32_t n_rows, int32_t n_cols,
                                const fs_csr_opts &o)
{
    return (o.reorder == FS_REORDER_RCM || o.reorder == FS_REORDER_AUTO) &&
           n_rows == n_cols && n_rows > 0;
}

fs_status layout_order(int32_t n_rows, int32_t n_cols, const int32_t *rowptr,
                       const int32_t *col, const fs_csr_opts &o,
                       HostLayout &L)
{
    const bool square = n_rows == n_cols;
    L.perm.resize(size_t(n_rows));
    std::iota(L.perm.begin(), L.perm.end(), 0);
    L.reorder = FS_REORDER_NONE;
    if (o.reorder == FS_REORDER_USER) {
        if (!o.perm) return set_error(FS_E_ARG, "FS_REORDER_USER needs perm");
        std::vector<char> seen(size_t(n_rows), 0);
        for (int32_t i = 0; i < n_rows; ++i) {
            int32_t v = o.perm[i];
            if (v < 0 || v >= n_rows || seen[v])
                return set_error(FS_E_ARG, "perm is not a permutation");
            seen[v] = 1;
            L.perm[i] = v;
        }
        L.reorder = FS_REORDER_USER;
    } else if (o.reorder == FS_REORDER_RCM || o.reorder == FS_REORDER_AUTO) {
        if (!square) {
            if (o.reorder == FS_REORDER_RCM)
                return set_error(FS_E_NOT_SQUARE,
                                 "RCM reordering needs a square matrix");
        } else if (n_rows > 0) {
            Graph g = symmetric_graph(n_rows, rowptr, col);
            std::vector<int32_t> ord = rcm_order_compressed(g);
            if (o.reorder == FS_REORDER_RCM) {
                L.perm = ord;
                L.reorder = FS_REORDER_RCM;
            } else {
                std::vector<int32_t> inv(static_cast<size_t>(n_rows));
                for (int32_t i = 0; i < n_rows; ++i) inv[ord[i]] = i;
                double b0 = mean_band(n_rows, rowptr, col, nullptr);
                double b1 = mean_band(n_rows, rowptr, col, inv.data());
                if (b1 < 0.8 * b0) {
                    L.perm = ord;
                    L.reorder = FS_REORDER_RCM;
                }
            }
        }
    } else if (o.reorder != FS_REORDER_NONE) {
        return set_error(FS_E_ARG, "unknown reorder option %d", o.reorder);
    }
    return FS_OK;
}

fs_status layout_groups(int32_t n_rows, int32_t n_cols, const int32_t *rowptr,
                        const fs_csr_opts &o, const LayoutParams &prm,
                        HostLayout &L)
{
    const int32_t threshold = prm.threshold, tmin = prm.tmin, tmax = prm.tmax;
    // ---- longest-first inside windows (stable, keeps locality order),
    // then row groups: one wavefront, T lanes per row, 64/T rows
    struct Raw { int32_t row0, rows, w, lt; };
    struct Plan {
        std::vector<int32_t> perm;
        std::vector<Raw> raw;
        int64_t slots1 = 0, slots2 = 0;
    };
    // row lengths in the initial order, read once: the window sorts and the
    // group cut below touch only this contiguous array
    std::vector<int32_t> len0(static_cast<size_t>(n_rows));
    parallel_chunks((n_rows + kRowChunk - 1) / kRowChunk, [&](int64_t c) {
        const int64_t i1 = std::min<int64_t>(n_rows, (c + 1) * kRowChunk);
        for (int64_t i = c * kRowChunk; i < i1; ++i) {
            const int32_t r = L.perm[size_t(i)];
            len0[size_t(i)] = rowptr[r + 1] - rowptr[r];
        }
    });
    auto make_plan = [&](int32_t window, Plan &P) {
        P.perm = L.perm;
        std::vector<int32_t> len = len0;      // lengths in the plan's order
        if (window > 1) {
            const int64_t nw = (n_rows + window - 1) / window;
            parallel_chunks(nw, [&](int64_t w) {
                const int64_t w0 = w * window;
                const int32_t m = int32_t(std::min<int64_t>(n_rows, w0 + window) - w0);
                std::vector<int32_t> ix(static_cast<size_t>(m)),
                    pv(static_cast<size_t>(m)), lv(static_cast<size_t>(m));
                std::iota(ix.begin(), ix.end(), 0);
                const int32_t *lw = len.data() + w0;
                std::stable_sort(ix.begin(), ix.end(), [&](int32_t a, int32_t b) {
                    return lw[a] > lw[b];
                });
                for (int32_t j = 0; j < m; ++j) {
                    pv[size_t(j)] = P.perm[size_t(w0 + ix[size_t(j)])];
                    lv[size_t(j)] = lw[ix[size_t(j)]];
                }
                std::copy(pv.begin(), pv.end(), P.perm.begin() + w0);
                std::copy(lv.begin(), lv.end(), len.begin() + w0);
            });
        }
        P.raw.clear();
        P.slots1 = P.slots2 = 0;
        for (int32_t i = 0; i < n_rows;) {
            int32_t T = tmin, rows = 0, w = 0;
            while (true) {
                rows = std::min<int32_t>(kWave / T, n_rows - i);
                int32_t maxlen = 0;
                for (int32_t j = 0; j < rows; ++j)
                    maxlen = std::max(maxlen, len[size_t(i + j)]);
                w = (maxlen + T - 1) / T;
                if (w <= threshold || T >= tmax) break;
                T *= 2;
            }
            int32_t lt = 0;
            while ((1 << lt) < T) ++lt;
            P.raw.push_back(Raw{i, rows, w, lt});
            P.slots1 += int64_t(w) * kWave;
            P.slots2 += int64_t((w + 1) / 2 * 2) * kWave;
            i += rows;
        }
    };
    Plan plan;
    if (o.sort_window > 0) {
        make_plan(o.sort_window, plan);
    } else {
        // auto window: sorting within wider windows lowers the padding of
        // matrices whose row lengths vary a lot locally (high-degree
        // nodes), at some cost in locality; take the narrowest window whose
        // slot count is within 2% of the fewest
        const int32_t cand[] = {256, 1024, 4096, 16384};
        std::vector<Plan> plans(4);
        int64_t best = INT64_MAX;
        for (int c = 0; c < 4; ++c) {
            make_plan(cand[c], plans[size_t(c)]);
            best = std::min(best, plans[size_t(c)].slots1);
            if (cand[c] >= n_rows) break;
        }
        for (int c = 0; c < 4; ++c)
            if (!plans[size_t(c)].raw.empty() || n_rows == 0)
                if (double(plans[size_t(c)].slots1) <= 1.02 * double(best)) {
                    plan = std::move(plans[size_t(c)]);
                    break;
                }
    }
    L.perm = std::move(plan.perm);
    L.iperm.assign(size_t(n_rows), 0);
    L.identity = true;
    for (int32_t i = 0; i < n_rows; ++i) {
        L.iperm[L.perm[i]] = i;
        if (L.perm[i] != i) L.identity = false;
    }
    L.symmetric_relabel = n_rows == n_cols;
    const std::vector<Raw> &raw = plan.raw;
    const int64_t slots1 = plan.slots1, slots2 = plan.slots2;
    // two slots per load halves the load instructions; one slot per load
    // avoids rounding each lane's slot count up to even.  Auto keeps the
    // wide loads unless they cost more than 6% extra padded slots.
    L.vec = o.vec ? o.vec : (double(slots2) <= 1.06 * double(slots1) ? 2 : 1);
    const int32_t V = L.vec;
    L.groups.clear();
    std::fill(std::begin(L.groups_by_lanes), std::end(L.groups_by_lanes), 0);
    int64_t slots = 0;
    for (const Raw &r : raw) {
        const int32_t width = (r.w + V - 1) / V * V;
        if (slots / kWave >= INT32_MAX)
            return set_error(FS_E_UNSUPPORTED, "layout too large");
        L.groups.push_back(Group{int32_t(slots / kWave), r.row0, r.rows,
                                 width | (r.lt << 24)});
        L.groups_by_lanes[r.lt]++;
        slots += int64_t(width) * kWave;
    }
    if (slots >= INT32_MAX)
        return set_error(FS_E_UNSUPPORTED,
                         "more than 2^31 padded slots (%lld)",
                         (long long)slots);
    L.slots = slots;
    return FS_OK;
}

fs_status build_layout(int32_t n_rows, int32_t n_cols, int64_t nnz,
                       const int32_t *rowptr, const int32_t *col,
                       const fs_csr_opts &o, HostLayout &L)
{
    FS_TRY(layout_check_rowptr(n_rows, nnz, rowptr));
    for (int64_t k = 0; k < nnz; ++k)
        if (col[k] < 0 || col[k] >= n_cols)
            return set_error(FS_E_BAD_CSR, "column %d out of range at %lld",
                             col[k], (long long)k);
    LayoutParams prm;
    FS_TRY(layout_params(o, prm));
    FS_TRY(layout_order(n_rows, n_cols, rowptr, col, o, L));
    FS_TRY(layout_groups(n_rows, n_cols, rowptr, o, prm, L));
    const bool square = n_rows == n_cols;
    L.band_before = square ? mean_band(n_rows, rowptr, col, nullptr) : 0.0;
    L.band_after = square ? mean_band(n_rows, rowptr, col, L.iperm.data())
                          : 0.0;
    const int64_t slots = L.slots;
    const int32_t V = L.vec;

    // ---- slot columns and the CSR-position -> slot map (groups are
    // independent: parallel over chunks of groups; the first duplicate
    // column in group order is reported)
    L.slot_col.assign(size_t(slots), -1);
    L.map.assign(size_t(nnz), -1);
    constexpr int64_t kGroupChunk = 1024;
    const int64_t ngr = int64_t(L.groups.size());
    const int64_t gch = (ngr + kGroupChunk - 1) / kGroupChunk;
    std::vector<int64_t> dup(size_t(gch), -1);   // first bad CSR position
    parallel_chunks(gch, [&](int64_t c) {
        std::vector<std::pair<int32_t, int32_t>> ent;  // (layout col, k)
        const int64_t g1 = std::min(ngr, (c + 1) * kGroupChunk);
        for (int64_t gi = c * kGroupChunk; gi < g1; ++gi) {
            const Group &g = L.groups[size_t(gi)];
            const int32_t lt = g.width_lt >> 24, T = 1 << lt;
            const int64_t base = int64_t(g.base64) * kWave;
            for (int32_t rr = 0; rr < g.nrows; ++rr) {
                const int32_t orow = L.perm[g.row0 + rr];
                const int32_t k0 = rowptr[orow], k1 = rowptr[orow + 1];
                ent.clear();
                for (int32_t k = k0; k < k1; ++k) {
                    int32_t cc = L.symmetric_relabel ? L.iperm[col[k]] : col[k];
                    ent.emplace_back(cc, k - k0);
                }
                std::sort(ent.begin(), ent.end());
                for (size_t e = 1; e < ent.size(); ++e)
                    if (ent[e].first == ent[e - 1].first) {
                        dup[size_t(c)] = k0 + ent[e].second;
                        return;
                    }
                for (size_t e = 0; e < ent.size(); ++e) {
                    const int32_t lane = rr * T + int32_t(e) % T;
                    const int32_t sl = int32_t(e) / T;
                    const int64_t idx = base + int64_t(sl / V) * kWave * V +
                                        int64_t(lane) * V + sl % V;
                    L.slot_col[size_t(idx)] = ent[e].first;
                    L.map[size_t(k0 + ent[e].second)] = int32_t(idx);
                }
            }
        }
    });
    for (int64_t c = 0; c < gch; ++c)
        if (dup[size_t(c)] >= 0) {
            const int64_t k = dup[size_t(c)];
            const int32_t row = int32_t(std::upper_bound(rowptr, rowptr + n_rows + 1,
                                                         int32_t(k)) - rowptr) - 1;
            return set_error(FS_E_BAD_CSR, "duplicate column %d in row %d",
                             col[k], row);
        }

    // ---- 16-bit column offsets when every group's columns fit: the index
    // stream shrinks from 4 to 2 bytes per slot
    L.index_bits = 32;
    L.slot_c16.clear();
    L.gbase.clear();
    if (o.index_bits == 0 && ngr > 0) {
        std::vector<int32_t> lo(size_t(ngr), 0), hi(size_t(ngr), -1);
        parallel_chunks(gch, [&](int64_t c) {
            const int64_t g1 = std::min(ngr, (c + 1) * kGroupChunk);
            for (int64_t gi = c * kGroupChunk; gi < g1; ++gi) {
                const Group &g = L.groups[size_t(gi)];
                const int64_t b0 = int64_t(g.base64) * kWave;
                const int64_t b1 = b0 + int64_t(g.width_lt & 0xffffff) * kWave;
                int32_t mn = INT32_MAX, mx = -1;
                for (int64_t e = b0; e < b1; ++e) {
                    const int32_t cc = L.slot_col[size_t(e)];
                    if (cc < 0) continue;
                    mn = std::min(mn, cc);
                    mx = std::max(mx, cc);
                }
                lo[size_t(gi)] = mx < 0 ? 0 : mn;
                hi[size_t(gi)] = mx;
            }
        });
        bool fits = true;
        for (int64_t gi = 0; gi < ngr && fits; ++gi)
            fits = hi[size_t(gi)] - lo[size_t(gi)] < 0xffff;
        if (fits) {
            L.index_bits = 16;
            L.gbase = lo;
            L.slot_c16.assign(size_t(slots), 0xffff);
            parallel_chunks(gch, [&](int64_t c) {
                const int64_t g1 = std::min(ngr, (c + 1) * kGroupChunk);
                for (int64_t gi = c * kGroupChunk; gi < g1; ++gi) {
                    const Group &g = L.groups[size_t(gi)];
                    const int64_t b0 = int64_t(g.base64) * kWave;
                    const int64_t b1 =
                        b0 + int64_t(g.width_lt & 0xffffff) * kWave;
                    for (int64_t e = b0; e < b1; ++e) {
                        const int32_t cc = L.slot_col[size_t(e)];
                        if (cc >= 0)
                            L.slot_c16[size_t(e)] =
                                uint16_t(cc - lo[size_t(gi)]);
                    }
                }
            });
        }
    }
    return FS_OK;
}

}  // namespace fs
