// Assembly plans (host side): which element entries sum into which output
// entry, in which order, and where the device kernel finds them.
//
// The paper assembles the global tangent matrix as an SpMV whose matrix has
// one row per global non-zero and the element contributions to that
// non-zero as entries, times a vector of ones (section "Description of
// Current GPU Methods"); writing the result directly in the solver's
// layout removes the value reorder (section "Cost of Reordering Matrix
// Values", conclusion).  Here the rows of that matrix are the value slots of
// the handle's layout (so the output lands where the products read it), an
// entry is the flat index of an element value, and a row's entries are kept
// in ascending flat index, i.e. element order.
#include <cstring>
#include <memory>
#include <new>

#include "host.h"

namespace fs {
namespace {

constexpr int64_t kWindow = 4096;       // output positions per sort window

// Uninitialised host array (whoever fills it writes every element).
template <class T> struct BufT {
    std::unique_ptr<T[]> p;
    size_t n = 0;
    void alloc(size_t m)
    {
        p.reset(m ? new T[m] : nullptr);
        n = m;
    }
    T *data() { return p.get(); }
    const T *data() const { return p.get(); }
    size_t size() const { return n; }
    bool empty() const { return n == 0; }
};
typedef BufT<int32_t> Buf;

// Host form of an AsmLdsPlan.
struct HostLds {
    bool built = false;
    int32_t nde = 0, rows = 0, region_max = 0;
    int64_t contrib = 0;
    Buf gdesc, bdesc, ea;
    BufT<uint16_t> off;
};

// Host form of an AsmPlan.
struct HostPlan {
    int64_t ntasks = 0, contrib = 0;
    Buf tpos, waves, aidx;
};

// One window of a plan, built independently of the others: its tasks (the
// output positions of the window with tag >= 0, longest list first, ties
// by position, padded with tasks of output -1 to whole waves), the widths
// of its waves and its interleaved index lists with window-local rows.
struct Window {
    std::vector<int32_t> tpos, width, aidx;
    int64_t contrib = 0;
    int64_t bad = -1;            // smallest element with a missing coupling
};

// Fill W from the (position, flat index) pairs of window [t0, t1).  Pairs of
// one position arrive in ascending flat index.
void finish_window(int64_t t0, int64_t t1, const int32_t *tag,
                   const std::vector<std::pair<int32_t, int32_t>> &pairs,
                   Window &W)
{
    const int64_t m = t1 - t0;
    std::vector<int32_t> cnt(size_t(m) + 1, 0);
    for (const auto &pr : pairs) ++cnt[size_t(pr.first - t0) + 1];
    std::vector<int32_t> len(cnt.begin() + 1, cnt.end());
    for (int64_t i = 0; i < m; ++i) cnt[size_t(i) + 1] += cnt[size_t(i)];
    std::vector<int32_t> lst(pairs.size());
    {
        std::vector<int32_t> cur(cnt.begin(), cnt.end() - 1);
        for (const auto &pr : pairs)       // stable: keeps ascending order
            lst[size_t(cur[size_t(pr.first - t0)]++)] = pr.second;
    }
    std::vector<int32_t> order;
    order.reserve(size_t(m) + kWave);
    for (int64_t i = 0; i < m; ++i)
        if (!tag || tag[t0 + i] >= 0) order.push_back(int32_t(i));
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return len[size_t(a)] > len[size_t(b)];
    });
    const size_t nt = order.size();
    const size_t ntp = (nt + kWave - 1) / kWave * kWave;
    W.tpos.assign(ntp, -1);
    for (size_t k = 0; k < nt; ++k) W.tpos[k] = int32_t(t0 + order[k]);
    W.width.assign(ntp / kWave, 0);
    int64_t rows = 0;
    for (size_t w = 0; w < W.width.size(); ++w) {
        int32_t wd = 0;
        for (size_t k = w * kWave; k < std::min(nt, (w + 1) * kWave); ++k)
            wd = std::max(wd, len[size_t(order[k])]);
        W.width[w] = wd;
        rows += wd;
    }
    W.aidx.assign(size_t(rows * kWave), -1);
    int64_t base = 0;
    for (size_t w = 0; w < W.width.size(); ++w) {
        for (size_t k = w * kWave; k < std::min(nt, (w + 1) * kWave); ++k) {
            const int32_t i = order[k];
            for (int32_t j = 0; j < len[size_t(i)]; ++j)
                W.aidx[size_t((base + j) * kWave + int64_t(k % kWave))] =
                    lst[size_t(cnt[size_t(i)] + j)];
        }
        base += W.width[w];
    }
    W.contrib = int64_t(pairs.size());
}

// Concatenate the windows: task offsets and index rows become global.
fs_status join_windows(std::vector<Window> &win, HostPlan &P)
{
    const size_t nw = win.size();
    std::vector<int64_t> toff(nw + 1, 0), woff(nw + 1, 0), roff(nw + 1, 0);
    P.contrib = 0;
    for (size_t w = 0; w < nw; ++w) {
        toff[w + 1] = toff[w] + int64_t(win[w].tpos.size());
        woff[w + 1] = woff[w] + int64_t(win[w].width.size());
        roff[w + 1] = roff[w] + int64_t(win[w].aidx.size()) / kWave;
        P.contrib += win[w].contrib;
    }
    if (woff[nw] > INT32_MAX || roff[nw] > INT32_MAX || toff[nw] > INT32_MAX)
        return set_error(FS_E_UNSUPPORTED, "assembly plan too large");
    P.ntasks = toff[nw];
    P.tpos.alloc(size_t(toff[nw]));
    P.waves.alloc(size_t(2 * woff[nw]));
    P.aidx.alloc(size_t(roff[nw] * kWave));
    parallel_chunks(int64_t(nw), [&](int64_t w) {
        const Window &W = win[size_t(w)];
        std::copy(W.tpos.begin(), W.tpos.end(),
                  P.tpos.data() + toff[size_t(w)]);
        int64_t r = roff[size_t(w)];
        int32_t *wv = P.waves.data() + 2 * woff[size_t(w)];
        for (size_t k = 0; k < W.width.size(); ++k) {
            wv[2 * k] = int32_t(r);
            wv[2 * k + 1] = W.width[k];
            r += W.width[k];
        }
        std::copy(W.aidx.begin(), W.aidx.end(),
                  P.aidx.data() + roff[size_t(w)] * kWave);
    });
    return FS_OK;
}

// Slot of layout column c in layout row i (entries of a row are stored in
// ascending layout column, entry e at lane e mod T, slot e / T of the row's
// lanes, padding after the last entry), or -1.
int64_t find_slot(const HostLayout &L, const int32_t *slot_col,
                  const Group &g, int32_t i, int32_t c)
{
    const int32_t lt = g.width_lt >> 24, T = 1 << lt;
    const int32_t width = g.width_lt & 0xffffff, V = L.vec;
    const int32_t rr = i - g.row0;
    const int64_t base = int64_t(g.base64) * kWave;
    auto idx = [&](int32_t e) {
        const int32_t lane = rr * T + e % T, sl = e / T;
        return base + int64_t(sl / V) * kWave * V + int64_t(lane) * V + sl % V;
    };
    int32_t lo = 0, hi = T * width;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        const int32_t cm = slot_col[idx(mid)];
        if (cm >= 0 && cm < c) lo = mid + 1;
        else hi = mid;
    }
    if (lo < T * width) {
        const int64_t s = idx(lo);
        if (slot_col[s] == c) return s;
    }
    return -1;
}

template <class T>
fs_status upload(T **d, const BufT<T> &h, int64_t &acct, hipStream_t s)
{
    FS_TRY(dalloc(d, int64_t(h.size()), acct));
    if (!h.empty())
        FS_HIP_TRY(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T),
                                  hipMemcpyHostToDevice, s));
    return FS_OK;
}

fs_status upload_lds(const HostLds &H, AsmLdsPlan &D, int64_t &acct,
                     hipStream_t s)
{
    D.ngroups = int32_t(H.gdesc.size() / 4);
    D.nde = H.nde;
    D.rows = H.rows;
    D.region_max = H.region_max;
    D.nbatch = int64_t(H.bdesc.size() / 2);
    D.nrec = int64_t(H.off.size() / kWave);
    D.contrib = H.contrib;
    FS_TRY(upload(&D.d_gdesc, H.gdesc, acct, s));
    FS_TRY(upload(&D.d_bdesc, H.bdesc, acct, s));
    FS_TRY(upload(&D.d_ea, H.ea, acct, s));
    FS_TRY(upload(&D.d_off, H.off, acct, s));
    return FS_OK;
}

fs_status upload_plan(const HostPlan &H, AsmPlan &D, int64_t &acct,
                      hipStream_t s)
{
    D.ntasks = H.ntasks;
    D.nwaves = int32_t(H.waves.size() / 2);
    D.stored = int64_t(H.aidx.size());
    D.contrib = H.contrib;
    FS_TRY(upload(&D.d_waves, H.waves, acct, s));
    FS_TRY(upload(&D.d_tpos, H.tpos, acct, s));
    FS_TRY(upload(&D.d_aidx, H.aidx, acct, s));
    return FS_OK;
}

void free_plan(AsmPlan &D)
{
    dfree(D.d_waves);
    dfree(D.d_tpos);
    dfree(D.d_aidx);
}

void free_asm(fs_asm *P)
{
    free_plan(P->km);
    free_plan(P->rv);
    dfree(P->kl.d_gdesc);
    dfree(P->kl.d_bdesc);
    dfree(P->kl.d_ea);
    dfree(P->kl.d_off);
}

// Row-group plan (LDS accumulation), when it applies: nde <= 64, no
// element repeats a kept DOF (two lanes of one step would add into the same
// slot at once), and every group's slot region fits kAsmLdsMax doubles.
// Returns FS_OK with H.built = false when it does not apply; *bad receives
// the smallest element with a coupling missing from the pattern (or -1).
fs_status build_lds(const HostLayout &L, const int32_t *slot_col, int32_t ne,
                    int32_t nde, const std::vector<int32_t> &edof,
                    const std::vector<int64_t> &doff,
                    const std::vector<int32_t> &dent, HostLds &H,
                    int64_t *bad)
{
    *bad = -1;
    H.built = false;
    if (nde < 1 || nde > kWave) return FS_OK;
    int32_t region_max = 0;
    for (const Group &g : L.groups) {
        const int32_t r = (g.width_lt & 0xffffff) * kWave;
        if (r > kAsmLdsMax) return FS_OK;
        region_max = std::max(region_max, r);
    }
    {
        std::vector<char> dup(size_t((int64_t(ne) + 4095) / 4096), 0);
        parallel_chunks(int64_t(dup.size()), [&](int64_t c) {
            std::vector<int32_t> t;
            const int64_t e1 = std::min<int64_t>(ne, (c + 1) * 4096);
            for (int64_t e = c * 4096; e < e1 && !dup[size_t(c)]; ++e) {
                t.clear();
                for (int32_t a = 0; a < nde; ++a)
                    if (edof[size_t(e * nde + a)] >= 0)
                        t.push_back(edof[size_t(e * nde + a)]);
                std::sort(t.begin(), t.end());
                if (std::adjacent_find(t.begin(), t.end()) != t.end())
                    dup[size_t(c)] = 1;
            }
        });
        for (char d : dup)
            if (d) return FS_OK;
    }
    const int32_t R = kWave / nde;
    const int64_t ng = int64_t(L.groups.size());
    constexpr int64_t kGC = 256;                // groups per work item
    const int64_t nch = (ng + kGC - 1) / kGC;
    struct Part {
        std::vector<int32_t> gdesc, bdesc, ea;
        std::vector<uint16_t> off;
        int64_t contrib = 0, bad = -1;
    };
    std::vector<Part> part(static_cast<size_t>(nch));
    parallel_chunks(nch, [&](int64_t c) {
        Part &P = part[size_t(c)];
        const int64_t g1 = std::min(ng, (c + 1) * kGC);
        for (int64_t gi = c * kGC; gi < g1; ++gi) {
            const Group &g = L.groups[size_t(gi)];
            const int64_t base = int64_t(g.base64) * kWave;
            const int32_t nb = (g.nrows + R - 1) / R;
            P.gdesc.insert(P.gdesc.end(),
                           {g.base64, g.width_lt & 0xffffff,
                            int32_t(P.bdesc.size() / 2), nb});
            for (int32_t j = 0; j < nb; ++j) {
                int32_t K = 0;
                for (int32_t q = 0; q < R && j * R + q < g.nrows; ++q) {
                    const int32_t I = L.perm[size_t(g.row0 + j * R + q)];
                    K = std::max<int32_t>(
                        K, int32_t(doff[size_t(I) + 1] - doff[size_t(I)]));
                }
                P.bdesc.insert(P.bdesc.end(),
                               {int32_t(P.off.size() / kWave), K});
                for (int32_t k = 0; k < K; ++k) {
                    const size_t o0 = P.off.size();
                    P.off.resize(o0 + kWave, 0xffff);
                    for (int32_t q = 0; q < R; ++q) {
                        const int32_t rr = j * R + q;
                        int32_t eav = -1;
                        if (rr < g.nrows) {
                            const int32_t i = g.row0 + rr;
                            const int32_t I = L.perm[size_t(i)];
                            if (k < doff[size_t(I) + 1] - doff[size_t(I)])
                                eav = dent[size_t(doff[size_t(I)] + k)];
                            if (eav >= 0) {
                                const int32_t *ed =
                                    edof.data() + int64_t(eav / nde) * nde;
                                for (int32_t b = 0; b < nde; ++b) {
                                    if (ed[b] < 0) continue;
                                    const int32_t cc =
                                        L.symmetric_relabel
                                            ? L.iperm[size_t(ed[b])] : ed[b];
                                    const int64_t sl =
                                        find_slot(L, slot_col, g, i, cc);
                                    if (sl < 0) {
                                        const int64_t e = eav / nde;
                                        if (P.bad < 0 || e < P.bad) P.bad = e;
                                        continue;
                                    }
                                    P.off[o0 + size_t(q * nde + b)] =
                                        uint16_t(sl - base);
                                    ++P.contrib;
                                }
                            }
                        }
                        P.ea.push_back(eav);
                    }
                }
            }
        }
    });
    for (const Part &P : part)
        if (P.bad >= 0 && (*bad < 0 || P.bad < *bad)) *bad = P.bad;
    if (*bad >= 0) return FS_OK;
    std::vector<int64_t> gb(size_t(nch) + 1, 0), bb(gb), rb(gb);
    H.contrib = 0;
    for (int64_t c = 0; c < nch; ++c) {
        const Part &P = part[size_t(c)];
        gb[size_t(c) + 1] = gb[size_t(c)] + int64_t(P.gdesc.size());
        bb[size_t(c) + 1] = bb[size_t(c)] + int64_t(P.bdesc.size());
        rb[size_t(c) + 1] = rb[size_t(c)] + int64_t(P.off.size()) / kWave;
        H.contrib += P.contrib;
    }
    if (bb[size_t(nch)] / 2 > INT32_MAX || rb[size_t(nch)] > INT32_MAX)
        return FS_OK;
    H.gdesc.alloc(size_t(gb[size_t(nch)]));
    H.bdesc.alloc(size_t(bb[size_t(nch)]));
    H.ea.alloc(size_t(rb[size_t(nch)] * R));
    H.off.alloc(size_t(rb[size_t(nch)] * kWave));
    parallel_chunks(nch, [&](int64_t c) {
        const Part &P = part[size_t(c)];
        int32_t *gd = H.gdesc.data() + gb[size_t(c)];
        for (size_t k = 0; k < P.gdesc.size(); k += 4) {
            gd[k] = P.gdesc[k];
            gd[k + 1] = P.gdesc[k + 1];
            gd[k + 2] = P.gdesc[k + 2] + int32_t(bb[size_t(c)] / 2);
            gd[k + 3] = P.gdesc[k + 3];
        }
        int32_t *bd = H.bdesc.data() + bb[size_t(c)];
        for (size_t k = 0; k < P.bdesc.size(); k += 2) {
            bd[k] = P.bdesc[k] + int32_t(rb[size_t(c)]);
            bd[k + 1] = P.bdesc[k + 1];
        }
        std::copy(P.ea.begin(), P.ea.end(), H.ea.data() + rb[size_t(c)] * R);
        std::copy(P.off.begin(), P.off.end(),
                  H.off.data() + rb[size_t(c)] * kWave);
    });
    H.nde = nde;
    H.rows = R;
    H.region_max = region_max;
    H.built = true;
    return FS_OK;
}

// Gather plan of the matrix: windows of whole row groups holding >=
// kWindow slots.
fs_status build_gather(const HostLayout &L, const int32_t *slot_col,
                       int32_t nde, const std::vector<int32_t> &edof,
                       const std::vector<int64_t> &doff,
                       const std::vector<int32_t> &dent, HostPlan &km)
{
    std::vector<int32_t> gcut{0};
    {
        int64_t acc = 0;
        for (size_t g = 0; g < L.groups.size(); ++g) {
            acc += int64_t(L.groups[g].width_lt & 0xffffff) * kWave;
            if (acc >= kWindow) {
                gcut.push_back(int32_t(g + 1));
                acc = 0;
            }
        }
        if (gcut.back() != int32_t(L.groups.size()))
            gcut.push_back(int32_t(L.groups.size()));
    }
    std::vector<Window> win(gcut.size() - 1);
    parallel_chunks(int64_t(win.size()), [&](int64_t w) {
        Window &W = win[size_t(w)];
        const Group &gf = L.groups[size_t(gcut[size_t(w)])];
        const Group &gl = L.groups[size_t(gcut[size_t(w) + 1] - 1)];
        const int64_t t0 = int64_t(gf.base64) * kWave;
        const int64_t t1 = int64_t(gl.base64) * kWave +
                           int64_t(gl.width_lt & 0xffffff) * kWave;
        std::vector<std::pair<int32_t, int32_t>> pairs;
        for (int32_t g = gcut[size_t(w)]; g < gcut[size_t(w) + 1]; ++g) {
            const Group &gd = L.groups[size_t(g)];
            for (int32_t rr = 0; rr < gd.nrows; ++rr) {
                const int32_t i = gd.row0 + rr;
                const int32_t I = L.perm[size_t(i)];
                for (int64_t k = doff[size_t(I)]; k < doff[size_t(I) + 1]; ++k) {
                    const int64_t ea = dent[size_t(k)];
                    const int32_t *ed = edof.data() + (ea / nde) * nde;
                    for (int32_t b = 0; b < nde; ++b) {
                        if (ed[b] < 0) continue;
                        const int32_t cc = L.symmetric_relabel
                                               ? L.iperm[size_t(ed[b])] : ed[b];
                        const int64_t sl = find_slot(L, slot_col, gd, i, cc);
                        if (sl < 0) {
                            const int64_t e = ea / nde;
                            if (W.bad < 0 || e < W.bad) W.bad = e;
                            continue;
                        }
                        pairs.emplace_back(int32_t(sl),
                                           int32_t(ea * nde + b));
                    }
                }
            }
        }
        if (W.bad < 0) finish_window(t0, t1, slot_col, pairs, W);
    });
    int64_t bad = -1;
    for (const Window &W : win)
        if (W.bad >= 0 && (bad < 0 || W.bad < bad)) bad = W.bad;
    if (bad >= 0)
        return set_error(FS_E_BAD_CSR,
                         "element %lld couples DOFs that are not a "
                         "structural non-zero of the matrix", (long long)bad);
    FS_TRY(join_windows(win, km));
    return FS_OK;
}

// Host half of asm_create on a host copy of edof.  Both plans are built
// from the DOF -> element entry lists (flat index e * nde + a, ascending):
// a row's matrix contributions are enumerated as (e, a) from its list, then
// b = 0 .. nde-1, i.e. in ascending flat index (e * nde + a) * nde + b.
fs_status build_asm(const HostLayout &L, const int32_t *slot_col, int32_t n,
                    int32_t ne, int32_t nde, const std::vector<int32_t> &edof,
                    HostPlan &km, HostPlan &rv, HostLds *kl)
{
    const int64_t nee = int64_t(ne) * nde;
    for (int64_t i = 0; i < nee; ++i) {
        const int32_t v = edof[size_t(i)];
        if (v < -1 || v >= n)
            return set_error(FS_E_ARG,
                             "edof[%lld][%d] = %d is outside [-1, %d)",
                             (long long)(i / nde), int(i % nde), v, n);
    }
    std::vector<int64_t> doff(size_t(n) + 1, 0);
    for (int64_t i = 0; i < nee; ++i)
        if (edof[size_t(i)] >= 0) ++doff[size_t(edof[size_t(i)]) + 1];
    for (int32_t r = 0; r < n; ++r) doff[size_t(r) + 1] += doff[size_t(r)];
    std::vector<int32_t> dent(static_cast<size_t>(doff[size_t(n)]));
    {
        std::vector<int64_t> cur(doff.begin(), doff.end() - 1);
        for (int64_t i = 0; i < nee; ++i)
            if (edof[size_t(i)] >= 0)
                dent[size_t(cur[size_t(edof[size_t(i)])]++)] = int32_t(i);
    }
    if (kl) {
        int64_t bad = -1;
        FS_TRY(build_lds(L, slot_col, ne, nde, edof, doff, dent, *kl, &bad));
        if (bad >= 0)
            return set_error(FS_E_BAD_CSR,
                             "element %lld couples DOFs that are not a "
                             "structural non-zero of the matrix",
                             (long long)bad);
    }
    if (!kl || !kl->built)
        FS_TRY(build_gather(L, slot_col, nde, edof, doff, dent, km));
    // vector: windows of kWindow rows in the caller's numbering
    std::vector<Window> vw(size_t((int64_t(n) + kWindow - 1) / kWindow));
    parallel_chunks(int64_t(vw.size()), [&](int64_t w) {
        const int64_t t0 = w * kWindow, t1 = std::min<int64_t>(n, t0 + kWindow);
        std::vector<std::pair<int32_t, int32_t>> pairs;
        for (int64_t I = t0; I < t1; ++I)
            for (int64_t k = doff[size_t(I)]; k < doff[size_t(I) + 1]; ++k)
                pairs.emplace_back(int32_t(I), dent[size_t(k)]);
        finish_window(t0, t1, nullptr, pairs, vw[size_t(w)]);
    });
    FS_TRY(join_windows(vw, rv));
    return FS_OK;
}

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" {

fs_status asm_create(fs_csr_t A, int32_t n_elem, int32_t nde,
                     const int32_t *edof, int32_t plan, hipStream_t s,
                     fs_asm_t *out)
{
    const double t0 = now_ms();
    if (!out) return set_error(FS_E_ARG, "NULL output plan pointer");
    *out = nullptr;
    if (!A) return set_error(FS_E_ARG, "NULL matrix handle");
    if (A->n_rows != A->n_cols)
        return set_error(FS_E_NOT_SQUARE, "assembly needs a square matrix");
    if (n_elem < 0 || nde < 0)
        return set_error(FS_E_ARG, "negative size (%d elements, %d DOFs)",
                         n_elem, nde);
    const int64_t nee = int64_t(n_elem) * nde;
    if (nee * nde >= INT32_MAX)
        return set_error(FS_E_UNSUPPORTED,
                         "n_elem * nde * nde must be below 2^31");
    if (nee > 0 && !edof) return set_error(FS_E_ARG, "NULL edof");
    if (plan < FS_ASM_AUTO || plan > FS_ASM_ROWGROUP)
        return set_error(FS_E_ARG, "unknown assembly plan kind %d", plan);
    DeviceGuard g(A->device);
    std::vector<int32_t> h(static_cast<size_t>(nee));
    if (nee > 0) {
        FS_HIP_TRY(hipMemcpyAsync(h.data(), edof, sizeof(int32_t) * size_t(nee),
                                  hipMemcpyDeviceToHost, s));
        FS_HIP_TRY(hipStreamSynchronize(s));
    }
    HostPlan km, rv;
    HostLds kl;
    try {
        // the handle keeps slot columns on the device only
        std::vector<int32_t> sc(static_cast<size_t>(A->slots));
        if (A->slots > 0) {
            FS_HIP_TRY(hipMemcpyAsync(sc.data(), A->d_col,
                                      sizeof(int32_t) * size_t(A->slots),
                                      hipMemcpyDeviceToHost, s));
            FS_HIP_TRY(hipStreamSynchronize(s));
        }
        FS_TRY(build_asm(A->host, sc.data(), A->n_rows, n_elem, nde, h, km,
                         rv, plan == FS_ASM_GATHER ? nullptr : &kl));
    } catch (const std::bad_alloc &) {
        return set_error(FS_E_OOM, "host allocation failed");
    }
    if (plan == FS_ASM_ROWGROUP && !kl.built)
        return set_error(FS_E_UNSUPPORTED,
                         "the row-group assembly plan does not apply (nde "
                         "> 64, a repeated DOF in an element, or a row group "
                         "wider than %d slots)", kAsmLdsMax);
    fs_asm *P = new (std::nothrow) fs_asm;
    if (!P) return set_error(FS_E_OOM, "host allocation failed");
    P->A = A;
    P->device = A->device;
    P->n_elem = n_elem;
    P->nde = nde;
    P->lds = kl.built;
    fs_status st = P->lds ? upload_lds(kl, P->kl, P->device_bytes, s)
                          : upload_plan(km, P->km, P->device_bytes, s);
    if (st == FS_OK) st = upload_plan(rv, P->rv, P->device_bytes, s);
    if (st == FS_OK && hipStreamSynchronize(s) != hipSuccess)
        st = set_error(FS_E_HIP, "upload of the assembly plan failed");
    if (st != FS_OK) {
        free_asm(P);
        delete P;
        return st;
    }
    P->t_build_ms = now_ms() - t0;
    *out = P;
    return FS_OK;
}

fs_status asm_plan_host(int32_t n_rows, int64_t nnz, const int32_t *rowptr,
                        const int32_t *colind, const fs_csr_opts *opts,
                        int32_t n_elem, int32_t nde, const int32_t *edof,
                        int32_t which, int64_t *ntasks, int32_t *nwaves,
                        int64_t *stored, int32_t *waves, int32_t *tpos,
                        int32_t *aidx)
{
    if (n_rows < 0 || nnz < 0 || n_elem < 0 || nde < 0)
        return set_error(FS_E_ARG, "negative size");
    if (!rowptr || (nnz > 0 && !colind) || !ntasks || !nwaves || !stored)
        return set_error(FS_E_ARG, "NULL argument");
    if (which != 0 && which != 1)
        return set_error(FS_E_ARG, "which must be 0 (matrix) or 1 (vector)");
    const int64_t nee = int64_t(n_elem) * nde;
    if (nee * nde >= INT32_MAX)
        return set_error(FS_E_UNSUPPORTED,
                         "n_elem * nde * nde must be below 2^31");
    if (nee > 0 && !edof) return set_error(FS_E_ARG, "NULL edof");
    fs_csr_opts o;
    csr_opts_default(&o);
    if (opts) o = *opts;
    HostLayout L;
    FS_TRY(build_layout(n_rows, n_rows, nnz, rowptr, colind, o, L));
    HostPlan km, rv;
    try {
        std::vector<int32_t> h(edof, edof + nee);
        FS_TRY(build_asm(L, L.slot_col.data(), n_rows, n_elem, nde, h, km,
                         rv, nullptr));
    } catch (const std::bad_alloc &) {
        return set_error(FS_E_OOM, "host allocation failed");
    }
    const HostPlan &H = which == 0 ? km : rv;
    *ntasks = H.ntasks;
    *nwaves = int32_t(H.waves.size() / 2);
    *stored = int64_t(H.aidx.size());
    if (waves && !H.waves.empty())
        std::memcpy(waves, H.waves.data(), H.waves.size() * sizeof(int32_t));
    if (tpos && !H.tpos.empty())
        std::memcpy(tpos, H.tpos.data(), H.tpos.size() * sizeof(int32_t));
    if (aidx && !H.aidx.empty())
        std::memcpy(aidx, H.aidx.data(), H.aidx.size() * sizeof(int32_t));
    return FS_OK;
}

fs_status asm_plan_host_groups(int32_t n_rows, int64_t nnz,
                               const int32_t *rowptr, const int32_t *colind,
                               const fs_csr_opts *opts, int32_t n_elem,
                               int32_t nde, const int32_t *edof,
                               int32_t *built, int32_t *ngroups,
                               int64_t *nbatch, int64_t *nrec, int32_t *rows,
                               int32_t *gdesc, int32_t *bdesc, int32_t *ea,
                               uint16_t *off)
{
    if (n_rows < 0 || nnz < 0 || n_elem < 0 || nde < 0)
        return set_error(FS_E_ARG, "negative size");
    if (!rowptr || (nnz > 0 && !colind) || !built || !ngroups || !nbatch ||
        !nrec || !rows)
        return set_error(FS_E_ARG, "NULL argument");
    const int64_t nee = int64_t(n_elem) * nde;
    if (nee * nde >= INT32_MAX)
        return set_error(FS_E_UNSUPPORTED,
                         "n_elem * nde * nde must be below 2^31");
    if (nee > 0 && !edof) return set_error(FS_E_ARG, "NULL edof");
    fs_csr_opts o;
    csr_opts_default(&o);
    if (opts) o = *opts;
    HostLayout L;
    FS_TRY(build_layout(n_rows, n_rows, nnz, rowptr, colind, o, L));
    HostPlan km, rv;
    HostLds kl;
    try {
        std::vector<int32_t> h(edof, edof + nee);
        FS_TRY(build_asm(L, L.slot_col.data(), n_rows, n_elem, nde, h, km,
                         rv, &kl));
    } catch (const std::bad_alloc &) {
        return set_error(FS_E_OOM, "host allocation failed");
    }
    *built = kl.built ? 1 : 0;
    *ngroups = int32_t(kl.gdesc.size() / 4);
    *nbatch = int64_t(kl.bdesc.size() / 2);
    *nrec = int64_t(kl.off.size() / kWave);
    *rows = kl.rows;
    if (gdesc && !kl.gdesc.empty())
        std::memcpy(gdesc, kl.gdesc.data(), kl.gdesc.size() * sizeof(int32_t));
    if (bdesc && !kl.bdesc.empty())
        std::memcpy(bdesc, kl.bdesc.data(), kl.bdesc.size() * sizeof(int32_t));
    if (ea && !kl.ea.empty())
        std::memcpy(ea, kl.ea.data(), kl.ea.size() * sizeof(int32_t));
    if (off && !kl.off.empty())
        std::memcpy(off, kl.off.data(), kl.off.size() * sizeof(uint16_t));
    return FS_OK;
}

fs_status asm_matrix(fs_asm_t P, const double *ke, hipStream_t s)
{
    if (!P) return set_error(FS_E_ARG, "NULL assembly plan");
    const int64_t contrib = P->lds ? P->kl.contrib : P->km.contrib;
    if (!ke && contrib > 0) return set_error(FS_E_ARG, "NULL ke");
    DeviceGuard g(P->device);
    const fs_csr *A = P->A;
    if (P->lds)
        FS_HIP_TRY(launch_assemble_lds(P->kl, ke, A->d_val, A->d_val_f32,
                                       A->d_val_bf16, A->d_groups, A->d_perm,
                                       nullptr, nullptr, false, s));
    else
        FS_HIP_TRY(launch_assemble(P->km, ke, A->d_val, A->d_val_f32,
                                   A->d_val_bf16, s));
    return FS_OK;
}

fs_status asm_system(fs_asm_t P, const double *ke, const double *re,
                     double *r, hipStream_t s)
{
    if (!P) return set_error(FS_E_ARG, "NULL assembly plan");
    if (!P->lds || !re) {          // gather plan, or no element entries
        FS_TRY(asm_matrix(P, ke, s));
        return asm_vector(P, re, r, s);
    }
    if (!ke && P->kl.contrib > 0) return set_error(FS_E_ARG, "NULL ke");
    if (!r && P->A->n_rows > 0) return set_error(FS_E_ARG, "NULL r");
    const int64_t nre = int64_t(P->n_elem) * P->nde;
    if (r && r < re + nre && re < r + P->A->n_rows)
        return set_error(FS_E_ARG, "r overlaps re");
    DeviceGuard g(P->device);
    const fs_csr *A = P->A;
    // every row belongs to one group of the plan, so every entry of r is
    // written
    FS_HIP_TRY(launch_assemble_lds(P->kl, ke, A->d_val, A->d_val_f32,
                                   A->d_val_bf16, A->d_groups, A->d_perm, re,
                                   r, false, s));
    return FS_OK;
}

fs_status asm_vector(fs_asm_t P, const double *re, double *r, hipStream_t s)
{
    if (!P) return set_error(FS_E_ARG, "NULL assembly plan");
    if (!r && P->rv.ntasks > 0) return set_error(FS_E_ARG, "NULL r");
    if (!re && P->rv.stored > 0) return set_error(FS_E_ARG, "NULL re");
    const int64_t nre = int64_t(P->n_elem) * P->nde;
    if (re && r && r < re + nre && re < r + P->rv.ntasks)
        return set_error(FS_E_ARG, "r overlaps re");
    DeviceGuard g(P->device);
    FS_HIP_TRY(launch_assemble(P->rv, re, r, nullptr, nullptr, s));
    return FS_OK;
}

fs_status asm_element_rows(fs_asm_t P, int32_t *pos, int64_t *rows)
{
    if (!P) return set_error(FS_E_ARG, "NULL assembly plan");
    if (!rows) return set_error(FS_E_ARG, "NULL rows");
    if (!P->lds)
        return set_error(FS_E_UNSUPPORTED,
                         "element-row order needs the row-group plan");
    const int64_t nr = P->kl.nrec * P->kl.rows;
    *rows = nr;
    if (!pos) return FS_OK;
    const int64_t nee = int64_t(P->n_elem) * P->nde;
    std::vector<int32_t> ea(static_cast<size_t>(nr));
    DeviceGuard g(P->device);
    if (nr > 0) {
        FS_HIP_TRY(hipMemcpy(ea.data(), P->kl.d_ea, sizeof(int32_t) * size_t(nr),
                             hipMemcpyDeviceToHost));
    }
    for (int64_t i = 0; i < nee; ++i) pos[i] = -1;
    for (int64_t i = 0; i < nr; ++i)
        if (ea[size_t(i)] >= 0) pos[ea[size_t(i)]] = int32_t(i);
    return FS_OK;
}

fs_status asm_matrix_ordered(fs_asm_t P, const double *ke_ordered,
                             hipStream_t s)
{
    if (!P) return set_error(FS_E_ARG, "NULL assembly plan");
    if (!P->lds)
        return set_error(FS_E_UNSUPPORTED,
                         "the ordered element buffer needs the row-group plan");
    if (!ke_ordered && P->kl.nrec > 0)
        return set_error(FS_E_ARG, "NULL ke_ordered");
    DeviceGuard g(P->device);
    const fs_csr *A = P->A;
    FS_HIP_TRY(launch_assemble_lds(P->kl, ke_ordered, A->d_val, A->d_val_f32,
                                   A->d_val_bf16, A->d_groups, A->d_perm,
                                   nullptr, nullptr, true, s));
    return FS_OK;
}

fs_status asm_info(fs_asm_t P, fs_asm_stats *st)
{
    if (!P) return set_error(FS_E_ARG, "NULL assembly plan");
    if (!st) return set_error(FS_E_ARG, "NULL stats");
    std::memset(st, 0, sizeof *st);
    st->n_elem = P->n_elem;
    st->nde = P->nde;
    st->plan = P->lds ? FS_ASM_ROWGROUP : FS_ASM_GATHER;
    st->contrib_matrix = P->lds ? P->kl.contrib : P->km.contrib;
    st->contrib_vector = P->rv.contrib;
    st->stored_matrix = P->lds ? P->kl.nrec * kWave : P->km.stored;
    st->stored_vector = P->rv.stored;
    st->bytes_algorithmic_matrix = 12 * st->contrib_matrix + 8 * P->A->nnz;
    st->bytes_algorithmic_vector = 12 * P->rv.contrib +
                                   8 * int64_t(P->A->n_rows);
    st->device_bytes = P->device_bytes;
    st->t_build_ms = P->t_build_ms;
    return FS_OK;
}

fs_status asm_destroy(fs_asm_t P)
{
    if (!P) return FS_OK;
    {
        DeviceGuard g(P->device);
        (void)hipDeviceSynchronize();
        free_asm(P);
    }
    delete P;
    return FS_OK;
}

}  // extern "C"
