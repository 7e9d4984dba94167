"""Host logic of the assembly plans (no GPU): the plan built by
asm_plan_host, executed by a numpy model of the device kernel (each task
adds its listed element values left to right from 0.0), must give bitwise
the oracle's element-loop assembly placed at the layout's slots."""
import numpy as np
import pytest

import workloads as W
from workloads.elements import (line_p1_elements, poisson_2d_p1_elements,
                                tet_p1_elements)


@pytest.fixture(scope="module")
def fs():
    import paper_1501_00324_amd as fs
    fs.load()
    return fs


def run_plan(plan, flat, n_out):
    """Numpy model of the assembly kernel."""
    waves, tpos, aidx = plan["waves"], plan["tpos"], plan["aidx"]
    nt = len(tpos)
    out = np.full(n_out, np.nan)
    if nt == 0:
        return out, np.zeros((0, 0), np.int32)
    width = int(waves[:, 1].max()) if len(waves) else 0
    t = np.arange(nt)
    w = t // 64
    j = np.arange(width)
    pos = (waves[w, 0][:, None] + j[None, :]) * 64 + (t % 64)[:, None]
    ok = j[None, :] < waves[w, 1][:, None]
    idx = np.where(ok, aidx[np.where(ok, pos, 0)], -1)
    vals = np.where(idx >= 0, flat[np.maximum(idx, 0)], 0.0)
    acc = np.cumsum(np.concatenate([np.zeros((nt, 1)), vals], axis=1),
                    axis=1)[:, -1]
    real = tpos >= 0
    out[tpos[real]] = acc[real]
    return out, idx


def bits(a):
    return np.ascontiguousarray(a).view(np.int64)


CASES = [
    ("line", lambda: (W.laplace_1d_p1(40)[0], line_p1_elements(40)), {}),
    ("p2d", lambda: (W.poisson_2d_p1(17, seed=(85, 0), bc="all",
                                     permute=True),
                     poisson_2d_p1_elements(17, seed=(85, 0), bc="all",
                                            permute=True)), {}),
    ("lap6", lambda: (W.tet_p1(6, "laplace", seed=(85, 1), permute=True),
                      tet_p1_elements(6, "laplace", seed=(85, 1),
                                      permute=True)), dict(vec=1)),
    ("ela5", lambda: (W.tet_p1(5, "elastic", seed=(85, 2), bc="x0",
                               permute=True),
                      tet_p1_elements(5, "elastic", seed=(85, 2), bc="x0",
                                      permute=True)), {}),
    ("ela5_nr", lambda: (W.tet_p1(5, "elastic", seed=(85, 3)),
                         tet_p1_elements(5, "elastic", seed=(85, 3))),
     dict(reorder=1, lanes_max=2)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_plan_reproduces_element_loop(fs, orc, case):
    name, gen, opts = CASES[case]
    A, E = gen()
    L = fs.csr_layout_host(A.rowptr, A.col, **opts)
    # matrix plan: tasks are exactly the non-padding slots
    P = fs.asm_plan_host(A.rowptr, A.col, E.edof, 0, **opts)
    tp = P["tpos"]
    assert len(tp) % 64 == 0
    assert np.array_equal(np.sort(tp[tp >= 0]), np.sort(L["map"]))
    got, idx = run_plan(P, E.ke.reshape(-1), L["slots"])
    want = orc.assemble_matrix(A, E.edof, E.ke)
    assert np.array_equal(bits(got[L["map"]]), bits(want))
    # every list is ascending (element order) and padding only at its end
    real = idx >= 0
    both = real[:, 1:] & real[:, :-1]
    assert np.all((np.diff(idx.astype(np.int64), axis=1) > 0) | ~both)
    assert np.all(real[:, :-1] | ~real[:, 1:])
    # padding stays modest: lists in a wave have nearly equal length
    assert len(P["aidx"]) <= 1.6 * real.sum() + 64 * len(P["waves"])
    # vector plan: one task per row
    V = fs.asm_plan_host(A.rowptr, A.col, E.edof, 1, **opts)
    assert np.array_equal(np.sort(V["tpos"][V["tpos"] >= 0]),
                          np.arange(A.n_rows))
    r, _ = run_plan(V, E.re.reshape(-1), A.n_rows)
    assert np.array_equal(bits(r), bits(orc.assemble_vector(A.n_rows, E.edof,
                                                            E.re)))


def test_plan_errors(fs):
    A = W.poisson_2d_p1(5, seed=(85, 4), bc="all")
    E = poisson_2d_p1_elements(5, seed=(85, 4), bc="all")
    bad = E.edof.copy()
    bad[0, 0] = -2
    with pytest.raises(fs.FsError) as ei:
        fs.asm_plan_host(A.rowptr, A.col, bad)
    assert ei.value.status == fs.FS_E_ARG
    n = A.n_rows
    rp = np.arange(n + 1, dtype=np.int32)
    with pytest.raises(fs.FsError) as ei:
        fs.asm_plan_host(rp, np.arange(n, dtype=np.int32), E.edof)
    assert ei.value.status == fs.FS_E_BAD_CSR
    # empty element set: every entry is a task with an empty list
    P = fs.asm_plan_host(A.rowptr, A.col, np.zeros((0, 3), np.int32))
    assert np.sum(P["tpos"] >= 0) == A.nnz and len(P["aidx"]) == 0


def run_groups(G, flat, n_slots, nde):
    """Numpy model of the row-group (LDS) assembly kernel."""
    out = np.full(n_slots, np.nan)
    rows = G["rows"]
    lane = np.arange(64)
    q, b = lane // nde, lane % nde
    act = q < rows
    for base64, width, b0, nb in G["gdesc"]:
        acc = np.zeros(width * 64)
        for j in range(b0, b0 + nb):
            r0, K = G["bdesc"][j]
            for rec in range(r0, r0 + K):
                e = np.where(act, G["ea"][rec][np.minimum(q, rows - 1)], -1)
                o = G["off"][rec].astype(np.int64)
                use = (e >= 0) & (o != 0xffff)
                # one step: distinct slots, added in step order
                assert len(np.unique(o[use])) == use.sum()
                acc[o[use]] += flat[e[use] * nde + b[use]]
        out[base64 * 64:(base64 + width) * 64] = acc
    return out


@pytest.mark.parametrize("case", range(len(CASES)))
def test_rowgroup_plan_reproduces_element_loop(fs, orc, case):
    name, gen, opts = CASES[case]
    A, E = gen()
    L = fs.csr_layout_host(A.rowptr, A.col, **opts)
    G = fs.asm_plan_host_groups(A.rowptr, A.col, E.edof, **opts)
    assert G is not None and G["rows"] == 64 // E.nde
    got = run_groups(G, E.ke.reshape(-1), L["slots"], E.nde)
    want = orc.assemble_matrix(A, E.edof, E.ke)
    assert np.array_equal(bits(got[L["map"]]), bits(want))
    # padding slots stay zero
    pad = np.ones(L["slots"], bool)
    pad[L["map"]] = False
    assert np.all(got[pad] == 0.0)
    # every element row is read exactly once
    ea = G["ea"][G["ea"] >= 0]
    assert np.array_equal(np.sort(ea), np.nonzero(E.edof.reshape(-1) >= 0)[0])
    # the same plan fed from a buffer stored in plan order (row rec * rows
    # + q holds element row ea[rec, q]): rows with offsets 0xffff only are
    # those without an element row
    rows = G["rows"]
    ko = np.full((G["ea"].size, E.nde), np.nan)
    flat = G["ea"].reshape(-1)
    ok = flat >= 0
    ko[np.nonzero(ok)[0]] = E.ke.reshape(-1, E.nde)[flat[ok]]
    assert np.all(G["off"].reshape(len(G["ea"]), -1)[:, :rows * E.nde]
                  .reshape(-1, rows, E.nde)[~ok.reshape(-1, rows)] == 0xffff)
    Go = dict(G)
    Go["ea"] = np.arange(G["ea"].size, dtype=np.int32).reshape(G["ea"].shape)
    got_o = run_groups(Go, np.nan_to_num(ko, nan=1e300).reshape(-1),
                       L["slots"], E.nde)
    assert np.array_equal(bits(got_o[L["map"]]), bits(want))


def test_rowgroup_plan_not_applicable(fs):
    A = W.poisson_2d_p1(6, seed=(85, 5), bc="none")
    E = poisson_2d_p1_elements(6, seed=(85, 5), bc="none")
    # an element that repeats a DOF
    ed = E.edof.copy()
    ed[4, 2] = ed[4, 0]
    assert fs.asm_plan_host_groups(A.rowptr, A.col, ed) is None
    # more than 64 DOFs per element
    wide = np.full((1, 65), -1, np.int32)
    wide[0, 0] = 0
    assert fs.asm_plan_host_groups(A.rowptr, A.col, wide) is None
    # the gather plan still covers both
    assert len(fs.asm_plan_host(A.rowptr, A.col, ed)["tpos"]) > 0
