"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, rejects bad arguments synchronously, and its layout builder (run on
the host through csr_layout_host) produces a valid slot layout whose
emulated product matches the oracle.  No GPU is needed."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

import paper_1501_00324_amd as fs
import workloads as W
from workloads.meshes import CSR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fespmv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(?:fs_status|const char \*)\s*(\w+)\s*\(",
                                 src)))


def test_library_exports_every_declared_symbol():
    L = fs.load()
    names = declared_functions()
    assert "csr_create" in names and "cg_solve" in names and "spmv" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(fs.EXPORTS) == names


def test_argument_errors_are_synchronous():
    L = fs.load()
    h = C.c_void_p()
    assert L.csr_create(4, 4, 0, None, None, None, None, None,
                        None) == fs.FS_E_ARG
    assert "NULL" in fs.last_error()
    assert L.csr_create(-1, 4, 0, None, None, None, None, None,
                        C.byref(h)) == fs.FS_E_ARG
    assert L.csr_create(4, 4, 2**31, 1, 1, 1, None, None,
                        C.byref(h)) == fs.FS_E_UNSUPPORTED
    assert L.spmv(None, None, None, None) == fs.FS_E_ARG
    assert L.spmv_perm(None, None, None, None) == fs.FS_E_ARG
    assert L.cg_solve(None, None, None, None, None, None) == fs.FS_E_ARG
    assert L.csr_info(None, None) == fs.FS_E_ARG
    assert L.csr_destroy(None) == fs.FS_OK
    o = fs.CgOpts()
    assert L.cg_opts_default(C.byref(o)) == fs.FS_OK
    assert o.rtol == 1e-8 and o.precond == fs.PC_JACOBI
    assert o.wg_threads == 0
    assert L.cg_solve_batch_wg(-1, None, None, None, None, None,
                               None) == fs.FS_E_ARG
    assert L.cg_solve_batch_wg(1, None, None, None, None, None,
                               None) == fs.FS_E_ARG
    o.wg_threads = 300
    assert L.cg_solve_batch_wg(0, None, None, None, C.byref(o), None,
                               None) == fs.FS_E_ARG
    assert "wg_threads" in fs.last_error()
    o.wg_threads = 0
    o.precision = fs.PREC_IR_F32
    assert L.cg_solve_batch_wg(0, None, None, None, C.byref(o), None,
                               None) == fs.FS_E_UNSUPPORTED


# ------------------------------------------------------------ host layout
def emulate(lay, x, n_rows):
    """Numpy emulation of the row-group kernel on the host layout (test
    code: checks the layout, not the kernel)."""
    y = np.zeros(n_rows)
    sc = lay["slot_col"]
    V = lay["vec"]
    for base64, row0, nrows, wlt in lay["groups"]:
        width, lt = wlt & 0xFFFFFF, wlt >> 24
        T = 1 << lt
        base = int(base64) * 64
        lanes = np.arange(64)
        s = np.arange(width)
        idx = base + (s[:, None] // V) * 64 * V + lanes[None, :] * V + \
            (s[:, None] % V)
        cols = sc[idx]
        vals = lay["val"][idx]
        prod = np.where(cols >= 0, vals * x[np.maximum(cols, 0)], 0.0)
        lane_sum = prod.sum(0)
        row_sum = lane_sum.reshape(64 // T, T).sum(1)
        y[row0:row0 + nrows] = row_sum[:nrows]
    return y


def check_layout(A, lay, square=True):
    n = A.n_rows
    perm = lay["perm"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    mp = lay["map"]
    sc = lay["slot_col"]
    assert len(np.unique(mp)) == A.nnz
    assert mp.min(initial=0) >= 0 and mp.max(initial=-1) < lay["slots"]
    exp_col = iperm[A.col] if square else A.col
    assert np.array_equal(sc[mp], exp_col)
    assert np.count_nonzero(sc >= 0) == A.nnz
    # groups cover the rows in order, slot ranges tile the slot array
    G = lay["groups"]
    row = 0
    slot = 0
    rl = A.row_lengths()
    for base64, row0, nrows, wlt in G:
        width, lt = wlt & 0xFFFFFF, wlt >> 24
        T = 1 << lt
        assert row0 == row and 1 <= nrows <= 64 // T
        assert base64 * 64 == slot and width % lay["vec"] == 0
        lens = rl[perm[row0:row0 + nrows]]
        assert width * T >= lens.max()
        row += nrows
        slot += width * 64
    assert row == n and slot == lay["slots"]


def layout_of(A, **opts):
    lay = fs.csr_layout_host(A.rowptr, A.col, A.n_rows, A.n_cols, **opts)
    val = np.zeros(lay["slots"])
    val[lay["map"]] = A.val
    lay["val"] = val
    return lay


CASES = [
    ("cfg0", lambda: W.config0_poisson2d(), {}),
    ("cfg0_t4", lambda: W.config0_poisson2d(), dict(lanes_min=4,
                                                     lanes_max=4)),
    ("ela_perm", lambda: W.tet_p1(6, "elastic", seed=(60, 0), bc="x0",
                                  permute=True), {}),
    ("ela_none", lambda: W.tet_p1(6, "elastic", seed=(60, 0), bc="x0",
                                  permute=True), dict(reorder=1)),
    ("p2_thr4", lambda: W.tet_p2(3, "laplace", seed=(60, 1)),
     dict(threshold=4)),
    ("q1_rcm_w1", lambda: W.hex_q1(5, "elastic", seed=(60, 2), permute=True),
     dict(reorder=2, sort_window=1)),
    ("ela_v1", lambda: W.tet_p1(6, "elastic", seed=(60, 3), bc="x0",
                                permute=True), dict(vec=1)),
    ("p2_v2_t2", lambda: W.tet_p2(3, "elastic", seed=(60, 4)),
     dict(vec=2, lanes_min=2, lanes_max=2)),
]


@pytest.mark.parametrize("name,gen,opts", CASES, ids=[c[0] for c in CASES])
def test_host_layout_valid_and_emulates_oracle(orc, name, gen, opts):
    A = gen()
    lay = layout_of(A, **opts)
    check_layout(A, lay)
    x = W.random_vector(A.n_cols, 60, W.XVEC)
    perm = lay["perm"]
    yp = emulate(lay, x[perm], A.n_rows)
    y = orc.spmv(A, x)
    assert np.all(np.abs(yp - y[perm]) <= 1e-13 * orc.spmv_abs(A, x)[perm])


def ragged(n_rows, n_cols, seed, maxlen=230):
    g = np.random.default_rng(seed)
    lens = g.integers(0, 12, n_rows)
    lens[g.choice(n_rows, max(1, n_rows // 20), replace=False)] = \
        g.integers(100, maxlen, max(1, n_rows // 20))
    lens = np.minimum(lens, n_cols)
    cols, vals = [], []
    for L in lens:
        cols.append(g.choice(n_cols, L, replace=False))  # unsorted columns
        vals.append(g.uniform(-1, 1, L))
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return CSR(n_rows, n_cols, rp, np.concatenate(cols).astype(np.int32),
               np.concatenate(vals))


@pytest.mark.parametrize("nr,nc", [(1, 1), (63, 63), (65, 65), (1000, 1000),
                                   (300, 1200), (1500, 40)])
def test_host_layout_ragged_rows(orc, nr, nc):
    A = ragged(nr, nc, seed=nr * 7 + nc)
    square = nr == nc
    lay = layout_of(A)
    # sorted columns ascending inside each row, in layout numbering
    check_layout(A, lay, square=square)
    x = W.random_vector(nc, 61, W.XVEC, nr)
    perm = lay["perm"]
    xl = x[perm] if square else x
    yp = emulate(lay, xl, nr)
    y = orc.spmv(A, x)
    assert np.all(np.abs(yp - y[perm]) <= 1e-13 * orc.spmv_abs(A, x)[perm])


def test_host_layout_empty_and_degenerate():
    e = fs.csr_layout_host(np.zeros(1, np.int32), np.zeros(0, np.int32), 0, 0)
    assert e["slots"] == 0 and len(e["groups"]) == 0
    z = fs.csr_layout_host(np.zeros(6, np.int32), np.zeros(0, np.int32), 5, 5)
    assert len(z["groups"]) == 1 and (z["groups"][0][3] & 0xFFFFFF) == 0


def test_host_layout_rejects_malformed_csr():
    L = fs
    with pytest.raises(fs.FsError) as e:
        L.csr_layout_host(np.array([1, 2], np.int32), np.array([0], np.int32))
    assert e.value.status == fs.FS_E_BAD_CSR
    with pytest.raises(fs.FsError) as e:
        L.csr_layout_host(np.array([0, 2, 1], np.int32),
                          np.array([0, 1], np.int32))
    assert e.value.status == fs.FS_E_BAD_CSR
    with pytest.raises(fs.FsError) as e:
        L.csr_layout_host(np.array([0, 1], np.int32), np.array([5], np.int32))
    assert e.value.status == fs.FS_E_BAD_CSR
    with pytest.raises(fs.FsError) as e:  # duplicate column
        L.csr_layout_host(np.array([0, 2], np.int32),
                          np.array([0, 0], np.int32))
    assert e.value.status == fs.FS_E_BAD_CSR
    with pytest.raises(fs.FsError) as e:
        L.csr_layout_host(np.array([0, 1, 2], np.int32),
                          np.array([0, 1], np.int32), perm=[0, 0])
    assert e.value.status == fs.FS_E_ARG
    with pytest.raises(fs.FsError) as e:
        L.csr_layout_host(np.array([0, 1], np.int32), np.array([0], np.int32),
                          lanes_min=3)
    assert e.value.status == fs.FS_E_ARG


def test_host_layout_worked_example():
    """The paper's one-row renumbering example inside a 7x7 matrix (other
    rows: the identity) with the paper's P as the user permutation: the
    layout row of that row holds the sorted relabelled columns c'' with
    the values A'' (section K1rs)."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden",
                                    "worked_example.json")))
    P = np.array(g["P"]) - 1
    rows = [list(zip(np.array(g["c"]) - 1, g["A"]))] + \
        [[(i, 1.0)] for i in range(1, 7)]
    rp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    col = np.array([c for r in rows for c, _ in r], np.int32)
    val = np.array([v for r in rows for _, v in r], float)
    A = CSR(7, 7, rp, col, val)
    lay = layout_of(A, perm=P, sort_window=1, lanes_min=1, lanes_max=1)
    assert np.array_equal(lay["perm"], P)
    r = int(np.nonzero(P == 0)[0][0])         # layout row holding row 0
    base64, row0, nrows, wlt = lay["groups"][0]
    lane = r - row0
    width = wlt & 0xFFFFFF
    s = np.arange(5)
    V = lay["vec"]
    idx = base64 * 64 + (s // V) * 64 * V + lane * V + s % V
    assert list(lay["slot_col"][idx] + 1) == g["c_dprime"]
    assert list(lay["val"][idx]) == g["A_dprime"]
    assert width >= 5
    x = np.array(g["x"], float)
    yp = emulate(lay, x[P], 7)
    assert yp[r] == g["y"]
