"""GPU parity of the FP64 SpMV against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import CSR
from tests.gpu_util import note, dev, host, make, assert_spmv_close
from tests.test_abi_cpu import ragged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


def run_spmv(fs, orc, A, opts, seed, what):
    note("spmv %s n=%d nnz=%d opts=%s" % (what, A.n_rows, A.nnz, opts))
    M = make(A, **opts)
    if opts.get("index_bits") == 32:
        assert fs.csr_info(M)["index_bits"] == 32
    x = W.random_vector(A.n_cols, 50, W.XVEC, seed)
    y = host(fs.spmv(M, dev(x)))
    assert_spmv_close(y, orc.spmv(A, x), orc.spmv_abs(A, x), what)
    if A.n_rows == A.n_cols:
        perm = fs.csr_get_perm(M)
        yp = host(fs.spmv_perm(M, dev(x[perm])))
        assert_spmv_close(yp, orc.spmv(A, x)[perm],
                          orc.spmv_abs(A, x)[perm], what + " perm")
    return M


LAYOUTS = [
    {},
    dict(lanes_min=1, lanes_max=1),
    dict(lanes_min=2, lanes_max=2),
    dict(lanes_min=4, lanes_max=4),
    dict(lanes_min=8, lanes_max=8),
    dict(lanes_min=16, lanes_max=16),
    dict(lanes_min=32, lanes_max=32),
    dict(lanes_min=64, lanes_max=64),
    dict(reorder=1),
    dict(reorder=2, sort_window=1),
    dict(sort_window=1024, threshold=4),
    dict(threshold=64),
    dict(vec=1),
    dict(vec=1, lanes_min=4, lanes_max=4),
    dict(vec=2, lanes_min=1, lanes_max=1, sort_window=1),
    dict(index_bits=32),
    dict(index_bits=32, vec=1),
    dict(index_bits=32, lanes_min=8, lanes_max=8),
]


@pytest.mark.parametrize("li", range(len(LAYOUTS)))
def test_config0_all_layouts(fs, orc, li):
    run_spmv(fs, orc, W.config0_poisson2d(), LAYOUTS[li], li, "cfg0")


@pytest.mark.parametrize("li", [0, 1, 3, 5, 8, 12, 13, 14])
def test_elasticity_layouts(fs, orc, li):
    A = W.tet_p1(12, "elastic", seed=(51, 0), bc="x0", permute=True)
    run_spmv(fs, orc, A, LAYOUTS[li], li, "ela12")


@pytest.mark.parametrize("i", [0, 3, 6, 9, 12])
@pytest.mark.parametrize("permuted", [False, True])
def test_sweep_small(fs, orc, i, permuted):
    A = W.sweep_matrix(i, permuted)
    run_spmv(fs, orc, A, {}, 100 + i, A.meta["name"])


@pytest.mark.parametrize("li", [0, 1, 3, 7, 9, 12])
def test_graded_layouts(fs, orc, li):
    """Skewed row lengths (3 .. 199 entries) under several layouts."""
    A = W.graded_2d_p1(60, seed=(52, 0), permute=True, hubs=None)
    run_spmv(fs, orc, A, LAYOUTS[li], li, "graded60")


@pytest.mark.parametrize("nr,nc", [(1, 1), (63, 63), (65, 65), (1000, 1000),
                                   (4099, 4099), (300, 1200), (1500, 40)])
@pytest.mark.parametrize("li", [0, 1, 4, 12])
def test_ragged_rows(fs, orc, nr, nc, li):
    A = ragged(nr, nc, seed=nr * 7 + nc)
    run_spmv(fs, orc, A, LAYOUTS[li], nr, "ragged%dx%d" % (nr, nc))


@pytest.mark.parametrize("vec", [1, 2])
def test_every_batch_count_and_tail(fs, orc, vec):
    """One lane per row and one row group per length: group k holds 64 rows
    of k entries, so the lanes own 1 .. 40 slots -- every count of full
    8-slot batches (0 .. 5, odd and even, where the pipelined loop pairs
    them) and every tail length after them; the caller-numbering and layout
    products are checked on every row against the oracle."""
    lens = np.repeat(np.arange(1, 41), 64)
    g = np.random.default_rng(77 + vec)
    n = len(lens)
    cols = [np.sort(g.choice(n, L, replace=False)) for L in lens]
    vals = [g.uniform(-1, 1, L) for L in lens]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    A = CSR(n, n, rp, np.concatenate(cols).astype(np.int32),
            np.concatenate(vals))
    M = run_spmv(fs, orc, A, dict(vec=vec, lanes_min=1, lanes_max=1,
                                  reorder=1, sort_window=1), vec,
                 "batches vec=%d" % vec)
    info = fs.csr_info(M)
    assert info["vec"] == vec and info["groups_by_lanes"][0] >= 40


def test_empty_and_zero_matrices(fs, orc):
    import torch
    note("spmv empty")
    A = CSR(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    M = make(A)
    fs.spmv(M, torch.zeros(0, dtype=torch.float64, device="cuda"))
    Z = CSR(70, 70, np.zeros(71, np.int32), np.zeros(0, np.int32),
            np.zeros(0))
    M = make(Z)
    y = host(fs.spmv(M, dev(np.ones(70))))
    assert not y.any()
    # a value update of a matrix without entries reads no values (the slot
    # refresh gathers only for slots that hold an entry)
    fs.csr_update_values(M, torch.zeros(0, dtype=torch.float64,
                                        device="cuda"))
    y = host(fs.spmv(M, dev(np.ones(70))))
    assert not y.any()


def test_padding_never_touches_x(fs, orc):
    """Padded slots must not multiply x: rows that do not reference column
    0 stay finite when x[0] is NaN or Inf."""
    A = ragged(500, 500, seed=3)
    keep = A.col != 0
    rows = np.repeat(np.arange(500), A.row_lengths())
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep],
                                                    minlength=500))])
    B = CSR(500, 500, rp.astype(np.int32), A.col[keep], A.val[keep])
    for li in (0, 1, 4):
        note("spmv padding nan layout %d" % li)
        M = make(B, **LAYOUTS[li])
        for bad in (np.nan, np.inf):
            x = W.random_vector(500, 52, W.XVEC)
            x[0] = bad
            y = host(fs.spmv(M, dev(x)))
            assert np.all(np.isfinite(y))
            assert_spmv_close(y, orc.spmv(B, x), orc.spmv_abs(B, x), "pad")


def test_permute_update_and_determinism(fs, orc):
    A = W.tet_p1(10, "elastic", seed=(53, 0), bc="x0", permute=True)
    note("spmv permute/update/determinism")
    M = make(A)
    x = W.random_vector(A.n_cols, 53, W.XVEC)
    xd = dev(x)
    xp = fs.csr_permute(M, fs.TO_LAYOUT, xd)
    perm = fs.csr_get_perm(M)
    assert np.array_equal(host(xp), x[perm])
    back = fs.csr_permute(M, fs.FROM_LAYOUT, xp)
    assert np.array_equal(host(back), x)
    y1 = host(fs.spmv(M, xd))
    y2 = host(fs.spmv(M, xd))
    assert np.array_equal(y1, y2)  # bitwise repeatable
    v2 = A.val * -1.5 + 0.25
    fs.csr_update_values(M, dev(v2))
    B = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, v2)
    y3 = host(fs.spmv(M, xd))
    assert_spmv_close(y3, orc.spmv(B, x), orc.spmv_abs(B, x), "update")


def test_config1_full_size(fs, orc):
    """The full config-1 matrix (774,144 rows, 33.97M nnz) in the launch
    configuration the benchmark times, every output row checked."""
    A = W.config1_elasticity3d()
    M = run_spmv(fs, orc, A, {}, 1, "cfg1")
    info = fs.csr_info(M)
    assert info["nnz"] == 33967818 and info["reorder"] == fs.REORDER_RCM
    assert info["padding"] < 0.15
    assert info["index_bits"] == 16      # the timed configuration
    M32 = run_spmv(fs, orc, A, dict(index_bits=32), 2, "cfg1 32-bit")
    assert fs.csr_info(M32)["slots"] == info["slots"]


# ------------------------------------------------------------ batched
def batch_matrices():
    """Mixed members: natural and relabelled numbering, both slot widths,
    a rectangular ragged matrix (rows permuted, columns not), a 1-row
    matrix."""
    return [
        (W.poisson_2d_p1(20, seed=(51, 0), bc="all"), {}),
        (W.tet_p1(6, "elastic", seed=(51, 1), bc="x0", permute=True), {}),
        (ragged(300, 157, seed=51), {}),
        (W.hex_q1(5, "laplace", seed=(51, 3), bc="all"), dict(vec=1)),
        (W.tet_p2(3, "laplace", seed=(51, 4), permute=True),
         dict(lanes_min=4, lanes_max=4)),
        (CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32),
             np.array([2.5])), {}),
    ]


def test_spmv_batch_equals_single(fs, orc):
    mats = batch_matrices()
    note("spmv_batch mixed, %d members" % len(mats))
    Ms = [make(A, **o) for A, o in mats]
    # every handle twice, the second time with another x (a relabelled
    # handle gathers into its own buffer: the batch must split there)
    order = list(range(len(mats))) * 2
    xs = [W.random_vector(mats[i][0].n_cols, 52, W.XVEC, j)
          for j, i in enumerate(order)]
    ys = fs.spmv_batch([Ms[i] for i in order], [dev(x) for x in xs])
    for j, i in enumerate(order):
        A = mats[i][0]
        y = host(ys[j])
        assert_spmv_close(y, orc.spmv(A, xs[j]), orc.spmv_abs(A, xs[j]),
                          "batch member %d" % j)
        y1 = host(fs.spmv(Ms[i], dev(xs[j])))
        assert np.array_equal(y, y1), j


def test_spmv_batch_many_members(fs, orc):
    """More members than one launch holds."""
    A = W.poisson_2d_p1(12, seed=(53, 0), bc="all", permute=True)
    B = W.poisson_2d_p1(9, seed=(53, 1), bc="all")
    note("spmv_batch 150 members")
    MA, MB = make(A), make(B)
    mats, xs = [], []
    for j in range(150):
        M, S = (MA, A) if j % 3 == 0 else (MB, B)
        mats.append((M, S))
        xs.append(W.random_vector(S.n_cols, 54, W.XVEC, j))
    ys = fs.spmv_batch([M for M, _ in mats], [dev(x) for x in xs])
    for j, ((M, S), x) in enumerate(zip(mats, xs)):
        assert_spmv_close(host(ys[j]), orc.spmv(S, x), orc.spmv_abs(S, x),
                          "member %d" % j)


def test_spmv_batch_rejects_aliasing(fs, orc):
    import torch
    A = W.poisson_2d_p1(8, seed=(55, 0), bc="all")
    note("spmv_batch argument errors")
    M = make(A)
    v = dev(np.ones(A.n_rows))
    w = torch.empty_like(v)
    with pytest.raises(fs.FsError) as e:
        fs.spmv_batch([M, M], [v, w], [w, torch.empty_like(v)])
    assert e.value.status == fs.FS_E_ARG
    with pytest.raises(fs.FsError) as e:
        fs.spmv_batch([M, M], [v, v], [w, w])
    assert e.value.status == fs.FS_E_ARG
    assert fs.spmv_batch([], []) == []


# ------------------------------------------------- plain CSR (no layout)
def long_rows(n_rows, n_cols, seed):
    """Rows of 300..1200 entries (mean above 256: 64 lanes per row)."""
    g = np.random.default_rng(seed)
    lens = g.integers(300, 1200, n_rows)
    cols = [np.sort(g.choice(n_cols, L, replace=False)) for L in lens]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return CSR(n_rows, n_cols, rp, np.concatenate(cols).astype(np.int32),
               g.uniform(-1, 1, int(rp[-1])))


CSR_CASES = [
    ("cfg0", W.config0_poisson2d),
    ("ela_perm", lambda: W.tet_p1(9, "elastic", seed=(57, 0), bc="x0",
                                  permute=True)),
    ("p2ela", lambda: W.tet_p2(4, "elastic", seed=(57, 1))),
    ("ragged", lambda: ragged(900, 411, seed=57)),
    ("long_rows", lambda: long_rows(70, 5000, seed=58)),
    ("no_entries", lambda: CSR(5, 3, np.zeros(6, np.int32),
                               np.zeros(0, np.int32), np.zeros(0))),
]


@pytest.mark.parametrize("name,gen", CSR_CASES, ids=[c[0] for c in CSR_CASES])
def test_spmv_csr_parity(fs, orc, name, gen):
    A = gen()
    note("spmv_csr %s n=%d nnz=%d" % (name, A.n_rows, A.nnz))
    x = W.random_vector(A.n_cols, 59, W.XVEC)
    y = host(fs.spmv_csr(dev(A.rowptr), dev(A.col), dev(A.val), A.n_rows,
                         A.n_cols, dev(x)))
    assert_spmv_close(y, orc.spmv(A, x), orc.spmv_abs(A, x), name)
