"""The device layout build (per-non-zero phases on the GPU) against the host
build: every layout array bit for bit, the statistics, and the product
(bitwise between the two handles, and against the CPU oracle)."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import CSR
from tests.gpu_util import note, dev, host, make, assert_spmv_close
from tests.test_abi_cpu import ragged
from tests.test_gpu_spmv import long_rows

pytestmark = pytest.mark.gpu

SAME_STATS = ("n_rows", "n_cols", "nnz", "slots", "n_groups", "reorder",
              "padding", "bytes_algorithmic", "bytes_layout",
              "groups_by_lanes", "vec", "mean_band_before", "mean_band_after",
              "index_bits", "device_bytes", "dtypes")


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


def compare_builds(fs, orc, A, what, expect_device=True, **opts):
    note("build %s n=%d nnz=%d opts=%s" % (what, A.n_rows, A.nnz, opts))
    Mh = make(A, build=fs.BUILD_HOST, **opts)
    Md = make(A, **opts)            # the default build
    sh, sd = fs.csr_info(Mh), fs.csr_info(Md)
    assert sh["build"] == fs.BUILD_HOST
    assert sd["build"] == (fs.BUILD_DEVICE if expect_device
                           else fs.BUILD_HOST)
    for k in SAME_STATS:
        assert sh[k] == sd[k], "%s: %s %r vs %r" % (what, k, sh[k], sd[k])
    assert np.array_equal(fs.csr_get_perm(Mh), fs.csr_get_perm(Md))
    lh, ld = fs.csr_get_layout(Mh), fs.csr_get_layout(Md)
    for k in ("groups", "slot_col", "map", "col16", "gbase"):
        if lh[k] is None:
            assert ld[k] is None, k
        else:
            assert np.array_equal(lh[k], ld[k]), "%s: %s differs" % (what, k)
    assert np.array_equal(host(fs.csr_get_values(Md)), A.val)
    x = W.random_vector(A.n_cols, 50, W.XVEC, A.n_rows)
    yh = host(fs.spmv(Mh, dev(x)))
    yd = host(fs.spmv(Md, dev(x)))
    assert np.array_equal(yh.view(np.uint64), yd.view(np.uint64)), what
    assert_spmv_close(yd, orc.spmv(A, x), orc.spmv_abs(A, x), what)
    return sh, sd


OPTS = [
    {},
    dict(reorder=1),
    dict(reorder=2, sort_window=1),
    dict(lanes_min=4, lanes_max=4),
    dict(lanes_min=64, lanes_max=64, vec=1),
    dict(sort_window=1024, threshold=4),
    dict(vec=1),
    dict(index_bits=32),
    dict(dtypes=6),
]


@pytest.mark.parametrize("oi", range(len(OPTS)))
def test_config0(fs, orc, oi):
    compare_builds(fs, orc, W.config0_poisson2d(), "cfg0", **OPTS[oi])


@pytest.mark.parametrize("oi", [0, 1, 3, 6])
def test_elasticity_permuted(fs, orc, oi):
    A = W.tet_p1(10, "elastic", seed=(91, 0), bc="x0", permute=True)
    compare_builds(fs, orc, A, "ela10", **OPTS[oi])


def test_user_permutation(fs, orc):
    A = W.tet_p1(8, "elastic", seed=(91, 1), bc="x0", permute=True)
    perm = np.random.default_rng(91).permutation(A.n_rows)
    compare_builds(fs, orc, A, "ela8 user perm", perm=perm)


@pytest.mark.parametrize("oi", [0, 2, 5])
@pytest.mark.parametrize("i,permuted", [(3, False), (12, True)])
def test_sweep(fs, orc, i, permuted, oi):
    """A P2 / graded sweep matrix (the graded one has skewed rows)."""
    A = W.sweep_matrix(i, permuted)
    compare_builds(fs, orc, A, A.meta["name"], **OPTS[oi])


@pytest.mark.parametrize("nr,nc", [(1, 1), (63, 63), (65, 65), (1000, 1000),
                                   (4099, 4099), (300, 1200), (1500, 40),
                                   (300, 70000)])
def test_ragged(fs, orc, nr, nc):
    """Unsorted columns, empty rows, rows of 100..230 entries (several
    64-entry chunks per row), non-square shapes, and a column span above
    65535 (32-bit indices chosen by both builders)."""
    A = ragged(nr, nc, seed=nr * 5 + nc)
    compare_builds(fs, orc, A, "ragged%dx%d" % (nr, nc))
    compare_builds(fs, orc, A, "ragged%dx%d T8" % (nr, nc), lanes_min=8,
                   lanes_max=8)


def test_long_rows(fs, orc):
    compare_builds(fs, orc, long_rows(70, 5000, seed=92), "long rows")


def test_empty_matrices(fs, orc):
    Z = CSR(70, 70, np.zeros(71, np.int32), np.zeros(0, np.int32),
            np.zeros(0))
    compare_builds(fs, orc, Z, "no entries")
    N = CSR(5, 3, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    compare_builds(fs, orc, N, "no entries 5x3")
    note("build 0x0")
    E = CSR(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    M = make(E, build=fs.BUILD_DEVICE)
    assert fs.csr_info(M)["build"] == fs.BUILD_DEVICE


def test_row_above_device_limit_falls_back(fs, orc):
    g = np.random.default_rng(93)
    lens = np.array([3, fs.BUILD_DEVICE_MAX_ROW + 1, 0, 7])
    cols = [g.choice(6000, L, replace=False) for L in lens]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    A = CSR(4, 6000, rp, np.concatenate(cols).astype(np.int32),
            g.uniform(-1, 1, int(rp[-1])))
    compare_builds(fs, orc, A, "fallback", expect_device=False)
    lens[1] = fs.BUILD_DEVICE_MAX_ROW
    cols = [g.choice(6000, L, replace=False) for L in lens]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    B = CSR(4, 6000, rp, np.concatenate(cols).astype(np.int32),
            g.uniform(-1, 1, int(rp[-1])))
    compare_builds(fs, orc, B, "at limit")


def test_bad_input_errors(fs, orc):
    base = ragged(200, 200, seed=94)
    note("build errors")
    # duplicate column inside a row
    col = base.col.copy()
    r = int(np.argmax(base.row_lengths() >= 3))
    k0 = int(base.rowptr[r])
    col[k0 + 2] = col[k0]
    dup = CSR(200, 200, base.rowptr, col, base.val)
    for b in (fs.BUILD_HOST, fs.BUILD_DEVICE):
        with pytest.raises(fs.FsError) as e:
            make(dup, build=b)
        assert e.value.status == fs.FS_E_BAD_CSR
        assert "duplicate column %d in row %d" % (col[k0], r) in str(e.value)
    # column out of range
    col = base.col.copy()
    col[17] = 200
    oor = CSR(200, 200, base.rowptr, col, base.val)
    for b in (fs.BUILD_HOST, fs.BUILD_DEVICE):
        with pytest.raises(fs.FsError) as e:
            make(oor, build=b)
        assert e.value.status == fs.FS_E_BAD_CSR
        assert "column 200 out of range at 17" in str(e.value)
    # decreasing row offsets
    rp = base.rowptr.copy()
    i = int(np.argmax(rp > 0))
    rp[i + 1] = rp[i] - 1
    bad = CSR(200, 200, rp, base.col, base.val)
    for b in (fs.BUILD_HOST, fs.BUILD_DEVICE):
        with pytest.raises(fs.FsError) as e:
            make(bad, build=b)
        assert e.value.status == fs.FS_E_BAD_CSR
    with pytest.raises(fs.FsError) as e:
        make(base, build=7)
    assert e.value.status == fs.FS_E_ARG


def test_config1_full_size(fs, orc):
    """The 64^3 elasticity matrix (774,144 rows, 33,967,818 non-zeros):
    identical layouts; the device build reports its time."""
    A = W.config1_elasticity3d()
    sh, sd = compare_builds(fs, orc, A, "config1")
    note("config1 build host %.1f ms, device %.1f ms" % (sh["t_build_ms"],
                                                         sd["t_build_ms"]))
    sh, sd = compare_builds(fs, orc, A, "config1 no reorder", reorder=1)
    note("config1 (no reorder) build host %.1f ms, device %.1f ms" % (
        sh["t_build_ms"], sd["t_build_ms"]))


def test_get_layout_rejects_offsets_of_32bit_layout(fs, orc):
    """csr_get_layout: 16-bit offsets exist only for a 16-bit layout."""
    A = ragged(300, 70000, seed=95)        # a group spans 69,969 columns
    note("get_layout 32-bit")
    M = make(A)
    st = fs.csr_info(M)
    assert st["index_bits"] == 32
    buf = np.empty(st["slots"], dtype=np.uint16)
    rc = fs.load().csr_get_layout(M._h, None, None, None, buf.ctypes.data,
                                  None)
    assert rc == fs.FS_E_ARG
    lay = fs.csr_get_layout(M)
    assert lay["col16"] is None and lay["gbase"] is None
    assert np.array_equal(np.sort(lay["map"]),
                          np.sort(np.nonzero(lay["slot_col"] >= 0)[0]))


def rows_of_lengths(lens, n_cols, seed):
    """Rows of the given lengths, distinct random columns, values in
    (-1, 1)."""
    g = np.random.default_rng(seed)
    cols = [g.choice(n_cols, L, replace=False) for L in lens]
    vals = [g.uniform(-1, 1, L) for L in lens]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return CSR(len(lens), n_cols, rp, np.concatenate(cols).astype(np.int32),
               np.concatenate(vals))


@pytest.mark.parametrize("name", ["cfg0", "ragged", "ragged_rect", "rows255",
                                  "rows256", "long_rows"])
def test_value_refresh_in_slot_order(fs, orc, name):
    """csr_update_values (slot-ordered gather: through row starts and
    byte-wide in-row positions when every row holds at most 255 entries,
    else through the inverse map) leaves every value array -- FP64 slots,
    FP32 and BF16 copies, padding -- equal to those of a handle created with
    the new values.  rows255 has rows of exactly 255 entries (largest
    position 254, next to the padding mark 255); rows256 and long_rows
    exceed the byte-wide range and refresh through the inverse map."""
    lens255 = np.array([255, 1, 0, 254, 255, 3] * 20)
    A = {"cfg0": W.config0_poisson2d,
         "ragged": lambda: ragged(1000, 1000, seed=96),
         "ragged_rect": lambda: ragged(300, 1200, seed=97),
         "rows255": lambda: rows_of_lengths(lens255, 400, 93),
         "rows256": lambda: rows_of_lengths(
             np.where(lens255 == 255, 256, lens255), 400, 94),
         "long_rows": lambda: ragged(400, 1000, seed=95, maxlen=600)}[name]()
    note("value refresh %s" % name)
    g = np.random.default_rng(98)
    v2 = g.uniform(-1, 1, A.nnz)
    B = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, v2)
    for build in (fs.BUILD_DEVICE, fs.BUILD_HOST):
        M = make(A, dtypes=6, build=build)
        fs.csr_update_values(M, dev(v2))
        N = make(B, dtypes=6, build=build)
        assert np.array_equal(host(fs.csr_get_values(M)), v2)
        x = W.random_vector(A.n_cols, 51, W.XVEC)
        assert np.array_equal(host(fs.spmv(M, dev(x))).view(np.uint64),
                              host(fs.spmv(N, dev(x))).view(np.uint64))
        if A.n_rows == A.n_cols:
            xp = dev(x.astype(np.float32))
            for dt in (fs.DT_F32, fs.DT_BF16):
                assert np.array_equal(
                    host(fs.spmv_lowp(M, dt, xp)).view(np.uint32),
                    host(fs.spmv_lowp(N, dt, xp)).view(np.uint32))
