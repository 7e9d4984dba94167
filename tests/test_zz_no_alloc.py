"""The allocation-free stream-ordered solve (cg_solve_async_noalloc)
against cg_solve_async, through the C ABI: bitwise the same solution and
result record on two calls in a row, the second on a smaller system (the
shared device workspace keeps the first call's contents), plus the
oracle's residual and the size limit."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import CSR
from tests.gpu_util import note, dev, host, make

pytestmark = pytest.mark.gpu

FIELDS = ("status", "iters", "replacements", "relres", "bytes")


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


def solve_both(fs, A, b, **opts):
    import torch
    M = make(A)
    bd = dev(b)
    ref = fs.cg_solve_async(M, bd, precond=fs.PC_JACOBI, **opts)
    ri = ref.info()
    x = torch.full((A.n_rows,), float("nan"), dtype=torch.float64,
                   device="cuda")
    buf = fs.info_buffer()
    got = fs.cg_solve_async_noalloc(M, bd, x, buf, precond=fs.PC_JACOBI,
                                    x0_zero=1, **opts)
    gi = got.info()
    return M, ref.x, ri, got.x, gi


def test_noalloc_matches_async_twice_then_smaller(fs, orc):
    big = W.config0_poisson2d()                       # 3,844 rows
    small = W.tet_p1(7, "elastic", seed=(90, 1), bc="x0", permute=True)
    assert small.n_rows < big.n_rows
    for A, seed in ((big, 0), (small, 1)):
        b = W.random_vector(A.n_rows, 90, W.BVEC, seed)
        note("noalloc solve n=%d" % A.n_rows)
        M, xr, ri, xg, gi = solve_both(fs, A, b)
        assert gi["status"] == fs.FS_OK
        assert all(ri[f] == gi[f] for f in FIELDS), (ri, gi)
        assert np.array_equal(host(xr), host(xg))
        rel = np.linalg.norm(b - orc.spmv(A, host(xg))) / np.linalg.norm(b)
        assert rel <= 1.001e-8


def test_noalloc_warm_start_and_limit(fs, orc):
    import torch
    A = W.poisson_2d_p1(30, seed=(91, 0), bc="all", permute=True)
    b = W.random_vector(A.n_rows, 91, W.BVEC)
    note("noalloc warm start")
    M = make(A)
    x0 = dev(W.random_vector(A.n_rows, 91, W.XVEC))
    ref = fs.cg_solve_async(M, dev(b), x=x0.clone(), precond=1, x0_zero=0)
    ri = ref.info()
    buf = fs.info_buffer()
    got = fs.cg_solve_async_noalloc(M, dev(b), x0.clone(), buf, precond=1,
                                    x0_zero=0)
    gi = got.info()
    assert all(ri[f] == gi[f] for f in FIELDS)
    assert np.array_equal(host(ref.x), host(got.x))
    # above the workspace's size: refused before any device work
    n = (1 << 18) + 1
    D = CSR(n, n, np.arange(n + 1, dtype=np.int32),
            np.arange(n, dtype=np.int32), np.full(n, 2.0))
    note("noalloc size limit")
    MD = make(D)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(fs.FsError) as e:
        fs.cg_solve_async_noalloc(MD, dev(np.ones(n)), x, buf)
    assert e.value.status == fs.FS_E_ARG and "262144" in str(e.value)
