"""GPU tests of the stream-ordered solve (cg_solve_async): one cooperative
launch per solve, parity with the oracle and with cg_solve, stream order,
status codes."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import CSR
from tests.gpu_util import note, dev, host, make
from tests.test_gpu_cg import kappa, true_relres, SPD

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


@pytest.mark.parametrize("name,gen", SPD, ids=[c[0] for c in SPD])
@pytest.mark.parametrize("precond", [0, 1])
def test_async_parity(fs, orc, name, gen, precond):
    A = gen()
    b = W.random_vector(A.n_rows, 60, W.BVEC, A.n_rows % 89)
    note("cg async %s pc=%d n=%d" % (name, precond, A.n_rows))
    M = make(A)
    res = fs.cg_solve_async(M, dev(b), precond=precond)
    info = res.info()
    xg = host(res.x)
    assert info["status"] == fs.FS_OK, info
    assert info["relres"] <= 1e-8
    assert true_relres(orc, A, xg, b) <= 1.001e-8
    xo, st, it, rr = orc.pcg(A, b, precond=precond)
    assert np.linalg.norm(xg - xo) <= 4e-8 * kappa(A) * np.linalg.norm(xo)
    _, i1 = fs.cg_solve(M, dev(b), precond=precond)
    assert abs(info["iters"] - i1["iters"]) <= max(3, i1["iters"] // 20)
    assert abs(info["iters"] - it) <= max(3, it // 20)
    assert info["ms"] > 0 and info["bytes"] > 0


def test_async_stream_order(fs, orc):
    """b made, solved and checked on a side stream with no host wait in
    between: every step sees its predecessor's result."""
    import torch
    A = W.tet_p1(8, "elastic", seed=(61, 0), bc="x0", permute=True)
    b = W.random_vector(A.n_rows, 61, W.BVEC)
    note("cg async stream order")
    M = make(A)
    bd = dev(b)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b2 = bd * 2.0                     # produced on s
        res = fs.cg_solve_async(M, b2, stream=s, precond=1)
        y = fs.spmv(M, res.x, stream=s)   # consumes x on s
        r = b2 - y
    info = res.info()
    s.synchronize()
    assert info["status"] == fs.FS_OK
    rn = np.linalg.norm(host(r)) / np.linalg.norm(2 * b)
    assert rn <= 1.001e-8
    assert abs(rn - info["relres"]) <= 1e-3 * rn + 1e-15


def test_async_warm_start_and_maxit(fs, orc):
    A = W.tet_p1(8, "laplace", seed=(62, 0), bc="all", permute=True)
    b = W.random_vector(A.n_rows, 62, W.BVEC)
    note("cg async maxit / warm start")
    M = make(A)
    res = fs.cg_solve_async(M, dev(b), precond=1, maxit=7)
    i0 = res.info()
    assert i0["status"] == fs.FS_E_NOT_CONVERGED and i0["iters"] == 7
    x7 = host(res.x)
    assert abs(i0["relres"] - true_relres(orc, A, x7, b)) <= \
        1e-10 * i0["relres"]
    res2 = fs.cg_solve_async(M, dev(b), x=dev(x7), precond=1)
    i1 = res2.info()
    assert i1["status"] == fs.FS_OK
    assert true_relres(orc, A, host(res2.x), b) <= 1.001e-8


def test_async_status_codes(fs, orc):
    note("cg async status codes")
    Ind = CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
              np.array([1.0, -1.0]))
    M = make(Ind)
    res = fs.cg_solve_async(M, dev(np.ones(2)), precond=0)
    assert res.info()["status"] == fs.FS_E_BREAKDOWN
    # b = 0: x = 0 after no iteration, whatever the initial guess
    A = W.poisson_2d_p1(10, seed=(63, 0), bc="all")
    MA = make(A)
    res = fs.cg_solve_async(MA, dev(np.zeros(A.n_rows)),
                            x=dev(np.ones(A.n_rows)), precond=1)
    inf = res.info()
    assert inf["status"] == fs.FS_OK and inf["iters"] == 0
    assert not host(res.x).any()
    with pytest.raises(fs.FsError) as e:
        fs.cg_solve_async(MA, dev(np.ones(A.n_rows)),
                          precision=fs.PREC_IR_F32)
    assert e.value.status == fs.FS_E_UNSUPPORTED


def test_async_config1(fs, orc):
    """The full elasticity system (random numbering), Jacobi."""
    A = W.config1_elasticity3d()
    b = W.random_vector(A.n_rows, 1, W.BVEC)
    note("cg async config1 n=%d" % A.n_rows)
    M = make(A)
    res = fs.cg_solve_async(M, dev(b), precond=1)
    info = res.info()
    assert info["status"] == fs.FS_OK, info
    xg = host(res.x)
    assert true_relres(orc, A, xg, b) <= 1.001e-8
    x1, i1 = fs.cg_solve(M, dev(b), precond=1)
    assert abs(info["iters"] - i1["iters"]) <= max(3, i1["iters"] // 20)
    print("async %d it %.1f ms (device), cg_solve %d it %.1f ms"
          % (info["iters"], info["ms"], i1["iters"], i1["ms"]))
