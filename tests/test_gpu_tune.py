"""GPU tests of the layout autotuner: the tuned layout is correct, the
choice is cached per matrix signature."""
import pytest

import workloads as W
from tests.gpu_util import note, dev, host, make, assert_spmv_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


@pytest.mark.parametrize("gen", [
    lambda: W.tet_p1(14, "elastic", seed=(35, 0), bc="x0", permute=True),
    lambda: W.tet_p2(6, "laplace", seed=(35, 1), permute=True),
])
def test_autotune_correct_and_cached(fs, orc, gen):
    A = gen()
    note("autotune n=%d" % A.n_rows)
    M = make(A, autotune=1)
    info = fs.csr_info(M)
    assert info["tuned"] == 1 and info["tune_candidates"] >= 2
    assert info["tune_best_us"] > 0
    x = W.random_vector(A.n_cols, 35, W.XVEC)
    y = host(fs.spmv(M, dev(x)))
    assert_spmv_close(y, orc.spmv(A, x), orc.spmv_abs(A, x), "tuned")
    perm = fs.csr_get_perm(M)
    yp = host(fs.spmv_perm(M, dev(x[perm])))
    assert_spmv_close(yp, orc.spmv(A, x)[perm], orc.spmv_abs(A, x)[perm],
                      "tuned perm")
    M2 = make(A, autotune=1)
    info2 = fs.csr_info(M2)
    assert info2["tuned"] == 2
    assert info2["slots"] == info["slots"]
    assert info2["groups_by_lanes"] == info["groups_by_lanes"]
    y2 = host(fs.spmv(M2, dev(x)))
    assert_spmv_close(y2, orc.spmv(A, x), orc.spmv_abs(A, x), "cached")
