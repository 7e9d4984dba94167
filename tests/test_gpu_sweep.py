"""GPU parity of the FP64 SpMV on every matrix of the sparsity sweep at full
size: 15 FEM matrices (P1/P2 tetrahedral Laplacian and elasticity, Q1
hexahedral Laplacian and elasticity, graded 2-D triangle meshes with skewed
row lengths), each in natural and random node numbering.  The sweep stands
in for the paper's benchmark matrix set (section "Benchmarks of SpMV
Methods"): a mix of FEM sizes and row-length shapes.

Every output row of both products the library offers -- the caller's
numbering (spmv: x gathered, y scattered) and the layout numbering
(spmv_perm, the product the CG iteration and the benchmark run) -- is
checked against the oracle's row sums at 1e-12 (|A||x|)_i, with the default
layout (the launch configuration the benchmark times).  Each matrix is
generated once for its test.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import note, dev, host, make, assert_spmv_close

pytestmark = pytest.mark.gpu

S12 = [i for i, r in enumerate(W.SWEEP) if r[0].startswith("S12")][0]


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


@pytest.mark.parametrize("permuted", [False, True], ids=["natural", "random"])
@pytest.mark.parametrize("i", range(len(W.SWEEP)),
                         ids=[r[0] for r in W.SWEEP])
def test_sweep_matrix_every_row(fs, orc, i, permuted):
    import torch
    name = W.SWEEP[i][0]
    note("sweep %s %s: generating" % (name, "random" if permuted
                                       else "natural"))
    A = W.sweep_matrix(i, permuted)
    note("sweep %s: n=%d nnz=%d, building the layout" % (name, A.n_rows,
                                                         A.nnz))
    M = make(A)
    info = fs.csr_info(M)
    x = W.random_vector(A.n_cols, 1, W.XVEC)
    y_ref = orc.spmv(A, x)
    scale = orc.spmv_abs(A, x)
    note("sweep %s: index_bits=%d slots=%d, products" % (
        name, info["index_bits"], info["slots"]))
    y = host(fs.spmv(M, dev(x)))
    assert_spmv_close(y, y_ref, scale, name + " caller numbering")
    perm = fs.csr_get_perm(M)
    yp = host(fs.spmv_perm(M, dev(x[perm])))
    assert_spmv_close(yp, y_ref[perm], scale[perm], name + " layout")
    # the padding stays bounded on every member of the set
    assert info["slots"] < 1.12 * max(A.nnz, 1)
    if i == S12:
        assert A.nnz == 156365811
    M.close()
    del M
    torch.cuda.synchronize()
