"""Mixed-precision refinement where it cannot converge: the BF16 copy of an
ill-conditioned matrix (rounding error times condition number far above 1).
The solve must stop by itself with a failure status and a message, and
return an x no worse than the one before the last correction."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import CSR
from tests.gpu_util import note, dev, host, make

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


def rough_1d(n_el, seed):
    """1-D P1 stiffness with element conductivities U(1, 2), both ends
    clamped: SPD, condition number ~ n_el^2, values not representable in
    BF16."""
    g = np.random.default_rng(seed)
    kap = g.uniform(1.0, 2.0, n_el) * n_el
    m = n_el - 1
    rows, cols, vals = [], [], []
    for i in range(m):
        for j, v in ((i - 1, -kap[i]), (i, kap[i] + kap[i + 1]),
                     (i + 1, -kap[i + 1])):
            if 0 <= j < m:
                rows.append(i)
                cols.append(j)
                vals.append(v)
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, np.array(rows) + 1, 1)
    return CSR(m, m, np.cumsum(rp).astype(np.int32),
               np.array(cols, np.int32), np.array(vals))


@pytest.mark.parametrize("restart", [0, 1])
def test_bf16_refinement_stops_when_it_stalls(fs, orc, restart):
    A = rough_1d(4000, 36)
    b = W.random_vector(A.n_rows, 36, W.BVEC)
    note("ir bf16 stall restart=%d" % restart)
    M = make(A)
    x, info = fs.cg_solve(M, dev(b), precond=1, precision=fs.PREC_IR_BF16,
                          inner_rtol=1e-2, check=False, ir_restart=restart)
    # the BF16 copy of so ill-conditioned a matrix need not even be positive
    # definite: the inner solve may break down (FS_E_BREAKDOWN) or only stall
    assert info["status"] in (fs.FS_E_NOT_CONVERGED, fs.FS_E_BREAKDOWN)
    assert info["outer"] < 50
    xg = host(x)
    rel = np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b)
    assert abs(rel - info["relres"]) <= 1e-6 * max(rel, 1e-300)
    assert rel <= 1.0 + 1e-12            # the failed correction was undone
    assert "stopped" in info["message"]
    # the same system in FP64 converges
    x64, i64 = fs.cg_solve(M, dev(b), precond=1)
    assert i64["status"] == fs.FS_OK
