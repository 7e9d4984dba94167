"""GPU tests of the continuous-batching solve server: every result equals the
same request solved alone (bitwise), admission respects the device-memory
budget, and a failing request does not perturb the others."""
import time

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


def relres(orc, A, x, b):
    return np.linalg.norm(b - orc.spmv(A, x)) / np.linalg.norm(b)


def request_mix():
    mats = [W.poisson_2d_p1(24, seed=(30, 0), bc="all"),
            W.tet_p1(7, "elastic", seed=(30, 1), bc="x0", permute=True),
            W.tet_p1(10, "laplace", seed=(30, 2), bc="all", permute=True),
            W.hex_q1(6, "elastic", seed=(30, 3), bc="x0")]
    g = np.random.default_rng([30, 5])
    reqs = []
    for i in range(14):
        mi = int(g.integers(0, len(mats)))
        k = int(g.integers(1, 6))
        reqs.append((mi, W.random_vector(mats[mi].n_rows, 30, W.BVEC, i, k=k)))
    return mats, reqs


def run_server(fs, Ms, reqs, stagger_s=0.0, **opts):
    srv = fs.Server(**opts)
    ids = []
    for mi, B in reqs:
        rid, X = srv.submit(Ms[mi], dev(B))
        ids.append((rid, X))
        if stagger_s:
            time.sleep(stagger_s)
    done = {d["req_id"]: d for d in srv.drain()}
    stats = srv.stats()
    srv.close()
    return ids, done, stats


def test_server_results_equal_alone(fs, orc):
    mats, reqs = request_mix()
    note("server mix of %d requests" % len(reqs))
    Ms = [make(A) for A in mats]
    alone = []
    for mi, B in reqs:
        X, _ = fs.cg_solve_multi(Ms[mi], dev(B), precond=1)
        alone.append(host(X))
    # arrivals spread over time so requests join a running batch
    ids, done, stats = run_server(fs, Ms, reqs, stagger_s=0.002,
                                  check_every=4)
    assert stats["completed"] == len(reqs)
    for (rid, X), (mi, B), Xa in zip(ids, reqs, alone):
        d = done[rid]
        assert d["info"]["status"] == fs.FS_OK
        Xh = host(X)
        assert np.array_equal(Xh, Xa)
        for c in range(B.shape[1]):
            assert relres(orc, mats[mi], Xh[:, c], B[:, c]) <= 1.001e-8
        assert d["t_submit_ms"] <= d["t_admit_ms"] <= d["t_done_ms"]
    assert stats["peak_active"] >= 2      # requests really overlapped


def test_server_budget_limits_admission(fs, orc):
    mats, reqs = request_mix()
    note("server small budget")
    Ms = [make(A) for A in mats]
    biggest = max(fs.csr_info(M)["device_bytes"] for M in Ms)
    budget = int(2.5 * biggest) + (4 << 20)
    ids, done, stats = run_server(fs, Ms, reqs, hbm_budget_bytes=budget)
    assert stats["completed"] == len(reqs)
    assert 0 < stats["peak_bytes"] <= budget
    for (rid, X), (mi, B) in zip(ids, reqs):
        assert done[rid]["info"]["status"] == fs.FS_OK
        Xh = host(X)
        for c in range(B.shape[1]):
            assert relres(orc, mats[mi], Xh[:, c], B[:, c]) <= 1.001e-8
    # a request that could never fit is refused at submission
    srv = fs.Server(hbm_budget_bytes=1024)
    with pytest.raises(fs.FsError) as e:
        srv.submit(Ms[0], dev(reqs[0][1]))
    assert e.value.status == fs.FS_E_BUDGET
    srv.close()


def test_server_failure_is_isolated(fs, orc):
    A = W.poisson_2d_p1(16, seed=(31, 0), bc="all")
    Ind = CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
              np.array([1.0, -1.0]))
    note("server breakdown isolation")
    MA, MI = make(A), make(Ind)
    b = W.random_vector(A.n_rows, 31, W.BVEC)
    xa, _ = fs.cg_solve(MA, dev(b), precond=0)
    srv = fs.Server(precond=0, check_every=2)
    r1, X1 = srv.submit(MA, dev(b))
    r2, X2 = srv.submit(MI, dev(np.ones(2)))
    r3, X3 = srv.submit(MA, dev(b))
    done = {d["req_id"]: d for d in srv.drain()}
    srv.close()
    assert done[r2]["info"]["status"] == fs.FS_E_BREAKDOWN
    for r, X in ((r1, X1), (r3, X3)):
        assert done[r]["info"]["status"] == fs.FS_OK
        assert np.array_equal(host(X).reshape(-1), host(xa))
