"""GPU tests of the one-workgroup batched solve (cg_solve_batch_wg): each
system's whole Jacobi-PCG solve in one workgroup of a single launch.
Parity with the oracle's PCG, results independent of the batch and of the
workgroup size, status codes and limits."""
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
def test_wg_parity(fs, orc, name, gen, precond):
    """Each system against the oracle's PCG: true residual (recomputed by
    the oracle), forward error within the conditioning bound, iteration
    count within 5% of the oracle's and of cg_solve's."""
    A = gen()
    b = W.random_vector(A.n_rows, 70, W.BVEC, A.n_rows % 83)
    note("cg wg %s pc=%d n=%d" % (name, precond, A.n_rows))
    M = make(A)
    xs, infos = fs.cg_solve_batch_wg([M], [dev(b)], precond=precond)
    info = infos[0]
    xg = host(xs[0])
    assert info["status"] == fs.FS_OK, info
    assert info["relres"] <= 1e-8
    assert true_relres(orc, A, xg, b) <= 1.001e-8
    xo, st, it, rr = orc.pcg(A, b, precond=precond)
    assert np.linalg.norm(xg - xo) <= 4e-8 * kappa(A) * np.linalg.norm(xo)
    assert abs(info["iters"] - it) <= max(3, it // 20)
    _, i1 = fs.cg_solve(M, dev(b), precond=precond)
    assert abs(info["iters"] - i1["iters"]) <= max(3, i1["iters"] // 20)
    assert info["ms"] > 0 and info["bytes"] > 0
    # the library's relres is the true residual of the returned x
    assert abs(info["relres"] - true_relres(orc, A, xg, b)) <= \
        1e-6 * info["relres"] + 1e-15


def wg_members():
    """Small systems of every layout kind: two- and one-slot loads, 16- and
    32-bit column streams, several row widths, one handle used twice."""
    return [
        (W.poisson_2d_p1(20, seed=(71, 0), bc="all"), {}),
        (W.tet_p1(6, "elastic", seed=(71, 1), bc="x0", permute=True), {}),
        (W.poisson_2d_p1(33, seed=(71, 2), bc="all", permute=True),
         {"vec": 1}),
        (W.hex_q1(5, "laplace", seed=(71, 3), bc="all"), {"index_bits": 32}),
        (W.tet_p2(3, "laplace", seed=(71, 4), bc="all"), {}),
        (W.config0_poisson2d(), {"vec": 1, "index_bits": 32}),
    ]


@pytest.mark.parametrize("precond", [0, 1])
def test_wg_alone_equals_mix(fs, orc, precond):
    """Every system gets bitwise the result of solving it alone, in any
    batch and order, and for every workgroup size."""
    mem = wg_members()
    note("cg wg batch of %d, precond %d" % (len(mem), precond))
    Ms = [make(A, **o) for A, o in mem]
    kinds = {(fs.csr_info(M)["vec"], fs.csr_info(M)["index_bits"]) for M in Ms}
    assert len(kinds) >= 3, kinds
    bs = [W.random_vector(A.n_rows, 72, W.BVEC, i)
          for i, (A, _) in enumerate(mem)]
    # the first handle twice, with another right-hand side
    Ms.append(Ms[0])
    bs.append(W.random_vector(mem[0][0].n_rows, 72, W.BVEC, 99))
    mats = [A for A, _ in mem] + [mem[0][0]]
    alone = []
    for M, b in zip(Ms, bs):
        xs, inf = fs.cg_solve_batch_wg([M], [dev(b)], precond=precond,
                                       wg_threads=256)
        alone.append((host(xs[0]), inf[0]["iters"]))
    for threads in (0, 256, 512, 1024):
        xs, infos = fs.cg_solve_batch_wg(Ms, [dev(b) for b in bs],
                                         precond=precond, wg_threads=threads)
        for A, x, b, (xa, ia), inf in zip(mats, xs, bs, alone, infos):
            xh = host(x)
            assert np.array_equal(xh, xa), threads
            assert inf["iters"] == ia
            assert inf["status"] == fs.FS_OK
            assert true_relres(orc, A, xh, b) <= 1.001e-8
    sub = list(range(len(Ms)))[::-2]
    xs, _ = fs.cg_solve_batch_wg([Ms[i] for i in sub],
                                 [dev(bs[i]) for i in sub], precond=precond)
    for i, x in zip(sub, xs):
        assert np.array_equal(host(x), alone[i][0])


def test_wg_z_in_lds_or_global(fs, orc):
    """A 29,929-row system (its z = D^-1 r does not fit in LDS beside the
    part sums, 8 bytes per row, so it stays in global memory) with small
    ones whose z does, and one whose z fits only above 64 KB of LDS:
    bitwise the same alone and together."""
    mats = [W.poisson_2d_p1(175, seed=(76, 0), bc="all"),
            W.poisson_2d_p1(20, seed=(76, 1), bc="all"),
            W.tet_p1(6, "elastic", seed=(76, 2), bc="x0", permute=True),
            # 12,100 rows: z in LDS needs 97 KB where the device allows
            # more than 64 KB per workgroup, else z stays in global memory
            W.poisson_2d_p1(112, seed=(76, 3), bc="all")]
    assert mats[0].n_rows == 29929 and mats[3].n_rows == 12100
    note("cg wg lds/global z, n=%s" % [A.n_rows for A in mats])
    Ms = [make(A) for A in mats]
    bs = [W.random_vector(A.n_rows, 76, W.BVEC, i) for i, A in
          enumerate(mats)]
    alone = [host(fs.cg_solve_batch_wg([M], [dev(b)], precond=1,
                                       wg_threads=1024)[0][0])
             for M, b in zip(Ms, bs)]
    xs, infos = fs.cg_solve_batch_wg(Ms, [dev(b) for b in bs], precond=1,
                                     wg_threads=1024)
    for A, x, b, xa, inf in zip(mats, xs, bs, alone, infos):
        assert inf["status"] == fs.FS_OK
        assert np.array_equal(host(x), xa)
        assert true_relres(orc, A, host(x), b) <= 1.001e-8


def test_wg_many_systems(fs, orc):
    """More workgroups than compute units: 300 jittered 2-D Poisson
    systems, each checked against the oracle."""
    m = 300
    mats = [W.poisson_2d_p1(24, seed=(73, i), bc="all") for i in range(m)]
    note("cg wg %d systems" % m)
    Ms = [make(A) for A in mats]
    bs = [W.random_vector(A.n_rows, 73, W.BVEC, i) for i, A in
          enumerate(mats)]
    xs, infos = fs.cg_solve_batch_wg(Ms, [dev(b) for b in bs], precond=1)
    for A, x, b, inf in zip(mats, xs, bs, infos):
        assert inf["status"] == fs.FS_OK
        assert true_relres(orc, A, host(x), b) <= 1.001e-8
    for M in Ms:
        M.close()


def test_wg_warm_start_maxit_and_status(fs, orc):
    A = W.tet_p1(8, "laplace", seed=(74, 0), bc="all", permute=True)
    b = W.random_vector(A.n_rows, 74, W.BVEC)
    note("cg wg maxit / warm start / status")
    M = make(A)
    xs, inf = fs.cg_solve_batch_wg([M], [dev(b)], precond=1, maxit=7,
                                   check=False)
    assert inf[0]["status"] == fs.FS_E_NOT_CONVERGED
    assert inf[0]["iters"] == 7
    x7 = host(xs[0])
    assert abs(inf[0]["relres"] - true_relres(orc, A, x7, b)) <= \
        1e-10 * inf[0]["relres"]
    # the oracle's PCG stopped after 7 iterations lands on the same iterate
    xo7, st, it, _ = orc.pcg(A, b, precond=1, maxit=7)
    assert it == 7
    assert np.linalg.norm(x7 - xo7) <= 1e-10 * np.linalg.norm(xo7)
    xs2, inf2 = fs.cg_solve_batch_wg([M], [dev(b)], [dev(x7)], precond=1)
    assert inf2[0]["status"] == fs.FS_OK
    assert true_relres(orc, A, host(xs2[0]), b) <= 1.001e-8
    # breakdown (indefinite), b = 0 (x = 0 whatever the guess), an empty
    # system, all in one batch beside a good one
    Ind = CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
              np.array([1.0, -1.0]))
    E = CSR(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32),
            np.zeros(0))
    Ms = [make(Ind), M, make(E), M]
    bs = [dev(np.ones(2)), dev(np.zeros(A.n_rows)),
          dev(np.zeros(0)), dev(b)]
    xs0 = [dev(np.zeros(2)), dev(np.ones(A.n_rows)), dev(np.zeros(0)),
           dev(np.zeros(A.n_rows))]
    xs, inf = fs.cg_solve_batch_wg(Ms, bs, xs0, precond=0, check=False)
    assert inf[0]["status"] == fs.FS_E_BREAKDOWN
    assert inf[1]["status"] == fs.FS_OK and inf[1]["iters"] == 0
    assert not host(xs[1]).any()
    assert inf[2]["status"] == fs.FS_OK and inf[2]["iters"] == 0
    assert inf[3]["status"] == fs.FS_OK
    assert true_relres(orc, A, host(xs[3]), b) <= 1.001e-8


def test_wg_limits_and_errors(fs, orc):
    note("cg wg limits")
    big = W.poisson_2d_p1(300, seed=(75, 0), bc="all")   # 88,804 rows
    assert big.n_rows > 65536
    Mb = make(big)
    with pytest.raises(fs.FsError) as e:
        fs.cg_solve_batch_wg([Mb], [dev(np.ones(big.n_rows))])
    assert e.value.status == fs.FS_E_ARG
    A = W.poisson_2d_p1(10, seed=(75, 1), bc="all")
    M = make(A)
    with pytest.raises(fs.FsError) as e:
        fs.cg_solve_batch_wg([M], [dev(np.ones(A.n_rows))], wg_threads=300)
    assert e.value.status == fs.FS_E_ARG
    with pytest.raises(fs.FsError) as e:
        fs.cg_solve_batch_wg([M], [dev(np.ones(A.n_rows))],
                             precision=fs.PREC_IR_F32)
    assert e.value.status == fs.FS_E_UNSUPPORTED
    xs, inf = fs.cg_solve_batch_wg([], [])
    assert xs == [] and inf == []
