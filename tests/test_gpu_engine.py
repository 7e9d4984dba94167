"""GPU parity of the multi-column products, the low-precision products, the
multi-right-hand-side CG and mixed-precision refinement (through the C
ABI), against the CPU oracle."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import CSR
from tests.gpu_util import note, dev, host, make, assert_spmv_close
from tests.test_abi_cpu import ragged
from tests.test_gpu_cg import kappa

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1501_00324_amd as fs
    fs.load(build_if_missing=False)
    return fs


def true_relres(orc, A, x, b):
    return np.linalg.norm(b - orc.spmv(A, x)) / np.linalg.norm(b)


# ------------------------------------------------------------------ SpMM
MATS = [
    ("cfg0", W.config0_poisson2d, {}),
    ("ela_perm", lambda: W.tet_p1(9, "elastic", seed=(40, 0), bc="x0",
                                  permute=True), {}),
    ("ela_v1_t4", lambda: W.tet_p1(7, "elastic", seed=(40, 1)),
     dict(vec=1, lanes_min=4, lanes_max=4)),
    ("ela_wide_idx", lambda: W.tet_p1(9, "elastic", seed=(40, 2),
                                      permute=True), dict(index_bits=32)),
    ("ragged_rect", lambda: ragged(700, 333, seed=5), {}),
]


@pytest.mark.parametrize("name,gen,opts", MATS, ids=[m[0] for m in MATS])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13, 16])
def test_spmm_parity(fs, orc, name, gen, opts, k):
    import torch
    A = gen()
    note("spmm %s k=%d" % (name, k))
    M = make(A, **opts)
    X = W.random_vector(A.n_cols, 41, W.XVEC, k, k=k)
    ld = k + 3
    Xp = np.zeros((A.n_cols, ld))
    Xp[:, :k] = X
    Yd = torch.full((A.n_rows, ld), 7.0, dtype=torch.float64, device="cuda")
    Xd = dev(Xp)
    st = fs.load().spmm(M._h, k, Xd.data_ptr(), ld, Yd.data_ptr(), ld,
                        torch.cuda.current_stream().cuda_stream)
    assert st == fs.FS_OK, fs.last_error()
    Y = host(Yd)
    Yo = orc.spmm(A, X)
    for c in range(k):
        assert_spmv_close(Y[:, c], Yo[:, c], orc.spmv_abs(A, X[:, c].copy()),
                          "spmm col %d" % c)
    assert np.all(Y[:, k:] == 7.0)          # padding columns untouched
    # k = 1 agrees bitwise with the single-vector product
    if k == 1:
        y1 = host(fs.spmv(M, dev(X[:, 0].copy())))
        assert np.array_equal(Y[:, 0], y1)


def test_spmm_rejects_bad_k(fs, orc):
    A = W.config0_poisson2d()
    M = make(A)
    import torch
    X = torch.zeros((A.n_rows, 17), dtype=torch.float64, device="cuda")
    for k, ld in [(0, 17), (17, 17), (4, 3)]:
        st = fs.load().spmm(M._h, k, X.data_ptr(), ld, X.data_ptr() + 8, ld,
                            0)
        assert st == fs.FS_E_ARG


# ------------------------------------------------------- low precision
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_lowp_storage_is_exact_rounding(fs, orc, dtype):
    """Unit vectors read back single columns of the stored copy: every
    stored value equals the oracle's rounding (FP32 nearest; BF16 nearest
    even of the FP32 value) bit for bit."""
    import torch
    A = W.tet_p1(6, "elastic", seed=(42, 0), bc="x0", permute=True)
    note("lowp storage %s" % dtype)
    M = make(A)
    dt = fs.DT_F32 if dtype == "f32" else fs.DT_BF16
    fs.csr_add_dtype(M, dt)
    if dtype == "f32":
        ref = orc.round_f32(A.val)
    else:
        ref = orc.bf16_bits_to_f32(orc.round_bf16(A.val))
    Alo = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, ref.astype(np.float64))
    D = Alo.to_dense()
    perm = fs.csr_get_perm(M)
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(len(perm))
    for j in range(0, A.n_cols, 37):
        e = np.zeros(A.n_cols, np.float32)
        e[iperm[j]] = 1.0            # layout position of column j
        y = host(fs.spmv_lowp(M, dt, dev(e)))
        col = y[iperm]               # back to caller numbering
        assert np.array_equal(col.astype(np.float64), D[:, j])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_lowp_product_error_bound(fs, orc, dtype):
    A = W.config0_poisson2d()
    note("lowp product %s" % dtype)
    M = make(A)
    dt = fs.DT_F32 if dtype == "f32" else fs.DT_BF16
    fs.csr_add_dtype(M, dt)
    a = orc.round_f32(A.val) if dtype == "f32" else \
        orc.bf16_bits_to_f32(orc.round_bf16(A.val))
    x = W.random_vector(A.n_cols, 43, W.XVEC).astype(np.float32)
    perm = fs.csr_get_perm(M)
    y = host(fs.spmv_lowp(M, dt, dev(x[perm])))
    yo = orc.spmv_f32(A, a, x)[perm]
    Af = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, a.astype(float))
    scale = orc.spmv_abs(Af, x.astype(float))[perm]
    m = A.row_lengths().max()
    u = 2.0 ** -24
    assert np.all(np.abs(y.astype(float) - yo.astype(float)) <=
                  2 * m * u * scale + 1e-30)


# ------------------------------------------------------- multi-RHS CG
def test_multi_rhs_columns_equal_single_solves(fs, orc):
    A = W.tet_p1(8, "elastic", seed=(44, 0), bc="x0", permute=True)
    k = 5
    B = W.random_vector(A.n_rows, 44, W.BVEC, 0, k=k)
    B[:, 3] = 0.0                          # a zero right-hand side
    note("cg multi k=%d" % k)
    M = make(A)
    X, infos = fs.cg_solve_multi(M, dev(B), precond=1)
    Xh = host(X)
    kap = kappa(A)
    for c in range(k):
        # one column alone runs the single-column kernels, whose sums are
        # ordered differently: equal up to rounding, not bitwise
        x1, i1 = fs.cg_solve(M, dev(B[:, c].copy()), precond=1)
        x1 = host(x1)
        assert np.linalg.norm(Xh[:, c] - x1) <= \
            4e-8 * kap * max(np.linalg.norm(x1), 1e-300), c
        assert abs(infos[c]["iters"] - i1["iters"]) <= \
            max(2, i1["iters"] // 20)
        if c == 3:
            assert infos[c]["iters"] == 0 and not Xh[:, c].any()
        else:
            assert infos[c]["status"] == fs.FS_OK
            assert true_relres(orc, A, Xh[:, c], B[:, c]) <= 1.001e-8


@pytest.mark.parametrize("k0,k1", [(5, 8), (3, 4), (9, 16)])
def test_multi_rhs_columns_depend_only_on_class(fs, k0, k1):
    """k0 and k1 share a column-count class: the first k0 columns of a
    k1-column solve equal the k0-column solve bit for bit."""
    A = W.tet_p1(8, "elastic", seed=(49, 0), bc="x0", permute=True)
    B = W.random_vector(A.n_rows, 49, W.BVEC, k1, k=k1)
    note("cg multi class k=%d,%d" % (k0, k1))
    M = make(A)
    X1, i1 = fs.cg_solve_multi(M, dev(B), precond=1)
    X0, i0 = fs.cg_solve_multi(M, dev(np.ascontiguousarray(B[:, :k0])),
                               precond=1)
    assert np.array_equal(host(X0), host(X1)[:, :k0])
    assert [i["iters"] for i in i0] == [i["iters"] for i in i1[:k0]]


@pytest.mark.parametrize("k", [2, 16])
def test_multi_rhs_parity(fs, orc, k):
    global KAPPA0
    A = W.config0_poisson2d()
    KAPPA0 = kappa(A)
    B = W.random_vector(A.n_rows, 45, W.BVEC, k, k=k)
    note("cg multi parity k=%d" % k)
    M = make(A)
    X, infos = fs.cg_solve_multi(M, dev(B), precond=0)
    Xh = host(X)
    for c in range(k):
        xo, st, it, rr = orc.pcg(A, B[:, c].copy(), precond=0)
        assert infos[c]["status"] == fs.FS_OK
        assert true_relres(orc, A, Xh[:, c], B[:, c]) <= 1.001e-8
        assert np.linalg.norm(Xh[:, c] - xo) <= 2e-8 * KAPPA0 * \
            np.linalg.norm(xo)


# ------------------------------------------------ mixed precision (IR)
IR_CASES = [
    ("cfg0", W.config0_poisson2d),
    ("ela8", lambda: W.tet_p1(8, "elastic", seed=(46, 0), bc="x0",
                              permute=True)),
]


@pytest.mark.parametrize("name,gen", IR_CASES, ids=[c[0] for c in IR_CASES])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("restart", [0, 1])
def test_ir_reaches_fp64_residual(fs, orc, name, gen, prec, restart):
    A = gen()
    b = W.random_vector(A.n_rows, 46, W.BVEC)
    note("ir %s %s restart=%d" % (name, prec, restart))
    M = make(A)
    p = fs.PREC_IR_F32 if prec == "f32" else fs.PREC_IR_BF16
    x, info = fs.cg_solve(M, dev(b), precond=1, precision=p, inner_rtol=1e-2,
                          ir_restart=restart)
    xg = host(x)
    assert info["status"] == fs.FS_OK, info
    assert info["outer"] >= 2
    assert info["relres"] <= 1e-8
    assert true_relres(orc, A, xg, b) <= 1.001e-8
    xo, st, it, rr = orc.pcg(A, b, precond=1)
    assert np.linalg.norm(xg - xo) <= 4e-8 * kappa(A) * np.linalg.norm(xo)
    if prec == "f32" and restart == 0:
        # the kept-direction refinement of the oracle takes about as many
        # inner iterations (sums are ordered differently)
        _, sto, outo, ino, _ = orc.ir_cg(A, orc.round_f32(A.val), b,
                                         inner_rtol=1e-2, keep=True)
        assert sto == orc.OK
        assert abs(info["iters"] - ino) <= max(5, ino // 10), (info, ino)


# ------------------------------------------------------- batched systems
def batch_members():
    return [
        (W.poisson_2d_p1(20, seed=(47, 0), bc="all"), 1),
        (W.tet_p1(6, "elastic", seed=(47, 1), bc="x0", permute=True), 3),
        (W.poisson_2d_p1(33, seed=(47, 2), bc="all", permute=True), 2),
        (W.hex_q1(5, "laplace", seed=(47, 3), bc="all"), 1),
        (W.tet_p1(9, "laplace", seed=(47, 4), bc="all"), 16),
    ]


@pytest.mark.parametrize("precond", [0, 1])
def test_batch_alone_equals_mix(fs, orc, precond):
    """Every system of a batch gets bitwise the result of solving it alone,
    whatever else shares the launches (the reductions depend only on the
    system's own grid)."""
    mem = batch_members()
    note("cg batch of %d, precond %d" % (len(mem), precond))
    Ms = [make(A) for A, _ in mem]
    Bs = [W.random_vector(A.n_rows, 48, W.BVEC, i, k=k)
          for i, (A, k) in enumerate(mem)]
    alone = []
    for M, B in zip(Ms, Bs):
        X, inf = fs.cg_solve_multi(M, dev(B), precond=precond)
        alone.append((host(X), [i["iters"] for i in inf]))
    Xs, infos = fs.cg_solve_batch(Ms, [dev(B) for B in Bs], precond=precond)
    j = 0
    for (A, k), X, B, (Xa, its) in zip(mem, Xs, Bs, alone):
        Xh = host(X)
        assert np.array_equal(Xh, Xa)
        for c in range(k):
            assert infos[j]["iters"] == its[c]
            assert infos[j]["status"] == fs.FS_OK
            assert true_relres(orc, A, Xh[:, c], B[:, c]) <= 1.001e-8
            j += 1
    # a different mix: reversed order, half the members
    sub = list(range(len(mem)))[::-2]
    Xs2, _ = fs.cg_solve_batch([Ms[i] for i in sub],
                               [dev(Bs[i]) for i in sub], precond=precond)
    for i, X in zip(sub, Xs2):
        assert np.array_equal(host(X), alone[i][0])


def test_batch_reports_per_rhs_status(fs, orc):
    Ind = CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
              np.array([1.0, -1.0]))
    A = W.poisson_2d_p1(12, seed=(49, 0), bc="all")
    note("cg batch status")
    Ms = [make(A), make(Ind)]
    Bs = [dev(W.random_vector(A.n_rows, 49, W.BVEC)), dev(np.ones(2))]
    Xs, infos = fs.cg_solve_batch(Ms, Bs, precond=0, check=False)
    assert infos[0]["status"] == fs.FS_OK
    assert infos[1]["status"] == fs.FS_E_BREAKDOWN
    assert true_relres(orc, A, host(Xs[0]).reshape(-1),
                       host(Bs[0])) <= 1.001e-8
