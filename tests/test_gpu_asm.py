"""GPU parity of finite-element assembly into the layout (asm_*) against the
oracle's element loop: bitwise, since both add the same contributions in
element order starting from 0.0."""
import numpy as np
import pytest

import workloads as W
from workloads.elements import (config1_elements, poisson_2d_p1_elements,
                                tet_p1_elements)
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


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.int64)


def same_bits(a, b):
    return np.array_equal(bits(a), bits(b))


CASES = [
    ("p2d_cfg0", lambda: (W.config0_poisson2d(),
                          poisson_2d_p1_elements(64, seed=(0, 0), bc="all")),
     {}),
    ("p2d_perm", lambda: (W.poisson_2d_p1(23, seed=(80, 0), bc="none",
                                          permute=True),
                          poisson_2d_p1_elements(23, seed=(80, 0), bc="none",
                                                 permute=True)),
     dict(dtypes=6)),
    ("lap9_perm", lambda: (W.tet_p1(9, "laplace", seed=(80, 1), bc="all",
                                    permute=True),
                           tet_p1_elements(9, "laplace", seed=(80, 1),
                                           bc="all", permute=True)),
     dict(vec=1)),
    ("ela8_x0", lambda: (W.tet_p1(8, "elastic", seed=(80, 2), bc="x0",
                                  permute=True),
                         tet_p1_elements(8, "elastic", seed=(80, 2), bc="x0",
                                         permute=True)),
     dict(dtypes=6, index_bits=32)),
    ("ela7_none", lambda: (W.tet_p1(7, "elastic", seed=(80, 3)),
                           tet_p1_elements(7, "elastic", seed=(80, 3))),
     dict(reorder=1, lanes_max=4)),
]


def test_config0_elements_match_config0_mesh():
    """The element data of the 2-D workload is that of config 0's mesh
    (same jitter seed, same removed rows) -- a host-side check."""
    A = W.config0_poisson2d()
    E = poisson_2d_p1_elements(64, seed=(0, 0), bc="all")
    assert E.n_rows == A.n_rows == 3844


@pytest.mark.parametrize("plan", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_assembly_bitwise(fs, orc, case, plan):
    name, gen, opts = CASES[case]
    A, E = gen()
    note("asm %s plan=%d n=%d nnz=%d elems=%d nde=%d opts=%s" % (
        name, plan, A.n_rows, A.nnz, E.n_elem, E.nde, opts))
    # the handle starts from unrelated values: assembly replaces them all
    M = make(CSR(A.n_rows, A.n_cols, A.rowptr, A.col, A.val * 3.0 + 1.0),
             **opts)
    P = fs.asm_create(M, dev(E.edof), plan=plan)
    info = fs.asm_info(P)
    assert info["plan"] == (fs.ASM_ROWGROUP if plan == 0 else fs.ASM_GATHER)
    want = orc.assemble_matrix(A, E.edof, E.ke)
    r_want = orc.assemble_vector(A.n_rows, E.edof, E.re)
    ne, nde = E.edof.shape
    assert info["contrib_matrix"] == int(np.sum(
        (E.edof[:, :, None] >= 0) & (E.edof[:, None, :] >= 0)))
    assert info["contrib_vector"] == int(np.sum(E.edof >= 0))
    assert info["stored_matrix"] >= info["contrib_matrix"]
    fs.asm_matrix(P, dev(E.ke))
    got = host(fs.csr_get_values(M))
    assert same_bits(got, want), "%d entries differ" % np.sum(
        bits(got) != bits(want))
    r = host(fs.asm_vector(P, dev(E.re)))
    assert same_bits(r, r_want)
    # the product reads what was assembled: bitwise a handle built from the
    # oracle's values with the same options
    Mo = make(CSR(A.n_rows, A.n_cols, A.rowptr, A.col, want), **opts)
    x = W.random_vector(A.n_cols, 80, W.XVEC, case)
    assert same_bits(host(fs.spmv(M, dev(x))), host(fs.spmv(Mo, dev(x))))
    dt = opts.get("dtypes", 0)
    if dt:
        import torch
        perm = fs.csr_get_perm(M)
        xp = dev(x[perm].astype(np.float32))
        for d in (fs.DT_F32, fs.DT_BF16):
            if dt & d:
                ya = host(fs.spmv_lowp(M, d, xp))
                yb = host(fs.spmv_lowp(Mo, d, xp))
                assert np.array_equal(ya.view(np.int32), yb.view(np.int32))
    # a second assembly with new element values replaces the first
    ke2 = E.ke * -0.5
    fs.asm_matrix(P, dev(ke2))
    assert same_bits(host(fs.csr_get_values(M)),
                     orc.assemble_matrix(A, E.edof, ke2))
    # element rows stored in the plan's order stream in (row-group plan)
    if plan == 0:
        pos, nrows = fs.asm_element_rows(P)
        assert np.array_equal(np.sort(pos[pos >= 0]),
                              np.unique(pos[pos >= 0]))
        assert np.all((pos >= 0) == (E.edof.reshape(-1) >= 0))
        ko = np.full((nrows, E.nde), np.nan)      # unused rows: never used
        keep = pos >= 0
        ko[pos[keep]] = E.ke.reshape(-1, E.nde)[keep] * 0.25
        fs.asm_matrix_ordered(P, dev(ko))
        assert same_bits(host(fs.csr_get_values(M)),
                         orc.assemble_matrix(A, E.edof, E.ke * 0.25))
    else:
        with pytest.raises(fs.FsError) as ei:
            fs.asm_element_rows(P)
        assert ei.value.status == fs.FS_E_UNSUPPORTED
    # matrix and vector in one pass: the same bits as the separate calls
    ke3, re3 = E.ke * 1.25 + 0.5, E.re - 0.75
    r3 = host(fs.asm_system(P, dev(ke3), dev(re3)))
    assert same_bits(host(fs.csr_get_values(M)),
                     orc.assemble_matrix(A, E.edof, ke3))
    assert same_bits(r3, orc.assemble_vector(A.n_rows, E.edof, re3))


def test_untouched_entries_and_dropped_dofs(fs, orc):
    """Pattern entries no element reaches come out 0; elements whose DOFs
    are all dropped contribute nothing; empty element sets give zeros."""
    A = W.tet_p1(5, "laplace", seed=(81, 0), bc="all", permute=True)
    E = tet_p1_elements(5, "laplace", seed=(81, 0), bc="all", permute=True)
    # keep every other element of the first half of the cells only
    sel = np.arange(0, E.n_elem // 2, 2)
    edof, ke, re = E.edof[sel], E.ke[sel], E.re[sel]
    note("asm subset n=%d elems=%d" % (A.n_rows, len(sel)))
    M = make(A)
    P = fs.asm_create(M, dev(edof))
    fs.asm_matrix(P, dev(ke))
    want = orc.assemble_matrix(A, edof, ke)
    assert np.any(want == 0.0)
    assert same_bits(host(fs.csr_get_values(M)), want)
    assert same_bits(host(fs.asm_vector(P, dev(re))),
                     orc.assemble_vector(A.n_rows, edof, re))
    # no elements at all
    note("asm empty element set")
    P0 = fs.asm_create(M, dev(np.zeros((0, 4), np.int32)))
    import torch
    fs.asm_matrix(P0, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert np.all(host(fs.csr_get_values(M)) == 0.0)
    r = fs.asm_vector(P0, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert np.all(host(r) == 0.0)
    fs.csr_update_values(M, dev(A.val))
    r = fs.asm_system(P0, torch.zeros(0, dtype=torch.float64, device="cuda"),
                      torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert np.all(host(r) == 0.0)
    assert np.all(host(fs.csr_get_values(M)) == 0.0)


def test_non_finite_contributions_stay_local(fs, orc):
    A = W.poisson_2d_p1(9, seed=(82, 0), bc="all", permute=True)
    E = poisson_2d_p1_elements(9, seed=(82, 0), bc="all", permute=True)
    ke = E.ke.copy()
    inner = np.nonzero(np.all(E.edof >= 0, axis=1))[0]
    ke[inner[0], 1, 1] = np.nan
    ke[inner[-1], 0, 2] = np.inf
    note("asm non-finite n=%d" % A.n_rows)
    M = make(A)
    P = fs.asm_create(M, dev(E.edof))
    fs.asm_matrix(P, dev(ke))
    got = host(fs.csr_get_values(M))
    want = orc.assemble_matrix(A, E.edof, ke)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    fin = ~np.isnan(want)
    assert same_bits(got[fin], want[fin])
    assert np.isnan(want).sum() >= 1 and np.isinf(want).sum() >= 1


def test_repeated_dof_falls_back_to_gather(fs, orc):
    """An element that lists a DOF twice adds both entries, in (a, b)
    order; the row-group plan does not apply, the gather plan does."""
    A = W.poisson_2d_p1(8, seed=(83, 1), bc="none")
    E = poisson_2d_p1_elements(8, seed=(83, 1), bc="none")
    ed = E.edof.copy()
    ed[7, 2] = ed[7, 0]
    note("asm repeated dof")
    M = make(A)
    with pytest.raises(fs.FsError) as ei:
        fs.asm_create(M, dev(ed), plan=fs.ASM_ROWGROUP)
    assert ei.value.status == fs.FS_E_UNSUPPORTED
    P = fs.asm_create(M, dev(ed))
    assert fs.asm_info(P)["plan"] == fs.ASM_GATHER
    fs.asm_matrix(P, dev(E.ke))
    assert same_bits(host(fs.csr_get_values(M)),
                     orc.assemble_matrix(A, ed, E.ke))


def test_errors(fs):
    A = W.poisson_2d_p1(6, seed=(83, 0), bc="all")
    E = poisson_2d_p1_elements(6, seed=(83, 0), bc="all")
    M = make(A)
    note("asm error paths")
    bad = E.edof.copy()
    bad[3, 1] = A.n_rows          # out of range
    with pytest.raises(fs.FsError) as ei:
        fs.asm_create(M, dev(bad))
    assert ei.value.status == fs.FS_E_ARG
    # a pattern that lacks couplings: the diagonal matrix
    n = A.n_rows
    D = CSR(n, n, np.arange(n + 1, dtype=np.int32),
            np.arange(n, dtype=np.int32), np.ones(n))
    MD = make(D)
    with pytest.raises(fs.FsError) as ei:
        fs.asm_create(MD, dev(E.edof))
    assert ei.value.status == fs.FS_E_BAD_CSR
    assert "element" in str(ei.value)


def test_newton_step_assemble_then_solve(fs, orc):
    """Assemble K and R straight into the layout, then solve K u = R: the
    same result as solving the oracle-assembled system (FP64 Jacobi-PCG)."""
    n = 10
    A = W.tet_p1(n, "elastic", seed=(84, 0), bc="x0", permute=True)
    E = tet_p1_elements(n, "elastic", seed=(84, 0), bc="x0", permute=True)
    note("asm+cg ela n=%d rows=%d" % (n, A.n_rows))
    M = make(A)
    P = fs.asm_create(M, dev(E.edof))
    fs.asm_matrix(P, dev(E.ke))
    R = fs.asm_vector(P, dev(E.re))
    x, info = fs.cg_solve(M, R)
    assert info["status"] == fs.FS_OK
    K = CSR(A.n_rows, A.n_cols, A.rowptr, A.col,
            orc.assemble_matrix(A, E.edof, E.ke))
    b = orc.assemble_vector(A.n_rows, E.edof, E.re)
    res = b - orc.spmv(K, host(x))
    assert np.linalg.norm(res) <= 1.001e-8 * np.linalg.norm(b)
    # gravity pulls the free end down
    assert host(x).reshape(-1, 3)[:, 2].min() < 0


def test_config1_full_size(fs, orc):
    """The 3-D elasticity workload at full size (774,144 rows, 1.5M
    elements): every assembled value and load entry against the oracle."""
    A = W.config1_elasticity3d()
    E = config1_elements()
    note("asm config1 rows=%d nnz=%d elems=%d" % (A.n_rows, A.nnz,
                                                   E.n_elem))
    M = make(A)
    ke = dev(E.ke)
    want = orc.assemble_matrix(A, E.edof, E.ke)
    for plan in (fs.ASM_ROWGROUP, fs.ASM_GATHER):
        note("asm config1 plan=%d" % plan)
        P = fs.asm_create(M, dev(E.edof), plan=plan)
        fs.asm_matrix(P, ke)
        got = host(fs.csr_get_values(M))
        assert same_bits(got, want)
        info = fs.asm_info(P)
        assert info["stored_matrix"] <= 1.2 * info["contrib_matrix"]
    rwant = orc.assemble_vector(A.n_rows, E.edof, E.re)
    assert same_bits(host(fs.asm_vector(P, dev(E.re))), rwant)
    note("asm config1 ordered")
    P = fs.asm_create(M, dev(E.edof))
    pos, nrows = fs.asm_element_rows(P)
    ko = np.zeros((nrows, E.nde))
    keep = pos >= 0
    ko[pos[keep]] = E.ke.reshape(-1, E.nde)[keep]
    import torch
    fs.csr_update_values(M, torch.zeros(A.nnz, dtype=torch.float64,
                                        device="cuda"))
    fs.asm_matrix_ordered(P, dev(ko))
    assert same_bits(host(fs.csr_get_values(M)), want)
    note("asm config1 system")
    P = fs.asm_create(M, dev(E.edof))
    import torch
    fs.csr_update_values(M, torch.zeros(A.nnz, dtype=torch.float64,
                                        device="cuda"))
    r = host(fs.asm_system(P, ke, dev(E.re)))
    assert same_bits(host(fs.csr_get_values(M)), want)
    assert same_bits(r, rwant)
