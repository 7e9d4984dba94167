"""Invariants of the seeded input generators (no oracle arithmetic here)."""
import numpy as np
import pytest

import workloads as W


def test_config0_sizes_and_determinism():
    A = W.config0_poisson2d()
    assert (A.n_rows, A.nnz) == (3844, 26414)
    rl = A.row_lengths()
    assert rl.min() == 3 and rl.max() == 7
    B = W.config0_poisson2d()
    assert np.array_equal(A.val, B.val) and np.array_equal(A.col, B.col)
    assert A.rowptr.dtype == np.int32 and A.col.dtype == np.int32


def test_config1_sizes():
    A = W.config1_elasticity3d()
    assert (A.n_rows, A.nnz) == (774144, 33967818)
    rl = A.row_lengths()
    assert rl.min() == 15 and rl.max() == 45
    # columns sorted and in range
    c = A.col
    starts = A.rowptr[:-1]
    assert c.min() >= 0 and c.max() < A.n_cols
    d = np.diff(c.astype(np.int64))
    inner = np.ones(len(d), bool)
    inner[starts[1:] - 1] = False
    assert np.all(d[inner] > 0)


@pytest.mark.parametrize("i,rows,nnz", [(0, 10648, 148366),
                                        (3, 10125, 408627),
                                        (6, 12167, 323093),
                                        (9, 10648, 262144)])
def test_sweep_small_sizes(i, rows, nnz):
    A = W.sweep_matrix(i, permuted=True)
    assert (A.n_rows, A.nnz) == (rows, nnz)


def test_unjittered_p2_row_lengths():
    A = W.tet_p2(4, "laplace", jitter=0.0)
    rl = A.row_lengths()
    assert rl.min() == 10 and rl.max() == 65


@pytest.mark.parametrize("gen", [
    lambda p: W.poisson_2d_p1(8, seed=(70, 0), bc="all", permute=p),
    lambda p: W.tet_p1(5, "elastic", seed=(70, 1), bc="x0", permute=p),
    lambda p: W.hex_q1(4, "laplace", seed=(70, 2), permute=p),
    lambda p: W.tet_p2(2, "elastic", seed=(70, 3), permute=p),
])
def test_permutation_is_a_relabelling(gen):
    """Natural and permuted orderings hold the same matrix, symmetrically
    renumbered by the node permutation (DOFs of a node stay adjacent)."""
    A, B = gen(False), gen(True)
    assert (A.n_rows, A.nnz) == (B.n_rows, B.nnz)
    dof = A.meta["dof"]
    pos = {nid: i for i, nid in enumerate(A.meta["node_ids"])}
    node_map = np.array([pos[n] for n in B.meta["node_ids"]])
    dmap = (dof * node_map[:, None] + np.arange(dof)).reshape(-1)
    Da, Db = A.to_dense(), B.to_dense()
    assert np.array_equal(Db, Da[np.ix_(dmap, dmap)])
    assert np.array_equal(Da, Da.T) or np.abs(Da - Da.T).max() < 1e-15


def test_jitter_keeps_boundary_and_bounds():
    X, idx = W.structured_grid((9, 9, 9), 0.2, seed=(71, 0))
    h = 1.0 / 8
    disp = X - idx * h
    bnd = np.any((idx == 0) | (idx == 8), axis=1)
    assert not disp[bnd].any()
    assert np.abs(disp).max() <= 0.2 * h
    assert np.abs(disp[~bnd]).max() > 0.15 * h


def test_random_vectors_are_seeded_uniform():
    a = W.random_vector(1000, 1, W.XVEC)
    b = W.random_vector(1000, 1, W.XVEC)
    c = W.random_vector(1000, 1, W.BVEC)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= -1 and a.max() <= 1


# ------------------------------------------------------ graded 2-D meshes
def graded_cases():
    return [W.graded_2d_p1(30, seed=(9, 0)),
            W.graded_2d_p1(30, seed=(9, 1), permute=True),
            W.graded_2d_p1(24, seed=(9, 2), hubs=[24 * 8 + 8, 24 * 15 + 15])]


@pytest.mark.parametrize("ci", range(3))
def test_graded_mesh_is_a_conforming_cover(ci):
    """Triangle areas add up to the unit square and every interior edge is
    shared by exactly two triangles, boundary edges by one (no gaps, no
    overlaps, no hanging nodes)."""
    A = graded_cases()[ci]
    X, T = A.meta["coords"], A.meta["triangles"]
    P = X[T]
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    assert np.all(det > 0)
    assert abs(0.5 * det.sum() - 1.0) < 1e-12
    E = np.sort(np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]]),
                axis=1)
    _, cnt = np.unique(E, axis=0, return_counts=True)
    assert set(np.unique(cnt)) <= {1, 2}
    ue, cnt = np.unique(E, axis=0, return_counts=True)
    mid = X[ue].mean(axis=1)
    on_bd = np.any((np.abs(mid) < 1e-12) | (np.abs(mid - 1) < 1e-12), axis=1)
    assert np.all(on_bd == (cnt == 1))


@pytest.mark.parametrize("ci", range(3))
def test_graded_laplacian_patch_test(ci):
    """P1 Laplacian: zero row sums (Neumann), symmetry, and A u = 0 at
    every interior node for a linear u -- fails for a non-conforming or
    mis-assembled mesh."""
    A = graded_cases()[ci]
    S = A.to_scipy()
    X = A.meta["coords"]
    assert np.max(np.abs(S @ np.ones(A.n_rows))) < 1e-12
    assert abs(S - S.T).max() < 1e-14
    u = 0.3 + 1.7 * X[:, 0] - 2.9 * X[:, 1]
    r = S @ u
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert np.max(np.abs(r[interior])) < 1e-11
    assert np.max(np.abs(r[~interior])) > 1e-3    # boundary flux is not 0


def test_graded_row_lengths():
    """Hub rows have 1 + 6 m entries; the distribution is skewed."""
    A = W.graded_2d_p1(24, seed=(9, 2), hubs=[24 * 8 + 8, 24 * 15 + 15],
                       max_row=200)
    L = A.row_lengths()
    assert L.max() == 1 + 6 * 33
    assert np.sum(L == L.max()) == 2
    B = W.sweep_matrix(13, permuted=False)
    LB = B.row_lengths()
    assert np.median(LB) == 7 and LB.max() > 100 and LB.min() >= 3
    C = W.sweep_matrix(13, permuted=False)
    assert np.array_equal(B.val, C.val)           # seeded: reproducible
