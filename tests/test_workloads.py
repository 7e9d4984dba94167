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
