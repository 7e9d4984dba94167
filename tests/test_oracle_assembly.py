"""Pins for the oracle's finite-element assembly (element loop, elements in
order).  Each check comes from the mathematics or from an independent
assembly, not from the oracle itself: closed-form 1-D and unjittered
stencils, the per-node stencil assembly of ``workloads.meshes`` (different
code, different summation order), null spaces, total load, and hand-derived
IEEE results that fix the summation order.
"""
import numpy as np
import pytest

import workloads as W
from workloads.elements import (line_p1_elements, poisson_2d_p1_elements,
                                tet_p1_elements)
from workloads.meshes import CSR

EPS = np.finfo(float).eps


def pair(kind, **kw):
    """(CSR from the stencil assembly, element data) of the same mesh."""
    if kind == "p2d":
        return W.poisson_2d_p1(**kw), poisson_2d_p1_elements(**kw)
    physics = kind.split("_")[1]
    return (W.tet_p1(physics=physics, **kw),
            tet_p1_elements(physics=physics, **kw))


CASES = [
    ("p2d", dict(n=5, seed=(70, 0), bc="none")),
    ("p2d", dict(n=8, seed=(70, 1), bc="all", permute=True)),
    ("tet_laplace", dict(n=3, seed=(70, 2))),
    ("tet_laplace", dict(n=5, seed=(70, 3), bc="all", permute=True)),
    ("tet_elastic", dict(n=4, seed=(70, 4), permute=True)),
    ("tet_elastic", dict(n=5, seed=(70, 5), bc="x0", permute=True)),
]


def test_1d_closed_form(orc):
    """P1 line elements: K = tridiag(-1, 2, -1) / h and R_i = h exactly
    (2 (1/h) = 2/h and h/2 + h/2 = h hold bitwise in IEEE arithmetic)."""
    for n_el in (2, 3, 7, 10, 64):
        A, load = W.laplace_1d_p1(n_el)
        E = line_p1_elements(n_el)
        val = orc.assemble_matrix(A, E.edof, E.ke)
        assert np.array_equal(val, A.val)
        r = orc.assemble_vector(E.n_rows, E.edof, E.re)
        assert np.array_equal(r, load)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_stencil_assembly(orc, case):
    """Same matrix as the per-node stencil assembly, to rounding: the two
    sum the same contributions in different orders, so they differ by at
    most (m - 1) eps times the sum of |contributions| (m <= 24 here)."""
    kind, kw = CASES[case]
    A, E = pair(kind, **kw)
    assert E.n_rows == A.n_rows
    val = orc.assemble_matrix(A, E.edof, E.ke)
    mag = orc.assemble_matrix(A, E.edof, np.abs(E.ke))
    assert np.all(np.abs(val - A.val) <= 24 * EPS * mag)
    # every pattern entry is reached by some element (values may be exact
    # zeros: unjittered boundary elements)
    hits = orc.assemble_matrix(A, E.edof, np.ones_like(E.ke))
    assert np.all(hits >= 1)


def test_unjittered_2d_is_five_point_stencil(orc):
    A, E = pair("p2d", n=10, jitter=0.0, bc="all")
    val = orc.assemble_matrix(A, E.edof, E.ke)
    D = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, val).to_dense()
    assert np.allclose(np.diag(D), 4.0, atol=1e-14)
    off = D - np.diag(np.diag(D))
    assert np.all(np.isclose(off, 0.0, atol=1e-15) |
                  np.isclose(off, -1.0, atol=1e-15))
    assert np.sum(np.isclose(off, -1.0)) == 2 * 2 * 8 * 7


def test_unjittered_kuhn_is_seven_point_stencil(orc):
    n = 6
    h = 1.0 / (n - 1)
    A, E = pair("tet_laplace", n=n, jitter=0.0, bc="all")
    val = orc.assemble_matrix(A, E.edof, E.ke)
    nz = val[np.abs(val) > 1e-14]
    assert np.allclose(np.sort(np.unique(np.round(nz / h, 12))), [-1, 6])
    D = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, val).to_dense()
    assert np.allclose(np.diag(D), 6 * h, atol=1e-14)


def test_neumann_row_sums_and_total_load(orc):
    """Pure Neumann Laplacian: rows sum to 0 (constants are in the null
    space); the load of f = 1 sums to the domain measure 1."""
    for kind, kw in [("p2d", dict(n=7, seed=(71, 0), bc="none")),
                     ("tet_laplace", dict(n=5, seed=(71, 1), permute=True))]:
        A, E = pair(kind, **kw)
        val = orc.assemble_matrix(A, E.edof, E.ke)
        rows = np.repeat(np.arange(A.n_rows), A.row_lengths())
        s = np.bincount(rows, val, A.n_rows)
        m = np.bincount(rows, np.abs(val), A.n_rows)
        assert np.all(np.abs(s) <= 1e-13 * m)
        r = orc.assemble_vector(E.n_rows, E.edof, E.re)
        assert abs(r.sum() - 1.0) < 1e-13
        assert np.all(r > 0)


def test_elasticity_null_space_and_gravity(orc):
    """Unconstrained elasticity annihilates the six rigid-body modes; the
    body force (0, 0, -1) over the unit cube sums to total force (0, 0, -1)."""
    A, E = pair("tet_elastic", n=4, seed=(72, 0), permute=True)
    val = orc.assemble_matrix(A, E.edof, E.ke)
    K = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, val)
    X = A.meta["coords"]
    modes = []
    for c in range(3):
        u = np.zeros((len(X), 3))
        u[:, c] = 1.0
        modes.append(u)
    for (i, j) in [(0, 1), (1, 2), (2, 0)]:
        u = np.zeros((len(X), 3))
        u[:, i] = -X[:, j]
        u[:, j] = X[:, i]
        modes.append(u)
    for u in modes:
        y = orc.spmv(K, u.reshape(-1))
        assert np.all(np.abs(y) <= 1e-12 * orc.spmv_abs(K, np.abs(u.reshape(-1))) + 1e-14)
    r = orc.assemble_vector(E.n_rows, E.edof, E.re).reshape(-1, 3)
    assert np.all(r[:, :2] == 0.0)
    assert abs(r[:, 2].sum() + 1.0) < 1e-13


def test_summation_order_is_element_order(orc):
    """Three one-DOF elements on the same entry with values 1, 1e-16, -1
    give exactly 0 in element order ((1 + 1e-16) rounds to 1); reversed they
    give 2^-53 (-1 + 1e-16 rounds up to -(1 - 2^-53))."""
    A = CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32),
            np.zeros(1))
    edof = np.zeros((3, 1), np.int32)
    fwd = np.array([1.0, 1e-16, -1.0]).reshape(3, 1, 1)
    assert orc.assemble_matrix(A, edof, fwd)[0] == 0.0
    assert orc.assemble_matrix(A, edof, fwd[::-1])[0] == 2.0 ** -53
    r = orc.assemble_vector(1, edof, fwd.reshape(3, 1))
    assert r[0] == 0.0


def test_dropped_dofs_and_untouched_entries(orc):
    """-1 entries of edof are skipped; pattern entries that no element
    touches come out 0; the sum over elements is the textbook one on a
    two-element chain."""
    # nodes 0-1-2, elements (0,1) and (1,2); node 0 dropped
    A = CSR(2, 2, np.array([0, 2, 4], np.int32),
            np.array([0, 1, 0, 1], np.int32), np.zeros(4))
    edof = np.array([[-1, 0], [0, 1]], np.int32)
    ke = np.array([[[1.0, -1.0], [-1.0, 1.0]],
                   [[2.0, -2.0], [-2.0, 2.0]]])
    val = orc.assemble_matrix(A, edof, ke)
    assert np.array_equal(val, [3.0, -2.0, -2.0, 2.0])
    # an extra pattern entry that no element reaches
    B = CSR(2, 2, np.array([0, 2, 4], np.int32),
            np.array([0, 1, 0, 1], np.int32), np.zeros(4))
    val = orc.assemble_matrix(B, np.array([[0, -1]], np.int32),
                              np.array([[[5.0, 7.0], [7.0, 9.0]]]))
    assert np.array_equal(val, [5.0, 0.0, 0.0, 0.0])
    r = orc.assemble_vector(2, edof, np.array([[1.0, 2.0], [3.0, 4.0]]))
    assert np.array_equal(r, [5.0, 4.0])


def test_missing_coupling_is_reported(orc):
    """A pattern without the (0, 1) entry cannot hold element 1's coupling."""
    A = CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
            np.zeros(2))
    edof = np.array([[0, -1], [0, 1]], np.int32)
    with pytest.raises(ValueError, match="element 1"):
        orc.assemble_matrix(A, edof, np.ones((2, 2, 2)))
