"""Finite-element meshes and their assembled stiffness matrices (CSR, FP64).

The paper's matrices come from unstructured finite element meshes: linear
tetrahedra of a heart geometry plus a public benchmark suite (benchmark
section, matrix information table).  Neither is available here, so this module
builds seeded synthetic stand-ins with the same character:

* P1 triangles on a jittered unit square (2-D Poisson);
* P1 tetrahedra from the Kuhn (Freudenthal) 6-tet split of a jittered cube
  grid, Laplacian or isotropic linear elasticity (3 DOF per node);
* P2 (10-node) tetrahedra on the same split;
* Q1 (8-node trilinear) hexahedra, 27-point connectivity;
* graded 2-D triangle meshes with a skewed row-length distribution.

All meshes are structured in *topology* (a grid of cells) but jittered in
geometry, and may be renumbered randomly, which is what makes them look
unstructured to a sparse kernel.  Assembly of a grid-topology mesh is done
per neighbour offset ("stencil" assembly) so that tens of millions of
non-zeros assemble in seconds with numpy; the graded meshes use a generic
element-by-element COO assembly.

Conventions
-----------
* node id of grid index (i0, i1, i2) is ``i0 + n0*(i1 + n1*i2)``;
* DOF id is ``dof*node + component`` (a node's components stay adjacent);
* the sparsity pattern is the element connectivity: every pair of nodes that
  share an element is a structural non-zero, and exact zeros produced by the
  geometry are *kept*, so ``nnz`` never depends on the values;
* columns are sorted ascending inside every row; indices are int32.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from .seeds import rng as _rng, JITTER, PERM


# --------------------------------------------------------------------------
# container
# --------------------------------------------------------------------------
@dataclass
class CSR:
    n_rows: int
    n_cols: int
    rowptr: np.ndarray  # int32, n_rows + 1
    col: np.ndarray     # int32, nnz
    val: np.ndarray     # float64, nnz
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def to_dense(self) -> np.ndarray:
        if self.n_rows * self.n_cols > 16_000_000:
            raise ValueError("to_dense is for tiny matrices only")
        a = np.zeros((self.n_rows, self.n_cols))
        rows = np.repeat(np.arange(self.n_rows), self.row_lengths())
        np.add.at(a, (rows, self.col), self.val)
        return a

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr),
                             shape=(self.n_rows, self.n_cols))


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def structured_grid(shape, jitter=0.2, seed=None):
    """Node coordinates of a grid on the unit square/cube.

    ``shape`` is the number of nodes per dimension.  Interior nodes are moved
    by an independent uniform draw in [-jitter*h, +jitter*h] per coordinate
    (h = 1/(n-1) per dimension); boundary nodes stay on the boundary so the
    domain is exact.  ``seed`` is a ``(cfg, idx)`` pair (draw purpose JITTER)
    or None for an unjittered grid.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    h = np.array([1.0 / (s - 1) for s in shape])
    idx = np.indices(shape[::-1]).reshape(d, -1)[::-1].T  # (N, d), i0 fastest
    X = idx * h
    if seed is not None and jitter > 0:
        g = _rng(seed[0], JITTER, seed[1])
        disp = g.uniform(-jitter, jitter, size=X.shape) * h
        interior = np.all((idx > 0) & (idx < np.array(shape) - 1), axis=1)
        X = X + disp * interior[:, None]
    return X, idx


def _lin(off, shape):
    """Linear node-id offset of an integer grid offset vector."""
    s = 1
    out = 0
    for k, n in enumerate(shape):
        out += int(off[k]) * s
        s *= n
    return out


# --------------------------------------------------------------------------
# reference elements: local node offsets (grid units) and shape-function
# derivatives at quadrature points
# --------------------------------------------------------------------------
def _kuhn_tets():
    """The 6 tetrahedra of the Kuhn split of the unit cube.

    Tet for permutation s of the axes: (0,0,0) -> e_s0 -> e_s0+e_s1 ->
    (1,1,1).  Vertices are reordered so the reference orientation is
    positive.  All 6 share the main diagonal; every interior node gets 14
    neighbours (the axis, face-diagonal and body-diagonal (1,1,...) ones).
    """
    tets = []
    for s in itertools.permutations(range(3)):
        v = [np.zeros(3, int)]
        for a in s:
            v.append(v[-1].copy())
            v[-1][a] = 1
        v = np.array(v)
        e = (v[1:] - v[0]).astype(float)
        if np.linalg.det(e) < 0:
            v[[1, 2]] = v[[2, 1]]
        tets.append(v)
    return tets


TRI_P1 = [np.array([[0, 0], [1, 0], [1, 1]]),   # SW, SE, NE
          np.array([[0, 0], [1, 1], [0, 1]])]   # SW, NE, NW (same diagonal)


def _p1_ref(d):
    g = np.zeros((d + 1, d))
    g[0, :] = -1.0
    g[1:, :] = np.eye(d)
    return g[None]  # (nq=1, nloc, d)


P1_WEIGHT = {2: 0.5, 3: 1.0 / 6.0}  # reference simplex measure


def _q1_ref():
    """Trilinear hex on [0,1]^3, 2x2x2 Gauss points; local node a has
    offset (a0, a1, a2) with a0 fastest."""
    offs = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    pts = np.array([[a, b, c] for c in gp for b in gp for a in gp])
    w = np.full(len(pts), 1.0 / 8.0)
    dN = np.zeros((len(pts), 8, 3))
    for q, xi in enumerate(pts):
        for a, o in enumerate(offs):
            f = [xi[k] if o[k] else 1.0 - xi[k] for k in range(3)]
            df = [1.0 if o[k] else -1.0 for k in range(3)]
            dN[q, a, 0] = df[0] * f[1] * f[2]
            dN[q, a, 1] = f[0] * df[1] * f[2]
            dN[q, a, 2] = f[0] * f[1] * df[2]
    return offs, dN, w


P2_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def _p2_ref():
    """10-node quadratic tet: barycentric L = (1-x-y-z, x, y, z); vertex
    functions L_i(2L_i-1), edge functions 4 L_i L_j; the 4-point degree-2
    rule (exact for stiffness of straight-sided elements)."""
    a, b = 0.5854101966249685, 0.1381966011250105
    bary = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    w = np.full(4, 1.0 / 24.0)
    dL = np.array([[-1.0, -1.0, -1.0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    dN = np.zeros((4, 10, 3))
    for q, L in enumerate(bary):
        for i in range(4):
            dN[q, i] = (4.0 * L[i] - 1.0) * dL[i]
        for e, (i, j) in enumerate(P2_EDGES):
            dN[q, 4 + e] = 4.0 * (L[j] * dL[i] + L[i] * dL[j])
    return dN, w


def _physical_gradients(dN, X):
    """dN (nq, nloc, d) reference derivatives, X (ne, nloc, d) coordinates.
    Returns G (ne, nq, nloc, d) physical gradients and detM (ne, nq)."""
    # M[k, i] = d x_i / d xi_k
    M = np.einsum("qak,eai->eqki", dN, X)
    det = np.linalg.det(M)
    Minv = np.linalg.inv(M)
    # grad_x N_a = M^{-1} grad_xi N_a   ->  G[a, i] = sum_k Minv[i, k] dN[a, k]
    G = np.einsum("eqik,qak->eqai", Minv, dN)
    return G, det


def _laplace_kernel(G, wdet):
    # K_ab = sum_q w|det| grad N_a . grad N_b, one batched product per
    # coordinate direction
    ne, nq, nloc, d = G.shape
    out = np.zeros((ne, nloc, nloc))
    for i in range(d):
        gi = np.ascontiguousarray(G[:, :, :, i])              # (ne, nq, nloc)
        wgt = np.ascontiguousarray((gi * wdet[:, :, None]).transpose(0, 2, 1))
        out += np.matmul(wgt, gi)
    return out


def _elastic_kernel(lam, mu):
    def k(G, wdet):
        # M[i][j][e, a, b] = sum_q w dN_a/dx_i dN_b/dx_j; the element matrix
        # K[a,i,b,j] = lam M[i][j] + mu M[j][i] + mu d_ij sum_k M[k][k]
        ne, nq, nloc, d = G.shape
        gd = [np.ascontiguousarray(G[:, :, :, i]) for i in range(d)]
        wgt = [np.ascontiguousarray((g * wdet[:, :, None]).transpose(0, 2, 1))
               for g in gd]
        M = [[np.matmul(wgt[i], gd[j]) for j in range(d)] for i in range(d)]
        tr = M[0][0].copy()
        for i in range(1, d):
            tr += M[i][i]
        K = np.empty((ne, nloc, d, nloc, d))
        for i in range(d):
            for j in range(d):
                blk = lam * M[i][j] + mu * M[j][i]
                if i == j:
                    blk += mu * tr
                K[:, :, i, :, j] = blk
        return K.reshape(ne, nloc * d, nloc * d)
    return k


def lame(E=1.0, nu=0.3):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu


# --------------------------------------------------------------------------
# stencil assembly over a grid of cells
# --------------------------------------------------------------------------
def _assemble_stencil(shape, X, etypes, cell_shape, stride, dN, w, kernel,
                      dof, chunk=16384, check_orientation=True):
    """Assemble element matrices of every cell into per-node stencils.

    Returns S (N, nD, dof, dof), cov (N, nD) and the offset list D (nD, d).
    Every (element type, local pair a, b) maps cells one-to-one onto the
    node of local vertex a, so plain fancy-index accumulation is exact.
    """
    d = len(shape)
    N = int(np.prod(shape))
    offs = set()
    for t in etypes:
        for a in t:
            for b in t:
                offs.add(tuple(int(v) for v in (b - a)))
    D = np.array(sorted(offs), dtype=np.int64).reshape(-1, d)
    dindex = {tuple(o): i for i, o in enumerate(D)}
    S = np.zeros((N, len(D), dof, dof))
    cov = np.zeros((N, len(D)), dtype=bool)

    cidx = np.indices(cell_shape[::-1]).reshape(d, -1)[::-1].T * stride
    clin = np.zeros(len(cidx), dtype=np.int64)
    s = 1
    for k in range(d):
        clin += cidx[:, k] * s
        s *= shape[k]
    for t in etypes:
        tl = np.array([_lin(o, shape) for o in t], dtype=np.int64)
        nl = len(t)
        # for a fixed local node a the offsets t[b] - t[a] are distinct, so
        # one scatter per a touches each (node, offset) slot at most once
        dis = np.array([[dindex[tuple(int(v) for v in (t[b] - t[a]))]
                         for b in range(nl)] for a in range(nl)])
        for c0 in range(0, len(clin), chunk):
            nodes = clin[c0:c0 + chunk, None] + tl[None, :]
            Xe = X[nodes]
            G, det = _physical_gradients(dN, Xe)
            if check_orientation and not np.all(det > 0):
                raise ValueError("inverted element after jitter")
            Ke = kernel(G, np.abs(det) * w[None, :])
            Kt = Ke.reshape(-1, nl, dof, nl, dof).transpose(0, 1, 3, 2, 4)
            for a in range(nl):
                ia = nodes[:, a, None]
                S[ia, dis[a][None, :]] += Kt[:, a]
                cov[ia, dis[a][None, :]] = True
    return S, cov, D


def _stencil_to_csr(S, cov, D, shape, keep, old_of_new, dof, chunk=131072):
    """Emit CSR rows for kept nodes in the order ``old_of_new``.

    Columns are the kept neighbours' new DOF ids, sorted ascending."""
    N = S.shape[0]
    Nk = len(old_of_new)
    new_of_old = np.full(N, -1, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(Nk)
    linD = np.array([_lin(o, shape) for o in D], dtype=np.int64)
    big = np.iinfo(np.int64).max
    rowlen = np.zeros(Nk * dof, dtype=np.int64)
    cols, vals = [], []
    for c0 in range(0, Nk, chunk):
        p = old_of_new[c0:c0 + chunk]
        q = p[:, None] + linD[None, :]
        qc = np.clip(q, 0, N - 1)
        valid = cov[p] & keep[qc]
        qnew = np.where(valid, new_of_old[qc], big)
        order = np.argsort(qnew, axis=1, kind="stable")
        qs = np.take_along_axis(qnew, order, 1)
        vs = np.take_along_axis(valid, order, 1)
        Sp = S[p[:, None], order]
        cc = dof * np.where(vs, qs, 0)[:, None, :, None] + \
            np.arange(dof)[None, None, None, :]
        cc = np.broadcast_to(cc, (len(p), dof, len(D), dof))
        vv = Sp.transpose(0, 2, 1, 3)
        m = np.broadcast_to(vs[:, None, :, None], cc.shape)
        cols.append(cc[m].astype(np.int32))
        vals.append(vv[m])
        rowlen[c0 * dof:(c0 + len(p)) * dof] = np.repeat(vs.sum(1) * dof, dof)
    rowptr = np.zeros(Nk * dof + 1, dtype=np.int64)
    np.cumsum(rowlen, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    return (rowptr.astype(np.int32), np.concatenate(cols),
            np.concatenate(vals))


def _numbering(keep, permute, seed):
    kept = np.nonzero(keep)[0]
    if permute:
        g = _rng(seed[0], PERM, seed[1])
        return kept[g.permutation(len(kept))]
    return kept


def _finish(shape, X, etypes, cell_shape, stride, dN, w, kernel, dof,
            keep, permute, seed, meta):
    S, cov, D = _assemble_stencil(shape, X, etypes, cell_shape, stride, dN,
                                  w, kernel, dof)
    old_of_new = _numbering(keep, permute, seed)
    rowptr, col, val = _stencil_to_csr(S, cov, D, shape, keep, old_of_new,
                                       dof)
    n = len(old_of_new) * dof
    meta = dict(meta)
    meta.update(node_ids=old_of_new, dof=dof, coords=X[old_of_new])
    return CSR(n, n, rowptr, col, val, meta)


def _keep_mask(idx, shape, bc):
    shape = np.array(shape)
    if bc == "none":
        return np.ones(len(idx), dtype=bool)
    if bc == "all":      # remove every boundary node (Dirichlet everywhere)
        return np.all((idx > 0) & (idx < shape - 1), axis=1)
    if bc == "x0":       # clamp the x = 0 face
        return idx[:, 0] > 0
    raise ValueError(bc)


# --------------------------------------------------------------------------
# public generators
# --------------------------------------------------------------------------
def poisson_2d_p1(n, jitter=0.2, seed=None, bc="all", permute=False):
    """P1 triangles on an n x n node unit square, every cell split along
    its SW-NE diagonal.  ``bc='all'`` removes the Dirichlet boundary rows and
    columns; ``bc='none'`` keeps the singular Neumann matrix."""
    shape = (n, n)
    X, idx = structured_grid(shape, jitter, seed)
    keep = _keep_mask(idx, shape, bc)
    meta = dict(kind="poisson2d_p1", n=n, bc=bc, h=1.0 / (n - 1))
    return _finish(shape, X, TRI_P1, (n - 1, n - 1), 1, _p1_ref(2),
                   np.array([P1_WEIGHT[2]]), _laplace_kernel, 1, keep,
                   permute, seed, meta)


def tet_p1(n, physics="laplace", jitter=0.2, seed=None, bc="none",
           permute=False, E=1.0, nu=0.3):
    """Kuhn 6-tet split of an n^3 node cube, linear tetrahedra."""
    shape = (n, n, n)
    X, idx = structured_grid(shape, jitter, seed)
    keep = _keep_mask(idx, shape, bc)
    if physics == "laplace":
        kern, dof = _laplace_kernel, 1
    else:
        kern, dof = _elastic_kernel(*lame(E, nu)), 3
    meta = dict(kind=f"tet_p1_{physics}", n=n, bc=bc, h=1.0 / (n - 1))
    return _finish(shape, X, _kuhn_tets(), (n - 1,) * 3, 1, _p1_ref(3),
                   np.array([P1_WEIGHT[3]]), kern, dof, keep, permute, seed,
                   meta)


def hex_q1(n, physics="laplace", jitter=0.2, seed=None, bc="none",
           permute=False, E=1.0, nu=0.3):
    """Trilinear hexahedra on an n^3 node cube (27-point connectivity)."""
    shape = (n, n, n)
    X, idx = structured_grid(shape, jitter, seed)
    keep = _keep_mask(idx, shape, bc)
    offs, dN, w = _q1_ref()
    if physics == "laplace":
        kern, dof = _laplace_kernel, 1
    else:
        kern, dof = _elastic_kernel(*lame(E, nu)), 3
    meta = dict(kind=f"hex_q1_{physics}", n=n, bc=bc, h=1.0 / (n - 1))
    return _finish(shape, X, [offs], (n - 1,) * 3, 1, dN, w, kern, dof,
                   keep, permute, seed, meta)


def tet_p2(cells, physics="laplace", jitter=0.2, seed=None, bc="none",
           permute=False, E=1.0, nu=0.3):
    """Quadratic 10-node tetrahedra on the Kuhn split of a cube with
    ``cells`` cells per side.  Vertices are jittered; mid-edge nodes sit at
    the midpoints of the (jittered) straight edges.  Every mid-edge node of
    the Kuhn split lies on the twice-refined grid, so the P2 nodes are the
    (2*cells+1)^3 refined grid points."""
    nc = cells + 1
    Xc, _ = structured_grid((nc,) * 3, jitter, seed)
    nf = 2 * cells + 1
    shape = (nf,) * 3
    fidx = np.indices(shape[::-1]).reshape(3, -1)[::-1].T
    lo, hi = fidx // 2, (fidx + 1) // 2

    def cl(ix):
        return ix[:, 0] + nc * (ix[:, 1] + nc * ix[:, 2])
    X = 0.5 * (Xc[cl(lo)] + Xc[cl(hi)])
    keep = _keep_mask(fidx, shape, bc)
    etypes = []
    for t in _kuhn_tets():
        v = 2 * t
        mids = [(v[i] + v[j]) // 2 for i, j in P2_EDGES]
        etypes.append(np.vstack([v] + mids))
    dN, w = _p2_ref()
    if physics == "laplace":
        kern, dof = _laplace_kernel, 1
    else:
        kern, dof = _elastic_kernel(*lame(E, nu)), 3
    meta = dict(kind=f"tet_p2_{physics}", cells=cells, bc=bc)
    return _finish(shape, X, etypes, (cells,) * 3, 2, dN, w, kern, dof,
                   keep, permute, seed, meta)


def laplace_1d_p1(n_el):
    """P1 line elements on [0, 1] with both ends clamped: the (n_el-1)
    interior rows of the stiffness matrix and the exact load vector for a
    unit source (each hat function integrates to h)."""
    h = 1.0 / n_el
    m = n_el - 1
    rows, cols, vals = [], [], []
    for i in range(m):
        for j, v in ((i - 1, -1.0 / h), (i, 2.0 / h), (i + 1, -1.0 / h)):
            if 0 <= j < m:
                rows.append(i)
                cols.append(j)
                vals.append(v)
    rowptr = np.zeros(m + 1, dtype=np.int32)
    np.add.at(rowptr, np.array(rows) + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    x = np.arange(1, n_el) * h
    return (CSR(m, m, rowptr, np.array(cols, np.int32), np.array(vals),
                dict(kind="laplace1d_p1", h=h, coords=x)),
            np.full(m, h))


def graded_2d_p1(n, hubs=None, seed=None, jitter=0.2, max_row=200,
                 permute=False):
    """Graded 2-D triangle mesh with a skewed row-length distribution.

    Start from the n x n structured P1 triangle mesh.  A seeded set of hub
    nodes (at least 4 grid steps apart) is refined: for hub v with fan factor
    m (geometric law, capped so the hub row stays within ``max_row``), every
    edge of v's 1-ring is subdivided into m pieces and each incident
    triangle is re-fanned from v through the new points; the neighbouring
    triangle across that ring edge is re-fanned from its opposite vertex so
    the mesh stays conforming.  Hub rows get up to ``max_row`` entries,
    ordinary rows keep 7.  P1 Laplacian, Neumann (singular, SpMV only).
    """
    from .graded import build_graded
    return build_graded(n, hubs=hubs, seed=seed, jitter=jitter,
                        max_row=max_row, permute=permute)
