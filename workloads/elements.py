"""Per-element inputs of finite-element assembly (element matrices, element
load vectors and the element-to-DOF map), for the same seeded meshes as
:mod:`workloads.meshes`.

Assembly itself (summing element contributions into global entries) is *not*
done here: that is the arithmetic under test.  These arrays are what an
element routine hands to the assembler: for element ``e``

* ``edof[e, a]`` -- row/column of local DOF ``a`` in the assembled matrix
  (the numbering of the matching CSR from :mod:`workloads.meshes`), or -1 for
  a DOF removed by a Dirichlet condition;
* ``ke[e, a, b]`` -- the element stiffness matrix;
* ``re[e, a]`` -- the element load vector (a body force).

Elements are numbered cell-major: element ``e`` is sub-element ``e % m`` of
grid cell ``e // m`` (``m`` elements per cell, cells with the first grid
index fastest).  Local DOF ``a`` is component ``a % dof`` of local node
``a // dof``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import (TRI_P1, P1_WEIGHT, _kuhn_tets, _p1_ref, _lin,
                     _physical_gradients, _laplace_kernel, _elastic_kernel,
                     _keep_mask, _numbering, lame, structured_grid)


@dataclass
class Elements:
    n_rows: int
    edof: np.ndarray   # int32 (ne, nde)
    ke: np.ndarray     # float64 (ne, nde, nde)
    re: np.ndarray     # float64 (ne, nde)
    meta: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.edof.shape[0])

    @property
    def nde(self) -> int:
        return int(self.edof.shape[1])


def _p1_elements(shape, X, etypes, kernel, dof, keep, permute, seed, force,
                 chunk=16384):
    d = len(shape)
    cell_shape = tuple(s - 1 for s in shape)
    cidx = np.indices(cell_shape[::-1]).reshape(d, -1)[::-1].T
    clin = np.zeros(len(cidx), dtype=np.int64)
    s = 1
    for k in range(d):
        clin += cidx[:, k] * s
        s *= shape[k]
    m = len(etypes)
    nl = d + 1
    nde = nl * dof
    tl = np.array([[_lin(o, shape) for o in t] for t in etypes],
                  dtype=np.int64)                           # (m, nl)
    nodes = (clin[:, None, None] + tl[None]).reshape(-1, nl)  # cell-major
    ne = len(nodes)
    dN, w = _p1_ref(d), np.array([P1_WEIGHT[d]])
    ke = np.empty((ne, nde, nde))
    vol = np.empty(ne)
    for e0 in range(0, ne, chunk):
        nd = nodes[e0:e0 + chunk]
        G, det = _physical_gradients(dN, X[nd])
        if not np.all(det > 0):
            raise ValueError("inverted element after jitter")
        wdet = np.abs(det) * w[None, :]
        ke[e0:e0 + chunk] = kernel(G, wdet)
        vol[e0:e0 + chunk] = wdet[:, 0]
    old_of_new = _numbering(keep, permute, seed)
    new_of_old = np.full(len(keep), -1, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(len(old_of_new))
    nn = new_of_old[nodes]                                   # (ne, nl)
    comp = np.arange(dof)
    edof = np.where(nn[:, :, None] >= 0, dof * nn[:, :, None] + comp, -1)
    edof = edof.reshape(ne, nde).astype(np.int32)
    # a P1 hat function integrates to |T| / (d + 1) over its element
    f = np.asarray(force, dtype=float).reshape(dof)
    re = (vol[:, None, None] / nl * f[None, None, :]).repeat(nl, 1)
    re = np.ascontiguousarray(re.reshape(ne, nde))
    return edof, ke, re, old_of_new


def tet_p1_elements(n, physics="laplace", jitter=0.2, seed=None, bc="none",
                    permute=False, E=1.0, nu=0.3):
    """Element data of :func:`workloads.meshes.tet_p1` with the same
    arguments (same geometry, numbering and removed DOFs).  Load: f = 1
    (Laplacian) or f = (0, 0, -1) (elasticity)."""
    shape = (n, n, n)
    X, idx = structured_grid(shape, jitter, seed)
    keep = _keep_mask(idx, shape, bc)
    if physics == "laplace":
        kern, dof, force = _laplace_kernel, 1, (1.0,)
    else:
        kern, dof, force = _elastic_kernel(*lame(E, nu)), 3, (0.0, 0.0, -1.0)
    edof, ke, re, old = _p1_elements(shape, X, _kuhn_tets(), kern, dof, keep,
                                     permute, seed, force)
    meta = dict(kind=f"tet_p1_{physics}", n=n, bc=bc, dof=dof,
                elems_per_cell=6)
    return Elements(len(old) * dof, edof, ke, re, meta)


def poisson_2d_p1_elements(n, jitter=0.2, seed=None, bc="all",
                           permute=False):
    """Element data of :func:`workloads.meshes.poisson_2d_p1` (f = 1)."""
    shape = (n, n)
    X, idx = structured_grid(shape, jitter, seed)
    keep = _keep_mask(idx, shape, bc)
    edof, ke, re, old = _p1_elements(shape, X, TRI_P1, _laplace_kernel, 1,
                                     keep, permute, seed, (1.0,))
    meta = dict(kind="poisson2d_p1", n=n, bc=bc, dof=1, elems_per_cell=2)
    return Elements(len(old), edof, ke, re, meta)


def line_p1_elements(n_el):
    """P1 line elements on [0, 1] with both ends clamped, unit source: the
    element data of :func:`workloads.meshes.laplace_1d_p1`."""
    h = 1.0 / n_el
    e = np.arange(n_el)
    edof = np.stack([e - 1, e], axis=1).astype(np.int32)   # node k -> row k-1
    edof[edof > n_el - 2] = -1
    ke = np.tile(np.array([[1.0, -1.0], [-1.0, 1.0]]) / h, (n_el, 1, 1))
    re = np.full((n_el, 2), h / 2.0)
    return Elements(n_el - 1, edof, ke, re, dict(kind="line_p1", h=h, dof=1))


def config1_elements(n=64, jitter=0.2):
    """Element data of the 3-D elasticity workload (Kuhn P1 tets, x = 0
    face clamped, random node numbering)."""
    return tet_p1_elements(n, "elastic", jitter=jitter, seed=(1, 0), bc="x0",
                           permute=True)
