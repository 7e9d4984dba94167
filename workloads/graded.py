"""Graded 2-D P1 triangle meshes with a skewed row-length distribution.

Base: the n x n node unit square, every cell split along its SW-NE diagonal
(interior nodes have 6 neighbours, rows of 7).  A seeded set of hub nodes,
at least 4 grid steps apart and 2 away from the boundary, is refined: hub v
gets a fan factor m (geometric law, capped so its row stays within
``max_row`` entries); every edge of v's 1-ring is cut into m pieces, each
triangle at v is re-fanned from v through the new points, and the triangle
across that ring edge is re-fanned from its opposite vertex, so the mesh
stays conforming.  Hub rows have 1 + 6m entries, the new edge points 5, the
opposite vertices 7 + (m - 1) per refined edge they face.

The stiffness matrix is the P1 Laplacian (Neumann), assembled element by
element (COO, duplicates summed in a fixed order).  Natural numbering keeps
the grid order with each hub's new points right after the hub; permuted
numbering draws a random node permutation.
"""
from __future__ import annotations

import numpy as np

from .seeds import rng as _rng, JITTER, PERM, SIZES


def _base_triangles(n):
    """Triangles of the n x n grid, lower (SW, SE, NE) then upper (SW, NE,
    NW) per cell; cell (i, j) has index i + (n - 1) j."""
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    i, j = i.ravel(), j.ravel()
    sw = i + n * j
    se, ne, nw = sw + 1, sw + 1 + n, sw + n
    lower = np.stack([sw, se, ne], 1)
    upper = np.stack([sw, ne, nw], 1)
    return np.concatenate([lower, upper]).astype(np.int64)


def _edge_partner(T, nnodes):
    """For every (triangle, local edge k) -- edge opposite local vertex k --
    the other triangle sharing that edge, or -1."""
    nt = len(T)
    a = np.stack([T[:, 1], T[:, 2], T[:, 0]], 1)
    b = np.stack([T[:, 2], T[:, 0], T[:, 1]], 1)
    key = (np.minimum(a, b) * nnodes + np.maximum(a, b)).ravel()
    order = np.argsort(key, kind="stable")
    ks = key[order]
    partner = np.full(3 * nt, -1, dtype=np.int64)
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    partner[order[same]] = order[same + 1] // 3
    partner[order[same + 1]] = order[same] // 3
    return partner.reshape(nt, 3)


def _pick_hubs(n, seed, density, mmax, p_geom):
    g = _rng(seed[0], SIZES, 1000 + seed[1])
    cand = [(i, j) for j in range(2, n - 2) for i in range(2, n - 2)]
    order = g.permutation(len(cand))
    want = max(1, int(density * n * n))
    blocked = np.zeros((n, n), dtype=bool)
    hubs = []
    for c in order:
        i, j = cand[c]
        if blocked[i, j]:
            continue
        hubs.append(i + n * j)
        blocked[max(0, i - 3):i + 4, max(0, j - 3):j + 4] = True
        if len(hubs) >= want:
            break
    m = np.minimum(mmax, 1 + g.geometric(p_geom, len(hubs)))
    return np.array(hubs, dtype=np.int64), m.astype(np.int64)


def _p1_laplace(X, T):
    """Element matrices of the P1 Laplacian: area * G G^T."""
    P = X[T]                                   # (nt, 3, 2)
    e1 = P[:, 1] - P[:, 0]
    e2 = P[:, 2] - P[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    if not np.all(det > 0):
        raise ValueError("inverted or degenerate triangle in graded mesh")
    # gradients of the barycentric functions: rows of inv([e1 e2])^T
    inv = np.empty((len(T), 2, 2))
    inv[:, 0, 0] = e2[:, 1] / det
    inv[:, 0, 1] = -e2[:, 0] / det
    inv[:, 1, 0] = -e1[:, 1] / det
    inv[:, 1, 1] = e1[:, 0] / det
    G = np.empty((len(T), 3, 2))
    G[:, 1] = inv[:, 0]
    G[:, 2] = inv[:, 1]
    G[:, 0] = -G[:, 1] - G[:, 2]
    area = 0.5 * det
    return area[:, None, None] * np.matmul(G, G.transpose(0, 2, 1))


def build_graded(n, hubs=None, seed=None, jitter=0.2, max_row=200,
                 density=1.0 / 64, p_geom=0.3, permute=False):
    from .meshes import CSR, structured_grid
    if seed is None:
        seed = (2, 0)
    X, idx = structured_grid((n, n), jitter, seed)
    T = _base_triangles(n)
    N0 = n * n
    mmax = max(1, (max_row - 1) // 6)
    if hubs is None:
        hubs, mfan = _pick_hubs(n, seed, density, mmax, p_geom)
    else:
        hubs = np.asarray(hubs, dtype=np.int64)
        mfan = np.full(len(hubs), mmax, dtype=np.int64)
    partner = _edge_partner(T, N0)
    # incident triangles of every hub
    hub_of = np.full(N0, -1, dtype=np.int64)
    hub_of[hubs] = np.arange(len(hubs))
    inc = [[] for _ in range(len(hubs))]
    for k in range(3):
        h = hub_of[T[:, k]]
        for t in np.nonzero(h >= 0)[0]:
            inc[h[t]].append((t, k))
    drop = np.zeros(len(T), dtype=bool)
    newX = [X]
    new_tris = []
    owner = [np.arange(N0, dtype=np.int64)]    # numbering key: (owner, sub)
    sub = [np.zeros(N0, dtype=np.int64)]
    nxt = N0
    for h, (v, m) in enumerate(zip(hubs, mfan)):
        if m <= 1:
            continue
        cnt = 1
        for t, k in inc[h]:
            p, q = T[t, (k + 1) % 3], T[t, (k + 2) % 3]
            # points s_1 .. s_{m-1} on p -> q
            f = np.arange(1, m)[:, None] / m
            pts = (1 - f) * X[p] + f * X[q]
            ids = nxt + np.arange(m - 1)
            nxt += m - 1
            newX.append(pts)
            owner.append(np.full(m - 1, v, dtype=np.int64))
            sub.append(cnt + np.arange(m - 1))
            cnt += m - 1
            chain = np.concatenate([[p], ids, [q]])
            for a, b in zip(chain[:-1], chain[1:]):
                new_tris.append((v, a, b))      # same orientation as (v,p,q)
            drop[t] = True
            u = partner[t, k]
            if u >= 0:
                ku = int(np.nonzero((T[u] != p) & (T[u] != q))[0][0])
                w = T[u, ku]
                pu, qu = T[u, (ku + 1) % 3], T[u, (ku + 2) % 3]
                # (w, pu, qu) is positively oriented; pu -> qu is q -> p
                ch = chain if pu == p else chain[::-1]
                for a, b in zip(ch[:-1], ch[1:]):
                    new_tris.append((w, a, b))
                drop[u] = True
    X = np.concatenate(newX)
    T = np.concatenate([T[~drop], np.array(new_tris, dtype=np.int64)
                        .reshape(-1, 3)])
    N = len(X)
    owner = np.concatenate(owner)
    sub = np.concatenate(sub)
    if permute:
        g = _rng(seed[0], PERM, seed[1])
        old_of_new = g.permutation(N)
    else:
        old_of_new = np.lexsort((sub, owner))
    new_of_old = np.empty(N, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(N)
    Tn = new_of_old[T]
    Ke = _p1_laplace(X, T)
    rows = np.repeat(Tn, 3, axis=1).ravel()
    cols = np.tile(Tn, (1, 3)).ravel()
    key = rows * N + cols
    order = np.argsort(key, kind="stable")
    ks = key[order]
    vs = Ke.reshape(-1)[order]
    start = np.concatenate([[0], np.nonzero(ks[1:] != ks[:-1])[0] + 1])
    val = np.add.reduceat(vs, start)
    uk = ks[start]
    r = uk // N
    c = (uk % N).astype(np.int32)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    meta = dict(kind="graded2d_p1", n=n, hubs=len(hubs),
                fan=mfan, coords=X[old_of_new], triangles=Tn)
    return CSR(N, N, rowptr, c, val, meta)
