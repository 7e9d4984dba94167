"""The five benchmark workloads as concrete seeded inputs.

* config 0: 2-D Poisson, P1 triangles, 64 x 64 nodes, interior jitter 0.2h,
  Dirichlet rows removed (3,844 rows).
* config 1: 3-D linear elasticity, P1 Kuhn tetrahedra, 64^3 nodes, jitter
  0.2h, E = 1, nu = 0.3, random node numbering, x = 0 face clamped by
  removing its DOFs (774,144 rows).
* config 2: the 15-matrix sweep below, each in natural and randomly
  permuted node order, full Neumann matrices (SpMV only).
* configs 3 and 4 reuse these generators (precision: the config-1 matrix;
  serving: P1 tet Laplacian / elasticity of drawn sizes).
"""
from __future__ import annotations

import numpy as np

from .meshes import poisson_2d_p1, tet_p1, tet_p2, hex_q1, graded_2d_p1
from .seeds import rng


def config0_poisson2d(jitter=0.2):
    return poisson_2d_p1(64, jitter=jitter, seed=(0, 0), bc="all")


def config1_elasticity3d(n=64, jitter=0.2):
    return tet_p1(n, "elastic", jitter=jitter, seed=(1, 0), bc="x0",
                  permute=True)


# name, builder, positional size, physics
SWEEP = [
    ("S1_p1tet_lap_22", tet_p1, 22, "laplace"),
    ("S2_p1tet_lap_59", tet_p1, 59, "laplace"),
    ("S3_p1tet_lap_126", tet_p1, 126, "laplace"),
    ("S4_p1tet_ela_15", tet_p1, 15, "elastic"),
    ("S5_p1tet_ela_41", tet_p1, 41, "elastic"),
    ("S6_p1tet_ela_87", tet_p1, 87, "elastic"),
    ("S7_p2tet_lap_11", tet_p2, 11, "laplace"),
    ("S8_p2tet_lap_50", tet_p2, 50, "laplace"),
    ("S9_p2tet_ela_20", tet_p2, 20, "elastic"),
    ("S10_q1hex_lap_22", hex_q1, 22, "laplace"),
    ("S11_q1hex_lap_126", hex_q1, 126, "laplace"),
    ("S12_q1hex_ela_87", hex_q1, 87, "elastic"),
    ("S13_graded2d_100", graded_2d_p1, 100, None),
    ("S14_graded2d_447", graded_2d_p1, 447, None),
    ("S15_graded2d_1414", graded_2d_p1, 1414, None),
]


def sweep_matrix(i, permuted=False):
    """Matrix ``i`` (0-based) of the sweep; seeds are (2, 2*i + permuted)."""
    name, fn, size, physics = SWEEP[i]
    seed = (2, 2 * i + int(bool(permuted)))
    if physics is None:
        A = fn(size, seed=seed, permute=permuted)
    else:
        A = fn(size, physics, jitter=0.2, seed=seed, bc="none",
               permute=permuted)
    A.meta["name"] = name + ("_perm" if permuted else "_nat")
    return A


def random_vector(n, cfg, purpose, idx=0, k=None):
    """Entries drawn from U(-1, 1); shape (n,) or (n, k)."""
    g = rng(cfg, purpose, idx)
    shape = (n,) if k is None else (n, k)
    return g.uniform(-1.0, 1.0, size=shape)
