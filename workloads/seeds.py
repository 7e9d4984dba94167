"""Seed convention shared by every generator.

``rng(cfg, purpose, idx)`` returns an independent PCG64 stream for workload
``cfg`` (0..4 for the five benchmark configurations, 90+ for test-only meshes),
draw ``purpose`` and matrix index ``idx``.
"""
import numpy as np

JITTER = 0     # interior node displacement
PERM = 1       # random node numbering
XVEC = 2       # SpMV input vectors
BVEC = 3       # right-hand sides
SIZES = 4      # request sizes (serving workload)
ARRIVALS = 5   # request arrival times (serving workload)


def rng(cfg: int, purpose: int, idx: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(cfg), int(purpose), int(idx)])
