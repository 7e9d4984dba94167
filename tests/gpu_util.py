"""Helpers shared by the GPU tests (marshalling and tolerances only)."""
import sys

import numpy as np


def note(msg):
    """Name the case on stdout before a GPU step (flushed)."""
    print("[gpu-case] " + msg, file=sys.stdout, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def make(A, **opts):
    import paper_1501_00324_amd as fs
    return fs.csr_create(dev(A.rowptr), dev(A.col), dev(A.val), A.n_rows,
                         A.n_cols, **opts)


# Componentwise FP64 SpMV bar: |y_i - y_i^oracle| <= 1e-12 (|A| |x|)_i.
# Summation-order and FMA differences are bounded by ~m eps (|A||x|)_i
# (m <= a few hundred entries per row), about 1e-13.
SPMV_RTOL = 1e-12


def assert_spmv_close(y, y_ref, scale, what=""):
    err = np.abs(y - y_ref)
    bad = ~(err <= SPMV_RTOL * scale)
    # rows whose exact value is +-inf/nan must agree in kind
    both_nan = np.isnan(y) & np.isnan(y_ref)
    same_inf = np.isinf(y) & (y == y_ref)
    bad &= ~(both_nan | same_inf)
    assert not bad.any(), "%s: %d rows off, first %s" % (
        what, bad.sum(), np.nonzero(bad)[0][:5])
