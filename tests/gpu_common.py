"""Helpers shared by the GPU parity tests (imported by tests/test_gpu_*.py).

Bars: FP64 path <= 1e-12, FP32 path (FP32 pair arithmetic, FP64 accumulation)
<= 1e-6, for the potential and for the field.  Every parity check applies the
bar twice: to the relative L2 error over the compared particles and to the
worst element, max |got - ref| / max |ref|, so that a defect confined to a few
particles (a source image on the near-ball sphere, a particle on a face, the
closest pair, K(0) = 0) cannot hide inside a norm.
"""
import os

import numpy as np
import pytest

TOL = {"fp64": 1e-12, "fp32": 1e-6}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    """Relative L2 distance ||a - b|| / ||b|| (the paper's eps_2, eq. (st2))."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst(a, b):
    """Worst element relative to the largest reference value."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def err(a, b):
    """The error a parity bar applies to: the larger of rel and worst."""
    return max(rel(a, b), worst(a, b))


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("reference %s not generated" % name)
    return np.load(path)


def run(ps, box, p, x, q, prec, R_b=None, lam=None, targets=None, **kw):
    pl = ps.Plan(box, p, R_b=R_b, lam=lam, precision=prec, n_max=len(q),
                 m_max=0 if targets is None else len(targets), **kw)
    phi, field = pl.eval(dev(x.T), dev(q), targets=None if targets is None else dev(targets.T))
    pl.status()
    return pl, phi.cpu().numpy(), field.cpu().numpy().T


def load_ps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_4374_amd as m
    m.lib()
    return m
