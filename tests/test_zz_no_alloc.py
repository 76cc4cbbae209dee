"""periodic_sum_eval_noalloc (the allocation-free eval, for callers that cannot
allocate device memory) against periodic_sum_eval through the C ABI: two calls
in a row, the second with fewer particles, give bitwise the results of the
ordinary eval (same kernels and work split; only the partial sums live in the
library's static device scratch); a request whose partial sums exceed that
scratch is refused with PS_E_UNSUPPORTED."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_common import dev, err, load_ps
from oracle.method import Plan as OPlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def _call(ps, name, plan, x, q, phi, field):
    L = ps._lib.lib()
    vp = ctypes.c_void_p
    return getattr(L, name)(plan.handle, x.shape[1], *(vp(t.data_ptr()) for t in (x[0], x[1], x[2], q, phi)),
                            *(vp(t.data_ptr()) for t in (field[0], field[1], field[2])),
                            vp(torch.cuda.current_stream().cuda_stream))


def _eval(ps, plan, x, q, noalloc):
    n = x.shape[1]
    phi = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    field = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda:0")
    if noalloc:
        ps._lib.check(_call(ps, "periodic_sum_eval_noalloc", plan, x, q, phi, field))
    else:
        L = ps._lib.lib()
        vp = ctypes.c_void_p
        ps._lib.check(L.periodic_sum_eval(plan.handle, n, *(vp(t.data_ptr()) for t in (x[0], x[1], x[2], q)), 0,
                                          None, None, None, vp(phi.data_ptr()),
                                          *(vp(t.data_ptr()) for t in (field[0], field[1], field[2])),
                                          vp(torch.cuda.current_stream().cuda_stream)))
    plan.status()
    return phi, field


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_eval_matches_eval(ps, prec):
    box = (1.0, 1.2, 0.9)
    pl = ps.Plan(box, 10, lam=1.6, precision=prec, n_max=3000)
    ref_pl = ps.Plan(box, 10, lam=1.6, precision=prec, n_max=3000)
    for n, seed in ((3000, 91), (1100, 92)):          # the second call with a smaller input
        x, q = W.uniform_box(n, box, charges="gauss", seed=seed)
        X, Q = dev(x.T), dev(q)
        phi_a, field_a = _eval(ps, pl, X, Q, noalloc=True)
        phi_b, field_b = _eval(ps, ref_pl, X, Q, noalloc=False)
        assert torch.equal(phi_a, phi_b) and torch.equal(field_a, field_b), n
        ref = OPlan(box, 10, lam=1.6).solve(x, q)
        tol = 1e-12 if prec == "fp64" else 1e-6
        assert err(phi_a.cpu().numpy(), ref[0]) <= tol and err(field_a.cpu().numpy().T, ref[1]) <= tol


def test_noalloc_eval_refuses_partials_beyond_the_scratch(ps):
    """64 source splits of 40,000 targets need 10.24 Mi doubles of partial sums,
    more than the scratch's 8 Mi: refused before any kernel runs, and the plan
    still evaluates after."""
    box = (1.0, 1.0, 1.0)
    n = 40000
    x, q = W.uniform_box(n, box, charges="gauss", seed=93)
    X, Q = dev(x.T), dev(q)
    pl = ps.Plan(box, 4, R_b=1.5, precision="fp32", n_max=n, n_split=64)
    phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    field = torch.empty(3, n, dtype=torch.float64, device="cuda:0")
    st = _call(ps, "periodic_sum_eval_noalloc", pl, X, Q, phi, field)
    assert st == ps._lib.PS_E_UNSUPPORTED
    assert b"static scratch" in ps._lib.lib().periodic_sum_last_error()
    p2, _ = pl.eval(X, Q)
    pl.status()
    assert np.isfinite(p2.cpu().numpy()).all()
