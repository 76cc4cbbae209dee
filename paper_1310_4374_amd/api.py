"""Python front end of the C ABI (torch tensors in, torch tensors out).

Positions are passed structure-of-arrays: a (3, N) float64 tensor on the plan's
device (rows x, y, z); charges an (N,) float64 tensor.  Calls enqueue work on
torch's current stream of that device and return at once.
"""
import ctypes

import torch

from . import _lib
from ._lib import check, lib, ps_params, ps_plan_info, ps_select_row

_PREC = {"fp64": _lib.PS_FP64, "fp32": _lib.PS_FP32_ACC64, "fp32_acc64": _lib.PS_FP32_ACC64}
_MEAN = {"zero": _lib.PS_MEAN_ZERO, "none": _lib.PS_MEAN_NONE}
_PERIODIC = {"xyz": 7, "xy": 3, "x": 1}
_KERNEL = {"coulomb": 0, "screened": 1, "biharmonic": 2}


def _host_points(a):
    """(k, 3) float64 C-contiguous host array (kept alive by the caller)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a.cpu() if hasattr(a, "cpu") else a, dtype=np.float64))
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("points must be (k, 3)")
    return a


def _params(box, p, R_b=None, lam=None, precision="fp64", mean="zero", rcond=1e-13, n_max=1, m_max=0,
            tile_targets=0, n_split=0, centres=None, check_points=None, keep=None, periodic="xyz", kernel="coulomb",
            kappa=0.0, dim=3):
    """keep: a list that receives the host arrays the struct points to.
    periodic: "xyz" (three periodic axes), "xy" (a slab, z free) or "x" (a wire, y and z free).
    kernel: "coulomb" (1/r; -log r in the plane), "screened" (exp(-kappa r)/r; needs centres) or
    "biharmonic" (r; spherical basis, three periodic axes).
    dim: 3, or 2 for the method in the plane (box (d1, d2))."""
    prm = ps_params()
    for k in range(len(box) if int(dim) == 2 else 3):
        prm.box[k] = float(box[k])
    prm.p = int(p)
    prm.R_b = float(R_b) if R_b is not None else 0.0
    prm.lambda_ = float(lam) if lam is not None else 0.0
    prm.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    prm.mean = _MEAN[mean] if isinstance(mean, str) else int(mean)
    prm.rcond = float(rcond)
    prm.n_max = int(n_max)
    prm.m_max = int(m_max)
    prm.tile_targets = int(tile_targets)
    prm.n_split = int(n_split)
    prm.periodic = _PERIODIC[periodic] if isinstance(periodic, str) else int(periodic)
    prm.kernel = _KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
    prm.kappa = float(kappa)
    prm.dim = int(dim)
    dp = ctypes.POINTER(ctypes.c_double)
    if centres is not None:
        c = _host_points(centres)
        keep.append(c)
        prm.basis = _lib.PS_BASIS_RBF
        prm.n_centres = c.shape[0]
        prm.centres = c.ctypes.data_as(dp)
    if check_points is not None:
        y = _host_points(check_points)
        keep.append(y)
        prm.n_check = y.shape[0]
        prm.check_points = y.ctypes.data_as(dp)
    return prm


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _soa(x, device, dim=3):
    """(3, N) or (N, 3) float64 positions -> contiguous (3, N) on the device.
    dim 2 (the plane): (2, N) or (N, 2) -> contiguous (2, N); a (3, N) or (N, 3)
    array gives its first two coordinates."""
    rows = (2, 3) if dim == 2 else (3,)
    if x.dim() != 2 or not any(r in x.shape for r in rows):
        r = "2|3" if dim == 2 else "3"
        raise ValueError("positions must be (%s, N) or (N, %s)" % (r, r))
    if x.shape[0] not in rows or (x.shape[1] in rows and not x.is_contiguous()):
        x = x.t()
    if x.dtype != torch.float64 or x.device != device:
        raise ValueError("positions must be float64 on %s" % device)
    return x[:dim].contiguous()


def _xyz(x):
    """Pointers to the coordinate rows; None for z in the plane."""
    return [_ptr(x[0]), _ptr(x[1]), _ptr(x[2]) if x.shape[0] > 2 else None]


def _vec(t, n, device, name):
    """t as a contiguous float64 device tensor of n elements, or ValueError (the
    library reads n doubles through the pointer; a wrong dtype, device or size
    must not reach it)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64 or t.device != device:
        raise ValueError("%s must be float64 on %s (got %s on %s)" % (name, device, t.dtype, t.device))
    if t.numel() != n:
        raise ValueError("%s must have %d elements (got %d)" % (name, n, t.numel()))
    return t.reshape(n).contiguous()


def _field_out(t, n, device, name, rows=3):
    """A (rows, n) float64 device output whose rows are contiguous."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != device:
        raise ValueError("%s must be a float64 tensor on %s" % (name, device))
    if tuple(t.shape) != (rows, n) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous (%d, %d) tensor" % (name, rows, n))
    return t


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """One periodic box: algorithm "set" at construction, "get" on each eval."""

    def __init__(self, box, p, R_b=None, lam=None, precision="fp64", mean="zero", rcond=1e-13, n_max=1, m_max=0,
                 tile_targets=0, n_split=0, centres=None, check_points=None, periodic="xyz", kernel="coulomb",
                 kappa=0.0, dim=3, device=0):
        """centres: (M, 3) RBF centres outside the box (eq. (5)); None for the
        spherical-harmonic basis.  check_points: (L, 3) points on the
        circumsphere; None for the Gauss spherical grid.  periodic: "xyz", or
        "xy" for a slab (periodic in x and y, vacuum above and below), or "x" for
        a wire (periodic in x, vacuum around it).
        kernel: "coulomb" (1/r), "screened" (exp(-kappa r)/r, any net charge,
        RBF centres required, no constant term) or "biharmonic" (r, neutral
        charges, P = p^2 + (p-2)^2).  dim=2: the method in the plane
        (box (d1, d2), kernel -log r, positions (2, N), field (2, N))."""
        self.device = torch.device("cuda", device)
        self.dim = int(dim) if int(dim) == 2 else 3
        keep = []
        self._prm = _params(box, p, R_b, lam, precision, mean, rcond, n_max, m_max, tile_targets, n_split,
                            centres, check_points, keep, periodic, kernel, kappa, dim)
        h = ctypes.c_void_p()
        check(lib().periodic_sum_plan(ctypes.byref(self._prm), int(device), ctypes.byref(h)))
        self._h = h
        self.n_max = int(n_max)

    def __del__(self):
        _destroy(self)

    @property
    def handle(self):
        return self._h

    def save(self, path):
        """Write the plan's set data and launch shape to a file (see load)."""
        _save(self, path)

    @classmethod
    def load(cls, path, device=0):
        """A plan rebuilt from a file written by save, without repeating the set phase."""
        obj = cls.__new__(cls)
        obj.device = torch.device("cuda", device)
        obj._h = _load(path, device)
        obj.n_max = None
        obj.dim = obj.info()["dim"]
        return obj

    def info(self):
        inf = ps_plan_info()
        check(lib().periodic_sum_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def tables(self):
        """Check points (L,3), partners (L,3), pseudo-inverse (P-1, n_rows), box means (P,) as CPU
        float64 tensors (n_rows = L, plus the decay rows of a slab)."""
        inf = self.info()
        L, P = inf["L"], inf["P"]
        yc = torch.empty(L, 3, dtype=torch.float64)
        yt = torch.empty(L, 3, dtype=torch.float64)
        pinv = torch.empty(P - 1, inf["n_rows"], dtype=torch.float64)
        bm = torch.empty(P, dtype=torch.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().periodic_sum_plan_tables(self._h, *(ctypes.cast(t.data_ptr(), dp) for t in (yc, yt, pinv, bm))))
        return yc, yt, pinv, bm

    def coefficients(self):
        P = self.info()["P"]
        C = torch.empty(P, dtype=torch.float64)
        check(lib().periodic_sum_last_coefficients(self._h, ctypes.cast(C.data_ptr(), ctypes.POINTER(ctypes.c_double))))
        return C

    def eval(self, x, q, targets=None, out=None):
        """phi (N,) and field -grad phi (3, N) at the particles, or at separate
        targets (3, M).  Returns device tensors; enqueued on the current stream."""
        x = _soa(x, self.device, self.dim)
        n = x.shape[1]
        q = _vec(q, n, self.device, "q")
        if targets is not None:
            t = _soa(targets, self.device, self.dim)
            m = t.shape[1]
            tp = _xyz(t)
        else:
            m = 0
            tp = [None, None, None]
        cnt = m if m else n
        if out is None:
            phi = torch.empty(cnt, dtype=torch.float64, device=self.device)
            field = torch.empty(self.dim, cnt, dtype=torch.float64, device=self.device)
        else:
            phi, field = out
            if phi.data_ptr() != _vec(phi, cnt, self.device, "phi").data_ptr():
                raise ValueError("phi must be contiguous")
            _field_out(field, cnt, self.device, "field", self.dim)
        check(lib().periodic_sum_eval(self._h, n, *_xyz(x), _ptr(q), m, *tp, _ptr(phi), *_xyz(field),
                                      _stream(self.device)))
        return phi, field

    def set_profiling(self, enable=True):
        check(lib().periodic_sum_set_profiling(self._h, int(bool(enable))))

    def stage_times(self):
        """Mean milliseconds per stage over the profiled evals since the previous
        read (or since set_profiling); synchronizes on the last of them."""
        arr = (ctypes.c_double * len(_lib.STAGES))()
        check(lib().periodic_sum_stage_times(self._h, arr, len(_lib.STAGES)))
        return dict(zip(_lib.STAGES, list(arr)))

    def autotune(self, x, q):
        """Pick targets per workgroup and the split scale by timing them on these inputs; returns ms per eval."""
        return _autotune(self, x, q, [0, _soa(x, self.device, self.dim).shape[1]])

    def near_counts(self):
        return _near_counts(self, 1)

    def status(self):
        """Synchronize and raise on a data error of the last eval."""
        check(lib().periodic_sum_status(self._h, _stream(self.device)))

    def energy(self, x, q, phi=None, field=None):
        x = _soa(x, self.device, self.dim)
        n = x.shape[1]
        q = _vec(q, n, self.device, "q")
        if phi is not None and phi.data_ptr() != _vec(phi, n, self.device, "phi").data_ptr():
            raise ValueError("phi must be contiguous")
        if field is not None:
            _field_out(field, n, self.device, "field", self.dim)
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        fp = _xyz(field) if field is not None else [None, None, None]
        check(lib().periodic_sum_energy(self._h, n, *_xyz(x), _ptr(q), _ptr(e), _ptr(phi), *fp,
                                        _stream(self.device)))
        return e

    def forward_epoch(self):
        """Counter of the forward passes enqueued on this plan (the last one is
        the pass whose state energy_vjp reuses); does not synchronize."""
        e = ctypes.c_int64()
        check(lib().periodic_sum_forward_epoch(self._h, ctypes.byref(e)))
        return e.value

    def energy_vjp(self, x, q, gE, exact=True, epoch=0):
        """Gradient of the last energy pass at these particles; epoch (from
        forward_epoch right after that pass, 0 = unchecked) makes the library
        refuse the call if another pass has run on the plan since."""
        x = _soa(x, self.device, self.dim)
        n = x.shape[1]
        q = _vec(q, n, self.device, "q")
        dx = torch.empty(self.dim, n, dtype=torch.float64, device=self.device)
        dq = torch.empty(n, dtype=torch.float64, device=self.device)
        gE = torch.as_tensor(gE).to(device=self.device, dtype=torch.float64).reshape(1).contiguous()
        check(lib().periodic_sum_energy_vjp(self._h, n, *_xyz(x), _ptr(q), _ptr(gE), *_xyz(dx), _ptr(dq),
                                            int(bool(exact)), int(epoch), _stream(self.device)))
        return dx, dq


def _autotune(obj, x, q, offsets):
    x = _soa(x, obj.device, obj.dim)
    n = x.shape[1]
    q = _vec(q, n, obj.device, "q")
    _check_offsets(offsets, n)
    off = (ctypes.c_int64 * len(offsets))(*[int(v) for v in offsets])
    phi = torch.empty(n, dtype=torch.float64, device=obj.device)
    field = torch.empty(obj.dim, n, dtype=torch.float64, device=obj.device)
    best = ctypes.c_double()
    check(lib().periodic_sum_autotune(obj._h, off, *_xyz(x), _ptr(q), _ptr(phi), *_xyz(field), ctypes.byref(best),
                                      _stream(obj.device)))
    return best.value


def _check_offsets(offsets, n):
    if len(offsets) < 2 or int(offsets[0]) != 0 or int(offsets[-1]) != n:
        raise ValueError("offsets must start at 0 and end at the particle count %d" % n)
    if any(int(b) <= int(a) for a, b in zip(offsets[:-1], offsets[1:])):
        raise ValueError("offsets must be strictly increasing")


def _destroy(obj):
    """Release the plan.  At interpreter exit the module globals may already be
    gone; the process is ending then and the plan's memory goes with it."""
    h = getattr(obj, "_h", None)
    if h is None or not h.value:
        return
    try:
        lib().periodic_sum_destroy(h)
    except (AttributeError, TypeError):
        pass
    obj._h = None


def _save(obj, path):
    check(lib().periodic_sum_plan_save(obj._h, str(path).encode()))


def _load(path, device):
    h = ctypes.c_void_p()
    check(lib().periodic_sum_plan_load(str(path).encode(), int(device), ctypes.byref(h)))
    return h


def _near_counts(obj, nsys):
    out = (ctypes.c_int64 * nsys)()
    check(lib().periodic_sum_near_counts(obj._h, out, nsys))
    return list(out)


class BatchedPlan:
    """Many independent boxes solved by one graph launch per eval."""

    def __init__(self, systems, p, lam=None, R_b=None, precision="fp32", mean="zero", rcond=1e-13, tile_targets=0,
                 n_split=0, kernel="coulomb", kappa=0.0, dim=3, device=0):
        """systems: list of dicts with 'box' and 'n_max' (and optional 'R_b'/'lam',
        'centres', 'check_points', 'periodic').  kernel, kappa and dim hold for every system."""
        self.device = torch.device("cuda", device)
        self.dim = int(dim) if int(dim) == 2 else 3
        arr = (ps_params * len(systems))()
        keep = []
        for k, s in enumerate(systems):
            arr[k] = _params(s["box"], s.get("p", p), s.get("R_b", R_b), s.get("lam", lam), precision, mean, rcond,
                             s["n_max"], 0, tile_targets, n_split, s.get("centres"), s.get("check_points"), keep,
                             s.get("periodic", "xyz"), kernel, kappa, dim)
        h = ctypes.c_void_p()
        check(lib().periodic_sum_plan_batched(len(systems), arr, int(device), ctypes.byref(h)))
        self._h = h
        self._arr = arr
        self.nsys = len(systems)

    def __del__(self):
        _destroy(self)

    def save(self, path):
        """Write the plan's set data and launch shape to a file (see load)."""
        _save(self, path)

    @classmethod
    def load(cls, path, device=0):
        """A batched plan rebuilt from a file written by save, without repeating the set phase."""
        obj = cls.__new__(cls)
        obj.device = torch.device("cuda", device)
        obj._h = _load(path, device)
        obj.nsys = obj.info()["nsys"]
        obj.dim = obj.info()["dim"]
        return obj

    def eval(self, x, q, offsets, out=None):
        """x: (3, sum N) packed positions, q: (sum N,), offsets: host sequence of nsys+1 ints.
        The captured graph is replayed while the particle counts and the buffers
        stay the same: in a loop, pass the same out=(phi, field) each time."""
        x = _soa(x, self.device, self.dim)
        n = x.shape[1]
        q = _vec(q, n, self.device, "q")
        if len(offsets) != self.nsys + 1:
            raise ValueError("offsets must have nsys + 1 = %d entries" % (self.nsys + 1))
        _check_offsets(offsets, n)
        off = (ctypes.c_int64 * (self.nsys + 1))(*[int(v) for v in offsets])
        if out is None:
            phi = torch.empty(n, dtype=torch.float64, device=self.device)
            field = torch.empty(self.dim, n, dtype=torch.float64, device=self.device)
        else:
            phi, field = out
            if phi.data_ptr() != _vec(phi, n, self.device, "phi").data_ptr():
                raise ValueError("phi must be contiguous")
            _field_out(field, n, self.device, "field", self.dim)
        check(lib().periodic_sum_eval_batched(self._h, off, *_xyz(x), _ptr(q), _ptr(phi), *_xyz(field),
                                              _stream(self.device)))
        return phi, field

    def autotune(self, x, q, offsets):
        """Pick targets per workgroup and the split scale by timing them on these inputs; returns ms per batch."""
        return _autotune(self, x, q, offsets)

    def near_counts(self):
        return _near_counts(self, self.nsys)

    def info(self):
        inf = ps_plan_info()
        check(lib().periodic_sum_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def status(self):
        check(lib().periodic_sum_status(self._h, _stream(self.device)))


def select_parameters(box, x, q, tol, lambdas=(1.3, 1.4, 1.5, 1.6, 1.7), precision="fp32", p_ref=0, rcond=1e-13,
                      tile_targets=0, device=0):
    """Smallest p meeting a relative L2 tolerance on phi for each candidate
    lambda, and the fastest candidate, measured on these charges (eq. (o1)).
    Returns (best, rows): best is the chosen row (a dict) or None, rows one dict
    per lambda with keys lambda, p, n_solves, B_P, err, err_prec, ms, set_s."""
    dev = torch.device("cuda", device)
    x = _soa(x, dev)
    n = x.shape[1]
    q = _vec(q, n, dev, "q")
    lam = [float(v) for v in lambdas]
    prm = _params(box, 8, lam=lam[0], precision=precision, rcond=rcond, n_max=n, tile_targets=tile_targets)
    arr = (ctypes.c_double * len(lam))(*lam)
    rows = (ps_select_row * len(lam))()
    best = ctypes.c_int32(-1)
    check(lib().periodic_sum_select(ctypes.byref(prm), device, n, _ptr(x[0]), _ptr(x[1]), _ptr(x[2]), _ptr(q),
                                    float(tol), arr, len(lam), int(p_ref), rows, ctypes.byref(best), _stream(dev)))
    out = [{"lambda": r.lambda_, "p": r.p, "n_solves": r.n_solves, "B_P": r.B_P, "err": r.err,
            "err_prec": r.err_prec, "ms": r.ms, "set_s": r.set_s} for r in rows]
    return (out[best.value] if best.value >= 0 else None), out


class PeriodicEnergy(torch.autograd.Function):
    """E = (1/2) sum q_i phi(x_i) with a hand-written adjoint (exact derivative of
    the discrete method, or the physical -q E / phi approximation)."""

    @staticmethod
    def forward(ctx, x, q, plan, exact=True):
        # the adjoint checks that it follows a pass at the same device arrays, so
        # the (3, N) contiguous form the library reads is kept for backward
        xs = _soa(x.detach(), plan.device, getattr(plan, "dim", 3))
        qs = _vec(q.detach(), xs.shape[1], plan.device, "q")
        e = plan.energy(xs, qs)
        ctx.save_for_backward(xs, qs)
        rows = (2, 3) if getattr(plan, "dim", 3) == 2 else (3,)
        ctx.x_rows = x.shape[0] in rows and not (x.shape[1] in rows and not x.is_contiguous())  # as _soa reads it
        ctx.x_shape = tuple(x.shape)
        ctx.plan = plan
        ctx.exact = exact
        ctx.epoch = plan.forward_epoch()
        return e[0]

    @staticmethod
    def backward(ctx, gE):
        x, q = ctx.saved_tensors
        plan = ctx.plan
        epoch = ctx.epoch
        if plan.forward_epoch() != epoch:
            # another pass ran on the plan since this forward (the plan keeps only
            # the last one): run this forward again so that the adjoint reuses
            # the state of these inputs
            plan.energy(x, q)
            epoch = plan.forward_epoch()
        dx, dq = plan.energy_vjp(x, q, gE, exact=ctx.exact, epoch=epoch)
        if dx.shape[0] == 2 and 3 in ctx.x_shape and 2 not in ctx.x_shape:   # plane positions given with a z row
            dx = torch.cat([dx, torch.zeros_like(dx[:1])])
        if not ctx.x_rows:
            dx = dx.t()
        return dx, dq, None, None
