"""The C-ABI library loads and exports every function include/periodic_sum.h
declares; argument errors are reported without touching a device."""
import ctypes
import os
import re

import pytest

from paper_1310_4374_amd import _lib

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "periodic_sum.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(periodic_sum_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("periodic_sum_plan", "periodic_sum_eval", "periodic_sum_energy", "periodic_sum_energy_vjp",
                     "periodic_sum_plan_batched", "periodic_sum_eval_batched", "periodic_sum_status",
                     "periodic_sum_destroy", "periodic_sum_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(_declared()) == sorted(_lib.EXPORTS)


def test_struct_layout_matches_header():
    """The ctypes mirror of ps_params has the C layout (no torch types cross)."""
    assert ctypes.sizeof(_lib.ps_params) == 3 * 8 + 4 + 4 + 8 + 8 + 4 + 4 + 8 + 8 + 8 + 4 + 4 + 4 + 4 + 8 + 4 + 4 + 8 \
        + 4 + 4 + 8 + 4 + 4
    assert _lib.ps_params.n_max.offset == 64
    assert _lib.ps_params.periodic.offset == 120
    assert _lib.ps_params.kernel.offset == 124 and _lib.ps_params.kappa.offset == 128
    assert _lib.ps_params.dim.offset == 136
    assert ctypes.sizeof(_lib.ps_plan_info) == 128 and _lib.ps_plan_info.kappa.offset == 96
    assert _lib.ps_plan_info.dim.offset == 108 and _lib.ps_plan_info.tune_second_ms.offset == 120


def _params(**kw):
    prm = _lib.ps_params()
    for k in range(3):
        prm.box[k] = 1.0
    prm.p = 8
    prm.R_b = 1.5
    prm.n_max = 100
    for k, v in kw.items():
        setattr(prm, k, v)
    return prm


@pytest.mark.parametrize("kw", [dict(p=1), dict(p=41), dict(n_max=0), dict(precision=7), dict(mean=3),
                                dict(tile_targets=100), dict(n_split=-1), dict(m_max=-5), dict(basis=2),
                                dict(basis=1, n_centres=0), dict(basis=1, n_centres=10), dict(n_check=5)])
def test_invalid_parameters_rejected_on_host(kw):
    L = _lib.lib()
    h = ctypes.c_void_p()
    st = L.periodic_sum_plan(ctypes.byref(_params(**kw)), 0, ctypes.byref(h))
    assert st == _lib.PS_E_INVALID
    assert not h.value
    assert L.periodic_sum_last_error()


def test_null_arguments_rejected():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.periodic_sum_plan(None, 0, ctypes.byref(h)) == _lib.PS_E_INVALID
    assert L.periodic_sum_plan(ctypes.byref(_params()), 0, None) == _lib.PS_E_INVALID
    assert L.periodic_sum_eval(None, 10, *([None] * 4), 0, *([None] * 3), *([None] * 4), None) == _lib.PS_E_INVALID
    assert L.periodic_sum_status(None, None) == _lib.PS_E_INVALID
    assert L.periodic_sum_eval_noalloc(None, 10, *([None] * 4), *([None] * 4), None) == _lib.PS_E_INVALID
    e = ctypes.c_int64(5)
    assert L.periodic_sum_forward_epoch(None, ctypes.byref(e)) == _lib.PS_E_INVALID
    assert L.periodic_sum_energy_vjp(None, 10, *([None] * 4), None, *([None] * 4), 1, 0, None) == _lib.PS_E_INVALID
    L.periodic_sum_destroy(None)


def test_screened_kernel_parameters_checked_on_host():
    """Unknown kernel, the screened kernel without the RBF basis or on a slab,
    and kappa outside (0, 64/R0] are refused before any device work."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    cen = (ctypes.c_double * 3)(2.0, 0.0, 0.0)
    dp = ctypes.cast(cen, ctypes.POINTER(ctypes.c_double))
    cases = [(dict(kernel=3), _lib.PS_E_INVALID), (dict(kernel=-1), _lib.PS_E_INVALID),
             (dict(kernel=1, kappa=1.0), _lib.PS_E_UNSUPPORTED),
             (dict(kernel=1, kappa=1.0, basis=1, n_centres=1, centres=dp, periodic=3), _lib.PS_E_UNSUPPORTED),
             (dict(kernel=1, kappa=0.0, basis=1, n_centres=1, centres=dp), _lib.PS_E_INVALID),
             (dict(kernel=1, kappa=-1.0, basis=1, n_centres=1, centres=dp), _lib.PS_E_INVALID),
             (dict(kernel=1, kappa=1e3, basis=1, n_centres=1, centres=dp), _lib.PS_E_INVALID)]
    for kw, status in cases:
        assert L.periodic_sum_plan(ctypes.byref(_params(**kw)), 0, ctypes.byref(h)) == status, kw
        assert h.value is None


def test_biharmonic_kernel_parameters_checked_on_host():
    """The biharmonic kernel with the RBF basis, fewer than three periodic axes,
    in the plane or with p outside [3, 30] is refused before any device work."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    cen = (ctypes.c_double * 3)(2.0, 0.0, 0.0)
    dp = ctypes.cast(cen, ctypes.POINTER(ctypes.c_double))
    cases = [dict(kernel=2, basis=1, n_centres=1, centres=dp), dict(kernel=2, periodic=3), dict(kernel=2, periodic=1),
             dict(kernel=2, dim=2), dict(kernel=2, p=2), dict(kernel=2, p=31)]
    for kw in cases:
        assert L.periodic_sum_plan(ctypes.byref(_params(**kw)), 0, ctypes.byref(h)) == _lib.PS_E_UNSUPPORTED, kw
        assert h.value is None


def test_periodic_axes_checked_on_host():
    """Masks other than 0, 7, 3 and 1, the RBF basis with fewer than three axes
    and the screened kernel on a wire are refused before any device work."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    cen = (ctypes.c_double * 3)(2.0, 0.0, 0.0)
    dp = ctypes.cast(cen, ctypes.POINTER(ctypes.c_double))
    cases = [dict(periodic=p) for p in (2, 4, 5, 6, 8, -1)]
    cases += [dict(periodic=1, basis=1, n_centres=1, centres=dp), dict(periodic=3, basis=1, n_centres=1, centres=dp),
              dict(periodic=1, kernel=1, kappa=1.0, basis=1, n_centres=1, centres=dp)]
    for kw in cases:
        assert L.periodic_sum_plan(ctypes.byref(_params(**kw)), 0, ctypes.byref(h)) == _lib.PS_E_UNSUPPORTED, kw
        assert h.value is None


def test_plane_parameters_checked_on_host():
    """dim other than 0, 2 or 3, and in the plane: the RBF basis, the screened
    kernel, caller check points, one periodic axis, p above 128, a bad box edge
    are refused before any device work (box[2] is not read in the plane)."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    cen = (ctypes.c_double * 3)(2.0, 0.0, 0.0)
    dp = ctypes.cast(cen, ctypes.POINTER(ctypes.c_double))
    cases = [(dict(dim=1), _lib.PS_E_INVALID), (dict(dim=4), _lib.PS_E_INVALID),
             (dict(dim=2, basis=1, n_centres=1, centres=dp), _lib.PS_E_UNSUPPORTED),
             (dict(dim=2, kernel=1, kappa=1.0), _lib.PS_E_UNSUPPORTED),
             (dict(dim=2, n_check=1, check_points=dp), _lib.PS_E_UNSUPPORTED),
             (dict(dim=2, periodic=1), _lib.PS_E_UNSUPPORTED),
             (dict(dim=2, p=129), _lib.PS_E_INVALID), (dict(dim=3, p=41), _lib.PS_E_INVALID)]
    for kw, status in cases:
        assert L.periodic_sum_plan(ctypes.byref(_params(**kw)), 0, ctypes.byref(h)) == status, kw
        assert h.value is None
    prm = _params(dim=2)
    prm.box[1] = -1.0
    assert L.periodic_sum_plan(ctypes.byref(prm), 0, ctypes.byref(h)) == _lib.PS_E_INVALID


@pytest.mark.parametrize("kw", [dict(R_b=0.5), dict(R_b=0.0, lambda_=0.9)])
def test_near_radius_must_exceed_circumradius(kw):
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.periodic_sum_plan(ctypes.byref(_params(**kw)), 0, ctypes.byref(h)) == _lib.PS_E_INVALID


def test_plan_file_errors_reported_before_any_device_work(tmp_path):
    """Loading a missing, foreign, truncated or corrupted plan file fails with
    PS_E_IO on the host; NULL arguments with PS_E_INVALID."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.periodic_sum_plan_load(None, 0, ctypes.byref(h)) == _lib.PS_E_INVALID
    assert L.periodic_sum_plan_load(b"x", 0, None) == _lib.PS_E_INVALID
    assert L.periodic_sum_plan_save(None, b"x") == _lib.PS_E_INVALID
    assert L.periodic_sum_plan_load(str(tmp_path / "missing.plan").encode(), 0, ctypes.byref(h)) == _lib.PS_E_IO
    assert h.value is None
    cases = {
        "empty": b"",
        "foreign": b"NOTAPLAN" + bytes(64),
        "short": b"PSPLAN01" + bytes(4),
        # right magic, wrong checksum
        "corrupt": b"PSPLAN01" + (1).to_bytes(4, "little") + (1).to_bytes(4, "little") + (256).to_bytes(4, "little")
                   + bytes(8) + bytes(8),
    }
    for name, data in cases.items():
        f = tmp_path / (name + ".plan")
        f.write_bytes(data)
        st = L.periodic_sum_plan_load(str(f).encode(), 0, ctypes.byref(h))
        assert st == _lib.PS_E_IO, name
        assert b"plan" in L.periodic_sum_last_error() or b"checksum" in L.periodic_sum_last_error(), name


def _fnv1a64(data):
    h = 0xcbf29ce484222325
    for b in data:
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_plan_file_with_valid_checksum_but_bad_contents_is_refused(tmp_path):
    """The reader checks every size and range, not only the checksum: a file
    whose system record claims p = 99 is refused with PS_E_IO."""
    import struct
    L = _lib.lib()
    head = b"PSPLAN01" + struct.pack("<Iiid", 4, 1, 256, 1.0)
    prm = struct.pack("<3didd", 1.0, 1.0, 1.0, 99, 1.5, 0.0) + struct.pack("<iid", 0, 0, 1e-13) \
        + struct.pack("<qqiiii", 100, 0, 0, 0, 0, 7) + struct.pack("<idi", 0, 0.0, 3)
    setup = struct.pack("<3di4d", 1.0, 1.0, 1.0, 0, 0.866, 1.5, 2.25, 1.0) + struct.pack("<4id", 99, 99 * 99, 10, 5, 1.0) \
        + struct.pack("<iii", 1, 0, 7) + struct.pack("<idi", 0, 0.0, 3)
    body = head + prm + setup
    f = tmp_path / "bad_p.plan"
    f.write_bytes(body + struct.pack("<Q", _fnv1a64(body)))
    h = ctypes.c_void_p()
    assert L.periodic_sum_plan_load(str(f).encode(), 0, ctypes.byref(h)) == _lib.PS_E_IO
    assert b"p out of range" in L.periodic_sum_last_error()


def test_plan_file_with_bad_image_list_is_refused(tmp_path):
    """A checksummed file whose image list repeats an image, or holds an image
    index beyond 2^16, is refused with PS_E_IO (the box-mean tables index a
    dense map over the image range)."""
    import struct
    L = _lib.lib()
    p, P, Lc = 2, 4, 6

    def plan_file(images):
        head = b"PSPLAN01" + struct.pack("<Iiid", 4, 1, 256, 1.0)
        prm = struct.pack("<3didd", 1.0, 1.0, 1.0, p, 1.5, 0.0) + struct.pack("<iid", 0, 0, 1e-13) \
            + struct.pack("<qqiiii", 100, 0, 0, 0, 0, 7) + struct.pack("<idi", 0, 0.0, 3)
        setup = struct.pack("<3di4d", 1.0, 1.0, 1.0, 0, 0.866, 1.5, 2.25, 1.0) \
            + struct.pack("<4id", p, P, Lc, P - 1, 1.0) + struct.pack("<iii", len(images), 0, 7) \
            + struct.pack("<idi", 0, 0.0, 3)
        arrays = struct.pack("<%dd" % (2 * 3 * Lc + (P - 1) * Lc + P), *([0.1] * (2 * 3 * Lc + (P - 1) * Lc + P)))
        arrays += struct.pack("<%di" % (3 * len(images)), *[v for im in images for v in im])
        body = head + prm + setup + arrays
        return body + struct.pack("<Q", _fnv1a64(body))

    h = ctypes.c_void_p()
    for name, images, msg in (("repeated", [(0, 0, 0), (1, 0, 0), (1, 0, 0)], b"repeated image"),
                              ("far", [(0, 0, 0), (0, 70000, 0)], b"image index out of range")):
        f = tmp_path / (name + ".plan")
        f.write_bytes(plan_file(images))
        assert L.periodic_sum_plan_load(str(f).encode(), 0, ctypes.byref(h)) == _lib.PS_E_IO, name
        assert msg in L.periodic_sum_last_error(), (name, L.periodic_sum_last_error())


def test_plan_file_with_bad_biharmonic_record_is_refused(tmp_path):
    """A checksummed file whose biharmonic system record has the harmonic basis
    size (p^2 instead of p^2 + (p-2)^2), or fewer than three periodic axes, is
    refused with PS_E_IO before any device work."""
    import struct
    L = _lib.lib()
    p = 4

    def plan_file(P, periodic):
        head = b"PSPLAN01" + struct.pack("<Iiid", 4, 1, 256, 1.0)
        prm = struct.pack("<3didd", 1.0, 1.0, 1.0, p, 1.5, 0.0) + struct.pack("<iid", 0, 0, 1e-13) \
            + struct.pack("<qqiiii", 100, 0, 0, 0, 0, periodic) + struct.pack("<idi", 2, 0.0, 3)
        setup = struct.pack("<3di4d", 1.0, 1.0, 1.0, 0, 0.866, 1.5, 2.25, 1.0) \
            + struct.pack("<4id", p, P, 28, P - 1, 1.0) + struct.pack("<iii", 1, 0, periodic) \
            + struct.pack("<idi", 2, 0.0, 3)
        body = head + prm + setup
        return body + struct.pack("<Q", _fnv1a64(body))

    h = ctypes.c_void_p()
    for name, P, per, msg in (("harmonic_size", p * p, 7, b"basis size does not match p"),
                              ("slab", p * p + (p - 2) ** 2, 3, b"bad biharmonic-kernel record")):
        f = tmp_path / (name + ".plan")
        f.write_bytes(plan_file(P, per))
        assert L.periodic_sum_plan_load(str(f).encode(), 0, ctypes.byref(h)) == _lib.PS_E_IO, name
        assert msg in L.periodic_sum_last_error(), (name, L.periodic_sum_last_error())


def _select(prm, tol=1e-6, lambdas=(1.3, 1.5), p_ref=0, n=10, null=None):
    """periodic_sum_select with stand-in particle pointers: every case here is
    rejected by the argument checks, before any device call."""
    L = _lib.lib()
    fake = ctypes.c_void_p(0x1000)
    lam = (ctypes.c_double * max(1, len(lambdas)))(*lambdas)
    rows = (_lib.ps_select_row * max(1, len(lambdas)))()
    best = ctypes.c_int32(7)
    args = [ctypes.byref(prm), 0, n, fake, fake, fake, fake, tol, lam, len(lambdas), p_ref, rows, ctypes.byref(best),
            None]
    if null is not None:
        args[null] = None
    return L.periodic_sum_select(*args), best.value


def test_select_row_layout():
    assert ctypes.sizeof(_lib.ps_select_row) == 8 + 4 + 4 + 5 * 8
    assert _lib.ps_select_row.B_P.offset == 16


@pytest.mark.parametrize("null", [0, 3, 6, 8, 11, 12])
def test_select_null_arguments_rejected(null):
    st, _ = _select(_params(), null=null)
    assert st == _lib.PS_E_INVALID


@pytest.mark.parametrize("kw", [dict(tol=0.0), dict(tol=1e-14), dict(tol=1.0), dict(tol=float("nan")),
                                dict(lambdas=()), dict(lambdas=(1.0,)), dict(lambdas=(1.5, 4.5)),
                                dict(p_ref=9), dict(p_ref=41), dict(n=0)])
def test_select_invalid_arguments_rejected(kw):
    st, best = _select(_params(), **kw)
    assert st == _lib.PS_E_INVALID
    assert best == -1
    assert _lib.lib().periodic_sum_last_error()


@pytest.mark.parametrize("kw", [dict(basis=1, n_centres=4), dict(n_check=10)])
def test_select_other_bases_unsupported(kw):
    st, _ = _select(_params(**kw))
    assert st == _lib.PS_E_UNSUPPORTED
