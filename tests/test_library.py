"""C-ABI library checks that need no GPU: the shared library loads, exports every entry
point include/cavity.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2008_01966_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "cavity.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cavity_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for name in ("cavity_plan_create", "cavity_solve", "cavity_rcs", "cavity_solve_batch"):
        assert name in syms
    assert sorted(P.EXPORTS) == syms


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_defaults_and_status_strings():
    lib = P.load_library()
    o = P.Opts()
    assert lib.cavity_opts_default(ctypes.byref(o)) == 0
    assert (o.precision, o.tbc_oversample, o.restart) == (0, 1, 60)
    assert o.tol == 1e-12 and o.max_iter == 400
    assert lib.cavity_status_string(0) == b"ok"
    assert lib.cavity_status_string(3) == b"resonant z-elimination pivot"


def _create(a=1.0, b=1.0, c=0.5, nx=16, ny=16, nz=8, eps=None, k=6.28, opts=None):
    lib = P.load_library()
    h = ctypes.c_void_p()
    st = lib.cavity_plan_create(a, b, c, nx, ny, nz, eps, k,
                                ctypes.byref(opts) if opts is not None else None,
                                ctypes.byref(h))
    return st, h, lib.cavity_last_error().decode()


@pytest.mark.parametrize("kw", [dict(a=-1.0), dict(c=0.0), dict(k=0.0), dict(nx=1), dict(nz=0)])
def test_invalid_arguments_rejected(kw):
    st, h, msg = _create(**kw)
    assert st == 1 and not h.value and msg


@pytest.mark.parametrize("kw", [dict(nx=17), dict(ny=19), dict(nx=46)])
def test_transform_lengths_beyond_the_radices_not_implemented(kw):
    """2 Nx or 2 Ny with a prime factor above 13 is a valid size the transforms do not
    cover: CAVITY_ENOTIMPL, not CAVITY_EINVAL."""
    st, h, msg = _create(**kw)
    assert st == 6 and not h.value and "prime factor" in msg


def test_invalid_layers_rejected():
    nzs = (ctypes.c_int * 2)(3, 4)
    eps = (P.C128 * 2)(P.C128(1, 0), P.C128(2, 0))
    stack = P.EpsStack(2, nzs, eps)
    st, h, msg = _create(nz=8, eps=ctypes.pointer(stack))
    assert st == 1 and "sum" in msg
    nzs0 = (ctypes.c_int * 2)(0, 8)
    st, h, msg = _create(nz=8, eps=ctypes.pointer(P.EpsStack(2, nzs0, eps)))
    assert st == 1


def test_invalid_layer_thickness_rejected():
    nzs = (ctypes.c_int * 2)(3, 5)
    eps = (P.C128 * 2)(P.C128(1, 0), P.C128(2, 0))
    for depth in ((0.2, 0.2), (0.6, -0.1), (0.25, float("nan"))):   # c = 0.5
        d = (ctypes.c_double * 2)(*depth)
        st, h, msg = _create(nz=8, eps=ctypes.pointer(P.EpsStack(2, nzs, eps, d)))
        assert st == 1 and not h.value and "thickness" in msg, depth


def test_invalid_options_rejected():
    lib = P.load_library()
    o = P.Opts()
    lib.cavity_opts_default(ctypes.byref(o))
    assert o.spectrum == 0
    o.spectrum = 2
    st, h, msg = _create(opts=o)
    assert st == 1 and "spectrum" in msg
    lib.cavity_opts_default(ctypes.byref(o))
    o.restart = 0
    assert _create(opts=o)[0] == 1
    lib.cavity_opts_default(ctypes.byref(o))
    o.precision = 7
    assert _create(opts=o)[0] == 1
    lib.cavity_opts_default(ctypes.byref(o))
    o.tbc_oversample = 0
    assert _create(opts=o)[0] == 1


def test_null_arguments_rejected():
    lib = P.load_library()
    assert lib.cavity_solve(None, 0.1, 0.0, 0, None) == 1
    assert lib.cavity_rcs(None, 0, 0, None, None, None) == 1
    assert lib.cavity_plan_info(None, None) == 1
    lib.cavity_plan_destroy(None)


def _footprint(a=1.0, b=1.0, c=0.5, nx=16, ny=16, nz=8, eps=None, k=6.28, opts=None):
    lib = P.load_library()
    out = ctypes.c_size_t()
    st = lib.cavity_plan_footprint(a, b, c, nx, ny, nz, eps, k,
                                   ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(out))
    return st, out.value


def test_footprint_needs_no_device_and_scales():
    """The device footprint is computed on the host: it grows with the grid, counts the
    Krylov basis of the restart length and the profiles of every level, and validates like
    plan creation."""
    st, small = _footprint()
    assert st == 0 and small > 0
    st, big = _footprint(a=8.0, b=8.0, c=2.0, nx=256, ny=256, nz=64)
    assert st == 0
    nm = 256 * 256
    assert big >= 16 * 2 * 65 * nm          # two profile arrays of 65 levels
    assert big >= 16 * 61 * 3 * nm          # restart 60: 61 basis vectors
    assert big < 4 << 30
    o = P.Opts()
    P.load_library().cavity_opts_default(ctypes.byref(o))
    o.restart = 20
    st, short = _footprint(a=8.0, b=8.0, c=2.0, nx=256, ny=256, nz=64, opts=o)
    assert st == 0 and short < big
    assert _footprint(nx=14)[0] == 0 and _footprint(nx=22)[0] == 0
    assert _footprint(nx=17)[0] == 6 and _footprint(c=-1.0)[0] == 1


def test_server_arguments_rejected_without_device():
    lib = P.load_library()
    o = P.ServerOpts()
    assert lib.cavity_server_opts_default(ctypes.byref(o)) == 0
    assert (o.streams, o.precision, o.tol) == (4, 1, 1e-12)
    h = ctypes.c_void_p()
    o.streams = 0
    assert lib.cavity_server_create(ctypes.byref(o), ctypes.byref(h)) == 1 and not h.value
    r = P.Request()
    t = ctypes.c_longlong()
    assert lib.cavity_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == 1
    assert lib.cavity_server_wait(None, 1, None) == 1
    assert lib.cavity_server_release(None, 1) == 1
    lib.cavity_server_destroy(None)


def test_direct_option_validated_without_device():
    """The direct-solve switch takes -1, 0 or 1; forcing it needs 3 Nx Ny <= 4096."""
    lib = P.load_library()
    o = P.Opts()
    lib.cavity_opts_default(ctypes.byref(o))
    assert o.direct == 0
    for val, nx, ny, want in ((2, 16, 16, 1), (-2, 16, 16, 1), (1, 16, 16, 0), (-1, 16, 16, 0),
                              (1, 40, 40, 1), (0, 40, 40, 0), (1, 32, 40, 0)):
        o.direct = val
        st, _ = _footprint(nx=nx, ny=ny, opts=o)
        assert st == want, (val, nx, ny, st)


def test_tbc_operator_option_validated_without_device():
    """tbc_operator takes CAVITY_TBC_TRAP (0, default) or CAVITY_TBC_SPEC (1); the spectral
    operator's transforms and product workspace show in the footprint."""
    lib = P.load_library()
    o = P.Opts()
    lib.cavity_opts_default(ctypes.byref(o))
    assert o.tbc_operator == 0
    st, trap = _footprint(opts=o)
    assert st == 0
    o.tbc_operator = 1
    st, spec = _footprint(opts=o)
    assert st == 0 and spec > trap
    for bad in (2, -1):
        o.tbc_operator = bad
        assert _footprint(opts=o)[0] == 1


def test_binding_validates_spectrum_and_thickness_arguments():
    """The binding refuses an unknown spectrum method and layer thicknesses without a layer
    stack before anything reaches the device."""
    with pytest.raises(ValueError):
        P.Plan(1.0, 1.0, 0.5, 16, 16, 8, stream=0, spectrum="hankel")
    with pytest.raises(ValueError):
        P.Plan(1.0, 1.0, 0.5, 16, 16, 8, stream=0, layer_depth=(0.5,))
    assert P.SPECTRA == {"exact": 0, "asymptotic": 1}


def test_fft_planner_radix_choice():
    """The transform planner's choice for the six lengths of a plan (2 s Nx, 2 s Ny, P1, P2,
    2 Nx, 2 Ny), host only: radices up to 8 where they need no more stages; all six in radices
    up to 8 when each needs at most one stage more and is at most 1000 points long; otherwise
    each length on its fewest stages.  Every factorisation multiplies out to its length."""
    small8 = [(8, 8, 8)] * 2 + [(5, 5, 5, 5)] * 2 + [(8, 8, 8)] * 2
    assert P.fft_plans((512, 512, 625, 625, 512, 512)) == small8
    # one stage more than 16.8 and 16.10 (2 wavelengths at 32 nodes per wavelength)
    assert P.fft_plans((128, 128, 160, 160, 128, 128)) == \
        [(8, 4, 4)] * 2 + [(8, 5, 4)] * 2 + [(8, 4, 4)] * 2
    # one stage more than 12.8.8 and 12.10.8 (12 wavelengths)
    assert P.fft_plans((768, 768, 960, 960, 768, 768)) == \
        [(8, 6, 4, 4)] * 2 + [(8, 6, 5, 4)] * 2 + [(8, 6, 4, 4)] * 2
    # above 1000 points no extra stage: 1024 and 1250 keep 16.8.8 and 10.5.5.5
    assert P.fft_plans((1024, 1024, 1250, 1250, 1024, 1024)) == \
        [(16, 8, 8)] * 2 + [(10, 5, 5, 5)] * 2 + [(16, 8, 8)] * 2
    # one length beyond the bound keeps the others on their fewest stages too
    assert P.fft_plans((768, 768, 2048, 2048, 960, 128)) == \
        [(12, 8, 8)] * 2 + [(16, 16, 8)] * 2 + [(12, 10, 8), (16, 8)]
    # the prime radix 11 (the M = N = 21 geometries of Section 7: 44 = 4 x 11)
    assert P.fft_plans((44, 44, 100, 100, 44, 44)) == [(11, 4)] * 2 + [(10, 10)] * 2 + [(11, 4)] * 2
    # no factorisation: a prime factor above 13
    assert P.fft_plans((34, 34, 40, 40, 34, 34))[0] == ()
    for n in (6, 30, 96, 250, 378, 486, 640, 729, 1000, 1452, 2000, 3125):
        for plan in P.fft_plans((n,) * 6):
            assert _product(plan) == n and max(plan) <= 16
    with pytest.raises(P.CavityError):
        P.fft_plans((0, 1, 2, 3, 4, 5))


def _product(t):
    out = 1
    for r in t:
        out *= r
    return out
