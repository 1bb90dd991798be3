"""Python binding of libcavity.so, the MI355X cavity-scattering solver.

Argument marshalling only: every step of the solver runs in the library's HIP kernels.
PyTorch provides device memory for the field output and the current stream.  The
library must have been built in-tree (``paper_2008_01966_amd.build``); importing the
binding without it raises immediately - there is no CPU fallback.

Entry points mirror the C ABI in include/cavity.h: plan creation, solve, batched
solve, radar cross section, aperture coefficients, plan info, and the inspection
calls used by the parity tests.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcavity.so")

TM, TE = 0, 1
STATUS = {0: "ok", 1: "EINVAL", 2: "ENOMEM", 3: "ERESONANT", 4: "ENOCONV", 5: "EDEVICE",
          6: "ENOTIMPL"}


class CavityError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class C128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class EpsStack(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int), ("layer_nz", ctypes.POINTER(ctypes.c_int)),
                ("eps_r", ctypes.POINTER(C128)), ("layer_depth", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tbc_oversample", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("restart", ctypes.c_int),
                ("hbm_budget", ctypes.c_size_t), ("stream", ctypes.c_void_p),
                ("batch", ctypes.c_int), ("direct", ctypes.c_int),
                ("tbc_operator", ctypes.c_int), ("spectrum", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("N", ctypes.c_int), ("Nz", ctypes.c_int),
                ("P1", ctypes.c_int), ("P2", ctypes.c_int), ("n_ap", ctypes.c_longlong),
                ("unknowns", ctypes.c_longlong), ("device_bytes", ctypes.c_size_t),
                ("min_pivot", ctypes.c_double), ("last_iterations", ctypes.c_int),
                ("last_rel_residual", ctypes.c_double), ("ms_spectrum", ctypes.c_double),
                ("ms_elimination", ctypes.c_double), ("ms_preconditioner", ctypes.c_double),
                ("ms_rhs", ctypes.c_double), ("ms_krylov", ctypes.c_double),
                ("ms_synthesis", ctypes.c_double), ("lds_budget", ctypes.c_int),
                ("last_direct", ctypes.c_int), ("ms_factor", ctypes.c_double),
                ("tbc_rows_in_place", ctypes.c_int)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int), ("hbm_budget", ctypes.c_size_t),
                ("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("plan_cache_bytes", ctypes.c_size_t)]


class Request(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("Nz", ctypes.c_int),
                ("n_layers", ctypes.c_int), ("layer_nz", ctypes.POINTER(ctypes.c_int)),
                ("eps_r", ctypes.POINTER(C128)), ("k", ctypes.c_double),
                ("theta", ctypes.c_double), ("phi", ctypes.c_double), ("pol", ctypes.c_int),
                ("E_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("sigma", ctypes.c_double * 2),
                ("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("unknowns", ctypes.c_longlong), ("device_bytes", ctypes.c_size_t),
                ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("plan_reused", ctypes.c_int),
                ("group_size", ctypes.c_int)]


EXPORTS = [
    "cavity_opts_default", "cavity_plan_create", "cavity_solve", "cavity_solve_batch",
    "cavity_solve_group",
    "cavity_rcs", "cavity_rcs_many", "cavity_rcs_many_noalloc", "cavity_aperture", "cavity_plan_footprint", "cavity_plan_info",
    "cavity_plan_destroy", "cavity_status_string", "cavity_last_error",
    "cavity_server_opts_default", "cavity_server_create", "cavity_server_submit",
    "cavity_server_wait", "cavity_server_release", "cavity_server_now_ms",
    "cavity_server_destroy", "cavity_debug_columns",
    "cavity_debug_profiles", "cavity_debug_spectrum", "cavity_debug_tbc",
    "cavity_debug_operator", "cavity_debug_rhs", "cavity_debug_fft_plans", "cavity_probe_kernel",
    "cavity_probe_read",
]
_NOT_INT = ("cavity_plan_destroy", "cavity_status_string", "cavity_last_error",
            "cavity_server_destroy", "cavity_server_now_ms")

KERNELS = {"spectrum": 0, "elimination": 1, "tbc_rows_fwd": 2, "tbc_cols": 3,
           "tbc_rows_bwd": 4, "epilogue": 5, "synth_rows": 6, "synth_cols": 7,
           "tbc_rows_fwd_f32": 8, "tbc_cols_f32": 9, "tbc_rows_bwd_f32": 10}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcavity.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2008_01966_amd.build`")
    # PyTorch ships its own HIP runtime.  Loading torch first makes the library bind to that
    # same runtime (identical soname), so the process holds one HIP runtime, not two.
    _torch()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, d, i = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    lib.cavity_opts_default.argtypes = [P(Opts)]
    lib.cavity_plan_create.argtypes = [d, d, d, i, i, i, P(EpsStack), d, P(Opts), P(vp)]
    lib.cavity_solve.argtypes = [vp, d, d, i, vp]
    lib.cavity_solve_batch.argtypes = [vp, i, P(d), P(d), P(i), vp, vp]
    lib.cavity_solve_group.argtypes = [i, P(vp), P(d), P(d), P(i), P(vp)]
    lib.cavity_rcs.argtypes = [vp, i, i, P(d), P(d), P(d)]
    lib.cavity_rcs_many.argtypes = [vp, i, P(i), P(d), P(d), P(d)]
    lib.cavity_rcs_many_noalloc.argtypes = [vp, i, P(i), P(d), P(d), P(d)]
    lib.cavity_aperture.argtypes = [vp, i, P(C128)]
    lib.cavity_plan_info.argtypes = [vp, P(Info)]
    lib.cavity_plan_destroy.argtypes = [vp]
    lib.cavity_plan_destroy.restype = None
    lib.cavity_status_string.argtypes = [i]
    lib.cavity_status_string.restype = ctypes.c_char_p
    lib.cavity_last_error.argtypes = []
    lib.cavity_last_error.restype = ctypes.c_char_p
    lib.cavity_debug_columns.argtypes = [vp, P(C128), P(C128), P(C128)]
    lib.cavity_debug_profiles.argtypes = [vp, P(C128), P(C128), P(C128)]
    lib.cavity_debug_spectrum.argtypes = [vp, P(C128)]
    lib.cavity_debug_tbc.argtypes = [vp, i, P(C128), P(C128)]
    lib.cavity_debug_operator.argtypes = [vp, P(C128), P(C128)]
    lib.cavity_debug_rhs.argtypes = [vp, d, d, i, P(C128), P(C128)]
    lib.cavity_debug_fft_plans.argtypes = [P(i), P(i), P(i)]
    lib.cavity_probe_kernel.argtypes = [i, i]
    lib.cavity_probe_read.argtypes = [P(i), P(d), P(d)]
    lib.cavity_plan_footprint.argtypes = [d, d, d, i, i, i, P(EpsStack), d, P(Opts),
                                          P(ctypes.c_size_t)]
    lib.cavity_server_opts_default.argtypes = [P(ServerOpts)]
    lib.cavity_server_create.argtypes = [P(ServerOpts), P(vp)]
    lib.cavity_server_submit.argtypes = [vp, P(Request), P(ctypes.c_longlong)]
    lib.cavity_server_wait.argtypes = [vp, ctypes.c_longlong, P(Result)]
    lib.cavity_server_release.argtypes = [vp, ctypes.c_longlong]
    lib.cavity_server_now_ms.argtypes = [vp]
    lib.cavity_server_now_ms.restype = d
    lib.cavity_server_destroy.argtypes = [vp]
    lib.cavity_server_destroy.restype = None
    for name in EXPORTS:
        if name not in _NOT_INT:
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().cavity_last_error().decode(errors="replace")
        raise CavityError(status, msg)


def _cbuf(arr: np.ndarray):
    assert arr.dtype == np.complex128 and arr.flags.c_contiguous
    return arr.ctypes.data_as(ctypes.POINTER(C128))


def _torch():
    import torch  # device memory and streams only
    return torch


# CAVITY_FP64: every step in double.  CAVITY_MIXED: the TBC convolutions inside the
# Krylov iterations in single precision, residuals (and everything else) in double.
PRECISIONS = {"fp64": 0, "mixed": 1}
# direct solve of the aperture system: automatic, always, never (GMRES only)
DIRECT = {"auto": 0, "always": 1, "never": -1}
# discrete TBC operator: trapezoid samples (D_trap) or exact trial transforms (D_spec)
OPERATORS = {"trap": 0, "spec": 1}
# kernel spectrum: quadrature everywhere, or the asymptotic (Case 2) form at large |xi|
SPECTRA = {"exact": 0, "asymptotic": 1}


class Plan:
    """One cavity geometry, grid and layer stack, with its resident device data."""

    def __init__(self, a: float, b: float, c: float, nx: int, ny: int, nz: int,
                 layer_nz: Optional[Sequence[int]] = None,
                 layer_eps: Optional[Sequence[complex]] = None, k: float = 2 * np.pi, *,
                 tol: float = 1e-12, restart: int = 60, max_iter: int = 400,
                 oversample: int = 1, hbm_budget: int = 0, stream: Optional[int] = None,
                 batch: int = 8, precision: str = "fp64", direct: str = "auto",
                 operator: str = "trap", layer_depth: Optional[Sequence[float]] = None,
                 spectrum: str = "exact"):
        lib = load_library()
        self._lib = lib
        self.a, self.b, self.c = float(a), float(b), float(c)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        opts = Opts()
        _check(lib.cavity_opts_default(ctypes.byref(opts)))
        opts.tol, opts.restart, opts.max_iter = float(tol), int(restart), int(max_iter)
        opts.tbc_oversample = int(oversample)
        opts.hbm_budget = int(hbm_budget)
        opts.batch = int(batch)
        if direct not in DIRECT:
            raise ValueError(f"direct must be one of {sorted(DIRECT)}")
        opts.direct = DIRECT[direct]
        if operator not in OPERATORS:
            raise ValueError(f"operator must be one of {sorted(OPERATORS)}")
        opts.tbc_operator = OPERATORS[operator]
        if spectrum not in SPECTRA:
            raise ValueError(f"spectrum must be one of {sorted(SPECTRA)}")
        opts.spectrum = SPECTRA[spectrum]
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        opts.precision = PRECISIONS[precision]
        self.precision = precision
        if stream is None:
            torch = _torch()
            stream = torch.cuda.current_stream().cuda_stream
        opts.stream = ctypes.c_void_p(int(stream))
        self._stream = stream
        eps_p = None
        if layer_nz is not None:
            nzs = (ctypes.c_int * len(layer_nz))(*[int(v) for v in layer_nz])
            epsv = (C128 * len(layer_eps))(*[C128(complex(e).real, complex(e).imag)
                                              for e in layer_eps])
            stack = EpsStack(len(layer_nz), nzs, epsv)
            depth = None
            if layer_depth is not None:
                depth = (ctypes.c_double * len(layer_depth))(*[float(v) for v in layer_depth])
                stack.layer_depth = depth
            self._keep = (nzs, epsv, depth)
            eps_p = ctypes.pointer(stack)
        elif layer_depth is not None:
            raise ValueError("layer_depth needs layer_nz and layer_eps")
        handle = ctypes.c_void_p()
        _check(lib.cavity_plan_create(self.a, self.b, self.c, self.nx, self.ny, self.nz, eps_p,
                                      float(k), ctypes.byref(opts), ctypes.byref(handle)))
        self._h = handle
        self.info_ = self.info()

    @classmethod
    def from_cavity(cls, cav, **kw) -> "Plan":
        kw.setdefault("oversample", cav.tbc_oversample)
        if getattr(cav, "layer_depth", None) is not None:
            kw.setdefault("layer_depth", cav.layer_depth)
        return cls(cav.a, cav.b, cav.c, cav.nx, cav.ny, cav.nz, cav.layer_nz, cav.layer_eps,
                   cav.k, **kw)

    # -- lifecycle -------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.cavity_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Info:
        out = Info()
        _check(self._lib.cavity_plan_info(self._h, ctypes.byref(out)))
        return out

    @property
    def grid_shape(self):
        inf = self.info_
        return (inf.M + 1, inf.N + 1)

    @property
    def field_shape(self):
        return (3, self.nz + 1, self.ny + 1, self.nx + 1)

    # -- solves ------------------------------------------------------------------------
    def empty_field(self, count: int = 1):
        torch = _torch()
        shape = self.field_shape if count == 1 else (count,) + self.field_shape
        return torch.empty(shape, dtype=torch.complex128, device="cuda")

    def solve(self, theta: float, phi: float, pol: int, out=None, field: bool = True):
        """Solve one incidence; returns the device field tensor (or None if field=False)."""
        if field and out is None:
            out = self.empty_field()
        ptr = ctypes.c_void_p(out.data_ptr()) if field else None
        _check(self._lib.cavity_solve(self._h, float(theta), float(phi), int(pol), ptr))
        return out if field else None

    def solve_batch(self, thetas, phis, pols, out=None, field: bool = True, aperture=None):
        n = len(thetas)
        th = (ctypes.c_double * n)(*map(float, thetas))
        ph = (ctypes.c_double * n)(*map(float, phis))
        po = (ctypes.c_int * n)(*map(int, pols))
        if field and out is None:
            out = self.empty_field(n)
        eptr = ctypes.c_void_p(out.data_ptr()) if field else None
        aptr = ctypes.c_void_p(aperture.data_ptr()) if aperture is not None else None
        _check(self._lib.cavity_solve_batch(self._h, n, th, ph, po, eptr, aptr))
        return out if field else None

    def rcs(self, index: int, theta_o, phi_o) -> np.ndarray:
        th = np.ascontiguousarray(np.atleast_1d(theta_o), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi_o), dtype=np.float64)
        sig = np.zeros((th.size, 2))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(self._lib.cavity_rcs(self._h, int(index), th.size, th.ctypes.data_as(dp),
                                    ph.ctypes.data_as(dp), sig.ctypes.data_as(dp)))
        return sig

    def rcs_many(self, indices, theta_o, phi_o) -> np.ndarray:
        """RCS of stored solution indices[i] at direction (theta_o[i], phi_o[i]) for every i,
        in one call; rows {sigma_theta, sigma_phi}."""
        idx = np.ascontiguousarray(np.atleast_1d(indices), dtype=np.int32)
        th = np.ascontiguousarray(np.atleast_1d(theta_o), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi_o), dtype=np.float64)
        if not idx.size == th.size == ph.size:
            raise ValueError("indices, theta_o and phi_o differ in length")
        sig = np.zeros((th.size, 2))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(self._lib.cavity_rcs_many(self._h, idx.size,
                                         idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                         th.ctypes.data_as(dp), ph.ctypes.data_as(dp),
                                         sig.ctypes.data_as(dp)))
        return sig

    def rcs_many_noalloc(self, indices, theta_o, phi_o) -> np.ndarray:
        """rcs_many through the library's no-allocation entry point (fixed device scratch;
        calls on one device must not overlap)."""
        idx = np.ascontiguousarray(np.atleast_1d(indices), dtype=np.int32)
        th = np.ascontiguousarray(np.atleast_1d(theta_o), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi_o), dtype=np.float64)
        if not idx.size == th.size == ph.size:
            raise ValueError("indices, theta_o and phi_o differ in length")
        sig = np.zeros((th.size, 2))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(self._lib.cavity_rcs_many_noalloc(self._h, idx.size,
                                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                                 th.ctypes.data_as(dp), ph.ctypes.data_as(dp),
                                                 sig.ctypes.data_as(dp)))
        return sig

    def aperture(self, index: int = 0) -> np.ndarray:
        out = np.zeros(self.info_.n_ap, dtype=np.complex128)
        _check(self._lib.cavity_aperture(self._h, int(index), _cbuf(out)))
        return out

    # -- inspection of individual steps ------------------------------------------------
    def debug_columns(self):
        shp = self.grid_shape
        rd, T, rn = (np.zeros(shp, np.complex128) for _ in range(3))
        _check(self._lib.cavity_debug_columns(self._h, _cbuf(rd), _cbuf(T), _cbuf(rn)))
        return rd, T, rn

    def debug_profiles(self):
        shp = (self.nz + 1,) + self.grid_shape
        pd, td, pn = (np.zeros(shp, np.complex128) for _ in range(3))
        _check(self._lib.cavity_debug_profiles(self._h, _cbuf(pd), _cbuf(td), _cbuf(pn)))
        return pd, td, pn

    def debug_spectrum(self):
        out = np.zeros((self.info_.P1, self.info_.P2), np.complex128)
        _check(self._lib.cavity_debug_spectrum(self._h, _cbuf(out)))
        return out

    def debug_tbc(self, family: int, coef: np.ndarray) -> np.ndarray:
        inp = np.ascontiguousarray(coef, dtype=np.complex128).reshape(self.grid_shape)
        out = np.zeros(self.grid_shape, np.complex128)
        _check(self._lib.cavity_debug_tbc(self._h, int(family), _cbuf(inp), _cbuf(out)))
        return out

    def debug_operator(self, e1, e2, e3):
        inp = np.ascontiguousarray(np.stack([e1, e2, e3]), dtype=np.complex128)
        out = np.zeros_like(inp)
        _check(self._lib.cavity_debug_operator(self._h, _cbuf(inp), _cbuf(out)))
        return out[0], out[1], out[2]

    def debug_rhs(self, theta: float, phi: float, pol: int):
        g1 = np.zeros(self.grid_shape, np.complex128)
        g2 = np.zeros(self.grid_shape, np.complex128)
        _check(self._lib.cavity_debug_rhs(self._h, float(theta), float(phi), int(pol), _cbuf(g1),
                                          _cbuf(g2)))
        return g1, g2


def fft_plans(lengths):
    """Stage radices the transform planner gives a plan whose six transform lengths are
    `lengths` (2 s Nx, 2 s Ny, P1, P2, 2 Nx, 2 Ny): a list of six tuples (empty when a length
    has no factorisation).  Host only (cavity_debug_fft_plans)."""
    lib = load_library()
    ln = (ctypes.c_int * 6)(*map(int, lengths))
    rad = (ctypes.c_int * 120)()
    nst = (ctypes.c_int * 6)()
    _check(lib.cavity_debug_fft_plans(ln, rad, nst))
    return [tuple(rad[20 * k + t] for t in range(nst[k])) for k in range(6)]


def solve_group(plans, thetas, phis, pols, fields: bool = True):
    """One incidence on each of several plans that share an aperture, solved as one lockstep
    group (cavity_solve_group); returns the list of device field tensors (or None)."""
    lib = load_library()
    n = len(plans)
    hs = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
    th = (ctypes.c_double * n)(*map(float, thetas))
    ph = (ctypes.c_double * n)(*map(float, phis))
    po = (ctypes.c_int * n)(*map(int, pols))
    outs = [p.empty_field() for p in plans] if fields else None
    eptr = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs]) if fields else None
    _check(lib.cavity_solve_group(n, hs, th, ph, po, eptr))
    return outs


def probe_start(kernel: str, capacity: int = 100000):
    """Start timing every launch of one kernel (HIP events on its launch stream)."""
    _check(load_library().cavity_probe_kernel(KERNELS[kernel], int(capacity)))


def probe_stop():
    """Return (launches, total device ms, total algorithmic bytes) and stop the probe."""
    lib = load_library()
    n, ms, by = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(lib.cavity_probe_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    _check(lib.cavity_probe_kernel(-1, 0))
    return n.value, ms.value, by.value


class Server:
    """Request server of the library: cavities of any size solved for one incidence each,
    several in flight on the GPU, the oldest queued request that fits admitted within a
    device-memory budget, plans of finished requests kept resident for repeated cavities.
    Results carry the backscatter RCS, iteration count and timestamps; the field goes to
    the caller's device tensor when one is given to submit()."""

    def __init__(self, streams: int = 4, hbm_budget: int = 0, precision: str = "mixed",
                 tol: float = 1e-12, plan_cache_bytes: Optional[int] = None):
        lib = load_library()
        self._lib = lib
        o = ServerOpts()
        _check(lib.cavity_server_opts_default(ctypes.byref(o)))
        o.streams, o.hbm_budget, o.tol = int(streams), int(hbm_budget), float(tol)
        if plan_cache_bytes is not None:
            o.plan_cache_bytes = int(plan_cache_bytes)
        o.precision = PRECISIONS[precision]
        h = ctypes.c_void_p()
        _check(lib.cavity_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, cav, theta: float, phi: float, pol: int, out=None) -> int:
        """Queue cavity `cav` (a workloads.Cavity-like object) at one incidence; `out`: an
        optional complex128 device tensor of shape (3, Nz+1, Ny+1, Nx+1) for the field,
        which must stay alive until wait() returns.  The server's plans use the common
        z-step, so a cavity with its own layer thicknesses is refused."""
        if getattr(cav, "layer_depth", None) is not None:
            raise ValueError("the request server does not take layer thicknesses; "
                             "use Plan(layer_depth=...)")
        nzs = (ctypes.c_int * len(cav.layer_nz))(*[int(v) for v in cav.layer_nz])
        eps = (C128 * len(cav.layer_eps))(*[C128(complex(e).real, complex(e).imag)
                                            for e in cav.layer_eps])
        eptr = None
        if out is not None:
            torch = _torch()
            assert out.dtype == torch.complex128 and out.is_cuda and out.is_contiguous()
            assert tuple(out.shape) == (3, cav.nz + 1, cav.ny + 1, cav.nx + 1)
            eptr = out.data_ptr()
        r = Request(cav.a, cav.b, cav.c, cav.nx, cav.ny, cav.nz, len(cav.layer_nz), nzs, eps,
                    cav.k, float(theta), float(phi), int(pol), eptr)
        t = ctypes.c_longlong()
        _check(self._lib.cavity_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = out
        return t.value

    def wait(self, ticket: int) -> Result:
        out = Result()
        _check(self._lib.cavity_server_wait(self._h, ctypes.c_longlong(ticket), ctypes.byref(out)))
        return out

    def release(self, ticket: int):
        _check(self._lib.cavity_server_release(self._h, ctypes.c_longlong(ticket)))
        self._keep.pop(ticket, None)

    def now_ms(self) -> float:
        return float(self._lib.cavity_server_now_ms(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.cavity_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
