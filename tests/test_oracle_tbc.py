"""Pins of the discrete single-layer operators S^f (Section 5 of the paper).

* The FFT form equals the double-sum definition with a directly summed discrete kernel.
* The separable diagonal equals the diagonal of the dense operator; S^f is complex
  symmetric (the kernel depends on |x - y| only).
* As the trapezoid grid is refined (s = 2, 4, 8, 16 quadrature intervals per mode
  interval) the operator converges to the exact Galerkin integrals (sig1)-(sig3),
  computed independently in polar coordinates around the singularity.
* The discrete kernel approaches g(x) = e^{ik|x|}/(4 pi |x|) away from x = 0 (loose).
* D_spec (exact trial transforms on the same lattice): its fast form equals its entry-by-
  entry definition, it is complex symmetric with the stated diagonal, and it converges to
  the same exact Galerkin integrals at second order in the lattice size, about ten times
  closer than D_trap on every lattice.
"""
import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import spectrum, tbc
from oracle.problem import Problem


def _tiny(s=1, nx=5, ny=4, a=0.8, b=0.6):
    return Problem.from_cavity(W.Cavity(a, b, 0.3, nx, ny, 3, (3,), (1.0 + 0j,), tbc_oversample=s))


@pytest.mark.parametrize("family", ["cs", "sc", "cc"])
@pytest.mark.parametrize("s", [1, 2])
def test_fft_equals_double_sum(family, s):
    prob = _tiny(s)
    kh = spectrum.kernel_spectrum(prob)
    dense = tbc.dense_matrix_direct(prob, kh, family)
    fft = tbc.dense_matrix_fft(prob, kh, family)
    assert np.abs(dense - fft).max() <= 1e-13 * np.abs(dense).max()
    assert np.abs(dense - dense.T).max() <= 1e-13 * np.abs(dense).max()
    diag = tbc.diagonal(prob, kh, family).ravel()
    assert np.abs(np.diag(dense) - diag).max() <= 1e-13 * np.abs(diag).max()


def _corr(kind, f, length, u):
    """int over the overlap of psi(x) psi(x - u), psi = cos(f x) or sin(f x) on [0, L]."""
    lo, hi = max(0.0, u), min(length, length + u)
    if hi <= lo:
        return 0.0
    if f == 0.0:
        return (hi - lo) if kind == "c" else 0.0
    osc = (np.sin(2 * f * hi - f * u) - np.sin(2 * f * lo - f * u)) / (2 * f)
    if kind == "c":
        return 0.5 * ((hi - lo) * np.cos(f * u) + osc)
    return 0.5 * ((hi - lo) * np.cos(f * u) - osc)


def _galerkin_exact(k, a, b, kind1, f1, kind2, f2):
    """int_Gamma int_Gamma psi(x) psi(y) g(x - y) dx dy with u = x - y in polar form."""
    def integrand_theta(th):
        c, s = np.cos(th), np.sin(th)
        rmax = min(a / abs(c) if abs(c) > 1e-15 else np.inf, b / abs(s) if abs(s) > 1e-15 else np.inf)
        fr = lambda r: np.exp(1j * k * r) / (4 * np.pi) * _corr(kind1, f1, a, r * c) * _corr(kind2, f2, b, r * s)  # noqa: E731
        re = integrate.quad(lambda r: fr(r).real, 0, rmax, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
        im = integrate.quad(lambda r: fr(r).imag, 0, rmax, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
        return re + 1j * im
    tc = np.arctan2(b, a)
    brk = [0, tc, np.pi - tc, np.pi, np.pi + tc, 2 * np.pi - tc, 2 * np.pi]
    total = 0.0
    for t0, t1 in zip(brk[:-1], brk[1:]):
        re = integrate.quad(lambda t: integrand_theta(t).real, t0, t1, epsabs=1e-12, epsrel=1e-11, limit=200)[0]
        im = integrate.quad(lambda t: integrand_theta(t).imag, t0, t1, epsabs=1e-12, epsrel=1e-11, limit=200)[0]
        total += re + 1j * im
    return total


@pytest.mark.slow
def test_converges_to_galerkin_integrals():
    a, b, nx, ny = 1.0, 0.75, 4, 3
    k = 2 * np.pi
    entries = [("cc", (0, 0), ("c", 0.0, "c", 0.0)),
               ("cs", (1, 1), ("c", np.pi / a, "s", np.pi / b)),
               ("sc", (2, 1), ("s", 2 * np.pi / a, "c", np.pi / b))]
    exact = {f: _galerkin_exact(k, a, b, *spec) for f, _, spec in entries}
    errs = {f: [] for f, _, _ in entries}
    for s in (2, 4, 8, 16):
        prob = Problem.from_cavity(W.Cavity(a, b, 0.3, nx, ny, 3, (3,), (1.0 + 0j,),
                                            tbc_oversample=s))
        kh = spectrum.kernel_spectrum(prob)
        for f, (m, n), _ in entries:
            d = tbc.diagonal(prob, kh, f)[m, n]
            errs[f].append(abs(d - exact[f]) / abs(exact[f]))
    for f in errs:
        e = np.array(errs[f])
        assert e[-1] < 5e-3, (f, e)
        assert np.all(e[1:] < e[:-1]), (f, e)
        assert np.log2(e[0] / e[-1]) / 3 > 1.2, (f, e)   # at least ~h^1.2 overall


def test_discrete_kernel_approaches_green_function():
    prob = Problem.from_cavity(W.Cavity(1.0, 1.0, 0.3, 64, 64, 3, (3,), (1.0 + 0j,)))
    kh = spectrum.kernel_spectrum(prob)
    kern = np.fft.ifft2(kh) / (prob.hq[0] * prob.hq[1])
    hq = prob.hq[0]
    for (i1, i2) in [(16, 0), (10, 20), (32, 32), (48, 8)]:
        r = hq * np.hypot(i1, i2)
        g = np.exp(1j * prob.k * r) / (4 * np.pi * r)
        assert abs(kern[i1, i2] - g) < 0.05 * abs(g)


@pytest.mark.parametrize("family", ["cs", "sc", "cc"])
def test_spec_fast_form_equals_definition(family):
    prob = _tiny(1)
    kh = spectrum.kernel_spectrum(prob)
    dense = tbc.dense_matrix_spec(prob, kh, family)
    shape = (prob.M + 1, prob.N + 1)
    n = shape[0] * shape[1]
    fast = np.zeros((n, n), dtype=complex)
    for col in range(n):
        e = np.zeros(n, dtype=complex)
        e[col] = 1.0
        fast[:, col] = tbc.apply_spec(prob, kh, family, e.reshape(shape)).ravel()
    scale = np.abs(dense).max()
    assert np.abs(dense - fast).max() <= 1e-13 * scale
    assert np.abs(dense - dense.T).max() <= 1e-13 * scale
    diag = tbc.diagonal_spec(prob, kh, family).ravel()
    assert np.abs(np.diag(dense) - diag).max() <= 1e-13 * scale


@pytest.mark.slow
def test_spec_converges_to_galerkin_integrals():
    a, b, nx, ny = 1.0, 0.75, 4, 3
    k = 2 * np.pi
    entries = [("cc", (0, 0), ("c", 0.0, "c", 0.0)),
               ("cs", (1, 1), ("c", np.pi / a, "s", np.pi / b)),
               ("sc", (2, 1), ("s", 2 * np.pi / a, "c", np.pi / b))]
    exact = {f: _galerkin_exact(k, a, b, *spec) for f, _, spec in entries}
    errs = {f: [] for f, _, _ in entries}
    for s in (1, 2, 4, 8):
        prob = Problem.from_cavity(W.Cavity(a, b, 0.3, nx, ny, 3, (3,), (1.0 + 0j,),
                                            tbc_oversample=s))
        kh = spectrum.kernel_spectrum(prob)
        for f, (m, n), _ in entries:
            d_spec = tbc.diagonal_spec(prob, kh, f)[m, n]
            d_trap = tbc.diagonal(prob, kh, f)[m, n]
            e_spec = abs(d_spec - exact[f]) / abs(exact[f])
            e_trap = abs(d_trap - exact[f]) / abs(exact[f])
            assert e_spec < e_trap / 4, (f, s, e_spec, e_trap)
            errs[f].append(e_spec)
    for f in errs:
        e = np.array(errs[f])
        assert e[-1] < 1e-3, (f, e)
        assert np.all(np.log2(e[:-1] / e[1:]) > 1.6), (f, e)     # about second order
