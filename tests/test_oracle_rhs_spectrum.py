"""Pins of the incident-field projections and of the truncated-kernel spectrum.

* C_m, S_n (Section 3 (nosig), Appendix A g2): closed forms against adaptive quadrature,
  including the removable points alpha = +-mu_m.
* G^_R(rho) = 1/2 int_0^R J0(rho r) e^{ikr} dr (Section 5.2): two independent quadratures
  (J0 panels vs. an angle midpoint rule), the rho = 0 closed form, the k = 0 closed form
  through Struve functions, and the infinite-range transform 1/sqrt(rho^2 - k^2) for a
  lossy wavenumber (where the tail beyond R is negligible).
"""
import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from oracle import incident, spectrum
from oracle.problem import Problem


def _quad_c(f, a, b):
    re = integrate.quad(lambda x: np.real(f(x)), a, b, epsabs=1e-15, epsrel=1e-14, limit=400)[0]
    im = integrate.quad(lambda x: np.imag(f(x)), a, b, epsabs=1e-15, epsrel=1e-14, limit=400)[0]
    return re + 1j * im


@pytest.mark.parametrize("alpha", [0.0, 1.3, -4.7, np.pi / 1.7 * 3, -np.pi / 1.7 * 2, 11.1])
def test_projections_vs_quadrature(alpha):
    L = 1.7
    freqs = np.pi * np.arange(8) / L
    c = incident.cos_proj(alpha, freqs, L)
    s = incident.sin_proj(alpha, freqs, L)
    for i, f in enumerate(freqs):
        cq = _quad_c(lambda x: np.cos(f * x) * np.exp(1j * alpha * x), 0, L)
        sq = _quad_c(lambda x: np.sin(f * x) * np.exp(1j * alpha * x), 0, L)
        assert abs(c[i] - cq) <= 1e-13 * max(1, abs(cq))
        assert abs(s[i] - sq) <= 1e-13 * max(1, abs(sq))


def test_rhs_structure():
    """g1 lives on N1, g2 on N2; at normal incidence with p = y^ only g2 survives and its
    x-projection vanishes for even m (sin(m pi x/a) integrates to zero)."""
    prob = Problem.from_cavity(W.vacuum_1x1x05().cavity)
    g1, g2 = incident.rhs(prob, 0.0, 0.0, W.TE)
    assert np.abs(g1).max() < 1e-14 * np.abs(g2).max()
    assert np.abs(g2[0, :]).max() == 0.0
    assert np.abs(g2[2::2, :]).max() < 1e-15 and np.abs(g2[1::2, 0]).min() > 1e-3
    # p = y^ at normal incidence: 2i beta p2 (h/c) S_m(0) C_n(0)
    k, h, a, b = prob.k, prob.h, prob.a, prob.b
    m = 3
    expect = (h / (a * b / 2)) * 2j * k * (a * (1 - (-1) ** m) / (m * np.pi)) * b
    assert abs(g2[m, 0] - expect) <= 1e-14 * abs(expect)


@pytest.mark.parametrize("rho", [0.0, 0.5, 3.0, 2 * np.pi, 17.0, 60.0, 142.0])
def test_ghat_two_quadratures(rho):
    k, R = 2 * np.pi, 8.0 * np.sqrt(2)
    a = spectrum.ghat_radial([rho], k, R)[0]
    b = spectrum.ghat_angle([rho], k, R)[0]
    # both sums carry rounding of order eps * R (terms of size R cancel to |G^|)
    assert abs(a - b) <= 1e-14 * R and abs(a - b) <= 5e-13 * abs(a)


def test_ghat_rho_zero_closed_form():
    k, R = 2 * np.pi, 1.3 * np.sqrt(2)
    expect = 0.5 * (np.exp(1j * k * R) - 1) / (1j * k)
    assert abs(spectrum.ghat_radial([0.0], k, R)[0] - expect) <= 1e-14


@pytest.mark.parametrize("rho", [0.7, 5.0, 33.0])
def test_ghat_static_struve(rho):
    R = 2.2
    x = rho * R
    integral_j0 = x * special.j0(x) + 0.5 * np.pi * x * (
        special.j1(x) * special.struve(0, x) - special.j0(x) * special.struve(1, x))
    expect = 0.5 * integral_j0 / rho
    assert abs(spectrum.ghat_radial([rho], 0.0, R)[0] - expect) <= 1e-13


@pytest.mark.parametrize("rho", [0.0, 3.0, 6.0, 25.0])
def test_ghat_lossy_infinite_range(rho):
    """For Im k > 0 and large R the truncated transform tends to 1/(2 sqrt(rho^2 - k^2))."""
    k, R = 2 * np.pi + 1.0j, 40.0
    s = -1j * k
    expect = 0.5 / np.sqrt(s * s + rho * rho)
    got = spectrum.ghat_radial([rho], k, R)[0]
    assert abs(got - expect) <= 1e-12 * abs(expect)


def test_kernel_spectrum_symmetry_and_lattice():
    prob = Problem.from_cavity(W.small_cases()[1].cavity)
    kh = spectrum.kernel_spectrum(prob)
    p1, p2 = prob.box
    assert kh.shape == (p1, p2)
    # K^ depends on |xi| only: even in each signed index
    i1 = (-np.arange(p1)) % p1
    i2 = (-np.arange(p2)) % p2
    assert np.array_equal(kh, kh[i1][:, i2])
    l1, l2 = prob.box_len
    rho = np.hypot(2 * np.pi * 3 / l1, 2 * np.pi * 5 / l2)
    assert abs(kh[3, p2 - 5] - spectrum.ghat_radial([rho], prob.k, prob.R)[0]) < 1e-15
