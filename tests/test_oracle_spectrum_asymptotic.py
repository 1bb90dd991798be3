"""Pins of the Case-2 (asymptotic) evaluation of the kernel spectrum (Section 5.2).

* The Fresnel tail int_Z^inf e^{ipz} / sqrt(z) dz against SciPy's oscillatory quadrature
  on the infinite interval (QUADPACK QAWF, independent of the Fresnel form) and against
  the exact Fresnel integrals (SciPy), for both signs of p.
* The whole Case-2 value against the quadrature spectrum within the error of the dropped
  O(z^-2) term of the J0 expansion: its tail integral oscillates, so the error falls like
  Z^{-5/2} / rho (Z = rho R); checked as |error| <= 0.05 Z^{-5/2} / rho over
  Z = 100 .. 3200, which a dropped 1/(8 z^{3/2}) term, a wrong Fresnel prefactor or a sign
  slip in either expansion exceeds by orders of magnitude.
* The case split: quadrature below the switch, Case 2 above it, on a whole lattice.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import fresnel

from oracle import spectrum as S
from oracle.problem import Problem

K = 2 * np.pi


@pytest.mark.parametrize("p,Z", [(1.3, 100.0), (-0.7, 150.0), (0.9, 400.0), (-1.6, 900.0)])
def test_fresnel_tail(p, Z):
    got = S.fresnel_tail(p, Z)
    re = quad(lambda z: 1.0 / np.sqrt(z), Z, np.inf, weight="cos", wvar=p)[0]
    im = quad(lambda z: 1.0 / np.sqrt(z), Z, np.inf, weight="sin", wvar=p)[0]
    ref = re + 1j * im
    assert abs(got - ref) <= 1e-6 * abs(ref)
    t = np.sqrt(2 * abs(p) * Z / np.pi)
    s_t, c_t = fresnel(t)
    ex = np.sqrt(np.pi / (2 * abs(p))) * ((1 - 2 * c_t) + 1j * (1 - 2 * s_t))
    ex = ex if p > 0 else np.conj(ex)
    assert abs(got - ex) <= 1e-6 * abs(ex)


@pytest.mark.parametrize("k,R", [(K, 8 * np.sqrt(2)), (2.5 * K, 3 * np.sqrt(2))])
def test_case2_within_expansion_error(k, R):
    Z = np.array([100.0, 200.0, 400.0, 800.0, 1600.0, 3200.0])
    rho = Z / R + k
    exact = S.ghat_radial(rho, k, R)
    asym = S.ghat_asymptotic(rho, k, R)
    zz = rho * R
    err = np.abs(asym - exact)
    assert np.all(err <= 0.05 * zz ** -2.5 / rho), err * rho * zz ** 2.5


def test_case_split_on_lattice():
    prob = Problem(2.0, 1.5, 0.5, 32, 24, 4, (4,), (1.0 + 0j,), K)
    exact = S.kernel_spectrum(prob, "exact")
    asym = S.kernel_spectrum(prob, "asymptotic")
    (p1, p2), (l1, l2) = prob.box, prob.box_len
    f1 = 2 * np.pi * S.signed_freq(p1) / l1
    f2 = 2 * np.pi * S.signed_freq(p2) / l2
    rho = np.sqrt(f1[:, None] ** 2 + f2[None, :] ** 2)
    far = (rho - prob.k) * prob.R >= S.ASYMPTOTIC_SWITCH
    assert far.mean() > 0.3 and (~far).any()
    assert np.array_equal(asym[~far], exact[~far])
    assert np.abs(asym[far] - exact[far]).max() <= 5e-8 * np.abs(exact).max()
    with pytest.raises(ValueError):
        S.kernel_spectrum(prob, "hankel")
