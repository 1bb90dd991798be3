"""Pins of the incident plane wave (oracle.incident.plane_wave) from geometry alone.

Section 2 states the incident wave as E_inc = p e^{i q.x} with q = (alpha1, alpha2, -beta)
and p.q = 0; Section 7 fixes q = k d with d = -(sin t cos f, sin t sin f, cos t) and the
polarisation p = cos(a) theta-hat + sin(a) phi-hat.  Nothing here reuses the oracle's
closed forms: theta-hat and phi-hat are the finite-difference derivatives of the radial
unit vector r^(theta, phi), d is minus that vector, and the frame (r^, theta-hat, phi-hat)
must be right-handed and orthonormal.  A sign slip in any component of theta-hat or
phi-hat, or in alpha1, alpha2, beta, fails one of these.
"""
import numpy as np
import pytest

from oracle import incident

K = 2.0 * np.pi


def r_hat(theta, phi):
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def _angles():
    rng = np.random.default_rng(20080196)
    th = rng.uniform(0.02, 0.5 * np.pi - 0.02, size=12)
    ph = rng.uniform(-np.pi, 3 * np.pi, size=12)
    return list(zip(th, ph)) + [(0.3, 0.0), (1.2, 0.5 * np.pi), (0.7, np.pi), (1.0, 4.0)]


@pytest.mark.parametrize("theta,phi", _angles())
def test_direction_is_minus_radial(theta, phi):
    a1, a2, beta, _ = incident.plane_wave(K, theta, phi, 0)
    q = np.array([a1, a2, -beta])
    assert np.abs(q - (-K) * r_hat(theta, phi)).max() <= 1e-14 * K


@pytest.mark.parametrize("theta,phi", _angles())
def test_polarisation_vectors_are_derivatives_of_radial(theta, phi):
    eps = 1e-6
    dth = (r_hat(theta + eps, phi) - r_hat(theta - eps, phi)) / (2 * eps)
    dph = (r_hat(theta, phi + eps) - r_hat(theta, phi - eps)) / (2 * eps * np.sin(theta))
    _, _, _, p_tm = incident.plane_wave(K, theta, phi, 0)
    _, _, _, p_te = incident.plane_wave(K, theta, phi, 1)
    assert np.abs(p_tm - dth).max() <= 1e-8
    assert np.abs(p_te - dph).max() <= 1e-8


@pytest.mark.parametrize("theta,phi", _angles())
def test_unit_transverse_right_handed(theta, phi):
    a1, a2, beta, p_tm = incident.plane_wave(K, theta, phi, 0)
    _, _, _, p_te = incident.plane_wave(K, theta, phi, 1)
    q = np.array([a1, a2, -beta])
    for p in (p_tm, p_te):
        assert abs(np.linalg.norm(p) - 1.0) <= 1e-14
        assert abs(p @ q) <= 1e-13 * K
    assert abs(p_tm @ p_te) <= 1e-14
    # (r^, theta^, phi^) is a right-handed frame: theta^ x phi^ = r^
    assert np.abs(np.cross(p_tm, p_te) - r_hat(theta, phi)).max() <= 1e-14


def test_normal_incidence_limits():
    """theta = 0: theta-hat = (cos f, sin f, 0) and phi-hat = (-sin f, cos f, 0), the wave
    travels along -z with beta = k."""
    for phi in (0.0, 0.4, 2.5):
        a1, a2, beta, p_tm = incident.plane_wave(K, 0.0, phi, 0)
        _, _, _, p_te = incident.plane_wave(K, 0.0, phi, 1)
        assert abs(a1) <= 1e-15 and abs(a2) <= 1e-15
        assert beta == K
        assert np.abs(p_tm - np.array([np.cos(phi), np.sin(phi), 0.0])).max() <= 1e-15
        assert np.abs(p_te - np.array([-np.sin(phi), np.cos(phi), 0.0])).max() <= 1e-15
