"""Incident plane wave and the TBC right-hand sides g1, g2 (oracle; test only).

Paper: Section 2 (incident and reflected waves, q = (alpha1, alpha2, -beta), p.q = 0),
Section 3 ((ENUC1): the source 2 i (alpha1 p3 + beta p1) e^{i(alpha1 x1 + alpha2 x2)};
g~1 of (nosig) and g1 = (h/q) 2 i (alpha1 p3 + beta p1) g~1), Appendix A (g2 with the
sin-cos projection and the normaliser c^(m,n)), Section 7 (E^inc = (cos a theta-hat +
sin a phi-hat) e^{i k d.x}, d = -(sin t cos f, sin t sin f, cos t)).

Readings: the exponent is e^{i k d.x}; polarisation 0 is theta-hat (alpha = 0),
polarisation 1 is phi-hat (alpha = pi/2).

The projections are separable products of 1D integrals, evaluated from their closed
forms through E(w) = int_0^L e^{i w x} dx = L e^{i w L/2} sinc(w L / 2), which has no
removable singularity left:
    C_m(alpha; a) = int_0^a cos(mu_m x) e^{i alpha x} dx = (E(alpha+mu_m) + E(alpha-mu_m)) / 2
    S_n(alpha; b) = int_0^b sin(nu_n y) e^{i alpha y} dy = (E(alpha+nu_n) - E(alpha-nu_n)) / 2i
"""
from __future__ import annotations

import numpy as np

from .problem import Problem


def plane_wave(k: float, theta: float, phi: float, pol: int):
    """Return (alpha1, alpha2, beta, p) for the incident wave of Section 7."""
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    alpha1 = -k * st * cp
    alpha2 = -k * st * sp
    beta = k * ct
    theta_hat = np.array([ct * cp, ct * sp, -st])
    phi_hat = np.array([-sp, cp, 0.0])
    ang = 0.0 if pol == 0 else 0.5 * np.pi
    p = np.cos(ang) * theta_hat + np.sin(ang) * phi_hat
    return alpha1, alpha2, beta, p


def exp_integral(w, length: float):
    """E(w) = int_0^length e^{i w x} dx, exact for all real or complex w."""
    w = np.asarray(w, dtype=complex)
    return length * np.exp(0.5j * w * length) * np.sinc(w * length / (2.0 * np.pi))


def cos_proj(alpha, freqs, length):
    """int_0^length cos(f x) e^{i alpha x} dx for each f in freqs."""
    return 0.5 * (exp_integral(alpha + freqs, length) + exp_integral(alpha - freqs, length))


def sin_proj(alpha, freqs, length):
    """int_0^length sin(f x) e^{i alpha x} dx for each f in freqs."""
    return (exp_integral(alpha + freqs, length) - exp_integral(alpha - freqs, length)) / 2j


def rhs(prob: Problem, theta: float, phi: float, pol: int):
    """g1 on the mode grid (valid on N1) and g2 (valid on N2), other entries zero."""
    a1, a2, beta, p = plane_wave(prob.k, theta, phi, pol)
    mu, nu = prob.mu, prob.nu
    n1, n2, _ = prob.masks()
    g1 = (prob.h / prob.q_norm()) * 2j * (a1 * p[2] + beta * p[0]) \
        * np.outer(cos_proj(a1, mu, prob.a), sin_proj(a2, nu, prob.b))
    g2 = (prob.h / prob.c_norm()) * 2j * (a2 * p[2] + beta * p[1]) \
        * np.outer(sin_proj(a1, mu, prob.a), cos_proj(a2, nu, prob.b))
    g1[~n1] = 0.0
    g2[~n2] = 0.0
    return g1, g2
