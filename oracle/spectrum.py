"""Fourier transform of the truncated free-space kernel (oracle; test only).

Paper: Section 5.2.  The inner single-layer integral is a convolution with
G(x) = g(x) 1{|x| <= R}, g = e^{i k |x|} / (4 pi |x|), R = sqrt(2) * max side.  Its 2D
Fourier transform at a frequency of modulus rho reduces, by the polar integral that
produces the Bessel function J0, to
    G^_R(rho) = (1/(4 pi)) * 2 pi * int_0^R J0(rho r) e^{i k r} dr
              = 1/2 * int_0^R J0(rho r) e^{i k r} dr.
(Reading: the paper's printed form drops the 2 pi of the angular integral.)

The paper evaluates the radial integral by Gaussian quadrature for small rho and by
Hankel/Fresnel asymptotics for large rho.  The asymptotic branch carries the truncation
error of a two-term J0 expansion, too coarse to define an operator that two
implementations can agree on to 1e-10, so the default spectrum uses composite
Gauss-Legendre quadrature on [0, R] with panels no longer than a fraction of the local
oscillation period, for every rho (SciPy's J0 supplies the Bessel function).  The
asymptotic branch is restated separately (``ghat_asymptotic``, the "asymptotic" method of
``kernel_spectrum``) as a faster plan option with its error stated.

Asymptotic branch (Case 2 of Section 5.2), with these readings of the garbled print:
* int_0^inf J0(rho r) e^{ikr} dr = 1 / sqrt(rho^2 - k^2) for rho > k (the Laplace
  transform of J0; the print drops the square root);
* int_Z^inf e^{ipz} / sqrt(z) dz = sqrt(pi / (2p)) (1 + i - 2 C(t) - 2i S(t)),
  t = sqrt(2 p Z / pi), for p > 0 (the print has sqrt(pi) / (2p)); its conjugate for p < 0;
* sin(z - pi/4) = (e^{i(z - pi/4)} - e^{-i(z - pi/4)}) / (2i) (the print repeats one
  exponent);
* Case 2 applies where (rho - k) R >= 100: the paper switches at frequency index 10 on a
  unit side with R = sqrt(2) side, i.e. at rho R of about 2 pi 10 sqrt(2) = 89; the
  expansions depend on the oscillation count (rho - k) R of the slower tail term, which
  the switch bounds from below.

K^[j] = G^_R(|xi_j|) on the full FFT lattice xi_j = 2 pi (j1/L1, j2/L2) with signed
j_d in (-P_d/2, P_d/2].
"""
from __future__ import annotations

import numpy as np
from scipy.special import j0

from .problem import Problem

_GL_ORDER = 24


def ghat_radial(rho, k: float, R: float) -> np.ndarray:
    """1/2 int_0^R J0(rho r) e^{i k r} dr for an array of rho >= 0 (J0 panel rule)."""
    rho = np.atleast_1d(np.asarray(rho, dtype=float))
    out = np.empty(rho.shape, dtype=complex)
    xg, wg = np.polynomial.legendre.leggauss(_GL_ORDER)
    # panel count: at most ~1/2 oscillation of the faster factor per panel
    npan = np.ceil((rho + abs(k)) * R / np.pi).astype(int) + 2
    order = np.argsort(npan, kind="stable")
    start = 0
    while start < order.size:
        npanels = npan[order[start]]
        # group all rho needing at most 1.25x this panel count
        cap = int(npanels * 1.25) + 1
        stop = start
        while stop < order.size and npan[order[stop]] <= cap:
            stop += 1
        idx = order[start:stop]
        edges = np.linspace(0.0, R, cap + 1)
        half = 0.5 * np.diff(edges)
        mid = 0.5 * (edges[1:] + edges[:-1])
        r = (mid[:, None] + half[:, None] * xg[None, :]).ravel()
        w = (half[:, None] * wg[None, :]).ravel()
        ew = w * np.exp(1j * k * r)
        rr = rho[idx]
        # chunk to bound memory
        chunk = max(1, int(4_000_000 // r.size))
        for c0 in range(0, rr.size, chunk):
            rc = rr[c0:c0 + chunk]
            out[idx[c0:c0 + chunk]] = 0.5 * (j0(rc[:, None] * r[None, :]) @ ew)
        start = stop
    return out


def ghat_angle(rho, k: float, R: float, n_nodes: int | None = None) -> np.ndarray:
    """Second, independent quadrature of the same integral (used only in tests).

    J0(x) = (1/pi) int_0^pi e^{i x cos t} dt turns the radial integral into
    (1/(2 pi)) int_0^pi E_R(k + rho cos t) dt, E_R(w) = (e^{i w R} - 1)/(i w); the
    integrand is smooth and periodic in t, so the midpoint rule converges geometrically."""
    rho = np.atleast_1d(np.asarray(rho, dtype=float))
    out = np.empty(rho.shape, dtype=complex)
    for i, r0 in enumerate(rho):
        n = n_nodes or int(np.ceil(0.5 * (r0 + abs(k)) * R)) + 48
        t = (np.arange(n) + 0.5) * np.pi / n
        w = k + r0 * np.cos(t)
        er = R * np.exp(0.5j * w * R) * np.sinc(w * R / (2 * np.pi))
        out[i] = er.sum() / (2.0 * n)
    return out


ASYMPTOTIC_SWITCH = 100.0


def fresnel_tail(p, Z):
    """int_Z^inf e^{ipz} / sqrt(z) dz for real p != 0, Z >> 1, through the Fresnel
    integrals and their two-term asymptotic expansions (Section 5.2, Case 2):
    C(t) = 1/2 + f sin(pi t^2 / 2) - g cos(pi t^2 / 2),
    S(t) = 1/2 - f cos(pi t^2 / 2) - g sin(pi t^2 / 2),
    f = (1 - 3 / (pi t^2)^2) / (pi t),  g = (1 - 15 / (pi t^2)^2) / (pi^2 t^3)."""
    p = np.asarray(p, dtype=float)
    ap = np.abs(p)
    t = np.sqrt(2.0 * ap * Z / np.pi)
    x2 = (np.pi * t * t) ** 2
    f = (1.0 - 3.0 / x2) / (np.pi * t)
    g = (1.0 - 15.0 / x2) / (np.pi ** 2 * t ** 3)
    phi = ap * Z                                   # pi t^2 / 2
    one_m_2c = -2.0 * f * np.sin(phi) + 2.0 * g * np.cos(phi)
    one_m_2s = 2.0 * f * np.cos(phi) + 2.0 * g * np.sin(phi)
    val = np.sqrt(np.pi / (2.0 * ap)) * (one_m_2c + 1j * one_m_2s)
    return np.where(p > 0, val, np.conj(val))


def ghat_asymptotic(rho, k: float, R: float) -> np.ndarray:
    """1/2 I with I = int_0^R J0(rho r) e^{ikr} dr by the Case-2 steps of Section 5.2, for
    rho > k: the infinite-range integral minus the tail beyond R, the tail with J0 replaced
    by its two-term Hankel expansion, written over z = rho r as sums of
    int_Z^inf e^{ipz} z^{-1/2} dz and int_Z^inf e^{iqz} z^{-3/2} dz (Z = rho R), the second
    by parts through the first, the first through the Fresnel integrals."""
    rho = np.atleast_1d(np.asarray(rho, dtype=float))
    Z = rho * R
    a = k / rho
    em, ep = np.exp(-0.25j * np.pi), np.exp(0.25j * np.pi)

    def tail_32(q):
        # int_Z^inf e^{iqz} z^{-3/2} dz = 2 e^{iqZ} / sqrt(Z) + 2 i q int_Z^inf e^{iqz} / sqrt(z)
        return 2.0 * np.exp(1j * q * Z) / np.sqrt(Z) + 2j * q * fresnel_tail(q, Z)

    # tail integrand [cos(z - pi/4) / sqrt(z) + sin(z - pi/4) / (8 z^{3/2})] e^{i a z}
    T = 0.5 * em * fresnel_tail(1.0 + a, Z) + 0.5 * ep * fresnel_tail(a - 1.0, Z) \
        + (em * tail_32(1.0 + a) - ep * tail_32(a - 1.0)) / 16j
    I = 1.0 / np.sqrt(rho * rho - k * k + 0j) - np.sqrt(2.0 / np.pi) / rho * T
    return 0.5 * I


def ghat_cases(rho, k: float, R: float) -> np.ndarray:
    """Case 1 (quadrature) where (rho - k) R < ASYMPTOTIC_SWITCH, Case 2 elsewhere."""
    rho = np.atleast_1d(np.asarray(rho, dtype=float))
    far = (rho - k) * R >= ASYMPTOTIC_SWITCH
    out = np.empty(rho.shape, dtype=complex)
    if (~far).any():
        out[~far] = ghat_radial(rho[~far], k, R)
    if far.any():
        out[far] = ghat_asymptotic(rho[far], k, R)
    return out


def signed_freq(p: int) -> np.ndarray:
    """DFT index j = 0..P-1 mapped to signed frequency in (-P/2, P/2]."""
    j = np.arange(p)
    return np.where(j <= p // 2, j, j - p)


def kernel_spectrum(prob: Problem, method: str = "exact") -> np.ndarray:
    """K^[j1, j2] = G^_R(|xi_j|) on the P1 x P2 lattice (FFT index order); method "exact"
    (quadrature everywhere) or "asymptotic" (Case 2 where it applies)."""
    (p1, p2), (l1, l2) = prob.box, prob.box_len
    # evaluate once per distinct (|j1|, |j2|) pair: quadrant symmetry
    a1 = np.abs(signed_freq(p1))
    a2 = np.abs(signed_freq(p2))
    u1 = np.arange(a1.max() + 1)
    u2 = np.arange(a2.max() + 1)
    rho = np.sqrt((2 * np.pi * u1[:, None] / l1) ** 2 + (2 * np.pi * u2[None, :] / l2) ** 2)
    flat, inv = np.unique(rho.ravel(), return_inverse=True)
    if method == "exact":
        vals = ghat_radial(flat, prob.k, prob.R)
    elif method == "asymptotic":
        vals = ghat_cases(flat, prob.k, prob.R)
    else:
        raise ValueError("method must be 'exact' or 'asymptotic'")
    quad = vals[inv].reshape(rho.shape)
    return quad[a1[:, None], a2[None, :]]
