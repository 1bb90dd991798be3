"""Fourier transform of the truncated free-space kernel (oracle; test only).

Paper: Section 5.2.  The inner single-layer integral is a convolution with
G(x) = g(x) 1{|x| <= R}, g = e^{i k |x|} / (4 pi |x|), R = sqrt(2) * max side.  Its 2D
Fourier transform at a frequency of modulus rho reduces, by the polar integral that
produces the Bessel function J0, to
    G^_R(rho) = (1/(4 pi)) * 2 pi * int_0^R J0(rho r) e^{i k r} dr
              = 1/2 * int_0^R J0(rho r) e^{i k r} dr.
(Reading: the paper's printed form drops the 2 pi of the angular integral.)

The paper evaluates the radial integral by Gaussian quadrature for small rho and by
Hankel/Fresnel asymptotics for large rho.  The asymptotic branch carries a truncation
error of 1e-6 .. 1e-9 (two-term J0 expansion), too coarse to define an operator that two
implementations can agree on to 1e-10, so the oracle uses composite Gauss-Legendre
quadrature on [0, R] with panels no longer than a fraction of the local oscillation
period, for every rho.  SciPy's J0 supplies the Bessel function.

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


def signed_freq(p: int) -> np.ndarray:
    """DFT index j = 0..P-1 mapped to signed frequency in (-P/2, P/2]."""
    j = np.arange(p)
    return np.where(j <= p // 2, j, j - p)


def kernel_spectrum(prob: Problem) -> np.ndarray:
    """K^[j1, j2] = G^_R(|xi_j|) on the P1 x P2 lattice (FFT index order)."""
    (p1, p2), (l1, l2) = prob.box, prob.box_len
    # evaluate once per distinct (|j1|, |j2|) pair: quadrant symmetry
    a1 = np.abs(signed_freq(p1))
    a2 = np.abs(signed_freq(p2))
    u1 = np.arange(a1.max() + 1)
    u2 = np.arange(a2.max() + 1)
    rho = np.sqrt((2 * np.pi * u1[:, None] / l1) ** 2 + (2 * np.pi * u2[None, :] / l2) ** 2)
    flat, inv = np.unique(rho.ravel(), return_inverse=True)
    vals = ghat_radial(flat, prob.k, prob.R)
    quad = vals[inv].reshape(rho.shape)
    return quad[a1[:, None], a2[None, :]]
