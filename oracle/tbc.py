"""Discrete single-layer operators of the transparent boundary condition (oracle).

Paper: Section 2 ((ENU1): the TBC operator built from S[phi](x) = int_Gamma g(x-y) phi(y)),
Section 3 ((sig1)-(sig3): Galerkin integrals F~, G~, H~ of the first TBC row; Appendix A
for the second row), Section 5.1 (integration by parts reduces G~ and H~ to the cos-cos
family I3, so only three families remain: I1 cos-sin, I2 sin-cos, I3 cos-cos), Section
5.2 (inner integral as a convolution with the truncated kernel, evaluated with the FFT
from the kernel's Fourier transform; outer integral by the trapezoidal rule).

Reading (the paper gives no grid, box or quadrature orders): for family f with 1D bases
(psi1, psi2), the operator on mode coefficients x is
    (S^f x)_alpha = sum_{i,i'} w_i psi_alpha(x_i) K[i - i' mod P] w_i' sum_beta x_beta psi_beta(x_i')
on the trapezoid grid x_i = (i1 hq1, i2 hq2), i_d = 0..s N_d, weights w_i, with the
discrete periodic kernel K[i] = (1/(L1 L2)) sum_j K^[j] e^{i xi_j . x_i} built from the
truncated kernel's spectrum on the P1 x P2 lattice.  The FFT form below computes exactly
that sum: synthesise, weight, zero-pad, FFT, multiply by K^/(hq1 hq2), inverse FFT, crop,
weight, project.

Spectral variant D_spec (the same lattice and kernel spectrum, exact trial transforms):
writing K[i - i'] as its lattice sum turns the double sum above into
    (S^f x)_alpha = (1/(L1 L2)) sum_j conj(A_alpha(xi_j)) K^[j] sum_beta A_beta(xi_j) x_beta,
with A_beta(xi) = sum_i w_i psi_beta(x_i) e^{-i xi . x_i}, the trapezoid rule for the
Fourier transform of the trial function over the aperture.  D_spec uses that transform
exactly, F_beta(xi) = int_Gamma psi_beta(x) e^{-i xi . x} dx (a product of two closed-form
1D integrals), with xi_j on the lattice centred at zero; it is a Galerkin discretisation of
the lattice-periodised truncated kernel and converges faster in the lattice size than the
trapezoid form (the paper's Section 5.2 evaluates the inner transform in closed form too).
"""
from __future__ import annotations

import numpy as np

from .incident import cos_proj, sin_proj
from .problem import Problem

FAMILIES = ("cs", "sc", "cc")


def bases(prob: Problem, nodes1: np.ndarray, nodes2: np.ndarray):
    """cos/sin basis matrices (modes x nodes) along both axes at the given nodes."""
    mu, nu = prob.mu, prob.nu
    c1 = np.cos(mu[:, None] * nodes1[None, :])
    s1 = np.sin(mu[:, None] * nodes1[None, :])
    c2 = np.cos(nu[:, None] * nodes2[None, :])
    s2 = np.sin(nu[:, None] * nodes2[None, :])
    return c1, s1, c2, s2


def quad_nodes(prob: Problem):
    (nq1, nq2), (hq1, hq2) = prob.nq, prob.hq
    return np.arange(nq1 + 1) * hq1, np.arange(nq2 + 1) * hq2


def family_bases(prob: Problem, family: str):
    x1, x2 = quad_nodes(prob)
    c1, s1, c2, s2 = bases(prob, x1, x2)
    return {"cs": (c1, s2), "sc": (s1, c2), "cc": (c1, c2)}[family]


def apply(prob: Problem, khat: np.ndarray, family: str, coef: np.ndarray) -> np.ndarray:
    """(S^f coef) on the (M+1) x (N+1) mode grid, FFT form."""
    b1, b2 = family_bases(prob, family)
    w1, w2 = prob.trapezoid_weights()
    (p1, p2), (hq1, hq2) = prob.box, prob.hq
    phi = w1[:, None] * (b1.T @ coef @ b2) * w2[None, :]
    pad = np.zeros((p1, p2), dtype=complex)
    pad[:phi.shape[0], :phi.shape[1]] = phi
    u = np.fft.ifft2(np.fft.fft2(pad) * khat) / (hq1 * hq2)
    u = u[:phi.shape[0], :phi.shape[1]]
    return b1 @ (w1[:, None] * u * w2[None, :]) @ b2.T


def discrete_kernel_direct(prob: Problem, khat: np.ndarray) -> np.ndarray:
    """K[i] = (1/(L1 L2)) sum_j K^[j] e^{i xi_j . x_i} by a direct double Fourier sum."""
    (p1, p2), (l1, l2), (hq1, hq2) = prob.box, prob.box_len, prob.hq
    j1 = np.arange(p1)
    j1s = np.where(j1 <= p1 // 2, j1, j1 - p1)
    j2 = np.arange(p2)
    j2s = np.where(j2 <= p2 // 2, j2, j2 - p2)
    e1 = np.exp(1j * (2 * np.pi * j1s[None, :] / l1) * (np.arange(p1)[:, None] * hq1))
    e2 = np.exp(1j * (2 * np.pi * j2s[None, :] / l2) * (np.arange(p2)[:, None] * hq2))
    return (e1 @ khat @ e2.T) / (l1 * l2)


def dense_matrix_direct(prob: Problem, khat: np.ndarray, family: str) -> np.ndarray:
    """Dense S^f on the full (M+1)(N+1) mode grid from the double-sum definition."""
    kern = discrete_kernel_direct(prob, khat)
    b1, b2 = family_bases(prob, family)
    w1, w2 = prob.trapezoid_weights()
    (p1, p2) = prob.box
    n1, n2 = b1.shape[1], b2.shape[1]
    i1 = np.arange(n1)
    i2 = np.arange(n2)
    d1 = (i1[:, None] - i1[None, :]) % p1
    d2 = (i2[:, None] - i2[None, :]) % p2
    # K over node pairs: [(i1, i2), (i1', i2')]
    kk = kern[d1[:, None, :, None], d2[None, :, None, :]].reshape(n1 * n2, n1 * n2)
    # psi_alpha(x_i) w_i as a matrix [node, mode]
    psi = np.einsum("im,jn->ijmn", w1[:, None] * b1.T, w2[:, None] * b2.T).reshape(
        n1 * n2, b1.shape[0] * b2.shape[0])
    return psi.T @ kk @ psi


def dense_matrix_fft(prob: Problem, khat: np.ndarray, family: str) -> np.ndarray:
    """Dense S^f by applying the FFT form to every unit vector (tiny sizes only)."""
    shape = (prob.M + 1, prob.N + 1)
    n = shape[0] * shape[1]
    out = np.zeros((n, n), dtype=complex)
    for col in range(n):
        e = np.zeros(n, dtype=complex)
        e[col] = 1.0
        out[:, col] = apply(prob, khat, family, e.reshape(shape)).ravel()
    return out


def diagonal(prob: Problem, khat: np.ndarray, family: str) -> np.ndarray:
    """Exact diagonal of S^f on the mode grid (separable form):
    S_aa = (1/(L1 L2)) sum_j K^[j] |A1_m(xi_j1)|^2 |A2_n(xi_j2)|^2,
    A_m(xi) = sum_i w_i psi_m(x_i) e^{i xi x_i}."""
    b1, b2 = family_bases(prob, family)
    w1, w2 = prob.trapezoid_weights()
    (p1, p2), (l1, l2), (hq1, hq2) = prob.box, prob.box_len, prob.hq
    n1, n2 = b1.shape[1], b2.shape[1]
    e1 = np.exp(2j * np.pi * np.outer(np.arange(n1), np.arange(p1)) / p1)
    e2 = np.exp(2j * np.pi * np.outer(np.arange(n2), np.arange(p2)) / p2)
    a1 = np.abs((w1[None, :] * b1) @ e1) ** 2  # (M+1) x P1
    a2 = np.abs((w2[None, :] * b2) @ e2) ** 2  # (N+1) x P2
    return (a1 @ khat @ a2.T) / (l1 * l2)


# ---- D_spec ------------------------------------------------------------------------
def lattice_freqs(prob: Problem):
    """xi on the P1 x P2 lattice, centred at zero, in FFT order along each axis."""
    (p1, p2), (l1, l2) = prob.box, prob.box_len
    j1 = np.arange(p1)
    j2 = np.arange(p2)
    j1s = np.where(j1 <= p1 // 2, j1, j1 - p1)
    j2s = np.where(j2 <= p2 // 2, j2, j2 - p2)
    return 2 * np.pi * j1s / l1, 2 * np.pi * j2s / l2


def spec_bases(prob: Problem, family: str):
    """F1[j1, m] = int_0^a psi_m(x) e^{-i xi_j1 x} dx and F2[j2, n] likewise along y, for
    the family's bases (cos or sin), closed form."""
    xi1, xi2 = lattice_freqs(prob)
    k1, k2 = {"cs": ("c", "s"), "sc": ("s", "c"), "cc": ("c", "c")}[family]
    proj = {"c": cos_proj, "s": sin_proj}
    f1 = proj[k1](-xi1[:, None], prob.mu[None, :], prob.a)
    f2 = proj[k2](-xi2[:, None], prob.nu[None, :], prob.b)
    return f1, f2


def apply_spec(prob: Problem, khat: np.ndarray, family: str, coef: np.ndarray) -> np.ndarray:
    """(S^f coef) of D_spec on the (M+1) x (N+1) mode grid."""
    f1, f2 = spec_bases(prob, family)
    l1, l2 = prob.box_len
    u = khat * (f1 @ coef @ f2.T) / (l1 * l2)
    return f1.conj().T @ u @ f2.conj()


def diagonal_spec(prob: Problem, khat: np.ndarray, family: str) -> np.ndarray:
    """Diagonal of D_spec's S^f: (1/(L1 L2)) sum_j K^[j] |F1_m(xi_j1)|^2 |F2_n(xi_j2)|^2."""
    f1, f2 = spec_bases(prob, family)
    l1, l2 = prob.box_len
    return (np.abs(f1).T ** 2) @ khat @ (np.abs(f2) ** 2) / (l1 * l2)


def dense_matrix_spec(prob: Problem, khat: np.ndarray, family: str) -> np.ndarray:
    """Dense S^f of D_spec from its definition entry by entry (tiny sizes only)."""
    f1, f2 = spec_bases(prob, family)
    l1, l2 = prob.box_len
    m1, m2 = f1.shape[1], f2.shape[1]
    out = np.zeros((m1 * m2, m1 * m2), dtype=complex)
    for a in range(m1 * m2):
        ma, na = divmod(a, m2)
        fa = np.outer(f1[:, ma], f2[:, na])
        for b in range(m1 * m2):
            mb, nb = divmod(b, m2)
            out[a, b] = np.sum(np.conj(fa) * khat * np.outer(f1[:, mb], f2[:, nb])) / (l1 * l2)
    return out
