"""Back-substitution into the cavity and the radar cross section (oracle; test only).

Paper: Section 3 ((EInter): interior values from the aperture values, column by column),
Section 4 (the same per layer), Section 2 ((EGa2): the scattered field is radiated by the
aperture's tangential field with image doubling), Section 7 (backscatter RCS for the
theta-theta and phi-phi polarisations).

Field synthesis: on the nodes x1 = i1 a/Nx, x2 = i2 b/Ny, z_j = -c + j h the field is the
truncated series (E123F) with the column values E_{l,j}^(m,n) = Pi_j E_l + (mu|nu) Theta_j
E3 (E3: Pi3_j E3).  Output layout [component][j][i2][i1].

RCS (reading; the paper defers the formula to its reference [J91]): from (EGa2) the far
field is |E_s| = (k / (2 pi r)) |r^ x L|, L = (-E^2(u), E^1(u), 0), with the aperture
transforms E^l(u) = int_Gamma E_l(y, 0) e^{-i u.y} dy at u = k (r^_1, r^_2).  Hence for a
unit incident amplitude sigma_theta = (k^2/pi) |phi^.L|^2, sigma_phi = (k^2/pi) |theta^.L|^2
(units lambda^2).
"""
from __future__ import annotations

import numpy as np

from .columns import Columns
from .incident import cos_proj, sin_proj
from .problem import Problem
from .tbc import bases


def synthesize(prob: Problem, cols: Columns, e1, e2, e3, levels=None) -> np.ndarray:
    """E_out[3, Nz+1, Ny+1, Nx+1] from the aperture mode values (padded mode grids); with
    `levels` (a list of z-nodes) only those levels, E_out[3, len(levels), Ny+1, Nx+1]."""
    x1 = np.arange(prob.nx + 1) * prob.a / prob.nx
    x2 = np.arange(prob.ny + 1) * prob.b / prob.ny
    c1, s1, c2, s2 = bases(prob, x1, x2)
    mu, nu = prob.mu[:, None], prob.nu[None, :]
    js = list(range(prob.nz + 1)) if levels is None else list(levels)
    out = np.zeros((3, len(js), prob.ny + 1, prob.nx + 1), dtype=complex)
    for o, j in enumerate(js):
        k1 = cols.pi_d[j] * e1 + mu * cols.theta_d[j] * e3
        k2 = cols.pi_d[j] * e2 + nu * cols.theta_d[j] * e3
        k3 = cols.pi_n[j] * e3
        out[0, o] = (c1.T @ k1 @ s2).T
        out[1, o] = (s1.T @ k2 @ c2).T
        out[2, o] = (s1.T @ k3 @ s2).T
    return out


def aperture_transform(prob: Problem, e1, e2, u1: float, u2: float):
    """E^1(u), E^2(u): transforms of the aperture series, closed-form 1D factors."""
    mu, nu = prob.mu, prob.nu
    f1 = np.outer(cos_proj(-u1, mu, prob.a), sin_proj(-u2, nu, prob.b))
    f2 = np.outer(sin_proj(-u1, mu, prob.a), cos_proj(-u2, nu, prob.b))
    return np.sum(e1 * f1), np.sum(e2 * f2)


def rcs(prob: Problem, e1, e2, theta_o: float, phi_o: float):
    """(sigma_theta, sigma_phi) in lambda^2 at the observation direction."""
    st, ct, sp_, cp = np.sin(theta_o), np.cos(theta_o), np.sin(phi_o), np.cos(phi_o)
    k = prob.k
    u1, u2 = k * st * cp, k * st * sp_
    h1, h2 = aperture_transform(prob, e1, e2, u1, u2)
    L = np.array([-h2, h1, 0.0])
    theta_hat = np.array([ct * cp, ct * sp_, -st])
    phi_hat = np.array([-sp_, cp, 0.0])
    s_theta = k ** 2 / np.pi * abs(phi_hat @ L) ** 2
    s_phi = k ** 2 / np.pi * abs(theta_hat @ L) ** 2
    return float(s_theta), float(s_phi)
