"""Pins of layers with their own grid steps in the oracle (a reading beyond Section 4).

The paper's layered derivation (Section 4) uses one step h.  Here each layer may have
its own step h_l = d_l / Nz_l; the one-sided differences of the interface conditions
keep the step of the layer they lie in.  Pinned by:
* thicknesses proportional to the interval counts reproduce the common-step result;
* the vectorised elimination against dense per-mode columns assembled row by row;
* convergence, as both steps shrink, to the continuum two-layer profiles: closed forms
  of the layer ODEs of Section 4 (E'' + lambda_l E = 0 per layer) with Dirichlet
  (E1, E2) or Neumann (E3) bottom, eps_up E3^+ = eps_lo E3^-, continuous E1, E2 and
  dE3/dz, and the jump dE1/dz^+ - dE1/dz^- = mu_m (E3^+ - E3^-) of the tangential curl;
* the full discrete system against the reduced solve, and the aperture rows' step (the
  top layer's) through a cavity split into two layers of one permittivity.
"""
import numpy as np
import pytest

import workloads as W
from oracle import columns, incident, solver, system
from oracle.problem import Problem

K = 2 * np.pi


def _two_layer(n_lo, n_up, d_lo=0.36, d_up=0.25, eps=(4.0 + 1.0j, 1.0 + 0j), nx=4, ny=4):
    return Problem(1.0, 1.0, d_lo + d_up, nx, ny, n_lo + n_up, (n_lo, n_up), eps, K,
                   layer_depth=(d_lo, d_up))


def _continuum(prob, m, n):
    """Continuum profiles at the nodes: Pi (E1, top value 1), Theta (E1 / mu_m for top
    E1 = 0, top E3 = 1) and Pi3 (E3 upper side, top value 1)."""
    d_lo, d_up = prob.layer_depth
    e_lo, e_up = prob.layer_eps
    g_lo, g_up = np.sqrt(prob.lam(0)[m, n] + 0j), np.sqrt(prob.lam(1)[m, n] + 0j)
    z = prob.z_nodes()
    low = z <= d_lo + 1e-12
    t = z - d_lo
    cu, su = np.cos(g_up * t), np.sin(g_up * t) / g_up

    # E3: A cos(g_lo z) below; E3^+ = (eps_lo / eps_up) E3^-, slope continuous
    e3m, s3 = np.cos(g_lo * d_lo), -g_lo * np.sin(g_lo * d_lo)
    e3p = e3m * e_lo / e_up
    up3 = e3p * cu + s3 * su
    pi3 = np.where(low, np.cos(g_lo * z), up3)
    top = up3[-1]
    pi3 = pi3 / top
    pi3[np.isclose(z, d_lo)] = e3p / top            # interface node: upper side
    jump = (e3p - e3m) / top                          # E3^+ - E3^- for top value 1

    # E1 with top value 1 and no E3: A sin(g_lo z), value and slope continuous
    es, sl = np.sin(g_lo * d_lo), g_lo * np.cos(g_lo * d_lo)
    up1 = es * cu + sl * su
    pi = np.where(low, np.sin(g_lo * z), up1) / up1[-1]

    # E1 with top value 0 and top E3 = 1: slope jumps by mu_m (E3^+ - E3^-)
    mu = prob.mu[m]
    a = -mu * jump * su[-1] / up1[-1]
    th = np.where(low, a * np.sin(g_lo * z), a * up1 + mu * jump * su) / mu
    return pi, th, pi3


def test_proportional_thickness_matches_common_step():
    wl = W.small_cases()[2]
    cav = wl.cavity
    base = Problem.from_cavity(cav)
    d = tuple(cav.c * nl / cav.nz for nl in cav.layer_nz)
    given = Problem(cav.a, cav.b, cav.c, cav.nx, cav.ny, cav.nz, tuple(cav.layer_nz),
                    tuple(cav.layer_eps), cav.k, cav.tbc_oversample, layer_depth=d)
    c0, c1 = columns.eliminate(base), columns.eliminate(given)
    for f in ("rho_d", "T", "rho_n", "pi_d", "theta_d", "pi_n"):
        x, y = getattr(c0, f), getattr(c1, f)
        assert np.abs(x - y).max() <= 1e-14 * max(np.abs(x).max(), 1.0), f


def test_invalid_thickness_rejected():
    with pytest.raises(ValueError):
        _two_layer(4, 8, d_lo=0.36, d_up=-0.25)
    with pytest.raises(ValueError):
        Problem(1.0, 1.0, 0.7, 4, 4, 12, (4, 8), (4.0, 1.0), K, layer_depth=(0.36, 0.25))


@pytest.mark.parametrize("eps", [(4.0 + 1.0j, 1.0 + 0j, 2.5 + 0.2j),
                                 (1.0 + 0j, 7.0 + 1.5j, 3.0 + 0j)])
def test_elimination_against_dense_columns(eps):
    # three layers, three steps (the second interface also carries the first's source)
    prob = Problem(1.0, 1.0, 0.61, 6, 5, 18, (5, 9, 4), eps, K, layer_depth=(0.36, 0.1, 0.15))
    assert len(set(prob.layer_h)) == 3
    cols = columns.eliminate(prob)
    for (m, n) in [(0, 2), (3, 0), (1, 1), (prob.M, prob.N), (2, 3)]:
        if m >= 1 and n >= 1:
            up, _ = columns.dense_e3_column(prob, m, n, 1.0)
            assert np.abs(cols.pi_n[:, m, n] - up).max() <= 1e-13 * np.abs(up).max()
        for comp in (1, 2):
            if (comp == 1 and n == 0) or (comp == 2 and m == 0):
                continue
            fac = prob.mu[m] if comp == 1 else prob.nu[n]
            e_only = columns.dense_tangential_column(prob, m, n, comp, 1.0, 0.0)
            e3_only = columns.dense_tangential_column(prob, m, n, comp, 0.0, 1.0)
            sc = max(np.abs(e_only).max(), 1.0)
            assert np.abs(cols.pi_d[:, m, n] - e_only).max() <= 1e-13 * sc
            assert np.abs(fac * cols.theta_d[:, m, n] - e3_only).max() <= 1e-13 * sc


@pytest.mark.parametrize("eps", [(4.0 + 1.0j, 1.0 + 0j), (2.0 + 0.1j, 6.0 + 0.5j)])
def test_continuum_limit_of_two_layer_profiles(eps):
    """Errors against the continuum profiles fall like h under refinement of both
    layers (steps 0.09 / 2^k below, 0.03125 / 2^k above; the interface rows are first
    order, as with the common step)."""
    errs = []
    for r in (1, 2, 4, 8, 16):
        prob = _two_layer(4 * r, 8 * r, eps=eps)
        cols = columns.eliminate(prob)
        e = 0.0
        for (m, n) in [(1, 1), (2, 1), (1, 3)]:
            pi, th, pi3 = _continuum(prob, m, n)
            e = max(e, np.abs(cols.pi_d[:, m, n] - pi).max() / np.abs(pi).max(),
                    np.abs(cols.theta_d[:, m, n] - th).max() / np.abs(th).max(),
                    np.abs(cols.pi_n[:, m, n] - pi3).max() / np.abs(pi3).max())
        errs.append(e)
    errs = np.array(errs)
    ratios = errs[1:] / errs[:-1]
    assert np.all(ratios < 0.7) and np.all(ratios[-2:] < 0.56), errs
    assert errs[-1] < 0.1, errs


def test_full_system_matches_reduced_solve():
    wl = W.small_cases()[4]
    prob = Problem.from_cavity(wl.cavity)
    assert prob.layer_h[0] != prob.layer_h[1]
    pl = solver.plan(prob)
    inc = wl.incidences[0]
    g1, g2 = incident.rhs(prob, inc.theta, inc.phi, inc.pol)
    full, A, b, x = system.solve_full(prob, pl.khat, g1, g2)
    sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
    e1, e2, e3 = sol.grids
    scale = max(np.abs(e1).max(), np.abs(e2).max(), np.abs(e3).max())
    c = pl.cols
    mu, nu = prob.mu[:, None], prob.nu[None, :]
    n1, n2, n3 = prob.masks()
    for j in range(1, prob.nz + 1):
        k1 = c.pi_d[j] * e1 + mu * c.theta_d[j] * e3
        k2 = c.pi_d[j] * e2 + nu * c.theta_d[j] * e3
        k3 = c.pi_n[j] * e3
        for got, ref, msk in ((k1, full[0][j], n1), (k2, full[1][j], n2), (k3, full[2][j], n3)):
            assert np.abs(got[msk] - ref[msk]).max() <= 1e-12 * scale
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_split_layer_converges_to_homogeneous_cavity():
    """One permittivity split into a coarse lower and a fine upper layer: the aperture
    solution approaches the single-layer one as the steps shrink (the aperture rows
    must use the top layer's step for this limit to hold)."""
    a, b, c, nx, ny = 1.0, 0.8, 0.4, 6, 5
    eps = 2.0 + 0.5j
    th, ph, pol = 0.5, 0.7, 0

    def aperture(n_lo, n_up, depth):
        prob = Problem(a, b, c, nx, ny, n_lo + n_up, (n_lo, n_up), (eps, eps), K,
                       layer_depth=depth)
        return solver.solve(solver.plan(prob), th, ph, pol, dense=True).x

    ref = aperture(96, 96, None)      # common fine step
    errs = [np.linalg.norm(aperture(2 * r, 6 * r, (0.24, 0.16)) - ref) / np.linalg.norm(ref)
            for r in (1, 2, 4)]
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs
