"""Pins of the reduced aperture system and of the whole oracle solve.

* Brute force: the full discrete system (every z-level of every mode, interface rows and
  the three aperture rows with dense S^f) solved by sparse LU equals the reduced path
  (elimination + reduced system + back-substitution) at every level.
* GMRES (right-preconditioned) reaches the dense LU solution of the reduced system.
* Energy balance (fixes the TBC sign and the RCS normalisation): for a lossless cavity the
  power radiated by the scattered field (hemisphere integral of the far field) cancels the
  interference term Re int (E_s x conj(H_0)).z over the aperture, up to the discretisation
  error of the TBC; a lossy cavity absorbs power.
* Mirror symmetry at phi = 0: theta-hat incidence excites only odd n, phi-hat only even n.
* Square aperture at normal incidence: the two co-polarised backscatter RCS coincide.
"""
import numpy as np
import pytest

import workloads as W
from oracle import columns, fields, incident, solver, system
from oracle.problem import Problem


def _prob(wl):
    return Problem.from_cavity(wl.cavity)


@pytest.mark.parametrize("case", [0, 1, 3, 5, 6])
def test_brute_force_full_system(case):
    wl = W.small_cases()[case]
    prob = _prob(wl)
    pl = solver.plan(prob)
    inc = wl.incidences[0]
    g1, g2 = incident.rhs(prob, inc.theta, inc.phi, inc.pol)
    full, A, b, x = system.solve_full(prob, pl.khat, g1, g2)
    sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
    e1, e2, e3 = sol.grids
    scale = max(np.abs(e1).max(), np.abs(e2).max(), np.abs(e3).max())
    c = pl.cols
    mu, nu = prob.mu[:, None], prob.nu[None, :]
    for j in range(1, prob.nz + 1):
        k1 = c.pi_d[j] * e1 + mu * c.theta_d[j] * e3
        k2 = c.pi_d[j] * e2 + nu * c.theta_d[j] * e3
        k3 = c.pi_n[j] * e3
        for got, ref, msk in ((k1, full[0][j], prob.masks()[0]), (k2, full[1][j], prob.masks()[1]),
                              (k3, full[2][j], prob.masks()[2])):
            assert np.abs(got[msk] - ref[msk]).max() <= 1e-12 * scale
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("case", [0, 1, 3])
def test_gmres_reaches_dense_solution(case):
    wl = W.small_cases()[case]
    prob = _prob(wl)
    pl = solver.plan(prob)
    for inc in wl.incidences:
        d = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
        g = solver.solve(pl, inc.theta, inc.phi, inc.pol, tol=1e-13)
        assert g.rel_residual <= 1e-13
        assert g.iterations < 60
        assert np.linalg.norm(g.x - d.x) <= 1e-11 * np.linalg.norm(d.x)


def aperture_power(prob, sol, theta, phi, pol):
    """(interference term, radiated power) in units eps0 = mu0 = 1, omega = k."""
    e1, e2, _ = sol.grids
    a1, a2, beta, p = incident.plane_wave(prob.k, theta, phi, pol)
    q = np.array([a1, a2, -beta])
    h0 = 2.0 / prob.k * np.cross(q, p)       # tangential H of incident + reflected at z = 0
    f1, f2 = fields.aperture_transform(prob, e1, e2, a1, a2)
    interference = 0.5 * np.real(f1 * np.conj(h0[1]) - f2 * np.conj(h0[0]))
    xg, wg = np.polynomial.legendre.leggauss(40)
    th = 0.25 * np.pi * (xg + 1)
    wth = 0.25 * np.pi * wg
    nph = 80
    total = 0.0
    for t, w in zip(th, wth):
        st, ct = np.sin(t), np.cos(t)
        for f in np.arange(nph) * 2 * np.pi / nph:
            sf, cf = np.sin(f), np.cos(f)
            t1, t2 = fields.aperture_transform(prob, e1, e2, prob.k * st * cf, prob.k * st * sf)
            L = np.array([-t2, t1, 0.0])
            r = np.array([st * cf, st * sf, ct])
            total += w * (2 * np.pi / nph) * st * np.linalg.norm(np.cross(r, L)) ** 2
    radiated = 0.5 * prob.k ** 2 / (4 * np.pi ** 2) * total
    return interference, radiated


@pytest.mark.slow
def test_energy_balance():
    lossless = [W.vacuum_1x1x05(),
                W.Workload("v", W.Cavity(1.0, 0.7, 0.3, 32, 24, 12, (12,), (1 + 0j,)),
                           (W.Incidence(0.6, 0.3, W.TM),))]
    for wl in lossless:
        prob = _prob(wl)
        pl = solver.plan(prob)
        inc = wl.incidences[0]
        sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
        inter, rad = aperture_power(prob, sol, inc.theta, inc.phi, inc.pol)
        assert rad > 0
        assert abs(inter + rad) <= 0.05 * rad, (inter, rad)
    wl = W.small_cases()[1]            # lossy bottom layer: absorbed power > 0
    prob = _prob(wl)
    pl = solver.plan(prob)
    inc = wl.incidences[0]
    sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
    inter, rad = aperture_power(prob, sol, inc.theta, inc.phi, inc.pol)
    assert -(inter + rad) > 0.01 * rad


@pytest.mark.parametrize("pol", [W.TM, W.TE])
def test_mirror_symmetry_phi0(pol):
    wl = W.small_cases()[2]
    prob = _prob(wl)
    pl = solver.plan(prob)
    sol = solver.solve(pl, 0.7, 0.0, pol, tol=1e-14)
    scale = max(np.abs(g).max() for g in sol.grids)
    zero_n = slice(0, None, 2) if pol == W.TM else slice(1, None, 2)
    for g in sol.grids:
        assert np.abs(g[:, zero_n]).max() <= 1e-12 * scale


def test_square_normal_incidence_tm_equals_te():
    wl = W.vacuum_1x1x05()
    prob = _prob(wl)
    pl = solver.plan(prob)
    s_tm = solver.solve(pl, 0.0, 0.0, W.TM, dense=True)
    s_te = solver.solve(pl, 0.0, 0.0, W.TE, dense=True)
    tt = solver.backscatter(pl, s_tm, 0.0, 0.0)[0]
    pp = solver.backscatter(pl, s_te, 0.0, 0.0)[1]
    assert abs(tt - pp) <= 1e-12 * tt


def test_resonance_guard_reports_small_pivot():
    """A real-eps geometry tuned to an exact discrete resonance drives the pivot to zero."""
    # Dirichlet column mode (m, n) with h^2 lam = 2 - 2 cos(p pi / Nz): E_j = sin(p pi j/Nz)
    a = b = 1.0
    nz, c = 8, 0.5
    h = c / nz
    m, n, p = 1, 1, 3
    lam = (2 - 2 * np.cos(p * np.pi / nz)) / h ** 2
    eps = (lam + (m * np.pi / a) ** 2 + (n * np.pi / b) ** 2) / (2 * np.pi) ** 2
    prob = Problem.from_cavity(W.Cavity(a, b, c, 6, 6, nz, (nz,), (complex(eps),)))
    cols = columns.eliminate(prob)
    assert cols.min_pivot < 1e-12


def test_divergence_free_interior():
    """Section 3 remark: the field is divergence free in the cavity.  The discrete
    divergence -mu E1 - nu E2 + (E3_j - E3_{j-1})/h of the resolved (low) modes must vanish
    at first order in h; a TBC third row without its h factor leaves an O(1) divergence."""
    worst = []
    for nz in (12, 24, 48):
        wl = W.Workload("v", W.Cavity(1.0, 0.7, 0.3, 32, 24, nz, (nz,), (1 + 0j,)),
                        (W.Incidence(0.6, 0.3, W.TM),))
        prob = _prob(wl)
        pl = solver.plan(prob)
        sol = solver.solve(pl, 0.6, 0.3, W.TM, tol=1e-13)
        e1, e2, e3 = sol.grids
        c = pl.cols
        mu, nu, h = prob.mu[:, None], prob.nu[None, :], prob.h
        low = prob.masks()[2].copy()
        low[prob.M // 4:, :] = False
        low[:, prob.N // 4:] = False
        ref = (np.abs(mu * e1) + np.abs(nu * e2))[low].max()
        w = 0.0
        for j in range(2, prob.nz + 1):
            d = -mu * (c.pi_d[j] * e1) - nu * (c.pi_d[j] * e2) + (c.pi_n[j] - c.pi_n[j - 1]) * e3 / h
            w = max(w, np.abs(d[low]).max() / ref)
        worst.append(w)
    assert worst[-1] < 0.02 and worst[0] / worst[-1] > 3.0, worst


def _direct_sum(prob, grid, comp):
    """Field of one component on the nodes from its mode values by the plain double sum
    of (E123F): cos(mu x) sin(nu y), sin(mu x) cos(nu y) or sin(mu x) sin(nu y)."""
    x1 = np.arange(prob.nx + 1) * prob.a / prob.nx
    x2 = np.arange(prob.ny + 1) * prob.b / prob.ny
    f1 = np.cos if comp == 0 else np.sin
    f2 = np.cos if comp == 1 else np.sin
    out = np.zeros((prob.ny + 1, prob.nx + 1), dtype=complex)
    for m in range(prob.M + 1):
        for n in range(prob.N + 1):
            if grid[m, n] != 0:
                out += grid[m, n] * np.outer(f2(prob.nu[n] * x2), f1(prob.mu[m] * x1))
    return out


@pytest.mark.parametrize("case", [1, 3, 4])
def test_field_synthesis_against_full_system(case):
    """fields.synthesize (through solver.field_out) at every z-level equals the full
    discrete system's mode values summed on the nodes.  The layered cases have nonzero
    Theta, so the mu / nu factors of its E3 term in E1 and E2 are exercised (the grids
    are not square, so a swap changes the result); E3 at an interface is the upper-side
    value and E3 at node 0 the bottom value of the full system."""
    wl = W.small_cases()[case]
    prob = _prob(wl)
    pl = solver.plan(prob)
    assert np.abs(pl.cols.theta_d).max() > 0.0
    inc = wl.incidences[0]
    g1, g2 = incident.rhs(prob, inc.theta, inc.phi, inc.pol)
    full, _, _, _ = system.solve_full(prob, pl.khat, g1, g2)
    sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
    got = solver.field_out(pl, sol)
    assert got.shape == (3, prob.nz + 1, prob.ny + 1, prob.nx + 1)
    scale = np.abs(got).max()
    for comp in range(3):
        for j in range(prob.nz + 1):
            ref = _direct_sum(prob, full[comp][j], comp)
            assert np.abs(got[comp, j] - ref).max() <= 1e-11 * scale, (comp, j)
