"""Pins of field synthesis, the 2D trigonometric transforms and the RCS.

* The cos/sin synthesis on the grid nodes equals SciPy's DCT-I / DST-I (an independent
  FFT-based routine), and DCT-I / DST-I on N+1 nodes invert exactly (round trip).
* The closed-form aperture transform used for the RCS equals a brute-force 2D
  Gauss-Legendre quadrature of the synthesised aperture series.
* The synthesised field obeys the bottom conditions (E1 = E2 = 0, dE3/dz = 0 discretely)
  and reproduces the aperture values at the top node.
"""
import numpy as np
import pytest
import scipy.fft as sfft

import workloads as W
from oracle import fields, solver
from oracle.problem import Problem
from oracle.tbc import bases


def test_dct_dst_match_scipy_and_round_trip():
    rng = np.random.default_rng(3)
    nx = 24
    x = np.arange(nx + 1) / nx
    prob = Problem.from_cavity(W.Cavity(1.0, 1.0, 0.2, nx, nx, 2, (2,), (1 + 0j,)))
    c1, s1, _, _ = bases(prob, x, x)
    coef = rng.standard_normal(nx) + 1j * rng.standard_normal(nx)   # m = 0..Nx-1
    # DCT-I on Nx+1 points: y_i = sum_m c_m cos(pi m i/Nx) with the last mode c_Nx = 0
    full = np.concatenate([coef, [0.0]])
    w = full.copy()
    w[0] *= 2.0
    w[-1] *= 2.0
    ref = 0.5 * sfft.dct(w, type=1)
    assert np.abs(c1.T @ coef - ref).max() <= 1e-13 * np.abs(ref).max()
    # DST-I on the Nx-1 interior points for m = 1..Nx-1
    ref_s = 0.5 * sfft.dst(coef[1:], type=1)
    assert np.abs((s1.T @ coef)[1:-1] - ref_s).max() <= 1e-13 * np.abs(ref_s).max()
    # round trips with the trapezoid-weighted projections
    tw = np.ones(nx + 1)
    tw[0] = tw[-1] = 0.5
    back_c = (2.0 / nx) * (c1 * tw[None, :]) @ (c1.T @ coef)
    back_c[0] *= 0.5
    assert np.abs(back_c - coef).max() <= 1e-13 * np.abs(coef).max()
    back_s = (2.0 / nx) * s1 @ (s1.T @ coef)
    assert np.abs(back_s[1:] - coef[1:]).max() <= 1e-13 * np.abs(coef).max()


def _solved(case=1):
    wl = W.small_cases()[case]
    prob = Problem.from_cavity(wl.cavity)
    pl = solver.plan(prob)
    inc = wl.incidences[0]
    sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, dense=True)
    return prob, pl, sol, inc


def test_rcs_closed_form_vs_quadrature():
    prob, pl, sol, inc = _solved(1)
    e1, e2, _ = sol.grids
    xg, wg = np.polynomial.legendre.leggauss(160)
    x1 = 0.5 * prob.a * (xg + 1)
    w1 = 0.5 * prob.a * wg
    x2 = 0.5 * prob.b * (xg + 1)
    w2 = 0.5 * prob.b * wg
    c1, s1, c2, s2 = bases(prob, x1, x2)
    f1 = c1.T @ e1 @ s2          # E1(x1, x2) on the Gauss grid
    f2 = s1.T @ e2 @ c2
    for (u1, u2) in [(0.3, -1.1), (4.0, 2.5), (-6.0, 0.0)]:
        ph = np.exp(-1j * u1 * x1)[:, None] * np.exp(-1j * u2 * x2)[None, :]
        q1 = np.sum(w1[:, None] * w2[None, :] * f1 * ph)
        q2 = np.sum(w1[:, None] * w2[None, :] * f2 * ph)
        t1, t2 = fields.aperture_transform(prob, e1, e2, u1, u2)
        assert abs(t1 - q1) <= 1e-12 * max(abs(q1), 1e-3)
        assert abs(t2 - q2) <= 1e-12 * max(abs(q2), 1e-3)
    st, sp = fields.rcs(prob, e1, e2, inc.theta, inc.phi)
    assert st >= 0 and sp >= 0 and st + sp > 0


def test_synthesis_boundary_and_top():
    prob, pl, sol, inc = _solved(3)
    out = solver.field_out(pl, sol)
    assert out.shape == (3, prob.nz + 1, prob.ny + 1, prob.nx + 1)
    scale = np.abs(out).max()
    assert np.abs(out[0, 0]).max() <= 1e-14 * scale
    assert np.abs(out[1, 0]).max() <= 1e-14 * scale
    # Neumann bottom E3_0 = E3_1 seen from the bottom layer (node 1 is an interface here:
    # the lower-side value is (eps_up / eps_lo) times the reported upper-side value)
    assert prob.layer_nz[0] == 1
    ratio = prob.layer_eps[1] / prob.layer_eps[0]
    assert np.abs(out[2, 0] - ratio * out[2, 1]).max() <= 1e-13 * scale
    # PEC side walls: tangential components vanish on x1 = 0, a (E2, E3) and x2 = 0, b (E1, E3)
    assert np.abs(out[1][:, :, [0, -1]]).max() <= 1e-13 * scale
    assert np.abs(out[2][:, :, [0, -1]]).max() <= 1e-13 * scale
    assert np.abs(out[0][:, [0, -1], :]).max() <= 1e-13 * scale
    # top node equals the aperture series
    x1 = np.arange(prob.nx + 1) * prob.a / prob.nx
    x2 = np.arange(prob.ny + 1) * prob.b / prob.ny
    c1, s1, c2, s2 = bases(prob, x1, x2)
    assert np.abs(out[0, -1] - (c1.T @ sol.grids[0] @ s2).T).max() <= 1e-13 * scale
