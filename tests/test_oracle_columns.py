"""Pins of the oracle's per-mode z-elimination (Sections 3-4 of the paper).

* Homogeneous cavity: closed-form discrete exponential solutions of the second-order
  difference equation (Dirichlet bottom for E1/E2, Neumann bottom E3_0 = E3_1 for E3).
* Layered cavity: the vectorised elimination against a dense solve of each mode's column
  assembled row by row, and against the paper's own two-layer formulas (con43)-(con63),
  A3, A4, d_l, s_l, (u31T1), (uTT1) evaluated with explicit LU factorisations.
"""
import numpy as np
import pytest

import workloads as W
from oracle import columns
from oracle.problem import Problem


def _roots(h, lam):
    """r with |r| <= 1 and r + 1/r = 2 - h^2 lam."""
    d = 2.0 - h * h * lam
    r = 0.5 * (d + np.sqrt(d * d - 4.0 + 0j))
    return np.where(np.abs(r) > 1.0, 1.0 / r, r)


def _homog(eps, nz=12, nx=12, ny=10, a=1.3, b=0.9, c=0.45):
    cav = W.Cavity(a, b, c, nx, ny, nz, (nz,), (eps,))
    return Problem.from_cavity(cav)


@pytest.mark.parametrize("eps", [1.0 + 0j, 4.0 + 1.0j, 2.5 + 0.01j])
def test_homogeneous_closed_forms(eps):
    prob = _homog(eps)
    cols = columns.eliminate(prob)
    lam = prob.lam(0)
    r = _roots(prob.h, lam)
    nz = prob.nz
    j = np.arange(nz + 1)[:, None, None]
    # Dirichlet: E_j ~ r^j - r^-j  =>  Pi_j = r^(Nz-j) (1 - r^(2j)) / (1 - r^(2Nz))
    pi_d = r ** (nz - j) * (1 - r ** (2 * j)) / (1 - r ** (2 * nz))
    # Neumann: E_j ~ r^(j-1/2) + r^-(j-1/2)
    pi_n = r ** (nz - j) * (1 + r ** (2 * j - 1)) / (1 + r ** (2 * nz - 1))
    _, _, n3 = prob.masks()
    ok = np.ones_like(n3)
    ok[0, 0] = False
    scale = np.abs(pi_d).max()
    assert np.abs(cols.pi_d[:, ok] - pi_d[:, ok]).max() <= 1e-13 * scale
    rel = np.abs(cols.rho_d[ok] - pi_d[nz - 1][ok]) / np.maximum(1, np.abs(pi_d[nz - 1][ok]))
    assert rel.max() <= 1e-13
    assert np.abs(cols.pi_n[:, n3] - pi_n[:, n3]).max() <= 1e-13 * np.abs(pi_n).max()
    rel = np.abs(cols.rho_n[n3] - pi_n[nz - 1][n3]) / np.maximum(1, np.abs(pi_n[nz - 1][n3]))
    assert rel.max() <= 1e-13
    # homogeneous: no interface source
    assert np.abs(cols.T).max() == 0.0 and np.abs(cols.theta_d).max() == 0.0


def test_homogeneous_continuum_limit():
    """Second-order convergence of rho to the ODE solution ratio E(-h)/E(0)."""
    errs = []
    for nz in (16, 32, 64):
        prob = _homog(1.0 + 0j, nz=nz, c=0.5)
        cols = columns.eliminate(prob)
        m, n = 1, 2
        lam = prob.lam(0)[m, n]
        g = np.sqrt(lam + 0j)
        z = -prob.h
        exact_d = np.sin(g * (z + prob.c)) / np.sin(g * prob.c)
        errs.append(abs(cols.pi_d[nz - 1, m, n] - exact_d))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


@pytest.mark.parametrize("case", [1, 2, 3])
def test_layered_against_dense_columns(case):
    wl = W.small_cases()[case]
    prob = Problem.from_cavity(wl.cavity)
    cols = columns.eliminate(prob)
    rng = np.random.default_rng(7 + case)
    modes = [(0, 3), (2, 0), (1, 1), (prob.M, prob.N), (prob.M // 2, 1)]
    modes += [(int(rng.integers(1, prob.M + 1)), int(rng.integers(1, prob.N + 1)))
              for _ in range(4)]
    for (m, n) in modes:
        if m >= 1 and n >= 1:
            up, lo = columns.dense_e3_column(prob, m, n, 1.0)
            assert np.allclose(cols.pi_n[:, m, n], up, rtol=0, atol=1e-13 * np.abs(up).max())
        for comp in (1, 2):
            if (comp == 1 and n == 0) or (comp == 2 and m == 0):
                continue
            fac = prob.mu[m] if comp == 1 else prob.nu[n]
            e_only = columns.dense_tangential_column(prob, m, n, comp, 1.0, 0.0)
            e3_only = columns.dense_tangential_column(prob, m, n, comp, 0.0, 1.0)
            sc = max(np.abs(e_only).max(), 1.0)
            assert np.abs(cols.pi_d[:, m, n] - e_only).max() <= 1e-13 * sc
            assert np.abs(fac * cols.theta_d[:, m, n] - e3_only).max() <= 1e-13 * sc
            # Schur data: E_{Nz-1} = rho E + tau E3
            assert abs(cols.rho_d[m, n] - e_only[prob.nz - 1]) <= 1e-13 * sc
            assert abs(fac * cols.T[m, n] - e3_only[prob.nz - 1]) <= 1e-13 * sc


def _lu_nopivot(A):
    n = A.shape[0]
    L = np.eye(n, dtype=complex)
    U = A.astype(complex).copy()
    for k in range(n - 1):
        for i in range(k + 1, n):
            L[i, k] = U[i, k] / U[k, k]
            U[i, :] -= L[i, k] * U[k, :]
    return L, U


def _tridiag(n, first, diag):
    A = np.diag(np.full(n, diag, dtype=complex)) + np.diag(np.ones(n - 1), 1) + np.diag(
        np.ones(n - 1), -1)
    A[0, 0] = first
    return A


@pytest.mark.parametrize("layers", [((5, 7), (3.0 + 0.05j, 7.0 + 1.5j)),
                                    ((8, 4), (4.0 + 1.0j, 1.0 + 0j)),
                                    ((3, 9), (1.0 + 0j, 2.0 + 0.3j))])
def test_two_layer_paper_formulas(layers):
    """rho_1, tau_1, rho_3 of the top layer from the paper's two-layer derivation."""
    nzs, eps = layers
    cav = W.Cavity(1.0, 1.2, 0.6, 10, 12, sum(nzs), nzs, eps)
    prob = Problem.from_cavity(cav)
    cols = columns.eliminate(prob)
    h = prob.h
    J, I = nzs[0] - 1, nzs[1] - 1   # unknowns below / above the interface
    eps2, eps1 = eps[0], eps[1]     # paper: 2 = bottom layer, 1 = top layer
    for (m, n) in [(1, 1), (2, 3), (5, 1), (9, 11), (3, 7)]:
        lam2 = prob.kappa2(0) - prob.mu[m] ** 2 - prob.nu[n] ** 2
        lam1 = prob.kappa2(1) - prob.mu[m] ** 2 - prob.nu[n] ** 2
        # bottom layer (dfv1M), (dfv3M), (LUd21), (LUd22) -> r_1(JJ), r_2(JJ)
        _, U1 = _lu_nopivot(_tridiag(J, -2 + h * h * lam2, -2 + h * h * lam2))
        _, U2 = _lu_nopivot(_tridiag(J, -1 + h * h * lam2, -2 + h * h * lam2))
        r1, r2 = U1[-1, -1], U2[-1, -1]
        ratio = eps1 / eps2
        # top layer E3: A4 (first diagonal from (con63)), (LUd13), (u31T1)
        first4 = 1.0 / ((1.0 / r2 + 1.0) * ratio + 1.0) - 2 + h * h * lam1
        _, U4 = _lu_nopivot(_tridiag(I, first4, -2 + h * h * lam1))
        r4 = U4[-1, -1]
        detU4 = np.prod(np.diag(U4))
        # top layer E1: A3 (first diagonal from (con43)), d_1, (LUd11), s_1
        first3 = 1.0 / (1.0 / r1 + 2.0) - 2 + h * h * lam1
        L3, U3 = _lu_nopivot(_tridiag(I, first3, -2 + h * h * lam1))
        r3 = U3[-1, -1]
        l_I1 = np.linalg.inv(L3)[-1, 0]
        d1 = ((ratio - 1.0) * prob.mu[m] * h / (1.0 / r1 + 2.0)) \
            * (1.0 / ((1.0 / r2 + 1.0) * ratio + 1.0)) * ((-1.0) ** (2 + I) / detU4)
        s1 = -l_I1 * d1
        # (uTT1): r3 u_I + u_{I+1} = s1 u3_{I+1};  r4 u3_I + u3_{I+1} = 0
        rho1, tau1, rho3 = -1.0 / r3, s1 / r3, -1.0 / r4
        assert abs(cols.rho_d[m, n] - rho1) <= 1e-12 * max(1, abs(rho1))
        assert abs(prob.mu[m] * cols.T[m, n] - tau1) <= 1e-12 * max(1, abs(tau1))
        assert abs(cols.rho_n[m, n] - rho3) <= 1e-12 * max(1, abs(rho3))
