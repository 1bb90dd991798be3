"""Per-mode z-columns: finite differences, bottom conditions, interface rows (oracle).

Paper: Section 3 (ODEs (ode1x3), (ode3x3); second-order differences and the bottom
conditions E_{1,0} = E_{2,0} = 0, E_{3,1} = E_{3,0}; matrices A1, A2, D^(m,n) in (dfE1M),
(dfE3M); LU elimination (LU1)-(EJJ1) giving r_JJ E_J + E_{J+1} = 0), Section 4 (layer ODEs
(odev1), (odev3), (odeu1); interface conditions (con11)-(con61) and their one-sided
discrete forms (con12)-(con63); the remark on more than two layers).

For one Fourier mode (m, n) the column unknowns are the values at nodes 1..Nz-1 (the
aperture value at node Nz is given).  E3 is two-valued at an interface node s: the lower
side E3^-_s and the upper side E3^+_s with eps_up E3^+_s = eps_lo E3^-_s (con32), and the
derivative continuity E3_{s+1} - E3^+_s = E3^-_s - E3_{s-1} (con61 discretised).  E1, E2
are single-valued; at an interface the tangential-curl continuity (con41), (con51) gives
    E1_{s-1} - 2 E1_s + E1_{s+1} = mu_m h (E3^+_s - E3^-_s)     (nu_n h for E2),
with zero right side when the mode has no E3 partner (m = 0 or n = 0).

Layers with their own steps (reading, beyond the paper's common h): the one-sided
differences keep their own steps, h_lo below and h_up above the interface.  With
q = h_up / h_lo the two interface rows become
    E3_{s+1} - E3^+_s = q (E3^-_s - E3_{s-1}),
    q E1_{s-1} - (1 + q) E1_s + E1_{s+1} = mu_m h_up (E3^+_s - E3^-_s),
(the derivative rows multiplied by h_up), which are the rows above when q = 1; interior
rows of layer l use h_l.

The eliminated quantities (reading: the paper's r_JJ relation, generalised to layers) are
    E_{l,Nz-1} = rho_l E_{l,Nz} + tau_l E_{3,Nz},     E_{3,Nz-1} = rho_3 E_{3,Nz},
and the profiles E_{l,j} = Pi_j E_{l,Nz} + (mu_m or nu_n) Theta_j E_{3,Nz},
E_{3,j} = Pi3_j E_{3,Nz}, with E3 at an interface reported on the upper side.

Two implementations, deliberately different:
* ``dense_column`` assembles one mode's column as a dense linear system from the rows
  above and solves it with numpy.linalg.solve (the plain definition; small sizes).
* ``eliminate`` runs Gaussian elimination bottom-up, vectorised over all modes, then the
  back-substitution top-down (the paper's LU route).  Tests pin it to ``dense_column``,
  to the homogeneous closed forms and to the paper's two-layer formulas.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .problem import Problem


# ----------------------------------------------------------------------------------------
# Dense, plain definition for one mode
# ----------------------------------------------------------------------------------------

def _e3_views(prob: Problem):
    """Variable bookkeeping for the two-valued E3 column.

    Returns (nvar, view) where view(ell, j) is the variable index of E3 at node j as seen
    from layer ell, or -1 for the given aperture value (node Nz)."""
    kinds = prob.node_kind()
    nz = prob.nz
    idx = {}
    nvar = 0
    for j in range(0, nz):
        idx[(j, "up")] = nvar  # node value; at an interface: the upper side
        nvar += 1
        if kinds[j][0] == "interface":
            idx[(j, "lo")] = nvar
            nvar += 1
    layer_top = np.cumsum(prob.layer_nz)
    layer_bot = layer_top - np.asarray(prob.layer_nz)

    def view(ell, j):
        if j == nz:
            return -1
        if kinds[j][0] == "interface" and j == layer_top[ell]:
            return idx[(j, "lo")]
        return idx[(j, "up")]

    return nvar, view, idx, layer_bot, layer_top


def dense_e3_column(prob: Problem, m: int, n: int, e3_top: complex = 1.0):
    """Solve the E3 column of mode (m, n) (m, n >= 1) densely for a given aperture value.

    Returns (upper-side values at nodes 0..Nz, lower-side values at interface nodes)."""
    kinds = prob.node_kind()
    nvar, view, idx, layer_bot, layer_top = _e3_views(prob)
    A = np.zeros((nvar, nvar), dtype=complex)
    rhs = np.zeros(nvar, dtype=complex)
    row = 0

    def put(r, ell, j, coef):
        v = view(ell, j)
        if v < 0:
            rhs[r] -= coef * e3_top
        else:
            A[r, v] += coef

    # bottom Neumann condition E3_0 = E3_1 (dfE3M), seen from layer 0
    put(row, 0, 0, 1.0)
    put(row, 0, 1, -1.0)
    row += 1
    for j in range(1, prob.nz):
        kd = kinds[j]
        if kd[0] == "interior":
            ell = kd[1]
            lam = prob.kappa2(ell) - prob.mu[m] ** 2 - prob.nu[n] ** 2
            put(row, ell, j - 1, 1.0)
            put(row, ell, j, -2.0 + prob.h_layer(ell) ** 2 * lam)
            put(row, ell, j + 1, 1.0)
            row += 1
        else:  # interface between layers lo and up
            lo, up = kd[1], kd[2]
            # eps_up E3^+ = eps_lo E3^-   (con32)
            A[row, idx[(j, "up")]] = prob.layer_eps[up]
            A[row, idx[(j, "lo")]] = -prob.layer_eps[lo]
            row += 1
            # E3_{j+1} - E3^+_j = q (E3^-_j - E3_{j-1})   (con61, one-sided differences)
            q = prob.h_layer(up) / prob.h_layer(lo)
            put(row, up, j + 1, 1.0)
            put(row, up, j, -1.0)
            put(row, lo, j, -q)
            put(row, lo, j - 1, q)
            row += 1
    assert row == nvar
    x = np.linalg.solve(A, rhs)
    upper = np.empty(prob.nz + 1, dtype=complex)
    for j in range(prob.nz):
        upper[j] = x[idx[(j, "up")]]
    upper[prob.nz] = e3_top
    lower = {j: x[idx[(j, "lo")]] for j in prob.interfaces}
    return upper, lower


def dense_tangential_column(prob: Problem, m: int, n: int, comp: int,
                            e_top: complex, e3_top: complex):
    """Solve the E1 (comp=1) or E2 (comp=2) column of mode (m, n) densely.

    Returns values at nodes 0..Nz (node 0 is the Dirichlet zero)."""
    kinds = prob.node_kind()
    nz = prob.nz
    coupled = m >= 1 and n >= 1
    if coupled:
        e3_up, e3_lo = dense_e3_column(prob, m, n, e3_top)
    factor = prob.mu[m] if comp == 1 else prob.nu[n]
    A = np.zeros((nz - 1, nz - 1), dtype=complex)
    rhs = np.zeros(nz - 1, dtype=complex)

    def put(r, j, coef):
        if j == 0:
            return  # E_0 = 0 (Dirichlet bottom)
        if j == nz:
            rhs[r] -= coef * e_top
        else:
            A[r, j - 1] += coef

    for j in range(1, nz):
        r = j - 1
        kd = kinds[j]
        if kd[0] == "interior":
            lam = prob.kappa2(kd[1]) - prob.mu[m] ** 2 - prob.nu[n] ** 2
            put(r, j - 1, 1.0)
            put(r, j, -2.0 + prob.h_layer(kd[1]) ** 2 * lam)
            put(r, j + 1, 1.0)
        else:
            h_up = prob.h_layer(kd[2])
            q = h_up / prob.h_layer(kd[1])
            put(r, j - 1, q)
            put(r, j, -1.0 - q)
            put(r, j + 1, 1.0)
            if coupled:
                rhs[r] += factor * h_up * (e3_up[j] - e3_lo[j])
    vals = np.zeros(nz + 1, dtype=complex)
    if nz > 1:
        vals[1:nz] = np.linalg.solve(A, rhs)
    vals[nz] = e_top
    return vals


# ----------------------------------------------------------------------------------------
# Gaussian elimination vectorised over modes (the paper's LU route, Sections 3-4)
# ----------------------------------------------------------------------------------------

@dataclass
class Columns:
    """Elimination results on the (M+1) x (N+1) mode grid.

    rho_d, T : Dirichlet (E1/E2) Schur data; tau_1 = mu_m T, tau_2 = nu_n T.
    rho_n    : Neumann (E3) Schur datum (meaningful on N3).
    pi_d, theta_d, pi_n : profiles at nodes 0..Nz, shape (Nz+1, M+1, N+1).
    min_pivot: smallest |pivot| met (resonance guard)."""
    rho_d: np.ndarray
    T: np.ndarray
    rho_n: np.ndarray
    pi_d: np.ndarray
    theta_d: np.ndarray
    pi_n: np.ndarray
    min_pivot: float


def eliminate(prob: Problem) -> Columns:
    kinds = prob.node_kind()
    nz = prob.nz
    shape = (prob.M + 1, prob.N + 1)
    _, _, n3 = prob.masks()
    min_piv = np.inf

    # E3, Neumann bottom: E3_0 = alpha_1 E3_1 with alpha_1 = 1.
    # alpha_j relates the two ends of interval [j-1, j] within its layer.
    alpha3 = np.zeros((nz + 1,) + shape, dtype=complex)
    alpha3[1] = 1.0
    for j in range(1, nz):
        kd = kinds[j]
        if kd[0] == "interior":
            piv = alpha3[j] + (-2.0 + prob.h_layer(kd[1]) ** 2 * prob.lam(kd[1]))
            min_piv = min(min_piv, float(np.abs(piv[n3]).min()))
            alpha3[j + 1] = -1.0 / piv
        else:
            # E3_{j-1} = alpha_j E3^-, E3^- = r E3^+ and the derivative row give
            # E3^+ = E3_{j+1} / (1 + q r (1 - alpha_j))
            lo, up = kd[1], kd[2]
            r = prob.layer_eps[up] / prob.layer_eps[lo]
            q = prob.h_layer(up) / prob.h_layer(lo)
            piv = 1.0 + (1.0 - alpha3[j]) * (q * r)
            min_piv = min(min_piv, float(np.abs(piv[n3]).min()))
            alpha3[j + 1] = 1.0 / piv
    rho_n = alpha3[nz].copy()
    # back-substitution, top-down; reported value at an interface is the upper side
    pi_n = np.zeros((nz + 1,) + shape, dtype=complex)
    pi_n[nz] = 1.0
    for j in range(nz, 0, -1):
        g = alpha3[j]
        if kinds[j][0] == "interface":
            lo, up = kinds[j][1], kinds[j][2]
            g = g * (prob.layer_eps[up] / prob.layer_eps[lo])  # E3^- = (eps_up/eps_lo) E3^+
        pi_n[j - 1] = g * pi_n[j]
    pi_n[:, ~n3] = 0.0

    # E1/E2, Dirichlet bottom: E_{j-1} = alpha_j E_j + b_j E3_top (times mu or nu).
    alpha = np.zeros((nz + 1,) + shape, dtype=complex)
    bcoef = np.zeros((nz + 1,) + shape, dtype=complex)
    for j in range(1, nz):
        kd = kinds[j]
        q = 1.0
        if kd[0] == "interior":
            piv = alpha[j] + (-2.0 + prob.h_layer(kd[1]) ** 2 * prob.lam(kd[1]))
            f = 0.0
        else:
            # q E_{j-1} - (1 + q) E_j + E_{j+1} = h_up (1 - r) E3^+ (times mu or nu)
            lo, up = kd[1], kd[2]
            h_up = prob.h_layer(up)
            q = h_up / prob.h_layer(lo)
            piv = q * alpha[j] - (1.0 + q)
            f = h_up * (1.0 - prob.layer_eps[up] / prob.layer_eps[lo]) * pi_n[j]
        mask = np.ones(shape, dtype=bool)
        mask[0, 0] = False
        min_piv = min(min_piv, float(np.abs(piv[mask]).min()))
        alpha[j + 1] = -1.0 / piv
        bcoef[j + 1] = (f - q * bcoef[j]) / piv
    rho_d = alpha[nz].copy()
    T = bcoef[nz].copy()
    pi_d = np.zeros((nz + 1,) + shape, dtype=complex)
    theta_d = np.zeros((nz + 1,) + shape, dtype=complex)
    pi_d[nz] = 1.0
    for j in range(nz, 0, -1):
        pi_d[j - 1] = alpha[j] * pi_d[j]
        theta_d[j - 1] = alpha[j] * theta_d[j] + bcoef[j]
    T[~n3] = 0.0
    theta_d[:, ~n3] = 0.0
    return Columns(rho_d, T, rho_n, pi_d, theta_d, pi_n, min_piv)
