"""Reduced aperture system, block preconditioner, GMRES and the brute-force full system.

Paper: Section 3 ((ENU14), (ENU24), (ENU34) assembled as (ENUGa); elimination (EJJ1) and
the reduced system (EJ1)), Section 4 ((uTT1), (uNUGa) and the layered reduced system
(uT1)), Section 5.1 (G~ = H~ = -nu_n I3 in row 1 and -mu_m I3 in row 2), Section 6 (the
paper solves the reduced system densely and names an iterative solver as the way to large
sizes).

Reading on the sign of the TBC operator.  The field representation (EGa2) gives
E = E_inc + E_ref + curl( 2 S[z x E] ) above the aperture, and curl curl = k^2 + grad div
there, so  z x curl E = g + 2k^2 z x S[z x E] + 2 z x grad S[div_Gamma(z x E)].
The printed operator T of (ENU1) carries the opposite sign (a sign slip between (EGa2)
and (ENU)); with the printed sign the transverse evanescent aperture modes see the
interior and exterior admittances subtract instead of add, which is the wrong physics
(an outgoing evanescent wave e^{i nu y - kappa z} has z x curl E = +kappa E, which the
sign below reproduces).  This build follows (EGa2): the F, G, H terms of (ENU14) and
(ENU24) enter with a plus sign.

With sigma = nu_n E1 - mu_m E2 on the cos-cos grid (the cos-cos coefficients of
div_Gamma(z x E)), the three aperture rows read (E = aperture values, node Nz):
  row 1, N1: E1_{Nz-1} - E1 + mu_m h E3 + (h/q)[2k^2 S^cs E1 - 2 nu_n S^cc sigma] = g1
  row 2, N2: E2_{Nz-1} - E2 + nu_n h E3 + (h/c)[2k^2 S^sc E2 + 2 mu_m S^cc sigma] = g2
  row 3, N3: E3_{Nz-1} - E3 + mu_m h E1 + nu_n h E2 = 0
and the elimination replaces E_{l,Nz-1} by rho_l E_l + tau_l E3 (tau_3 = 0).  The G~, H~
terms of Section 3 / Appendix A collapse to the sigma terms above after the integration
by parts of Section 5.1 (the third TBC row carries the h that the printed (ENU33) omits,
as its matrix form (ENU34) with I~3, I~4 shows).  With layers of their own steps, h in
these rows is the top layer's step (the one-sided difference at the aperture lies in the
top layer).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import tbc
from .columns import Columns
from .problem import Problem

# +1: the sign implied by the field representation (EGa2); -1 would be the printed (ENU1).
TBC_SIGN = +1.0


class ReducedSystem:
    """Matrix-free reduced aperture operator on the compact (paper-ordered) vector."""

    def __init__(self, prob: Problem, cols: Columns, khat: np.ndarray, operator: str = "trap"):
        self.prob, self.cols, self.khat = prob, cols, khat
        self.single = {"trap": tbc.apply, "spec": tbc.apply_spec}[operator]
        self.mu = prob.mu[:, None]
        self.nu = prob.nu[None, :]
        self.hq_ = prob.h / prob.q_norm()
        self.hc_ = prob.h / prob.c_norm()
        self.n_applies = 0

    def apply_grid(self, e1, e2, e3):
        p, c, k2 = self.prob, self.cols, self.prob.k ** 2
        mu, nu, h = self.mu, self.nu, p.h
        sigma = nu * e1 - mu * e2
        s_cs = self.single(p, self.khat, "cs", e1)
        s_sc = self.single(p, self.khat, "sc", e2)
        s_cc = self.single(p, self.khat, "cc", sigma)
        r1 = (c.rho_d - 1.0) * e1 + mu * (c.T + h) * e3 \
            + TBC_SIGN * self.hq_ * (2 * k2 * s_cs - 2 * nu * s_cc)
        r2 = (c.rho_d - 1.0) * e2 + nu * (c.T + h) * e3 \
            + TBC_SIGN * self.hc_ * (2 * k2 * s_sc + 2 * mu * s_cc)
        r3 = (c.rho_n - 1.0) * e3 + mu * h * e1 + nu * h * e2
        self.n_applies += 1
        return r1, r2, r3

    def matvec(self, x):
        e1, e2, e3 = self.prob.unpack(x)
        return self.prob.pack(*self.apply_grid(e1, e2, e3))

    def dense(self):
        n = self.prob.n_ap
        out = np.zeros((n, n), dtype=complex)
        for j in range(n):
            e = np.zeros(n, dtype=complex)
            e[j] = 1.0
            out[:, j] = self.matvec(e)
        return out


class BlockPreconditioner:
    """Per-mode 3x3 blocks of the reduced operator with S^f replaced by its diagonal.

    A design choice of this build (the paper proposes no preconditioner): only the
    convergence speed depends on it, never the solution."""

    def __init__(self, prob: Problem, cols: Columns, khat: np.ndarray, operator: str = "trap"):
        self.prob = prob
        k2, h = prob.k ** 2, prob.h
        mu, nu = prob.mu[:, None], prob.nu[None, :]
        diag = {"trap": tbc.diagonal, "spec": tbc.diagonal_spec}[operator]
        d_cs = diag(prob, khat, "cs")
        d_sc = diag(prob, khat, "sc")
        d_cc = diag(prob, khat, "cc")
        hq_, hc_ = h / prob.q_norm(), h / prob.c_norm()
        shape = (prob.M + 1, prob.N + 1)
        A = np.zeros(shape + (3, 3), dtype=complex)
        sg = TBC_SIGN
        A[..., 0, 0] = (cols.rho_d - 1) + sg * hq_ * (2 * k2 * d_cs - 2 * nu * nu * d_cc)
        A[..., 0, 1] = sg * hq_ * 2 * nu * mu * d_cc
        A[..., 0, 2] = mu * (cols.T + h)
        A[..., 1, 0] = sg * hc_ * 2 * mu * nu * d_cc
        A[..., 1, 1] = (cols.rho_d - 1) + sg * hc_ * (2 * k2 * d_sc - 2 * mu * mu * d_cc)
        A[..., 1, 2] = nu * (cols.T + h)
        A[..., 2, 0] = np.broadcast_to(mu * h, shape)
        A[..., 2, 1] = np.broadcast_to(nu * h, shape)
        A[..., 2, 2] = cols.rho_n - 1
        n1, n2, n3 = prob.masks()
        for comp, msk in enumerate((n1, n2, n3)):
            A[~msk, comp, :] = 0.0
            A[~msk, :, comp] = 0.0
            A[~msk, comp, comp] = 1.0
        self.inv = np.linalg.inv(A)
        self.diag = (d_cs, d_sc, d_cc)

    def solve_grid(self, r1, r2, r3):
        r = np.stack([r1, r2, r3], axis=-1)
        z = np.einsum("mnij,mnj->mni", self.inv, r)
        return z[..., 0], z[..., 1], z[..., 2]

    def solve(self, x):
        e = self.prob.unpack(x)
        return self.prob.pack(*self.solve_grid(*e))


def gmres(matvec, precond, b, tol=1e-13, restart=60, max_iter=2000, x0=None):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt.

    Stops when the true residual ||b - A x|| <= tol ||b||.  Returns (x, iterations,
    history of relative residual estimates)."""
    n = b.size
    x = np.zeros(n, dtype=complex) if x0 is None else x0.astype(complex).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    hist = []
    it = 0
    while it < max_iter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta <= tol * bnorm:
            break
        V = np.zeros((restart + 1, n), dtype=complex)
        H = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart, dtype=complex)
        sn = np.zeros(restart, dtype=complex)
        g = np.zeros(restart + 1, dtype=complex)
        V[0] = r / beta
        g[0] = beta
        Z = np.zeros((restart, n), dtype=complex)
        j_last = -1
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            # rotation [[c, s], [-conj(s), conj(c)]] with c = conj(a)/d, s = conj(b)/d
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            cs[j] = np.conj(H[j, j]) / den
            sn[j] = np.conj(H[j + 1, j]) / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_last = j
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= 0.5 * tol * bnorm or it >= max_iter:
                break
        m = j_last + 1
        y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
        x = x + y @ Z[:m]
    return x, it, hist


# ----------------------------------------------------------------------------------------
# Brute force: the full discrete system of Sections 3-4 assembled as one sparse matrix
# ----------------------------------------------------------------------------------------

def assemble_full(prob: Problem, khat: np.ndarray, g1: np.ndarray, g2: np.ndarray):
    """Assemble every z-level of every mode plus the aperture rows, with dense S^f.

    Returns (A, b, index) where index maps (comp, m, n, j[, 'lo']) to a column."""
    kinds = prob.node_kind()
    nz, h, k2 = prob.nz, prob.h, prob.k ** 2   # h: the top layer's step (aperture rows)
    n1, n2, n3 = prob.masks()
    modes = {1: list(zip(*np.nonzero(n1))), 2: list(zip(*np.nonzero(n2))),
             3: list(zip(*np.nonzero(n3)))}
    idx = {}
    for comp in (1, 2):
        for (m, n) in modes[comp]:
            for j in range(1, nz + 1):
                idx[(comp, m, n, j)] = len(idx)
    for (m, n) in modes[3]:
        for j in range(0, nz + 1):
            idx[(3, m, n, j)] = len(idx)
            if kinds[j][0] == "interface":
                idx[(3, m, n, j, "lo")] = len(idx)
    nvar = len(idx)
    rows, cols_, vals = [], [], []
    b = np.zeros(nvar, dtype=complex)
    row = [0]

    def add(r, key, v):
        if key is None:
            return
        rows.append(r)
        cols_.append(idx[key])
        vals.append(v)

    layer_top = np.cumsum(prob.layer_nz)

    def e3key(m, n, ell, j):
        if kinds[j][0] == "interface" and j == layer_top[ell]:
            return (3, m, n, j, "lo")
        return (3, m, n, j)

    mu, nu = prob.mu, prob.nu
    # tangential columns
    for comp in (1, 2):
        for (m, n) in modes[comp]:
            fac = mu[m] if comp == 1 else nu[n]
            for j in range(1, nz):
                r = row[0]
                kd = kinds[j]
                key = lambda jj: None if jj == 0 else (comp, m, n, jj)  # noqa: E731
                add(r, key(j + 1), 1.0)
                if kd[0] == "interior":
                    lam = prob.kappa2(kd[1]) - mu[m] ** 2 - nu[n] ** 2
                    add(r, key(j - 1), 1.0)
                    add(r, key(j), -2.0 + prob.h_layer(kd[1]) ** 2 * lam)
                else:
                    h_up = prob.h_layer(kd[2])
                    q = h_up / prob.h_layer(kd[1])
                    add(r, key(j - 1), q)
                    add(r, key(j), -1.0 - q)
                    if m >= 1 and n >= 1:
                        add(r, (3, m, n, j), -fac * h_up)
                        add(r, (3, m, n, j, "lo"), fac * h_up)
                row[0] += 1
    # normal column
    for (m, n) in modes[3]:
        r = row[0]
        add(r, e3key(m, n, 0, 0), 1.0)
        add(r, e3key(m, n, 0, 1), -1.0)
        row[0] += 1
        for j in range(1, nz):
            kd = kinds[j]
            r = row[0]
            if kd[0] == "interior":
                ell = kd[1]
                lam = prob.kappa2(ell) - mu[m] ** 2 - nu[n] ** 2
                add(r, e3key(m, n, ell, j - 1), 1.0)
                add(r, e3key(m, n, ell, j), -2.0 + prob.h_layer(ell) ** 2 * lam)
                add(r, e3key(m, n, ell, j + 1), 1.0)
                row[0] += 1
            else:
                lo, up = kd[1], kd[2]
                add(r, (3, m, n, j), prob.layer_eps[up])
                add(r, (3, m, n, j, "lo"), -prob.layer_eps[lo])
                row[0] += 1
                r = row[0]
                q = prob.h_layer(up) / prob.h_layer(lo)
                add(r, e3key(m, n, up, j + 1), 1.0)
                add(r, e3key(m, n, up, j), -1.0)
                add(r, e3key(m, n, lo, j), -q)
                add(r, e3key(m, n, lo, j - 1), q)
                row[0] += 1
    # aperture rows with dense single-layer matrices
    shape = (prob.M + 1, prob.N + 1)
    S = {f: tbc.dense_matrix_fft(prob, khat, f) for f in tbc.FAMILIES}
    flat = lambda m, n: m * shape[1] + n  # noqa: E731
    qn, cn = prob.q_norm(), prob.c_norm()
    top = len(prob.layer_nz) - 1
    for (m, n) in modes[1]:
        r = row[0]
        add(r, (1, m, n, nz - 1) if nz > 1 else None, 1.0)
        add(r, (1, m, n, nz), -1.0)
        if m >= 1:
            add(r, (3, m, n, nz), mu[m] * h)
        c0 = TBC_SIGN * (h / qn[m, n])
        for (mm, nn) in modes[1]:
            v = c0 * 2 * k2 * S["cs"][flat(m, n), flat(mm, nn)]
            v += c0 * (-2 * nu[n]) * S["cc"][flat(m, n), flat(mm, nn)] * nu[nn]
            add(r, (1, mm, nn, nz), v)
        for (mm, nn) in modes[2]:
            v = c0 * (-2 * nu[n]) * S["cc"][flat(m, n), flat(mm, nn)] * (-mu[mm])
            add(r, (2, mm, nn, nz), v)
        b[r] = g1[m, n]
        row[0] += 1
    for (m, n) in modes[2]:
        r = row[0]
        add(r, (2, m, n, nz - 1) if nz > 1 else None, 1.0)
        add(r, (2, m, n, nz), -1.0)
        if n >= 1:
            add(r, (3, m, n, nz), nu[n] * h)
        c0 = TBC_SIGN * (h / cn[m, n])
        for (mm, nn) in modes[2]:
            v = c0 * 2 * k2 * S["sc"][flat(m, n), flat(mm, nn)]
            v += c0 * (2 * mu[m]) * S["cc"][flat(m, n), flat(mm, nn)] * (-mu[mm])
            add(r, (2, mm, nn, nz), v)
        for (mm, nn) in modes[1]:
            v = c0 * (2 * mu[m]) * S["cc"][flat(m, n), flat(mm, nn)] * nu[nn]
            add(r, (1, mm, nn, nz), v)
        b[r] = g2[m, n]
        row[0] += 1
    for (m, n) in modes[3]:
        r = row[0]
        add(r, e3key(m, n, top, nz - 1), 1.0)
        add(r, (3, m, n, nz), -1.0)
        add(r, (1, m, n, nz), mu[m] * h)
        add(r, (2, m, n, nz), nu[n] * h)
        row[0] += 1
    assert row[0] == nvar, (row[0], nvar)
    A = sp.csr_matrix((vals, (rows, cols_)), shape=(nvar, nvar))
    return A, b, idx


def solve_full(prob: Problem, khat, g1, g2):
    """Solve the full discrete system; return per-component (Nz+1, M+1, N+1) arrays
    (E3 at interfaces on the upper side; E3 at node 0 included)."""
    A, b, idx = assemble_full(prob, khat, g1, g2)
    x = spla.spsolve(A.tocsc(), b)
    shape = (prob.nz + 1, prob.M + 1, prob.N + 1)
    out = [np.zeros(shape, dtype=complex) for _ in range(3)]
    for key, col in idx.items():
        if len(key) == 4:
            comp, m, n, j = key
            out[comp - 1][j, m, n] = x[col]
    return out, A, b, x
