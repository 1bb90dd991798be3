"""Whole path: plan (elimination, kernel spectrum, preconditioner) and solve (oracle).

Paper: Section 6, Algorithms I and II (Step 1: singular-integral data and right-hand
sides; Step 2: per-mode LU elimination; Step 3: the aperture system), Section 7 (the four
phase timers T_singular, T_assemble, T_solve, T_RCS).  The aperture system is solved by
GMRES with the true residual checked at the end; on tiny grids a dense LU is available.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict

import numpy as np

from . import columns, fields, incident, spectrum, system
from .problem import Problem


@dataclass
class Plan:
    prob: Problem
    cols: columns.Columns
    khat: np.ndarray
    op: system.ReducedSystem
    pre: system.BlockPreconditioner
    timers: Dict[str, float] = field(default_factory=dict)


def plan(prob: Problem, operator: str = "trap", spectrum_method: str = "exact") -> Plan:
    """operator: the discrete TBC, "trap" (D_trap) or "spec" (D_spec); spectrum_method:
    "exact" (quadrature) or "asymptotic" (Case 2 of Section 5.2 at large frequencies)."""
    t0 = time.perf_counter()
    khat = spectrum.kernel_spectrum(prob, spectrum_method)
    t1 = time.perf_counter()
    cols = columns.eliminate(prob)
    op = system.ReducedSystem(prob, cols, khat, operator)
    pre = system.BlockPreconditioner(prob, cols, khat, operator)
    t2 = time.perf_counter()
    return Plan(prob, cols, khat, op, pre, {"spectrum": t1 - t0, "assemble": t2 - t1})


@dataclass
class Solution:
    x: np.ndarray            # compact aperture vector (paper order)
    grids: tuple             # padded (E1, E2, E3) aperture mode grids
    iterations: int
    rel_residual: float
    timers: Dict[str, float]


def solve(pl: Plan, theta: float, phi: float, pol: int, tol: float = 1e-13,
          dense: bool = False, restart: int = 60) -> Solution:
    prob = pl.prob
    t0 = time.perf_counter()
    g1, g2 = incident.rhs(prob, theta, phi, pol)
    b = prob.pack(g1, g2, np.zeros_like(g1))
    if dense:
        A = pl.op.dense()
        x = np.linalg.solve(A, b)
        its = 0
    else:
        x, its, _ = system.gmres(pl.op.matvec, pl.pre.solve, b, tol=tol, restart=restart)
    r = b - pl.op.matvec(x)
    rel = float(np.linalg.norm(r) / max(np.linalg.norm(b), 1e-300))
    t1 = time.perf_counter()
    return Solution(x, prob.unpack(x), its, rel, {"solve": t1 - t0})


def field_out(pl: Plan, sol: Solution) -> np.ndarray:
    return fields.synthesize(pl.prob, pl.cols, *sol.grids)


def backscatter(pl: Plan, sol: Solution, theta: float, phi: float):
    return fields.rcs(pl.prob, sol.grids[0], sol.grids[1], theta, phi)
