"""Write tests/golden/layered_16x16x4.npz: oracle values for the three-layer 16 x 16 x 4
wavelength cavity on the 512 x 512 x 128 grid (eps_r 4+1i / 2.5+0.5i / 1 over 25/50/25 %),
theta = 45 deg, phi = 0, both polarisations.

Only the CPU oracle is called.  Stored: a seeded sample of 4000 aperture coefficients and
20000 field values per incidence (flat indices into the paper-ordered aperture vector and
into E_out[3][Nz+1][Ny+1][Nx+1]), the backscatter RCS, and the oracle's GMRES data.

Run from the repository root:  python tests/golden/make_layered_16x16x4.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import solver  # noqa: E402
from oracle.problem import Problem  # noqa: E402


def main():
    wl = W.layered_16x16x4()
    prob = Problem.from_cavity(wl.cavity)
    pl = solver.plan(prob)
    rng = np.random.default_rng(20080196)
    n_field = 3 * (prob.nz + 1) * (prob.ny + 1) * (prob.nx + 1)
    ap_idx = np.sort(rng.choice(prob.n_ap, size=4000, replace=False))
    fe_idx = np.sort(rng.choice(n_field, size=20000, replace=False))
    out = {"ap_idx": ap_idx, "field_idx": fe_idx}
    for i, inc in enumerate(wl.incidences):
        sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, tol=1e-13)
        field = solver.field_out(pl, sol).ravel()
        out[f"ap_{i}"] = sol.x[ap_idx]
        out[f"ap_norm_{i}"] = np.linalg.norm(sol.x)
        out[f"field_{i}"] = field[fe_idx]
        out[f"field_norm_{i}"] = np.linalg.norm(field)
        out[f"rcs_{i}"] = np.array(solver.backscatter(pl, sol, inc.theta, inc.phi))
        out[f"relres_{i}"] = sol.rel_residual
        print(f"incidence {i}: iterations {sol.iterations}, residual {sol.rel_residual:.2e}",
              flush=True)
        del field
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "layered_16x16x4.npz")
    np.savez_compressed(path, **out)
    print(path)


if __name__ == "__main__":
    main()
