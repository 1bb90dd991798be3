"""The spectral discrete TBC operator (D_spec, exact trial-function transforms on the kernel
spectrum lattice, Section 5.2) against the oracle's D_spec: each single-layer operator and
the full operator to 1e-12, the field of iterative, direct and mixed-precision solves to
1e-10 and the RCS to 1e-9.  Its RCS differs from D_trap's by the discretisation change
(a sanity check that the option is in effect)."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver, tbc
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

CASES = W.small_cases()[:3] + [
    W.Workload("edge_5x6x4", W.Cavity(0.7, 0.9, 0.35, 5, 6, 4, (2, 2), (3.0 + 0.5j, 1.0 + 0j)),
               (W.Incidence(0.4, 1.3, W.TM),))]


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("wl", CASES, ids=[c.name for c in CASES])
def test_spec_operator_and_solves(wl):
    import torch
    print(f"\n[case] {wl.name} spec", flush=True)
    prob = Problem.from_cavity(wl.cavity)
    ora = solver.plan(prob, operator="spec")
    gpu = P.Plan.from_cavity(wl.cavity, operator="spec")
    rng = np.random.default_rng(8)
    for f, fam in enumerate(tbc.FAMILIES):
        x = rng.standard_normal(gpu.grid_shape) + 1j * rng.standard_normal(gpu.grid_shape)
        got = gpu.debug_tbc(f, x)
        ref = tbc.apply_spec(prob, ora.khat, fam, x)
        if fam == "cs":
            got[:, 0] = ref[:, 0] = 0
        if fam == "sc":
            got[0, :] = ref[0, :] = 0
        assert rel(got, ref) <= 1e-12, fam
    e = []
    for msk in prob.masks():
        x = rng.standard_normal(msk.shape) + 1j * rng.standard_normal(msk.shape)
        x[~msk] = 0
        e.append(x)
    got = gpu.debug_operator(*e)
    ref = ora.op.apply_grid(*e)
    scale = max(np.abs(r).max() for r in ref)
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= 1e-12 * scale
    gpu.close()
    inc = wl.incidences[0]
    ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
    oe = solver.field_out(ora, ref)
    o = np.array(solver.backscatter(ora, ref, inc.theta, inc.phi))
    sig = {}
    for precision, direct, tol in (("fp64", "never", 1e-10), ("fp64", "always", 1e-10),
                                   ("mixed", "never", 1e-10)):
        plan = P.Plan.from_cavity(wl.cavity, operator="spec", precision=precision, direct=direct)
        field = plan.solve(inc.theta, inc.phi, inc.pol)
        torch.cuda.synchronize()
        assert plan.info().last_rel_residual <= 1e-12
        eo = field.cpu().numpy()
        err = np.linalg.norm(eo - oe) / np.linalg.norm(oe)
        s = plan.rcs(0, inc.theta, inc.phi)[0]
        print(f"[compare] {precision} {direct}: field {err:.1e}", flush=True)
        assert err <= tol
        assert np.abs(s - o).max() <= 1e-9 * o.max()
        sig[(precision, direct)] = s
        plan.close()
    trap = P.Plan.from_cavity(wl.cavity)
    trap.solve(inc.theta, inc.phi, inc.pol, field=False)
    st = trap.rcs(0, inc.theta, inc.phi)[0]
    trap.close()
    co = inc.pol
    assert abs(st[co] - sig[("fp64", "never")][co]) > 1e-6 * st[co]
