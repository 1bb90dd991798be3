"""Several small cavities in one lockstep group (cavity_solve_group): cavities sharing the
aperture (1.5 x 1 wavelengths, 24 x 12 nodes) but with their own depth, z-grid and layer
stack, one incidence each, solved together.  Each field and backscatter RCS equals that of
the plan solved alone (the group's kernels keep every right-hand side's arithmetic separate)
in double and mixed precision, and the double-precision results match the oracle; plans
that do not share the aperture are refused."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

GROUP = [
    (W.Cavity(1.5, 1.0, 0.4, 24, 12, 10, (3, 7), (2.0 + 0.3j, 1.0 + 0j)), W.Incidence(0.6, 0.35, W.TM)),
    (W.Cavity(1.5, 1.0, 0.6, 24, 12, 14, (14,), (4.0 + 1.0j,)), W.Incidence(0.2, 1.3, W.TE)),
    (W.Cavity(1.5, 1.0, 0.3, 24, 12, 9, (3, 3, 3), (3.0 + 0.2j, 1.5 + 0j, 1.0 + 0j)),
     W.Incidence(1.1, 4.0, W.TE)),
    (W.Cavity(1.5, 1.0, 0.25, 24, 12, 6, (6,), (1.0 + 0j,)), W.Incidence(0.0, 0.0, W.TM)),
    (W.Cavity(1.5, 1.0, 0.5, 24, 12, 20, (8, 12), (6.0 + 2.0j, 2.5 + 0.5j)), W.Incidence(0.9, 2.2, W.TM)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_group_equals_alone(precision):
    import torch
    print(f"\n[case] group of {len(GROUP)} cavities, {precision}", flush=True)
    plans = [P.Plan.from_cavity(c, precision=precision, batch=1) for c, _ in GROUP]
    outs = P.solve_group(plans, [i.theta for _, i in GROUP], [i.phi for _, i in GROUP],
                         [i.pol for _, i in GROUP])
    sig = [p.rcs(0, i.theta, i.phi)[0] for p, (_, i) in zip(plans, GROUP)]
    its = plans[0].info().last_iterations
    for p in plans:
        p.close()
    torch.cuda.synchronize()
    for k, ((cav, inc), o, s) in enumerate(zip(GROUP, outs, sig)):
        alone = P.Plan.from_cavity(cav, precision=precision, batch=1)
        f = alone.solve(inc.theta, inc.phi, inc.pol)
        sa = alone.rcs(0, inc.theta, inc.phi)[0]
        alone.close()
        d = float((o - f).abs().max()) / float(f.abs().max())
        ds = float(np.abs(s - sa).max() / sa.max())
        print(f"[compare] cavity {k} ({cav.nz} intervals, {len(cav.layer_nz)} layers): group vs "
              f"alone field {d:.1e}, rcs {ds:.1e}", flush=True)
        assert d <= 1e-12 and ds <= 1e-12
        if precision == "fp64" and k in (0, 2, 4):
            ora = solver.plan(Problem.from_cavity(cav))
            ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
            oe = solver.field_out(ora, ref)
            err = np.linalg.norm(o.cpu().numpy() - oe) / np.linalg.norm(oe)
            so = solver.backscatter(ora, ref, inc.theta, inc.phi)
            co = inc.pol
            er = abs(s[co] - so[co]) / so[co]
            print(f"[compare] cavity {k} vs oracle: field {err:.2e}, rcs {er:.2e}", flush=True)
            assert err <= 1e-10 and er <= 1e-9
    assert its > 0


def test_group_refuses_mismatched_plans():
    a = P.Plan.from_cavity(GROUP[0][0])
    b = P.Plan.from_cavity(W.Cavity(1.5, 1.0, 0.4, 20, 12, 10, (10,), (1.0 + 0j,)))
    c = P.Plan.from_cavity(GROUP[1][0], precision="mixed")
    d = P.Plan.from_cavity(GROUP[1][0], operator="spec")
    for plans, status in (([a, b], 1), ([a, c], 1), ([a, a], 1)):
        with pytest.raises(P.CavityError) as e:
            P.solve_group(plans, [0.1] * len(plans), [0.0] * len(plans), [0] * len(plans))
        assert e.value.status == status
    with pytest.raises(P.CavityError) as e:
        P.solve_group([d], [0.1], [0.0], [0])
    assert e.value.status == 6
    for p in (a, b, c, d):
        p.close()
