"""Backscatter RCS sweeps on the geometries of the paper's numerical examples (Section 7):
one plan per geometry, many incidences solved together without field output, RCS from the
stored aperture solutions.  Each geometry: the GPU sweep against the oracle at two angles
(1e-9 relative, both polarisations), the mixed-precision sweep against the double one
(1e-8), and the phi = 0 mirror rule (the cross-polarised backscatter vanishes).  Example 3
runs with both readings of its interval counts: one common step, and each layer with its
own step."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver
from oracle.problem import Problem

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
@pytest.mark.parametrize("make", [W.example1_sweep, W.example1_sweep_m21, W.example1_small_sweep,
                                  W.example2_sweep, W.example3_sweep, W.example3_sweep_steps],
                         ids=["example1", "example1_m21", "example1_small", "example2", "example3",
                              "example3_steps"])
def test_sweep_against_oracle(make):
    import torch
    wl = make()
    # every tenth angle, both polarisations (incidences alternate TM, TE per angle)
    incs = [inc for k, inc in enumerate(wl.incidences) if (k // 2) % 10 == 0]
    print(f"\n[case] {wl.name}: {len(incs)} of {len(wl.incidences)} incidences", flush=True)
    th = [i.theta for i in incs]
    ph = [i.phi for i in incs]
    po = [i.pol for i in incs]
    res = {}
    for prec in ("fp64", "mixed"):
        plan = P.Plan.from_cavity(wl.cavity, precision=prec, batch=16)
        plan.solve_batch(th, ph, po, field=False)
        res[prec] = np.array([plan.rcs(i, t, f)[0] for i, (t, f) in enumerate(zip(th, ph))])
        its = plan.info().last_iterations
        plan.close()
        print(f"[gpu] {prec}: last iterations {its}", flush=True)
    torch.cuda.synchronize()
    for i, inc in enumerate(incs):
        co, cross = inc.pol, 1 - inc.pol
        s64, smx = res["fp64"][i], res["mixed"][i]
        assert abs(smx[co] - s64[co]) <= 1e-8 * s64[co]
        assert s64[cross] <= 1e-12 * s64[co] + 1e-300, (i, s64)
    ora = solver.plan(Problem.from_cavity(wl.cavity))
    for i in (2, len(incs) - 1):          # a TM and a TE incidence
        inc = incs[i]
        ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
        o = solver.backscatter(ora, ref, inc.theta, inc.phi)
        co = inc.pol
        err = abs(res["fp64"][i][co] - o[co]) / o[co]
        print(f"[compare] theta {np.degrees(inc.theta):.1f} pol {inc.pol}: rcs rel err {err:.2e}",
              flush=True)
        assert err <= 1e-9


@pytest.mark.timeout(600)
def test_graph_replays_match_direct_launches():
    """With CAVITY_GRAPHS=1 the Arnoldi steps run as captured graphs (one per step index and
    group size, replayed across lockstep groups, restarts and solve calls); they give the
    same RCS as direct launches, bit for bit, on every replay: three solve calls in a row,
    with eager work and synchronisations between them."""
    import os

    import torch
    wl = W.example2_sweep()
    incs = [inc for k, inc in enumerate(wl.incidences) if (k // 2) % 6 == 0][:48]
    th = [i.theta for i in incs]
    ph = [i.phi for i in incs]
    po = [i.pol for i in incs]
    out = {}
    old = os.environ.get("CAVITY_GRAPHS")
    try:
        for mode in ("0", "1"):
            os.environ["CAVITY_GRAPHS"] = mode
            plan = P.Plan.from_cavity(wl.cavity, precision="mixed", batch=16)
            runs = []
            for rep in range(3):
                plan.solve_batch(th, ph, po, field=False)
                runs.append(np.array([plan.rcs(i, t, f)[0] for i, (t, f) in enumerate(zip(th, ph))]))
                torch.cuda.synchronize()
                _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between
            plan.close()
            out[mode] = runs
    finally:
        if old is None:
            os.environ.pop("CAVITY_GRAPHS", None)
        else:
            os.environ["CAVITY_GRAPHS"] = old
    ref = out["0"][0]
    for mode in ("0", "1"):
        for rep, r in enumerate(out[mode]):
            d = float(np.abs(r - ref).max() / ref.max())
            print(f"[compare] graphs={mode} call {rep}: max rel diff {d:.1e}", flush=True)
            assert d == 0.0
