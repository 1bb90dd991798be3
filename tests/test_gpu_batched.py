"""Batched mixed precision at full size: the three-layer 8 x 8 x 2 wavelength cavity on the
256 x 256 x 64 grid with all 128 right-hand sides (8 theta x 8 phi x 2 polarisations),
iterated 32 at a time, as the benchmark runs it.  The mixed-precision batch (single-precision
TBC convolutions, double-precision refinement residuals, tolerance 1e-10) against the
double-precision batch (tolerance 1e-12) on every incidence, and both against the oracle on
the subset 0, 17, ..., 119.

Bars: mixed vs double and mixed vs oracle 1e-8 relative on the whole field and on the
co-polarised backscatter RCS; double vs oracle 1e-10 (field) and 1e-9 (RCS)."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

SUBSET = (0, 17, 34, 51, 68, 85, 102, 119)


@pytest.mark.timeout(900)
def test_batched_layered_8x8x2_mixed_vs_fp64_and_oracle():
    import torch
    wl = W.batched_layered_8x8x2()
    incs = wl.incidences
    print(f"\n[case] {wl.name}: all {len(incs)} incidences, batch 32", flush=True)
    th = [i.theta for i in incs]
    ph = [i.phi for i in incs]
    po = [i.pol for i in incs]
    idx = np.arange(len(incs))
    mix = P.Plan.from_cavity(wl.cavity, precision="mixed", tol=wl.tol, batch=32)
    f_mix = mix.solve_batch(th, ph, po)
    s_mix = mix.rcs_many(idx, th, ph)
    mix.close()
    dbl = P.Plan.from_cavity(wl.cavity, tol=1e-12, batch=32)
    f_dbl = dbl.solve_batch(th, ph, po)
    s_dbl = dbl.rcs_many(idx, th, ph)
    dbl.close()
    torch.cuda.synchronize()
    worst, worst_r = 0.0, 0.0
    for i, inc in enumerate(incs):
        e = float(torch.linalg.vector_norm(f_mix[i] - f_dbl[i]) / torch.linalg.vector_norm(f_dbl[i]))
        co = inc.pol
        er = abs(s_mix[i][co] - s_dbl[i][co]) / s_dbl[i][co]
        worst, worst_r = max(worst, e), max(worst_r, er)
        assert e <= 1e-8 and er <= 1e-8, (i, e, er)
    print(f"[compare] mixed vs double, {len(incs)} incidences: worst field {worst:.2e}, "
          f"rcs {worst_r:.2e}", flush=True)
    ora = solver.plan(Problem.from_cavity(wl.cavity))
    for i in SUBSET:
        inc = incs[i]
        ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
        oe = solver.field_out(ora, ref)
        nrm = np.linalg.norm(oe)
        em = np.linalg.norm(f_mix[i].cpu().numpy() - oe) / nrm
        ed = np.linalg.norm(f_dbl[i].cpu().numpy() - oe) / nrm
        o = solver.backscatter(ora, ref, inc.theta, inc.phi)
        co = inc.pol
        rm = abs(s_mix[i][co] - o[co]) / o[co]
        rd = abs(s_dbl[i][co] - o[co]) / o[co]
        print(f"[compare] incidence {i}: field mixed {em:.2e} double {ed:.2e}; "
              f"rcs mixed {rm:.2e} double {rd:.2e}", flush=True)
        assert em <= 1e-8 and rm <= 1e-8
        assert ed <= 1e-10 and rd <= 1e-9
