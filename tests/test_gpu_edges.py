"""Edge cases of the hot path against the oracle: the smallest grids the method allows
(one mode per direction, one z-interval, layers of one interval), a very elongated
aperture, normal and grazing incidence (beta = 0), right-hand sides in ragged lockstep
groups, and the direct and iterative solves of each.  Bars as for the other small cases:
field within 1e-10 and RCS within 1e-9 of the oracle's dense solve.  Grazing TE incidence
excites nothing (beta and the normal polarisation component both vanish in the right-hand
side), so its field is rounding noise on both sides: errors are taken relative to at
least 1e-4 of the case's largest field (and RCS), and that field is checked to be at
rounding level."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

EDGE = [
    ("min_2x2x1_vacuum", W.Cavity(0.3, 0.3, 0.1, 2, 2, 1, (1,), (1.0 + 0j,))),
    ("3x2x2_two_layers_of_one", W.Cavity(0.5, 0.4, 0.2, 3, 2, 2, (1, 1), (4.0 + 1.0j, 1.5 + 0j))),
    ("elongated_2x40x3", W.Cavity(0.25, 5.0, 0.3, 2, 40, 3, (3,), (2.0 + 0.3j,))),
    ("5x6x4_lossy", W.Cavity(0.7, 0.9, 0.35, 5, 6, 4, (2, 2), (3.0 + 0.5j, 1.0 + 0j))),
]
INCS = [(0.0, 0.0, W.TM), (0.0, 0.0, W.TE), (np.pi / 2, 0.7, W.TM), (np.pi / 2, 2.1, W.TE),
        (0.4, 1.3, W.TM), (1.1, 4.0, W.TE), (0.8, 0.2, W.TE)]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("direct", ["never", "always"])
def test_edge_case_against_oracle(case, direct):
    import torch
    name, cav = case
    print(f"\n[case] {name} direct={direct}", flush=True)
    prob = Problem.from_cavity(cav)
    ora = solver.plan(prob)
    th = [i[0] for i in INCS]
    ph = [i[1] for i in INCS]
    po = [i[2] for i in INCS]
    plan = P.Plan.from_cavity(cav, batch=3, direct=direct)    # groups of 3, 3, 1
    fields = plan.solve_batch(th, ph, po)
    torch.cuda.synchronize()
    info = plan.info()
    assert info.last_rel_residual <= 1e-12
    assert info.last_direct == (1 if direct == "always" else 0)
    sig = plan.rcs_many(np.arange(len(INCS)), th, ph)
    refs = [solver.solve(ora, t, f, pol, tol=1e-13, dense=True) for t, f, pol in INCS]
    oes = [solver.field_out(ora, r) for r in refs]
    os_ = [np.array(solver.backscatter(ora, r, t, f)) for r, (t, f, _) in zip(refs, INCS)]
    fscale = max(np.linalg.norm(o) for o in oes)
    sscale = max(o.max() for o in os_)
    for i, (t, f, pol) in enumerate(INCS):
        eo = fields[i].cpu().numpy()
        ferr = np.linalg.norm(eo - oes[i]) / max(np.linalg.norm(oes[i]), 1e-4 * fscale)
        serr = np.abs(sig[i] - os_[i]).max() / max(os_[i].max(), 1e-4 * sscale)
        print(f"[compare] {name} inc {i}: field {ferr:.1e} rcs {serr:.1e}", flush=True)
        assert ferr <= 1e-10 and serr <= 1e-9, (name, i, ferr, serr)
    grazing_te = [i for i, (t, f, pol) in enumerate(INCS) if t == np.pi / 2 and pol == W.TE]
    for i in grazing_te:                     # no excitation: noise-level field on both sides
        assert np.linalg.norm(oes[i]) <= 1e-12 * fscale
        assert float(fields[i].abs().max()) <= 1e-12 * fscale
    plan.close()


def test_misaligned_field_output_is_refused():
    """Device outputs of complex values must be 16-byte aligned (the kernels move each value
    as one 16-byte access): a field pointer 8 bytes into a buffer gives CAVITY_EINVAL from
    cavity_solve, cavity_solve_batch and cavity_solve_group before any work is queued, and
    the aligned call then succeeds."""
    import ctypes

    import torch
    cav = EDGE[0][1]
    plan = P.Plan.from_cavity(cav)
    buf = torch.zeros(plan.nz + 2, 3 * (plan.ny + 1) * (plan.nx + 1), dtype=torch.complex128,
                      device="cuda").reshape(-1)
    bad = ctypes.c_void_p(buf.data_ptr() + 8)
    lib = plan._lib
    assert lib.cavity_solve(plan._h, 0.3, 0.2, W.TM, bad) == 1
    th, ph, po = (ctypes.c_double * 1)(0.3), (ctypes.c_double * 1)(0.2), (ctypes.c_int * 1)(W.TM)
    assert lib.cavity_solve_batch(plan._h, 1, th, ph, po, bad, None) == 1
    plans = (ctypes.c_void_p * 1)(plan._h.value)
    outs = (ctypes.c_void_p * 1)(bad.value)
    assert lib.cavity_solve_group(1, plans, th, ph, po, outs) == 1
    torch.cuda.synchronize()
    assert float(buf.abs().max()) == 0.0
    good = plan.solve(0.3, 0.2, W.TM)
    torch.cuda.synchronize()
    assert float(good.abs().max()) > 0.0
    plan.close()
