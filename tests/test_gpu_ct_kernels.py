"""The kernel variants with the transform shapes fixed at compile time (extension
transform 8 x 8 x 8 = 512, box transform 5 x 5 x 5 x 5 = 625: the 256 x 256 grid of the
8 x 8 x 2 wavelength cavity) against the oracle and against the generic kernels (the
radix-16 build, chosen with CAVITY_FFT_MAXR=16) on the same inputs.

Tolerances: the single-layer operators 1e-12 against the oracle (as for the other cases)
and 1e-13 between the two builds (same stages, same twiddles, same operation order); whole
solves 1e-11 between the builds in double precision (both stop at a relative residual of
1e-12) and 1e-9 in mixed precision (the single-precision inner cycles round differently).
"""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver, tbc
from oracle.problem import Problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def plans():
    wl = W.lossy_8x8x2()
    print(f"\n[case] {wl.name}: compile-time and generic kernels", flush=True)
    ct = P.Plan.from_cavity(wl.cavity, direct="never")
    assert (ct.info().P1, ct.info().P2) == (625, 625)
    mp = pytest.MonkeyPatch()
    mp.setenv("CAVITY_FFT_MAXR", "16")
    try:
        gen = P.Plan.from_cavity(wl.cavity, direct="never")
    finally:
        mp.undo()
    yield wl, ct, gen
    ct.close()
    gen.close()


def test_single_layer_families(plans):
    wl, ct, gen = plans
    prob = Problem.from_cavity(wl.cavity)
    ora = solver.plan(prob)
    rng = np.random.default_rng(625)
    for i, fam in enumerate(tbc.FAMILIES):
        x = rng.standard_normal(ct.grid_shape) + 1j * rng.standard_normal(ct.grid_shape)
        a = ct.debug_tbc(i, x)
        b = gen.debug_tbc(i, x)
        ref = tbc.apply(prob, ora.khat, fam, x)
        for arr in (a, b, ref):   # entries outside the family's modes
            if fam == "cs":
                arr[:, 0] = 0
            if fam == "sc":
                arr[0, :] = 0
        print(f"[compare] {fam}: vs oracle {rel(a, ref):.2e}, vs generic {rel(a, b):.2e}",
              flush=True)
        assert rel(a, ref) <= 1e-12
        assert rel(a, b) <= 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_matches_generic(plans, precision):
    wl, ct, gen = plans
    if precision == "mixed":
        ct = P.Plan.from_cavity(wl.cavity, precision="mixed", direct="never")
        mp = pytest.MonkeyPatch()
        mp.setenv("CAVITY_FFT_MAXR", "16")
        try:
            gen = P.Plan.from_cavity(wl.cavity, precision="mixed", direct="never")
        finally:
            mp.undo()
    inc = wl.incidences[0]
    fa = ct.solve(inc.theta, inc.phi, inc.pol)
    fb = gen.solve(inc.theta, inc.phi, inc.pol)
    err = float((fa - fb).abs().max() / fb.abs().max())
    print(f"[compare] {precision} field, compile-time vs generic: {err:.2e}", flush=True)
    assert err <= (1e-11 if precision == "fp64" else 1e-9)
    if precision == "mixed":
        ct.close()
        gen.close()
