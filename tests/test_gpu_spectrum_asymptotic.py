"""GPU parity of the asymptotic (Case 2) kernel spectrum (Section 5.2) against the oracle's
restatement of the same steps, on a parity case and at the 256 x 256 aperture of the
8 x 8 wavelength workload (P = 625), the aperture cache keeping the two spectra apart,
and a solve with the asymptotic spectrum against the oracle's solve with it."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver, spectrum
from oracle.problem import Problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("cav", [W.small_cases()[2].cavity, W.lossy_8x8x2().cavity],
                         ids=["lossy_2x1.25x0.5", "lossy_8x8x2_256"])
def test_asymptotic_spectrum_matches_oracle(cav):
    import torch
    print(f"\n[case] asymptotic spectrum {cav.a}x{cav.b} {cav.nx}x{cav.ny}", flush=True)
    prob = Problem.from_cavity(cav)
    # the spectrum depends on the aperture only: two-level plans
    mk = lambda m: P.Plan(cav.a, cav.b, cav.c, cav.nx, cav.ny, 2, k=cav.k, spectrum=m)  # noqa
    gx, ga = mk("exact"), mk("asymptotic")
    kx, ka = gx.debug_spectrum(), ga.debug_spectrum()
    torch.cuda.synchronize()
    gx.close()
    ga.close()
    ref_a = spectrum.kernel_spectrum(prob, "asymptotic")
    assert rel(ka, ref_a) <= 1e-12
    d = rel(ka, kx)                    # the two methods differ by the expansion error
    assert 0 < d <= 1e-7, d
    print(f"[compare] asymptotic vs exact spectrum {d:.2e}", flush=True)


def test_solve_with_asymptotic_spectrum():
    import torch
    wl = W.small_cases()[1]
    print(f"\n[case] {wl.name} asymptotic spectrum solve", flush=True)
    prob = Problem.from_cavity(wl.cavity)
    ora = solver.plan(prob, spectrum_method="asymptotic")
    gpu = P.Plan.from_cavity(wl.cavity, spectrum="asymptotic")
    inc = wl.incidences[0]
    gpu.solve(inc.theta, inc.phi, inc.pol)
    got = gpu.aperture(0)
    torch.cuda.synchronize()
    gpu.close()
    ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
    err = np.linalg.norm(got - ref.x) / np.linalg.norm(ref.x)
    print(f"[compare] aperture rel err {err:.2e}", flush=True)
    assert err <= 1e-10
