"""GPU parity of every hot-path step against the CPU oracle on small cavities.

The cases span several tiles and ragged (non power-of-two, non-square) sizes, one to four
layers, layers of a single interval, lossless and lossy media.  Each step is called through
the C ABI (inspection entry points for the individual steps, cavity_solve / cavity_rcs for
the whole path) and compared element by element with the oracle on the same inputs.

Tolerances: individual steps 1e-12 relative (double rounding of FFT-based vs. dense sums);
whole solves 1e-10 relative on the field (both solvers stop at a relative residual of
1e-12..1e-13 and the reduced system's condition number is a few tens) and 1e-9 on the RCS.
"""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import incident, solver, tbc
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

CASES = W.small_cases()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", params=list(range(len(CASES))), ids=[c.name for c in CASES])
def pair(request):
    wl = CASES[request.param]
    print(f"\n[case] {wl.name}", flush=True)
    prob = Problem.from_cavity(wl.cavity)
    gpu = P.Plan.from_cavity(wl.cavity)
    ora = solver.plan(prob)
    yield wl, prob, gpu, ora
    gpu.close()


def test_spectrum(pair):
    wl, prob, gpu, ora = pair
    assert (gpu.info_.P1, gpu.info_.P2) == prob.box
    assert rel(gpu.debug_spectrum(), ora.khat) <= 1e-12


def test_elimination(pair):
    wl, prob, gpu, ora = pair
    rd, T, rn = gpu.debug_columns()
    pd, td, pn = gpu.debug_profiles()
    c = ora.cols
    n1, n2, n3 = prob.masks()
    ok = np.ones_like(n3)
    ok[0, 0] = False
    assert rel(rd[ok], c.rho_d[ok]) <= 1e-12
    assert rel(rn[n3], c.rho_n[n3]) <= 1e-12
    assert rel(pd[:, ok], c.pi_d[:, ok]) <= 1e-12
    assert rel(pn[:, n3], c.pi_n[:, n3]) <= 1e-12
    if len(prob.layer_nz) > 1:
        assert rel(T[n3], c.T[n3]) <= 1e-12
        assert rel(td, c.theta_d) <= 1e-12
    else:
        assert np.abs(T).max() == 0 and np.abs(td).max() == 0
    assert abs(gpu.info_.min_pivot - c.min_pivot) <= 1e-12 * c.min_pivot


def test_single_layer_families(pair):
    wl, prob, gpu, ora = pair
    rng = np.random.default_rng(11)
    for f, fam in enumerate(tbc.FAMILIES):
        x = rng.standard_normal(gpu.grid_shape) + 1j * rng.standard_normal(gpu.grid_shape)
        got = gpu.debug_tbc(f, x)
        ref = tbc.apply(prob, ora.khat, fam, x)
        if fam == "cs":
            got[:, 0] = ref[:, 0] = 0
        if fam == "sc":
            got[0, :] = ref[0, :] = 0
        assert rel(got, ref) <= 1e-12, fam


def test_rhs(pair):
    wl, prob, gpu, ora = pair
    for inc in wl.incidences + (W.Incidence(0.3, 2.0, W.TM),):
        g1, g2 = gpu.debug_rhs(inc.theta, inc.phi, inc.pol)
        o1, o2 = incident.rhs(prob, inc.theta, inc.phi, inc.pol)
        scale = max(np.abs(o1).max(), np.abs(o2).max())
        assert np.abs(g1 - o1).max() <= 1e-13 * scale
        assert np.abs(g2 - o2).max() <= 1e-13 * scale


def test_operator(pair):
    wl, prob, gpu, ora = pair
    rng = np.random.default_rng(5)
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


def test_solve_field_and_rcs(pair):
    wl, prob, gpu, ora = pair
    for inc in wl.incidences:
        field = gpu.solve(inc.theta, inc.phi, inc.pol)
        info = gpu.info()
        assert info.last_rel_residual <= 1e-12
        ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
        ap = gpu.aperture(0)
        assert np.linalg.norm(ap - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
        eo = field.cpu().numpy()
        oe = solver.field_out(ora, ref)
        assert np.linalg.norm(eo - oe) <= 1e-10 * np.linalg.norm(oe)
        sig = gpu.rcs(0, [inc.theta, 0.2], [inc.phi, 1.0])
        for i, (t, f) in enumerate([(inc.theta, inc.phi), (0.2, 1.0)]):
            o = solver.backscatter(ora, ref, t, f)
            assert np.abs(sig[i] - np.array(o)).max() <= 1e-9 * max(o)


def test_batch_matches_single(pair):
    wl, prob, gpu, ora = pair
    incs = list(wl.incidences) + [W.Incidence(0.9, 0.4, W.TE)]
    th = [i.theta for i in incs]
    ph = [i.phi for i in incs]
    po = [i.pol for i in incs]
    fields = gpu.solve_batch(th, ph, po)
    for i, inc in enumerate(incs):
        single = gpu.solve(inc.theta, inc.phi, inc.pol)
        assert float((fields[i] - single).abs().max()) <= 1e-13 * float(single.abs().max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_call_of_several_groups_matches_single(pair, precision):
    """A call of several lockstep groups (5 incidences in groups of 2, the last one alone):
    every field equals the field of the same incidence solved alone (the kernels do not
    depend on the group), read on the caller's stream right after the call."""
    wl, prob, gpu, ora = pair
    plan = P.Plan.from_cavity(wl.cavity, batch=2, precision=precision, direct="never")
    incs = [W.Incidence(0.1 + 0.15 * i, 0.3 * i, W.TM if i % 2 else W.TE) for i in range(5)]
    fields = plan.solve_batch([i.theta for i in incs], [i.phi for i in incs],
                              [i.pol for i in incs])
    peaks = [float(f.abs().max()) for f in fields]
    for i, inc in enumerate(incs):
        single = plan.solve(inc.theta, inc.phi, inc.pol)
        assert abs(peaks[i] - float(single.abs().max())) <= 1e-13 * peaks[i]
        assert float((fields[i] - single).abs().max()) <= 1e-13 * float(single.abs().max())
    plan.close()


def test_mixed_precision_solve(pair):
    """Mixed precision (single-precision convolutions inside GMRES, double-precision
    residuals at every restart): the field and RCS against the double-precision oracle
    within 1e-8 relative, the stated target of the refined solve, and a batch of
    incidences equal to the single solves."""
    wl, prob, gpu, ora = pair
    mix = P.Plan.from_cavity(wl.cavity, precision="mixed")
    incs = list(wl.incidences) + [W.Incidence(0.9, 0.4, W.TE)]
    fields = mix.solve_batch([i.theta for i in incs], [i.phi for i in incs],
                             [i.pol for i in incs])
    assert mix.info().last_rel_residual <= 1e-12
    # the batch's RCS first: a later solve call replaces the stored solutions
    sigs = [mix.rcs(i, [inc.theta], [inc.phi])[0] for i, inc in enumerate(incs)]
    for i, inc in enumerate(incs):
        ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
        oe = solver.field_out(ora, ref)
        err = np.linalg.norm(fields[i].cpu().numpy() - oe) / np.linalg.norm(oe)
        print(f"[compare] mixed incidence {i}: field rel err {err:.2e}", flush=True)
        assert err <= 1e-8
        o = solver.backscatter(ora, ref, inc.theta, inc.phi)
        assert np.abs(sigs[i] - np.array(o)).max() <= 1e-8 * max(o)
        single = mix.solve(inc.theta, inc.phi, inc.pol)
        assert float((fields[i] - single).abs().max()) <= 1e-13 * float(single.abs().max())
    mix.close()


def test_no_convergence_reported():
    cav = W.vacuum_1x1x05().cavity
    gpu = P.Plan.from_cavity(cav, max_iter=1)
    with pytest.raises(P.CavityError) as exc:
        gpu.solve(0.3, 0.0, W.TM)
    assert exc.value.status == 4
    gpu.close()


def test_resonant_geometry_refused():
    # Dirichlet mode (1,1) tuned to the discrete eigenvalue h^2 lam = 2 - 2 cos(3 pi / Nz)
    a = b = 1.0
    nz, c = 8, 0.5
    h = c / nz
    lam = (2 - 2 * np.cos(3 * np.pi / nz)) / h ** 2
    eps = (lam + 2 * np.pi ** 2) / (2 * np.pi) ** 2
    with pytest.raises(P.CavityError) as exc:
        P.Plan(a, b, c, 6, 6, nz, [nz], [complex(eps)])
    assert exc.value.status == 3


def test_invalid_angle_rejected():
    gpu = P.Plan.from_cavity(W.vacuum_1x1x05().cavity)
    with pytest.raises(P.CavityError) as exc:
        gpu.solve(2.0, 0.0, W.TM)
    assert exc.value.status == 1
    gpu.close()


@pytest.mark.parametrize("form", ["0", "1"], ids=["rows_pingpong", "rows_in_place"])
def test_tbc_row_pass_forms(form, monkeypatch):
    """Both forms of the TBC row passes (two LDS buffers, or in place with one work item per
    thread) give the oracle's single-layer operators and the full operator to 1e-12."""
    monkeypatch.setenv("CAVITY_TBC_ROWS_IP", form)
    rng = np.random.default_rng(21)
    for wl in CASES[:3]:
        prob = Problem.from_cavity(wl.cavity)
        ora = solver.plan(prob)
        for precision in ("fp64", "mixed"):
            gpu = P.Plan.from_cavity(wl.cavity, precision=precision)
            assert gpu.info().tbc_rows_in_place == int(form)
            for fam in tbc.FAMILIES:
                x = rng.standard_normal(gpu.grid_shape) + 1j * rng.standard_normal(gpu.grid_shape)
                got = gpu.debug_tbc(tbc.FAMILIES.index(fam), x)
                ref = tbc.apply(prob, ora.khat, fam, x)
                if fam == "cs":
                    got[:, 0] = ref[:, 0] = 0
                if fam == "sc":
                    got[0, :] = ref[0, :] = 0
                assert rel(got, ref) <= 1e-12, (wl.name, fam)
            inc = wl.incidences[0]
            gpu.solve(inc.theta, inc.phi, inc.pol, field=False)
            ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
            tol = 1e-10 if precision == "fp64" else 1e-8
            assert np.linalg.norm(gpu.aperture(0) - ref.x) <= tol * np.linalg.norm(ref.x)
            gpu.close()
