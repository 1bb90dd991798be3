"""The request server on the GPU: a mix of cavities (sizes, layer stacks, shared and
distinct apertures) submitted at once to four workers must give every request exactly the
result it gets alone (plan + solve + RCS on one stream), the mixed-precision results must
match the oracle within 1e-8, admission must respect the device-memory budget, and plans
that share an aperture (spectrum and diagonal taken from the library's cache) must equal a
plan computed from scratch."""
import ctypes
import os

import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W
from oracle import solver
from oracle.problem import Problem

pytestmark = pytest.mark.gpu


def _mix():
    """Ten requests: the four small parity cavities, permittivity variants of two of them
    (same aperture, different columns), and a 48 x 48 x 16 lossy cavity."""
    cases = W.small_cases()[:4]       # the server builds its plans with the common step
    reqs = []
    for wl in cases:
        reqs.append((wl.cavity, wl.incidences[0]))
    base = cases[1].cavity
    for eps in ((2.0 + 0.3j, 1.0 + 0j), (5.5 + 1.2j, 1.5 + 0.1j), (1.2 + 0j, 3.0 + 0.5j)):
        reqs.append((W.Cavity(base.a, base.b, base.c, base.nx, base.ny, base.nz, base.layer_nz,
                              eps), W.Incidence(0.4, 1.1, W.TE)))
    big = W.Cavity(1.5, 1.5, 0.5, 48, 48, 16, (8, 8), (4.0 + 1.0j, 1.0 + 0j))
    reqs.append((big, W.Incidence(0.7, 0.3, W.TM)))
    reqs.append((big, W.Incidence(0.7, 0.3, W.TE)))
    reqs.append((cases[0].cavity, W.Incidence(0.9, 2.0, W.TM)))
    return reqs


def _alone(cav, inc, precision):
    import torch
    plan = P.Plan.from_cavity(cav, precision=precision, batch=1)
    field = plan.solve(inc.theta, inc.phi, inc.pol)
    sig = plan.rcs(0, [inc.theta], [inc.phi])[0]
    torch.cuda.synchronize()
    plan.close()
    return field, sig


@pytest.mark.timeout(600)
def test_mix_equals_alone_and_oracle():
    import torch
    reqs = _mix()
    print(f"\n[case] server mix of {len(reqs)} requests, 4 streams", flush=True)
    srv = P.Server(streams=4, precision="mixed")
    outs = [torch.empty((3, c.nz + 1, c.ny + 1, c.nx + 1), dtype=torch.complex128, device="cuda")
            for c, _ in reqs]
    tickets = [srv.submit(c, i.theta, i.phi, i.pol, out=o) for (c, i), o in zip(reqs, outs)]
    results = [srv.wait(t) for t in tickets]
    for t in tickets:
        srv.release(t)
    srv.close()
    for k, ((cav, inc), res, out) in enumerate(zip(reqs, results, outs)):
        assert res.status == 0, (k, res.status)
        assert res.t_submit_ms <= res.t_start_ms <= res.t_done_ms
        field, sig = _alone(cav, inc, "mixed")
        d = float((out - field).abs().max()) / float(field.abs().max())
        ds = float(np.abs(np.array(res.sigma[:]) - sig).max() / max(sig))
        print(f"[compare] request {k}: mix vs alone field {d:.1e}, rcs {ds:.1e}, "
              f"{res.iterations} its, {res.t_done_ms - res.t_start_ms:.2f} ms", flush=True)
        assert d <= 1e-13 and ds <= 1e-13
    for k in (1, len(reqs) - 4):
        cav, inc = reqs[k]
        ora = solver.plan(Problem.from_cavity(cav))
        ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
        oe = solver.field_out(ora, ref)
        err = np.linalg.norm(outs[k].cpu().numpy() - oe) / np.linalg.norm(oe)
        o = solver.backscatter(ora, ref, inc.theta, inc.phi)
        co = inc.pol
        err_r = abs(results[k].sigma[co] - o[co]) / o[co]
        print(f"[compare] request {k} vs oracle: field {err:.2e}, rcs {err_r:.2e}", flush=True)
        assert err <= 1e-8 and err_r <= 1e-8


@pytest.mark.timeout(300)
def test_budget_admission():
    import torch
    lib = P.load_library()
    reqs = _mix()[:4]
    fps = []
    for cav, _ in reqs:
        nzs = (ctypes.c_int * len(cav.layer_nz))(*cav.layer_nz)
        eps = (P.C128 * len(cav.layer_eps))(*[P.C128(e.real, e.imag) for e in map(complex, cav.layer_eps)])
        o = P.Opts()
        lib.cavity_opts_default(ctypes.byref(o))
        o.precision, o.batch = 1, 1
        b = ctypes.c_size_t()
        assert lib.cavity_plan_footprint(cav.a, cav.b, cav.c, cav.nx, cav.ny, cav.nz,
                                         ctypes.pointer(P.EpsStack(len(cav.layer_nz), nzs, eps)),
                                         cav.k, ctypes.byref(o), ctypes.byref(b)) == 0
        fields = 3 * (cav.nz + 1) * (cav.ny + 1) * (cav.nx + 1) * 16
        fps.append(b.value + fields)
    # room for the largest request only: requests run one at a time, in order
    srv = P.Server(streams=4, hbm_budget=max(fps) + 1024, precision="mixed")
    tickets = [srv.submit(c, i.theta, i.phi, i.pol) for c, i in reqs]
    res = [srv.wait(t) for t in tickets]
    assert all(r.status == 0 for r in res)
    budget = max(fps) + 1024
    # at every start, the requests running together fit in the budget
    for r in res:
        t = r.t_start_ms
        held = sum(q.device_bytes for q in res if q.t_start_ms <= t < q.t_done_ms)
        assert held <= budget, (held, budget)
    assert sorted(q.device_bytes for q in res) == sorted(fps)
    print(f"\n[case] budget {budget} bytes, footprints {fps}", flush=True)
    # a request larger than the whole budget is refused, not queued forever
    small = P.Server(streams=1, hbm_budget=1 << 20, precision="mixed")
    t = small.submit(reqs[0][0], 0.1, 0.2, W.TM)
    assert small.wait(t).status == 2
    small.close()
    srv.close()
    torch.cuda.synchronize()


@pytest.mark.timeout(300)
def test_aperture_cache_reuse_is_exact():
    import torch
    base = W.small_cases()[2].cavity
    other = W.Cavity(base.a, base.b, base.c, base.nx, base.ny, base.nz, base.layer_nz,
                     tuple(complex(e) * 1.1 for e in base.layer_eps))
    p1 = P.Plan.from_cavity(base)
    p2 = P.Plan.from_cavity(other)          # same aperture: spectrum and diagonal from cache
    k1, k2 = p1.debug_spectrum(), p2.debug_spectrum()
    assert np.array_equal(k1, k2)
    f2 = p2.solve(0.3, 0.5, W.TM)
    torch.cuda.synchronize()
    p1.close()
    p2.close()
    ora = solver.plan(Problem.from_cavity(other))
    ref = solver.solve(ora, 0.3, 0.5, W.TM, tol=1e-13)
    oe = solver.field_out(ora, ref)
    assert np.linalg.norm(f2.cpu().numpy() - oe) <= 1e-10 * np.linalg.norm(oe)


@pytest.mark.timeout(900)
def test_served_stream_first_requests():
    """The first 20 requests of the served stream (cavities of 2 to 12 wavelengths, one to
    three layers) submitted together to the server in mixed precision: every field and
    backscatter RCS within 1e-8 of the same request solved alone in double precision, and
    those of side at most 4 wavelengths within 1e-8 of the oracle."""
    import torch
    stream = W.served_stream(20)
    print(f"\n[case] served stream, first {len(stream)} requests", flush=True)
    srv = P.Server(streams=4, precision="mixed")
    outs, tickets = [], []
    for req in stream:
        cav, inc = req.workload.cavity, req.workload.incidences[0]
        o = torch.empty((3, cav.nz + 1, cav.ny + 1, cav.nx + 1), dtype=torch.complex128,
                        device="cuda")
        outs.append(o)
        tickets.append(srv.submit(cav, inc.theta, inc.phi, inc.pol, out=o))
    results = [srv.wait(t) for t in tickets]
    for t in tickets:
        srv.release(t)
    srv.close()
    torch.cuda.synchronize()
    n_oracle = 0
    for k, (req, r, o) in enumerate(zip(stream, results, outs)):
        cav, inc = req.workload.cavity, req.workload.incidences[0]
        assert r.status == 0, (k, r.status)
        co = inc.pol
        f64, s64 = _alone(cav, inc, "fp64")
        e = float(torch.linalg.vector_norm(o - f64) / torch.linalg.vector_norm(f64))
        er = abs(r.sigma[co] - s64[co]) / s64[co]
        del f64
        msg = f"[compare] request {k} ({cav.a:g} lambda, {cav.nx}x{cav.ny}x{cav.nz}): " \
              f"vs double alone field {e:.2e} rcs {er:.2e}"
        assert e <= 1e-8 and er <= 1e-8, msg
        if cav.a <= 4.0:
            ora = solver.plan(Problem.from_cavity(cav))
            ref = solver.solve(ora, inc.theta, inc.phi, inc.pol, tol=1e-13)
            oe = solver.field_out(ora, ref)
            eo = np.linalg.norm(o.cpu().numpy() - oe) / np.linalg.norm(oe)
            so = solver.backscatter(ora, ref, inc.theta, inc.phi)
            ro = abs(r.sigma[co] - so[co]) / so[co]
            msg += f"; vs oracle field {eo:.2e} rcs {ro:.2e}"
            assert eo <= 1e-8 and ro <= 1e-8, msg
            n_oracle += 1
        print(msg, flush=True)
    assert n_oracle >= 5


def _footprint(cav, field=True):
    lib = P.load_library()
    nzs = (ctypes.c_int * len(cav.layer_nz))(*cav.layer_nz)
    eps = (P.C128 * len(cav.layer_eps))(*[P.C128(e.real, e.imag) for e in map(complex, cav.layer_eps)])
    o = P.Opts()
    lib.cavity_opts_default(ctypes.byref(o))
    o.precision, o.batch = 1, 1
    b = ctypes.c_size_t()
    assert lib.cavity_plan_footprint(cav.a, cav.b, cav.c, cav.nx, cav.ny, cav.nz,
                                     ctypes.pointer(P.EpsStack(len(cav.layer_nz), nzs, eps)),
                                     cav.k, ctypes.byref(o), ctypes.byref(b)) == 0
    return b.value + (3 * (cav.nz + 1) * (cav.ny + 1) * (cav.nx + 1) * 16 if field else 0)


@pytest.mark.timeout(300)
def test_resident_plan_reuse_is_exact():
    """Requests on a cavity seen before run on its resident plan (no plan creation) and
    give exactly the result of the request alone; another cavity in between stays resident
    beside it."""
    import torch
    a = W.small_cases()[1].cavity
    b = W.small_cases()[2].cavity
    seq = [(a, W.Incidence(0.3, 0.4, W.TM)), (b, W.Incidence(0.5, 1.0, W.TE)),
           (a, W.Incidence(0.7, 2.0, W.TE)), (a, W.Incidence(0.2, 5.0, W.TM)),
           (b, W.Incidence(1.1, 0.1, W.TM))]
    print(f"\n[case] {len(seq)} requests on two cavities, one at a time", flush=True)
    srv = P.Server(streams=2, precision="mixed")
    res, outs = [], []
    for cav, inc in seq:
        o = torch.empty((3, cav.nz + 1, cav.ny + 1, cav.nx + 1), dtype=torch.complex128,
                        device="cuda")
        t = srv.submit(cav, inc.theta, inc.phi, inc.pol, out=o)
        res.append(srv.wait(t))
        srv.release(t)
        outs.append(o)
    srv.close()
    assert [r.plan_reused for r in res] == [0, 0, 1, 1, 1]
    for k, ((cav, inc), r, o) in enumerate(zip(seq, res, outs)):
        assert r.status == 0
        field, sig = _alone(cav, inc, "mixed")
        d = float((o - field).abs().max()) / float(field.abs().max())
        ds = float(np.abs(np.array(r.sigma[:]) - sig).max() / max(sig))
        print(f"[compare] request {k} reused {r.plan_reused}: vs alone field {d:.1e} rcs {ds:.1e}, "
              f"{r.t_done_ms - r.t_start_ms:.2f} ms", flush=True)
        assert d <= 1e-13 and ds <= 1e-13
    # no plan reuse when the resident budget is 0
    srv = P.Server(streams=1, precision="mixed", plan_cache_bytes=0)
    rr = []
    for cav, inc in seq[:3]:
        t = srv.submit(cav, inc.theta, inc.phi, inc.pol)
        rr.append(srv.wait(t).plan_reused)
        srv.release(t)
    srv.close()
    assert rr == [0, 0, 0]


@pytest.mark.timeout(300)
def test_admission_passes_a_large_head():
    """With room for the large request alone, a small request queued behind it starts while
    another small one runs, before the large head (which then runs alone).  An attempt in
    which the small request could not start while the first one ran (it was queued after
    the first one ended, or a worker thread was not scheduled in time) says nothing about
    the admission rule and is repeated, at most five times; the rule itself would fail
    every attempt."""
    import time

    import torch
    # 64 z-levels make the first request last a few ms while its footprint stays below the
    # large one's
    slow = W.Cavity(2.0, 2.0, 1.0, 64, 64, 64, (32, 32), (4.0 + 1.0j, 1.0 + 0j))
    big = W.Cavity(3.0, 3.0, 1.0, 96, 96, 32, (32,), (2.0 + 0.5j,))
    small = W.small_cases()[0].cavity
    f_slow, f_big, f_small = _footprint(slow), _footprint(big), _footprint(small)
    assert f_slow + f_big > f_big + 1024 >= f_slow + f_small
    for attempt in range(5):
        # the server's admission trace (stderr) goes into the captured output of a failure
        os.environ["CAVITY_SERVER_TRACE"] = "1"
        try:
            srv = P.Server(streams=2, hbm_budget=f_big + 1024, precision="mixed",
                           plan_cache_bytes=0)
        finally:
            del os.environ["CAVITY_SERVER_TRACE"]
        c0 = time.perf_counter()
        t1 = srv.submit(slow, 0.3, 0.2, W.TM)
        t2 = srv.submit(big, 0.3, 0.2, W.TM)
        t3 = srv.submit(small, 0.3, 0.2, W.TE)
        c1 = time.perf_counter()
        r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
        srv.close()
        torch.cuda.synchronize()
        print(f"\n[case] attempt {attempt}: starts slow {r1.t_start_ms:.2f}, big "
              f"{r2.t_start_ms:.2f}, small {r3.t_start_ms:.2f} ms; slow done {r1.t_done_ms:.2f}; "
              f"queued at {r1.t_submit_ms:.2f}, {r2.t_submit_ms:.2f}, {r3.t_submit_ms:.2f} "
              f"(three submits {1e3 * (c1 - c0):.2f} ms)", flush=True)
        assert r1.status == r2.status == r3.status == 0
        # the budget holds the large head alone: it never starts while the first one runs
        assert r2.t_start_ms >= r1.t_done_ms - 1e-6
        if r3.t_start_ms < r1.t_done_ms:
            break
    assert r3.t_start_ms < r1.t_done_ms, "the small request never started beside the first"
    assert r3.t_start_ms < r2.t_start_ms
    assert r2.t_start_ms >= max(r1.t_done_ms, r3.t_done_ms) - 1e-6


@pytest.mark.timeout(300)
def test_same_aperture_requests_are_grouped():
    """Requests queued behind a running one, on cavities that share an aperture, are taken
    together and solved as one lockstep group; each result equals the request alone."""
    import torch
    from test_gpu_group import GROUP
    busy = W.Cavity(3.0, 3.0, 1.0, 96, 96, 32, (32,), (2.0 + 0.5j,))
    srv = P.Server(streams=1, precision="mixed", plan_cache_bytes=0)
    t0 = srv.submit(busy, 0.3, 0.2, W.TM)
    outs, tickets = [], []
    for cav, inc in GROUP:
        o = torch.empty((3, cav.nz + 1, cav.ny + 1, cav.nx + 1), dtype=torch.complex128,
                        device="cuda")
        outs.append(o)
        tickets.append(srv.submit(cav, inc.theta, inc.phi, inc.pol, out=o))
    r0 = srv.wait(t0)
    res = [srv.wait(t) for t in tickets]
    srv.close()
    torch.cuda.synchronize()
    print(f"\n[case] group sizes {[r.group_size for r in res]}, first request alone "
          f"{r0.group_size}", flush=True)
    assert r0.status == 0 and r0.group_size == 1
    assert [r.group_size for r in res] == [len(GROUP)] * len(GROUP)
    for k, ((cav, inc), r, o) in enumerate(zip(GROUP, res, outs)):
        assert r.status == 0
        field, sig = _alone(cav, inc, "mixed")
        d = float((o - field).abs().max()) / float(field.abs().max())
        ds = float(np.abs(np.array(r.sigma[:]) - sig).max() / max(sig))
        print(f"[compare] grouped request {k}: vs alone field {d:.1e} rcs {ds:.1e}", flush=True)
        assert d <= 1e-13 and ds <= 1e-13
