#!/usr/bin/env python3
"""Benchmark of the cavity-scattering hot path on one MI355X.

One step = the solve of every incidence of the workload (right-hand side, preconditioned
GMRES with the FFT-applied TBC operator), the field synthesis on all (Nz+1) x (Ny+1) x
(Nx+1) nodes and the backscatter RCS.  The plan (truncated-kernel spectrum, per-mode
z-elimination, preconditioner) is built before the timed region; its build time is
reported on its own as plan_ms.

value = unknowns solved per second = steps * incidences * n_ap * Nz / wall time.

The default workload is the 8 x 8 x 2 wavelength cavity filled with eps_r = 4+1i on a
256 x 256 x 64 grid (h = lambda/32), incidence theta = 30 deg, phi = 45 deg, both
polarisations.  Inputs are synthetic (the paper's workloads are geometries, not data).

Also reported: the average-launch roofline of the dominant kernel (timed with HIP events on
its launch stream through the library's probe) and the CPU oracle timed on the host cores
on the same workload (reported baseline), plus the GPU field's error against that oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cavity unknowns solved/s + p50/p99 latency, mixed vs FP64 at ≤1e-8 rel err"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(wl, gpu_fields, gpu_sigma, sample):
    """Time the CPU oracle on the same workload: plan + the first `sample` incidences (field
    and RCS each), a bounded sample of the workload."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import solver
    from oracle.problem import Problem

    prob = Problem.from_cavity(wl.cavity)
    t0 = time.perf_counter()
    pl = solver.plan(prob)
    fields, sig = [], []
    incs = wl.incidences[:sample]
    for inc in incs:
        sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, tol=1e-13)
        if gpu_fields is not None:
            fields.append(solver.field_out(pl, sol))
        sig.append(solver.backscatter(pl, sol, inc.theta, inc.phi))
    t1 = time.perf_counter()
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    errs = ([float(np.linalg.norm(g - o) / np.linalg.norm(o)) for g, o in zip(gpu_fields, fields)]
            if gpu_fields is not None else [])
    rerr = []
    for i, (g, o) in enumerate(zip(gpu_sigma, sig)):
        co = int(wl.incidences[i].pol)      # co-polarised component of this incidence
        rerr.append(float(abs(g[co] - o[co]) / abs(o[co])))
    unknowns = len(incs) * prob.unknowns
    what = ("whole workload once" if len(incs) == len(wl.incidences) else
            f"first {len(incs)} of {len(wl.incidences)} incidences")
    return {
        "value": unknowns / (t1 - t0), "unit": "unknowns/s", "cores": int(threads),
        "kind": "oracle",
        "sample": (f"{what}: plan + {len(incs)} solves + "
                   f"{'fields + ' if gpu_fields is not None else ''}RCS, {t1 - t0:.1f} s wall"),
        "phases_s": {"spectrum": pl.timers["spectrum"], "assemble": pl.timers["assemble"]},
    }, (max(errs) if errs else None), max(rerr)


# Sources that define the TBC kernels: a traffic measurement is only used while they match.
KERNEL_SOURCES = ("device.hpp", "fft.hpp", "kernels.hpp", "solve_kernels.hip")


def sources_sha256() -> str:
    """Hash of the device sources of the TBC kernels."""
    import hashlib
    d = os.path.join(ROOT, "paper_2008_01966_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed hardware-counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None when
    there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None, None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    rel = os.path.relpath(path, ROOT)
    if kv.get("source_sha256") != sources_sha256():
        return None, rel + " (stale: kernel sources changed since)"
    return float(kv["traffic_bytes_per_launch"]), rel



SERVED = "served_stream_2000_poisson40"


def served_main(args) -> int:
    """Replay the served stream in real time: each request (random cavity, one incidence)
    is submitted to the library's request server at its seeded Poisson arrival time; the
    latency of a request runs from its arrival to its field and backscatter RCS being
    ready.  value = unknowns of all requests / (last completion - first arrival)."""
    import numpy as np
    import torch

    import paper_2008_01966_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    stream = W.served_stream(args.requests)
    # warm-up on a cavity outside the stream (loads the kernels; no aperture of the stream)
    warm = P.Plan(0.75, 0.75, 0.25, 24, 24, 8, precision="mixed")
    warm.solve(0.2, 0.1, 0)
    warm.close()
    torch.cuda.synchronize()
    prec = "mixed" if args.precision in ("mixed", "both") else "fp64"
    srv = P.Server(streams=args.streams, precision=prec)
    tickets = []
    t_origin = srv.now_ms() + 50.0
    for req in stream:
        due = t_origin + 1e3 * req.arrival_s
        while True:
            now = srv.now_ms()
            if now >= due:
                break
            time.sleep(min(0.002, (due - now) * 1e-3))
        inc = req.workload.incidences[0]
        tickets.append((srv.submit(req.workload.cavity, inc.theta, inc.phi, inc.pol), due))
    res = []
    for t, due in tickets:
        r = srv.wait(t)
        res.append((r, due))
        srv.release(t)
    srv.close()
    bad = [k for k, (r, _) in enumerate(res) if r.status != 0]
    lat = np.array([r.t_done_ms - due for r, due in res])
    queue = np.array([r.t_start_ms - due for r, due in res])
    unknowns = float(sum(r.unknowns for r, _ in res))
    span_s = (max(r.t_done_ms for r, _ in res) - t_origin) * 1e-3
    its = [r.iterations for r, _ in res]
    out = {
        "metric": METRIC,
        "value": unknowns / span_s,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": len(res),
        "warmup": 1,
        "ms_per_step": float(np.mean(lat)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": SERVED,
            "requests": len(res),
            "arrivals": "Poisson 40/s, seed 200801966, replayed in real time",
            "streams": args.streams,
            "precision": prec,
            "step": "one request: plan (aperture data from the cache when seen before) + "
                    "GMRES + field on all nodes + backscatter RCS",
        },
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "of": "arrival to field and RCS ready"},
        "queueing_ms": {"p50": float(np.percentile(queue, 50)),
                        "p99": float(np.percentile(queue, 99))},
        "failed_requests": bad,
        "gmres_iterations": {"min": int(min(its)), "max": int(max(its))},
        "span_s": span_s,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["oracle_check"] = served_oracle(stream, res, prec)
    print(json.dumps(out), flush=True)
    return 0


def served_oracle(stream, res, prec):
    """The oracle serves the stream's requests in order, serially, for about 20 s of host
    time (at least one); the same requests are solved alone on the GPU with their field
    kept and compared with the oracle's field and RCS."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info

    import paper_2008_01966_amd as P
    from oracle import solver
    from oracle.problem import Problem

    t0 = time.perf_counter()
    done, unknowns, errs = 0, 0, []
    for req, (r, _) in zip(stream, res):
        cav = req.workload.cavity
        inc = req.workload.incidences[0]
        prob = Problem.from_cavity(cav)
        pl = solver.plan(prob)
        sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, tol=1e-13)
        field = solver.field_out(pl, sol)
        sig = solver.backscatter(pl, sol, inc.theta, inc.phi)
        done += 1
        unknowns += prob.unknowns
        plan = P.Plan.from_cavity(cav, precision=prec, batch=1)
        g = plan.solve(inc.theta, inc.phi, inc.pol).cpu().numpy()
        plan.close()
        co = inc.pol
        errs.append({"request": done - 1, "side": cav.a, "grid": [cav.nx, cav.ny, cav.nz],
                     "field_rel_err": float(np.linalg.norm(g - field) / np.linalg.norm(field)),
                     "rcs_rel_err_server": float(abs(r.sigma[co] - sig[co]) / sig[co])})
        if time.perf_counter() - t0 > 20.0:
            break
    t1 = time.perf_counter()
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    torch.cuda.synchronize()
    return ({"value": unknowns / (t1 - t0), "unit": "unknowns/s", "cores": int(threads),
             "kind": "oracle",
             "sample": f"first {done} requests of the stream served serially, {t1 - t0:.1f} s "
                       "wall (includes the GPU re-solve of each for the field check)"}, errs)

def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lossy_8x8x2_256x256x64")
    ap.add_argument("--probe", default=None,
                    help="kernel timed for the roofline (default: the column pass of the TBC "
                         "convolution in the headline precision); none: no probe (the "
                         "Arnoldi steps may then run as captured graphs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (reference "
                         "kernel for scaling hardware traffic counters) and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=0,
                    help="right-hand sides iterated together (0: the workload's choice)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="incidences the CPU oracle solves (0: all when at most 2, else 1)")
    ap.add_argument("--requests", type=int, default=2000, help="served stream: requests")
    ap.add_argument("--streams", type=int, default=4, help="served stream: concurrent requests")
    ap.add_argument("--operator", choices=["trap", "spec"], default="trap",
                    help="discrete TBC operator: trapezoid samples with FFT convolution, or "
                         "exact trial transforms on the spectrum lattice (D_spec)")
    ap.add_argument("--spectrum", choices=["exact", "asymptotic"], default="exact",
                    help="kernel spectrum at plan time: quadrature everywhere, or the "
                         "large-frequency asymptotic form where it applies")
    ap.add_argument("--direct", choices=["auto", "always", "never"], default="auto",
                    help="direct solve of the aperture system (inverse built once per plan, "
                         "in the warm-up; its time is reported as direct_factor_ms)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both",
                    help="both: time the double-precision path, then the mixed one (headline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent incidences and requests shard across GPUs with no exchange).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 16
        a = torch.ones(n, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": int(n * 16), "launches": 3}), flush=True)
        return 0

    if args.workload == SERVED:
        return served_main(args)

    import paper_2008_01966_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    wl = W.by_name(args.workload)
    batch = args.batch or wl.batch
    cav = wl.cavity
    incs = wl.incidences
    th = [i.theta for i in incs]
    ph = [i.phi for i in incs]
    po = [i.pol for i in incs]
    fields = (torch.empty((len(incs), 3, cav.nz + 1, cav.ny + 1, cav.nx + 1),
                          dtype=torch.complex128, device="cuda") if wl.fields else None)

    def timed(precision, out, probe):
        """Create the plan (timed on its own, outside the step: the first creation computes
        the aperture data, the second takes it from the library's aperture cache), warm up,
        then time `steps` steps of solve + fields + RCS; each step ends with host-side RCS
        values, so the per-step wall times are step latencies."""
        plan_ms = []
        for _ in range(2):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            plan = P.Plan.from_cavity(cav, precision=precision, tol=wl.tol, batch=batch,
                                      direct=args.direct, operator=args.operator,
                                      spectrum=args.spectrum)
            torch.cuda.synchronize()
            plan_ms.append(1e3 * (time.perf_counter() - tp))
            if len(plan_ms) < 2:
                plan.close()

        def step():
            plan.solve_batch(th, ph, po, out=out, field=out is not None)
            sig = list(plan.rcs_many(np.arange(len(incs)), th, ph))
            return sig, plan.info()

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        probe = probe and args.probe != "none"
        if probe:
            P.probe_start(args.probe)
            torch.cuda.synchronize()
        lat, infos = [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            sig, info = step()
            lat.append(time.perf_counter() - ts)
            infos.append(info)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        probe_res = P.probe_stop() if probe else (0, 0.0, 0.0)
        plan.close()
        unknowns_step = len(incs) * infos[-1].unknowns
        res = {
            "value": args.steps * unknowns_step / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / args.steps,
            "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "plan_ms": plan_ms[0],
            "plan_ms_same_aperture": plan_ms[-1],
            "gmres_iterations_last": int(infos[-1].last_iterations),
            "lds_budget": int(infos[-1].lds_budget),
            "tbc_rows_in_place": bool(infos[-1].tbc_rows_in_place),
            "direct": bool(infos[-1].last_direct),
            "direct_factor_ms": float(infos[-1].ms_factor),
        }
        return res, sig, infos[-1], probe_res

    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    head = precisions[-1]
    if args.probe is None:
        args.probe = "tbc_cols_f32" if head == "mixed" else "tbc_cols"
    runs, sigs = {}, {}
    fields_by = {}
    for prec in precisions:
        out = None if fields is None else (fields if prec == head else torch.empty_like(fields))
        res, sig, info_p, probe_res = timed(prec, out, probe=(prec == head))
        runs[prec] = res
        sigs[prec] = sig
        fields_by[prec] = out
        if prec == head:
            info, (launches, k_ms, k_bytes) = info_p, probe_res

    unknowns_step = len(incs) * info.unknowns
    value = runs[head]["value"]
    traffic, traffic_src = measured_traffic(args.probe, wl.name)
    achieved = (k_bytes / (k_ms * 1e-3)) / 1e9 if k_ms > 0 else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": runs[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "geometry_lambda": [cav.a, cav.b, cav.c],
            "grid": [cav.nx, cav.ny, cav.nz],
            "layers": [[n, str(e)] for n, e in zip(cav.layer_nz, cav.layer_eps)],
            "incidences": len(incs),
            "unknowns_per_rhs": int(info.unknowns),
            "aperture_unknowns": int(info.n_ap),
            "fft_box": [int(info.P1), int(info.P2)],
            "precision": head,
            "tol": wl.tol,
            "batch": batch,
            "fields": bool(wl.fields),
            "step": ("all incidences (RHS, GMRES or the direct solve) + field synthesis (when "
                     "fields) + backscatter RCS; the plan (spectrum, elimination, "
                     "preconditioner) is built once before the timed region and its time "
                     "reported as plan_ms; when the direct solve is taken, its inverse is "
                     "built once in the warm-up and its time reported as direct_factor_ms"),
            "direct": args.direct,
            "tbc_operator": args.operator,
            "spectrum": args.spectrum,
            "layer_depth": None if cav.layer_depth is None else list(cav.layer_depth),
        },
        "latency_ms": {"p50": runs[head]["p50_ms"], "p99": runs[head]["p99_ms"],
                       "of": "one step"},
        "plan_ms": runs[head]["plan_ms"],
        "plan_ms_same_aperture": runs[head]["plan_ms_same_aperture"],
        "by_precision": runs,
        "gmres_iterations_last": int(info.last_iterations),
        "phases_ms_last_step": {
            "spectrum": info.ms_spectrum, "elimination": info.ms_elimination,
            "preconditioner": info.ms_preconditioner, "rhs_last": info.ms_rhs,
            "krylov_last": info.ms_krylov, "synthesis_last": info.ms_synthesis,
        },
        "roofline": {
            "kernel": args.probe,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
            "traffic": traffic,
            "traffic_source": traffic_src,
            "launches": launches,
            "avg_launch_ms": k_ms / max(launches, 1),
            "algorithmic_bytes_per_launch": k_bytes / max(launches, 1),
        },
    }
    if "fp64" in fields_by and "mixed" in fields_by:
        a64, amx = fields_by["fp64"], fields_by["mixed"]
        if a64 is not None:
            errs = [float(torch.linalg.vector_norm(amx[i] - a64[i]) /
                          torch.linalg.vector_norm(a64[i])) for i in range(len(incs))]
            out["mixed_vs_fp64_field_rel_err"] = max(errs)
        out["mixed_vs_fp64_rcs_rel_err"] = max(
            abs(sigs["mixed"][i][incs[i].pol] - sigs["fp64"][i][incs[i].pol]) /
            abs(sigs["fp64"][i][incs[i].pol]) for i in range(len(incs)))
        out["mixed_speedup_vs_fp64"] = runs["mixed"]["value"] / runs["fp64"]["value"]
    if not args.no_cpu_baseline:
        sample = args.cpu_sample or (len(incs) if len(incs) <= 2 else 1)
        sample = min(sample, len(incs))
        gpu_fields = ([fields[i].cpu().numpy() for i in range(sample)] if fields is not None
                      else None)
        base, ferr, rerr = cpu_baseline(wl, gpu_fields, sigs[head][:sample], sample)
        out["cpu_baseline"] = base
        out["field_rel_err_vs_oracle"] = ferr
        out["rcs_rel_err_vs_oracle"] = rerr
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
