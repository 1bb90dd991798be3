#!/usr/bin/env python3
"""Benchmark of the cavity-scattering hot path on one MI355X.

One step = the solve of every incidence of the workload (right-hand side, preconditioned
GMRES with the FFT-applied TBC operator), the field synthesis on all (Nz+1) x (Ny+1) x
(Nx+1) nodes and the backscatter RCS.  The plan (truncated-kernel spectrum, per-mode
z-elimination, preconditioner) is built before the timed region; its build time is
reported on its own as plan_ms.

value = unknowns solved per second = steps * incidences * n_ap * Nz / wall time.

The default workload is the batched layered cavity: 8 x 8 x 2 wavelengths, three layers
(eps_r = 4+1i, 2.5+0.5i, 1 over 25 / 50 / 25 % of the depth), 256 x 256 x 64 grid, 128
right-hand sides (8 theta in [0, 80 deg] x 8 phi x 2 polarisations) solved to 1e-10.  It
runs in double precision and then in mixed precision (the headline), and the two fields are
compared.  A prefix of the served stream (random cavities of 2-12 wavelengths, Poisson
arrivals at 40/s, replayed in real time through the library's request server) gives the
p50/p99 latency of the same JSON line.  Inputs are synthetic (the paper's workloads are
geometries, not data).

Also reported: the average-launch roofline of the dominant kernel (timed with HIP events on
its launch stream through the library's probe) and the CPU oracle timed on the host cores
on a bounded sample of the same workload (reported baseline), plus the GPU field's error
against that oracle.
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

def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


METRIC = "cavity unknowns solved/s + p50/p99 latency, mixed vs FP64 at ≤1e-8 rel err"
HBM_PEAK_GBS = 8000.0
# published vector peaks of the chip (fp32 counts packed two-wide FMA; code without packed
# math tops out at half of it, the fp64 figure)
VECTOR_PEAK_TFLOPS = {"tbc_cols_f32": 157.3, "tbc_cols": 78.6}


def fft_flops(n):
    """Nominal arithmetic of one complex transform of length n (5 n log2 n)."""
    import math
    return 5.0 * n * math.log2(n)


def tbc_cols_flops(info, nq1, bytes_per_launch, elem):
    """Algorithmic flops of one column-pass launch: per column of the 3 families of every
    right-hand side, the extension transform (length 2 nq1) in and out, the box transform
    (length P1) forward and inverse, and the product with the spectrum (6 flops per entry).
    The right-hand sides per launch come from the probe's algorithmic bytes, elem bytes per
    entry times (2 x 3 nb (M+1) P2 [X in, Y out] + P1 P2 [spectrum])."""
    P1, P2, M = int(info.P1), int(info.P2), int(info.M)
    nb = (bytes_per_launch / elem - P1 * P2) / (6.0 * (M + 1) * P2)
    per_column = 2 * fft_flops(2 * nq1) + 2 * fft_flops(P1) + 6.0 * P1
    return 3.0 * nb * P2 * per_column


def cpu_baseline(wl, gpu_fields, gpu_sigma, indices):
    """Time the CPU oracle on a bounded sample of the workload: the plan + the incidences
    `indices` (field and RCS each); gpu_fields / gpu_sigma hold the GPU results of the same
    incidences, in the same order."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import solver
    from oracle.problem import Problem

    prob = Problem.from_cavity(wl.cavity)
    t0 = time.perf_counter()
    pl = solver.plan(prob)
    fields, sig = [], []
    incs = [wl.incidences[i] for i in indices]
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
    for inc, g, o in zip(incs, gpu_sigma, sig):
        co = int(inc.pol)      # co-polarised component of this incidence
        rerr.append(float(abs(g[co] - o[co]) / abs(o[co])))
    unknowns = len(incs) * prob.unknowns
    what = ("whole workload once" if len(incs) == len(wl.incidences) else
            f"incidences {list(indices)} of {len(wl.incidences)}")
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


def measured_traffic(kernel, workload, info=None):
    """HBM bytes per launch of `kernel` on `workload` from the committed hardware-counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None when
    there is none, the kernel's sources changed since it was taken, or this run's tuned
    launch configuration (info: LDS budget, row passes in place) is not the measured one."""
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
    if info is not None and "lds_budget" in kv:
        # lds_budget 0: the library's default, 40000 bytes or CAVITY_LDS_BUDGET
        lds = int(info.lds_budget) or int(os.environ.get("CAVITY_LDS_BUDGET", "40000"))
        run_cfg = (lds, int(info.tbc_rows_in_place))
        file_cfg = (int(kv["lds_budget"]), int(kv["tbc_rows_in_place"]))
        if run_cfg != file_cfg:
            return None, (rel + f" (measured at LDS budget {file_cfg[0]}, rows in place "
                          f"{file_cfg[1]}; this run tuned {run_cfg[0]}, {run_cfg[1]})")
    return float(kv["traffic_bytes_per_launch"]), rel



SERVED = "served_stream_2000_poisson40"
DEFAULT_WORKLOAD = "batched_layered_8x8x2_256x256x64_x128"
# incidences the oracle solves for a batched workload: every 17th of the 128
ORACLE_SUBSET = (0, 17, 34, 51, 68, 85, 102, 119)


def replay_served(n_requests, streams, prec):
    """Submit the first n_requests of the served stream to the library's request server at
    their seeded Poisson arrival times (real time) and collect the results."""
    import torch

    import paper_2008_01966_amd as P
    import workloads as W

    stream = W.served_stream(n_requests)
    # warm-up on a cavity outside the stream (loads the kernels; no aperture of the stream)
    warm = P.Plan(0.75, 0.75, 0.25, 24, 24, 8, precision=prec)
    warm.solve(0.2, 0.1, 0)
    warm.close()
    torch.cuda.synchronize()
    srv = P.Server(streams=streams, precision=prec)
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
    return stream, res, t_origin


def served_summary(res, t_origin, streams, prec):
    """Latency from arrival to field and RCS ready, queueing, throughput of a replay."""
    import numpy as np

    bad = [k for k, (r, _) in enumerate(res) if r.status != 0]
    lat = np.array([r.t_done_ms - due for r, due in res])
    queue = np.array([r.t_start_ms - due for r, due in res])
    unknowns = float(sum(r.unknowns for r, _ in res))
    span_s = (max(r.t_done_ms for r, _ in res) - t_origin) * 1e-3
    its = [r.iterations for r, _ in res]
    return {
        "workload": SERVED,
        "requests": len(res),
        "arrivals": "Poisson 40/s, seed 200801966, replayed in real time",
        "streams": streams,
        "precision": prec,
        "unknowns_per_s": unknowns / span_s,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "mean": float(lat.mean()),
                       "of": "arrival to field and RCS ready"},
        "queueing_ms": {"p50": float(np.percentile(queue, 50)),
                        "p99": float(np.percentile(queue, 99))},
        "failed_requests": bad,
        "gmres_iterations": {"min": int(min(its)), "max": int(max(its))},
        "span_s": span_s,
        "step": "one request: plan (aperture data from the cache when seen before) + GMRES + "
                "field on all nodes + backscatter RCS",
    }


def served_oracle(stream, res, prec, budget_s, max_side=None):
    """The oracle serves the stream's requests in order, serially (those of side at most
    max_side when given), for about budget_s of host time (at least one); the same requests
    are solved alone on the GPU with their field kept and compared with the oracle's field
    and RCS; the server's RCS is compared too."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info

    import paper_2008_01966_amd as P
    from oracle import solver
    from oracle.problem import Problem

    t_cpu = 0.0
    done, unknowns, errs = 0, 0, []
    for k, (req, (r, _)) in enumerate(zip(stream, res)):
        cav = req.workload.cavity
        if max_side is not None and max(cav.a, cav.b) > max_side:
            continue
        inc = req.workload.incidences[0]
        t0 = time.perf_counter()
        prob = Problem.from_cavity(cav)
        pl = solver.plan(prob)
        sol = solver.solve(pl, inc.theta, inc.phi, inc.pol, tol=1e-13)
        field = solver.field_out(pl, sol)
        sig = solver.backscatter(pl, sol, inc.theta, inc.phi)
        t_cpu += time.perf_counter() - t0
        done += 1
        unknowns += prob.unknowns
        plan = P.Plan.from_cavity(cav, precision=prec, batch=1)
        g = plan.solve(inc.theta, inc.phi, inc.pol).cpu().numpy()
        plan.close()
        co = inc.pol
        errs.append({"request": k, "side": cav.a, "grid": [cav.nx, cav.ny, cav.nz],
                     "field_rel_err": float(np.linalg.norm(g - field) / np.linalg.norm(field)),
                     "rcs_rel_err_server": float(abs(r.sigma[co] - sig[co]) / sig[co])})
        if t_cpu > budget_s:
            break
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    torch.cuda.synchronize()
    which = "" if max_side is None else f" of side <= {max_side:g} wavelengths"
    return ({"value": unknowns / max(t_cpu, 1e-9), "unit": "unknowns/s", "cores": int(threads),
             "kind": "oracle",
             "sample": f"first {done} requests{which} of the stream served serially, "
                       f"{t_cpu:.1f} s of oracle time"}, errs)


def served_main(args) -> int:
    """The whole served stream on its own: value = unknowns of all requests / (last
    completion - first arrival)."""
    import torch

    torch.cuda.set_device(0)
    prec = "mixed" if args.precision in ("mixed", "both") else "fp64"
    stream, res, t_origin = replay_served(args.requests, args.streams, prec)
    summ = served_summary(res, t_origin, args.streams, prec)
    out = {
        "metric": METRIC,
        "value": summ["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": len(res),
        "warmup": 1,
        "ms_per_step": summ["latency_ms"]["mean"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {k: summ[k] for k in ("workload", "requests", "arrivals", "streams",
                                         "precision", "step")},
        "latency_ms": summ["latency_ms"],
        "queueing_ms": summ["queueing_ms"],
        "failed_requests": summ["failed_requests"],
        "gmres_iterations": summ["gmres_iterations"],
        "span_s": summ["span_s"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["oracle_check"] = served_oracle(stream, res, prec, 20.0)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
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
                    help="incidences the CPU oracle solves (0: all when at most 2, the "
                         "subset 0, 17, ..., 119 of a 128-incidence batch, else 1)")
    ap.add_argument("--requests", type=int, default=2000, help="served stream: requests")
    ap.add_argument("--streams", type=int, default=4, help="served stream: concurrent requests")
    ap.add_argument("--served-prefix", type=int, default=320,
                    help="requests of the served stream replayed after the batched workload "
                         "for the p50/p99 latency of the same line (0: none)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain double-precision run (one incidence per solve)")
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

    def timed(precision, out, probe, nb):
        """Create the plan (timed on its own, outside the step: the first creation computes
        the aperture data, the second takes it from the library's aperture cache), warm up,
        then time `steps` steps of solve + fields + RCS; each step ends with host-side RCS
        values, so the per-step wall times are step latencies."""
        plan_ms = []
        for _ in range(2):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            plan = P.Plan.from_cavity(cav, precision=precision, tol=wl.tol, batch=nb,
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
        slow = int(np.argmax(lat))
        res = {
            "value": args.steps * unknowns_step / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / args.steps,
            "batch": nb,
            "step_ms": [round(1e3 * v, 3) for v in lat],
            "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            # phases of the last lockstep group of the slowest step (device time)
            "slowest_step": {"index": slow, "ms": 1e3 * lat[slow],
                             "krylov_ms_last_group": infos[slow].ms_krylov,
                             "synthesis_ms_last_group": infos[slow].ms_synthesis,
                             "gmres_iterations": int(infos[slow].last_iterations)},
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
    other = None
    if fields is not None and len(precisions) > 1:
        other = torch.empty_like(fields)
    if args.precision == "both" and len(incs) > 1 and not args.no_plain:
        # the plain method: double precision, one incidence per solve (no lockstep group)
        res, _, _, _ = timed("fp64", other, probe=False, nb=1)
        runs["fp64_plain"] = res
        log(f"fp64, one incidence per solve: {res['ms_per_step']:.1f} ms per step")
    for prec in precisions:
        out = None if fields is None else (fields if prec == head else other)
        res, sig, info_p, probe_res = timed(prec, out, probe=(prec == head), nb=batch)
        runs[prec] = res
        sigs[prec] = sig
        log(f"{prec}, batch {batch}: {res['ms_per_step']:.1f} ms per step")
        fields_by[prec] = out
        if prec == head:
            info, (launches, k_ms, k_bytes) = info_p, probe_res

    value = runs[head]["value"]
    traffic, traffic_src = measured_traffic(args.probe, wl.name, info)
    achieved = (k_bytes / (k_ms * 1e-3)) / 1e9 if k_ms > 0 else None
    avg_ms = k_ms / max(launches, 1)
    bytes_per_launch = k_bytes / max(launches, 1)
    roofline = {
        "kernel": args.probe,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
        "traffic": traffic,
        "traffic_source": traffic_src,
        "launches": launches,
        "avg_launch_ms": avg_ms,
        "algorithmic_bytes_per_launch": bytes_per_launch,
    }
    if args.probe in VECTOR_PEAK_TFLOPS and k_ms > 0:
        # the column pass runs its four transforms per column in LDS on one HBM round trip:
        # about 25 flop per byte in single precision, above the vector ALU's ridge, so the
        # vector ALU bounds it; the HBM figures stay beside it
        elem = 8 if args.probe.endswith("_f32") else 16
        flops = tbc_cols_flops(info, wl.cavity.tbc_oversample * wl.cavity.nx, bytes_per_launch,
                               elem)
        tflops = flops / (avg_ms * 1e-3) / 1e12
        peak = VECTOR_PEAK_TFLOPS[args.probe]
        roofline.update({
            "bound": "alu", "achieved": tflops, "peak": peak, "unit": "TFLOP/s",
            "frac": tflops / peak, "algorithmic_flops_per_launch": flops,
            "hbm_achieved_gbs": achieved, "hbm_peak_gbs": HBM_PEAK_GBS,
            "hbm_frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
        })
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
                       "of": "one step (all incidences)"},
        "plan_ms": runs[head]["plan_ms"],
        "plan_ms_same_aperture": runs[head]["plan_ms_same_aperture"],
        "by_precision": runs,
        "gmres_iterations_last": int(info.last_iterations),
        "phases_ms_last_step": {
            "spectrum": info.ms_spectrum, "elimination": info.ms_elimination,
            "preconditioner": info.ms_preconditioner, "rhs_last": info.ms_rhs,
            "krylov_last": info.ms_krylov, "synthesis_last": info.ms_synthesis,
        },
        "roofline": roofline,
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
        if "fp64_plain" in runs:
            out["mixed_speedup_vs_fp64_plain"] = runs["mixed"]["value"] / runs["fp64_plain"]["value"]
    del other
    if not args.no_cpu_baseline:
        if args.cpu_sample:
            idx = list(range(min(args.cpu_sample, len(incs))))
        elif len(incs) <= 2:
            idx = list(range(len(incs)))
        elif len(incs) == 128:
            idx = list(ORACLE_SUBSET)
        else:
            idx = [0]
        gpu_fields = ([fields[i].cpu().numpy() for i in idx] if fields is not None else None)
        log(f"oracle on incidences {idx}")
        base, ferr, rerr = cpu_baseline(wl, gpu_fields, [sigs[head][i] for i in idx], idx)
        log(f"oracle done: {base['sample']}")
        del gpu_fields
        out["cpu_baseline"] = base
        out["field_rel_err_vs_oracle"] = ferr
        out["rcs_rel_err_vs_oracle"] = rerr
    del fields, fields_by
    torch.cuda.empty_cache()
    if args.served_prefix > 0:
        prec = "mixed" if args.precision in ("mixed", "both") else "fp64"
        log(f"served stream, first {args.served_prefix} requests")
        stream, res, t_origin = replay_served(args.served_prefix, args.streams, prec)
        summ = served_summary(res, t_origin, args.streams, prec)
        log(f"served: p50 {summ['latency_ms']['p50']:.2f} ms, p99 {summ['latency_ms']['p99']:.2f} ms")
        if not args.no_cpu_baseline:
            base, errs = served_oracle(stream, res, prec, 10.0, max_side=4.0)
            summ["oracle_check"] = errs
            summ["cpu_baseline"] = base
        out["served"] = summ
        out["latency_ms"] = dict(summ["latency_ms"])
        out["latency_ms"]["of"] = (f"served stream, first {len(res)} requests: "
                                   "arrival to field and RCS ready")
        out["step_latency_ms"] = {"p50": runs[head]["p50_ms"], "p99": runs[head]["p99_ms"],
                                  "of": "one step of the batched workload"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
