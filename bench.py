"""Benchmark of the FC-Gram RK step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line: grid-point RK-substeps per second (physical points
nx*ny*nz times RK stages, o = 2 per step) over K timed steps after W warmup
steps, with inputs resident in HBM; the roofline of the dominant kernel
(algorithmic bytes per launch over its mean event-timed duration on the
solver stream); and the FP64 oracle timed on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
from dataclasses import replace
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("grid-point RK-substeps/sec (FP64 & mixed) + p50/p99 step latency in batched "
          "serving")
UNIT = "grid-point RK-substeps/s"
HBM_PEAK_GBPS = 8000.0
BREAKDOWN_STEPS = 2  # steps with every kernel class event-timed, before the timed region
CSRC = os.path.join(ROOT, "paper_2002_01392_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    """Hash of the device code and the host code that launches it (the serving
    loop, which launches nothing itself, is left out)."""
    h = hashlib.sha256()
    for fn in sorted(os.listdir(CSRC)):
        if fn == "fcns_server.cpp":
            continue
        with open(os.path.join(CSRC, fn), "rb") as fh:
            h.update(fn.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def field_bytes(w):
    """(M, S): bytes of one complex128 mixed field and one continued field."""
    nkx = w.nx // 2 + 1
    M = w.nz * w.ny * nkx * 16
    S = (w.nz + w.C) * w.ny * nkx * 16
    return M, S


# timing classes that span several kernels (never the roofline kernel)
CHAINS = ("xy_slabs",)


def algorithmic_bytes(w, cls, stage, keep_pressure=False):
    """Bytes one launch of a kernel class must move (each array read or written
    once).  F = transported fields, M / S = one mixed / continued field."""
    F = w.nfields
    M, S = field_bytes(w)
    rb = w.boussinesq
    if cls == "y_back_dy":
        return 3 * F * M            # read q^, write q and dq/dy
    if cls == "y_back_dz":
        return 2 * F * M
    if cls == "x_nl":
        return 4 * F * M            # read q, dq/dy, dq/dz; write NL
    if cls == "y_fwd":
        return 2 * F * M
    if cls == "z_stageA":
        reads_state = F * S if stage == 1 else 2 * F * S   # V^t (= W at stage 1), W
        return F * M + reads_state + F * S + (2 * M if rb else 0)
    if cls == "z_stageB":
        return 6 * S + (M if keep_pressure else 0)   # read V*, write V
    if cls == "z_back":
        return F * S + 2 * F * M                     # read V, write v and dv/dz
    if cls == "z_pass":
        # the fused z pass: read NL, V^t and W (W = V^t at stage 1), write the
        # new state and its v, dv/dz
        reads_state = F * S if stage == 1 else 2 * F * S
        return F * M + reads_state + F * S + 2 * F * M + (M if keep_pressure else 0)
    if cls == "xy_slabs":
        # the y back, x and y forward passes of one stage run slab by slab in z
        # (several launches): their arrays, each read or written once
        return 11 * F * M
    raise KeyError(cls)


def pass_model_bytes(w):
    """The four-pass model per substep: 14 F M + 3 F S."""
    M, S = field_bytes(w)
    return 14 * w.nfields * M + 3 * w.nfields * S


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(w, steps=1, side=128):
    """The FP64 oracle (as it stands) on a bounded sample: `steps` RK steps of
    the same workload parameters and wall-normal grid on a reduced horizontal
    grid, timed twice: with its matrix products (the oracle's own DFTs and the
    continuation) on every host core, and on one thread.  numpy's elementwise
    work is single-threaded either way."""
    from dataclasses import replace
    from threadpoolctl import threadpool_limits

    from oracle.ns import Oracle, Problem
    nxs = max(16, min(w.nx, side))
    nys = max(16, min(w.ny, side))
    ws = replace(w, nx=nxs, ny=nys, lx=w.lx * nxs / w.nx, ly=w.ly * nys / w.ny)
    v0, th0 = ws.initial_state()
    pts = ws.nx * ws.ny * ws.nz
    cores = host_cores()
    rates = {}
    for threads in (cores, 1):
        with threadpool_limits(limits=threads):
            o = Oracle(Problem(**ws.problem_kwargs()))
            o.set_state(v0, th0)
            t0 = time.perf_counter()
            o.rk_step(ws.dt, steps)
            el = time.perf_counter() - t0
        rates[threads] = (pts * 2 * steps / el, el)
        del o
    return {"value": rates[cores][0], "unit": UNIT, "cores": cores, "kind": "oracle",
            "one_core": {"value": rates[1][0], "cores": 1},
            "sample": (f"{steps} RK2 step(s) ({2 * steps} substeps) of {w.name}'s parameters, "
                       f"nz={w.nz}, C={w.C}, on a {nxs}x{nys} horizontal grid (box scaled to "
                       f"keep dx, dy): {rates[cores][1]:.1f} s with BLAS on {cores} threads, "
                       f"{rates[1][1]:.1f} s on 1; the oracle's own FFTs (no FFT library)")}


def precision_run(name="channel_256x256x257", steps=100, warmup=2):
    """The mixed-precision step on the channel grid: rate of the FP64 and the
    mixed step (same initial state, same number of steps), and the mixed
    result's per-field relative L2 distance from the FP64 one (which matches
    the FP64 oracle to 1e-11 in the parity tests)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01392_amd import Solver

    w = W.get(name)
    v0, th0 = w.initial_state()
    v0 = torch.from_numpy(v0)
    out = {}
    res = {}
    for prec in ("fp64", "mixed"):
        s = Solver.from_workload(w, keep_pressure=True, precision=prec)
        s.set_state(v0)
        out[prec + "_autotune"] = s.autotune()
        s.rk_step(w.dt, warmup)
        s.set_state(v0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.rk_step(w.dt, steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        v, _, pr = s.get_state(pressure=True)
        torch.cuda.synchronize()
        res[prec] = (v.cpu().numpy(), pr.cpu().numpy())
        out[prec] = {"ms_per_step": ms / steps,
                     "value": w.nx * w.ny * w.nz * 2 * steps / (ms / 1e3)}
        s.close()
        del s
    (vd, pd), (vm, pm) = res["fp64"], res["mixed"]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err = {c: rel(vm[i], vd[i]) for i, c in enumerate("uvw")}
    err["p"] = rel(pm, pd)
    return {"workload": name, "steps": steps, "unit": UNIT,
            "fp64": out["fp64"], "mixed": out["mixed"],
            "autotune": {"fp64": out["fp64_autotune"], "mixed": out["mixed_autotune"]},
            "speedup": out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"],
            "rel_l2_vs_fp64": err,
            "note": "nonlinear term in FP32 (back transforms of the state, x and y FFTs, "
                    "products, mixed-space arrays); FP64 state, FC extension, the "
                    "transforms that form v*, and the projection"}


def serving_run(max_active=8, max_bytes=64 << 30, n=64, rate=20.0, steps=20, max_large=1,
                large_points=4 << 20):
    """The serving workload: n requests with Poisson arrivals at `rate`/s, each
    a `steps`-step solve (channel or Rayleigh-Benard, side 32..192), served by
    the library's request loop with up to max_active overlapping requests, and
    the same arrivals served one at a time (max_active = 1) for comparison.
    Inputs are generated before the clock starts; arrivals are replayed in
    real time; latency = result detected - submission (host clock)."""
    import numpy as np

    import workloads as W
    from paper_2002_01392_amd import Server, workload_problem

    import torch

    from paper_2002_01392_amd import Solver

    stream = W.serving_stream(n=n, rate=rate, steps=steps)
    reqs = []
    for t, w in stream:
        v0, th0 = w.initial_state()
        prob, tab = workload_problem(w)
        reqs.append((t, w, prob, tab, v0, th0))
    # launch choices tuned once per shape before the clock starts (a serving
    # system keeps such a table; the contexts it creates take them)
    tuned = {}
    for _, w, prob, _tab, v0, th0 in reqs:
        key = (w.nx, w.ny, w.nz, w.C, w.boussinesq)
        if key in tuned:
            continue
        s = Solver.from_workload(w)
        s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
        s.autotune()
        tuned[key] = (prob, s.choices())
        s.close()
        del s
    torch.cuda.empty_cache()

    def run(slots, replay=True, tune=True, mix=True):
        srv = Server(max_active=slots, max_bytes=max_bytes)
        if tune:
            for prob, text in tuned.values():
                srv.set_choices(prob, text)
        if mix and slots > 1:
            # at most max_large of the largest shapes (192^2 x 193: 7.1e6
            # points) at a time (one keeps their latency tail short); the
            # smaller ones fill the device around them
            srv.set_mix(max_large, large_points)
        t0 = srv.now()
        ids, k = [], 0
        while True:
            now = srv.now() - t0
            while k < len(reqs) and (reqs[k][0] <= now or not replay):
                _, w, prob, _tab, v0, th0 = reqs[k]
                ids.append((srv.submit(prob, v0, th0, w.dt, w.steps), w))
                k += 1
            _, _, done = srv.poll()
            if k == len(reqs) and done == len(reqs):
                break
        lat, step_ms, work, t_end, finite = [], [], 0, 0.0, True
        for rid, w in ids:
            _, _, info = srv.result(rid)
            finite = finite and info["finite"]
            lat.append(1e3 * (info["t_done"] - info["t_submit"]))
            step_ms.extend(srv.step_times(rid).tolist())
            work += w.nx * w.ny * w.nz * 2 * w.steps
            t_end = max(t_end, info["t_done"] - t0)
        srv.close()
        t_first = reqs[0][0] if replay else 0.0
        pct = lambda a, q: float(np.percentile(np.asarray(a), q))
        return {"max_active": slots, "makespan_s": t_end - t_first,
                "value": work / (t_end - t_first), "unit": UNIT,
                "request_ms_p50": pct(lat, 50), "request_ms_p99": pct(lat, 99),
                "step_ms_p50": pct(step_ms, 50), "step_ms_p99": pct(step_ms, 99),
                "all_finite": finite}

    seq = run(1)
    bat = run(max_active)
    # the same requests all submitted at once (offered load above capacity)
    seq_sat = run(1, replay=False)
    bat_sat = run(max_active, replay=False)
    # and with the default launch choices (no tuning table) and plain
    # arrival-order admission
    seq_def = run(1, replay=False, tune=False)
    bat_def = run(max_active, replay=False, tune=False, mix=False)
    return {"requests": n, "rate_per_s": rate, "steps_each": steps,
            "sides": list(W.SERVING_SIDES), "tuned_shapes": len(tuned),
            "mix_limit": {"max_large": max_large, "large_points": large_points},
            "batched": bat, "sequential": seq,
            "throughput_gain": bat["value"] / seq["value"],
            "p99_request_gain": seq["request_ms_p99"] / bat["request_ms_p99"],
            "saturated": {"batched": bat_sat, "sequential": seq_sat,
                          "throughput_gain": bat_sat["value"] / seq_sat["value"],
                          "p99_request_gain": seq_sat["request_ms_p99"]
                          / bat_sat["request_ms_p99"]},
            "saturated_default_choices_arrival_order": {
                "batched": bat_def, "sequential": seq_def,
                "throughput_gain": bat_def["value"] / seq_def["value"],
                "p99_request_gain": seq_def["request_ms_p99"] / bat_def["request_ms_p99"]}}


def batch_leg(steps=20, sides=(32, 64, 96), per_side=3):
    """Small problems of mixed shapes (the serving stream's smaller sizes,
    channel and Rayleigh-Benard, C = 31): one after another, interleaved on
    their own streams (fcns_batch_step), and with one fused z-pass launch per
    stage for all of them (fcns_batch_run)."""
    import torch

    import workloads as W
    from paper_2002_01392_amd import Batch, Solver, batch_step

    ws = []
    for i, side in enumerate([s for s in sides for _ in range(per_side)]):
        if i % 2:
            w = W.channel(side, side, side + 1, 2000.0, C=31, seed=900 + i)
        else:
            w = W.rayleigh_benard(side, side, side + 1, 1e6, C=31, seed=900 + i)
        ws.append(replace(w, dt=W.stable_dt(w)))
    states = [w.initial_state() for w in ws]

    def fresh():
        out = []
        for w, (v0, th0) in zip(ws, states):
            s = Solver.from_workload(w, stream=torch.cuda.Stream())
            s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
            s.autotune()
            s.set_finite_check("deferred")
            out.append(s)
        torch.cuda.synchronize()
        return out

    work = sum(w.nx * w.ny * w.nz * 2 * steps for w in ws)
    res = {"members": [w.name.split("_", 1)[-1] if "_" in w.name else w.name for w in ws],
           "steps": steps, "unit": UNIT}
    for mode in ("sequential", "interleaved", "one_launch"):
        S = fresh()
        b = Batch(S, [w.dt for w in ws]) if mode == "one_launch" else None
        for _ in range(2):   # warmup, then timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "sequential":
                for s, w in zip(S, ws):
                    s.rk_step(w.dt, steps)
                    s.synchronize()
            elif mode == "interleaved":
                batch_step(S, [w.dt for w in ws], [steps] * len(ws))
            else:
                b.run(steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        for s in S:
            s.check_finite()
        res[mode] = {"s": el, "value": work / el}
        if b is not None:
            b.close()
        for s in S:
            s.close()
    res["one_launch_vs_sequential"] = res["one_launch"]["value"] / res["sequential"]["value"]
    res["one_launch_vs_interleaved"] = res["one_launch"]["value"] / res["interleaved"]["value"]
    return res


def graph_run(name="channel_32x32x33", steps=200, warmup=5):
    """Launch-bound small problem: eager rk_step against the replayed HIP graph
    of one step (same state, same steps)."""
    import torch

    import workloads as W
    from paper_2002_01392_amd import Solver

    w = W.get(name)
    v0, th0 = w.initial_state()
    out = {"workload": name, "steps": steps, "unit": UNIT}
    for mode in ("eager", "graph"):
        s = Solver.from_workload(w)
        s.set_finite_check("deferred")
        s.set_state(torch.from_numpy(v0))
        run = s.rk_step if mode == "eager" else s.rk_graph
        run(w.dt, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run(w.dt, 1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = {"ms_per_step": 1e3 * el / steps,
                     "value": w.nx * w.ny * w.nz * 2 * steps / el}
        s.check_finite()
        s.close()
    out["speedup"] = out["eager"]["ms_per_step"] / out["graph"]["ms_per_step"]
    return out


def load_traffic(w, kernel, src_hash):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources and workload."""
    p = os.path.join(PROFILES, f"pmc_{kernel}_{w.name}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != src_hash or d.get("workload") != w.name:
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rb_512x512x257")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing", type=int, default=1,
                    help="1: event-time every kernel class over %d steps before the timed "
                         "region and the dominant class inside it; 2: every class inside "
                         "it; 0: none" % BREAKDOWN_STEPS)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run on the channel grid")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch choices")
    ap.add_argument("--choices", default="",
                    help="apply these launch choices (the 'choices' text of an earlier run) "
                         "instead of autotuning")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP graph comparison")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the one-launch batch of small mixed shapes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 1 GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01392_amd import Solver

    w = W.get(args.workload)
    print(f"[bench] workload {w.name}: building initial state", file=sys.stderr, flush=True)
    v0, th0 = w.initial_state()
    s = Solver.from_workload(w)
    s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
    del v0, th0
    torch.cuda.synchronize()
    tuned = None
    if args.choices:
        # launch choices saved from an earlier run (no autotuning trials, so a
        # profiler sees only the steps)
        s.set_choices(args.choices)
        tuned = "given"
    elif not args.no_autotune:
        print("[bench] autotune", file=sys.stderr, flush=True)
        tuned = s.autotune()
    choices = s.choices()
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    s.rk_step(w.dt, args.warmup)
    torch.cuda.synchronize()

    breakdown = {}
    if args.timing == 1:
        # every class event-timed over a few steps before the timed region
        # (per-kernel breakdown, and which class dominates); in the timed
        # region only the dominant class carries events
        s.set_timing(True)
        s.timing_reset()
        s.rk_step(w.dt, BREAKDOWN_STEPS)
        breakdown = s.timing_report()
        tot = {k: ms for k, (n, ms) in breakdown.items() if n > 0 and k not in CHAINS}
        s.set_timing(True, classes=[max(tot, key=tot.get)])
        s.timing_reset()
    elif args.timing:
        s.set_timing(True)
        s.timing_reset()
    stream = s.stream
    # the steps stay asynchronous in the timed region; the non-finite flag
    # is read once after it
    s.set_finite_check("deferred")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        s.rk_step(w.dt, 1)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    total_ms = float(ev[0].elapsed_time(ev[-1]))
    rep = s.timing_report() if args.timing else {}
    try:
        s.check_finite()
        finite = True
    except Exception:
        finite = False
    torch.cuda.synchronize()

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    pts = w.nx * w.ny * w.nz
    substeps = 2 * args.steps
    ms_per_step = total_ms / args.steps
    value = pts * substeps / (total_ms / 1e3)

    roof = None
    kernels = {}
    src_hash = kernel_source_hash()
    if rep:
        tot = {k: ms for k, (n, ms) in rep.items() if n > 0 and k not in CHAINS}
        dom = max(tot, key=tot.get)
        n_dom, ms_dom = rep[dom]
        per_launch_s = ms_dom / n_dom / 1e3
        b = 0.5 * (algorithmic_bytes(w, dom, 1) + algorithmic_bytes(w, dom, 2))
        ach = b / per_launch_s / 1e9
        traffic = load_traffic(w, dom, src_hash)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "bytes_per_launch": int(b), "mean_launch_ms": round(ms_dom / n_dom, 4)}
        brk = breakdown if breakdown else rep
        btot = sum(ms for n, ms in brk.values() if n > 0)
        for k, (n, ms) in brk.items():
            if n == 0:
                continue
            bk = 0.5 * (algorithmic_bytes(w, k, 1) + algorithmic_bytes(w, k, 2))
            kernels[k] = {"launches": n, "mean_ms": round(ms / n, 4),
                          "GBps": round(bk / (ms / n / 1e3) / 1e9, 1),
                          "share": round(ms / btot, 4)}
    pm = pass_model_bytes(w)
    pass_model = {"bytes_per_substep": pm,
                  "GBps": round(pm / (total_ms / 1e3 / substeps) / 1e9, 1),
                  "frac": round(pm / (total_ms / 1e3 / substeps) / 1e9 / HBM_PEAK_GBPS, 4)}

    mixed = None
    s.close()
    del s
    torch.cuda.empty_cache()
    if not args.no_mixed:
        print("[bench] mixed precision on the channel grid", file=sys.stderr, flush=True)
        mixed = precision_run()

    graph = None
    if not args.no_graph:
        print("[bench] HIP graph replay on the small channel", file=sys.stderr, flush=True)
        graph = graph_run()

    batch = None
    if not args.no_batch:
        print("[bench] small mixed shapes: sequential, interleaved, one launch", file=sys.stderr,
              flush=True)
        batch = batch_leg()

    serving = None
    if not args.no_serving:
        print("[bench] serving: 64 requests, sequential then overlapped", file=sys.stderr,
              flush=True)
        serving = serving_run()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, steps=2)

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "box": [w.lx, w.ly, w.lz],
                   "fc_d": w.d, "fc_C": w.C, "N_prime": w.nz + w.C, "fields": w.nfields,
                   "dt": w.dt, "rk_order": 2, "nu": w.nu, "kappa": w.kappa, "gamma": w.gamma,
                   "forcing_x": w.forcing_x},
        "step_ms_p50": float(np.percentile(step_ms, 50)),
        "step_ms_p99": float(np.percentile(step_ms, 99)),
        "wall_s": wall, "state_finite": finite,
        "roofline": roof, "pass_model": pass_model, "kernels": kernels,
        "kernels_timed": ("%d steps before the timed region, every class event-timed; in "
                          "the timed region only the roofline kernel" % BREAKDOWN_STEPS)
        if breakdown else "the timed region",
        "precision": mixed,
        "serving": serving, "graph": graph, "batch": batch, "autotune": tuned, "choices": choices,
        "cpu_baseline": cpu, "kernel_source_hash": src_hash,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
