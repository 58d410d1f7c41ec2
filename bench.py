#!/usr/bin/env python3
"""Throughput of the sliced multi-amplitude contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C2]
                    [--precision c64|chalf] [--slice-batch B] [--no-cpu-baseline]

One step is one complete pass of the hot path over the workload's batch:
the slice-invariant (stem) nodes, every slice of the sliced network in
batches of B slices (gathered branch contractions over the reuse tree), the
FP64 slice-sum into the amplitudes and the FP64 linear XEB.  Inputs (leaf
tensors, reuse maps, offset tables) are resident in HBM before the timed
region; planning and upload are reported separately.

Prints one JSON line: amplitudes/s of the whole job (value), sustained
complex TFLOP/s, the error of the amplitudes against the stored FP64
oracle values, a roofline entry for the dominant kernel (HIP-event timings
of a profiled pass on the plan's stream) and the oracle timed on the host
cores on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "fp16": 2516.6}  # dense MFMA
PEAK_HBM_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="C2", choices=["C1", "C2", "C3", "C4", "C5"])
    p.add_argument("--max-est-s", type=float, default=100.0,
                   help="uneven batch (C5): leave out circuits whose plan's estimated time exceeds this")
    p.add_argument("--precision", default="c64", choices=["c64", "chalf"])
    p.add_argument("--slice-batch", type=int, default=0, help="0 = workload default")
    p.add_argument("--trials", type=int, default=32, help="order-search candidates")
    p.add_argument("--partition-trials", type=int, default=-1,
                   help="bisection candidates of the order search (-1: 16 for the 36- and 53-qubit "
                        "workloads, none otherwise)")
    p.add_argument("--slice-subset", type=int, default=0, metavar="N",
                   help="time N consecutive slices (seeded start) instead of all of them and project the "
                        "full-job rate (the large workloads); 0 = every slice")
    p.add_argument("--replan", action="store_true",
                   help="6x6 and 53-qubit workloads: search a plan instead of loading the stored one")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--beside", action="store_true",
                   help="complex64 runs: also time complex-half on the same plan (default for the small workloads)")
    p.add_argument("--no-beside", action="store_true")
    p.add_argument("--no-autotune", action="store_true", help="keep the heuristic MFMA tile choice")
    p.add_argument("--profile-out", default="", help="write the per-step profile as JSON")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of MIB MiB five times (calibrates the "
                        "HBM byte counters of a profiler against a known traffic) and exit")
    return p.parse_args()


def copy_probe(mib: int) -> None:
    """Five launches of torch's copy kernel moving exactly mib MiB in and out."""
    import torch
    n = mib << 18  # float32 elements
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    best = min(ms)
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5,
                      "best_ms": best, "copy_gbs": 2 * n * 4 / (best / 1e3) / 1e9}))


TUNING = os.path.join(ROOT, "paper_2212_04749_amd", "tuning_mi355x.json")


def autotune(run) -> None:
    """Pick tile configurations with the library's autotuner, starting from
    $MATNC_AUTOTUNE_CACHE if set, else from a scratch copy of the shipped
    MI355X choices (the step classes of the default workloads, measured with
    this library), so that a default run uses the configurations its profile
    was taken with; classes not in the file are timed and added to the copy
    only, which is removed afterwards."""
    env = os.environ.get("MATNC_AUTOTUNE_CACHE")
    if env:
        run.autotune(reps=3, cache_path=env)
        return
    import shutil
    import tempfile
    fd, path = tempfile.mkstemp(prefix="matnc_tune_", suffix=".json")
    os.close(fd)
    try:
        shutil.copyfile(TUNING, path)
        run.autotune(reps=3, cache_path=path)
    finally:
        os.remove(path)


def workload_description(name, w, info, spec):
    g = w.grid
    shape = f"{g.rows}x{g.cols}" + (f" minus {len(g.removed)} site" if g.removed else "")
    return {
        "workload": f"{name}: {shape} grid RQC ({w.n_qubits} qubits), depth {w.depth}, "
                    f"fSim(pi/2,pi/6), {w.k} uniform bitstrings" +
                    (f" x 2^{len(w.open_qubits)} open legs" if w.open_qubits else "") +
                    f", rank cap {spec.cap}, {info.n_slices} slices",
        "n_qubits": w.n_qubits,
        "depth": w.depth,
        "bitstrings": w.k,
        "open_qubits": len(w.open_qubits),
        "amplitudes": int(info.n_amplitudes),
        "rank_cap": spec.cap,
        "n_slices": int(info.n_slices),
        "max_rank": int(info.max_rank),
        "cmac_total": float(info.cmac_total),
        "kS_over_Sk": float(info.n_unique * info.cmac_single / info.cmac_multi),
        "plan": spec.method,
    }


def reference_error(name, run, amps_np):
    """Relative error vs the stored FP64 oracle amplitudes, where stored."""
    import numpy as np
    path = {"C2": "c2_subset.json", "C1": None}.get(name)
    if name == "C1":
        from oracle import statevector
        from workload import CONFIGS
        w = CONFIGS["C1"]
        ref = statevector.amplitudes(w.circuit(), w.bitstrings())
        got = amps_np[:, 0]
    elif path and os.path.exists(os.path.join(ROOT, "tests", "golden", path)):
        g = json.load(open(os.path.join(ROOT, "tests", "golden", path)))
        ref = np.array([complex(a, b) for a, b in g["amps"]])
        got = amps_np[np.array(g["indices"]), 0]
    else:
        return None
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    max_over_rms = float(np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)))
    n = run.net.n_qubits
    xeb_gpu = float(np.ldexp(np.mean(np.abs(got) ** 2), n) - 1)
    xeb_ref = float(np.ldexp(np.mean(np.abs(ref) ** 2), n) - 1)
    return {"rel_err": err, "max_abs_err_over_rms": max_over_rms, "samples": int(len(ref)),
            "xeb_abs_err_on_samples": abs(xeb_gpu - xeb_ref)}


def roofline(run, precision, n_batches, nb_last, workload):
    """Roofline of the dominant launch of a profiled pass.  Every contraction
    step is one launch of one kernel configuration on one shape; the
    dominant one is the step with the largest share of the pass
    (slice-dependent steps run once per slice batch).  Its bound is the
    larger of its algorithmic flops over the MFMA peak of its kernel and its
    algorithmic bytes over the HBM peak, and achieved is that quantity per
    launch over the launch's time.  Also returns per-kernel-id aggregates
    and the pass's summed per-step roofline time (ms)."""
    prof = run.profile(0, min(run.slice_batch, run.n_slices))
    per = {}
    steps = []
    t_roof = 0.0  # sum over steps of max(flops / MFMA peak, bytes / HBM peak), ms
    for j, ((ms, kid, cmac, by), dep) in enumerate(zip(prof, run.step_dep())):
        if ms < 0:
            continue
        reps = n_batches if dep else 1
        # 100/200 + c: FP32 MFMA (complex64, and the FP32 steps of
        # complex-half); 300/400 + c: FP16 MFMA; 0: streaming (vector ALU)
        peak = PEAK_TFLOPS["fp16" if kid >= 300 else "fp32"]
        tf, tb = 8 * cmac / (peak * 1e12), by / (PEAK_HBM_GBS * 1e9)
        t_roof += reps * max(tf, tb) * 1e3
        e = per.setdefault(kid, {"ms": 0.0, "cmac": 0.0, "bytes": 0.0, "launches": 0})
        e["ms"] += ms * reps
        e["cmac"] += cmac * reps
        e["bytes"] += by * reps
        e["launches"] += reps
        steps.append((ms * reps, j, ms, kid, cmac, by, reps, tf, tb, peak))
    total = sum(x[0] for x in steps)
    share, j, ms, kid, cmac, by, reps, tf, tb, peak = max(steps)
    t = ms / 1e3
    if kid >= 100 and tf >= tb:
        r = {"bound": "mfma", "achieved": 8 * cmac / t / 1e12, "peak": peak, "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": by / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = pmc_traffic(workload, precision, kid, j)
    r["algorithmic_bytes_per_launch"] = by
    r["algorithmic_flops_per_launch"] = 8 * cmac
    r["kernel"] = ("streaming" if kid < 100 else
                   f"{'fp16' if kid >= 300 else 'fp32'} mfma{' fan-out' if (kid // 100) % 2 == 0 else ''} "
                   f"cfg {kid % 100}") + f", step {j}"
    r["kernel_id"] = kid
    r["step"] = j
    r["launches"] = reps
    r["mean_launch_ms"] = ms
    r["share_of_step"] = share / total
    return r, per, t_roof


def pmc_traffic(workload: str, precision: str, kernel_id: int, step: int):
    """HBM bytes per launch of one step's kernel as measured by rocprofv3
    counters (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel calibration)
    and recorded in profiles/*.md, or None when no record matches or the
    kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for m in re.finditer(r"<!-- traffic (\{.*?\}) -->", open(path).read()):
            rec = json.loads(m.group(1))
            if (rec["workload"], rec["precision"], rec["kernel_id"], rec["step"]) != \
                    (workload, precision, kernel_id, step):
                continue
            same = all(os.path.exists(os.path.join(ROOT, f)) and
                       hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest() == h
                       for f, h in rec["sources"].items())
            return float(rec["bytes_per_launch"]) if same else None
    return None


def cpu_baseline(name, w):
    """The oracle (plain-C FP64 state vector) on a bounded sample: the set-up
    and the first G_s gates are timed and the full-circuit time is
    extrapolated linearly in the gate count; the oracle's amplitudes/s for
    this workload is k over that time."""
    from oracle import sv_native
    from oracle.circuit import gate_list
    circ, words = w.circuit(), w.bitstrings()
    if w.n_qubits > 30:
        return None
    n, glist = gate_list(circ)
    t0 = time.perf_counter()
    sv_native.amplitudes(circ, words, max_gates=0)
    t_setup = time.perf_counter() - t0
    gs = min(len(glist), 60)
    t0 = time.perf_counter()
    sv_native.amplitudes(circ, words, max_gates=gs)
    t_sample = time.perf_counter() - t0
    per_gate = max(t_sample - t_setup, 1e-9) / gs
    t_full = t_setup + per_gate * len(glist)
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": w.k / t_full, "unit": "amplitudes/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 state vector (oracle/sv.c) of the same {w.n_qubits}-qubit circuit: set-up plus the "
                      f"first {gs} of {len(glist)} gates timed ({t_sample:.1f} s), full run extrapolated to "
                      f"{t_full:.1f} s for all {w.k} bitstrings"}


GROUP_EST_S = 30.0


def run_in_parts(api, w, e, net, prec, need, stream, args, gi):
    """One plan too large for a bounded queue pass: its slices run in
    parts of about GROUP_EST_S estimated seconds, each timed with HIP events
    and reported when it ends; the pass starts from an empty stem cache, so
    the parts add up to one complete contraction."""
    import math
    import torch
    spec = api.PlanSpec([tuple(x) for x in e["pairs"]], e["sliced"], (), e["cap"])
    r = api.Contraction(net, spec, w.bitstrings(), precision=prec, slice_batch=1, stream=stream,
                        memory_budget=need)
    n = r.n_slices
    parts = min(n, max(1, math.ceil(e["est_seconds"] / GROUP_EST_S)))
    bounds = [n * i // parts for i in range(parts + 1)]
    log(f"group {gi}: {w.name} alone, estimated {e['est_seconds']:.1f} s per pass, {n} slices in {parts} parts")
    amps = None
    for rep in range(args.warmup + args.steps):
        timed = rep >= args.warmup
        r.reset_cache()
        amps = r.new_amplitudes() if amps is None else amps.zero_()
        ms = 0.0
        for i in range(parts):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            r.execute(amps, bounds[i], bounds[i + 1])
            ev1.record(stream)
            stream.synchronize()
            ms += ev0.elapsed_time(ev1)
            log(f"group {gi}: {'timed' if timed else 'warm-up'} pass {rep}, slices [{bounds[i]}, {bounds[i + 1]}) "
                f"done, {ms / 1e3:.1f} s so far")
    x = r.xeb(amps)
    out = (ms, x, r.k, r.info.cmac_total)
    r.close()
    return out


def run_uneven(args) -> None:
    """The uneven batch: the 32 seeded circuits of workload.configs with the
    stored plans (plans/c5_cap30.json), in complex-half by default. Plans
    are packed, largest workspace first, into groups whose workspaces fit
    the device memory; each group is one queue (one captured graph of all
    of its plans' launches, slice-sums and XEBs). The timed step replays
    every group's queue once; amplitudes/s counts every amplitude of every
    circuit in the batch."""
    import torch
    from paper_2212_04749_amd import api, binding as B
    from paper_2212_04749_amd.circuit_tn import build_network
    from paper_2212_04749_amd.plans import make_c5
    from workload.configs import uneven_batch_c5

    plans = make_c5.load()
    prec = args.precision
    sel, skipped = [], []
    for w in uneven_batch_c5():
        e = plans[w.name]
        (sel if e["est_seconds"] <= args.max_est_s else skipped).append((w, e))
    free, _ = torch.cuda.mem_get_info()
    cap_bytes = int(0.85 * free)
    # workspace each plan needs (chunked down to the device budget if larger)
    items = []
    for w, e in sel:
        net = build_network(w.circuit())
        ranks, ids, data = api.network_arrays(net)
        h = B.matnc_network_create(ranks, ids, data, net.n_qubits, net.output_index)
        p = B.matnc_plan_create(h, [tuple(x) for x in e["pairs"]], e["sliced"], [], w.bitstrings(),
                                api.PRECISIONS[prec], e["cap"], 1, cap_bytes)
        need = int(B.matnc_plan_info(p).workspace_bytes)
        B.matnc_plan_destroy(p)
        B.matnc_network_destroy(h)
        items.append((need, w, e, net))
    items.sort(key=lambda x: -x[0])
    # first fit, largest workspace first; a group also stays under about
    # GROUP_EST_S of estimated work so that each pass over it reports back
    # within a bounded time (a single larger plan gets a group of its own)
    groups = []
    for it in items:
        est = it[2]["est_seconds"]
        for g in groups:
            if g["bytes"] + it[0] <= cap_bytes and g["est"] + est <= GROUP_EST_S:
                g["items"].append(it)
                g["bytes"] += it[0]
                g["est"] += est
                break
        else:
            groups.append({"bytes": it[0], "est": est, "items": [it]})
    log(f"uneven batch: {len(sel)} circuits in {len(groups)} queue groups, {len(skipped)} left out "
        f"(estimated over {args.max_est_s} s each)")
    total_ms = 0.0
    xebs, n_amps, cmac = {}, 0, 0.0
    stream = torch.cuda.Stream()
    for gi, g in enumerate(groups):
        if len(g["items"]) == 1 and g["est"] > GROUP_EST_S:
            need, w, e, net = g["items"][0]
            ms, x, k, cm = run_in_parts(api, w, e, net, prec, need, stream, args, gi)
            total_ms += ms
            xebs[w.name] = x
            n_amps += k
            cmac += cm
            torch.cuda.empty_cache()
            continue
        runs = []
        for need, w, e, net in g["items"]:
            spec = api.PlanSpec([tuple(x) for x in e["pairs"]], e["sliced"], (), e["cap"])
            runs.append(api.Contraction(net, spec, w.bitstrings(), precision=prec, slice_batch=1, stream=stream,
                                        memory_budget=need))
        q = api.Queue(runs)
        log(f"group {gi}: {len(runs)} circuits ({', '.join(it[1].name for it in g['items'])}), "
            f"estimated {g['est']:.1f} s per pass; capturing")
        t0 = time.perf_counter()
        amps, xeb = q.execute()  # capture
        stream.synchronize()
        log(f"group {gi}: first pass {time.perf_counter() - t0:.1f} s")
        for _ in range(args.warmup):
            q.execute(amps, xeb)
            stream.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            q.execute(amps, xeb)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        total_ms += ms
        xs = xeb.cpu().numpy()
        for (need, w, e, net), r, x in zip(g["items"], runs, xs):
            xebs[w.name] = float(x)
            n_amps += r.k
            cmac += r.info.cmac_total
        log(f"group {gi}: {len(runs)} circuits, {g['bytes'] / 2**30:.1f} GiB, {ms:.2f} ms per pass")
        q.close()
        for r in runs:
            r.close()
        del amps, xeb
        torch.cuda.empty_cache()
    secs = total_ms / 1e3
    out = {
        "metric": "sustained complex TFLOP/s + amplitudes/sec per slice-batch at stated err vs FP64",
        "value": n_amps / secs, "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "complex64" if prec == "c64" else "complex-half", "data": "synthetic",
        "complex_tflops": 8 * cmac / secs / 1e12,
        "config": {"workload": f"C5: uneven batch of {len(sel)} seeded grid RQCs (20-36 qubits, depth 10-16, "
                               f"256-4096 bitstrings), stored plans at rank cap 30, one queue per memory group",
                   "circuits": len(sel), "left_out": [w.name for w, _ in skipped], "groups": len(groups),
                   "amplitudes": n_amps, "precision": prec},
        "xeb_per_circuit": xebs,
    }
    print(json.dumps(out), flush=True)


def beside_pass(api, torch, net, spec, words, name, batch, args):
    """The same workload and plan in complex-half, timed with the same
    protocol (every step a full pass from an empty stem cache), for the
    complex-half rate beside the complex64 one."""
    run = api.Contraction(net, spec, words, precision="chalf", slice_batch=batch)
    if not args.no_autotune:
        autotune(run)
    amps = run.new_amplitudes()

    def step():
        run.reset_cache()
        with torch.cuda.stream(run.stream):
            amps.zero_()
        run.execute(amps)
        return run.xeb_dev(amps)

    for _ in range(args.warmup):
        step()
        run.synchronize()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(run.stream)
    for _ in range(args.steps):
        x = step()
    ev1.record(run.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"complex-half beside: {ms:.2f} ms/step")
    a = amps.cpu().numpy()
    err = reference_error(name, run, a[..., 0] + 1j * a[..., 1])
    n_batches = -(-run.n_slices // batch)
    roof, _, t_roof_ms = roofline(run, "chalf", n_batches, run.n_slices - (n_batches - 1) * batch, name)
    info = run.info
    tflops = 8 * info.cmac_total / (ms / 1e3) / 1e12
    out = {"dtype": "complex-half", "ms_per_step": ms, "value": info.n_amplitudes / (ms / 1e3),
           "unit": "amplitudes/s", "complex_tflops": tflops, "mfma_peak_frac": tflops / PEAK_TFLOPS["fp16"],
           "step_roofline_frac": t_roof_ms / ms, "xeb": float(x.cpu().item()), "error_vs_fp64": err,
           "roofline": roof}
    run.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; multi-GPU slice sharding is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.workload == "C5":
        run_uneven(args)
        return
    from paper_2212_04749_amd import api, planner
    from paper_2212_04749_amd.circuit_tn import build_network
    from workload import CONFIGS

    name = args.workload
    w = CONFIGS[name]
    batch = args.slice_batch or {"C1": 1, "C2": 4, "C3": 8, "C4": 1}[name]
    circ, words = w.circuit(), w.bitstrings()
    t0 = time.perf_counter()
    net = build_network(circ)
    cap = w.cap if w.cap is not None else 32
    # at least the workload's slice count; a cheaper plan that needs more
    # sliced indices to meet the rank cap keeps its real count
    pt = args.partition_trials if args.partition_trials >= 0 else (16 if name in ("C3", "C4") else 0)
    if name in ("C3", "C4") and not args.replan:
        # the stored plan (plans/make_c3.py, make_c4.py: minutes to tens of
        # minutes of host planning)
        import importlib
        e = importlib.import_module(f"paper_2212_04749_amd.plans.make_{name.lower()}").load()
        pairs = [tuple(x) for x in e["pairs"]]
        st0 = planner.Structure.from_network(net, w.open_qubits)
        plan = planner.Plan(pairs, list(e["sliced"]), planner.costs(
            st0, planner.build_tree(st0, pairs, sum(1 << i for i in e["sliced"])),
            planner.widths(planner.build_tree(st0, pairs), words), sum(1 << i for i in e["sliced"])),
            planner.widths(planner.build_tree(st0, pairs), words), "stored:" + e["method"])
        cap = e["cap"]
    else:
        plan = planner.find_plan(net, words, w.open_qubits, w.cap, seed=0, trials=args.trials, partition_trials=pt,
                                 min_slices=w.n_slices_target.bit_length() - 1 if w.n_slices_target else 0,
                                 progress=lambda msg: log(f"planning: {msg}"))
    spec = api.PlanSpec(plan.pairs, plan.sliced, tuple(w.open_qubits), cap, plan.method)
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    run = api.Contraction(net, spec, words, precision=args.precision, slice_batch=batch)
    torch.cuda.synchronize()
    t_bind = time.perf_counter() - t0
    t_tune = 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        autotune(run)
        t_tune = time.perf_counter() - t0
    info = run.info
    log(f"plan {t_plan:.2f}s bind {t_bind:.2f}s autotune {t_tune:.2f}s workspace {info.workspace_bytes / 2**30:.2f} GiB "
        f"slices {info.n_slices} cmac_total {info.cmac_total:.3e}")

    amps = run.new_amplitudes()
    xeb_out = None
    s_begin, s_end = 0, run.n_slices
    if args.slice_subset and args.slice_subset < run.n_slices:
        rng = np.random.default_rng(2004)
        n_sub = -(-args.slice_subset // batch) * batch
        s_begin = int(rng.integers(0, (run.n_slices - n_sub) // batch + 1)) * batch
        s_end = min(run.n_slices, s_begin + n_sub)
        log(f"timing slices [{s_begin}, {s_end}) of {run.n_slices}")

    def step():
        nonlocal xeb_out
        run.reset_cache()
        with torch.cuda.stream(run.stream):
            amps.zero_()
        run.execute(amps, s_begin, s_end)
        xeb_out = run.xeb_dev(amps)

    for i in range(args.warmup):
        step()
        run.synchronize()
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(run.stream)
    for i in range(args.steps):
        step()
    ev1.record(run.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step (wall {wall / args.steps * 1e3:.2f} ms/step)")
    full = (s_begin, s_end) == (0, run.n_slices)
    ms_slices = None
    if not full:
        # the same slices again with the stem cache kept: the per-slice part
        # of the step, so that the projection counts the slice-invariant
        # prologue once for the job
        with torch.cuda.stream(run.stream):
            amps.zero_()
        ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev2.record(run.stream)
        run.execute(amps, s_begin, s_end)
        ev3.record(run.stream)
        torch.cuda.synchronize()
        ms_slices = ev2.elapsed_time(ev3)
        log(f"slices [{s_begin}, {s_end}) with the stem cache kept: {ms_slices:.2f} ms "
            f"({ms_slices / (s_end - s_begin):.2f} ms per slice)")

    amps_np = amps.cpu().numpy()
    amps_c = amps_np[..., 0] + 1j * amps_np[..., 1]
    xeb = float(xeb_out.cpu().item()) if full else None
    err = reference_error(name, run, amps_c) if full else None
    n_batches = -(-run.n_slices // batch)
    roof, per, t_roof_ms = roofline(run, args.precision, n_batches, run.n_slices - (n_batches - 1) * batch, name)
    if args.profile_out:
        from paper_2212_04749_amd import planner as P
        st = P.Structure.from_network(net, w.open_qubits)
        smask = sum(1 << i for i in spec.sliced)
        tree = P.build_tree(st, spec.pairs, smask)
        prof = run.profile(0, min(batch, run.n_slices))
        steps = []
        for j, ((ms, kid, cm, by), dep) in enumerate(zip(prof, run.step_dep())):
            a, b_ = spec.pairs[j]
            ma, mb = tree.masks[a], tree.masks[b_]
            if mb.bit_count() > ma.bit_count():
                ma, mb = mb, ma
            k_ = (ma & mb).bit_count()
            steps.append({"step": j, "ms": ms, "kernel": kid, "cmac": cm, "bytes": by, "dep": dep,
                          "m": ma.bit_count() - k_, "n": mb.bit_count() - k_, "k": k_,
                          "w": plan.widths[st.n_tensors + j]})
        with open(args.profile_out, "w") as f:
            json.dump({"per_kernel": {str(k): v for k, v in per.items()}, "steps": steps}, f, indent=1)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        try:
            cpu = cpu_baseline(name, w)
        except MemoryError:
            cpu = None
    # a slice subset is projected to the whole job: the slice-invariant
    # prologue once, the per-slice work for every slice
    n_timed = s_end - s_begin
    frac = n_timed / run.n_slices
    if full:
        secs = ms_step / 1e3
    else:
        prologue_ms = max(0.0, ms_step - ms_slices)
        secs = (prologue_ms + ms_slices / n_timed * run.n_slices) / 1e3
    cmac_timed = info.cmac_invariant + (info.cmac_total - info.cmac_invariant) * frac
    out = {
        "metric": "sustained complex TFLOP/s + amplitudes/sec per slice-batch at stated err vs FP64",
        "value": info.n_amplitudes / secs,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64" if args.precision == "c64" else "complex-half",
        "data": "synthetic",
        "complex_tflops": 8 * cmac_timed / (ms_step / 1e3) / 1e12,
        # whole-step rate over the MFMA peak of the precision (FP32 for
        # complex64, FP16 for complex-half, whose stem still runs on FP32)
        "mfma_peak_frac": 8 * cmac_timed / (ms_step / 1e3) / 1e12 /
                          PEAK_TFLOPS["fp32" if args.precision == "c64" else "fp16"],
        # sum over the steps of each one's roofline time (the larger of its
        # flops over the MFMA peak of its kernel and its algorithmic bytes
        # over 8 TB/s), over the measured step time
        # (for a slice subset both are whole-job figures: the projected time)
        "step_roofline_ms": t_roof_ms,
        "step_roofline_frac": t_roof_ms / (secs * 1e3),
        "xeb": xeb,
        "error_vs_fp64": err,
        "plan_s": t_plan,
        "bind_s": t_bind,
        "autotune_s": t_tune,
        "config": workload_description(name, w, info, spec) | {"slice_batch": batch, "precision": args.precision}
        | ({} if full else {"slices_timed": [s_begin, s_end], "value_is_projected": True,
                            "projected_job_s": secs, "per_slice_ms": ms_slices / n_timed,
                            "prologue_ms": max(0.0, ms_step - ms_slices)}),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    run.close()
    if args.precision == "c64" and full and not args.no_beside and (args.beside or name in ("C1", "C2")):
        torch.cuda.empty_cache()
        out["complex_half"] = beside_pass(api, torch, net, spec, words, name, batch, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
