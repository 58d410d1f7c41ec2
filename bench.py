#!/usr/bin/env python3
"""Throughput of the sliced multi-amplitude contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C3]
                    [--precision chalf|c64] [--beside-steps K2] [--no-secondary]
                    [--slice-batch B] [--no-cpu-baseline]

One step is one complete pass of the hot path over the workload's batch:
the slice-invariant (stem) nodes, every slice of the sliced network in
batches of B slices (gathered branch contractions over the reuse tree), the
FP64 slice-sum into the amplitudes and the FP64 linear XEB.  Inputs (leaf
tensors, reuse maps, offset tables) are resident in HBM before the timed
region; planning and upload are reported separately.

Default: the 6x6 depth-14 batching workload (2^14 amplitudes as 64 bitstring
groups x 8 open legs, 256 slices, its stored plan), complex-half for the
headline (W warm-up passes, K timed passes), complex64 on the same plan
beside it (one warm-up, K2 timed passes), and the 5x6 depth-12 workload
(4096 bitstrings) in both precisions as a secondary entry.  The first
warm-up pass of the 6x6 legs runs the permutation circuit of the same grid
(its leaves swapped in with matnc_plan_set_tensor; exact amplitudes known,
stored in tests/golden/c3_permutation.json): its error is the error figure
of the line, since the random circuit is beyond any FP64 reference.

Prints one JSON line: amplitudes/s of the whole job (value), sustained
complex TFLOP/s, the error of the amplitudes against stored FP64 oracle
values, a roofline entry for the dominant kernel (HIP-event timings of a
profiled pass on the plan's stream) and the oracle timed on the host cores
on a bounded sample.
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
GOLDEN = os.path.join(ROOT, "tests", "golden")
METRIC = "sustained complex TFLOP/s + amplitudes/sec per slice-batch at stated err vs FP64"
PRECISION_NAME = {"c64": "complex64", "chalf": "complex-half"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="C3", choices=["C1", "C2", "C3", "C4", "C5", "PT"],
                   help="C1..C5 the workloads; PT the fidelity workload (Eq. (2), Fig. 4)")
    p.add_argument("--max-est-s", type=float, default=100.0,
                   help="uneven batch (C5): leave out circuits whose plan's estimated time exceeds this")
    p.add_argument("--precision", default=None, choices=["c64", "chalf"],
                   help="headline precision (default: complex-half, complex64 for the 4x4 and 5x6 workloads)")
    p.add_argument("--slice-batch", type=int, default=0, help="0 = workload default")
    p.add_argument("--trials", type=int, default=32, help="order-search candidates (--replan, 4x4)")
    p.add_argument("--partition-trials", type=int, default=-1,
                   help="bisection candidates of the order search (-1: 16 for the 36- and 53-qubit "
                        "workloads, none otherwise)")
    p.add_argument("--slice-subset", type=int, default=0, metavar="N",
                   help="time N consecutive slices (seeded start) instead of all of them and project the "
                        "full-job rate (the large workloads); 0 = every slice, except on the 53-qubit workload "
                        "(C4), whose default is 64 (a full pass takes hours)")
    p.add_argument("--replan", action="store_true",
                   help="search a plan instead of loading the stored one (5x6, 6x6 and 53-qubit workloads)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--beside-steps", type=int, default=2,
                   help="timed passes of the other precision on the same plan (0: leave it out)")
    p.add_argument("--no-secondary", action="store_true", help="6x6 default: leave out the 5x6 entry")
    p.add_argument("--no-autotune", action="store_true", help="keep the heuristic MFMA tile choice")
    p.add_argument("--profile-out", default="", help="write the per-step profile of the headline leg as JSON")
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


def stored_plan(name, net, words, open_qubits):
    """The stored plan of a workload (plans/make_*.py: seconds to tens of
    minutes of host search) with its cost reports."""
    import importlib
    from paper_2212_04749_amd import planner
    e = importlib.import_module(f"paper_2212_04749_amd.plans.make_{name.lower()}").load()
    plan = planner.plan_from(net, words, open_qubits, e["pairs"], e["sliced"], "stored:" + e["method"])
    return plan, e


def workload_description(name, w, info, spec, e, net=None):
    g = w.grid
    shape = f"{g.rows}x{g.cols}" + (f" minus {len(g.removed)} site" if g.removed else "")
    greedy = (e or {}).get("greedy_report") or {}
    plan_txt = f"; plan: {spec.method}"
    if (e or {}).get("time_model"):
        plan_txt += f", searched under the {e['time_model']} time model"
    if greedy.get("cmac_total"):
        plan_txt += f" (the greedy order sliced to the same cap: {greedy['cmac_total']:.2e} CMAC)"
    return {
        "workload": f"{name}: {shape} grid RQC ({w.n_qubits} qubits), depth {w.depth}, "
                    f"fSim(pi/2,pi/6), {w.k} uniform bitstrings" +
                    (f" x 2^{len(w.open_qubits)} open legs" if w.open_qubits else "") +
                    f", rank cap {spec.cap}, {info.n_slices} slices" + plan_txt,
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
        "plan_time_model": (e or {}).get("time_model", "c64") if e else None,
        "greedy_plan": greedy or None,
        "workspace_bytes": int(info.workspace_bytes),
    } | ({} if net is None else {"reuse_tree_memory": reuse_tree_memory(net, w, spec)})


def reuse_tree_memory(net, w, spec):
    """The paper's breadth- and depth-first memory figures of the plan's reuse
    tree (planner.memory_figures, per slice, in tensor elements) beside the
    library's workspace, which holds every node's instances of a slice batch."""
    from paper_2212_04749_amd import planner
    st = planner.Structure.from_network(net, w.open_qubits)
    tree = planner.build_tree(st, list(spec.pairs), sum(1 << i for i in spec.sliced))
    m = planner.memory_figures(tree, w.bitstrings())
    return {"M_BFT_elements": m["M_BFT"], "M_DFT_elements": m["M_DFT"], "layers": len(m["layers"])}


def _golden_amps(g):
    import numpy as np
    return np.array([complex(a, b) for a, b in g["amps"]])


def errors(got, ref, n_qubits):
    import numpy as np
    got, ref = np.asarray(got).reshape(-1), np.asarray(ref).reshape(-1)
    xeb_gpu = float(np.ldexp(np.mean(np.abs(got) ** 2), n_qubits) - 1)
    xeb_ref = float(np.ldexp(np.mean(np.abs(ref) ** 2), n_qubits) - 1)
    return {"rel_err": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "max_abs_err_over_rms": float(np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))),
            "samples": int(got.size), "xeb_abs_err_on_samples": abs(xeb_gpu - xeb_ref)}


def reference_error(name, amps_c, n_qubits):
    """Error against the stored FP64 oracle amplitudes of the workload's
    random circuit (tests/golden, written by oracle-only scripts), where
    stored: all 64 of the 4x4 batch, a 256-bitstring subset of the 5x6 one."""
    import numpy as np
    path = {"C1": "c1_all.json", "C2": "c2_subset.json"}.get(name)
    if not path or not os.path.exists(os.path.join(GOLDEN, path)):
        return None
    g = json.load(open(os.path.join(GOLDEN, path)))
    ref = _golden_amps(g)
    idx = np.array(g["indices"]) if "indices" in g else np.arange(len(ref))
    out = errors(amps_c[idx, 0], ref, n_qubits)
    out["reference"] = f"FP64 state vector of the same circuit (tests/golden/{path})"
    return out


def permutation_check(name, w, net):
    """For the 6x6 workload: the permutation circuit of the same grid and
    depth, whose fused network has the same structure (so the plan is
    unchanged and only leaf data differs), with its exact amplitudes on a
    subset of the groups (tests/golden/c3_permutation.json)."""
    if name != "C3":
        return None
    from paper_2212_04749_amd.circuit_tn import build_network
    from workload import permutation_circuit
    g = json.load(open(os.path.join(GOLDEN, "c3_permutation.json")))
    pnet = build_network(permutation_circuit(w.grid, w.depth, g["permutation_seed"]))
    if pnet.indices != net.indices:
        raise RuntimeError("permutation network differs in structure")
    return {"net": net, "pnet": pnet, "groups": g["groups"], "ref": _golden_amps(g),
            "seed": g["permutation_seed"]}


def run_leg(api, torch, name, w, net, spec, precision, batch, steps, warmup, args, e=None, check=None,
            s_range=None, profile_out=""):
    """One precision on one plan: warm-up passes, then `steps` timed passes
    (each from an empty stem cache with zeroed amplitudes: every slice of the
    range, slice-sums and XEB) between HIP events on the plan's stream; the
    host waits for pass i-1 while pass i is queued, so it reports progress
    without idling the GPU.  With `check`, the first warm-up pass runs the
    permutation circuit's leaves and gives the error figure."""
    import numpy as np
    words = w.bitstrings()
    t0 = time.perf_counter()
    run = api.Contraction(net, spec, words, precision=precision, slice_batch=batch)
    torch.cuda.synchronize()
    t_bind = time.perf_counter() - t0
    t_tune = 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        autotune(run)
        t_tune = time.perf_counter() - t0
    info = run.info
    log(f"{name} {precision}: bind {t_bind:.2f}s autotune {t_tune:.2f}s workspace "
        f"{info.workspace_bytes / 2**30:.2f} GiB, {info.n_chunks} key chunks, {info.n_slices} slices")
    amps = run.new_amplitudes()
    s_begin, s_end = s_range or (0, run.n_slices)
    xeb_out = None

    def step():
        nonlocal xeb_out
        run.reset_cache()
        with torch.cuda.stream(run.stream):
            amps.zero_()
        run.execute(amps, s_begin, s_end)
        xeb_out = run.xeb_dev(amps)

    err = None
    done = 0
    check_ms = None
    if check is not None:
        for t, x in enumerate(check["pnet"].tensors):
            run.set_tensor(t, x)
        ev_c = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev_c[0].record(run.stream)
        step()
        ev_c[1].record(run.stream)
        run.synchronize()
        check_ms = ev_c[0].elapsed_time(ev_c[1])
        a = amps.cpu().numpy()
        blocks = (a[..., 0] + 1j * a[..., 1])[np.array(check["groups"])]
        err = errors(blocks, check["ref"], w.n_qubits)
        # every |a| of a permutation circuit is 2^(-n/2): its XEB error is
        # about twice the mean relative error, not a statistic of the
        # random circuit's batch (see xeb_vs_complex64 for that)
        err.pop("xeb_abs_err_on_samples")
        err["reference"] = (f"exact amplitudes of the permutation circuit (seed {check['seed']}) on the same "
                            f"network and plan, full pass with its leaves swapped in "
                            f"(tests/golden/c3_permutation.json, oracle.closed_forms)")
        for t, x in enumerate(check["net"].tensors):
            run.set_tensor(t, x)
        done = 1
        log(f"{name} {precision}: warm-up pass on the permutation circuit, rel err {err['rel_err']:.2e}")
    ev_w = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    graph_ms = check_ms
    for i in range(max(0, warmup - done)):
        ev_w[0].record(run.stream)
        step()
        ev_w[1].record(run.stream)
        run.synchronize()
        graph_ms = ev_w[0].elapsed_time(ev_w[1])
        log(f"{name} {precision}: warm-up {i + done} done ({graph_ms:.1f} ms, graph replay)")
    # the dominant step, from one profiled batch; its launches are then timed
    # with HIP events inside the timed passes
    n_batches = -(-run.n_slices // batch)
    dom = dominant_step(run, precision, n_batches)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    dom_ms, dom_n = 0.0, 0
    evs[0].record(run.stream)
    for i in range(steps):
        run.reset_cache()
        with torch.cuda.stream(run.stream):
            amps.zero_()
        ms, n = run.execute_timed(amps, dom["step"], s_begin, s_end)
        xeb_out = run.xeb_dev(amps)
        evs[i + 1].record(run.stream)
        dom_ms += ms
        dom_n += n
        log(f"{name} {precision}: timed pass {i} queued, step {dom['step']}: {n} launches, {ms / max(n, 1):.3f} ms each")
    torch.cuda.synchronize()
    ms_step = evs[0].elapsed_time(evs[steps]) / steps
    ms_passes = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    log(f"{name} {precision}: {steps} timed passes, {ms_step:.2f} ms per pass")
    full = (s_begin, s_end) == (0, run.n_slices)
    ms_slices = None
    if not full:
        # the same slices again with the stem cache kept: the per-slice part
        # of the step, so that the projection counts the slice-invariant
        # prologue once for the job
        with torch.cuda.stream(run.stream):
            amps.zero_()
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(run.stream)
        run.execute(amps, s_begin, s_end)
        e3.record(run.stream)
        torch.cuda.synchronize()
        ms_slices = e2.elapsed_time(e3)
    a = amps.cpu().numpy()
    amps_c = a[..., 0] + 1j * a[..., 1]
    xeb = float(xeb_out.cpu().item()) if full else None
    if err is None and full:
        err = reference_error(name, amps_c, w.n_qubits)
    roof = roofline(dom, dom_ms, dom_n, precision, name)
    per, t_roof_ms = dom["per"], dom["t_roof_ms"]
    if profile_out:
        write_profile(profile_out, run, spec, net, w, batch, per)
    n_timed = s_end - s_begin
    frac = n_timed / run.n_slices
    if full:
        secs = ms_step / 1e3
    else:
        secs = (max(0.0, ms_step - ms_slices) + ms_slices / n_timed * run.n_slices) / 1e3
    cmac_timed = info.cmac_invariant + (info.cmac_total - info.cmac_invariant) * frac
    tflops = 8 * cmac_timed / (ms_step / 1e3) / 1e12
    out = {
        "dtype": PRECISION_NAME[precision],
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        # a warm-up pass replayed from the captured graphs (the timed passes
        # launch the same kernels one by one, with events around the
        # dominant step's launches)
        "ms_per_step_graph": graph_ms,
        # each timed pass (the mean of these is ms_per_step)
        "ms_per_pass": ms_passes,
        "ms_per_pass_median": sorted(ms_passes)[len(ms_passes) // 2],
        "value": info.n_amplitudes / secs,
        "unit": "amplitudes/s",
        "complex_tflops": tflops,
        # whole-step rate over the MFMA peak of the precision's arithmetic
        "mfma_peak_frac": tflops / PEAK_TFLOPS["fp32" if precision == "c64" else "fp16"],
        # sum over the steps of each one's roofline time (the larger of its
        # flops over the MFMA peak of its kernel and its algorithmic bytes
        # over 8 TB/s), over the measured (or, for a slice subset, projected) time
        "step_roofline_ms": t_roof_ms,
        "step_roofline_frac": t_roof_ms / (secs * 1e3),
        "xeb": xeb,
        "error_vs_fp64": err,
        "bind_s": t_bind,
        "autotune_s": t_tune,
        "config": workload_description(name, w, info, spec, e, net) | {"slice_batch": batch, "precision": precision,
                                                                     "key_chunks": int(info.n_chunks)}
        | ({} if full else {"slices_timed": [s_begin, s_end], "value_is_projected": True,
                            "projected_job_s": secs, "per_slice_ms": ms_slices / n_timed,
                            "prologue_ms": max(0.0, ms_step - ms_slices)}),
        "roofline": roof,
        # the random circuit's amplitudes of a full pass (removed before output)
        "_amps": amps_c if full else None,
    }
    run.close()
    del amps
    torch.cuda.empty_cache()
    return out


def write_profile(path, run, spec, net, w, batch, per):
    from paper_2212_04749_amd import planner as P
    st = P.Structure.from_network(net, w.open_qubits)
    smask = sum(1 << i for i in spec.sliced)
    tree = P.build_tree(st, spec.pairs, smask)
    wid = P.widths(P.build_tree(st, spec.pairs), w.bitstrings())
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
                      "w": wid[st.n_tensors + j]})
    with open(path, "w") as f:
        json.dump({"per_kernel": {str(k): v for k, v in per.items()}, "steps": steps}, f, indent=1)


def cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return len(os.sched_getaffinity(0))


def cpu_baseline_sv(w):
    """The oracle's plain-C FP64 state vector (oracle/sv.c) over the whole
    circuit for the workload's whole batch, timed (n <= 30 qubits)."""
    from oracle import sv_native
    circ, words = w.circuit(), w.bitstrings()
    t0 = time.perf_counter()
    sv_native.amplitudes(circ, words)
    t = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": w.k / t, "unit": "amplitudes/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_info(),
            "sample": f"the whole job: FP64 state vector (oracle/sv.c) of the {w.n_qubits}-qubit circuit and all "
                      f"{w.k} amplitudes, {t:.1f} s, not extrapolated"}


def cpu_baseline_tn(w, cap: int = 25, seed: int = 2025, min_s: float = 10.0, max_slices: int = 32):
    """The oracle's plain tensor-network contraction (oracle/tn.py: unfused
    network, its own greedy order, numpy tensordot in complex128), sliced by
    its own slicer to rank `cap` so that one slice is a bounded sample;
    seeded (group, slice) contractions are timed until at least min_s
    seconds of work, and the whole-job time is their mean x the oracle's
    slice count x the number of groups (every slice of every group is the
    same contraction with other values)."""
    import numpy as np
    from oracle import tn as otn
    from oracle.circuit import words_to_bits
    circ, words = w.circuit(), w.bitstrings()
    plan = otn.Plan(circ, w.open_qubits, cap)
    rng = np.random.default_rng(seed)
    times = []
    while len(times) < max_slices and sum(times) < min_s:
        g = int(rng.integers(0, len(words)))
        assignment = [int(x) for x in rng.integers(0, 2, len(plan.sliced))]
        bits = words_to_bits(words[g:g + 1], plan.net.n)[0]
        t0 = time.perf_counter()
        plan.slice_partial(bits, assignment)
        times.append(time.perf_counter() - t0)
    t = sum(times) / len(times)
    n_sl = 2 ** len(plan.sliced)
    job_s = t * n_sl * len(words)
    amps = len(words) << len(w.open_qubits)
    return {"value": amps / job_s, "unit": "amplitudes/s", "cores": blas_threads(), "kind": "oracle",
            "cpu_model": cpu_info(),
            "sample": f"{len(times)} of the oracle tensor network's {n_sl} slices (its own greedy order and slicer "
                      f"at rank {cap}) of seeded groups among the {len(words)} bitstring groups (2^"
                      f"{len(w.open_qubits)} amplitudes each), {sum(times):.1f} s in all, {t:.2f} s per slice, "
                      f"scaled by {n_sl} slices x {len(words)} groups to {job_s:.3g} s for the whole job"}


def dominant_step(run, precision, n_batches):
    """The step with the largest share of a pass, from one profiled batch
    (slice-dependent steps run once per slice batch).  Also returns per-
    kernel-id aggregates and the pass's summed per-step roofline time (ms):
    for every step the larger of its algorithmic flops over the MFMA peak of
    its kernel and its algorithmic bytes over the HBM peak."""
    prof = run.profile(0, min(run.slice_batch, run.n_slices))
    per = {}
    steps = []
    t_roof = 0.0
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
    return {"step": j, "profile_ms": ms, "kid": kid, "cmac": cmac, "bytes": by, "tf": tf, "tb": tb, "peak": peak,
            "share": share / total, "per": per, "t_roof_ms": t_roof}


def roofline(dom, ms_total, launches, precision, workload):
    """Roofline of the dominant step's kernel: its bound is the larger of its
    algorithmic flops over the MFMA peak of the kernel and its algorithmic
    bytes over the HBM peak; achieved is that quantity per launch over the
    mean launch time measured with HIP events in the timed passes."""
    j, kid, cmac, by, peak = dom["step"], dom["kid"], dom["cmac"], dom["bytes"], dom["peak"]
    ms = ms_total / max(launches, 1)
    t = ms / 1e3
    if kid >= 100 and dom["tf"] >= dom["tb"]:
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
    r["launches"] = launches
    r["mean_launch_ms"] = ms
    r["timing"] = "HIP events on the plan's stream around each launch of the step in the timed passes"
    r["profile_pass_ms"] = dom["profile_ms"]
    r["share_of_step"] = dom["share"]
    return r


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


def run_uneven(args) -> None:
    """The uneven batch: the 32 seeded circuits of workload.configs with the
    stored plans (plans/c5_cap30.json), complex-half by default, as ONE queue
    bound to one workspace (every plan's static region plus one arena shared
    by all, matnc_queue_bind) and captured as one graph: every plan's stem,
    slices, slice-sums and XEB.  The timed step replays that graph once;
    amplitudes/s counts every amplitude of every circuit."""
    import torch
    from paper_2212_04749_amd import api
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
    budget = int(0.75 * free)
    stream = torch.cuda.Stream()
    runs = []
    for w, e in sel:
        spec = api.PlanSpec([tuple(x) for x in e["pairs"]], e["sliced"], (), e["cap"])
        runs.append(api.Contraction(build_network(w.circuit()), spec, w.bitstrings(), precision=prec, slice_batch=1,
                                    stream=stream, memory_budget=budget, bind=False))
    q = api.Queue(runs, shared=True)
    log(f"uneven batch: {len(runs)} circuits in one queue, shared workspace {q.workspace.numel() / 2**30:.1f} GiB "
        f"(the plans' own workspaces add up to {sum(r.info.workspace_bytes for r in runs) / 2**30:.1f} GiB), "
        f"{len(skipped)} left out (estimated over {args.max_est_s} s each)")
    t0 = time.perf_counter()
    amps, xeb = q.execute()  # captures the queue's graph; the first warm-up pass
    stream.synchronize()
    log(f"capture and first pass {time.perf_counter() - t0:.1f} s")
    for i in range(max(0, args.warmup - 1)):
        q.execute(amps, xeb)
        stream.synchronize()
        log(f"warm-up pass {i + 1} done")
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for i in range(args.steps):
        q.execute(amps, xeb)
        evs[i + 1].record(stream)
        if i >= 1:
            evs[i].synchronize()
            log(f"timed pass {i - 1} done")
    torch.cuda.synchronize()
    total_ms = evs[0].elapsed_time(evs[args.steps]) / args.steps
    xs = xeb.cpu().numpy()
    xebs = {w.name: float(x) for (w, _), x in zip(sel, xs)}
    n_amps = sum(r.k for r in runs)
    cmac = sum(r.info.cmac_total for r in runs)
    secs = total_ms / 1e3
    out = {
        "metric": METRIC,
        "value": n_amps / secs, "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": PRECISION_NAME[prec], "data": "synthetic",
        "complex_tflops": 8 * cmac / secs / 1e12,
        "config": {"workload": f"C5: uneven batch of {len(sel)} seeded grid RQCs (20-36 qubits, depth 10-16, "
                               f"256-4096 bitstrings), stored plans at rank cap 30 ("
                               f"{sum(e.get('time_model') == 'chalf' for e in plans.values())} searched under the "
                               f"chalf time model, the others under c64), one queue, one workspace, one graph",
                   "circuits": len(sel), "left_out": [w.name for w, _ in skipped],
                   "shared_workspace_bytes": int(q.workspace.numel()),
                   "amplitudes": n_amps, "precision": prec},
        "xeb_per_circuit": xebs,
    }
    q.close()
    for r in runs:
        r.close()
    print(json.dumps(out), flush=True)


def run_fidelity(args) -> None:
    """The fidelity workload (main text Eq. (2), Fig. 4): bitstrings of a
    20-qubit circuit sampled from the mixture of its exact distribution
    (weight F) and the uniform one, stored with their exact x = 2^n p
    (tests/golden/pt_samples.json, written by the oracle).  Their amplitudes
    are computed on the GPU in both precisions; F is estimated by the linear
    XEB (on the GPU) and by maximum likelihood under Eq. (2); the histogram
    of x against Eq. (2)'s density at the fitted F is the data of Fig. 4."""
    import numpy as np
    import torch
    from paper_2212_04749_amd import analysis, api
    from workload import GridSpec, random_circuit
    g = json.load(open(os.path.join(GOLDEN, "pt_samples.json")))
    circ = random_circuit(GridSpec(*g["grid"]), g["depth"], g["circuit_seed"])
    n = g["n_qubits"]
    sets = []
    for st in g["sets"]:
        words = np.array([int(x) for x in st["words"]], dtype=np.uint64)
        x_ref = np.array(st["x"])
        entry = {"fidelity": st["fidelity"], "samples": len(words),
                 "expected_linear_xeb": st["fidelity"] * g["ideal_linear_xeb"]}
        for prec in ("c64", "chalf"):
            run = api.Contraction.from_circuit(circ, words, cap=18, precision=prec, slice_batch=2, trials=4)
            amps = run.execute()
            run.synchronize()
            torch.cuda.synchronize()
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            evs[0].record(run.stream)
            for _ in range(max(1, args.steps)):
                run.reset_cache()
                with torch.cuda.stream(run.stream):
                    amps.zero_()
                run.execute(amps)
            evs[1].record(run.stream)
            torch.cuda.synchronize()
            ms = evs[0].elapsed_time(evs[1]) / max(1, args.steps)
            f_lin = run.xeb(amps)
            a = amps.cpu().numpy()
            x = analysis.x_values(a[:, 0, 0] + 1j * a[:, 0, 1], n)
            f_mle = analysis.fit_fidelity(x)
            entry[PRECISION_NAME[prec]] = {
                "linear_xeb_gpu": f_lin, "mle_fidelity": f_mle, "ms_per_pass": ms,
                "amplitudes_per_s": len(words) / (ms / 1e3),
                "x_rel_err": float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)),
                "histogram": analysis.porter_thomas_histogram(x, f_mle, bins=24, x_max=6.0)}
            run.close()
            log(f"F = {st['fidelity']} {prec}: linear XEB {f_lin:.4f}, MLE {f_mle:.4f}, {ms:.2f} ms per pass")
        sets.append(entry)
    print(json.dumps({"workload": "PT: 4x5 grid RQC (20 qubits), depth 12, 4096 bitstrings per fidelity sampled "
                                  "from the mixture of the exact distribution and the uniform one",
                      "sets": sets}), flush=True)


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
    name = args.workload
    if args.precision is None:
        args.precision = "chalf" if name in ("C3", "C4", "C5") else "c64"
    if name == "C5":
        run_uneven(args)
        return
    if name == "PT":
        run_fidelity(args)
        return
    from paper_2212_04749_amd import api, planner
    from paper_2212_04749_amd.circuit_tn import build_network
    from workload import CONFIGS

    w = CONFIGS[name]
    batch = args.slice_batch or {"C1": 1, "C2": 4, "C3": 8, "C4": 1}[name]
    words = w.bitstrings()
    t0 = time.perf_counter()
    net = build_network(w.circuit())
    e = None
    if name in ("C2", "C3", "C4") and not args.replan:
        plan, e = stored_plan(name, net, words, w.open_qubits)
        cap = e["cap"]
    else:
        cap = w.cap if w.cap is not None else 32
        pt = args.partition_trials if args.partition_trials >= 0 else (16 if name in ("C3", "C4") else 0)
        plan = planner.find_plan(net, words, w.open_qubits, w.cap, seed=0, trials=args.trials, partition_trials=pt,
                                 min_slices=w.n_slices_target.bit_length() - 1 if w.n_slices_target else 0,
                                 progress=lambda msg: log(f"planning: {msg}"))
    spec = api.PlanSpec(plan.pairs, plan.sliced, tuple(w.open_qubits), cap, plan.method)
    t_plan = time.perf_counter() - t0
    check = permutation_check(name, w, net)
    s_range = None
    if name == "C4" and not args.slice_subset:
        args.slice_subset = 64
    if args.slice_subset:
        n_sl = 2 ** len(plan.sliced)
        if args.slice_subset < n_sl:
            rng = np.random.default_rng(2004)
            n_sub = -(-args.slice_subset // batch) * batch
            s0 = int(rng.integers(0, (n_sl - n_sub) // batch + 1)) * batch
            s_range = (s0, min(n_sl, s0 + n_sub))
            log(f"timing slices [{s_range[0]}, {s_range[1]}) of {n_sl}")

    head = run_leg(api, torch, name, w, net, spec, args.precision, batch, args.steps, args.warmup, args, e,
                   check, s_range, args.profile_out)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
    }
    out |= {k: head[k] for k in ("ms_per_step_graph", "ms_per_pass", "ms_per_pass_median", "complex_tflops",
                                 "mfma_peak_frac", "step_roofline_ms",
                                 "step_roofline_frac",
                                 "xeb", "error_vs_fp64", "bind_s", "autotune_s")}
    out["plan_s"] = t_plan
    out["config"] = head["config"]
    out["roofline"] = head["roofline"]
    out["cpu_baseline"] = None
    other = "c64" if args.precision == "chalf" else "chalf"
    if args.beside_steps > 0:
        leg = run_leg(api, torch, name, w, net, spec, other, batch, args.beside_steps, 1, args, e, check, s_range)
        leg.pop("config")
        out["beside"] = {PRECISION_NAME[other]: leg}
        if head["xeb"] is not None and leg["xeb"] is not None:
            # the random circuit's linear XEB over the whole batch, the two
            # precisions on the same plan and bitstrings
            out["xeb_vs_" + PRECISION_NAME[other].replace("-", "_")] = abs(head["xeb"] - leg["xeb"])
        if head["_amps"] is not None and leg["_amps"] is not None:
            # complex-half against complex64 on the random circuit itself (its
            # complex64 error is ~1e-6 on the workloads the oracle reaches)
            h, c = (head["_amps"], leg["_amps"]) if args.precision == "chalf" else (leg["_amps"], head["_amps"])
            d = h - c
            rms = float(np.sqrt(np.mean(np.abs(c) ** 2)))
            out["complex_half_vs_complex64"] = {
                "rel_diff": float(np.linalg.norm(d) / np.linalg.norm(c)),
                "max_abs_diff_over_rms": float(np.max(np.abs(d)) / rms), "amplitudes": int(c.size)}
        leg.pop("_amps")
    head.pop("_amps")
    if name == "C3" and not args.no_secondary:
        # the 5x6 workload (4096 bitstrings, stored plan) in both precisions
        w2 = CONFIGS["C2"]
        net2 = build_network(w2.circuit())
        plan2, e2 = stored_plan("C2", net2, w2.bitstrings(), ())
        spec2 = api.PlanSpec(plan2.pairs, plan2.sliced, (), e2["cap"], plan2.method)
        sec = {}
        for prec in ("c64", "chalf"):
            sec[PRECISION_NAME[prec]] = run_leg(api, torch, "C2", w2, net2, spec2, prec, 4, 3, 1, args, e2)
            sec[PRECISION_NAME[prec]].pop("_amps")
        out["secondary"] = {"C2": sec}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        t0 = time.perf_counter()
        try:
            out["cpu_baseline"] = cpu_baseline_sv(w) if w.n_qubits <= 30 else cpu_baseline_tn(w)
        except MemoryError:
            out["cpu_baseline"] = None
        log(f"cpu baseline: {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
