#!/usr/bin/env python3
"""Throughput of the device-resident search iteration (Algorithm 1, GPU
version): candidate evaluations per second on one MI355X.

A step is one full iteration on the device: eq. (6) base pick, n candidates
drawn (Philox) and evaluated (walk, eq. (2), HU and SU rebalancing, cost,
gate), argmin, reconstruction and commit of the winner.  Inputs are seeded
synthetic instances resident in HBM before the timed region.

Prints one JSON line.  The default workload is the 500-field clustered
instance (2^22 candidates per iteration).  The roofline object prices the
evaluation kernel's algorithmic LDS bytes per candidate (one full evaluation:
the walk of every tour, eq. (2), the units of the rebalancing rounds) against
the LDS peak, over the evaluation launches of the very iterations that
`value` times (the deterministic search is restarted and those iterations
run again with HIP events around the launches); its integer-ALU figure and
its measured HBM traffic sit beside it.  `full_search` covers every
iteration of the workload's search from the initial solution.  The
cpu_baseline object times the CPU oracle on a bounded sample of the same
iteration's candidates; cpu_version runs the oracle's Algorithm 1, CPU
version, against the GPU version's best cost on the 12-field instance.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz = 78643 GB/s
# 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (no FMA or dual
# issue doubling, unlike the fp32 figure) = 39.3 T lane-ops/s.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic integer lane-operations of one full candidate evaluation (walk,
# eq. (2), rebalancing rounds, cost), per workload.
ALU_OPS_PER_CANDIDATE = {"tiny12": 400, "mid100": 1200, "clust500": 4000}

DESCR = {
    "tiny12": "12 fields, 3 BPs, 2 tours, 4 HUs, 8 SUs, 50 km square",
    "mid100": "100 fields, 10 BPs, 5 tours, 12 HUs, 40 SUs, 100 km square",
    "clust500": "500 fields in 20 clusters, 20 BPs, 10 tours, 30 HUs, 120 SUs, 200 km square",
}


HBM_PEAK_GBS = 8000.0
# Instances (and batches whose members all have) at most this many tours are
# evaluated one candidate per lane (k_eval_lane, k_eval_multi_lane), larger
# ones on a segment of lanes per candidate (k_eval, k_eval_multi).
LANE_MAX_TOURS = 12
KERNEL_SOURCES = ("paper_1909_10286_amd/csrc/eval.hip", "paper_1909_10286_amd/csrc/device.h",
                  "paper_1909_10286_amd/csrc/lane_eval.h", "paper_1909_10286_amd/csrc/bl_internal.h")


def kernel_source_digest():
    """sha256 over the evaluation kernel's sources, to tell whether recorded
    counter figures still describe the kernel being run."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload):
    """HBM bytes per evaluation step (a lane kernel's two passes) from the
    committed counter summary of this workload (FETCH_SIZE and WRITE_SIZE,
    scaled by a plain copy's readings), or None when there is none or the
    kernel has changed since."""
    path = os.path.join(ROOT, "profiles", "k_eval_search_%s.md" % workload)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def lds_bytes_per_candidate(nf, nb, nt, nhu, nsu):
    """Algorithmic LDS bytes of one full evaluation: per field visited 22 B
    (position 2, successor leg 4, field-BP distance 4, area 4, supply 4,
    shuttle drives 4), per BP 12 B (list entry 2, start 2, length 2, demand 4,
    tour offset 2), per tour 28 B (offsets 4, unit masks 24) and 4 B per unit
    (rate or fill time)."""
    return 22 * nf + 12 * nb + 28 * nt + 4 * (nhu + nsu)


def cpu_baseline(inst, x0, n_sample):
    from oracle import search as S
    from tests.oracle_pool import OraclePool, n_procs
    st = S.start(inst, x0)
    thr = S.eps_threshold(0.5)
    from oracle.moves import exploit_draw
    base = st.x_best if exploit_draw(0, 0, 0, thr) else st.x_old
    job = (inst, base, 0, 0, 0, False, "le", st.t_best, None, True)
    procs = n_procs()
    pool = OraclePool(procs)
    pool(job, procs)  # start the workers outside the timed region
    t0 = time.perf_counter()
    pool(job, n_sample)
    dt = time.perf_counter() - t0
    pool.close()
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=n_sample / dt, unit="evals/s", cores=procs, kind="oracle",
                sample="first %d candidates of iteration 0 (seed 0, eps 0.5), %d processes, %.1f s"
                % (n_sample, procs, dt), cpu_model=model)


# Oracle candidates per cpu_baseline sample, per workload: about 10-30 s on
# 16 host cores (clust500: about 5.6 ms per candidate on one core).
CPU_SAMPLE = {"tiny12": 1 << 19, "mid100": 1 << 19, "clust500": 1 << 16}


def cpu_version_baseline(budget_s=10.0):
    """Algorithm 1's CPU version (one candidate per iteration, x_old <- x after
    every draw) in the oracle, on the tiny12 instance, for `budget_s` seconds
    of one host core: its evaluations per second, and when it first comes
    within 1 % of, and first matches, the best cost of the GPU version's
    search on the same instance (4096 candidates x 100 iterations, seed 0,
    eps 0.5)."""
    from oracle import search as S
    from paper_1909_10286_amd import bl, inputs
    from tests.gpu_common import from_csr
    import torch

    wl = inputs.WORKLOADS["tiny12"]
    ctx = bl.Context(0)
    ctx.set_stream(torch.cuda.current_stream())
    inst = inputs.make_instance("tiny12", 0, accept=_accepting(ctx, bl))
    iid = ctx.instance_upload(inst)
    x0 = ctx.init_solution(iid)
    ctx.solution_upload(iid, bl.SLOT_BASE, x0)
    ctx.search_start(iid, 0)
    thr = S.eps_threshold(0.5)
    for _ in range(wl["iters"]):
        ctx.search_step(iid, 0, thr, wl["n_cand"])
    gpu_best = ctx.search_state(iid)["cost_best_m"]
    ctx.close()
    target = 1.01 * gpu_best
    st = S.start(inst, from_csr(x0))
    start_cost = st.cost_best
    hits = {"target": None, "gpu_best": None}
    t0 = time.perf_counter()
    iters = 0
    while time.perf_counter() - t0 < budget_s:
        st = S.cpu_version_step(inst, st, 0, thr)
        st.trace = []   # the harness keeps no trace: only the best cost is read
        iters += 1
        for k, c in (("target", target), ("gpu_best", gpu_best)):
            if hits[k] is None and st.cost_best <= c:
                hits[k] = (time.perf_counter() - t0, iters)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "algorithm": "Algorithm 1, CPU version (one candidate per iteration)",
            "workload": "tiny12: %s, seed 0, eps 0.5" % DESCR["tiny12"], "cores": 1,
            "evals_per_s": iters / dt, "iterations": iters, "seconds": dt,
            "start_km": start_cost / 1e3, "gpu_version_best_km": gpu_best / 1e3, "target_km": target / 1e3,
            "best_km": st.cost_best / 1e3,
            "time_to_target_s": hits["target"] and hits["target"][0],
            "iterations_to_target": hits["target"] and hits["target"][1],
            "time_to_gpu_version_best_s": hits["gpu_best"] and hits["gpu_best"][0],
            "iterations_to_gpu_version_best": hits["gpu_best"] and hits["gpu_best"][1]}


def bench_batch(a):
    """256 uneven instances searched together: one persistent evaluation
    launch per iteration, autotuned schedule, iterations replayed from a
    captured HIP graph."""
    import tempfile

    import torch

    from paper_1909_10286_amd import bl, inputs

    wl = inputs.WORKLOADS["batch256"]
    n, K = a.n or wl["n_cand"], wl["n_instances"]
    ctx = bl.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)

    def accept(inst):
        iid = ctx.instance_upload(inst)
        try:
            ctx.init_solution(iid)
            return True
        except bl.BlError as e:
            if e.status == bl.EINFEASIBLE:
                return False
            raise
    insts, ids = [], []
    for k in range(K):
        inst = inputs.make_batch_instance(k, accept=accept)
        iid = ctx.instance_upload(inst)
        ctx.solution_upload(iid, bl.SLOT_BASE, ctx.init_solution(iid))
        insts.append(inst)
        ids.append(iid)
    b = ctx.batch_create(ids, n)
    chunk = 10 if a.steps % 10 == 0 else 1
    ctx.batch_start(b, a.warmup + a.steps + 1)
    seed, thr = 0, 1 << 31
    cache = os.path.join(tempfile.gettempdir(), "bl_batch_schedule.json")
    sched = ctx.batch_autotune(b, seed, thr, cache)
    for _ in range(a.warmup):
        ctx.batch_step(b, seed, thr)
    g = ctx.batch_capture(b, seed, thr, chunk)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps // chunk):
        ctx.graph_launch(g)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # Evaluation-kernel time of a few eager iterations (graphs are not bracketed).
    ctx.timing_enable(True)
    for _ in range(5):
        ctx.batch_step(b, seed, thr)
    eval_ms, launches = ctx.timing_read()
    ctx.timing_enable(False)
    per_launch_s = eval_ms / 1e3 / max(launches, 1)
    bytes_iter = sum(lds_bytes_per_candidate(i.n_fields, i.n_bps, i.n_tours, i.n_hus, i.n_sus) * n
                     for i in insts)
    achieved = bytes_iter / per_launch_s / 1e9
    total = K * n * a.steps
    out = {
        "metric": "candidate evals/s", "value": total / (ms / 1e3), "unit": "evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batch256: 256 instances (fields U{20..300}, BPs U{3..15}, tours "
                               "U{2..8}), %d candidates/iteration each, graph-replayed" % n,
                   "n_candidates": n, "n_instances": K, "schedule": sched,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / LDS_PEAK_GBS, "traffic": None,
                     "kernel": "k_eval_multi_lane" if max(i.n_tours for i in insts) <= LANE_MAX_TOURS
                     else "k_eval_multi", "kernel_ms_per_launch": per_launch_s * 1e3},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def _accepting(ctx, bl):
    def accept(inst):
        iid = ctx.instance_upload(inst)
        try:
            ctx.init_solution(iid)
            return True
        except bl.BlError as e:
            if e.status == bl.EINFEASIBLE:
                return False
            raise
    return accept


def _timed_run(ctx, stream, iid, x0, iters, step):
    """Search from x0 for `iters` iterations of `step()`; returns the
    cumulative seconds after each iteration (HIP events) and the trace's
    best cost after each iteration (exact, metres)."""
    import numpy as np
    import torch

    from paper_1909_10286_amd import bl
    ctx.solution_upload(iid, bl.SLOT_BASE, x0)
    ctx.search_start(iid, iters)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(iters):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    t = np.array([ev[0].elapsed_time(e) for e in ev[1:]]) / 1e3
    c = np.array([r["cost_m"] for r in ctx.search_trace(iid)], dtype=np.float64)
    return t, c


# Algorithmic bf16 FLOP of one screened proposal: three changed field rows,
# each through 16 -> 128 -> 128 -> 64 (the pooled-embedding rows of W3).
SCREEN_FLOPS_PER_PROPOSAL = 3 * 2 * (16 * 128 + 128 * 128 + 128 * 64)
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense bf16 MFMA


def screen_comparison(iters=300, n_plain=1 << 22, n_prop=1 << 24, k=1 << 18, pairs=1 << 22,
                      per_base=1 << 16, max_examples=1024, mk_margin=0.05, err_threshold=0.1,
                      n_control=1 << 12):
    """Wall time to within 1 % of the plain search's best cost: the plain
    search (n_plain exact candidates per iteration) against the screened
    search (n_prop proposals ranked by the learned screen, the k best
    evaluated exactly, the plain batch as fallback), on the clust500
    instance.  The network is trained first on `pairs` exact (candidate,
    cost) pairs drawn against the bases of a plain trajectory."""
    import numpy as np
    import torch

    from paper_1909_10286_amd import bl, inputs

    ctx = bl.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)
    inst = inputs.make_instance("clust500", 0, accept=_accepting(ctx, bl))
    iid = ctx.instance_upload(inst)
    x0 = ctx.init_solution(iid)
    seed, thr = 0, 1 << 31

    # Plain search.
    tp, cp = _timed_run(ctx, stream, iid, x0, iters, lambda: ctx.search_step(iid, seed, thr, n_plain))
    target = 1.01 * cp[-1]

    # Training on exact labels along a plain trajectory (its own seed).
    ctx.solution_upload(iid, bl.SLOT_BASE, x0)
    ctx.search_start(iid, 0)
    st = ctx.search_state(iid)
    w = bl.sur_glorot_weights(inputs.surrogate_init_words(1))
    sur = ctx.sur_create(iid, w, float(st["cost_best_m"]), float(st["t_best_s"]),
                         max_examples=max_examples, lr=1e-3)
    d_mv = torch.empty(per_base, dtype=torch.int64, device="cuda")
    d_key = torch.empty(per_base, dtype=torch.int64, device="cuda")
    d_c = torch.empty(per_base, dtype=torch.float32, device="cuda")
    d_m = torch.empty(per_base, dtype=torch.int32, device="cuda")
    d_loss = torch.zeros(2, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_bases = max(1, pairs // per_base)
    for b in range(n_bases):
        ctx.search_step(iid, seed + 1, thr, 1 << 16)
        ctx.generate(iid, seed + 2 + b, 0, 0, 0, per_base, d_mv)
        ctx.evaluate_batch(iid, d_mv, per_base, 1 << 40, d_key, d_c, d_m, None)
        last = b == n_bases - 1
        for j in range(0, per_base, max_examples):
            m = min(max_examples, per_base - j)
            ctx.sur_train_step(sur, d_mv[j:], d_c[j:], d_m[j:], m, d_loss if last else None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    lv = d_loss.cpu().numpy()
    loss = float(lv[0] / max(lv[1], 1.0))

    # Screened search (one eager call first sizes the screen's buffers):
    # without a control sample (the screen alone) and with one (an exact
    # sample that joins the argmin and sends the iteration to the plain batch
    # when it holds an improvement the shortlist misses).
    def screened(nc):
        ctx.solution_upload(iid, bl.SLOT_BASE, x0)
        ctx.search_start(iid, 1)
        ctx.sur_search_step(sur, seed, thr, n_prop, k, n_plain, mk_margin=mk_margin,
                            err_threshold=err_threshold, n_control=nc)
        s0 = ctx.sur_stats(sur)
        ts, cs = _timed_run(ctx, stream, iid, x0, iters, lambda: ctx.sur_search_step(
            sur, seed, thr, n_prop, k, n_plain, mk_margin=mk_margin, err_threshold=err_threshold,
            n_control=nc))
        s1 = ctx.sur_stats(sur)
        th, ih = reach(ts, cs)
        return {"n_control": nc, "best_km": cs[-1] / 1e3, "ms_per_iteration": ts[-1] / iters * 1e3,
                "time_to_target_s": th, "iterations_to_target": ih,
                "time_to_target_with_training_s": None if th is None else th + t_train,
                "fallback_iterations": s1["fallbacks"] - s0["fallbacks"],
                "last_mean_rel_error": s1["last_error"]}

    def reach(t, c):
        hit = np.nonzero(c <= target)[0]
        return (float(t[hit[0]]), int(hit[0]) + 1) if hit.size else (None, None)
    runs = [screened(0), screened(n_control)]
    # The scoring kernel alone, timed with HIP events on its stream.
    ctx.timing_read()
    ctx.timing_enable(True, bl.TIMING_SCREEN)
    for _ in range(10):
        ctx.sur_search_step(sur, seed, thr, n_prop, k, n_plain, mk_margin=mk_margin,
                            err_threshold=err_threshold, n_control=n_control)
    scr_ms, scr_n = ctx.timing_read()
    ctx.timing_enable(False)
    ctx.close()
    scr_ms /= max(scr_n, 1)
    scr_tflops = n_prop * SCREEN_FLOPS_PER_PROPOSAL / (scr_ms * 1e-3) / 1e12

    tp_hit, ip_hit = reach(tp, cp)
    return {
        "workload": "clust500 instance; plain: %d exact candidates/iteration; screened: %d proposals -> "
                    "%d exact (+ %d control, fallback %d); %d iterations each, seed 0, eps 0.5"
                    % (n_plain, n_prop, k, n_control, n_plain, iters),
        "target_km": target / 1e3,
        "plain": {"best_km": cp[-1] / 1e3, "ms_per_iteration": tp[-1] / iters * 1e3,
                  "time_to_target_s": tp_hit, "iterations_to_target": ip_hit},
        "screened": runs[0],
        "screened_with_control": runs[1],
        "training": {"pairs": n_bases * per_base, "seconds": t_train, "final_loss": loss,
                     "examples_per_step": max_examples},
        # The algorithmic work is bf16 MFMA, priced against that peak; what
        # binds the kernel is VALU issue (counters: VALU busy 59 %, MFMA busy
        # 29 %, from the feature rows, bf16 rounding and ReLU between layers
        # and the per-lane score arithmetic).
        "roofline": {"kernel": "k_scr_fused", "bound": "mfma", "binding_unit": "valu",
                     "achieved": scr_tflops,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": scr_tflops / BF16_PEAK_TFLOPS,
                     "flops_per_proposal": SCREEN_FLOPS_PER_PROPOSAL, "kernel_ms_per_launch": scr_ms},
    }


def bench_replica(a):
    """The paper's experiment at its scale (sec. 3.1-3.2, Table 1): fresh
    seeded replicas of 1200 fields / 20 BPs / 7 tours, Cases 1-4, the epsilon
    grid {0, .25, .5, .75, 1}, 5000 iterations; the best cost over epsilon per
    seed and case.  All seeds and cases of one epsilon run as one batch."""
    import numpy as np
    import torch

    from paper_1909_10286_amd import bl, inputs

    ctx = bl.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)
    n = a.n or (1 << 14)
    iters = a.steps
    seeds = list(range(a.replica_seeds))
    cases = {2: bl.FIXED_FIELD_BP | bl.NO_EMBEDDED_MIN | bl.GATE_OFF, 3: bl.FIXED_FIELD_BP, 4: 0}
    grid = [0.0, 0.25, 0.5, 0.75, 1.0]
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), "bl_batch_schedule.json")
    members, case1 = [], {}
    t0 = time.perf_counter()
    for sd in seeds:
        inst = inputs.make_replica_instance(sd, accept=_accepting(ctx, bl))
        fixed = ctx.instance_upload(inst, flags=bl.NO_EMBEDDED_MIN)
        x0 = ctx.init_solution(fixed)
        ctx.solution_upload(fixed, bl.SLOT_BASE, x0)
        ctx.search_start(fixed, 0)
        st = ctx.search_state(fixed)
        case1[sd] = (st["cost_best_m"], st["t_best_s"])
        for cs, fl in cases.items():
            members.append((sd, cs, ctx.instance_upload(inst, flags=fl), x0))
    # The schedule is tuned on bases 200 iterations into a search (the share
    # of candidates that break eq. (2) changes as the search goes on), then
    # read from the cache for every epsilon.
    for _, _, iid, x0 in members:
        ctx.solution_upload(iid, bl.SLOT_BASE, x0)
    b = ctx.batch_create([m[2] for m in members], n)
    ctx.batch_start(b, 0)
    for _ in range(200):
        ctx.batch_step(b, 1, 1 << 31)
    ctx.batch_autotune(b, 1, 1 << 31, cache)
    best = {}
    eval_s = 0.0
    for eps in grid:
        thr = min(int(round(eps * 2.0 ** 32)), 1 << 32)
        for _, _, iid, x0 in members:
            ctx.solution_upload(iid, bl.SLOT_BASE, x0)
        b = ctx.batch_create([m[2] for m in members], n)
        ctx.batch_start(b, 0)
        sched = ctx.batch_autotune(b, 0, thr, cache)   # timed once, then read from the cache
        chunk = 50 if iters % 50 == 0 else 1
        g = ctx.batch_capture(b, 0, thr, chunk)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(iters // chunk):
            ctx.graph_launch(g)
        e1.record(stream)
        torch.cuda.synchronize()
        eval_s += e0.elapsed_time(e1) / 1e3
        for sd, cs, iid, _ in members:
            st = ctx.search_state(iid)
            key = (sd, cs)
            if key not in best or st["cost_best_m"] < best[key][0]:
                best[key] = (st["cost_best_m"], st["t_best_s"], eps)
    ctx.close()
    rows = {1: {"cost_km": float(np.mean([case1[sd][0] for sd in seeds])) / 1e3,
                "worst_completion_h": float(np.mean([case1[sd][1] for sd in seeds])) / 3600}}
    for cs in cases:
        c = [best[(sd, cs)][0] for sd in seeds]
        rows[cs] = {"cost_km": float(np.mean(c)) / 1e3,
                    "delta_pct": float(np.mean([(best[(sd, cs)][0] / case1[sd][0] - 1) * 100 for sd in seeds])),
                    "worst_completion_h": float(np.mean([best[(sd, cs)][1] for sd in seeds])) / 3600,
                    "eps_star": float(np.mean([best[(sd, cs)][2] for sd in seeds]))}
    total = len(members) * n * iters * len(grid)
    print(json.dumps({
        "metric": "candidate evals/s", "value": total / eval_s, "unit": "evals/s", "n_gpus": 1,
        "steps": iters, "warmup": 0, "ms_per_step": eval_s / (iters * len(grid)) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "paper replica: 1200 fields, 20 BPs, 7 tours, 7 HUs, 14 + 28 SUs, 80 km "
                               "square; %d seeds x Cases 2-4 per batch, %d candidates/iteration, "
                               "epsilon grid of 5" % (len(seeds), n),
                   "schedule": sched, "parallelism": "single GPU"},
        "cases": rows, "wall_s": time.perf_counter() - t0}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="clust500", choices=sorted(DESCR) + ["batch256", "replica"])
    ap.add_argument("--replica-seeds", type=int, default=10)
    ap.add_argument("--n", type=int, default=0, help="candidates per iteration (default: workload's)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="candidates the oracle evaluates for cpu_baseline (default: the workload's, "
                         "about 10-30 s on 16 host cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-screen", action="store_true",
                    help="skip the plain vs screened wall-time comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (scale for the HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1909_10286_amd import bl, inputs

    if a.copy_calibration:
        src = torch.ones((256 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 256 << 20, "copies": 3}), flush=True)
        return
    if a.workload == "batch256":
        return bench_batch(a)
    if a.workload == "replica":
        return bench_replica(a)
    return bench_search(a)


def _replay(ctx, stream, iid, x0, seed, thr, n, warmup, steps, graph_chunk=0, timing=False):
    """Searches from x0: `warmup` eager iterations, then `steps` timed ones,
    replayed from a captured graph of `graph_chunk` iterations (eager when
    0).  Returns (ms of the timed iterations from events on the library's
    stream, evaluation-kernel ms and launches within them when `timing`)."""
    import torch

    from paper_1909_10286_amd import bl
    ctx.solution_upload(iid, bl.SLOT_BASE, x0)
    ctx.search_start(iid, warmup + steps)
    for _ in range(warmup):
        ctx.search_step(iid, seed, thr, n)
    g = ctx.search_capture(iid, seed, thr, n, graph_chunk) if graph_chunk else None
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    if timing:
        ctx.timing_read()
        ctx.timing_enable(True)
    e0.record(stream)
    if g is not None:
        for _ in range(steps // graph_chunk):
            ctx.graph_launch(g)
    else:
        for _ in range(steps):
            ctx.search_step(iid, seed, thr, n)
    e1.record(stream)
    torch.cuda.synchronize()
    kern = None
    if timing:
        kern = ctx.timing_read()
        ctx.timing_enable(False)
    return e0.elapsed_time(e1), kern


def bench_search(a):
    """One instance, Algorithm 1's GPU version on the device: `warmup`
    eager iterations, then `steps` iterations timed (graph replays).  The
    evaluation kernel's duration is taken over the same iterations: the
    search is deterministic, so it is restarted from the initial solution,
    the warm-up redone and the timed iterations run again eagerly with HIP
    events around every evaluation launch."""
    import torch

    from paper_1909_10286_amd import bl, inputs

    wl = inputs.WORKLOADS[a.workload]
    n = a.n or wl["n_cand"]
    ctx = bl.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)
    inst = inputs.make_instance(a.workload, 0, accept=_accepting(ctx, bl))
    iid = ctx.instance_upload(inst)
    x0 = ctx.init_solution(iid)
    seed, thr = 0, 1 << 31  # eps = 0.5
    chunk = 10 if a.steps % 10 == 0 else 1
    t0 = time.perf_counter()
    ms, _ = _replay(ctx, stream, iid, x0, seed, thr, n, a.warmup, a.steps, graph_chunk=chunk)
    wall = time.perf_counter() - t0
    state = ctx.search_state(iid)
    # The same iterations again, eagerly, with the evaluation launches timed.
    _, (eval_ms, launches) = _replay(ctx, stream, iid, x0, seed, thr, n, a.warmup, a.steps, timing=True)
    again = ctx.search_state(iid)
    # The whole search of the workload (every iteration from the initial
    # solution), graph-replayed, and its evaluation launches timed the same way.
    full_iters = wl["iters"]
    fchunk = 10 if full_iters % 10 == 0 else 1
    full_ms, _ = _replay(ctx, stream, iid, x0, seed, thr, n, 0, full_iters, graph_chunk=fchunk)
    full_state = ctx.search_state(iid)
    _, (full_eval_ms, full_launches) = _replay(ctx, stream, iid, x0, seed, thr, n, 0, full_iters,
                                               timing=True)
    hbm_meas, lds_meas = ctx.measure_peaks()
    ctx.close()

    value = n * a.steps / (ms / 1e3)
    step_s = eval_ms / 1e3 / max(launches, 1)   # one evaluation step (a lane kernel's two passes)
    bpc = lds_bytes_per_candidate(inst.n_fields, inst.n_bps, inst.n_tours, inst.n_hus, inst.n_sus)
    achieved = bpc * n / step_s / 1e9
    ops = ALU_OPS_PER_CANDIDATE.get(a.workload)
    traffic = recorded_traffic(a.workload) if n == wl["n_cand"] else None
    full_step_s = full_eval_ms / 1e3 / max(full_launches, 1)
    kernel = ("k_eval_lane" if inst.n_tours <= LANE_MAX_TOURS else "k_eval") + " (search mode)"
    out = {
        "metric": "candidate evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "%s: %s, %d candidates/iteration" % (a.workload, DESCR[a.workload], n),
                   "n_candidates": n, "instance_seed": 0, "search_seed": seed, "eps": 0.5,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / LDS_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "bytes_per_candidate": bpc,
                     "kernel_ms_per_launch": step_s * 1e3,
                     "launches_timed": launches,
                     "same_iterations_as_value": again["cost_best_m"] == state["cost_best_m"]
                     and again["it"] == state["it"],
                     "peak_measured": lds_meas, "frac_measured": achieved / lds_meas,
                     "alu": None if ops is None else {
                         "achieved": ops * n / step_s / 1e12, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                         "frac": ops * n / step_s / 1e12 / ALU_PEAK_TOPS, "ops_per_candidate": ops},
                     "hbm": None if traffic is None else {
                         "achieved": traffic / step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": traffic / step_s / 1e9 / HBM_PEAK_GBS,
                         "peak_measured": hbm_meas, "frac_measured": traffic / step_s / 1e9 / hbm_meas}},
        "measured_peaks": {"hbm_copy_gbs": hbm_meas, "lds_read_gbs": lds_meas},
        "search": {"cost_best_km": state["cost_best_m"] / 1000.0, "t_best_h": state["t_best_s"] / 3600.0,
                   "iterations": state["it"], "wall_s": wall},
        "full_search": {"iterations": full_iters, "value": n * full_iters / (full_ms / 1e3),
                        "ms_per_step": full_ms / full_iters, "kernel_ms_per_launch": full_step_s * 1e3,
                        "lds_frac": bpc * n / full_step_s / 1e9 / LDS_PEAK_GBS,
                        "cost_best_km": full_state["cost_best_m"] / 1000.0},
    }
    if not a.no_screen and a.workload == "clust500":
        out["screen"] = screen_comparison()
    if not a.no_cpu_baseline:
        from tests.gpu_common import from_csr
        out["cpu_baseline"] = cpu_baseline(inst, from_csr(x0), a.cpu_sample or CPU_SAMPLE[a.workload])
        out["cpu_version"] = cpu_version_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
