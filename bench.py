"""Benchmark: Aggregate Risk Analysis on one MI355X.

One step = one analysis request on resident tables: ara_run_layers (fold +
trial pass over the whole 1M x Poisson(1000) Year Event Table, 16 ELTs) and
ara_risk_metrics (mean, PML/TVaR at 99% and 99.6%).  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

Also measured: the trial-pass kernel's own duration (HIP events on its launch
stream, in a second pass over the same steps, since recording them adds idle
gaps between launches) for the roofline, the gradient/forward time ratio (forward with S
checkpoints + metrics vs ara_backward), and the CPU oracle on a bounded
sample of the same workload.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_pass_kernel_config1_traffic.json")
NETS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "event_nets_config1_traffic.json")
CSRC = os.path.join(ROOT, "paper_1606_04473_amd", "csrc")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="config1")
    ap.add_argument("--cpu-sample-trials", type=int, default=300_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--literal-steps", type=int, default=0,
                    help="also time the literal per-ELT lookup kernel this many times")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the multi-tenant serving study (config 4)")
    ap.add_argument("--serving-per-tenant", type=int, default=6)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-layer batched run (config 2)")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-portfolio", action="store_true",
                    help="skip the portfolio run (10 programs of the 64 library layers, YET split 1-8 ways)")
    ap.add_argument("--portfolio-steps", type=int, default=3)
    ap.add_argument("--no-event-nets", action="store_true",
                    help="skip the per-event net-loss run on the main workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for counter scaling)")
    return ap.parse_args()


def copy_probe() -> None:
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch.
    Hardware counters of this launch scale those of the trial pass."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "launches": 3}), flush=True)


def cpu_model() -> str:
    """The host CPU's model name."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def time_oracle(oracle, yet, pool, layer, threads: int, min_s: float = 1.0) -> float:
    """Seconds per oracle run of one layer, repeated until min_s has passed."""
    reps, t0 = 0, time.time()
    while True:
        oracle.run_layer(yet, pool, layer, threads=threads)
        reps += 1
        if time.time() - t0 >= min_s:
            return (time.time() - t0) / reps


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary, if it was taken on the current source of the kernel's file."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src_file = os.path.join(CSRC, rec.get("kernel_source", "kernels_parts.hip"))
    if not os.path.exists(src_file):
        return None
    src = hashlib.sha256(open(src_file, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != src:
        return None
    return rec.get("traffic_bytes_per_launch")


def batched_study(ara, tables, w, library, steps, stream):
    """All 64 layers of the shared-YET library in one ara_run_layers call.
    The autotuner picks the pass variant and launch shape for this shape
    (timing every candidate on it); then, each timed with HIP events over
    `steps` calls: the tuned choice replayed from a HIP graph and eagerly,
    the per-layer streaming sequences, and the persistent batched launch
    (pass_variant 1), eagerly and from a graph."""
    import tempfile
    import torch
    from paper_1606_04473_amd import autotune
    off = w.yet.offsets
    lookups = sum(float(off[l.trial_begin + l.trial_count] - off[l.trial_begin]) * l.n_elts for l in library)
    events = sum(float(off[l.trial_begin + l.trial_count] - off[l.trial_begin]) for l in library)
    total = sum(l.trial_count for l in library)
    C = w.yet.catalogue_size
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()            # graph capture needs a stream of its own
    res = {"layers": len(library), "lookups": lookups, "ylt_values": total, "event_layer_pairs": events}
    # Alg. 1 order (a YET pass per layer) and a fused single pass, as algorithmic bytes
    res["alg1_bytes"] = 4.0 * events + sum(8.0 * l.n_elts * C + 16.0 * l.trial_count for l in library)
    res["fused_bytes"] = 4.0 * w.yet.n_events + 8.0 * len({int(j) for l in library for j in l.elt_index}) * C \
        + 8.0 * total
    report = {}
    with torch.cuda.stream(stream):
        best = autotune.tuned(tables, library, out, path=os.path.join(tempfile.mkdtemp(), "tune.json"), repeats=2,
                              report=report)
    res["autotune"] = {"chosen": best, "candidates": report.get("detail")}
    log(f"batched 64 layers: autotuner chose {best}")
    legs = (("tuned_graph", best, ara.ARA_GRAPH), ("tuned", best, 0),
            ("stream_per_layer", dict(pass_variant=0), 0),
            ("persistent", dict(pass_variant=1, part_lanes_per_trial=16), 0),
            ("persistent_graph", dict(pass_variant=1, part_lanes_per_trial=16), ara.ARA_GRAPH))
    for name, knobs, flags in legs:
        ara.set_tuning(tables, **knobs)
        torch.cuda.synchronize()
        for _ in range(2):
            ara.run_layers(tables, library, out=out, flags=flags, stream=stream)
        stream.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            ara.run_layers(tables, library, out=out, flags=flags, stream=stream)
        b.record(stream)
        stream.synchronize()
        ms = a.elapsed_time(b) / steps
        res[name] = {"knobs": knobs, "graph": bool(flags & ara.ARA_GRAPH), "ms": round(ms, 3),
                     "lookups_per_s": lookups / (ms / 1e3),
                     "event_layer_pairs_per_s": events / (ms / 1e3),
                     "pct_hbm_fused_bytes": round(res["fused_bytes"] / (ms / 1e3) / (HBM_PEAK_GBS * 1e9), 4),
                     "pct_hbm_alg1_bytes": round(res["alg1_bytes"] / (ms / 1e3) / (HBM_PEAK_GBS * 1e9), 4)}
        log(f"batched 64 layers ({name}): {ms:.3f} ms, {lookups / (ms / 1e3):.3e} lookups/s, "
            f"{events / (ms / 1e3):.3e} event-layer pairs/s")
    ara.set_tuning(tables)
    del out
    return res


def portfolio_study(ara, tables, w, steps):
    """Algorithm 1 over a portfolio: the 64 library layers grouped in order
    into 10 programs, every layer over all trials, the YET split 1, 2, 4 and
    8 ways.  Per split count: time per portfolio (HIP events), whether the
    program and portfolio YLTs are bit-identical to the unsplit run, and the
    program/portfolio sum kernel's duration and HBM rate."""
    import torch
    from workloads import portfolio_programs
    N = w.yet.n_trials
    progs = portfolio_programs(w.layers, 10, 0, N, seed=w.meta["seed"] + 100)
    specs = [[ara.LayerSpec.from_layer(l, w.pool, N) for l in p] for p in progs]
    n_layers = sum(len(p) for p in progs)
    lookups = float(w.yet.n_events) * sum(l.n_elts for p in progs for l in p)
    sum_bytes = 8.0 * N * (n_layers + len(progs) + 1)
    outs = {"program": torch.empty((len(progs), N), dtype=torch.float64, device="cuda"),
            "portfolio": torch.empty(N, dtype=torch.float64, device="cuda")}
    stream = torch.cuda.Stream()
    res = {"programs": len(progs), "layers": n_layers, "layers_per_program": [len(p) for p in progs],
           "trials": N, "lookups": lookups, "sum_kernel_bytes": sum_bytes, "by_splits": {}}
    ref = None
    for n_splits in (1, 2, 4, 8):
        ara.run_portfolio(tables, specs, n_splits, outs=outs, stream=stream)
        stream.synchronize()
        if ref is None:
            ref = {k: v.clone() for k, v in outs.items()}
            identical = True
        else:
            identical = all(bool(torch.equal(outs[k], ref[k])) for k in outs)
        ara.kernel_stats(tables, ara.KERNEL_AGGREGATE, reset=True)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            ara.run_portfolio(tables, specs, n_splits, outs=outs, stream=stream, flags=ara.ARA_PROFILE)
        b.record(stream)
        stream.synchronize()
        ms = a.elapsed_time(b) / steps
        n_sum, ms_sum = ara.kernel_stats(tables, ara.KERNEL_AGGREGATE, reset=True)
        sum_ms = ms_sum / max(n_sum, 1)
        res["by_splits"][str(n_splits)] = {
            "ms": round(ms, 3), "lookups_per_s": lookups / (ms / 1e3), "bit_identical_to_1": identical,
            "sum_kernel_ms": round(sum_ms, 4),
            "sum_kernel_gbs": round(sum_bytes / (sum_ms / 1e3) / 1e9, 1)}
        log(f"portfolio {len(progs)} programs / {n_layers} layers, {n_splits} splits: {ms:.3f} ms, "
            f"{lookups / (ms / 1e3):.3e} lookups/s, sums {sum_ms:.4f} ms, identical={identical}")
    del outs, ref
    return res


def main() -> None:
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the analysis shards by trials "
                                   "across GPUs, but runs on several GPUs are not measured",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1606_04473_amd import ara
    from workloads import make_config

    torch.cuda.set_device(0)
    torch.cuda.init()
    t0 = time.time()
    w = make_config(args.config)
    yet, pool, layer = w.yet, w.pool, w.layers[0]
    J = layer.n_elts
    N, n_ev, C = yet.n_trials, yet.n_events, yet.catalogue_size
    log(f"generated {args.config}: N={N} events={n_ev} C={C} J={J} in {time.time() - t0:.1f}s")
    t0 = time.time()
    tables = ara.create_tables(yet.offsets, yet.ids, pool.losses)
    log(f"tables resident ({tables.bytes() / 1e9:.2f} GB) in {time.time() - t0:.1f}s")
    spec = ara.LayerSpec.from_layer(layer, pool, N)
    probs = list(w.probs)
    out = torch.empty(N, dtype=torch.float64, device="cuda")
    res = torch.empty(1 + 2 * len(probs), dtype=torch.float64, device="cuda")
    # a stream of the bench's own (the legacy default stream synchronises with
    # every other stream, and graph replay needs a real stream)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    def step(flags=0):
        if flags & ara.ARA_GRAPH:
            # the layer call and the metrics as one replayed graph (ara_analyze)
            ara.analyze(tables, spec, probs, ylt=out, metrics=res, flags=flags, stream=stream)
        else:
            ara.run_layers(tables, [spec], out=out, flags=flags, stream=stream)
            ara.risk_metrics(out, probs, outputs=res, stream=stream)

    def step_layer_graph():
        # the layer call's own graph (ara_run_layers with ARA_GRAPH), metrics eager
        ara.run_layers(tables, [spec], out=out, flags=ara.ARA_GRAPH, stream=stream)
        ara.risk_metrics(out, probs, outputs=res, stream=stream)

    for _ in range(args.warmup):
        step()
        step(ara.ARA_GRAPH)                 # the first ones capture the graphs
        step_layer_graph()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed(flags, fn=None):
        torch.cuda.synchronize()
        w0 = time.time()
        start.record(stream)
        for _ in range(args.steps):
            if fn is None:
                step(flags)
            else:
                fn()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / args.steps, time.time() - w0

    # the steps as a user runs them, no per-kernel events: eagerly (two calls),
    # with the layer call's own graph and eager metrics, and as one graph of
    # the whole step (ara_analyze with ARA_GRAPH: fold, pass, combine and the
    # metrics kernels), which is the headline
    ms_step_eager, _ = timed(0)
    ms_step_layer_graph, _ = timed(0, step_layer_graph)
    ms_step, wall = timed(ara.ARA_GRAPH)
    # the same steps again with HIP events around each launch (ARA_PROFILE), for
    # the per-kernel durations; recording them adds idle gaps between launches
    ara.kernel_stats(tables, ara.KERNEL_TRIAL_PASS, reset=True)
    ara.kernel_stats(tables, ara.KERNEL_FOLD, reset=True)
    ara.kernel_stats(tables, ara.KERNEL_COMBINE, reset=True)
    start.record(stream)
    for _ in range(args.steps):
        step(ara.ARA_PROFILE)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_step_profiled = start.elapsed_time(stop) / args.steps
    n_tp, ms_tp = ara.kernel_stats(tables, ara.KERNEL_TRIAL_PASS)
    n_fold, ms_fold = ara.kernel_stats(tables, ara.KERNEL_FOLD)
    n_comb, ms_comb = ara.kernel_stats(tables, ara.KERNEL_COMBINE)
    tp_avg = ms_tp / max(n_tp, 1)
    fold_avg = ms_fold / max(n_fold, 1)
    comb_avg = ms_comb / max(n_comb, 1)
    log(f"step {ms_step:.4f} ms as one graph (wall {wall / args.steps * 1e3:.4f} ms), {ms_step_layer_graph:.4f} ms "
        f"with the layer graph and eager metrics, {ms_step_eager:.4f} ms "
        f"eager, {ms_step_profiled:.4f} ms with per-kernel events; trial pass {tp_avg:.4f} ms; "
        f"combine {comb_avg:.4f} ms; fold {fold_avg:.4f} ms")
    h = res.cpu().numpy()
    log(f"mean={h[0]:.6e} PML={h[1:1 + len(probs)]} TVaR={h[1 + len(probs):]}")

    lookups = float(n_ev) * J
    value = lookups / (ms_step / 1e3)
    step_bytes = 4.0 * n_ev + 8.0 * (N + 1) + 8.0 * J * C + 8.0 * N
    # the pass's algorithmic bytes per launch: 4 B per event (its ID), 16 B per
    # trial (offsets in, year loss out), 8 B per catalogue event (o)
    tp_bytes = 4.0 * n_ev + 8.0 * (N + 1) + 8.0 * N + 8.0 * C
    achieved = tp_bytes / (tp_avg / 1e3) / 1e9
    lay = tables.layout()
    streaming = lay["stream_parts"] > 0
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if streaming else None,
                "kernel": "stream_pass_kernel" if streaming else "xcd_pass_kernel",
                "algorithmic_bytes_per_launch": tp_bytes, "avg_launch_ms": round(tp_avg, 5)}
    if streaming:
        # the 16-bit layout's own bytes: its IDs (2 B each, padding included),
        # each group's 32 trial ends (2 B) and start (4 B) per part, and the
        # per-(part, trial) partial sums written (8 + 4 B)
        P16, NG = lay["stream_parts"], lay["stream_groups"]
        lay_bytes = 2.0 * lay["stream_ids"] + P16 * NG * (64.0 + 4.0) + 12.0 * P16 * N
        roofline["layout_bytes_per_launch"] = lay_bytes
        roofline["layout_achieved"] = round(lay_bytes / (tp_avg / 1e3) / 1e9, 1)
        roofline["layout_frac"] = round(lay_bytes / (tp_avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        roofline["layout"] = {"stream_parts": P16, "group_trials": lay["stream_group_trials"],
                              "groups_per_part": NG, "stream_ids": lay["stream_ids"]}

    extra = {"pct_hbm_step": round(step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
             "step_algorithmic_bytes": step_bytes, "fold_ms": round(fold_avg, 5),
             "combine_ms": round(comb_avg, 5),
             "combine_bytes": 12.0 * lay["stream_parts"] * N + 16.0 * N if streaming else 16.0 * lay["image_parts"] * N + 16.0 * N,
             "ms_per_step_with_kernel_events": round(ms_step_profiled, 5),
             "ms_per_step_eager": round(ms_step_eager, 5),
             "ms_per_step_layer_graph_metrics_eager": round(ms_step_layer_graph, 5),
             "lookups_per_s_eager": lookups / (ms_step_eager / 1e3),
             "trial_pass_ms": round(tp_avg, 5)}

    if args.literal_steps > 0:
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.literal_steps):
            ara.run_layers(tables, [spec], out=out, flags=ara.ARA_LITERAL, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        lit_ms = a.elapsed_time(b) / args.literal_steps
        extra["literal_run_layers_ms"] = round(lit_ms, 4)
        extra["literal_lookups_per_s"] = lookups / (lit_ms / 1e3)
        log(f"literal run_layers {lit_ms:.3f} ms")

    if not args.no_backward:
        gm = torch.empty(2 * J + 4, dtype=torch.float64, device="cuda")
        gt = torch.empty(2 * J + 4, dtype=torch.float64, device="cuda")
        for _ in range(2):
            step(ara.ARA_CHECKPOINT_S)
            ara.backward(tables, spec, 0.99, grad_mean=gm, grad_tvar=gt, stream=stream)
        torch.cuda.synchronize()
        reps = max(3, args.steps // 2)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        fwd = bwd = 0.0
        for _ in range(reps):
            e[0].record(stream)
            step(ara.ARA_CHECKPOINT_S)
            e[1].record(stream)
            ara.backward(tables, spec, 0.99, grad_mean=gm, grad_tvar=gt, stream=stream)
            e[2].record(stream)
            torch.cuda.synchronize()
            fwd += e[0].elapsed_time(e[1])
            bwd += e[1].elapsed_time(e[2])
        extra["fwd_checkpointed_ms"] = round(fwd / reps, 4)
        extra["backward_ms"] = round(bwd / reps, 4)
        extra["grad_fwd_ratio"] = round(bwd / fwd, 4)
        extra["grad_fwd_ratio_vs_plain_step"] = round((bwd / reps) / ms_step, 4)
        log(f"forward+ckpt {fwd / reps:.4f} ms, backward {bwd / reps:.4f} ms")
        # the forward that also keeps prefix sums of S every 64 events in time
        # order (the time-ordered pass over the 32-bit YET)
        step(ara.ARA_CHECKPOINT_STRIDE)
        torch.cuda.synchronize()
        e[0].record(stream)
        for _ in range(reps):
            step(ara.ARA_CHECKPOINT_STRIDE)
        e[1].record(stream)
        torch.cuda.synchronize()
        extra["fwd_stride_checkpointed_ms"] = round(e[0].elapsed_time(e[1]) / reps, 4)
        log(f"forward+stride checkpoints {extra['fwd_stride_checkpointed_ms']:.4f} ms")

    if not args.no_event_nets:
        # per-event net losses of every event of the workload, to a device buffer
        nets = torch.empty(n_ev, dtype=torch.float64, device="cuda")
        ara.event_nets(tables, spec, out=nets, stream=stream)
        torch.cuda.synchronize()
        reps = 3
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ara.event_nets(tables, spec, out=nets, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        nets_ms = a.elapsed_time(b) / reps
        # the nets of a trial add up to its year loss (A_0 = 0): first 200 trials
        head = nets[:int(yet.offsets[200])].cpu().numpy()
        ylt_h = out[:200].cpu().numpy()
        worst = max(abs(math.fsum(head[yet.offsets[t]:yet.offsets[t + 1]].tolist()) - ylt_h[t])
                    / max(ylt_h[t], 1.0) for t in range(200))
        nets_bytes = 4.0 * n_ev + 8.0 * (N + 1) + 8.0 * n_ev + 8.0 * J * C + 16.0 * C
        extra["event_nets"] = {"ms": round(nets_ms, 4), "events_per_s": n_ev / (nets_ms / 1e3),
                               "algorithmic_bytes": nets_bytes,
                               "pct_hbm": round(nets_bytes / (nets_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                               "telescoping_rel_err_200_trials": worst,
                               "traffic": measured_traffic(NETS_TRAFFIC_FILE)}
        log(f"event nets: {nets_ms:.4f} ms for {n_ev} events, telescoping error {worst:.2e}")
        del nets

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from workloads import Layer
        n_s = min(args.cpu_sample_trials, N)
        sub = Layer(layer.elt_index, layer.occ_retention, layer.occ_limit, layer.agg_retention,
                    layer.agg_limit, 0, n_s)
        ev_s = int(yet.offsets[n_s])
        n_all = oracle.max_threads()        # before a one-thread run changes the default
        t1 = time.time()
        oracle.run_layer(yet, pool, sub, threads=n_all)
        dt = time.time() - t1
        cpu = {"value": ev_s * J / dt, "unit": "event-ELT lookups/s", "cores": n_all,
               "kind": "oracle",
               "sample": f"first {n_s} trials ({ev_s} events x {J} ELTs) of the same workload, "
                         f"{dt:.1f} s, exact-sum FP64 C oracle",
               "cpu_model": cpu_model()}
        log(f"cpu oracle: {cpu['value']:.3e} lookups/s on {cpu['cores']} threads ({dt:.1f}s)")
        # one core on a smaller sample of the same workload, and the small
        # 10,000-trial workload on all cores and on one
        n1 = min(20_000, N)
        sub1 = Layer(layer.elt_index, layer.occ_retention, layer.occ_limit, layer.agg_retention,
                     layer.agg_limit, 0, n1)
        ev1 = int(yet.offsets[n1])
        dt1 = time_oracle(oracle, yet, pool, sub1, threads=1)
        cpu["single_core"] = {"value": ev1 * J / dt1, "cores": 1,
                              "sample": f"first {n1} trials ({ev1} events x {J} ELTs), {dt1:.2f} s per run"}
        w0 = make_config("config0")
        l0 = w0.layers[0]
        lk0 = float(w0.yet.offsets[-1]) * l0.n_elts
        small = {}
        for name, th in (("all_cores", n_all), ("single_core", 1)):
            d0 = time_oracle(oracle, w0.yet, w0.pool, l0, threads=th)
            small[name] = {"value": lk0 / d0, "cores": th, "seconds_per_run": round(d0, 5)}
        cpu["small_workload"] = dict(small, workload=f"{w0.yet.n_trials} trials x Poisson(100) events, "
                                                     f"{w0.yet.catalogue_size}-event catalogue, {l0.n_elts} ELTs")
        log(f"cpu oracle: one core {cpu['single_core']['value']:.3e} lookups/s; small workload "
            f"{small['all_cores']['value']:.3e} (all cores) / {small['single_core']['value']:.3e} (one core)")

    tables.close()
    del out, res
    serving = None
    batched = None
    portfolio = None
    if not (args.no_serving and args.no_batched and args.no_portfolio):
        t1 = time.time()
        w4 = make_config("config4")
        base = ara.create_tables(w4.yet.offsets, w4.yet.ids, w4.pool.losses)
        library = [ara.LayerSpec.from_layer(l, w4.pool, w4.yet.n_trials) for l in w4.layers]
        log(f"config2/4 tables resident ({base.bytes() / 1e9:.2f} GB) in {time.time() - t1:.1f}s")
        if not args.no_batched:
            batched = batched_study(ara, base, w4, library, args.batched_steps, stream)
        if not args.no_portfolio:
            portfolio = portfolio_study(ara, base, w4, args.portfolio_steps)
        if not args.no_serving:
            from paper_1606_04473_amd import serving as srv
            serving = srv.run_tenant_study(base, w4.yet.offsets, w4.yet.ids, library, n_tenants=8,
                                           per_tenant=args.serving_per_tenant, log=log)
            extra["tenant_p99_ms"] = serving["concurrent_8t"]["p99_ms"]
            extra["tenant_p99_ms_single_tenant"] = serving["concurrent_1t"]["p99_ms"]
            # one analysis (the whole YET, 4 layers) split over 1-8 tenants: time,
            # energy and the deployment model fitted on one tenant
            serving["split"] = srv.split_study(base, w4.yet.offsets, srv.pin_ids(w4.yet.ids), library,
                                               layer_ids=[0, 1, 2, 3], log=log)
        base.close()

    line = {
        "metric": "event-ELT lookups/s + % HBM peak (1M×1000 YET); grad/fwd time; tenant p99",
        "value": value,
        "unit": "event-ELT lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain ARA paper-scale one-GPU share: 1,000,000 trials x Poisson(1000) "
                               "events over a 2,000,000-event catalogue, 1 layer over 16 dense ELTs "
                               "(20,000 lognormal(10,2) losses each), PML/TVaR at 99% and 99.6%",
                   "trials": N, "events": n_ev, "catalogue": C, "elts_per_layer": J},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    if batched is not None:
        line["batched_config2"] = batched
    if portfolio is not None:
        line["portfolio_config2_layers"] = portfolio
    if serving is not None:
        line["serving"] = serving
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
