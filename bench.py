#!/usr/bin/env python3
"""Events/s of the GNN track-finding hot path on one MI355X.

One step = one pass of the whole path (features, embedding MLP, radius graph,
interaction network, score cut, components) over one batch of synthetic
events already resident in HBM.  The default workload is the full-size plain
FP32 batch: 1000 events, 26 planes at z in [-290, 750] mm, Poisson(200)
tracks per event (~2500 hits incl. 5 % noise), embedding 3-128-128-12, radius
0.12, at most 64 neighbours, interaction network hidden 64 with 8 steps,
random Xavier weights.

Prints one JSON line with the throughput, the roofline of the dominant kernel
(timed live with HIP events on the stream the kernels run on) and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "int8": 5000.0}   # dense MFMA (int8: TOP/s)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c5"],
                    help="c5: the c3 workload with trained weights and the learned prefilter, trained before timing")
    ap.add_argument("--pf-train-events", type=int, default=50000, help="c5: prefilter training events")
    ap.add_argument("--pf-recall", type=float, default=0.995, help="c5: positive-edge recall that fixes tau")
    ap.add_argument("--events", type=int, default=None, help="override the number of events")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8", "int8"])
    ap.add_argument("--emb-precision", default=None, choices=["fp32", "bf16", "fp8", "int8"],
                    help="the embedding MLP's own operand precision (default: --precision)")
    ap.add_argument("--compact-state", type=int, default=0,
                    help="bf16/fp8: store node and edge encodings in low precision (default: FP32 master copies)")
    ap.add_argument("--graph", type=int, default=0, help="replay the batch as one captured HIP graph")
    ap.add_argument("--autotune", type=int, default=0, help="tune the launch schedule on the batch before timing")
    ap.add_argument("--autotune-log", default=None, help="append the autotuner's trials to this JSON-lines file")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (counter calibration) and exit")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-threads", type=int, default=None)
    ap.add_argument("--profile-stages", type=int, default=1)
    return ap.parse_args()


def stage_roofline(stage, ms_total, launches, n_edges, n_hits, H, dtype, compact):
    """Algorithmic work per launch of a stage and its roofline."""
    if launches == 0 or ms_total <= 0:
        return None
    t = ms_total / launches * 1e-3          # seconds per launch
    # bytes per stored edge-encoding feature: FP32 master copies unless the state is compact
    es = {"f32": 4, "bf16": 2, "fp8": 1, "int8": 1}[dtype] if compact else 4
    if stage in ("edge_step", "edge_step_final"):
        # edge net: Linear(3H->H) + Linear(H->H) per edge (the last step adds the
        # classifier Linear(H->H) + Linear(H->1)); bytes: e read and written once
        # (the last step writes a 4-byte score instead), src and dst indices
        flops = n_edges * (8 * H * H + (2 * H * H + 2 * H if stage == "edge_step_final" else 0))
        # executed on MFMA: layer 1 is factorised (the node products are gathered), so the
        # per-edge products are H x H twice (plus the classifier's H x H)
        xflops = n_edges * (4 * H * H + (2 * H * H if stage == "edge_step_final" else 0))
        nbytes = n_edges * (H * es + (4 if stage == "edge_step_final" else H * es) + 8)
        peak = PEAK_TFLOPS[dtype]
        if flops / (peak * 1e12) >= nbytes / (PEAK_HBM_GBS * 1e9):
            achieved = flops / t / 1e12
            return dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                        units_per_launch=n_edges, per_unit=f"{flops // max(n_edges, 1)} flop/edge (algorithmic)",
                        executed_per_unit=f"{xflops // max(n_edges, 1)} flop/edge (MFMA)",
                        executed_achieved=xflops / t / 1e12, executed_frac=xflops / t / 1e12 / peak)
        achieved = nbytes / t / 1e9
        return dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                    units_per_launch=n_edges, per_unit=f"{nbytes // max(n_edges, 1)} B/edge")
    if stage == "node_step":
        flops = n_hits * (2 * 3 * H * H + 2 * H * H + 2 * 2 * H * H)
        achieved = flops / t / 1e12
        peak = PEAK_TFLOPS[dtype]
        return dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                    units_per_launch=n_hits, per_unit=f"{12 * H * H} flop/hit")
    if stage == "segsum":
        # each edge encoding read once, one 4-byte CSC index per edge, both sums written
        nbytes = n_edges * (H * es + 4) + n_hits * (2 * H * 4 + 16)
        achieved = nbytes / t / 1e9
        return dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                    units_per_launch=n_edges, per_unit=f"{H * es + 4} B/edge + {2 * H * 4 + 16} B/hit")
    return None


def kernel_source_hash(kernel):
    """sha256 of the HIP source that defines a stage's kernel."""
    import hashlib
    src = {"edge_step": "gnn.hip", "edge_step_final": "gnn.hip", "segsum": "gnn.hip", "node_step": "gnn.hip"}[kernel]
    h = hashlib.sha256()
    for f in (src, "tile.hpp"):
        with open(os.path.join(ROOT, "paper_2508_07423_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, dtype):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current source of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)["records"]
    for r in recs:
        if r["kernel"] == kernel and r["workload"] == workload and r["dtype"] == dtype:
            return r["bytes_per_launch"] if r["source_sha256"] == kernel_source_hash(kernel) else None
    return None


def copy_calibration(gib):
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, weights, batch, threads):
    """The FP64 oracle on the host: one thread per event over `threads`
    events, and one event on a single thread."""
    from oracle import oracle as O
    O.lib()
    n = min(threads, len(batch["hit_off"]) - 1)
    t0 = time.perf_counter()
    O.run_batch(batch, w, weights, events=list(range(n)), threads=threads)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    O.run_batch(batch, w, weights, events=[n % max(len(batch["hit_off"]) - 1, 1)], threads=1)
    dt1 = time.perf_counter() - t1
    return dict(value=n / dt, unit="events/s", cores=threads, kind="oracle",
                sample=f"first {n} events of the same batch, one oracle thread per event ({dt:.1f} s wall)",
                single_thread_events_per_s=round(1.0 / dt1, 4), cpu_model=cpu_model(), nproc=os.cpu_count())


def main():
    args = parse()
    if args.copy_gib > 0:
        copy_calibration(args.copy_gib)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              "events are independent, so a multi-GPU run would split the batch by events with no exchange.",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        raise SystemExit("--steps must be at least 1")

    import torch
    from paper_2508_07423_amd import etx, synth

    w = synth.WORKLOADS[args.workload]
    n_events = args.events or w.n_events
    precs = {"fp32": etx.ETX_FP32, "bf16": etx.ETX_BF16, "fp8": etx.ETX_FP8_E4M3, "int8": etx.ETX_INT8}
    prec = precs[args.precision]
    dtype = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8", "int8": "int8"}[args.precision]
    t_gen = time.perf_counter()
    batch = synth.generate_batch(w, n_events)
    use_pf = w.name == "c5"
    # the prefilter learns from what the full pipeline keeps, which needs a trained network
    weights = synth.trained_weights(w) if use_pf else synth.xavier_weights(w)
    print(f"[bench] workload {w.name}: {n_events} events, {int(batch['hit_off'][-1])} hits "
          f"(generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)

    pf_info = None
    if use_pf:
        from paper_2508_07423_amd import evaluate
        from paper_2508_07423_amd import prefilter_train as PT
        t_tr = time.perf_counter()
        tr = PT.train_prefilter(w, weights, n_events=args.pf_train_events, batch_events=20, lr=1e-2,
                                log=lambda m: print(m, file=sys.stderr, flush=True))
        t_tr = time.perf_counter() - t_tr
        sel = PT.choose_tau(w, weights, tr["params"], synth.generate_batch(w, 100, seed_space=6000 + w.cid),
                            recall=args.pf_recall)
        print(f"[bench] prefilter: {args.pf_train_events} training events, {tr['steps']} steps in {t_tr:.1f} s, "
              f"tau {sel['tau']:.4f} keeps {sel['kept_fraction']:.3f} of validation candidates", file=sys.stderr,
              flush=True)
        pf_info = dict(train_events=args.pf_train_events, train_steps=tr["steps"], train_s=round(t_tr, 1),
                       tau=round(sel["tau"], 5), recall_target=args.pf_recall,
                       validation_kept=round(sel["kept_fraction"], 4))

    stream = torch.cuda.Stream()
    cal = None
    if prec in (etx.ETX_FP8_E4M3, etx.ETX_INT8) or (args.emb_precision in ("fp8", "int8")):
        # static calibration on events of a disjoint seed space (on the unpruned graph, before the prefilter is on)
        cal = etx.to_device(synth.generate_batch(w, 20, seed_space=1000 + w.cid))

    def calibrated(pipe):
        if cal is not None:
            with torch.cuda.stream(stream):
                pipe.calibrate(cal, stream=stream)
        return pipe

    compact = bool(args.compact_state) and prec in (etx.ETX_BF16, etx.ETX_FP8_E4M3)
    emb_prec = precs[args.emb_precision or args.precision]

    def configured(pipe):
        etx.etx_set_option(pipe.ctx, etx.ETX_OPT_COMPACT_STATE, int(compact))
        if emb_prec != prec:
            etx.etx_set_option(pipe.ctx, etx.ETX_OPT_EMBED_PRECISION, emb_prec)
        return calibrated(pipe)

    p = configured(etx.Pipeline(w, weights, precision=prec))
    if use_pf:
        etx.etx_prefilter_set(p.ctx, tr["params"])
        etx.etx_prefilter_config(p.ctx, 1, sel["tau"])
    b = etx.to_device(batch)
    tuned = None
    if args.autotune:
        with torch.cuda.stream(stream):
            out = p.allocate(b)
            path = args.autotune_log
            etx.etx_autotune(p.ctx, p.hits_struct(b), out, p.ws_ptr, p.ws_bytes, stream.cuda_stream, path)
        tuned = {k: etx.etx_get_option(p.ctx, v) for k, v in (("edge_threads", etx.ETX_OPT_EDGE_WG_SIZE),
                                                               ("edge_wg_per_cu", etx.ETX_OPT_EDGE_WG_PER_CU),
                                                               ("edge_pipeline", etx.ETX_OPT_EDGE_PIPELINE),
                                                               ("node_wg_per_cu", etx.ETX_OPT_NODE_WG_PER_CU),
                                                               ("fuse_messages", etx.ETX_OPT_FUSE_MESSAGES),
                                                               ("segsum_unroll", etx.ETX_OPT_SEGSUM_UNROLL),
                                                               ("radius_sort_min", etx.ETX_OPT_RADIUS_SORT_MIN),
                                                               ("radius_fast", etx.ETX_OPT_RADIUS_FAST),
                                                               ("xcd_map", etx.ETX_OPT_XCD_MAP),
                                                               ("edge_products", etx.ETX_OPT_EDGE_PRODUCTS),
                                                               ("csc_place", etx.ETX_OPT_CSC_PLACE))}
        print(f"[bench] autotuned: {tuned}", file=sys.stderr, flush=True)
    if args.graph:
        etx.etx_set_option(p.ctx, etx.ETX_OPT_USE_GRAPH, 1)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            p.run(b, stream=stream)
        stream.synchronize()
        if args.warmup > 0:
            res = p.results(b)
            print(f"[bench] warmup done: {int(res['edge_off'][-1])} edges ({int(res['edge_off'][-1]) / b.n_hits:.1f}"
                  f"/hit), kept {(res['score'] >= 0.5).mean():.3f}", file=sys.stderr, flush=True)
        if args.profile_stages and not args.graph:
            etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 1)
            etx.etx_profile_reset(p.ctx)
        torch.cuda.synchronize()
        # HIP events between the passes (on the stream they run on) for the median
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        marks[0].record(stream)
        for k in range(args.steps):
            p.run(b, stream=stream)
            marks[k + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps))
    res = p.results(b)      # raises on a non-zero device status
    n_edges = int(res["edge_off"][-1])
    dt = t1 - t0
    value = n_events * args.steps / dt
    stages = {}
    roof = None
    if args.profile_stages and not args.graph:
        prof = etx.etx_profile_read(p.ctx)
        etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 0)
        stages = {k: dict(ms=round(v[0] / args.steps, 3), launches=v[1]) for k, v in prof.items() if v[1] > 0}
        gnn = {k: v for k, v in prof.items() if k in ("edge_step", "edge_step_final", "segsum", "node_step")}
        dom = max(gnn, key=lambda k: gnn[k][0])
        roof = stage_roofline(dom, gnn[dom][0], gnn[dom][1], n_edges, b.n_hits, w.gnn_hidden, dtype, compact)
        if roof is not None:
            roof = dict(kernel=dom, **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in roof.items()},
                        traffic=measured_traffic(dom, w.name, dtype + ("-compact" if compact else "")))
        print(f"[bench] stages (ms/step): " + ", ".join(f"{k} {v['ms']}" for k, v in stages.items()),
              file=sys.stderr, flush=True)
    if use_pf:
        # the unpruned pipeline on the same batch: its throughput and efficiency are the reference
        p0 = configured(etx.Pipeline(w, weights, precision=prec))
        # the same launch schedule as the pruned pipeline (tuned or default)
        for key in range(etx.ETX_OPT_COMPACT_STATE + 1):
            if key not in (etx.ETX_OPT_PROFILE,):
                etx.etx_set_option(p0.ctx, key, etx.etx_get_option(p.ctx, key))
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                p0.run(b, stream=stream)
            torch.cuda.synchronize()
            u0 = time.perf_counter()
            for _ in range(args.steps):
                p0.run(b, stream=stream)
            torch.cuda.synchronize()
            u1 = time.perf_counter()
        r0 = p0.results(b)
        m0, m1 = evaluate.batch_metrics(r0["labels"], batch), evaluate.batch_metrics(res["labels"], batch)
        pf_info.update(edges_unpruned=int(r0["edge_off"][-1]), edges_kept=n_edges,
                       kept_fraction=round(n_edges / max(int(r0["edge_off"][-1]), 1), 4),
                       unpruned_events_per_s=round(n_events * args.steps / (u1 - u0), 2),
                       efficiency=round(m1["efficiency"], 5), efficiency_unpruned=round(m0["efficiency"], 5))
        p0.close()
    cpu = None
    if args.cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        print(f"[bench] timing the FP64 oracle on {threads} events with {threads} threads", file=sys.stderr,
              flush=True)
        cpu = cpu_baseline(w, weights, batch, threads)
    line = {
        "metric": "events/s (GNN track finding, 1 GPU) at fixed track efficiency vs plain FP32",
        "value": round(value, 2),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "ms_per_step_median": round(step_ms[len(step_ms) // 2], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded straight-track events, " + ("trained weights, learned prefilter)" if use_pf
                                                                  else "random Xavier weights)"),
        "config": {
            "workload": f"{w.name}: {n_events} events, {w.n_planes} planes, tracks {w.tracks[0]}({w.tracks[1]}), "
                        f"emb 3-{w.emb_hidden}x{w.emb_layers}-{w.emb_dim}, radius {w.radius}, k {w.k_max}, "
                        f"IN hidden {w.gnn_hidden} x {w.gnn_steps} steps, {args.precision}"
                        + (f", {args.emb_precision} embedding" if emb_prec != prec else "")
                        + (", compact state" if compact else "") + (", hip graph" if args.graph else ""),
            "events": n_events, "hits": int(b.n_hits), "edges": n_edges, "schedule": tuned,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "prefilter": pf_info,
        "stages_ms_per_step": stages,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
