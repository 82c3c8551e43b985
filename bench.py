#!/usr/bin/env python3
"""Events/s of the GNN track-finding hot path on one MI355X.

One step = one pass of the whole path (features, embedding MLP, radius graph,
interaction network, score cut, components) over one batch of synthetic
events already resident in HBM.  The default workload is the full-size plain
FP32 batch: 1000 events, 26 planes at z in [-290, 750] mm, Poisson(200)
tracks per event (~2500 hits incl. 5 % noise), embedding 3-128-128-12, radius
0.12, at most 64 neighbours, interaction network hidden 64 with 8 steps,
random Xavier weights.

Measurement order for the headline workload: warm-up passes; instrumented
passes (a HIP event pair around every stage) for the per-stage times, which
also name the dominant interaction-network kernel; then the timed passes, in
which only that kernel's launches carry HIP event pairs (its average launch
time gives the roofline); the throughput is events x passes over the host
wall time between two device synchronisations around the timed passes.

With the default ``--spec 1`` the same run adds the comparison the
metric is quoted as: the 10,000-event uneven batch (plain FP32, autotuned, one
HIP graph per pass), and the same batch with trained weights with and without
the learned prefilter (trained first, on the GPU), in FP32 and with BF16
operands, each with its events/s, the kept fraction of candidate edges and the
track efficiency against the unpruned FP32 pipeline.

Prints one JSON line.
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
DTYPES = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8", "int8": "int8"}
GNN_KERNELS = ("edge_step", "edge_step_final", "segsum", "node_step", "edge_encode")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
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
    ap.add_argument("--profile-stages", type=int, default=1,
                    help="instrumented passes before the timed ones (per-stage times, the roofline kernel)")
    ap.add_argument("--north-star", type=int, default=None,
                    help="add the uneven-batch and prefilter comparison (default: on for the c2 headline)")
    ap.add_argument("--ns-steps", type=int, default=20, help="timed passes of each north-star leg")
    ap.add_argument("--triplets-only", type=int, default=0,
                    help="1: only the conversion-pair comparison (components against the triplet stage), "
                         "printed as one JSON line")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# algorithmic work per launch
# ---------------------------------------------------------------------------

def stage_roofline(stage, ms_total, launches, n_edges, n_hits, H, dtype, compact):
    """Roofline of one interaction-network kernel from its average launch time.

    MFMA-bound kernels are priced on the products they execute on the matrix
    cores: the edge step's first layer is factorised (the node products
    h W_src, h W_dst are formed per node and gathered), so an edge step
    executes two H x H products per edge (4H^2 flop) where the unfactorised
    edge network would need 8H^2; the 8H^2 rate is reported beside it as the
    algorithmic-equivalent rate and never compared with the peak."""
    if launches == 0 or ms_total <= 0:
        return None
    t = ms_total / launches * 1e-3          # seconds per launch
    # bytes per stored edge-encoding feature: FP32 master copies unless the state is compact
    es = {"f32": 4, "bf16": 2, "fp8": 1, "int8": 1}[dtype] if compact else 4
    peak = PEAK_TFLOPS[dtype]
    if stage in ("edge_step", "edge_step_final"):
        fin = stage == "edge_step_final"
        # edge net Linear(3H->H) + Linear(H->H) per edge; the last step adds the classifier
        # Block(H->H) + Linear(H->1)
        alg = n_edges * (8 * H * H + (2 * H * H + 2 * H if fin else 0))
        xflops = n_edges * (4 * H * H + (2 * H * H if fin else 0))
        nbytes = n_edges * (H * es + (4 if fin else H * es) + 8)
        if xflops / (peak * 1e12) >= nbytes / (PEAK_HBM_GBS * 1e9):
            ach = xflops / t / 1e12
            return dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                        units_per_launch=n_edges, per_unit=f"{xflops // max(n_edges, 1)} flop/edge (MFMA, executed)",
                        algorithmic_per_unit=f"{alg // max(n_edges, 1)} flop/edge (unfactorised edge network)",
                        algorithmic_equivalent_tflops=alg / t / 1e12, hbm_bytes_per_launch=nbytes,
                        hbm_frac=nbytes / t / 1e9 / PEAK_HBM_GBS)
        ach = nbytes / t / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS,
                    units_per_launch=n_edges, per_unit=f"{nbytes // max(n_edges, 1)} B/edge",
                    mfma_frac=xflops / t / 1e12 / peak)
    if stage == "node_step":
        # node net Linear(3H->H) + Linear(H->H), plus the two edge-net node products h W_src, h W_dst
        xflops = n_hits * (2 * 3 * H * H + 2 * H * H + 2 * 2 * H * H)
        ach = xflops / t / 1e12
        return dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    units_per_launch=n_hits, per_unit=f"{12 * H * H} flop/hit")
    if stage == "segsum":
        nbytes = segsum_bytes(n_edges, n_hits, H, es)
        ach = nbytes / t / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS,
                    units_per_launch=n_edges, per_unit=f"{H * es + 4} B/edge + {2 * H * 4 + 16} B/hit")
    if stage == "edge_encode":
        nbytes = edge_encode_bytes(n_edges, n_hits, H, es)
        ach = nbytes / t / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS,
                    units_per_launch=n_edges, per_unit=f"{H * es + 8} B/edge + {3 * H * 4} B/hit",
                    mfma_frac=n_edges * 2 * H * H / t / 1e12 / peak)
    return None


def segsum_bytes(E, N, H, es):
    # each edge encoding read once through the CSC, one 4-byte CSC id per edge; both sums written per hit
    return E * (H * es + 4) + N * (2 * H * 4 + 16)


def edge_encode_bytes(E, N, H, es):
    # per edge: src, dst and the stored encoding; per hit: the two node-product rows read once and the
    # out-sum row written
    return E * (H * es + 8) + N * (3 * H * 4)


def stage_hbm(stages, E_cand, E, E_kept, N, D, H, es):
    """Gather/scatter stages against the HBM roofline, on algorithmic bytes.

    radius (search + scan + row copy): the embedding read once per hit (D floats), the edges written
    (src, dst) with their row offsets; edge encoder, message sums: as above; score cut: every score
    read, the kept edge ids written."""
    def frac(nbytes, ms):
        return None if ms <= 0 else dict(bytes=int(nbytes), ms=round(ms, 4), tbs=round(nbytes / ms / 1e9, 3),
                                         frac=round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 4))
    get = lambda k: stages.get(k, {"ms": 0.0, "launches": 0})
    rad_ms = sum(get(k)["ms"] for k in ("radius_count", "scan", "radius_emit"))
    out = {"a3_radius": frac(N * (4 * D + 4) + E_cand * 8 + (N + 1) * 8, rad_ms),
           "a5_edge_encode": frac(edge_encode_bytes(E, N, H, es), get("edge_encode")["ms"]),
           "a8_compact": frac(E * 4 + E_kept * 4, get("compact")["ms"])}
    s = get("segsum")
    if s["launches"]:
        per = s["ms"] / max(s["launches"], 1)
        steps = s["launches"]
        out["a6_segsum"] = frac(segsum_bytes(E, N, H, es), per)
        out["a6_segsum"]["per_launch"] = True
        out["a6_segsum"]["launches_per_pass"] = steps
    return out


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def kernel_source_hash(kernel):
    """sha256 of the HIP source that defines a stage's kernel."""
    import hashlib
    src = {"edge_step": "gnn.hip", "edge_step_final": "gnn.hip", "segsum": "gnn.hip", "node_step": "gnn.hip",
           "edge_encode": "gnn.hip"}[kernel]
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


TUNED_KEYS = ("EDGE_WG_SIZE", "EDGE_WG_PER_CU", "EDGE_PIPELINE", "NODE_WG_PER_CU", "FUSE_MESSAGES", "SEGSUM_UNROLL",
              "RADIUS_SORT_MIN", "RADIUS_FAST", "XCD_MAP", "EDGE_PRODUCTS", "CSC_PLACE",
              "RADIUS_SPLIT")


def schedule(etx, ctx):
    return {k.lower(): etx.etx_get_option(ctx, getattr(etx, "ETX_OPT_" + k)) for k in TUNED_KEYS}


def make_pipeline(etx, synth, w, weights, prec, emb_prec, compact, cal_batch, stream):
    import torch
    p = etx.Pipeline(w, weights, precision=prec)
    etx.etx_set_option(p.ctx, etx.ETX_OPT_COMPACT_STATE, int(compact))
    if emb_prec != prec:
        etx.etx_set_option(p.ctx, etx.ETX_OPT_EMBED_PRECISION, emb_prec)
    scaled = (etx.ETX_FP8_E4M3, etx.ETX_INT8)
    if prec in scaled or emb_prec in scaled:
        # static calibration on events of a disjoint seed space (the unpruned graph)
        with torch.cuda.stream(stream):
            p.calibrate(cal_batch, stream=stream)
    return p


def timed_passes(p, b, stream, steps, warmup):
    """Warm-up, then `steps` passes between two device synchronisations; returns
    (events/s, ms per pass, median ms per pass from HIP events between passes)."""
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            p.run(b, stream=stream)
        torch.cuda.synchronize()
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        marks[0].record(stream)
        for k in range(steps):
            p.run(b, stream=stream)
            marks[k + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    med = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))[steps // 2]
    return b.n_events * steps / (t1 - t0), (t1 - t0) / steps * 1e3, med


def autotune(etx, p, b, stream, path):
    import torch
    with torch.cuda.stream(stream):
        out = p.allocate(b)
        etx.etx_autotune(p.ctx, p.hits_struct(b), out, p.ws_ptr, p.ws_bytes, stream.cuda_stream, path)
    return schedule(etx, p.ctx)


# ---------------------------------------------------------------------------
# the comparison the metric is quoted as
# ---------------------------------------------------------------------------

def north_star(args, stream):
    """Uneven 10,000-event batch: plain FP32 with random weights (autotuned, HIP
    graph); then trained weights with and without the learned prefilter, FP32
    and BF16 operands, efficiency against the unpruned FP32 pipeline."""
    import torch
    from paper_2508_07423_amd import etx, evaluate, synth
    from paper_2508_07423_amd import prefilter_train as PT
    res = {}
    steps = args.ns_steps

    def leg(w, weights, batch, prec, pf=None, name="", compact=False):
        p = make_pipeline(etx, synth, w, weights, prec, prec, compact, None, stream)
        if pf is not None:
            etx.etx_prefilter_set(p.ctx, pf["params"])
            etx.etx_prefilter_config(p.ctx, 1, pf["tau"])
            etx.etx_prefilter_band(p.ctx, *pf["band"])
        b = etx.to_device(batch)
        t0 = time.perf_counter()
        tuned = autotune(etx, p, b, stream, args.autotune_log)
        t_tune = time.perf_counter() - t0
        etx.etx_set_option(p.ctx, etx.ETX_OPT_USE_GRAPH, 1)
        eps, ms, med = timed_passes(p, b, stream, steps, 2)
        torch.cuda.synchronize()
        st = p.status.cpu().numpy()
        if st[0] != etx.ETX_OK:
            raise etx.EtxError(int(st[0]), f"{name}: device status")
        r = dict(edge_off=p.edge_off.cpu().numpy(), labels=p.labels[:b.n_hits].cpu().numpy())
        fallback = None
        if pf is not None:
            fallback = int(p.view(b, etx.ETX_VIEW_PF_FALLBACK, torch.int32).sum().item())
        p.close()
        del b
        torch.cuda.empty_cache()
        log(f"[bench] {name}: {eps:.0f} events/s ({ms:.2f} ms per pass, tuning {t_tune:.0f} s)")
        out = dict(events_per_s=round(eps, 1), ms_per_pass=round(ms, 3), ms_per_pass_median=round(med, 3),
                   steps=steps, edges=int(r["edge_off"][-1]), schedule=tuned, tune_s=round(t_tune, 1))
        if fallback is not None:
            out["fallback_events"] = fallback
        return out, r

    # c3: uneven batch, plain FP32, random weights
    w3 = synth.WORKLOADS["c3"]
    t0 = time.perf_counter()
    batch3 = synth.generate_batch(w3, w3.n_events)
    log(f"[bench] c3: {w3.n_events} events, {int(batch3['hit_off'][-1])} hits "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    r3, _ = leg(w3, synth.xavier_weights(w3), batch3, etx.ETX_FP32, name="c3 fp32 graph autotuned")
    hits = np.diff(batch3["hit_off"])
    r3.update(workload=f"c3: {w3.n_events} events, tracks lognormal-mixed Poisson(150) clipped [20, 600], "
                       f"{int(hits.min())}-{int(hits.max())} hits/event, IN hidden {w3.gnn_hidden} x "
                       f"{w3.gnn_steps}, fp32, random Xavier weights, hip graph, autotuned",
              hits=int(batch3["hit_off"][-1]))
    res["c3_fp32"] = r3
    del batch3

    # c5: the same kind of batch with trained weights; the prefilter trained on the GPU first
    w5 = synth.WORKLOADS["c5"]
    weights5 = synth.trained_weights(w5)
    t0 = time.perf_counter()
    tr = PT.train_prefilter(w5, weights5, n_events=args.pf_train_events, batch_events=20, lr=1e-2, log=log)
    t_tr = time.perf_counter() - t0
    sel = PT.choose_tau(w5, weights5, tr["params"], synth.generate_batch(w5, 100, seed_space=6000 + w5.cid),
                        recall=args.pf_recall)
    pf = dict(params=tr["params"], tau=sel["tau"], band=sel["band"])
    log(f"[bench] prefilter: {args.pf_train_events} events, {tr['steps']} steps, {t_tr:.1f} s; "
        f"tau {sel['tau']:.4f} keeps {sel['kept_fraction']:.3f} of validation candidates")
    batch5 = synth.generate_batch(w5, w5.n_events)
    legs = {}
    for name, prec, use_pf, compact in (("fp32_unpruned", etx.ETX_FP32, False, False),
                                        ("fp32_pruned", etx.ETX_FP32, True, False),
                                        ("bf16_pruned", etx.ETX_BF16, True, False),
                                        ("bf16_compact_pruned", etx.ETX_BF16, True, True),
                                        ("bf16_unpruned", etx.ETX_BF16, False, False)):
        r, out = leg(w5, weights5, batch5, prec, pf if use_pf else None, name=f"c5 {name}", compact=compact)
        m = evaluate.batch_metrics(out["labels"], batch5)
        r.update(efficiency=round(m["efficiency"], 5), ghost_rate=round(m["ghost_rate"], 5))
        legs[name] = r
    base = legs["fp32_unpruned"]
    for name, r in legs.items():
        r["kept_fraction"] = round(r["edges"] / max(base["edges"], 1), 4)
        r["delta_efficiency_vs_fp32_unpruned"] = round(r["efficiency"] - base["efficiency"], 5)
        r["speedup_vs_fp32_unpruned"] = round(r["events_per_s"] / base["events_per_s"], 3)
    del batch5
    res["c6"] = triplet_legs(args, stream)
    res["c5"] = dict(workload=f"c5: {w5.n_events} events as c3, trained weights, learned prefilter "
                              f"6-32-32-1, hip graph, autotuned per leg",
                     prefilter=dict(train_events=args.pf_train_events, train_steps=tr["steps"],
                                    train_s=round(t_tr, 1), tau=round(sel["tau"], 5),
                                    recall_target=args.pf_recall,
                                    validation_kept=round(sel["kept_fraction"], 4),
                                    fallback_band=[round(x, 4) for x in sel["band"]]),
                     legs=legs)
    return res


def timed_track_passes(p, b, stream, steps, warmup, caps):
    """timed_passes for etx_run_tracks (eager) with fixed capacities."""
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            p.run_tracks(b, stream=stream, **caps)
        torch.cuda.synchronize()
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        marks[0].record(stream)
        for k in range(steps):
            p.run_tracks(b, stream=stream, **caps)
            marks[k + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    med = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))[steps // 2]
    return b.n_events * steps / (t1 - t0), (t1 - t0) / steps * 1e3, med


def triplet_legs(args, stream):
    """Conversion-pair batch (c6): the plain pipeline's components (the c3
    network) against the triplet stage's tracks (the network and triplet
    classifiers trained together on the GPU), events/s and track metrics with
    shared hits counted for both particles; stage times of the triplet stage
    from a separate instrumented run, and the triplet classifiers' roofline."""
    import torch
    from paper_2508_07423_amd import etx, evaluate, synth
    w = synth.WORKLOADS["c6"]
    steps = args.ns_steps
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    batch = synth.generate_batch(w, w.n_events)
    log(f"[bench] c6: {w.n_events} events, {int(batch['hit_off'][-1])} hits, "
        f"{int((batch['particle2'] >= 0).sum())} shared (generated in {time.perf_counter() - t0:.1f} s)")
    b = etx.to_device(batch)
    out = {}
    # plain pipeline: components of the kept graph
    p = etx.Pipeline(w, synth.trained_weights(synth.WORKLOADS["c3"]))
    tuned = autotune(etx, p, b, stream, args.autotune_log)
    etx.etx_set_option(p.ctx, etx.ETX_OPT_USE_GRAPH, 1)
    eps, ms, med = timed_passes(p, b, stream, steps, 2)
    res = p.results(b)
    m = evaluate.track_list_metrics(*evaluate.tracks_from_labels(res["labels"], batch), batch)
    out["components"] = dict(events_per_s=round(eps, 1), ms_per_pass=round(ms, 3), ms_per_pass_median=round(med, 3),
                             steps=steps, schedule=tuned, **{k: round(v, 5) if isinstance(v, float) else v
                                                            for k, v in m.items()})
    log(f"[bench] c6 components: {eps:.0f} events/s ({ms:.2f} ms per pass), efficiency {m['efficiency']:.4f}, "
        f"pair efficiency {m['pair_efficiency']:.4f}")
    # the triplet leg's graph is the same (same embedding): size its edge buffers from it, not from k_max per hit
    edge_cap = int(res["edge_off"][-1] * 1.25) + 1024
    p.close()
    del p, res
    torch.cuda.empty_cache()
    # triplet stage
    p = etx.Pipeline(w, synth.trained_weights(w))
    p.set_triplets(synth.trained_triplets(w))
    with torch.cuda.stream(stream):
        out_ = p.allocate(b, edge_capacity=edge_cap)
        etx.etx_autotune(p.ctx, p.hits_struct(b), out_, p.ws_ptr, p.ws_bytes, stream.cuda_stream, args.autotune_log)
    tuned = schedule(etx, p.ctx)
    with torch.cuda.stream(stream):
        p.run_tracks_sized(b, stream=stream, edge_capacity=edge_cap)
    tc, kc, hc = p._trk_shape[:3]
    caps = dict(triplet_capacity=tc, track_capacity=kc, hit_capacity=hc, edge_capacity=edge_cap)
    eps, ms, med = timed_track_passes(p, b, stream, steps, 2, caps)
    tres = p.track_results(b)
    res = p.results(b)
    m = evaluate.track_list_metrics(tres["tracks"], tres["event_track_off"], batch)
    n_tri = int(tres["elb_off"][-1])
    n_art = int(tres["art_off"][-1])
    # instrumented passes: stage times
    etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 1)
    etx.etx_profile_reset(p.ctx)
    n_prof = 3
    with torch.cuda.stream(stream):
        for _ in range(n_prof):
            p.run_tracks(b, stream=stream, **caps)
    torch.cuda.synchronize()
    prof = etx.etx_profile_read(p.ctx)
    etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 0)
    stage_ms = {k: round(v[0] / n_prof, 3) for k, v in prof.items() if v[1] > 0}
    H = w.gnn_hidden
    ms_score = prof["triplet_score"][0] / prof["triplet_score"][1]          # both classifiers' launches of a pass
    flops = 6 * H * H * n_tri                                              # 2 x (2H x H + H x H) on the matrix cores
    nbytes = (2 * 4 * H + 12) * n_tri                                      # two gathered rows, the pair, the score
    out["triplets"] = dict(
        events_per_s=round(eps, 1), ms_per_pass=round(ms, 3), ms_per_pass_median=round(med, 3), steps=steps,
        schedule=tuned, triplets=n_tri, articulations=n_art, track_list=len(tres["tracks"]),
        edges=int(res["edge_off"][-1]), stage_ms=stage_ms,
        classifier_roofline=dict(kernel="tri_score", bound="mfma", ms_per_pass=round(ms_score, 4),
                                 achieved=round(flops / ms_score / 1e9, 2), peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                                 frac=round(flops / ms_score / 1e9 / PEAK_TFLOPS["f32"], 4),
                                 per_unit=f"{6 * H * H} flop/triplet (MFMA)",
                                 hbm_frac=round(nbytes / ms_score / 1e6 / PEAK_HBM_GBS, 4)),
        **{k: round(v, 5) if isinstance(v, float) else v for k, v in m.items()})
    log(f"[bench] c6 triplets: {eps:.0f} events/s ({ms:.2f} ms per pass), efficiency {m['efficiency']:.4f}, "
        f"pair efficiency {m['pair_efficiency']:.4f}; {n_tri} triplets, stages {stage_ms}")
    p.close()
    del p
    torch.cuda.empty_cache()
    # the same with BF16 operands and the compact BF16 state (the classifiers read BF16 edge encodings)
    p = etx.Pipeline(w, synth.trained_weights(w), precision=etx.ETX_BF16)
    etx.etx_set_option(p.ctx, etx.ETX_OPT_COMPACT_STATE, 1)
    p.set_triplets(synth.trained_triplets(w))
    with torch.cuda.stream(stream):
        out_ = p.allocate(b, edge_capacity=edge_cap)
        etx.etx_autotune(p.ctx, p.hits_struct(b), out_, p.ws_ptr, p.ws_bytes, stream.cuda_stream, args.autotune_log)
        p.run_tracks_sized(b, stream=stream, edge_capacity=edge_cap)
    tc, kc, hc = p._trk_shape[:3]
    caps = dict(triplet_capacity=tc, track_capacity=kc, hit_capacity=hc, edge_capacity=edge_cap)
    eps, ms, med = timed_track_passes(p, b, stream, steps, 2, caps)
    tres = p.track_results(b)
    m = evaluate.track_list_metrics(tres["tracks"], tres["event_track_off"], batch)
    out["triplets_bf16_compact"] = dict(events_per_s=round(eps, 1), ms_per_pass=round(ms, 3),
                                        ms_per_pass_median=round(med, 3), steps=steps, schedule=schedule(etx, p.ctx),
                                        triplets=int(tres["elb_off"][-1]),
                                        **{k: round(v, 5) if isinstance(v, float) else v for k, v in m.items()})
    log(f"[bench] c6 triplets bf16 compact: {eps:.0f} events/s ({ms:.2f} ms per pass), efficiency "
        f"{m['efficiency']:.4f}, pair efficiency {m['pair_efficiency']:.4f}")
    p.close()
    c, t = out["components"], out["triplets"]
    out["workload"] = (f"c6: {w.n_events} events as c3 with conversion pairs (a tenth of the tracks shares its first "
                       f"1-3 hits with a partner), eager triplet stage after an autotuned network")
    out["delta_efficiency_triplets_vs_components"] = round(t["efficiency"] - c["efficiency"], 5)
    out["delta_pair_efficiency"] = round(t["pair_efficiency"] - c["pair_efficiency"], 5)
    out["throughput_ratio"] = round(t["events_per_s"] / c["events_per_s"], 3)
    del b
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------

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

    if args.triplets_only:
        stream = torch.cuda.Stream()
        print(json.dumps(dict(c6=triplet_legs(args, stream))), flush=True)
        return
    w = synth.WORKLOADS[args.workload]
    n_events = args.events or w.n_events
    precs = {"fp32": etx.ETX_FP32, "bf16": etx.ETX_BF16, "fp8": etx.ETX_FP8_E4M3, "int8": etx.ETX_INT8}
    prec = precs[args.precision]
    dtype = DTYPES[args.precision]
    t_gen = time.perf_counter()
    batch = synth.generate_batch(w, n_events)
    use_pf = w.name == "c5"
    # the prefilter learns from what the full pipeline keeps, which needs a trained network
    weights = synth.trained_weights(w) if use_pf else synth.xavier_weights(w)
    log(f"[bench] workload {w.name}: {n_events} events, {int(batch['hit_off'][-1])} hits "
        f"(generated in {time.perf_counter() - t_gen:.1f} s)")

    pf_info = None
    if use_pf:
        from paper_2508_07423_amd import prefilter_train as PT
        t_tr = time.perf_counter()
        tr = PT.train_prefilter(w, weights, n_events=args.pf_train_events, batch_events=20, lr=1e-2, log=log)
        t_tr = time.perf_counter() - t_tr
        sel = PT.choose_tau(w, weights, tr["params"], synth.generate_batch(w, 100, seed_space=6000 + w.cid),
                            recall=args.pf_recall)
        log(f"[bench] prefilter: {args.pf_train_events} training events, {tr['steps']} steps in {t_tr:.1f} s, "
            f"tau {sel['tau']:.4f} keeps {sel['kept_fraction']:.3f} of validation candidates")
        pf_info = dict(train_events=args.pf_train_events, train_steps=tr["steps"], train_s=round(t_tr, 1),
                       tau=round(sel["tau"], 5), recall_target=args.pf_recall,
                       validation_kept=round(sel["kept_fraction"], 4))

    stream = torch.cuda.Stream()
    cal = etx.to_device(synth.generate_batch(w, 20, seed_space=1000 + w.cid))
    compact = bool(args.compact_state) and prec in (etx.ETX_BF16, etx.ETX_FP8_E4M3)
    emb_prec = precs[args.emb_precision or args.precision]
    p = make_pipeline(etx, synth, w, weights, prec, emb_prec, compact, cal, stream)
    if use_pf:
        etx.etx_prefilter_set(p.ctx, tr["params"])
        etx.etx_prefilter_config(p.ctx, 1, sel["tau"])
        etx.etx_prefilter_band(p.ctx, *sel["band"])
    b = etx.to_device(batch)
    tuned = autotune(etx, p, b, stream, args.autotune_log) if args.autotune else None
    if tuned:
        log(f"[bench] autotuned: {tuned}")
    if args.graph:
        etx.etx_set_option(p.ctx, etx.ETX_OPT_USE_GRAPH, 1)
    profiled = args.profile_stages and not args.graph
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            p.run(b, stream=stream)
        stream.synchronize()
        if args.warmup > 0:
            res = p.results(b)
            log(f"[bench] warmup done: {int(res['edge_off'][-1])} edges ({int(res['edge_off'][-1]) / b.n_hits:.1f}"
                f"/hit), kept {(res['score'] >= 0.5).mean():.3f}")
        stages, dom = {}, None
        if profiled:
            # instrumented passes: every stage between HIP events (per-stage times, the dominant kernel)
            n_prof = min(args.steps, 5)
            etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 1)
            etx.etx_profile_reset(p.ctx)
            for _ in range(n_prof):
                p.run(b, stream=stream)
            prof = etx.etx_profile_read(p.ctx)
            stages = {k: dict(ms=round(v[0] / n_prof, 3), launches=v[1] // n_prof) for k, v in prof.items()
                      if v[1] > 0}
            gnn = {k: v for k, v in prof.items() if k in GNN_KERNELS and v[1] > 0}
            dom = max(gnn, key=lambda k: gnn[k][0])
            # the timed passes then carry HIP events around the dominant kernel's launches only
            names = [etx.etx_stage_name(i) for i in range(etx.N_STAGES)]
            etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE_STAGES, 1 << names.index(dom))
            etx.etx_profile_reset(p.ctx)
            log("[bench] stages (ms/pass, instrumented): " + ", ".join(f"{k} {v['ms']}" for k, v in stages.items()))
        torch.cuda.synchronize()
    value, ms_step, ms_med = timed_passes(p, b, stream, args.steps, 0)
    res = p.results(b)      # raises on a non-zero device status
    n_edges = int(res["edge_off"][-1])
    n_kept = int((res["score"] >= w.threshold).sum())
    roof, hbm = None, None
    if profiled:
        tprof = etx.etx_profile_read(p.ctx)[dom]
        etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 0)
        es = (4 if not compact else {"bf16": 2, "fp8": 1}[dtype])
        roof = stage_roofline(dom, tprof[0], tprof[1], n_edges, b.n_hits, w.gnn_hidden, dtype, compact)
        if roof is not None:
            roof = dict(kernel=dom, launches_timed=tprof[1], ms_per_launch=round(tprof[0] / max(tprof[1], 1), 4),
                        **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in roof.items()},
                        traffic=measured_traffic(dom, w.name, dtype + ("-compact" if compact else "")))
        # (with the prefilter the radius stage writes the candidates, here counted as the kept edges)
        hbm = stage_hbm(stages, n_edges, n_edges, n_kept, b.n_hits, w.emb_dim, w.gnn_hidden, es)
    if use_pf:
        # the unpruned pipeline on the same batch: its throughput and efficiency are the reference
        from paper_2508_07423_amd import evaluate
        p0 = make_pipeline(etx, synth, w, weights, prec, emb_prec, compact, cal, stream)
        for key in range(etx.ETX_OPT_COMPACT_STATE + 1):
            if key != etx.ETX_OPT_PROFILE:
                etx.etx_set_option(p0.ctx, key, etx.etx_get_option(p.ctx, key))
        u_eps, _, _ = timed_passes(p0, b, stream, args.steps, args.warmup)
        r0 = p0.results(b)
        m0, m1 = evaluate.batch_metrics(r0["labels"], batch), evaluate.batch_metrics(res["labels"], batch)
        pf_info.update(edges_unpruned=int(r0["edge_off"][-1]), edges_kept=n_edges,
                       kept_fraction=round(n_edges / max(int(r0["edge_off"][-1]), 1), 4),
                       unpruned_events_per_s=round(u_eps, 2),
                       efficiency=round(m1["efficiency"], 5), efficiency_unpruned=round(m0["efficiency"], 5))
        p0.close()
    cpu = None
    if args.cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        log(f"[bench] timing the FP64 oracle on {threads} events with {threads} threads")
        cpu = cpu_baseline(w, weights, batch, threads)
    p.close()
    del b
    torch.cuda.empty_cache()
    ns = None
    if args.north_star if args.north_star is not None else (args.workload == "c2" and args.events is None):
        ns = north_star(args, stream)
    line = {
        "metric": "events/s (GNN track finding, 1 GPU) at fixed track efficiency vs plain FP32",
        "value": round(value, 2),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_per_step_median": round(ms_med, 3),
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
            "events": n_events, "hits": int(b_hits(batch)), "edges": n_edges, "schedule": tuned,
        },
        "timed_region": ("HIP event pair around each launch of the roofline kernel only; per-stage times from "
                         "separate instrumented passes") if profiled else "uninstrumented",
        "roofline": roof,
        "stage_hbm": hbm,
        "cpu_baseline": cpu,
        "prefilter": pf_info,
        "stages_ms_per_step": stages,
        "north_star": ns,
    }
    print(json.dumps(line), flush=True)


def b_hits(batch):
    return batch["hit_off"][-1]


if __name__ == "__main__":
    main()
