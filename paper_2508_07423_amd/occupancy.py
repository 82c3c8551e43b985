"""Occupancy scaling of the pipeline: throughput and per-stage time against
hits per event.

The thesis finds its GPU k-NN graph building scaling worst of all stages with
detector occupancy (ch. 9, throughput against occupancy).  Here the uneven
batch (events of ~250 to ~7,600 hits) is cut into bins of hits per event;
every bin runs as a batch of its own, and the stage times (HIP events around
each stage) are reported per hit and per event, so a stage whose cost grows
faster than the hit count shows up as a rising time per hit.

    python -m paper_2508_07423_amd.occupancy --workload c3 [--precision fp32]

prints one JSON line per bin.
"""
import argparse
import json
import sys
import time
from typing import Dict, Sequence

import numpy as np

BIN_EDGES = (0, 500, 1000, 1500, 2000, 3000, 4500, 1 << 30)


def sub_batch(batch: Dict[str, np.ndarray], events: Sequence[int]) -> Dict[str, np.ndarray]:
    """The given events of a packed batch, packed back to back in that order."""
    ho = batch["hit_off"]
    events = [int(i) for i in events]
    parts = {k: [batch[k][ho[i]:ho[i + 1]] for i in events] for k in ("x", "y", "z", "plane", "particle")}
    counts = np.array([ho[i + 1] - ho[i] for i in events], dtype=np.int64)
    out = {k: (np.concatenate(v) if v else batch[k][:0].copy()) for k, v in parts.items()}
    out["hit_off"] = np.zeros(len(events) + 1, dtype=np.int64)
    np.cumsum(counts, out=out["hit_off"][1:])
    return out


def bins_of(hit_off: np.ndarray, edges: Sequence[int] = BIN_EDGES, max_events: int = 0):
    """(lo, hi, event indices) of every non-empty bin lo <= hits < hi."""
    n = np.diff(hit_off)
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        idx = np.nonzero((n >= lo) & (n < hi))[0]
        if max_events:
            idx = idx[:max_events]
        if len(idx):
            out.append((int(lo), int(hi), idx))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="c3", choices=["c3", "c5"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8", "int8"])
    ap.add_argument("--events", type=int, default=None, help="events generated (default: the workload's)")
    ap.add_argument("--max-events-per-bin", type=int, default=2000)
    ap.add_argument("--passes", type=int, default=5)
    args = ap.parse_args(argv)

    import torch
    from . import etx, synth

    w = synth.WORKLOADS[args.workload]
    batch = synth.generate_batch(w, args.events or w.n_events)
    weights = synth.trained_weights(w) if w.name == "c5" else synth.xavier_weights(w)
    prec = {"fp32": etx.ETX_FP32, "bf16": etx.ETX_BF16, "fp8": etx.ETX_FP8_E4M3, "int8": etx.ETX_INT8}[args.precision]
    p = etx.Pipeline(w, weights, precision=prec)
    if prec in (etx.ETX_FP8_E4M3, etx.ETX_INT8):
        p.calibrate(etx.to_device(synth.generate_batch(w, 20, seed_space=1000 + w.cid)))
    stream = torch.cuda.Stream()
    for lo, hi, idx in bins_of(batch["hit_off"], max_events=args.max_events_per_bin):
        sb = sub_batch(batch, idx)
        b = etx.to_device(sb)
        with torch.cuda.stream(stream):
            p.run(b, stream=stream)                      # warm-up (and workspace)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.passes):
                p.run(b, stream=stream)
            stream.synchronize()
            dt = (time.perf_counter() - t0) / args.passes
            etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 1)
            etx.etx_profile_reset(p.ctx)
            for _ in range(args.passes):
                p.run(b, stream=stream)
            prof = etx.etx_profile_read(p.ctx)
            etx.etx_set_option(p.ctx, etx.ETX_OPT_PROFILE, 0)
        res = p.results(b)
        hits, events = b.n_hits, b.n_events
        edges = int(res["edge_off"][-1])
        stage_ms = {k: v[0] / args.passes for k, v in prof.items() if v[1] > 0}
        line = dict(workload=w.name, precision=args.precision, bin=[lo, hi], events=events,
                    hits_per_event=round(hits / events, 1), edges_per_hit=round(edges / max(hits, 1), 2),
                    ms_per_pass=round(dt * 1e3, 3), events_per_s=round(events / dt, 1),
                    mhits_per_s=round(hits / dt / 1e6, 2),
                    ns_per_hit={k: round(v * 1e6 / hits, 2) for k, v in stage_ms.items()},
                    us_per_event={k: round(v * 1e3 / events, 3) for k, v in stage_ms.items()})
        print(json.dumps(line), flush=True)
    p.close()


if __name__ == "__main__":
    sys.exit(main())
