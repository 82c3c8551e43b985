"""The batched path as it is benchmarked: an uneven batch of the 26-plane
geometry (events of 20 to 600 tracks), tuned by etx_autotune, replayed through
the captured HIP graph, and the tuning table saved and loaded back.

Every launch schedule computes the same bits, so tuned, graph-replayed and
table-restored runs must equal the untuned eager run bit for bit; the eager
run is compared with the FP64 oracle on the smallest, the median and the
largest event, with trained weights (track-like components, so the label
comparison covers almost every hit)."""
import json

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_07423_amd import synth
from tests import gpu_helpers as G
from tests.test_gpu_parity import event_parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("src", "dst", "score", "labels", "edge_off")


def _etx():
    from paper_2508_07423_amd import etx
    return etx


def concat(batches):
    out = {k: np.concatenate([b[k] for b in batches]) for k in ("x", "y", "z", "plane", "particle")}
    counts = np.concatenate([np.diff(b["hit_off"]) for b in batches])
    out["hit_off"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return out


@pytest.fixture(scope="module")
def uneven():
    w = synth.C3
    small = synth.generate_batch(w.with_(tracks=("fixed", 20)), 1, seed_space=9100)
    big = synth.generate_batch(w.with_(tracks=("fixed", 600)), 1, seed_space=9101)
    batch = concat([small, synth.generate_batch(w, 200), big])
    return w, synth.trained_weights(w), batch


def test_autotune_graph_and_table_round_trip(uneven, tmp_path):
    etx = _etx()
    w, W, batch = uneven
    hits = np.diff(batch["hit_off"])
    assert hits.min() < 400 and hits.max() > 6000      # the uneven spread of the workload
    b = etx.to_device(batch)
    p0 = etx.Pipeline(w, W)
    p0.run(b)
    ref = p0.results(b)
    p0.close()

    p = etx.Pipeline(w, W)
    s = torch.cuda.Stream()
    log = tmp_path / "trials.jsonl"
    with torch.cuda.stream(s):
        out = p.allocate(b)
        etx.etx_autotune(p.ctx, p.hits_struct(b), out, p.ws_ptr, p.ws_bytes, s.cuda_stream, str(log))
    rec = json.loads(log.read_text().splitlines()[-1])
    assert rec["n_events"] == len(hits) and rec["arch"].startswith("gfx")
    assert "edge_threads_x_wg_per_cu" in rec["choice"] and "radius_sort_min" in rec["choice"]
    tuned = {k: etx.etx_get_option(p.ctx, getattr(etx, "ETX_OPT_" + k))
             for k in ("EDGE_WG_SIZE", "EDGE_WG_PER_CU", "EDGE_PIPELINE", "NODE_WG_PER_CU", "FUSE_MESSAGES",
                       "SEGSUM_UNROLL", "RADIUS_SORT_MIN", "RADIUS_FAST", "XCD_MAP", "EDGE_PRODUCTS", "CSC_PLACE",
                       "RADIUS_SPLIT")}
    p.run(b)
    r = p.results(b)
    for k in KEYS:
        assert np.array_equal(r[k], ref[k]), ("tuned eager", k)
    # the captured graph, replayed with eager work and host synchronisations between replays
    etx.etx_set_option(p.ctx, etx.ETX_OPT_USE_GRAPH, 1)
    for rep in range(3):
        with torch.cuda.stream(s):
            p.run(b, stream=s)
        s.synchronize()
        g = p.results(b)
        for k in KEYS:
            assert np.array_equal(g[k], ref[k]), ("graph replay", rep, k)
        torch.zeros(1 << 20, device="cuda").sum().item()
    # the tuning table: saved, then loaded by a fresh context, whose first run applies the entry
    table = tmp_path / "tuning.txt"
    etx.etx_tuning_save(p.ctx, str(table))
    text = table.read_text()
    assert any(line.startswith(rec["arch"]) and f"h{int(round(np.log2(hits.mean())))}" in line
               for line in text.splitlines()), text
    p.close()
    q = etx.Pipeline(w, W)
    etx.etx_tuning_load(q.ctx, str(table))
    q.run(b)
    rq = q.results(b)
    for k, v in tuned.items():
        assert etx.etx_get_option(q.ctx, getattr(etx, "ETX_OPT_" + k)) == v, k
    for k in KEYS:
        assert np.array_equal(rq[k], ref[k]), ("table-restored", k)
    q.close()
    _check_events_against_oracle(w, W, batch, ref)


def _check_events_against_oracle(w, W, batch, res):
    hits = np.diff(batch["hit_off"])
    order = np.argsort(hits, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    for i in picks:
        # the trained network amplifies FP32 rounding: the score bound is the FP32 tolerance, or twice
        # the distance between the oracle and the same network evaluated in FP32 arithmetic
        ev = synth.event_slice(batch, i)
        r64, r32 = O.run_event(ev, w, W), O.run_event(ev, w, W, f32=True)
        floor = np.abs(r64["score"] - r32["score"]).max(initial=0.0) if np.array_equal(r64["src"], r32["src"]) \
            and np.array_equal(r64["dst"], r32["dst"]) else G.SCORE_TOL
        tol = max(G.SCORE_TOL, 2 * floor)
        ref, n_undec, frac = event_parity(w, W, batch, res, i, score_tol=tol)
        print(f"event {i}: {hits[i]} hits, {len(ref['src'])} edges, undecidable rows {n_undec}, "
              f"labels compared on {frac:.4f} of the hits, FP32-evaluation floor {floor:.2e}, score bound {tol:.2e}")
        assert frac >= 0.95, (i, frac)


def test_autotune_reports_device_errors_and_restores_options(uneven):
    """A batch that overflows its edge capacity: the tuner reads the device
    status of its first trial, returns the error and leaves the options as
    they were."""
    etx = _etx()
    w, W, batch = uneven
    small = {k: batch[k] for k in ("x", "y", "z", "plane", "particle", "hit_off")}
    sub = synth.event_slice(small, 1)
    one = dict(sub, hit_off=np.array([0, len(sub["x"])], np.int64))
    b = etx.to_device(one)
    p = etx.Pipeline(w, W)
    etx.etx_set_option(p.ctx, etx.ETX_OPT_EDGE_WG_PER_CU, 3)
    before = {k: etx.etx_get_option(p.ctx, k) for k in range(etx.ETX_OPT_COMPACT_STATE + 1)}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = p.allocate(b, edge_capacity=4)
        with pytest.raises(etx.EtxError) as e:
            etx.etx_autotune(p.ctx, p.hits_struct(b), out, p.ws_ptr, p.ws_bytes, s.cuda_stream, None)
    assert e.value.code == etx.ETX_ERR_CAPACITY
    after = {k: etx.etx_get_option(p.ctx, k) for k in range(etx.ETX_OPT_COMPACT_STATE + 1)}
    assert after == before
    p.close()
