"""Edge cases of the HIP path: empty and ragged batches, degenerate events,
the k_max cap with exact ties, windows larger than LDS, and the device-side
error paths (capacity, invalid input, unsupported sizes) forced from the host.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_07423_amd import synth
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _etx():
    from paper_2508_07423_amd import etx
    return etx


def pack(events):
    """Pack a list of event dicts (x, y, z, plane) into a batch."""
    counts = [len(e["x"]) for e in events]
    off = np.zeros(len(events) + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    cat = lambda k, dt: (np.concatenate([np.asarray(e[k], dt) for e in events]) if events and off[-1] > 0
                         else np.zeros(0, dt))
    return dict(x=cat("x", np.float32), y=cat("y", np.float32), z=cat("z", np.float32),
                plane=cat("plane", np.int32), particle=np.full(int(off[-1]), -1, np.int32), hit_off=off)


def run(w, weights, batch, cap=None, check=True):
    etx = _etx()
    p = etx.Pipeline(w, weights)
    b = etx.to_device(batch)
    p.run(b, edge_capacity=cap)
    torch.cuda.synchronize()
    st = p.status.cpu().numpy()
    res = p.results(b) if (check and st[0] == 0) else None
    return p, b, st, res


def oracle_batch_check(w, W, batch, res):
    for i in range(len(batch["hit_off"]) - 1):
        a, e = int(batch["hit_off"][i]), int(batch["hit_off"][i + 1])
        ev = {k: batch[k][a:e] for k in ("x", "y", "z", "plane")}
        ref = O.run_event(ev, w, W, with_margins=True)
        e0, e1 = int(res["edge_off"][i]), int(res["edge_off"][i + 1])
        gs, gd, sc = res["src"][e0:e1] - a, res["dst"][e0:e1] - a, res["score"][e0:e1]
        if e - a == 0:
            assert e1 == e0
            continue
        G.check_edges(gs, gd, ref, ev["plane"], w, ref["emb"])
        _, cart = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
        G.check_scores(gs, gd, sc, cart, W, w, ref)
        G.check_labels(e - a, gs, gd, sc, res["labels"][a:e] - a, ref)


def test_empty_batch():
    w = synth.C1
    W = synth.xavier_weights(w)
    p, b, st, res = run(w, W, pack([]))
    assert st[0] == 0
    assert res["edge_off"].tolist() == [0] and len(res["src"]) == 0


def test_ragged_batch_with_degenerate_events():
    w = synth.C1
    W = synth.xavier_weights(w)
    e0 = synth.generate_event(w, 0)
    e3 = synth.generate_event(w, 3)
    one = {k: e0[k][:1] for k in ("x", "y", "z", "plane")}
    same_plane = {k: e3[k][e3["plane"] == 4] for k in ("x", "y", "z", "plane")}
    empty = {k: e0[k][:0] for k in ("x", "y", "z", "plane")}
    last_plane = {k: e0[k][e0["plane"] == w.n_planes - 1] for k in ("x", "y", "z", "plane")}
    batch = pack([empty, e0, one, empty, same_plane, last_plane, e3, empty])
    p, b, st, res = run(w, W, batch)
    assert st[0] == 0
    eo = res["edge_off"]
    # events with no pair of planes in reach have no edges and singleton labels
    for i in (0, 2, 3, 4, 5, 7):
        assert eo[i + 1] == eo[i]
    a, e = int(batch["hit_off"][4]), int(batch["hit_off"][5])
    assert np.array_equal(res["labels"][a:e], np.arange(a, e))
    oracle_batch_check(w, W, batch, res)


def _identity_embedding_weights(w):
    """Embedding = (r/R_s, phi/pi, z/Z_s, 0, ...) exactly: ReLU(x) - ReLU(-x)."""
    W = synth.xavier_weights(w)
    Wd = w.emb_hidden
    W1 = np.zeros((3, Wd), np.float32)
    for k in range(3):
        W1[k, k] = 1.0
        W1[k, k + 3] = -1.0
    W2 = np.zeros((Wd, Wd), np.float32)
    for k in range(6):
        W2[k, k] = 1.0
    W3 = np.zeros((Wd, w.emb_dim), np.float32)
    for k in range(3):
        W3[k, k] = 1.0
        W3[k + 3, k] = -1.0
    W["emb"] = [(W1, np.zeros(Wd, np.float32)), (W2, np.zeros(Wd, np.float32)),
                (W3, np.zeros(w.emb_dim, np.float32))]
    return W


@pytest.mark.parametrize("k_max", [1, 2, 3])
def test_cap_tie_break_by_smaller_index(k_max):
    w = synth.C1.with_(k_max=k_max, radius=0.5)
    W = _identity_embedding_weights(w)
    # source (index 5) on plane 0 at phi = 0; targets on plane 1 in mirrored
    # pairs (phi = +-a), exactly equidistant in the embedding
    xs = [20.0, 20.0, 20.0, 20.0, 20.0, 20.0]
    ys = [3.0, -1.0, 1.0, -3.0, 2.5, 0.0]
    pl = [1, 1, 1, 1, 3, 0]
    zs = [50.0, 50.0, 50.0, 50.0, 150.0, 0.0]
    batch = pack([dict(x=xs, y=ys, z=zs, plane=pl)])
    p, b, st, res = run(w, W, batch)
    assert st[0] == 0
    row = res["dst"][res["src"] == 5].tolist()
    # nearest pair is {1, 2} (|y| = 1), then {0, 3} (|y| = 3)
    expect = sorted([1, 2, 0, 3][:k_max]) if k_max != 1 else [1]
    assert row == expect
    ref = O.run_event({k: batch[k] for k in ("x", "y", "z", "plane")}, w, W)
    assert ref["dst"][ref["src"] == 5].tolist() == expect


@pytest.mark.parametrize("tracks", [1100, 400])
def test_window_larger_than_lds_and_long_lists(tracks):
    """A wide radius puts more than 256 candidates inside r of most sources
    (longer than a wave's list: the k_max cut scans the candidates again).
    1,100 tracks on 10 planes: windows of ~2,200 hits, read from HBM; 400
    tracks: windows of ~800 hits, staged in LDS."""
    w = synth.C1.with_(tracks=("fixed", tracks), radius=0.3, k_max=16)
    W = synth.xavier_weights(w)
    batch = synth.generate_batch(w, 1)
    assert batch["hit_off"][-1] < 16384
    p, b, st, res = run(w, W, batch)
    assert st[0] == 0
    etx = _etx()
    etx.etx_set_option(p.ctx, etx.ETX_OPT_RADIUS_LDS, 0)
    p.run(b)
    r2 = p.results(b)
    for k in ("src", "dst", "score", "labels"):
        assert np.array_equal(r2[k], res[k]), k
    oracle_batch_check(w, W, batch, res)


def test_capacity_overflow_reports_required_edges():
    w = synth.C1
    W = synth.xavier_weights(w)
    batch = synth.generate_batch(w, 1)
    _, _, st_ok, res = run(w, W, batch)
    need = int(res["edge_off"][-1])
    p, b, st, _ = run(w, W, batch, cap=need - 1, check=False)
    assert st[0] == _etx().ETX_ERR_CAPACITY and st[1] == need
    p, b, st, res2 = run(w, W, batch, cap=need)
    assert st[0] == 0 and np.array_equal(res2["src"], res["src"])


@pytest.mark.parametrize("bad", ["nan_x", "inf_z", "plane_high", "plane_negative", "hit_off_order", "hit_off_total"])
def test_invalid_input_sets_status(bad):
    etx = _etx()
    w = synth.C1
    W = synth.xavier_weights(w)
    batch = synth.generate_batch(w, 2)
    batch = {k: v.copy() for k, v in batch.items()}
    if bad == "nan_x":
        batch["x"][5] = np.nan
    elif bad == "inf_z":
        batch["z"][7] = np.inf
    elif bad == "plane_high":
        batch["plane"][3] = w.n_planes
    elif bad == "plane_negative":
        batch["plane"][3] = -1
    elif bad == "hit_off_order":
        batch["hit_off"][1] = batch["hit_off"][2] + 1
        batch["hit_off"][2] = batch["hit_off"][1] - 5
    elif bad == "hit_off_total":
        batch["hit_off"][-1] -= 1
    # the host total stays the real hit count: the device check must catch the mismatch
    b = etx.to_device(batch)
    b.n_hits = len(batch["x"])
    p = etx.Pipeline(w, W)
    p.run(b)
    torch.cuda.synchronize()
    assert p.status.cpu().numpy()[0] == etx.ETX_ERR_INPUT


def test_event_size_limit():
    etx = _etx()
    w = synth.C1
    W = synth.xavier_weights(w)
    rng = np.random.default_rng(0)
    for n, want in ((etx.ETX_MAX_EVENT_HITS, etx.ETX_OK), (etx.ETX_MAX_EVENT_HITS + 1, etx.ETX_ERR_UNSUPPORTED)):
        ev = dict(x=rng.uniform(-30, 30, n), y=rng.uniform(-30, 30, n), z=np.zeros(n),
                  plane=rng.integers(0, w.n_planes, n))
        ev["z"] = np.asarray(w.z_planes)[ev["plane"]]
        p, b, st, _ = run(w, W, pack([ev]), check=False)
        assert st[0] == want


def test_host_argument_errors():
    etx = _etx()
    w = synth.C1
    W = synth.xavier_weights(w)
    cfg = etx.make_config(w)
    blob = etx.pack_weights(w, W)
    with pytest.raises(etx.EtxError) as e:
        etx.etx_create(cfg, blob[:-4])
    assert e.value.code == etx.ETX_ERR_WEIGHTS
    p = etx.Pipeline(w, W)
    batch = synth.generate_batch(w, 1)
    b = etx.to_device(batch)
    out = p.allocate(b)
    with pytest.raises(etx.EtxError) as e:
        etx.etx_run(p.ctx, p.hits_struct(b), out, p.ws_ptr, p.ws_bytes - 256, 0)
    assert e.value.code == etx.ETX_ERR_INVALID_ARG
    with pytest.raises(etx.EtxError) as e:
        etx.etx_run(p.ctx, p.hits_struct(b), out, p.ws_ptr + 4, p.ws_bytes, 0)
    assert e.value.code == etx.ETX_ERR_INVALID_ARG


def test_checkpoint_round_trip():
    """etx_save / etx_load carry weights, FP8 scales, prefilter state and band,
    triplet classifiers and launch options: the loaded context computes the
    same bits, and saves the same checkpoint."""
    etx = _etx()
    w = synth.C1
    W = synth.xavier_weights(w)
    cal = etx.to_device(synth.generate_batch(w, 3, seed_space=1001))
    batch = synth.generate_batch(w, 1)
    p = etx.Pipeline(w, W, precision=etx.ETX_FP8_E4M3)
    p.calibrate(cal)
    rng = np.random.default_rng(5)
    state = rng.normal(0, 0.1, 3 * etx.ETX_PF_NPARAM).astype(np.float32)
    etx.etx_prefilter_state(p.ctx, state)
    etx.etx_set_option(p.ctx, etx.ETX_OPT_EDGE_PIPELINE, 2)
    etx.etx_prefilter_band(p.ctx, 0.25, 0.75)
    heads = synth.xavier_triplets(w, seed=3)
    p.set_triplets(heads)
    b = etx.to_device(batch)
    p.run(b)
    r0 = p.results(b)
    blob = etx.etx_save(p.ctx)
    q = etx.Pipeline(w, W, precision=etx.ETX_FP8_E4M3)
    etx.etx_destroy(q.ctx)
    q.ctx = etx.etx_load(blob)
    assert etx.etx_get_option(q.ctx, etx.ETX_OPT_EDGE_PIPELINE) == 2
    assert np.array_equal(etx.etx_prefilter_state(q.ctx), state)
    assert np.array_equal(etx.etx_get_scales(q.ctx), etx.etx_get_scales(p.ctx))
    assert np.array_equal(etx.etx_triplet_get(q.ctx, etx.ETX_TRIPLET_NPARAM(w.gnn_hidden)), etx.pack_triplets(heads))
    q.run(b)
    r1 = q.results(b)
    for k in ("src", "dst", "score", "labels", "edge_off"):
        assert np.array_equal(r0[k], r1[k]), k
    assert etx.etx_save(q.ctx) == blob
