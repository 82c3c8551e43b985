"""Learned edge prefilter: on-device forward/backward/Adam against the FP64
oracle's hand-written gradient (itself pinned by finite differences and torch
autograd on the CPU), determinism and checkpoint/resume, the pruning decision,
and the unpruned fallback."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_07423_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _etx():
    from paper_2508_07423_amd import etx
    return etx


def pf_params(seed=3):
    layers = synth.xavier_prefilter(seed)
    rng = np.random.default_rng(seed)
    layers = [(W, rng.normal(0, 0.1, b.shape).astype(np.float32)) for W, b in layers]
    flat = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers]).astype(np.float32)
    return layers, flat


def oracle_candidates(w, W, ev):
    cyl, _ = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    emb = O.embed(cyl, W["emb"])
    src, dst = O.radius_graph(ev["plane"], emb, float(np.float32(w.radius)), w.k_max, w.plane_window)
    f = O.prefilter_features(src, dst, ev["x"], ev["y"], ev["z"], emb, w.r_scale, w.z_scale)
    return src, dst, f


@pytest.fixture(scope="module")
def setup():
    etx = _etx()
    w = synth.C1
    W = synth.xavier_weights(w)
    batch = synth.generate_batch(w, 1)
    ev = synth.event_slice(batch, 0)
    src, dst, f = oracle_candidates(w, W, ev)
    rng = np.random.default_rng(7)
    labels = (rng.uniform(0, 1, len(src)) < 0.3).astype(np.uint8)
    layers, flat = pf_params()
    p = etx.Pipeline(w, W)
    b = etx.to_device(batch)
    return etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b


U32 = 2.0 ** -24            # FP32 unit roundoff
# FP32 rounding level of the six features as the GPU forms them: differences of
# FP32 coordinates (and of hypotf / atan2f values) relative to O(1) normalised
# values, and the embedding distance, which carries the FP32 embedding's error
FEAT_EPS = np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-5])


def _dense_terms(f, labels, layers, pos_weight):
    """FP64 dense forward/backward (no rounding) for the magnitudes behind the
    per-parameter bounds: S_p = sum over edges of |per-edge gradient term| and
    M_p, an upper bound of one edge's |term|."""
    (W1, b1), (W2, b2), (W3, b3) = [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in layers]
    E = len(f)
    z1 = f @ W1 + b1
    a1 = np.maximum(z1, 0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0)
    z3 = a2 @ W3[:, 0] + b3[0]
    y = labels.astype(np.float64)
    wt = np.where(labels != 0, pos_weight, 1.0)
    dz = wt * (1 / (1 + np.exp(-z3)) - y) / E
    d2 = (z2 > 0) * (W3[:, 0][None, :] * dz[:, None])
    d1 = (z1 > 0) * (d2 @ W2.T)
    adz, ad2, ad1 = np.abs(dz), np.abs(d2), np.abs(d1)
    S = np.concatenate([(np.abs(f).T @ ad1).ravel(), ad1.sum(0), (np.abs(a1).T @ ad2).ravel(), ad2.sum(0),
                        np.abs(a2).T @ adz, [adz.sum()]])
    M = np.concatenate([np.outer(np.abs(f).max(0), ad1.max(0)).ravel(), ad1.max(0),
                        np.outer(np.abs(a1).max(0), ad2.max(0)).ravel(), ad2.max(0),
                        np.abs(a2).max(0) * adz.max(), [adz.max()]])
    return S, M, a1, d2


def _near_bf16_boundary(v, rel=2.0 ** -20):
    """Count values within `rel` (relative) of a BF16 rounding midpoint: an
    FP32 evaluation can round those to the other neighbouring code."""
    v = np.abs(np.asarray(v, np.float64).ravel())
    v = v[v > 0]
    ulp = np.exp2(np.floor(np.log2(v)) - 7)
    frac = v / ulp - np.floor(v / ulp)
    return int((np.abs(frac - 0.5) * ulp < rel * v).sum())


def test_features_match_oracle(setup):
    """Each of the six features of every candidate edge against the oracle's
    (the difference of the stored phi values wrapped to (-pi, pi]; where the FP64
    difference lies within the features' rounding of +-pi either side of the
    wrap is correct)."""
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    q = etx.Pipeline(w, W, prefilter=1, prefilter_tau=0.0)
    etx.etx_set_option(q.ctx, etx.ETX_OPT_PF_FEATURES, 1)
    etx.etx_prefilter_set(q.ctx, flat)
    q.run(b)
    q.results(b)
    g = q.view(b, etx.ETX_VIEW_PF_FEAT, torch.float32).cpu().numpy().reshape(-1, 8)[:len(src)].astype(np.float64)
    assert np.all(g[:, 6:] == 0)
    d = np.abs(g[:, :6] - f)
    at_wrap = np.abs(np.abs(f[:, 4]) - 1.0) <= FEAT_EPS[4]
    d[at_wrap, 4] = np.minimum(d[at_wrap, 4], np.abs(np.abs(g[at_wrap, 4]) - np.abs(f[at_wrap, 4])))
    for k in range(6):
        assert d[:, k].max() <= FEAT_EPS[k], (k, d[:, k].max())
    print(f"feature max |gpu - oracle|: {d.max(0)}")
    q.close()


def test_probabilities_match_oracle(setup):
    """Every candidate's probability against the oracle's forward pass with the
    same BF16 rounding at the 32 x 32 product.  Bound per edge: the spread of
    the oracle's own probability under input perturbations at the features'
    FP32 rounding level (two draws, times four), plus FP32 accumulation."""
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    q = etx.Pipeline(w, W, prefilter=1, prefilter_tau=0.0)
    etx.etx_prefilter_set(q.ctx, flat)
    q.run(b)
    q.results(b)
    prob = q.view(b, etx.ETX_VIEW_PF_PROB, torch.float32).cpu().numpy()[:len(src)].astype(np.float64)
    L64 = [(Wl.astype(np.float64), bl.astype(np.float64)) for Wl, bl in layers]
    po = O.sigmoid(O.prefilter_forward(f, L64, 1))
    rng = np.random.default_rng(11)
    spread = np.zeros(len(f))
    for _ in range(2):
        fp = f + FEAT_EPS * rng.standard_normal(f.shape)
        spread = np.maximum(spread, np.abs(O.sigmoid(O.prefilter_forward(fp, L64, 1)) - po))
    tol = 4 * spread + 64 * U32
    err = np.abs(prob - po)
    bad = err > tol
    print(f"probabilities: max |gpu - oracle| {err.max():.2e}, above 1e-6: {(err > 1e-6).sum()} of {len(err)}, "
          f"outside the bound: {bad.sum()}")
    assert not bad.any(), (err[bad][:5], tol[bad][:5])
    q.close()


def test_gradient_and_loss_match_oracle(setup):
    """Loss and every parameter's gradient against the oracle's hand-written
    BF16 backward.  Bound per parameter p: FP32 accumulation of the mean over E
    edges (16 log2(E) u32 S_p, S_p the sum of the edges' |terms|), plus one BF16
    step (2^-7 relative of one edge's term, M_p) for each operand of the two
    BF16 products that lies within FP32 rounding of a rounding midpoint (counted
    on the exact intermediates), plus four times the oracle's own change under
    feature perturbations at the FP32 rounding level."""
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    etx.etx_prefilter_set(p.ctx, flat)
    lab = torch.as_tensor(labels).cuda()
    loss = p.prefilter_train_step(b, lab, 1e-3, 2.5, 1)
    torch.cuda.synchronize()
    assert np.array_equal(p.src[:len(src)].cpu().numpy(), src) and np.array_equal(p.dst[:len(dst)].cpu().numpy(), dst)
    g = p.view(b, etx.ETX_VIEW_PF_GRAD, torch.float32).cpu().numpy().astype(np.float64)
    L64 = [(Wl.astype(np.float64), bl.astype(np.float64)) for Wl, bl in layers]
    lo, go = O.prefilter_loss_grad(f, labels, L64, 2.5, qmode=1)
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo) + 1e-7
    assert abs(g[-1] - lo) <= 1e-5 * abs(lo) + 1e-7
    E = len(f)
    S, M, a1, d2 = _dense_terms(f, labels, layers, 2.5)
    n_near = _near_bf16_boundary(a1) + _near_bf16_boundary(d2)
    rng = np.random.default_rng(12)
    spread = np.zeros_like(go)
    for _ in range(2):
        fp = f + FEAT_EPS * rng.standard_normal(f.shape)
        spread = np.maximum(spread, np.abs(O.prefilter_loss_grad(fp, labels, L64, 2.5, qmode=1)[1] - go))
    tol = 16 * np.log2(max(E, 2)) * U32 * S + (n_near + 1) * 2.0 ** -7 * M + 4 * spread
    err = np.abs(g[:-1] - go)
    bad = err > tol
    print(f"gradient: {len(go)} parameters, max |gpu - oracle| {err.max():.2e} (max |g| {np.abs(go).max():.2e}), "
          f"operands near a BF16 midpoint {n_near}, outside the bound: {bad.sum()}")
    assert not bad.any(), (np.nonzero(bad)[0][:5], err[bad][:5], tol[bad][:5])
    # the Adam step moved every parameter with a clear gradient by lr against its sign
    new = etx.etx_prefilter_get(p.ctx).astype(np.float64)
    clear = np.abs(go) > 1e-2 * np.abs(go).max()
    step = new - flat.astype(np.float64)
    np.testing.assert_allclose(step[clear], -1e-3 * np.sign(go[clear]), rtol=1e-3, atol=1e-7)


def test_training_is_deterministic_and_resumable(setup):
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    lab = torch.as_tensor(labels).cuda()

    def train(steps, start=1):
        for t in range(start, start + steps):
            p.prefilter_train_step(b, lab, 1e-2, 2.5, t)
        torch.cuda.synchronize()
        return etx.etx_prefilter_state(p.ctx)

    etx.etx_prefilter_set(p.ctx, flat)
    two = train(2)
    etx.etx_prefilter_set(p.ctx, flat)
    one = train(1)
    ckpt = one.copy()
    etx.etx_prefilter_set(p.ctx, np.zeros_like(flat))      # clobber, then resume from the checkpoint
    etx.etx_prefilter_state(p.ctx, ckpt)
    resumed = train(1, start=2)
    assert np.array_equal(resumed, two)
    etx.etx_prefilter_set(p.ctx, flat)
    assert np.array_equal(train(2), two)


def test_loss_decreases_with_training(setup):
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    # a learnable target: edges with a small transverse step
    target = (np.abs(f[:, 3]) < np.median(np.abs(f[:, 3]))).astype(np.uint8)
    lab = torch.as_tensor(target).cuda()
    etx.etx_prefilter_set(p.ctx, flat)
    losses = [float(p.prefilter_train_step(b, lab, 1e-2, 1.0, t).item()) for t in range(1, 201)]
    assert losses[-1] < 0.7 * losses[0]


def test_pruning_matches_oracle_and_tau_zero_is_the_plain_path(setup):
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    tau = 0.5
    q = etx.Pipeline(w, W, prefilter=1, prefilter_tau=tau)
    etx.etx_prefilter_set(q.ctx, flat)
    q.run(b)
    res = q.results(b)
    keep = q.view(b, etx.ETX_VIEW_PF_KEEP, torch.uint8).cpu().numpy()[:len(src)].astype(bool)
    prob = O.sigmoid(O.prefilter_forward(f, [(Wl.astype(np.float64), bl.astype(np.float64)) for Wl, bl in layers], 1))
    far = np.abs(prob - tau) > 1e-3
    assert np.array_equal(keep[far], prob[far] >= tau)
    assert 0 < keep.sum() < len(keep)
    assert np.array_equal(res["src"], src[keep]) and np.array_equal(res["dst"], dst[keep])
    # the network then sees only the surviving edges
    _, cart = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    s64 = O.sigmoid(O.gnn(cart, res["src"], res["dst"], W, w.gnn_hidden, w.gnn_steps))
    assert np.abs(res["score"] - s64).max() <= 1e-5
    # tau = 0 keeps every candidate: identical to the plain path
    z = etx.Pipeline(w, W, prefilter=1, prefilter_tau=0.0)
    etx.etx_prefilter_set(z.ctx, flat)
    z.run(b)
    rz = z.results(b)
    p.run(b)
    rp = p.results(b)
    for k in ("src", "dst", "score", "labels", "edge_off"):
        assert np.array_equal(rz[k], rp[k]), k


def test_fallback_band_runs_events_unpruned(setup):
    """Events whose kept fraction leaves the validated band run unpruned: their
    edges are the unpruned pipeline's (scores to FP32 rounding: the batch's
    tile boundaries move), the other events' are the pruned run's; the
    fallback flags name exactly the events outside the band."""
    etx, w, W, batch, ev, src, dst, f, labels, layers, flat, p, b = setup
    bat = synth.generate_batch(w.with_(tracks=("fixed", 40)), 6, seed_space=9200)
    bb = etx.to_device(bat)

    def run(tau, band=None, prefilter=1):
        q = etx.Pipeline(w, W, prefilter=prefilter, prefilter_tau=tau)
        etx.etx_prefilter_set(q.ctx, flat)
        if band is not None:
            etx.etx_prefilter_band(q.ctx, *band)
        q.run(bb)
        r = q.results(bb)
        fb = q.view(bb, etx.ETX_VIEW_PF_FALLBACK, torch.int32).cpu().numpy().copy() if prefilter else None
        q.close()
        return r, fb

    unpruned, _ = run(0.0, prefilter=0)
    pruned, fb0 = run(0.5)
    assert not fb0.any()
    frac = np.diff(pruned["edge_off"]) / np.maximum(np.diff(unpruned["edge_off"]), 1)
    s = np.sort(frac)
    lo = 0.5 * (s[2] + s[3])              # three events below the band, three inside
    assert s[2] < lo < s[3]
    got, fb = run(0.5, (float(lo), 1.0))
    assert np.array_equal(fb.astype(bool), frac < lo)
    ho = bat["hit_off"]
    for e in range(6):
        ref = unpruned if fb[e] else pruned
        a0, a1 = got["edge_off"][e], got["edge_off"][e + 1]
        r0, r1 = ref["edge_off"][e], ref["edge_off"][e + 1]
        assert np.array_equal(got["src"][a0:a1], ref["src"][r0:r1]), e
        assert np.array_equal(got["dst"][a0:a1], ref["dst"][r0:r1]), e
        assert np.abs(got["score"][a0:a1].astype(np.float64) - ref["score"][r0:r1]).max(initial=0) <= 1e-5
    with pytest.raises(etx.EtxError):
        etx.etx_prefilter_band(p.ctx, 0.6, 0.5)


@pytest.mark.parametrize("tau", [0.5, 1.5])
def test_pruned_graph_is_the_filtered_candidate_list_across_events(tau):
    """A 30-event batch with an empty event: the pruned graph is exactly the
    candidate list (the plain path's graph) filtered by the keep flags, in
    order, with per-event offsets that follow; with tau above every
    probability nothing is kept and every hit is its own component."""
    etx = _etx()
    w = synth.C3
    W = synth.xavier_weights(w)
    batch = dict(synth.generate_batch(w, 30))
    ho = batch["hit_off"]
    batch["hit_off"] = np.insert(ho, 5, ho[5]).astype(np.int64)
    _, flat = pf_params()
    b = etx.to_device(batch)
    plain = etx.Pipeline(w, W)
    plain.run(b)
    rp = plain.results(b)
    q = etx.Pipeline(w, W, prefilter=1, prefilter_tau=tau)
    etx.etx_prefilter_set(q.ctx, flat)
    q.run(b)
    r = q.results(b)
    keep = q.view(b, etx.ETX_VIEW_PF_KEEP, torch.uint8).cpu().numpy()[:len(rp["src"])].astype(bool)
    assert np.array_equal(r["src"], rp["src"][keep]) and np.array_equal(r["dst"], rp["dst"][keep])
    kept_before = np.concatenate([[0], np.cumsum(keep)])
    assert np.array_equal(r["edge_off"], kept_before[rp["edge_off"]])
    if tau > 1:
        assert len(r["src"]) == 0 and not keep.any()
        assert np.array_equal(r["labels"], np.arange(len(r["labels"])))
    else:
        assert 0 < keep.sum() < len(keep)
