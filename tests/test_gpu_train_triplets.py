"""In-library training with the triplet term of eq. gnn-loss against the FP64
oracle (pinned on the CPU by torch autograd, central differences and its
reduction to the edge loss): the step's triplets are those of its own
purified graph, its triplet labels follow the generator truth, and the
gradients of every network parameter and both triplet classifiers match the
oracle's parameter by parameter, within the bound of the network step's test
(FP32 rounding of forward and backward, plus the oracle's response to FP32
input perturbations)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_07423_amd import synth
from tests.test_gpu_train import _bound, _gnn_param_offset, _mods

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def triplet_labels(ta, tb, kind, src, dst, t):
    """Genuine: one particle through A -> C -> B along its successor chain
    (articulation), or one particle owning all three hits (elbow)."""
    part, part2, succ, succ2 = t["particle"], t["particle2"], t["succ"], t["succ2"]

    def parts(h):
        return {int(p) for p in (part[h], part2[h]) if p >= 0}

    def nxt(h, p):
        return succ[h] if part[h] == p else (succ2[h] if part2[h] == p else -1)

    out = np.zeros(len(ta), np.uint8)
    for i, (a, b, k) in enumerate(zip(ta, tb, kind)):
        if k == 0:
            A, C, B = src[a], dst[a], dst[b]
            out[i] = any(nxt(A, p) == C and nxt(C, p) == B for p in parts(A))
        else:
            C, A, B = (src[a], dst[a], dst[b]) if k == 1 else (dst[a], src[a], src[b])
            out[i] = bool(parts(C) & parts(A) & parts(B))
    return out


def _heads(w, seed):
    rng = np.random.default_rng(seed)
    H = synth.xavier_triplets(w, seed)
    return {h: [(W, rng.normal(0, 0.2, b.shape).astype(np.float32)) for W, b in L] for h, L in H.items()}


def test_triplet_step_gradient_matches_oracle():
    etx, T = _mods()
    w = synth.C6
    batch = synth.generate_batch(w, 1, first=41)
    W = synth.trained_weights(w)
    heads = _heads(w, 3)
    tr = T.Trainer(w, W)
    tr.set_triplets(heads)
    truth = T.truth_arrays(batch, w, np.random.default_rng(0))
    assert (truth["particle2"] >= 0).any()
    ts, _ = T.truth_to_device(truth)
    b = etx.to_device(batch)
    losses = tr.triplet_step(b, ts, 0.25, 2.0, 0.0, 1).cpu().numpy()
    g = tr.gradient(b)
    tg = tr.triplet_view(b, 0, torch.float32).cpu().numpy().astype(np.float64)
    E = int(tr.iview(b, etx.ETX_VIEW_ROW_PTR, torch.int64)[-1].item())
    src, dst = tr.src[:E].cpu().numpy(), tr.dst[:E].cpu().numpy()
    keep = tr.score[:E].cpu().numpy() >= np.float32(w.threshold)
    n = len(batch["x"])
    ao = tr.triplet_view(b, 5, torch.int64).cpu().numpy()
    eo = tr.triplet_view(b, 6, torch.int64).cpu().numpy()
    nt = int(eo[-1])
    ta = tr.triplet_view(b, 2, torch.int32)[:nt].cpu().numpy()
    tb = tr.triplet_view(b, 3, torch.int32)[:nt].cpu().numpy()
    kind = tr.triplet_view(b, 4, torch.uint8)[:nt].cpu().numpy()
    # the step's triplets are those of its own purified graph
    ra, rb, rk = O.triplets(n, src, dst, batch["plane"], keep)
    assert np.array_equal(ta, ra) and np.array_equal(tb, rb) and np.array_equal(kind, rk)
    assert int(ao[-1]) == int((kind == 0).sum())
    # labels from the generator truth (edges: succ or succ2; triplets: the rule above)
    lab = ((truth["succ"][src] == dst) | (truth["succ2"][src] == dst)).astype(np.uint8)
    assert np.array_equal(tr.train_view(b, 2, torch.uint8)[:E].cpu().numpy(), lab)
    tlab = triplet_labels(ta, tb, kind, src, dst, truth)
    assert np.array_equal(tr.triplet_view(b, 1, torch.uint8)[:nt].cpu().numpy(), tlab)
    assert 0 < tlab.sum() < len(tlab)
    # gradients against the oracle
    ev = synth.event_slice(batch, 0)
    _, cart = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    args = (src, dst, W, w.gnn_hidden, w.gnn_steps, lab, ta, tb, kind, tlab, heads, 0.25, 2.0)
    lo, go, tgo = O.gnn_triplet_loss_grad(cart, *args)
    rng = np.random.default_rng(3)
    spread, tspread = np.zeros_like(go), np.zeros_like(tgo)
    for _ in range(2):
        cp = cart * (1 + 2.0 ** -23 * rng.standard_normal(cart.shape))
        _, gp, tgp = O.gnn_triplet_loss_grad(cp, *args)
        spread = np.maximum(spread, np.abs(gp - go))
        tspread = np.maximum(tspread, np.abs(tgp - tgo))
    o = _gnn_param_offset(w)
    gg = g[o:o + len(go)]
    for name, got, ref, sp in (("network", gg, go, spread), ("triplet classifiers", tg, tgo, tspread)):
        err = np.abs(got - ref)
        tol = _bound(ref, sp)
        bad = err > tol
        print(f"{name} gradient: {len(ref)} parameters, max |gpu - oracle| {err.max():.2e} (max |g| "
              f"{np.abs(ref).max():.2e}), outside the bound {bad.sum()}")
        assert not bad.any(), (name, np.nonzero(bad)[0][:8], err[bad][:8], tol[bad][:8])
    print(f"losses gpu {losses} (sum {losses.sum():.7f}) oracle {lo:.7f}; {nt} triplets, {int(tlab.sum())} genuine")
    assert abs(float(losses.sum()) - lo) <= 1e-5 * abs(lo)
    # an optimiser step moves the network and the classifiers, not the embedding
    p0 = tr.params()
    h0 = etx.pack_triplets(tr.triplet_heads())
    tr.triplet_step(b, ts, 0.25, 2.0, 1e-3, 1)
    p1 = tr.params()
    h1 = etx.pack_triplets(tr.triplet_heads())
    assert np.array_equal(p1[:o], p0[:o]) and np.any(p1[o:] != p0[o:]) and np.any(h1 != h0)
    tr.close()


def test_triplet_training_learns_and_separates_shared_starts():
    """A short run of the triplet term on conversion-pair events lowers both
    triplet losses, and the trained classifiers reconstruct more of the
    particles that share their first hits than plain components do."""
    etx, T = _mods()
    from paper_2508_07423_amd import evaluate
    w = synth.C6
    r = T.train_triplets(w, synth.trained_weights(w), n_events=60, epochs=4, log=print)
    h = np.array(r["history"])
    assert h[-1, 1] < 0.7 * h[0, 1] and h[-1, 2] < h[0, 2]
    batch = synth.generate_batch(w, 40)
    p = etx.Pipeline(w, r["weights"])
    p.set_triplets(r["heads"])
    b = etx.to_device(batch)
    p.run_tracks_sized(b)
    res = p.results(b)
    tres = p.track_results(b)
    m_trk = evaluate.track_list_metrics(tres["tracks"], tres["event_track_off"], batch)
    m_lab = evaluate.track_list_metrics(*evaluate.tracks_from_labels(res["labels"], batch), batch)
    print(f"triplet tracks: {m_trk}; components: {m_lab}")
    assert m_trk["pair_efficiency"] > m_lab["pair_efficiency"]
