"""In-library training against the FP64 oracle's losses and gradients (which
are pinned on the CPU by torch autograd and central differences), and a
training run's behaviour.

Gradients are compared parameter by parameter.  The GPU runs the same network
in FP32, so every parameter's gradient may differ from the FP64 one by the
FP32 rounding of its forward and backward (relative 1e-4 of the value, plus
1e-6 of the largest gradient for parameters whose terms cancel), and by the
oracle's own change under input perturbations at the FP32 rounding level
(two draws, times four), which covers terms that switch at a ReLU or hinge
kink."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_07423_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _mods():
    from paper_2508_07423_amd import etx
    from paper_2508_07423_amd import train as T
    return etx, T


def _bound(go, spread):
    return 1e-4 * np.abs(go) + 1e-6 * np.abs(go).max() + 4 * spread


def _gnn_param_offset(w):
    return sum(K * M + M for K, M in synth.layer_shapes(w)["emb"])


@pytest.fixture(scope="module")
def c1_event():
    w = synth.C1
    batch = synth.generate_batch(w, 1)
    return w, batch


def test_gnn_step_gradient_matches_oracle(c1_event):
    etx, T = _mods()
    w, batch = c1_event
    W = synth.xavier_weights(w)
    tr = T.Trainer(w, W)
    truth = T.truth_arrays(batch, w, np.random.default_rng(0))
    ts, keep = T.truth_to_device(truth)
    b = etx.to_device(batch)
    loss = tr.gnn_step(b, ts, 0.25, 2.0, 0.0, 1)
    g = tr.gradient(b)
    E = int(tr.iview(b, etx.ETX_VIEW_ROW_PTR, torch.int64)[-1].item())
    src = tr.src[:E].cpu().numpy()
    dst = tr.dst[:E].cpu().numpy()
    ev = synth.event_slice(batch, 0)
    ref = O.run_event(ev, w, W, with_margins=True)
    assert np.array_equal(src, ref["src"]) and np.array_equal(dst, ref["dst"])
    lab = (truth["succ"][src] == dst).astype(np.uint8)
    glab = tr.train_view(b, 2, torch.uint8)[:E].cpu().numpy()
    assert np.array_equal(glab, lab) and 0 < lab.sum() < len(lab)
    _, cart = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    lo, go = O.gnn_focal_loss_grad(cart, src, dst, W, w.gnn_hidden, w.gnn_steps, lab, 0.25, 2.0)
    rng = np.random.default_rng(3)
    spread = np.zeros_like(go)
    for _ in range(2):
        cp = cart * (1 + 2.0 ** -23 * rng.standard_normal(cart.shape))
        spread = np.maximum(spread, np.abs(O.gnn_focal_loss_grad(cp, src, dst, W, w.gnn_hidden, w.gnn_steps, lab,
                                                                 0.25, 2.0)[1] - go))
    o = _gnn_param_offset(w)
    gg = g[o:o + len(go)]
    err = np.abs(gg - go)
    tol = _bound(go, spread)
    bad = err > tol
    print(f"network gradient: {len(go)} parameters, max |gpu - oracle| {err.max():.2e} (max |g| "
          f"{np.abs(go).max():.2e}), max relative {np.max(err / (np.abs(go) + 1e-30)):.2e}, outside the bound "
          f"{bad.sum()}; loss gpu {float(loss.item()):.7f} oracle {lo:.7f}")
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo)
    assert not bad.any(), (np.nonzero(bad)[0][:8], err[bad][:8], tol[bad][:8])
    # an optimiser step moves the network's parameters only
    p0 = tr.params()
    tr.gnn_step(b, ts, 0.25, 2.0, 1e-3, 1)
    p1 = tr.params()
    moved, clear = p1[o:] != p0[o:], np.abs(gg) > 1e-6 * np.abs(gg).max()
    assert np.array_equal(p1[:o], p0[:o]) and not np.any(moved & (gg == 0)) and np.all(moved[clear])
    tr.close()


def _oracle_embedding_pairs(w, ev, W, truth, r_train, a):
    cyl, _ = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    emb = O.embed(cyl, W["emb"])
    r32 = float(np.float32(r_train))
    src, dst = O.radius_graph(ev["plane"], emb, r32, w.k_max, w.plane_window)
    rm, kg = O.radius_margins(ev["plane"], emb, r32, w.k_max, w.plane_window)
    succ = truth["succ"][a:a + len(cyl)] - a
    succ[truth["succ"][a:a + len(cyl)] < 0] = -1
    q = truth["query"][a:a + len(cyl)].astype(bool)
    part = truth["particle"][a:a + len(cyl)]
    rnd = truth["rnd"][a:a + len(cyl)]
    rnd = np.where(rnd >= 0, rnd - a, -1)
    qi = np.nonzero(q & (succ >= 0))[0]
    gen = (qi, succ[qi])
    fm = q[src] & (part[dst] >= 0) & (dst != succ[src])
    rq = np.nonzero(q & (rnd >= 0) & (rnd != succ))[0]
    fake = (np.concatenate([src[fm], rq]), np.concatenate([dst[fm], rnd[rq]]))
    return cyl, emb, src, dst, rm, kg, gen, fake


def _embedding_abs_terms(cyl, layers, gen, fake, margin, w_gen):
    """FP64 dense forward/backward of the embedding (no rounding) for the
    magnitude of every gradient's terms: S_p = sum over hits of |x_k dz_m| (|dz_m|
    for a bias), the scale of its FP32 accumulation error."""
    a = [np.asarray(cyl, np.float64)]
    zs = []
    for i, (W, b) in enumerate(layers):
        z = a[-1] @ W + b
        zs.append(z)
        a.append(np.maximum(z, 0) if i + 1 < len(layers) else z)
    e = a[-1]
    de = np.zeros_like(e)
    gs, gd = gen
    cg = 2 * w_gen / max(len(gs), 1)
    np.add.at(de, gs, cg * (e[gs] - e[gd]))
    np.add.at(de, gd, -cg * (e[gs] - e[gd]))
    fs, fd = fake
    act = ((e[fs] - e[fd]) ** 2).sum(1) < margin
    cf = -2.0 / max(len(fs), 1)
    np.add.at(de, fs[act], cf * (e[fs[act]] - e[fd[act]]))
    np.add.at(de, fd[act], -cf * (e[fs[act]] - e[fd[act]]))
    S = []
    dz = de
    for i in range(len(layers) - 1, -1, -1):
        W = layers[i][0]
        S.append(np.concatenate([(np.abs(a[i]).T @ np.abs(dz)).ravel(), np.abs(dz).sum(0)]))
        if i > 0:
            dz = (dz @ W.T) * (zs[i - 1] > 0)
    return np.concatenate(S[::-1])


def test_embedding_step_gradient_matches_oracle(c1_event):
    etx, T = _mods()
    w, batch = c1_event
    W = synth.xavier_weights(w)
    tr = T.Trainer(w, W)
    truth = T.truth_arrays(batch, w, np.random.default_rng(1))
    ts, keep = T.truth_to_device(truth)
    b = etx.to_device(batch)
    margin = w.radius ** 2 / 0.9
    r_train = float(np.sqrt(1.5 * margin))
    loss = tr.embed_step(b, ts, margin, 3.0, r_train, 0.0, 1)
    g = tr.gradient(b)
    E = int(tr.iview(b, etx.ETX_VIEW_ROW_PTR, torch.int64)[-1].item())
    gsrc, gdst = tr.src[:E].cpu().numpy(), tr.dst[:E].cpu().numpy()
    ev = synth.event_slice(batch, 0)
    cyl, emb, src, dst, rm, kg, gen, fake = _oracle_embedding_pairs(w, ev, W, truth, r_train, 0)
    # the training graph: decidable rows equal the oracle's exactly
    dec = (rm > 1e-6) & (kg > 1e-6)
    assert dec.mean() > 0.99
    n = len(cyl)
    gr = np.split(gdst, np.searchsorted(gsrc, np.arange(1, n)))
    orr = np.split(dst, np.searchsorted(src, np.arange(1, n)))
    for i in np.nonzero(dec)[0]:
        assert np.array_equal(gr[i], orr[i]), i
    if not dec.all():
        pytest.skip("a training-graph row lies within 1e-6 of the radius or the k boundary")
    L64 = [(Wl.astype(np.float64), bl.astype(np.float64)) for Wl, bl in W["emb"]]
    lo, go = O.embed_hinge_loss_grad(cyl, L64, gen, fake, margin, 3.0)
    # fake pairs within FP32 rounding of the hinge's kink (d^2 = m) may be active on one side only: the GPU's
    # gradient must then match the oracle's with any subset of those pairs switched
    d2f = ((emb[fake[0]] - emb[fake[1]]) ** 2).sum(1)
    near = np.nonzero(np.abs(margin - d2f) <= 1e-6)[0]
    assert len(near) <= 4
    none = (np.zeros(0, np.int32), np.zeros(0, np.int32))
    flips = []
    for i in near:
        one = (fake[0][i:i + 1], fake[1][i:i + 1])
        gi = O.embed_hinge_loss_grad(cyl, L64, none, one, d2f[i] + 1.0, 3.0)[1] / len(fake[0])
        flips.append(-gi if d2f[i] < margin else gi)
    rng = np.random.default_rng(4)
    spread = np.zeros_like(go)
    for _ in range(2):
        cp = cyl * (1 + 2.0 ** -23 * rng.standard_normal(cyl.shape))
        spread = np.maximum(spread, np.abs(O.embed_hinge_loss_grad(cp, L64, gen, fake, margin, 3.0)[1] - go))
    gg = g[:len(go)]
    # FP32 accumulation of the sums over hits (their terms cancel exactly in the last layer's bias: a pair's
    # terms at its two hits are opposite), relative FP32 error of the value, and the input-perturbation spread
    S = _embedding_abs_terms(cyl, L64, gen, fake, margin, 3.0)
    tol = 1e-4 * np.abs(go) + 16 * np.log2(len(cyl)) * 2.0 ** -24 * S + 4 * spread
    best = None
    for mask in range(1 << len(flips)):
        ref = go + sum((f for j, f in enumerate(flips) if mask >> j & 1), np.zeros_like(go))
        err = np.abs(gg - ref)
        if best is None or (err > tol).sum() < (best[1] > tol).sum():
            best = (mask, err)
    mask, err = best
    bad = err > tol
    print(f"embedding gradient: {len(go)} parameters, {len(gen[0])} genuine / {len(fake[0])} fake pairs "
          f"({len(near)} at the kink, switched {bin(mask).count('1')}), max |gpu - oracle| {err.max():.2e} "
          f"(max |g| {np.abs(go).max():.2e}), outside the bound {bad.sum()}; "
          f"loss gpu {float(loss.item()):.7f} oracle {lo:.7f}")
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo)
    assert not bad.any(), (np.nonzero(bad)[0][:8], err[bad][:8], tol[bad][:8])
    # an optimiser step moves the embedding's parameters only
    p0 = tr.params()
    tr.embed_step(b, ts, margin, 3.0, r_train, 1e-3, 1)
    p1 = tr.params()
    moved = p1[:len(go)] != p0[:len(go)]
    clear = np.abs(gg) > 1e-6 * np.abs(gg).max()
    assert np.array_equal(p1[len(go):], p0[len(go):]) and not np.any(moved & (gg == 0)) and np.all(moved[clear])
    tr.close()


def test_training_is_reproducible_and_learns():
    """Two runs from the same start give the same bits; a few hundred steps on
    a handful of events lower both losses."""
    etx, T = _mods()
    w = synth.C3
    evs = [synth.generate_batch(w, 1, first=i, seed_space=2100) for i in range(4)]

    def run(steps_emb, steps_gnn):
        tr = T.Trainer(w, synth.xavier_weights(w, 5))
        rng = np.random.default_rng(0)
        dev = [(etx.to_device(e), T.truth_to_device(T.truth_arrays(e, w, rng))) for e in evs]
        margin = w.radius ** 2 / 0.9
        r_train = float(np.sqrt(1.5 * margin))
        le, lg = [], []
        for s in range(steps_emb):
            b, (ts, _) = dev[s % len(dev)]
            le.append(float(tr.embed_step(b, ts, margin, 3.0, r_train, 3e-3, s + 1).item()))
        tr.apply()
        for s in range(steps_gnn):
            b, (ts, _) = dev[s % len(dev)]
            lg.append(float(tr.gnn_step(b, ts, 0.25, 2.0, 2e-3, s + 1).item()))
        p = tr.params()
        tr.close()
        return p, le, lg

    p1, le, lg = run(80, 80)
    p2, _, _ = run(80, 80)
    assert np.array_equal(p1, p2)
    print(f"embedding loss {np.mean(le[:8]):.4f} -> {np.mean(le[-8:]):.4f}; network loss {np.mean(lg[:8]):.4f} -> "
          f"{np.mean(lg[-8:]):.4f}")
    assert np.mean(le[-8:]) < 0.7 * np.mean(le[:8])
    assert np.mean(lg[-8:]) < 0.7 * np.mean(lg[:8])


def test_gpu_training_reaches_the_trained_weights_efficiency():
    """The whole recipe on the GPU (200 generator events of the training seed
    space, 6 embedding and 6 network epochs from Xavier weights): track
    efficiency on 200 events of the uneven-batch workload at least that of the
    committed trained weights, less 0.5 %."""
    etx, T = _mods()
    from paper_2508_07423_amd import evaluate
    w = synth.C3
    r = T.train(w, n_events=200, epochs_emb=6, epochs_gnn=6, log=print)
    batch = synth.generate_batch(w, 200)
    effs = {}
    for name, W in (("gpu-trained", r["weights"]), ("committed", synth.trained_weights(w))):
        p = etx.Pipeline(w, W)
        b = etx.to_device(batch)
        p.run(b)
        res = p.results(b)
        p.close()
        m = evaluate.batch_metrics(res["labels"], batch)
        effs[name] = m["efficiency"]
        print(f"{name}: efficiency {m['efficiency']:.4f}, ghost rate {m['ghost_rate']:.4f}, "
              f"{len(res['src']) / len(batch['x']):.2f} edges per hit")
    print(f"training took {r['seconds']:.1f} s; losses {r['history']}")
    assert effs["gpu-trained"] >= effs["committed"] - 0.005
