"""Pins of the oracle's training losses and gradients (CPU only).

The embedding's pairwise hinge loss (thesis ch. 8, eqs. loss1-loss3) and the
edge classifier's sigmoid focal loss (eq. gnn-loss, Lin et al.) with their
gradients through the embedding MLP and the whole interaction network are
checked against routes that share nothing with the oracle's code:
  - torch float64 autograd through the dense incidence-matrix formulation of
    the network (the oracle hand-writes every backward step);
  - central finite differences of the oracle's own loss (the gradient is the
    derivative of the value it returns);
  - special cases with closed forms: gamma = 0 makes the focal loss torch's
    class-weighted binary cross-entropy; a genuine pair's hinge term is the
    squared distance, a fake pair beyond the margin contributes nothing.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import oracle as O
from paper_2508_07423_amd import synth
from tests.test_oracle_pins import _random_gnn_weights


def _emb_layers(seed, dims=(3, 16, 16, 4)):
    rng = np.random.default_rng(seed)
    return [(rng.normal(0, 0.6, (a, b)), rng.normal(0, 0.2, b)) for a, b in zip(dims[:-1], dims[1:])]


def _torch_emb(cyl, layers):
    ps = []
    t = torch.tensor(cyl, dtype=torch.float64)
    for i, (W, b) in enumerate(layers):
        Wt = torch.tensor(W, dtype=torch.float64, requires_grad=True)
        bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
        ps += [Wt, bt]
        t = t @ Wt + bt
        if i + 1 < len(layers):
            t = torch.relu(t)
    return t, ps


def _pairs(n, rng, k):
    s = rng.integers(0, n, k)
    d = rng.integers(0, n, k)
    ok = s != d
    return s[ok].astype(np.int32), d[ok].astype(np.int32)


def test_hinge_gradient_matches_torch_autograd():
    rng = np.random.default_rng(1)
    n = 40
    cyl = rng.normal(0, 1, (n, 3))
    layers = _emb_layers(2)
    gen = _pairs(n, rng, 30)
    fake = _pairs(n, rng, 60)
    margin, w_gen = 2.5, 3.0
    loss, g = O.embed_hinge_loss_grad(cyl, layers, gen, fake, margin, w_gen)
    e, ps = _torch_emb(cyl, layers)
    d2g = ((e[gen[0]] - e[gen[1]]) ** 2).sum(1)
    d2f = ((e[fake[0]] - e[fake[1]]) ** 2).sum(1)
    assert 0 < int((d2f < margin).sum()) < len(d2f)          # both sides of the hinge occur
    lt = torch.relu(margin - d2f).mean() + w_gen * d2g.mean()
    lt.backward()
    gt = np.concatenate([p.grad.numpy().ravel() for p in ps])
    assert abs(loss - float(lt.detach())) <= 1e-12 * abs(loss)
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_hinge_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    n = 25
    cyl = rng.normal(0, 1, (n, 3))
    layers = _emb_layers(4)
    gen = _pairs(n, rng, 15)
    fake = _pairs(n, rng, 30)
    _, g = O.embed_hinge_loss_grad(cyl, layers, gen, fake, 2.0, 2.0)
    flat = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])
    sizes = [(W.shape, b.shape) for W, b in layers]

    def unflat(v):
        out, o = [], 0
        for (ws, bs) in sizes:
            nw, nb = int(np.prod(ws)), int(np.prod(bs))
            out.append((v[o:o + nw].reshape(ws), v[o + nw:o + nw + nb]))
            o += nw + nb
        return out

    h = 1e-6
    for i in rng.choice(len(flat), 40, replace=False):
        vp, vm = flat.copy(), flat.copy()
        vp[i] += h
        vm[i] -= h
        lp, _ = O.embed_hinge_loss_grad(cyl, unflat(vp), gen, fake, 2.0, 2.0)
        lm, _ = O.embed_hinge_loss_grad(cyl, unflat(vm), gen, fake, 2.0, 2.0)
        assert abs((lp - lm) / (2 * h) - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_hinge_special_cases():
    """One genuine pair: the loss is w_gen d^2; a fake pair beyond the margin
    adds nothing (and no gradient); no pairs: zero."""
    layers = [(np.eye(3)[:, :2] * 1.0, np.zeros(2))]       # linear: e = (x, y)
    cyl = np.array([[0.0, 0.0, 5.0], [3.0, 4.0, -1.0], [10.0, 0.0, 0.0]])
    loss, g = O.embed_hinge_loss_grad(cyl, layers, (np.array([0]), np.array([1])), (np.array([0]), np.array([2])),
                                      margin=50.0, w_gen=2.0)
    assert loss == pytest.approx(2.0 * 25.0)
    loss0, g0 = O.embed_hinge_loss_grad(cyl, layers, (np.zeros(0), np.zeros(0)), (np.zeros(0), np.zeros(0)), 1.0, 2.0)
    assert loss0 == 0.0 and not np.any(g0)


def _dense_focal_torch(cart, src, dst, weights, H, S, labels, alpha, gamma):
    """The network in torch float64 with dense incidence matrices, every
    parameter a leaf; focal loss from torch's binary cross-entropy."""
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64)
    n, E = len(cart), len(src)
    Bs = torch.zeros(E, n, dtype=torch.float64); Bs[torch.arange(E), torch.tensor(src, dtype=torch.long)] = 1
    Bd = torch.zeros(E, n, dtype=torch.float64); Bd[torch.arange(E), torch.tensor(dst, dtype=torch.long)] = 1
    leaves = []

    def lin(x, Wb):
        W = T(Wb[0]).requires_grad_(True)
        b = T(Wb[1]).requires_grad_(True)
        leaves.extend([W, b])
        return x @ W + b

    def mlp2(x, layers):
        for Wb in layers:
            x = torch.relu(F.layer_norm(lin(x, Wb), (H,), eps=1e-5))
        return x

    h = mlp2(T(cart), weights["node_enc"])
    e = mlp2(torch.cat([Bs @ h, Bd @ h], 1), weights["edge_enc"])
    for k in range(S):
        mo, mi = Bs.T @ e, Bd.T @ e
        h = h + mlp2(torch.cat([h, mo, mi], 1), weights[f"node{k}"])
        e = e + mlp2(torch.cat([e, Bs @ h, Bd @ h], 1), weights[f"edge{k}"])
    c = torch.relu(F.layer_norm(lin(e, weights["cls"][0]), (H,), eps=1e-5))
    z = lin(c, weights["cls"][1])[:, 0]
    y = T(labels)
    ce = F.binary_cross_entropy_with_logits(z, y, reduction="none")
    p = torch.sigmoid(z)
    pt = p * y + (1 - p) * (1 - y)
    at = alpha * y + (1 - alpha) * (1 - y)
    loss = (at * (1 - pt) ** gamma * ce).mean()
    loss.backward()
    return float(loss.detach()), np.concatenate([t.grad.numpy().ravel() for t in leaves])


def _small_graph(seed, n=14, E=30):
    rng = np.random.default_rng(seed)
    cart = rng.normal(0, 0.5, (n, 3))
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    order = np.lexsort((dst, src))
    return cart, src[order], dst[order], rng.integers(0, 2, len(src)).astype(np.uint8)


@pytest.mark.parametrize("H,S", [(8, 1), (8, 3), (16, 2)])
def test_focal_gradient_matches_torch_autograd(H, S):
    cart, src, dst, lab = _small_graph(H + S)
    W = _random_gnn_weights(H, S, seed=7 + S)
    loss, g = O.gnn_focal_loss_grad(cart, src, dst, W, H, S, lab, 0.25, 2.0)
    lt, gt = _dense_focal_torch(cart, src, dst, W, H, S, lab, 0.25, 2.0)
    assert abs(loss - lt) <= 1e-12 * abs(lt)
    np.testing.assert_allclose(g, gt, rtol=1e-8, atol=1e-14)


def test_focal_gradient_matches_central_differences():
    H, S = 8, 2
    cart, src, dst, lab = _small_graph(5)
    W = _random_gnn_weights(H, S, seed=3)
    _, g = O.gnn_focal_loss_grad(cart, src, dst, W, H, S, lab, 0.25, 2.0)
    blocks = O.gnn_param_blocks(W)
    flat = np.concatenate([np.concatenate([np.ravel(a), np.ravel(b)]) for a, b in blocks]).astype(np.float64)
    keys = []
    for k in ["node_enc", "edge_enc"] + [f"{t}{s}" for s in range(S) for t in ("node", "edge")] + ["cls"]:
        for li in range(len(W[k])):
            keys.append((k, li))

    def with_flat(v):
        out, o = {k: list(x) for k, x in W.items()}, 0
        for k, li in keys:
            Wl, bl = W[k][li]
            nw, nb = Wl.size, bl.size
            out[k][li] = (v[o:o + nw].reshape(Wl.shape), v[o + nw:o + nw + nb])
            o += nw + nb
        return out

    rng = np.random.default_rng(9)
    h = 1e-6
    for i in rng.choice(len(flat), 60, replace=False):
        vp, vm = flat.copy(), flat.copy()
        vp[i] += h
        vm[i] -= h
        lp, _ = O.gnn_focal_loss_grad(cart, src, dst, with_flat(vp), H, S, lab)
        lm, _ = O.gnn_focal_loss_grad(cart, src, dst, with_flat(vm), H, S, lab)
        assert abs((lp - lm) / (2 * h) - g[i]) <= 2e-6 * max(1e-2, abs(g[i])), (i, (lp - lm) / (2 * h), g[i])


def test_focal_with_gamma_zero_is_weighted_bce():
    H, S = 8, 1
    cart, src, dst, lab = _small_graph(11)
    W = _random_gnn_weights(H, S, seed=1)
    loss, _ = O.gnn_focal_loss_grad(cart, src, dst, W, H, S, lab, 0.3, 0.0)
    z = torch.tensor(O.gnn(cart, src, dst, W, H, S))
    y = torch.tensor(lab, dtype=torch.float64)
    ref = F.binary_cross_entropy_with_logits(z, y, weight=0.3 * y + 0.7 * (1 - y))
    assert loss == pytest.approx(float(ref), rel=1e-12)


def test_focal_on_a_generator_event_is_finite_and_matches_oracle_forward():
    """The training forward is the inference network: with gamma = 0 and alpha
    = 1/2 the loss equals half the BCE of the oracle's logits on a real event."""
    w = synth.C1
    W = synth.xavier_weights(w)
    ev = synth.event_slice(synth.generate_batch(w, 1), 0)
    r = O.run_event(ev, w, W)
    _, cart = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    lab = (np.arange(len(r["src"])) % 3 == 0).astype(np.uint8)
    loss, g = O.gnn_focal_loss_grad(cart, r["src"], r["dst"], W, w.gnn_hidden, w.gnn_steps, lab, 0.5, 0.0)
    ref = F.binary_cross_entropy_with_logits(torch.tensor(r["logit"]), torch.tensor(lab, dtype=torch.float64))
    assert loss == pytest.approx(0.5 * float(ref), rel=1e-10)
    assert np.all(np.isfinite(g))


# --------------------------------------------------------------------------
# eq. gnn-loss with its triplet term (two triplet classifiers on [e_S(a), e_S(b)])
# --------------------------------------------------------------------------

def _dense_triplet_torch(cart, src, dst, weights, H, S, labels, ta, tb, kind, tlab, heads, alpha, gamma):
    """The network and both triplet classifiers in torch float64 (dense
    incidence, every parameter a leaf); each loss term a focal loss built from
    torch's binary cross-entropy."""
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64)
    n, E = len(cart), len(src)
    Bs = torch.zeros(E, n, dtype=torch.float64); Bs[torch.arange(E), torch.tensor(src, dtype=torch.long)] = 1
    Bd = torch.zeros(E, n, dtype=torch.float64); Bd[torch.arange(E), torch.tensor(dst, dtype=torch.long)] = 1
    leaves, tleaves = [], []

    def lin(x, Wb, into):
        W = T(Wb[0]).requires_grad_(True)
        b = T(Wb[1]).requires_grad_(True)
        into.extend([W, b])
        return x @ W + b

    def blk(x, Wb, into):
        return torch.relu(F.layer_norm(lin(x, Wb, into), (H,), eps=1e-5))

    def focal(z, y):
        ce = F.binary_cross_entropy_with_logits(z, y, reduction="none")
        p = torch.sigmoid(z)
        pt = p * y + (1 - p) * (1 - y)
        at = alpha * y + (1 - alpha) * (1 - y)
        return (at * (1 - pt) ** gamma * ce).mean()

    h = blk(blk(T(cart), weights["node_enc"][0], leaves), weights["node_enc"][1], leaves)
    e = blk(blk(torch.cat([Bs @ h, Bd @ h], 1), weights["edge_enc"][0], leaves), weights["edge_enc"][1], leaves)
    for k in range(S):
        mo, mi = Bs.T @ e, Bd.T @ e
        x = torch.cat([h, mo, mi], 1)
        h = h + blk(blk(x, weights[f"node{k}"][0], leaves), weights[f"node{k}"][1], leaves)
        x = torch.cat([e, Bs @ h, Bd @ h], 1)
        e = e + blk(blk(x, weights[f"edge{k}"][0], leaves), weights[f"edge{k}"][1], leaves)
    c = blk(e, weights["cls"][0], leaves)
    loss = focal(lin(c, weights["cls"][1], leaves)[:, 0], T(labels))
    ta_t, tb_t = torch.tensor(ta, dtype=torch.long), torch.tensor(tb, dtype=torch.long)
    for name, sel in (("art", kind == 0), ("elb", kind > 0)):
        L = heads[name]
        if not sel.any():
            # keep the leaf layout: unused classifier parameters get zero gradients
            for Wb in L:
                for a in Wb:
                    tleaves.append(T(a).requires_grad_(True))
            continue
        s = torch.tensor(np.nonzero(sel)[0], dtype=torch.long)
        x = torch.cat([e[ta_t[s]], e[tb_t[s]]], 1)
        y = blk(blk(x, L[0], tleaves), L[1], tleaves)
        loss = loss + focal(lin(y, L[2], tleaves)[:, 0], T(tlab)[s])
    loss.backward()
    g = np.concatenate([t.grad.numpy().ravel() for t in leaves])
    tg = np.concatenate([(t.grad.numpy() if t.grad is not None else np.zeros(t.shape)).ravel() for t in tleaves])
    return float(loss.detach()), g, tg


def _triplet_case(seed, H, E=30, n=14, T=40):
    cart, src, dst, lab = _small_graph(seed, n, E)
    rng = np.random.default_rng(seed + 100)
    ta = rng.integers(0, E, T).astype(np.int32)
    tb = rng.integers(0, E, T).astype(np.int32)
    kind = rng.integers(0, 3, T).astype(np.uint8)
    tlab = rng.integers(0, 2, T).astype(np.uint8)
    heads = {h: [(rng.normal(0, 0.4, (a, b)), rng.normal(0, 0.2, b)) for a, b in [(2 * H, H), (H, H), (H, 1)]]
             for h in ("art", "elb")}
    return cart, src, dst, lab, ta, tb, kind, tlab, heads


@pytest.mark.parametrize("H,S", [(8, 1), (8, 2), (16, 2)])
def test_triplet_loss_gradient_matches_torch_autograd(H, S):
    cart, src, dst, lab, ta, tb, kind, tlab, heads = _triplet_case(H + 3 * S, H)
    W = _random_gnn_weights(H, S, seed=5 + S)
    loss, g, tg = O.gnn_triplet_loss_grad(cart, src, dst, W, H, S, lab, ta, tb, kind, tlab, heads, 0.25, 2.0)
    lt, gt, tgt = _dense_triplet_torch(cart, src, dst, W, H, S, lab, ta, tb, kind, tlab, heads, 0.25, 2.0)
    assert abs(loss - lt) <= 1e-12 * abs(lt)
    np.testing.assert_allclose(g, gt, rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(tg, tgt, rtol=1e-8, atol=1e-14)


def test_triplet_loss_with_one_kind_only_and_without_triplets():
    H, S = 8, 1
    cart, src, dst, lab, ta, tb, kind, tlab, heads = _triplet_case(21, H)
    W = _random_gnn_weights(H, S, seed=2)
    art = kind == 0
    loss, g, tg = O.gnn_triplet_loss_grad(cart, src, dst, W, H, S, lab, ta[art], tb[art], kind[art], tlab[art],
                                          heads)
    lt, gt, tgt = _dense_triplet_torch(cart, src, dst, W, H, S, lab, ta[art], tb[art], kind[art], tlab[art], heads,
                                       0.25, 2.0)
    np.testing.assert_allclose(g, gt, rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(tg, tgt, rtol=1e-8, atol=1e-14)
    hs = len(tg) // 2
    assert not np.any(tg[hs:]) and np.any(tg[:hs])           # the elbow classifier sees no triplet
    # no triplets: exactly the edge loss and its gradient
    z = np.zeros(0, np.int32)
    l0, g0, tg0 = O.gnn_triplet_loss_grad(cart, src, dst, W, H, S, lab, z, z, z.astype(np.uint8),
                                          z.astype(np.uint8), heads)
    le, ge = O.gnn_focal_loss_grad(cart, src, dst, W, H, S, lab)
    assert l0 == le and np.array_equal(g0, ge) and not np.any(tg0)


def test_triplet_head_gradient_matches_central_differences():
    H, S = 8, 1
    cart, src, dst, lab, ta, tb, kind, tlab, heads = _triplet_case(33, H)
    W = _random_gnn_weights(H, S, seed=6)
    _, _, tg = O.gnn_triplet_loss_grad(cart, src, dst, W, H, S, lab, ta, tb, kind, tlab, heads)
    flat = O.triplet_params(heads)
    shapes = [(a.shape, b.shape) for h in ("art", "elb") for a, b in heads[h]]

    def unflat(v):
        out, o, L = {"art": [], "elb": []}, 0, []
        for ws, bs in shapes:
            nw, nb = int(np.prod(ws)), int(np.prod(bs))
            L.append((v[o:o + nw].reshape(ws), v[o + nw:o + nw + nb]))
            o += nw + nb
        out["art"], out["elb"] = L[:3], L[3:]
        return out

    rng = np.random.default_rng(4)
    h = 1e-6
    for i in rng.choice(len(flat), 50, replace=False):
        vp, vm = flat.copy(), flat.copy()
        vp[i] += h
        vm[i] -= h
        lp = O.gnn_triplet_loss_grad(cart, src, dst, W, H, S, lab, ta, tb, kind, tlab, unflat(vp))[0]
        lm = O.gnn_triplet_loss_grad(cart, src, dst, W, H, S, lab, ta, tb, kind, tlab, unflat(vm))[0]
        assert abs((lp - lm) / (2 * h) - tg[i]) <= 2e-6 * max(1e-2, abs(tg[i])), (i, (lp - lm) / (2 * h), tg[i])
