"""Offline tool: trained weights for the efficiency workloads.

Random Xavier weights make the interaction network keep either almost no
edge or almost every edge, so track efficiency (and the labels of the learned
prefilter) are meaningless with them.  This tool trains the same
architectures on generator events of a disjoint seed space, with the
thesis's losses, using PyTorch autograd on the CPU:

  embedding  pairwise hinge loss (ch. 8, eqs. loss1-3): L = L_fake +
             w_genuine L_genuine, L_genuine = mean d^2 over genuine pairs,
             L_fake = mean max(0, m - d^2) over fake pairs; the training set
             merges hard negatives (k-NN in the current embedding on planes
             p+1, p+2 under a training radius), one random pair per query and
             all genuine pairs; queries are hits of particles with >= 3 hits
  GNN        sigmoid focal loss on the edge scores of the rough graph
             (ch. 8, eq. gnn-loss without the triplet term)

Genuine edges are successive hits of one particle along the beam (appendix,
true-edge definition).  The weights are written as .npz (float32) with the
layout of synth.xavier_weights and read back with synth.load_weights.  The
margin follows the thesis's ratio of graph radius to margin (d^2_max = 0.9 m),
scaled to the workload's radius.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from typing import Dict, List, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2508_07423_amd import synth  # noqa: E402


def _torch():
    import torch
    return torch


def true_edges(plane: np.ndarray, particle: np.ndarray, z: np.ndarray) -> set:
    out = set()
    for p in np.unique(particle[particle >= 0]):
        idx = np.nonzero(particle == p)[0]
        idx = idx[np.argsort(z[idx], kind="stable")]
        for a, b in zip(idx[:-1], idx[1:]):
            if plane[b] > plane[a]:
                out.add((int(a), int(b)))
    return out


class Nets:
    def __init__(self, w, seed):
        torch = _torch()
        init = synth.xavier_weights(w, seed)
        self.p = {k: [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in v]
                  for k, v in init.items()}
        self.w = w

    def params(self, nets):
        return [t for k in nets for Wb in self.p[k] for t in Wb]

    def export(self) -> Dict:
        return {k: [(W.detach().numpy().astype(np.float32), b.detach().numpy().astype(np.float32)) for W, b in v]
                for k, v in self.p.items()}


def features(ev, w):
    torch = _torch()
    x = torch.tensor(ev["x"], dtype=torch.float32)
    y = torch.tensor(ev["y"], dtype=torch.float32)
    z = torch.tensor(ev["z"], dtype=torch.float32)
    cyl = torch.stack([torch.hypot(x, y) / w.r_scale, torch.atan2(y, x) / np.pi, z / w.z_scale], 1)
    cart = torch.stack([x / w.r_scale, y / w.r_scale, z / w.z_scale], 1)
    return cyl, cart


def embed(nets, cyl):
    torch = _torch()
    h = cyl
    L = nets.p["emb"]
    for i, (W, b) in enumerate(L):
        h = h @ W + b
        if i + 1 < len(L):
            h = torch.relu(h)
    return h


def knn_pairs(emb, plane, r2, k, window=2):
    """Edges i -> j (1 <= plane_j - plane_i <= window, d^2 < r2, k nearest)."""
    torch = _torch()
    with torch.no_grad():
        src, dst = [], []
        pl = torch.as_tensor(plane)
        P = int(pl.max().item()) + 1 if len(pl) else 0
        for p in range(P):
            s = torch.nonzero(pl == p)[:, 0]
            t = torch.nonzero((pl > p) & (pl <= p + window))[:, 0]
            if len(s) == 0 or len(t) == 0:
                continue
            d2 = torch.cdist(emb[s], emb[t]) ** 2
            d2 = torch.where(d2 < r2, d2, torch.full_like(d2, float("inf")))
            kk = min(k, len(t))
            val, idx = torch.topk(d2, kk, dim=1, largest=False)
            ok = torch.isfinite(val)
            rows = s[:, None].expand(-1, kk)[ok]
            cols = t[idx][ok]
            src.append(rows)
            dst.append(cols)
        if not src:
            return torch.zeros(0, dtype=torch.long), torch.zeros(0, dtype=torch.long)
        return torch.cat(src), torch.cat(dst)


def train_embedding(nets, events, w, epochs, lr, w_genuine=3.0, log=print, on_epoch=None):
    torch = _torch()
    opt = torch.optim.Adam(nets.params(["emb"]), lr=lr)
    margin = w.radius ** 2 / 0.9
    r2_train = 1.5 * margin
    rng = np.random.default_rng(0)
    for ep in range(epochs):
        tot = 0.0
        for ev in events:
            keep = ev["particle"] >= 0
            cyl, _ = features(ev, w)
            te = ev["true"]
            emb = embed(nets, cyl)
            # queries: hits of particles with >= 3 hits (noise excluded)
            part = ev["particle"]
            pids, cnt = np.unique(part[keep], return_counts=True)
            good = set(pids[cnt >= 3].tolist())
            q_ok = np.array([p in good for p in part])
            gs = np.array([a for a, b in te if q_ok[a]], dtype=np.int64)
            gd = np.array([b for a, b in te if q_ok[a]], dtype=np.int64)
            hs, hd = knn_pairs(emb.detach(), ev["plane"], r2_train, 50)
            hs, hd = hs.numpy(), hd.numpy()
            m = q_ok[hs] & (part[hs] >= 0) & (part[hd] >= 0)
            hs, hd = hs[m], hd[m]
            # one random pair per query on the next two planes
            qs = np.nonzero(q_ok)[0]
            rs, rd = [], []
            for q in qs:
                cand = np.nonzero((ev["plane"] > ev["plane"][q]) & (ev["plane"] <= ev["plane"][q] + 2) & (part >= 0))[0]
                if len(cand):
                    rs.append(q)
                    rd.append(int(rng.choice(cand)))
            fs = np.concatenate([hs, np.array(rs, np.int64)])
            fd = np.concatenate([hd, np.array(rd, np.int64)])
            tset = set(zip(gs.tolist(), gd.tolist()))
            fm = np.array([(a, b) not in tset for a, b in zip(fs.tolist(), fd.tolist())], dtype=bool)
            fs, fd = fs[fm], fd[fm]
            d2g = ((emb[gs] - emb[gd]) ** 2).sum(1)
            d2f = ((emb[fs] - emb[fd]) ** 2).sum(1)
            loss = torch.relu(margin - d2f).mean() + w_genuine * d2g.mean()
            opt.zero_grad()
            loss.backward()
            opt.step()
            tot += float(loss)
        log(f"[emb] epoch {ep} loss {tot / len(events):.5f}")
        if on_epoch is not None:
            on_epoch("emb", ep)


def block(x, Wb):
    torch = _torch()
    W, b = Wb
    return torch.relu(torch.nn.functional.layer_norm(x @ W + b, (W.shape[1],), eps=1e-5))


def gnn_forward(nets, cart, src, dst):
    torch = _torch()
    P = nets.p
    S = nets.w.gnn_steps
    h = block(block(cart, P["node_enc"][0]), P["node_enc"][1])
    e = block(block(torch.cat([h[src], h[dst]], 1), P["edge_enc"][0]), P["edge_enc"][1])
    n = cart.shape[0]
    for k in range(S):
        mo = torch.zeros(n, e.shape[1]).index_add_(0, src, e)
        mi = torch.zeros(n, e.shape[1]).index_add_(0, dst, e)
        h = h + block(block(torch.cat([h, mo, mi], 1), P[f"node{k}"][0]), P[f"node{k}"][1])
        e = e + block(block(torch.cat([e, h[src], h[dst]], 1), P[f"edge{k}"][0]), P[f"edge{k}"][1])
    c = block(e, P["cls"][0])
    W, b = P["cls"][1]
    return (c @ W + b)[:, 0]


def focal_loss(logit, y, alpha=0.25, gamma=2.0):
    torch = _torch()
    p = torch.sigmoid(logit)
    ce = torch.nn.functional.binary_cross_entropy_with_logits(logit, y, reduction="none")
    pt = p * y + (1 - p) * (1 - y)
    a = alpha * y + (1 - alpha) * (1 - y)
    return (a * (1 - pt) ** gamma * ce).mean()


def train_gnn(nets, events, w, epochs, lr, log=print, on_epoch=None):
    torch = _torch()
    names = ["node_enc", "edge_enc", "cls"] + [f"node{k}" for k in range(w.gnn_steps)] + \
            [f"edge{k}" for k in range(w.gnn_steps)]
    opt = torch.optim.Adam(nets.params(names), lr=lr)
    for ep in range(epochs):
        tot, acc = 0.0, 0.0
        for ev in events:
            cyl, cart = features(ev, w)
            with torch.no_grad():
                emb = embed(nets, cyl)
            src, dst = knn_pairs(emb, ev["plane"], w.radius ** 2, w.k_max)
            if len(src) == 0:
                continue
            te = ev["true"]
            y = torch.tensor([float((a, b) in te) for a, b in zip(src.tolist(), dst.tolist())])
            logit = gnn_forward(nets, cart, src, dst)
            loss = focal_loss(logit, y)
            opt.zero_grad()
            loss.backward()
            opt.step()
            tot += float(loss)
            acc += float(((logit > 0).float() == y).float().mean())
        log(f"[gnn] epoch {ep} loss {tot / len(events):.5f} edge accuracy {acc / len(events):.4f}")
        if on_epoch is not None:
            on_epoch("gnn", ep)


def train(w, n_events: int, epochs_emb: int, epochs_gnn: int, seed: int = 5, threads: int = 8, log=print,
          init: Dict = None, checkpoint: str = None) -> Dict:
    """Train both phases; ``init`` starts from a saved weight set (with
    ``epochs_emb=0`` it resumes at the GNN phase), ``checkpoint`` is rewritten
    after every epoch so an interrupted run leaves its latest weights."""
    torch = _torch()
    torch.manual_seed(seed)
    torch.set_num_threads(threads)
    evs = []
    for i in range(n_events):
        ev = synth.generate_event(w, i, seed_space=2000 + w.cid)
        ev["true"] = true_edges(ev["plane"], ev["particle"], ev["z"])
        evs.append(ev)
    nets = Nets(w, seed)
    if init is not None:
        nets.p = {k: [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in v]
                  for k, v in init.items()}

    def on_epoch(phase, ep):
        if checkpoint is not None:
            save(nets.export(), checkpoint)
            log(f"[{phase}] checkpoint after epoch {ep}: {checkpoint}")

    t0 = time.time()
    train_embedding(nets, evs, w, epochs_emb, 3e-3, log=log, on_epoch=on_epoch)
    log(f"[emb] {time.time() - t0:.0f} s")
    train_gnn(nets, evs, w, epochs_gnn, 2e-3, log=log, on_epoch=on_epoch)
    log(f"[gnn] {time.time() - t0:.0f} s")
    return nets.export()


def save(weights: Dict, path: str) -> None:
    flat = {}
    for k, v in weights.items():
        for i, (W, b) in enumerate(v):
            flat[f"{k}.{i}.W"] = W
            flat[f"{k}.{i}.b"] = b
    tmp = path + ".tmp.npz"
    np.savez(tmp, **flat)
    os.replace(tmp, path)      # an interrupted run never leaves a torn file


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--events", type=int, default=200)
    ap.add_argument("--epochs-emb", type=int, default=6)
    ap.add_argument("--epochs-gnn", type=int, default=6)
    ap.add_argument("--out", default=None)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--resume", default=None, help="start from this saved weight set")
    a = ap.parse_args()
    w = synth.WORKLOADS[a.workload]
    out = a.out or os.path.join(HERE, "weights", f"{w.name}_trained.npz")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    init = synth.load_weights(a.resume) if a.resume else None
    W = train(w, a.events, a.epochs_emb, a.epochs_gnn, threads=a.threads, log=lambda s: print(s, flush=True),
              init=init, checkpoint=out)
    save(W, out)
    print(out)
