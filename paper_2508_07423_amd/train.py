"""In-library training of the embedding MLP and the interaction network (host
orchestration only; every numerical step runs in the library's kernels).

The training set follows thesis ch. 8 "Hit Embedding and Rough Graph
Construction": each step is one event (or a small batch of events); queries
are hits of particles with hits on at least three planes; genuine pairs are
successive hits of a particle along the beam; fake pairs are the hard
negatives (the radius graph of the current embedding at a training radius)
that are not genuine, plus one random pair per query on the next two planes.
The embedding minimises L_fake + w_gen L_gen (eqs. loss1-loss3, margin m); the
network then minimises the mean sigmoid focal loss of its edge scores on the
rough graph of the trained embedding (eq. gnn-loss without the triplet term).

The random pairs are drawn here, from a seeded generator, and handed to the
library as data.
"""
from __future__ import annotations

import os
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import etx, synth


def truth_arrays(batch: Dict[str, np.ndarray], w, rng: np.random.Generator) -> Dict[str, np.ndarray]:
    """Generator truth of a packed batch in the library's etx_truth form (global
    hit indices): successor / predecessor along each particle (in z), query
    flags, one random partner per query on the next two planes (a hit of a
    particle), and the random pairs grouped by partner."""
    n = len(batch["x"])
    ho = batch["hit_off"]
    particle = batch["particle"].astype(np.int32)
    plane = batch["plane"]
    z = batch["z"]
    succ = np.full(n, -1, np.int32)
    pred = np.full(n, -1, np.int32)
    query = np.zeros(n, np.uint8)
    rnd = np.full(n, -1, np.int32)
    for e in range(len(ho) - 1):
        a, b = int(ho[e]), int(ho[e + 1])
        p = particle[a:b]
        real = np.nonzero(p >= 0)[0]
        if len(real) == 0:
            continue
        order = real[np.lexsort((z[a:b][real], p[real]))]
        same = p[order[1:]] == p[order[:-1]]
        later = plane[a:b][order[1:]] > plane[a:b][order[:-1]]
        link = same & later
        s_from, s_to = order[:-1][link] + a, order[1:][link] + a
        succ[s_from] = s_to
        pred[s_to] = s_from
        # queries: particles with hits on at least three planes
        pids = np.unique(p[real])
        for pid in pids:
            idx = real[p[real] == pid]
            if len(np.unique(plane[a:b][idx])) >= 3:
                query[idx + a] = 1
        # one random partner per query among the particle hits on the next two planes
        pl = plane[a:b]
        for q in np.nonzero(query[a:b])[0]:
            cand = real[(pl[real] > pl[q]) & (pl[real] <= pl[q] + w.plane_window)]
            if len(cand):
                rnd[a + q] = a + int(rng.choice(cand))
    has = rnd >= 0
    qs = np.nonzero(has)[0].astype(np.int32)
    order = np.lexsort((qs, rnd[qs]))
    rnd_src = qs[order]
    counts = np.bincount(rnd[qs], minlength=n)
    rnd_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    # hits two particles share (conversion pairs): the second particle's successor of each such hit
    particle2 = batch.get("particle2", np.full(n, -1, np.int32)).astype(np.int32)
    succ2 = np.full(n, -1, np.int32)
    for h in np.nonzero(particle2 >= 0)[0]:
        e = int(np.searchsorted(ho, h, side="right")) - 1
        a, b = int(ho[e]), int(ho[e + 1])
        q = particle2[h]
        chain = np.nonzero((particle[a:b] == q) | (particle2[a:b] == q))[0] + a
        chain = chain[np.argsort(z[chain], kind="stable")]
        k = int(np.nonzero(chain == h)[0][0])
        if k + 1 < len(chain) and plane[chain[k + 1]] > plane[h]:
            succ2[h] = chain[k + 1]
    return dict(particle=particle, succ=succ, pred=pred, query=query, rnd=rnd, rnd_ptr=rnd_ptr,
                rnd_src=rnd_src.astype(np.int32), particle2=particle2, succ2=succ2)


def truth_to_device(t: Dict[str, np.ndarray], device="cuda"):
    import torch
    d = {k: torch.as_tensor(np.ascontiguousarray(v)).to(device) for k, v in t.items()}
    if d["rnd_src"].numel() == 0:
        d["rnd_src"] = torch.zeros(1, dtype=torch.int32, device=device)
    s = etx.etx_truth(d["particle"].data_ptr(), d["succ"].data_ptr(), d["pred"].data_ptr(), d["query"].data_ptr(),
                      d["rnd"].data_ptr(), d["rnd_ptr"].data_ptr(), d["rnd_src"].data_ptr(),
                      d["particle2"].data_ptr() if "particle2" in d else None,
                      d["succ2"].data_ptr() if "succ2" in d else None)
    return s, d


class Trainer(etx.Pipeline):
    """A context whose weights train on the device; outputs and the training
    workspace are torch-allocated per batch shape."""

    def __init__(self, w, weights: Dict, device: int = 0):
        super().__init__(w, weights, device=device)
        etx.etx_train_begin(self.ctx)
        self.n_params = sum(W.size + b.size for v in weights.values() for W, b in v)
        self._tshape = None

    def allocate_train(self, b: "etx.Batch"):
        import torch
        out = self.allocate(b)
        shape = (b.n_events, b.n_hits, self.cap)
        if self._tshape != shape:
            nbytes = etx.etx_train_workspace_size(self.ctx, b.n_events, b.n_hits, self.cap)
            self.tws = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device("cuda", self.device))
            self.tws_ptr = (self.tws.data_ptr() + 255) & ~255
            self.tws_bytes = nbytes
            self._tshape = shape
            if not hasattr(self, "_loss"):
                self._loss = torch.zeros(1, dtype=torch.float32, device=torch.device("cuda", self.device))
        return out

    def embed_step(self, b, truth, margin: float, w_gen: float, r_train: float, lr: float, step: int, stream=None):
        import torch
        out = self.allocate_train(b)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        etx._check(etx.lib().etx_train_embed_step(self.ctx, etx.C.byref(self.hits_struct(b)), etx.C.byref(out),
                                                   etx.C.byref(truth), margin, w_gen, r_train, lr, step,
                                                   etx.C.c_void_p(self._loss.data_ptr()),
                                                   etx.C.c_void_p(self.tws_ptr), self.tws_bytes,
                                                   etx.C.c_void_p(s.cuda_stream)), "etx_train_embed_step")
        return self._loss

    def gnn_step(self, b, truth, alpha: float, gamma: float, lr: float, step: int, stream=None):
        import torch
        out = self.allocate_train(b)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        etx._check(etx.lib().etx_train_gnn_step(self.ctx, etx.C.byref(self.hits_struct(b)), etx.C.byref(out),
                                                 etx.C.byref(truth), alpha, gamma, lr, step,
                                                 etx.C.c_void_p(self._loss.data_ptr()),
                                                 etx.C.c_void_p(self.tws_ptr), self.tws_bytes,
                                                 etx.C.c_void_p(s.cuda_stream)), "etx_train_gnn_step")
        return self._loss

    def triplet_step(self, b, truth, alpha: float, gamma: float, lr: float, step: int, stream=None):
        """One network step with the triplet term of eq. gnn-loss; returns the device float[3] losses (edges,
        articulations, elbows).  The triplet buffers grow when a step needs more."""
        import torch
        out = self.allocate_train(b)
        if not hasattr(self, "_tcap"):
            self._tcap = 4 * b.n_hits + 1024
        if not hasattr(self, "_loss3"):
            self._loss3 = torch.zeros(3, dtype=torch.float32, device=torch.device("cuda", self.device))
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        for _ in range(4):
            need = etx.etx_train_triplet_workspace_size(self.ctx, b.n_events, b.n_hits, self.cap, self._tcap)
            if self.tws_bytes < need:
                self.tws = None
                self.tws = torch.empty(need + 256, dtype=torch.uint8, device=torch.device("cuda", self.device))
                self.tws_ptr = (self.tws.data_ptr() + 255) & ~255
                self.tws_bytes = need
            needed = etx.C.c_int64(0)
            code = etx.lib().etx_train_triplet_step(self.ctx, etx.C.byref(self.hits_struct(b)), etx.C.byref(out),
                                                    etx.C.byref(truth), alpha, gamma, lr, step, self._tcap,
                                                    etx.C.byref(needed), etx.C.c_void_p(self._loss3.data_ptr()),
                                                    etx.C.c_void_p(self.tws_ptr), self.tws_bytes,
                                                    etx.C.c_void_p(s.cuda_stream))
            if code != etx.ETX_ERR_CAPACITY:
                etx._check(code, "etx_train_triplet_step")
                return self._loss3
            self._tcap = int(needed.value * 1.25) + 1024
        raise etx.EtxError(etx.ETX_ERR_CAPACITY, "etx_train_triplet_step")

    def triplet_view(self, b, which: int, dtype):
        off, nbytes = etx.etx_train_triplet_view(self.ctx, b.n_events, b.n_hits, self.cap, self._tcap, which)
        base = self.tws_ptr - self.tws.data_ptr()
        return self.tws[base + off: base + off + nbytes].view(dtype)

    def triplet_heads(self) -> Dict:
        H = self.w.gnn_hidden
        p = etx.etx_train_triplet_params(self.ctx, n=etx.ETX_TRIPLET_NPARAM(H))
        return etx.unpack_triplets(p, H)

    def iview(self, b, which: int, dtype):
        """An inference buffer (etx_workspace_view) of the training workspace."""
        off, nbytes = etx.etx_workspace_view(self.ctx, b.n_events, b.n_hits, self.cap, which)
        base = self.tws_ptr - self.tws.data_ptr()
        return self.tws[base + off: base + off + nbytes].view(dtype)

    def train_view(self, b, which: int, dtype):
        off, nbytes = etx.etx_train_view(self.ctx, b.n_events, b.n_hits, self.cap, which)
        base = self.tws_ptr - self.tws.data_ptr()
        return self.tws[base + off: base + off + nbytes].view(dtype)

    def gradient(self, b) -> np.ndarray:
        import torch
        torch.cuda.synchronize(self.device)
        return self.train_view(b, 0, torch.float32).cpu().numpy().astype(np.float64)

    def params(self) -> np.ndarray:
        return etx.etx_train_params(self.ctx, n=self.n_params)

    def weights(self) -> Dict:
        """The training parameters in the layout of synth.xavier_weights."""
        p = self.params()
        out, o = {}, 0
        for net, shapes in weight_order(self.w):
            out[net] = []
            for K, M in shapes:
                W = p[o:o + K * M].reshape(K, M).copy()
                o += K * M
                bb = p[o:o + M].copy()
                o += M
                out[net].append((W, bb))
        return out

    def apply(self):
        etx.etx_train_apply(self.ctx)


def weight_order(w):
    shapes = synth.layer_shapes(w)
    order = ["emb", "node_enc", "edge_enc"]
    for k in range(w.gnn_steps):
        order += [f"node{k}", f"edge{k}"]
    order.append("cls")
    return [(k, shapes[k]) for k in order]


def train(w, n_events: int = 200, epochs_emb: int = 6, epochs_gnn: int = 6, lr_emb: float = 3e-3,
          lr_gnn: float = 2e-3, w_gen: float = 3.0, seed: int = 5, seed_space: Optional[int] = None,
          log: Callable[[str], None] = print, device: int = 0) -> Dict:
    """Train both phases on the GPU, one event per step: the embedding (hinge
    loss; margin m = r^2 / 0.9, the thesis's ratio of graph radius to margin
    scaled to the workload's radius; hard negatives at d^2 < 1.5 m), then the
    network on the rough graph of the trained embedding (focal loss, alpha
    0.25, gamma 2).  Starts from Xavier weights drawn with `seed`."""
    import torch
    ss = 2000 + w.cid if seed_space is None else seed_space
    init = synth.xavier_weights(w, seed)
    tr = Trainer(w, init, device=device)
    rng = np.random.default_rng(seed)
    events = [synth.generate_batch(w, 1, first=i, seed_space=ss) for i in range(n_events)]
    truths = [truth_arrays(ev, w, rng) for ev in events]
    dev = [(etx.to_device(ev, f"cuda:{device}"), truth_to_device(t, f"cuda:{device}")) for ev, t in zip(events, truths)]
    margin = w.radius ** 2 / 0.9
    r_train = float(np.sqrt(1.5 * margin))
    t0 = time.time()
    step = 0
    history = {"emb": [], "gnn": []}
    for ep in range(epochs_emb):
        tot = 0.0
        for b, (ts, _) in dev:
            step += 1
            tot += float(tr.embed_step(b, ts, margin, w_gen, r_train, lr_emb, step).item())
        history["emb"].append(tot / len(dev))
        log(f"[train] embedding epoch {ep} loss {tot / len(dev):.5f} ({time.time() - t0:.1f} s)")
    tr.apply()                        # the network trains on the rough graph of the trained embedding
    step = 0
    for ep in range(epochs_gnn):
        tot = 0.0
        for b, (ts, _) in dev:
            step += 1
            tot += float(tr.gnn_step(b, ts, 0.25, 2.0, lr_gnn, step).item())
        history["gnn"].append(tot / len(dev))
        log(f"[train] network epoch {ep} loss {tot / len(dev):.5f} ({time.time() - t0:.1f} s)")
    weights = tr.weights()
    tr.close()
    torch.cuda.synchronize()
    return dict(weights=weights, history=history, seconds=time.time() - t0)


def train_triplets(w, weights: Dict, n_events: int = 200, epochs: int = 6, lr: float = 1e-3, seed: int = 5,
                   heads: Optional[Dict] = None, seed_space: Optional[int] = None,
                   log: Callable[[str], None] = print, device: int = 0) -> Dict:
    """The triplet term of eq. gnn-loss on the GPU: starting from a trained
    embedding and network (``weights``) and Xavier triplet classifiers, train
    the network and both classifiers on L_edges + L_art + L_elb, one event per
    step, on generator events of ``w`` (with conversion pairs when
    w.pair_fraction > 0).  Returns the network weights, the classifiers and
    the loss history."""
    import torch
    ss = 3000 + w.cid if seed_space is None else seed_space
    tr = Trainer(w, weights, device=device)
    tr.set_triplets(synth.xavier_triplets(w, seed) if heads is None else heads)
    etx.etx_train_begin(tr.ctx)
    rng = np.random.default_rng(seed)
    events = [synth.generate_batch(w, 1, first=i, seed_space=ss) for i in range(n_events)]
    dev = [(etx.to_device(ev, f"cuda:{device}"), truth_to_device(truth_arrays(ev, w, rng), f"cuda:{device}"))
           for ev in events]
    t0 = time.time()
    step = 0
    history = []
    for ep in range(epochs):
        tot = np.zeros(3)
        for b, (ts, _) in dev:
            step += 1
            tot += tr.triplet_step(b, ts, 0.25, 2.0, lr, step).cpu().numpy()
        history.append((tot / len(dev)).tolist())
        log(f"[train] triplet epoch {ep} losses edges {tot[0] / len(dev):.5f} articulations {tot[1] / len(dev):.5f} "
            f"elbows {tot[2] / len(dev):.5f} ({time.time() - t0:.1f} s)")
    out = dict(weights=tr.weights(), heads=tr.triplet_heads(), history=history, seconds=time.time() - t0)
    tr.close()
    torch.cuda.synchronize()
    return out


def save(weights: Dict, path: str) -> None:
    flat = {}
    for k, v in weights.items():
        for i, (W, b) in enumerate(v):
            flat[f"{k}.{i}.W"] = np.asarray(W, np.float32)
            flat[f"{k}.{i}.b"] = np.asarray(b, np.float32)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **flat)
    os.replace(tmp, path)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="train the embedding and the interaction network on the GPU")
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--events", type=int, default=200)
    ap.add_argument("--epochs-emb", type=int, default=6)
    ap.add_argument("--epochs-gnn", type=int, default=6)
    ap.add_argument("--out", required=True)
    ap.add_argument("--triplets", action="store_true",
                    help="train the triplet term from the workload's trained weights; --out receives the network, "
                         "--out-triplets the classifiers")
    ap.add_argument("--epochs-tri", type=int, default=6)
    ap.add_argument("--out-triplets")
    a = ap.parse_args()
    wl = synth.WORKLOADS[a.workload]
    if a.triplets:
        r = train_triplets(wl, synth.trained_weights(wl), a.events, a.epochs_tri, log=lambda s: print(s, flush=True))
        save(r["weights"], a.out)
        save(r["heads"], a.out_triplets)
    else:
        r = train(wl, a.events, a.epochs_emb, a.epochs_gnn, log=lambda s: print(s, flush=True))
        save(r["weights"], a.out)
    print(a.out, f"{r['seconds']:.1f} s")
