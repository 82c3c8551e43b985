"""Training loop of the learned edge prefilter (host orchestration only).

Every numerical step runs in the library: the full pipeline labels the
candidate edges of a batch (an edge is positive when the unpruned pipeline
keeps it, score >= 0.5), and ``etx_prefilter_train_step`` runs the forward,
backward, gradient reduction and Adam kernels.  The threshold tau is chosen on
a validation batch so that a target fraction of the positive edges survive.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import etx, synth


def labels_from_full_pipeline(pipe: "etx.Pipeline", b: "etx.Batch", threshold: float):
    """Run the unpruned pipeline and return (uint8 device labels per candidate
    edge in the candidate order, number of candidates)."""
    import torch
    etx.etx_prefilter_config(pipe.ctx, 0, 0.0)
    pipe.run(b)
    torch.cuda.synchronize()
    st = pipe.status.cpu().numpy()
    if st[0] != etx.ETX_OK:
        raise etx.EtxError(int(st[0]), "labelling run")
    E = int(pipe.edge_off[-1].item())
    return (pipe.score[:max(E, 1)] >= threshold).to(torch.uint8), E


def train_prefilter(w, weights: Dict, n_events: int, batch_events: int = 20, epochs: int = 1, lr: float = 1e-2,
                    pos_weight: float = 4.0, seed_space: Optional[int] = None, init_seed: int = 7,
                    log: Callable[[str], None] = print, device: int = 0) -> Dict:
    """Train on ``n_events`` generated events (disjoint seed space) in
    minibatches of ``batch_events``; returns params, optimiser state and the
    loss history.  Every step averages over all candidate edges of its events
    (tens of thousands per event), so small event batches (many Adam steps)
    train far better than large ones."""
    import torch
    ss = 5000 + w.cid if seed_space is None else seed_space
    pipe = etx.Pipeline(w, weights, device=device)
    init = synth.xavier_prefilter(init_seed)
    etx.etx_prefilter_set(pipe.ctx, np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in init]))
    n_batches = max(1, n_events // batch_events)
    history: List[float] = []
    step = 0
    t0 = time.time()
    cache = []
    for ep in range(epochs):
        for bi in range(n_batches):
            if ep == 0:
                batch = synth.generate_batch(w, batch_events, first=bi * batch_events, seed_space=ss)
                cache.append(batch)
            b = etx.to_device(cache[bi], f"cuda:{device}")
            labels, E = labels_from_full_pipeline(pipe, b, w.threshold)
            step += 1
            loss = pipe.prefilter_train_step(b, labels, lr, pos_weight, step)
            history.append(float(loss.item()))
            if bi % max(1, n_batches // 5) == 0:
                log(f"[prefilter] epoch {ep} batch {bi}/{n_batches} candidates {E} positives "
                    f"{float(labels.float().mean().item()):.3f} loss {history[-1]:.4f} ({time.time() - t0:.0f} s)")
    state = etx.etx_prefilter_state(pipe.ctx)
    pipe.close()
    return dict(params=state[:etx.ETX_PF_NPARAM].copy(), state=state, history=history, steps=step)


def fallback_band(kept_per_event: np.ndarray, candidates_per_event: np.ndarray, quantile: float = 0.005,
                  margin: float = 0.8) -> tuple:
    """Band of an event's kept fraction inside which the prefilter is trusted:
    from `margin` times the `quantile` of the validation events' kept fractions
    up to 1 (keeping more candidates than validated costs time, never
    efficiency).  Events with no candidates do not count."""
    kept = np.asarray(kept_per_event, np.float64)
    cand = np.asarray(candidates_per_event, np.float64)
    frac = kept[cand > 0] / cand[cand > 0]
    if len(frac) == 0:
        return 0.0, 1.0
    return float(margin * np.quantile(frac, quantile)), 1.0


def choose_tau(w, weights: Dict, params: np.ndarray, batch: Dict, recall: float = 0.995, device: int = 0) -> Dict:
    """Threshold keeping `recall` of the positive edges of a validation batch,
    and the fallback band of the per-event kept fraction at that threshold."""
    import torch
    pipe = etx.Pipeline(w, weights, device=device)
    etx.etx_prefilter_set(pipe.ctx, params)
    b = etx.to_device(batch, f"cuda:{device}")
    labels, E = labels_from_full_pipeline(pipe, b, w.threshold)
    etx.etx_prefilter_config(pipe.ctx, 1, 0.0)      # keep all: the probabilities of every candidate
    pipe.run(b)
    torch.cuda.synchronize()
    prob = pipe.view(b, etx.ETX_VIEW_PF_PROB, torch.float32).cpu().numpy()[:E]
    lab = labels[:E].cpu().numpy().astype(bool)
    pos = np.sort(prob[lab])
    tau = float(pos[int(np.floor((1.0 - recall) * len(pos)))]) if len(pos) else 0.0
    kept = float((prob >= tau).mean()) if E else 1.0
    eo = pipe.edge_off.cpu().numpy()
    cand_ev = np.diff(eo)
    cs = np.concatenate([[0], np.cumsum(prob >= tau)])
    kept_ev = cs[eo[1:]] - cs[eo[:-1]]
    lo, hi = fallback_band(kept_ev, cand_ev)
    pipe.close()
    return dict(tau=tau, kept_fraction=kept, positive_fraction=float(lab.mean()) if E else 0.0,
                positive_recall=float((prob[lab] >= tau).mean()) if lab.any() else 1.0, band=(lo, hi))
