"""Track-finding metrics (thesis ch. 7 "Track reconstruction", LHCb Run-3
conventions) from per-hit component labels and generator truth.

A track is a component with at least three hits (thesis ch. 8, minimum track
length).  A particle is reconstructible when it left hits on at least three
distinct planes.  A track is matched to a particle when at least 70 % of its
hits come from that particle (noise hits count in the denominator); an
unmatched track is a ghost (fake).  Efficiency = reconstructed reconstructible
particles / reconstructible particles; ghost rate = fake tracks / tracks;
clone rate = extra tracks matched to an already matched particle / tracks;
hit purity and hit efficiency are averaged over matched tracks.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np


def event_metrics(labels: np.ndarray, particle: np.ndarray, plane: np.ndarray, min_hits: int = 3,
                  match_frac: float = 0.7) -> Dict[str, float]:
    """Counts for one event.  labels: component label per hit (any integers);
    particle: generator particle id per hit (-1 = noise)."""
    labels = np.asarray(labels)
    particle = np.asarray(particle)
    plane = np.asarray(plane)
    # reconstructible particles
    real = particle >= 0
    pids = np.unique(particle[real])
    n_planes_of = {int(p): len(np.unique(plane[particle == p])) for p in pids}
    n_hits_of = {int(p): int((particle == p).sum()) for p in pids}
    reco_able = {p for p, k in n_planes_of.items() if k >= min_hits}
    # tracks
    uniq, inv, counts = np.unique(labels, return_inverse=True, return_counts=True)
    n_tracks = n_fake = n_clone = 0
    matched_particles = set()
    purity, hit_eff = [], []
    for t in np.nonzero(counts >= min_hits)[0]:
        members = particle[inv == t]
        n_tracks += 1
        ids, c = np.unique(members[members >= 0], return_counts=True)
        if len(ids) == 0:
            n_fake += 1
            continue
        best = int(np.argmax(c))
        pid, nbest = int(ids[best]), int(c[best])
        if nbest < match_frac * len(members):
            n_fake += 1
            continue
        if pid in matched_particles:
            n_clone += 1
        matched_particles.add(pid)
        purity.append(nbest / len(members))
        hit_eff.append(nbest / n_hits_of[pid])
    n_reco = len(matched_particles & reco_able)
    return dict(reconstructible=len(reco_able), reconstructed=n_reco, tracks=n_tracks, fake=n_fake, clone=n_clone,
                purity_sum=float(np.sum(purity)), hit_eff_sum=float(np.sum(hit_eff)), matched=len(purity))


def batch_metrics(labels: np.ndarray, batch: Dict[str, np.ndarray], events: Sequence[int] = None) -> Dict[str, float]:
    """Aggregate metrics over the events of a packed batch (labels may be
    global indices; only the partition matters)."""
    ho = batch["hit_off"]
    idx = range(len(ho) - 1) if events is None else events
    tot = dict(reconstructible=0, reconstructed=0, tracks=0, fake=0, clone=0, purity_sum=0.0, hit_eff_sum=0.0,
               matched=0)
    for i in idx:
        a, b = int(ho[i]), int(ho[i + 1])
        m = event_metrics(labels[a:b], batch["particle"][a:b], batch["plane"][a:b])
        for k in tot:
            tot[k] += m[k]
    return dict(efficiency=tot["reconstructed"] / max(tot["reconstructible"], 1),
                ghost_rate=tot["fake"] / max(tot["tracks"], 1),
                clone_rate=tot["clone"] / max(tot["tracks"], 1),
                hit_purity=tot["purity_sum"] / max(tot["matched"], 1),
                hit_efficiency=tot["hit_eff_sum"] / max(tot["matched"], 1),
                tracks=tot["tracks"], reconstructible=tot["reconstructible"])
