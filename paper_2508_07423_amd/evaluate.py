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


def batch_metrics(labels: np.ndarray, batch: Dict[str, np.ndarray], events: Sequence[int] = None,
                  min_hits: int = 3, match_frac: float = 0.7) -> Dict[str, float]:
    """Aggregate metrics over the events of a packed batch (labels may be
    global indices or any int32 values; only the partition inside an event
    matters).  The same definitions as ``event_metrics``, evaluated for every
    event at once with sorted keys (event, label) and (event, particle)."""
    ho = np.asarray(batch["hit_off"], np.int64)
    n_ev = len(ho) - 1
    idx = np.arange(n_ev) if events is None else np.asarray(list(events), np.int64)
    cnt = ho[idx + 1] - ho[idx]
    hit = np.concatenate([np.arange(ho[i], ho[i + 1]) for i in idx]) if events is not None else np.arange(ho[-1])
    ev = np.repeat(np.arange(len(idx), dtype=np.int64), cnt)
    lab = np.asarray(labels)[hit].astype(np.int64)
    part = np.asarray(batch["particle"])[hit].astype(np.int64)
    pl = np.asarray(batch["plane"])[hit].astype(np.int64)
    # particles: dense ids over (event, particle); reconstructible on >= min_hits distinct planes
    real = part >= 0
    pkey = (ev << 32) | (part & 0xFFFFFFFF)
    pu, pinv, pcount = np.unique(pkey[real], return_inverse=True, return_counts=True)
    pdense = np.full(len(part), -1, np.int64)
    pdense[real] = pinv
    planes_of = np.bincount(np.unique(pinv * 64 + pl[real]) // 64, minlength=len(pu))
    reco_able = planes_of >= min_hits
    # tracks: components of >= min_hits hits
    lkey = (ev << 32) | ((lab + (1 << 31)) & 0xFFFFFFFF)
    lu, linv, lcount = np.unique(lkey, return_inverse=True, return_counts=True)
    is_track = lcount >= min_hits
    n_tracks = int(is_track.sum())
    # per track, the particle with the most hits (ties: the smallest particle id)
    sel = real & is_track[linv]
    pair = linv[sel] * max(len(pu), 1) + pdense[sel]
    pairs, pc = np.unique(pair, return_counts=True)
    ptrack, ppart = pairs // max(len(pu), 1), pairs % max(len(pu), 1)
    order = np.lexsort((ppart, -pc, ptrack))
    first = np.ones(len(order), bool)
    first[1:] = ptrack[order][1:] != ptrack[order][:-1]
    best = order[first]
    bt, bp, bn = ptrack[best], ppart[best], pc[best]
    members = lcount[bt]
    ok = ~(bn < match_frac * members)
    bt, bp, bn, members = bt[ok], bp[ok], bn[ok], members[ok]
    matched_ids = np.unique(bp)
    n_matched = len(bt)
    n_fake = n_tracks - n_matched
    n_clone = n_matched - len(matched_ids)
    n_reco = int(reco_able[matched_ids].sum())
    purity_sum = float(np.sum(bn / members))
    hit_eff_sum = float(np.sum(bn / pcount[bp]))
    return dict(efficiency=n_reco / max(int(reco_able.sum()), 1),
                ghost_rate=n_fake / max(n_tracks, 1),
                clone_rate=n_clone / max(n_tracks, 1),
                hit_purity=purity_sum / max(n_matched, 1),
                hit_efficiency=hit_eff_sum / max(n_matched, 1),
                tracks=n_tracks, reconstructible=int(reco_able.sum()))


def tracks_from_labels(labels: np.ndarray, batch: Dict[str, np.ndarray]):
    """Component labels as a track list: (tracks, event_track_off), each track
    the ascending global hit indices of one label of one event."""
    ho = np.asarray(batch["hit_off"], np.int64)
    lab = np.asarray(labels, np.int64)
    ev = np.repeat(np.arange(len(ho) - 1), np.diff(ho))
    order = np.lexsort((np.arange(len(lab)), lab, ev))
    key = (ev[order] << 32) | (lab[order] & 0xFFFFFFFF)
    cut = np.nonzero(np.diff(key))[0] + 1
    groups = np.split(order, cut) if len(order) else []
    tev = ev[order][np.r_[0, cut]] if len(order) else np.zeros(0, np.int64)
    eto = np.searchsorted(tev, np.arange(len(ho)), side="left").astype(np.int64)
    return [np.sort(g) for g in groups], eto


def track_list_metrics(tracks, event_track_off, batch: Dict[str, np.ndarray], min_hits: int = 3,
                       match_frac: float = 0.7) -> Dict[str, float]:
    """The metrics of ``batch_metrics`` for a list of tracks that may share
    hits (the triplet stage's output), with hits that two particles share
    (``particle2``) counted for both.  Also the efficiency over the particles
    that share hits with another (pair_efficiency)."""
    ho = np.asarray(batch["hit_off"], np.int64)
    part = np.asarray(batch["particle"], np.int64)
    part2 = np.asarray(batch.get("particle2", np.full(len(part), -1)), np.int64)
    plane = np.asarray(batch["plane"], np.int64)
    ev = np.repeat(np.arange(len(ho) - 1, dtype=np.int64), np.diff(ho))
    # memberships (hit, particle key)
    mh = np.r_[np.nonzero(part >= 0)[0], np.nonzero(part2 >= 0)[0]]
    mp = np.r_[part[part >= 0], part2[part2 >= 0]]
    mkey = (ev[mh] << 32) | mp
    pu, pinv = np.unique(mkey, return_inverse=True)
    pcount = np.bincount(pinv, minlength=len(pu))
    planes_of = np.bincount(np.unique(pinv * 64 + plane[mh]) // 64, minlength=len(pu))
    reco_able = planes_of >= min_hits
    shared_p = np.zeros(len(pu), bool)
    sh = np.nonzero(part2 >= 0)[0]
    if len(sh):
        shared_p[np.searchsorted(pu, (ev[sh] << 32) | part[sh])] = True
        shared_p[np.searchsorted(pu, (ev[sh] << 32) | part2[sh])] = True
    # tracks of >= min_hits hits
    lens = np.array([len(t) for t in tracks], np.int64)
    is_track = lens >= min_hits
    n_tracks = int(is_track.sum())
    hits = np.concatenate([t for t in tracks]) if len(tracks) else np.zeros(0, np.int64)
    tid = np.repeat(np.arange(len(tracks), dtype=np.int64), lens)
    # (track, particle) pairs through every membership of every hit
    first = np.full(len(part), -1, np.int64)
    second = np.full(len(part), -1, np.int64)
    m1 = part >= 0
    first[m1] = np.searchsorted(pu, (ev[m1] << 32) | part[m1])
    m2 = part2 >= 0
    second[m2] = np.searchsorted(pu, (ev[m2] << 32) | part2[m2])
    pt = np.r_[tid, tid]
    pp = np.r_[first[hits], second[hits]]
    ok = (pp >= 0) & is_track[pt]
    npu = max(len(pu), 1)
    pairs, pc = np.unique(pt[ok] * npu + pp[ok], return_counts=True)
    ptrack, ppart = pairs // npu, pairs % npu
    order = np.lexsort((ppart, -pc, ptrack))
    head = np.ones(len(order), bool)
    head[1:] = ptrack[order][1:] != ptrack[order][:-1]
    best = order[head]
    bt, bp, bn = ptrack[best], ppart[best], pc[best]
    good = ~(bn < match_frac * lens[bt])
    bt, bp, bn = bt[good], bp[good], bn[good]
    matched = np.unique(bp)
    n_matched = len(bt)
    n_fake = n_tracks - n_matched
    reco = np.zeros(len(pu), bool)
    reco[matched] = True
    ra = reco_able & shared_p
    return dict(efficiency=float((reco & reco_able).sum() / max(int(reco_able.sum()), 1)),
                pair_efficiency=float((reco & ra).sum() / max(int(ra.sum()), 1)),
                ghost_rate=n_fake / max(n_tracks, 1),
                clone_rate=(n_matched - len(matched)) / max(n_tracks, 1),
                hit_purity=float(np.sum(bn / lens[bt]) / max(n_matched, 1)),
                tracks=n_tracks, reconstructible=int(reco_able.sum()), pair_reconstructible=int(ra.sum()))
