"""Tracking metrics (thesis ch. 7 definitions) on hand-built events with known truth."""
import numpy as np
import pytest

from paper_2508_07423_amd import evaluate as E


def test_perfect_reconstruction():
    # particles 0 (4 hits), 1 (3 hits), 2 (2 hits: not reconstructible), noise
    particle = np.array([0, 0, 0, 0, 1, 1, 1, 2, 2, -1])
    plane = np.array([0, 1, 2, 3, 0, 1, 2, 0, 1, 5])
    labels = np.array([0, 0, 0, 0, 4, 4, 4, 7, 7, 9])
    m = E.batch_metrics(labels, dict(particle=particle, plane=plane, hit_off=np.array([0, 10])))
    assert m["efficiency"] == 1.0 and m["ghost_rate"] == 0.0 and m["clone_rate"] == 0.0
    assert m["tracks"] == 2 and m["reconstructible"] == 2
    assert m["hit_purity"] == 1.0 and m["hit_efficiency"] == 1.0


def test_seventy_percent_matching_ghosts_and_clones():
    # particle 0 has 10 hits split into two tracks (clone); particle 1's track has
    # 7 of its hits + 3 foreign hits (70 %: matched); a track of 2+2+1 hits is a ghost
    particle = np.array([0] * 10 + [1] * 7 + [2] * 3 + [3, 3, 4, 4, -1])
    plane = np.concatenate([np.arange(10), np.arange(7), np.arange(3), [0, 1, 2, 3, 4]])
    labels = np.array([0] * 5 + [5] * 5 + [10] * 7 + [10] * 3 + [20] * 5)
    m = E.batch_metrics(labels, dict(particle=particle, plane=plane, hit_off=np.array([0, len(particle)])))
    # reconstructible: 0 (10 planes), 1 (7), 2 (3 planes); 3 and 4 have 2 hits
    assert m["reconstructible"] == 3
    assert m["tracks"] == 4
    assert np.isclose(m["ghost_rate"], 1 / 4)
    assert np.isclose(m["clone_rate"], 1 / 4)
    assert np.isclose(m["efficiency"], 2 / 3)            # particles 0 and 1 found, 2 absorbed into 1's track
    assert np.isclose(m["hit_purity"], (1 + 1 + 0.7) / 3)
    assert np.isclose(m["hit_efficiency"], (0.5 + 0.5 + 1.0) / 3)


def test_short_components_are_not_tracks():
    particle = np.array([0, 0, 0, 1, 1, 1])
    plane = np.array([0, 1, 2, 0, 1, 2])
    labels = np.array([0, 0, 2, 3, 3, 5])                # every component has < 3 hits
    m = E.batch_metrics(labels, dict(particle=particle, plane=plane, hit_off=np.array([0, 6])))
    assert m["tracks"] == 0 and m["efficiency"] == 0.0


def test_batch_metrics_equals_the_per_event_definition():
    """The vectorised batch aggregate equals the sum of the per-event counts of
    ``event_metrics`` (random partitions, particles and noise)."""
    rng = np.random.default_rng(5)
    ho = [0]
    parts, planes, labels = [], [], []
    for ev in range(40):
        n = int(rng.integers(0, 60))
        parts.append(rng.integers(-1, 8, n))
        planes.append(rng.integers(0, 6, n))
        labels.append(ho[-1] + rng.integers(0, max(n // 3, 1), n))   # global-index-like labels
        ho.append(ho[-1] + n)
    batch = dict(particle=np.concatenate(parts), plane=np.concatenate(planes), hit_off=np.array(ho))
    lab = np.concatenate(labels)
    tot = dict(reconstructible=0, reconstructed=0, tracks=0, fake=0, clone=0, purity_sum=0.0, hit_eff_sum=0.0,
               matched=0)
    for i in range(40):
        a, b = ho[i], ho[i + 1]
        m = E.event_metrics(lab[a:b], batch["particle"][a:b], batch["plane"][a:b])
        for k in tot:
            tot[k] += m[k]
    m = E.batch_metrics(lab, batch)
    assert m["reconstructible"] == tot["reconstructible"] and m["tracks"] == tot["tracks"]
    assert np.isclose(m["efficiency"], tot["reconstructed"] / tot["reconstructible"])
    assert np.isclose(m["ghost_rate"], tot["fake"] / tot["tracks"])
    assert np.isclose(m["clone_rate"], tot["clone"] / tot["tracks"])
    assert np.isclose(m["hit_purity"], tot["purity_sum"] / tot["matched"])
    assert np.isclose(m["hit_efficiency"], tot["hit_eff_sum"] / tot["matched"])
    sub = [3, 7, 11]
    ms = E.batch_metrics(lab, batch, events=sub)
    t2 = dict(reconstructible=0, reconstructed=0)
    for i in sub:
        a, b = ho[i], ho[i + 1]
        mm = E.event_metrics(lab[a:b], batch["particle"][a:b], batch["plane"][a:b])
        t2["reconstructible"] += mm["reconstructible"]
        t2["reconstructed"] += mm["reconstructed"]
    assert ms["reconstructible"] == t2["reconstructible"]
    assert np.isclose(ms["efficiency"], t2["reconstructed"] / max(t2["reconstructible"], 1))


def test_track_list_metrics_equal_batch_metrics_without_shared_hits():
    from paper_2508_07423_amd import synth
    w = synth.C3
    batch = synth.generate_batch(w, 6)
    rng = np.random.default_rng(2)
    # a noisy partition: true particles, some merged, some split, noise spread around
    labels = batch["particle"].astype(np.int64).copy()
    noise = labels < 0
    labels[noise] = rng.integers(0, 40, noise.sum())
    labels[rng.uniform(size=len(labels)) < 0.05] = 7
    labels = labels + (np.repeat(np.arange(6), np.diff(batch["hit_off"])) << 20)
    tracks, eto = E.tracks_from_labels(labels, batch)
    m1 = E.track_list_metrics(tracks, eto, batch)
    m0 = E.batch_metrics(labels, batch)
    for k in ("efficiency", "ghost_rate", "clone_rate", "hit_purity", "tracks", "reconstructible"):
        assert m1[k] == pytest.approx(m0[k], abs=1e-12), k


def test_track_list_metrics_count_shared_hits_for_both_particles():
    # particles 0 and 1 share hits 0, 1 (planes 0, 1); 0 continues on 2, 3, particle 1 on 4, 5
    batch = dict(hit_off=np.array([0, 6]), particle=np.array([0, 0, 0, 0, 1, 1]),
                 particle2=np.array([1, 1, -1, -1, -1, -1]), plane=np.array([0, 1, 2, 3, 2, 3]))
    both = [np.array([0, 1, 2, 3]), np.array([0, 1, 4, 5])]
    m = E.track_list_metrics(both, np.array([0, 2]), batch)
    assert m["efficiency"] == 1.0 and m["pair_efficiency"] == 1.0 and m["ghost_rate"] == 0.0
    merged = [np.arange(6)]             # 4 of 6 hits from either particle: below 70 %, a ghost
    m = E.track_list_metrics(merged, np.array([0, 1]), batch)
    assert m["efficiency"] == 0.0 and m["ghost_rate"] == 1.0 and m["tracks"] == 1
