"""The conversion-pair generator (workload c6) and the training truth built
from it (CPU)."""
import numpy as np

from paper_2508_07423_amd import synth
from paper_2508_07423_amd import train as T


def test_pairs_share_the_parents_first_hits_then_leave_them():
    w = synth.C6
    n_pairs = n_tracks = 0
    for i in range(5):
        ev = synth.generate_event(w, i)
        part, part2, plane = ev["particle"], ev["particle2"], ev["plane"]
        assert np.all(part[part2 >= 0] >= 0)                 # only particle hits are shared
        for q in np.unique(part2[part2 >= 0]):
            shared = np.nonzero(part2 == q)[0]
            parents = np.unique(part[shared])
            assert len(parents) == 1
            p = parents[0]
            s = len(shared)
            assert w.pair_shared[0] <= s <= w.pair_shared[1]
            own_p = np.sort(plane[part == p])
            assert np.array_equal(np.sort(plane[shared]), own_p[:s])   # the parent's first s hits
            own_q = plane[part == q]
            assert len(own_q) >= 1 and own_q.min() > own_p[s - 1]       # then the partner's own hits
            n_pairs += 1
        n_tracks += len(np.unique(part[(part >= 0) & (part2 < 0)]))
    assert 0.04 < n_pairs / n_tracks < 0.15


def test_no_pairs_without_the_fraction():
    ev = synth.generate_event(synth.C3, 3)
    assert np.all(ev["particle2"] == -1)
    ev2 = synth.generate_event(synth.C3.with_(pair_fraction=0.0), 3)
    for k in ev:
        assert np.array_equal(ev[k], ev2[k])


def test_truth_follows_both_particles_through_shared_hits():
    w = synth.C6
    batch = synth.generate_batch(w, 3)
    t = T.truth_arrays(batch, w, np.random.default_rng(0))
    part, part2, z = batch["particle"], batch["particle2"], batch["z"]
    for h in np.nonzero(part2 >= 0)[0][:200]:
        q = part2[h]
        e = int(np.searchsorted(batch["hit_off"], h, side="right")) - 1
        a, b = batch["hit_off"][e], batch["hit_off"][e + 1]
        chain = np.arange(a, b)[(part[a:b] == q) | (part2[a:b] == q)]
        chain = chain[np.argsort(z[chain], kind="stable")]
        k = int(np.nonzero(chain == h)[0][0])
        assert t["succ2"][h] == (chain[k + 1] if k + 1 < len(chain) else -1)
    assert np.all(t["succ2"][part2 < 0] == -1)
