"""Host logic of the occupancy study: binning by hits per event and packing
the selected events back to back."""
import numpy as np

from paper_2508_07423_amd import occupancy, synth


def test_bins_partition_events_by_hit_count():
    batch = synth.generate_batch(synth.C3, 60)
    n = np.diff(batch["hit_off"])
    bins = occupancy.bins_of(batch["hit_off"])
    seen = np.concatenate([idx for _, _, idx in bins])
    assert sorted(seen.tolist()) == list(range(60))
    for lo, hi, idx in bins:
        assert np.all((n[idx] >= lo) & (n[idx] < hi))
    capped = occupancy.bins_of(batch["hit_off"], max_events=2)
    assert all(len(idx) <= 2 for _, _, idx in capped)


def test_sub_batch_packs_the_chosen_events():
    batch = synth.generate_batch(synth.C3, 12)
    pick = [7, 2, 11]
    sb = occupancy.sub_batch(batch, pick)
    assert sb["hit_off"][0] == 0 and len(sb["hit_off"]) == 4
    for j, i in enumerate(pick):
        a, b = sb["hit_off"][j], sb["hit_off"][j + 1]
        ev = synth.event_slice(batch, i)
        for k in ("x", "y", "z", "plane", "particle"):
            assert np.array_equal(sb[k][a:b], ev[k])
    empty = occupancy.sub_batch(batch, [])
    assert len(empty["x"]) == 0 and list(empty["hit_off"]) == [0]
