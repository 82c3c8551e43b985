"""Pins of the oracle's triplet stage (CPU only; thesis ch. 8 "Triplet
Building" and "Track Building").

Checked against routes that share nothing with the oracle's code:
  - triplet enumeration: brute force over every ordered pair of kept edges
    (a triplet is two kept edges sharing one hit), and the closed-form counts
    sum_C in_C * out_C, sum_C C(out_C, 2) + C(in_C, 2);
  - triplet classifiers: torch float64 (linear, layer_norm, relu) on the
    gathered encodings; the final edge encodings the oracle hands out
    reproduce its own edge logits through torch's classifier;
  - track building: the thesis's motivating cases written out by hand (two
    tracks sharing their first hits come out as two tracks that both hold
    the shared hits, where plain components merge them; a skipped plane
    bridged by two elbows leaves one track), and graphs without branching,
    where the tracks must equal scipy's connected components of the kept
    hit graph.
"""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from oracle import oracle as O
from paper_2508_07423_amd import synth
from tests.test_oracle_pins import _random_gnn_weights


def _random_graph(seed, n=14, n_planes=6, E=40, window=2):
    rng = np.random.default_rng(seed)
    plane = np.sort(rng.integers(0, n_planes, n)).astype(np.int32)
    pairs = set()
    for _ in range(E * 4):
        i, j = rng.integers(0, n, 2)
        if 1 <= plane[j] - plane[i] <= window:
            pairs.add((int(i), int(j)))
        if len(pairs) >= E:
            break
    pairs = sorted(pairs)
    src = np.array([p[0] for p in pairs], np.int32)
    dst = np.array([p[1] for p in pairs], np.int32)
    keep = rng.uniform(0, 1, len(src)) < 0.7
    return plane, src, dst, keep


def _brute_triplets(plane, src, dst, keep):
    kept = [e for e in range(len(src)) if keep[e]]
    out = set()
    for p, q in itertools.permutations(kept, 2):
        if dst[p] == src[q]:
            out.add((0, p, q))
        if src[p] == src[q] and p < q:
            a, b = (q, p) if plane[dst[q]] < plane[dst[p]] else (p, q)
            out.add((1, a, b))
        if dst[p] == dst[q] and p < q:
            a, b = (q, p) if plane[src[q]] > plane[src[p]] else (p, q)
            out.add((2, a, b))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_triplets_equal_brute_force_over_edge_pairs(seed):
    plane, src, dst, keep = _random_graph(seed)
    n = len(plane)
    ta, tb, kind = O.triplets(n, src, dst, plane, keep)
    got = list(zip(kind.tolist(), ta.tolist(), tb.tolist()))
    assert len(got) == len(set(got))
    assert set(got) == _brute_triplets(plane, src, dst, keep)
    # closed-form counts around every hit
    ind = np.bincount(dst[keep], minlength=n)
    outd = np.bincount(src[keep], minlength=n)
    assert int((kind == 0).sum()) == int((ind * outd).sum())
    assert int((kind == 1).sum()) == int((outd * (outd - 1) // 2).sum())
    assert int((kind == 2).sum()) == int((ind * (ind - 1) // 2).sum())
    # order: articulations first, each block hit by hit (the shared hit C ascending)
    assert np.all(np.diff(kind.astype(int) > 0) >= 0)
    shared_hit = np.where(kind == 0, dst[ta], np.where(kind == 1, src[ta], dst[ta]))
    art = kind == 0
    assert np.all(np.diff(shared_hit[art]) >= 0) and np.all(np.diff(shared_hit[~art]) >= 0)
    # the unpurified graph holds more triplets; an empty purified graph none
    assert len(O.triplets(n, src, dst, plane, np.zeros_like(keep))[0]) == 0


def _heads(H, seed):
    rng = np.random.default_rng(seed)
    return {h: [(rng.normal(0, 0.3, (a, b)), rng.normal(0, 0.2, b)) for a, b in [(2 * H, H), (H, H), (H, 1)]]
            for h in ("art", "elb")}


def _torch_head(x, layers):
    t = torch.tensor(x, dtype=torch.float64)
    for i, (W, b) in enumerate(layers):
        t = t @ torch.tensor(W, dtype=torch.float64) + torch.tensor(b, dtype=torch.float64)
        if i < 2:
            t = torch.relu(F.layer_norm(t, (t.shape[-1],), eps=1e-5))
    return t[:, 0].numpy()


@pytest.mark.parametrize("H", [32, 64])
def test_triplet_logits_match_torch(H):
    rng = np.random.default_rng(H)
    E, T = 30, 50
    e = rng.normal(0, 1, (E, H))
    ta = rng.integers(0, E, T).astype(np.int32)
    tb = rng.integers(0, E, T).astype(np.int32)
    kind = rng.integers(0, 3, T).astype(np.uint8)
    heads = _heads(H, 3)
    got = O.triplet_logits(ta, tb, kind, e, heads)
    x = np.concatenate([e[ta], e[tb]], 1)
    ref = np.where(kind == 0, _torch_head(x, heads["art"]), _torch_head(x, heads["elb"]))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    # the input order matters: [e_a, e_b] is not [e_b, e_a]
    swapped = O.triplet_logits(tb, ta, kind, e, heads)
    assert np.max(np.abs(swapped - got)) > 1e-3
    assert O.triplet_head_size(H) == sum(W.size + b.size for W, b in heads["art"])


def test_final_edge_encodings_reproduce_the_edge_logits():
    H, S = 32, 2
    rng = np.random.default_rng(5)
    n, E = 30, 90
    cart = rng.uniform(-1, 1, (n, 3))
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    W = _random_gnn_weights(H, S, 4)
    logit, e = O.gnn(cart, src, dst, W, H, S, return_e=True)
    np.testing.assert_array_equal(logit, O.gnn(cart, src, dst, W, H, S))
    (W1, b1), (w2, b2) = W["cls"]
    t = torch.tensor(e) @ torch.tensor(W1, dtype=torch.float64) + torch.tensor(b1, dtype=torch.float64)
    t = torch.relu(F.layer_norm(t, (H,), eps=1e-5))
    ref = (t @ torch.tensor(w2, dtype=torch.float64))[:, 0] + float(b2[0])
    np.testing.assert_allclose(logit, ref.numpy(), rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# track building: hand-built purified graphs
# --------------------------------------------------------------------------

def _build(plane, edges, keep_triplet):
    """edges: list of (src, dst) in (src, dst) order; keep_triplet(kind, (a_src, a_dst), (b_src, b_dst)) -> bool."""
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    assert list(zip(src, dst)) == sorted(zip(src, dst))
    plane = np.asarray(plane, np.int32)
    keep = np.ones(len(src), bool)
    n = len(plane)
    ta, tb, kind = O.triplets(n, src, dst, plane, keep)
    tkeep = np.array([keep_triplet(int(k), (int(src[a]), int(dst[a])), (int(src[b]), int(dst[b])))
                      for k, a, b in zip(kind, ta, tb)], bool)
    r = O.build_tracks(n, src, dst, plane, keep, ta, tb, kind, tkeep)
    r["labels"] = O.components(n, src, dst, keep)
    return r


def _sets(tracks):
    return sorted(tuple(t.tolist()) for t in tracks)


def test_single_chain_is_one_track():
    r = _build([0, 1, 2, 3, 4], [(0, 1), (1, 2), (2, 3), (3, 4)], lambda k, a, b: True)
    assert _sets(r["tracks"]) == [(0, 1, 2, 3, 4)]
    assert not r["dup"].any()


def _shared_start_event():
    # hits: 0 (plane 0), 1 (plane 1) shared; track a: 2 (plane 2), 3 (plane 3); track b: 4 (plane 2), 5 (plane 3)
    plane = [0, 1, 2, 3, 2, 3]
    edges = [(0, 1), (1, 2), (1, 4), (2, 3), (4, 5)]
    return plane, edges


def test_tracks_sharing_their_first_hits_are_separated():
    plane, edges = _shared_start_event()
    # the elbow between the two tracks' first own edges is rejected; every articulation kept
    r = _build(plane, edges, lambda k, a, b: k == 0)
    assert _sets(r["tracks"]) == [(0, 1, 2, 3), (0, 1, 4, 5)]
    # plain components merge both particles into one group
    assert len(set(r["labels"].tolist())) == 1
    # the shared edge 0->1 (index 0) is its own component; both tracks hold it
    assert sorted(zip(r["c1"].tolist(), r["c2"].tolist())) == [(0, 1), (0, 2)]


def test_rejected_articulation_splits_at_the_shared_hit():
    plane, edges = _shared_start_event()
    r = _build(plane, edges, lambda k, a, b: k == 0 and not (a == (0, 1) and b == (1, 4)))
    assert _sets(r["tracks"]) == [(0, 1, 2, 3), (1, 4, 5)]


def _skip_event():
    # one particle on planes 0..3 and a skip edge 0 -> 2 across plane 1
    return [0, 1, 2, 3], [(0, 1), (0, 2), (1, 2), (2, 3)]


def test_skip_edge_bridged_by_two_elbows_is_a_duplicate():
    plane, edges = _skip_event()
    r = _build(plane, edges, lambda k, a, b: True)
    assert r["dup"].tolist() == [0, 1, 0, 0]
    assert _sets(r["tracks"]) == [(0, 1, 2, 3)]


def test_skip_edge_with_one_elbow_is_not_a_duplicate():
    plane, edges = _skip_event()
    # the right elbow (1->2, 0->2) at hit 2 is rejected: 0->2 stays, 2->3 then has two predecessors
    r = _build(plane, edges, lambda k, a, b: k != 2)
    assert not r["dup"].any()
    assert _sets(r["tracks"]) == [(0, 1, 2, 3), (0, 2, 3)]


def test_no_kept_triplet_leaves_every_edge_a_track():
    plane, edges = _shared_start_event()
    r = _build(plane, edges, lambda k, a, b: False)
    assert _sets(r["tracks"]) == sorted(edges)


def test_empty_graph_has_no_tracks():
    z = np.zeros(0, np.int32)
    r = O.build_tracks(3, z, z, np.array([0, 1, 2], np.int32), np.zeros(0, bool), z, z, np.zeros(0, np.uint8),
                       np.zeros(0, bool))
    assert r["tracks"] == []


@pytest.mark.parametrize("seed", range(5))
def test_unbranched_graph_tracks_are_its_components(seed):
    # disjoint chains (every hit at most one kept in- and out-edge) plus isolated hits
    rng = np.random.default_rng(seed)
    n_planes, n_chains = 8, 12
    plane, edges, hit = [], [], 0
    for _ in range(n_chains):
        length = int(rng.integers(1, n_planes))
        p0 = int(rng.integers(0, n_planes - length + 1))
        ids = list(range(hit, hit + length))
        plane += list(range(p0, p0 + length))
        edges += list(zip(ids[:-1], ids[1:]))
        hit += length
    perm = rng.permutation(hit)                  # shuffle hit indices
    inv = np.argsort(perm)
    plane = np.asarray(plane)[perm]
    edges = sorted((int(inv[a]), int(inv[b])) for a, b in edges)
    r = _build(plane, edges, lambda k, a, b: True)
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    g = coo_matrix((np.ones(len(src)), (src, dst)), shape=(hit, hit))
    nc, lab = connected_components(g, directed=True, connection="weak")
    deg = np.bincount(src, minlength=hit) + np.bincount(dst, minlength=hit)
    comps = sorted(tuple(np.nonzero((lab == c) & (deg > 0))[0].tolist()) for c in range(nc))
    comps = [c for c in comps if c]
    assert _sets(r["tracks"]) == comps


@pytest.mark.parametrize("seed", range(4))
def test_every_kept_edge_lies_in_a_track(seed):
    plane, src, dst, keep = _random_graph(seed + 10, n=20, E=60)
    n = len(plane)
    ta, tb, kind = O.triplets(n, src, dst, plane, keep)
    tkeep = np.random.default_rng(seed).uniform(0, 1, len(ta)) < 0.6
    r = O.build_tracks(n, src, dst, plane, keep, ta, tb, kind, tkeep)
    hits_of = [set(t.tolist()) for t in r["tracks"]]
    for e in np.nonzero(keep)[0]:
        if r["dup"][e]:
            continue
        assert any(src[e] in h and dst[e] in h for h in hits_of)
        assert r["comp"][e] >= 0 and r["comp"][e] <= e
    assert np.all(r["comp"][~keep] == -1)
    for t in r["tracks"]:
        assert np.all(np.diff(t) > 0)


def test_event_pipeline_with_triplets_is_consistent():
    w = synth.C1
    ev = synth.event_slice(synth.generate_batch(w, 1), 0)
    heads = synth.xavier_triplets(w)
    out = O.run_event_triplets(ev, w, synth.xavier_weights(w), heads)
    ref = O.run_event(ev, w, synth.xavier_weights(w))
    np.testing.assert_array_equal(out["logit"], ref["logit"])
    np.testing.assert_array_equal(out["labels"], ref["labels"])
    assert len(out["ta"]) == len(O.triplets(len(ev["x"]), out["src"], out["dst"], ev["plane"], out["keep"])[0])
