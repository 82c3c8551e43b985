"""Shared helpers of the GPU parity tests (comparison protocol against the oracle).

Protocol (spec tolerances):
  edges   for every source whose candidates are decidable (no |d - r| within
          1e-6 and, when the k_max cap binds, a gap above 1e-6 between the
          k-th and (k+1)-th nearest) the GPU row equals the oracle row exactly;
          otherwise the GPU row lies inside the rows possible within 1e-6 and
          holds at most k_max targets
  scores  FP32 path: |s_gpu - s_oracle| <= 1e-5 on every edge, with the
          oracle's interaction network evaluated on the GPU's edge list
  keep    equal wherever |s_oracle - 0.5| > 1e-4
  labels  bit-exact against BFS over the GPU's own kept edges; equal to the
          oracle's labels for hits whose oracle component touches no
          undecidable edge
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

EDGE_EPS = 1e-6
SCORE_TOL = 1e-5
KEEP_BAND = 1e-4


def oracle_event(ev, w, weights):
    return O.run_event(ev, w, weights, with_margins=True)


def check_edges(gsrc, gdst, ref, ev_plane, w, emb64):
    """gsrc/gdst: the GPU's edges of one event in local indices."""
    n = len(ev_plane)
    osrc, odst = ref["src"], ref["dst"]
    decidable = (ref["r_margin"] > EDGE_EPS) & (ref["k_gap"] > EDGE_EPS)
    g_rows = np.split(gdst, np.searchsorted(gsrc, np.arange(1, n)))
    o_rows = np.split(odst, np.searchsorted(osrc, np.arange(1, n)))
    r = float(np.float32(w.radius))
    n_undec = 0
    for i in range(n):
        g, o = g_rows[i], o_rows[i]
        if decidable[i]:
            assert np.array_equal(g, o), f"row {i}: gpu {g} oracle {o}"
        else:
            n_undec += 1
            check_undecidable_row(i, g, ev_plane, emb64, r, w)
    return n_undec, ~decidable


def check_undecidable_row(i, g, ev_plane, emb64, r, w):
    """A row with a candidate within EDGE_EPS of r, or a near tie at the k_max
    boundary: the GPU row holds only possible targets (window, d < r + eps),
    ascending, at most k_max of them, and every certain target: one with
    d < r - eps that at most k_max - 1 other possible candidates could precede
    (d' < d + eps).  It holds at least min(k_max, #(d < r - eps)) targets."""
    assert len(g) <= w.k_max
    assert np.all(np.diff(g) > 0)
    dp = ev_plane - ev_plane[i]
    win = np.nonzero((dp >= 1) & (dp <= w.plane_window))[0]
    d = np.sqrt(((emb64[win] - emb64[i]) ** 2).sum(1))
    possible = win[d < r + EDGE_EPS]
    assert np.all(np.isin(g, possible)), f"row {i}: {np.setdiff1d(g, possible)} not within r + eps"
    dpos = np.sort(d[d < r + EDGE_EPS])
    inside = d < r - EDGE_EPS
    ahead = np.searchsorted(dpos, d + EDGE_EPS, side="left")     # possible candidates with d' < d + eps
    certain = win[inside & (ahead <= w.k_max)]
    missing = np.setdiff1d(certain, g)
    assert len(missing) == 0, f"row {i}: certain targets {missing} missing"
    assert len(g) >= min(w.k_max, int(inside.sum())), f"row {i}: {len(g)} targets"


def check_scores(gsrc, gdst, gscore, cart64, weights, w, ref=None, tol=SCORE_TOL):
    if ref is not None and np.array_equal(gsrc, ref["src"]) and np.array_equal(gdst, ref["dst"]):
        s64 = ref["score"]
    else:
        s64 = O.sigmoid(O.gnn(cart64, gsrc, gdst, weights, w.gnn_hidden, w.gnn_steps))
    err = np.abs(gscore.astype(np.float64) - s64)
    assert err.max(initial=0.0) <= tol, f"max score error {err.max()} (bound {tol})"
    far = np.abs(s64 - 0.5) > KEEP_BAND
    assert np.array_equal(gscore[far] >= 0.5, s64[far] >= 0.5)
    return s64, err


def check_labels(n, gsrc, gdst, gscore, glabels_local, ref):
    keep = gscore >= np.float32(0.5)
    bfs = O.components(n, gsrc, gdst, keep)
    assert np.array_equal(glabels_local, bfs)
    # hits touching an edge present on one side only, or an edge whose score
    # lies in the undecidable band; their oracle components are excluded
    g = set(zip(gsrc.tolist(), gdst.tolist()))
    o = set(zip(ref["src"].tolist(), ref["dst"].tolist()))
    bad_hits = set()
    for a, b in g ^ o:
        bad_hits.update((a, b))
    near = np.abs(ref["score"] - 0.5) <= KEEP_BAND
    bad_hits.update(ref["src"][near].tolist())
    bad_hits.update(ref["dst"][near].tolist())
    lab = ref["labels"]
    bad = set(lab[list(bad_hits)].tolist()) if bad_hits else set()
    ok = ~np.isin(lab, list(bad))
    assert np.array_equal(glabels_local[ok], lab[ok])
    return ok.mean()
