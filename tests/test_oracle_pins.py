"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test reaches the expected value by another route: a closed form of the
geometry, a library routine (torch float64, scipy), brute force over all small
inputs, or an invariant the definition implies.  A dropped term, a wrong sign
or index, or a transposed operand anywhere in the oracle fails one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import oracle as O
from paper_2508_07423_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# features (ch. 8: normalised cylindrical input, normalised Cartesian node input)
# ---------------------------------------------------------------------------

def test_features_special_points():
    R, Z = 40.0, 450.0
    x = np.array([40.0, 0.0, -40.0, 0.0, 20.0], np.float32)
    y = np.array([0.0, 40.0, 0.0, -40.0, 20.0], np.float32)
    z = np.array([450.0, -225.0, 0.0, 90.0, 45.0], np.float32)
    cyl, cart = O.features(x, y, z, R, Z)
    # r / R_s on the axes, phi / pi = 0, 1/2, 1 (the (-pi, pi] branch), -1/2, 1/4
    np.testing.assert_allclose(cyl[:, 0], [1, 1, 1, 1, math.sqrt(800) / 40], rtol=0, atol=1e-15)
    np.testing.assert_allclose(cyl[:, 1], [0, 0.5, 1.0, -0.5, 0.25], rtol=0, atol=1e-15)
    np.testing.assert_allclose(cyl[:, 2], [1, -0.5, 0, 0.2, 0.1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(cart, np.stack([x / R, y / R, z / Z], 1), rtol=0, atol=1e-7)


# ---------------------------------------------------------------------------
# embedding MLP (Linear, ReLU between layers, linear output)
# ---------------------------------------------------------------------------

def _torch_mlp(x, layers):
    t = torch.tensor(x, dtype=torch.float64)
    for i, (W, b) in enumerate(layers):
        t = F.linear(t, torch.tensor(W.T, dtype=torch.float64), torch.tensor(b, dtype=torch.float64))
        if i + 1 < len(layers):
            t = F.relu(t)
    return t.numpy()


def test_embed_matches_torch_float64():
    w = synth.C2
    W = synth.xavier_weights(w)["emb"]
    rng = np.random.default_rng(0)
    W = [(Wi, rng.normal(0, 0.1, bi.shape).astype(np.float32)) for Wi, bi in W]  # nonzero biases
    cyl = rng.uniform(-1, 1, (300, 3))
    np.testing.assert_allclose(O.embed(cyl, W), _torch_mlp(cyl, W), rtol=1e-13, atol=1e-13)


def test_embed_special_weights():
    # zero weights: output = last bias; one-hot first layer passes a coordinate through ReLU
    cyl = np.array([[0.3, -0.7, 0.1], [-0.2, 0.4, 0.9]])
    W1 = np.zeros((3, 4), np.float32); W1[0, 0] = 1; W1[1, 1] = 1; W1[2, 2] = 1; W1[0, 3] = -1
    W2 = np.eye(4, 2, dtype=np.float32)
    out = O.embed(cyl, [(W1, np.zeros(4, np.float32)), (W2, np.array([0.5, -0.25], np.float32))])
    np.testing.assert_allclose(out, [[0.3 + 0.5, 0.0 - 0.25], [0.0 + 0.5, 0.4 - 0.25]], atol=1e-15)
    zero = [(np.zeros((3, 5), np.float32), np.ones(5, np.float32)), (np.zeros((5, 2), np.float32), np.array([2.0, -3.0], np.float32))]
    np.testing.assert_allclose(O.embed(cyl, zero), [[2, -3], [2, -3]], atol=0)


# ---------------------------------------------------------------------------
# radius graph (squared-distance equation, k-NN algorithm, planes p+1..p+W)
# ---------------------------------------------------------------------------

def _brute_force_py(plane, emb, r, k, W):
    """Pure-Python loops (tiny inputs): the candidate relation then the cap."""
    n = len(plane)
    edges = []
    for i in range(n):
        cands = []
        for j in range(n):
            if 1 <= plane[j] - plane[i] <= W:
                d2 = sum((emb[i][c] - emb[j][c]) ** 2 for c in range(len(emb[i])))
                if d2 < r * r:
                    cands.append((d2, j))
        cands.sort()
        edges += [(i, j) for j in sorted(j for _, j in cands[:k])]
    return edges


def test_radius_hand_event():
    # 1-D embedding on three planes: exact pair set by inspection
    plane = np.array([0, 1, 2, 1, 0, 3], np.int32)
    emb = np.array([[0.0], [0.05], [0.12], [0.30], [0.29], [0.21]])
    src, dst = O.radius_graph(plane, emb, 0.1, 8, 2)
    # 0->1 (0.05), 0->2 (0.12 no), 1->2 (0.07), 1->5 (0.16 no), 2->5 (0.09), 3->2 (0.18 no),
    # 3->5 (0.09), 4->3 (0.01), 4->1 (0.24 no)
    assert list(zip(src.tolist(), dst.tolist())) == [(0, 1), (1, 2), (2, 5), (3, 5), (4, 3)]


def test_radius_matches_kdtree_uncapped():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(3)
    n, D = 400, 5
    plane = rng.integers(0, 8, n).astype(np.int32)
    emb = rng.uniform(0, 1, (n, D))
    r = 0.35
    src, dst = O.radius_graph(plane, emb, r, n, 2)
    pairs = cKDTree(emb).query_pairs(r, output_type="ndarray")
    expect = set()
    for a, b in pairs:
        if np.sum((emb[a] - emb[b]) ** 2) >= r * r:
            continue  # query_pairs includes the boundary; the relation is strict
        if 1 <= plane[b] - plane[a] <= 2:
            expect.add((int(a), int(b)))
        elif 1 <= plane[a] - plane[b] <= 2:
            expect.add((int(b), int(a)))
    got = set(zip(src.tolist(), dst.tolist()))
    assert got == expect
    order = np.lexsort((dst, src))
    assert np.all(order == np.arange(len(src)))          # sorted by (src, dst)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_radius_cap_matches_python_loops(k):
    rng = np.random.default_rng(k)
    n = 60
    plane = rng.integers(0, 4, n).astype(np.int32)
    emb = rng.uniform(0, 1, (n, 3))
    src, dst = O.radius_graph(plane, emb, 0.6, k, 2)
    assert list(zip(src.tolist(), dst.tolist())) == _brute_force_py(plane.tolist(), emb.tolist(), 0.6, k, 2)


def test_radius_cap_tie_break_by_index():
    # source 0 with four candidates at exactly equal distance; k=2 keeps the two smallest indices
    plane = np.array([0, 1, 1, 2, 1], np.int32)
    emb = np.array([[0.0, 0.0], [0.25, 0.0], [0.0, 0.25], [-0.25, 0.0], [0.0, -0.25]])
    src, dst = O.radius_graph(plane, emb, 0.3, 2, 2)
    assert dst[src == 0].tolist() == [1, 2]


def test_radius_mirror_symmetry_when_cap_does_not_bind():
    # plane -> P-1-plane reverses every edge; with no cap the unordered pair sets agree
    w = synth.C1
    ev = synth.generate_event(w, 0)
    W = synth.xavier_weights(w)
    cyl, _ = O.features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    emb = O.embed(cyl, W["emb"])
    src, dst = O.radius_graph(ev["plane"], emb, 0.1, 10 ** 6, 2)
    mplane = (w.n_planes - 1 - ev["plane"]).astype(np.int32)
    ms, md = O.radius_graph(mplane, emb, 0.1, 10 ** 6, 2)
    assert set(zip(src.tolist(), dst.tolist())) == set(zip(md.tolist(), ms.tolist()))
    assert len(src) > 100


# ---------------------------------------------------------------------------
# interaction network (node/edge encoders, message equation, residual updates)
# ---------------------------------------------------------------------------

def _dense_gnn(cart, src, dst, weights, H, S):
    """Independent formulation with dense incidence matrices in torch float64:
    out-sum = B_src^T E, in-sum = B_dst^T E, gathers = B h."""
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64)
    n, E = len(cart), len(src)
    Bs = torch.zeros(E, n, dtype=torch.float64); Bs[torch.arange(E), torch.tensor(src, dtype=torch.long)] = 1
    Bd = torch.zeros(E, n, dtype=torch.float64); Bd[torch.arange(E), torch.tensor(dst, dtype=torch.long)] = 1

    def block(x, Wb):
        W, b = Wb
        return F.relu(F.layer_norm(x @ T(W) + T(b), (H,), eps=1e-5))

    def mlp2(x, layers):
        return block(block(x, layers[0]), layers[1])

    h = mlp2(T(cart), weights["node_enc"])
    e = mlp2(torch.cat([Bs @ h, Bd @ h], 1), weights["edge_enc"])
    for k in range(S):
        mo, mi = Bs.T @ e, Bd.T @ e
        h = h + mlp2(torch.cat([h, mo, mi], 1), weights[f"node{k}"])
        e = e + mlp2(torch.cat([e, Bs @ h, Bd @ h], 1), weights[f"edge{k}"])
    c = block(e, weights["cls"][0])
    W, b = weights["cls"][1]
    return (c @ T(W) + T(b))[:, 0].numpy()


def _random_gnn_weights(H, S, seed):
    w = synth.C1.with_(gnn_hidden=H, gnn_steps=S)
    W = synth.xavier_weights(w, seed)
    rng = np.random.default_rng(seed)
    # nonzero biases so that a dropped bias term is visible
    return {k: [(Wi, rng.normal(0, 0.2, bi.shape).astype(np.float32)) for Wi, bi in v] for k, v in W.items()}


@pytest.mark.parametrize("H,S", [(32, 1), (32, 4), (64, 2)])
def test_gnn_matches_dense_incidence_torch(H, S):
    rng = np.random.default_rng(H + S)
    n, E = 40, 150
    cart = rng.uniform(-1, 1, (n, 3))
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    W = _random_gnn_weights(H, S, 11)
    got = O.gnn(cart, src, dst, W, H, S)
    ref = _dense_gnn(cart, src, dst, W, H, S)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def _pow2_at_or_above(m):
    """The FP8 per-tensor scale from its definition: the smallest power of two
    s with m / s <= 448, found by walking powers of two (1 for m = 0)."""
    if not m > 0:
        return 1.0
    s = 1.0
    while m / s > 448.0:
        s *= 2.0
    while m / (s / 2.0) <= 448.0:
        s /= 2.0
    return s


def _dense_gnn_quantised(cart, src, dst, weights, H, S, qmode, act_scale, compact):
    """The quantised network in the dense formulation, rounding with torch's
    own bfloat16 / float8_e4m3fn casts and torch.round (INT8): every GEMM
    operand is rounded where it enters the GEMM (FP8, INT8: per-tensor
    activation scales, per-matrix weight scales); the 3-wide first layer, LayerNorm, residual additions, sums and
    the H -> 1 output layer are not.  compact: h is stored as BF16 and e in
    the operand format after every write."""
    T = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64)
    n, E = len(cart), len(src)
    Bs = torch.zeros(E, n, dtype=torch.float64); Bs[torch.arange(E), torch.tensor(src, dtype=torch.long)] = 1
    Bd = torch.zeros(E, n, dtype=torch.float64); Bd[torch.arange(E), torch.tensor(dst, dtype=torch.long)] = 1

    def q(x, s):
        if qmode == 1:
            return x.to(torch.bfloat16).to(torch.float64)
        if qmode == 3:      # torch.round: half to even
            return torch.round(x / s).clamp(-127.0, 127.0) * s
        return (x / s).clamp(-448.0, 448.0).to(torch.float8_e4m3fn).to(torch.float64) * s

    def bf(x):
        return x.to(torch.bfloat16).to(torch.float64)

    def qw(W):
        W = T(W)
        m = float(W.abs().max())
        return q(W, m / 127.0 if qmode == 3 else _pow2_at_or_above(m))

    def ln(x):
        return F.relu(F.layer_norm(x, (H,), eps=1e-5))

    sc = lambda i: float(act_scale[i]) if act_scale is not None else 1.0
    (W1, b1), (W2, b2) = weights["node_enc"]
    t = ln(T(cart) @ T(W1) + T(b1))
    h = ln(q(t, sc(0)) @ qw(W2) + T(b2))
    if compact:
        h = bf(h)
    (W1, b1), (W2, b2) = weights["edge_enc"]
    t = ln(torch.cat([q(Bs @ h, sc(1)), q(Bd @ h, sc(1))], 1) @ qw(W1) + T(b1))
    e = ln(q(t, sc(4)) @ qw(W2) + T(b2))
    if compact:
        e = q(e, sc(7))
    for k in range(S):
        mo, mi = Bs.T @ e, Bd.T @ e
        (W1, b1), (W2, b2) = weights[f"node{k}"]
        t = ln(torch.cat([q(h, sc(1)), q(mo, sc(2)), q(mi, sc(3))], 1) @ qw(W1) + T(b1))
        h = h + ln(q(t, sc(5)) @ qw(W2) + T(b2))
        if compact:
            h = bf(h)
        (W1, b1), (W2, b2) = weights[f"edge{k}"]
        t = ln(torch.cat([q(e, sc(7 + k)), q(Bs @ h, sc(1)), q(Bd @ h, sc(1))], 1) @ qw(W1) + T(b1))
        e = e + ln(q(t, sc(6)) @ qw(W2) + T(b2))
        if compact:
            e = q(e, sc(8 + k))
    (W1, b1), (W2, b2) = weights["cls"]
    c = ln(q(e, sc(7 + S)) @ qw(W1) + T(b1))
    return (c @ T(W2) + T(b2))[:, 0].numpy()


@pytest.mark.parametrize("qmode,compact", [(1, False), (1, True), (2, False), (2, True), (3, False), (3, True)])
def test_gnn_quantised_matches_dense_torch(qmode, compact):
    """The quantised oracle network (ch. 4 "Quantization": BF16, FP8-E4M3,
    symmetric INT8), with node and edge state kept in full precision or stored
    in low precision."""
    rng = np.random.default_rng(21 + qmode)
    n, E, H, S = 30, 120, 32, 3
    cart = rng.uniform(-1, 1, (n, 3))
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    W = _random_gnn_weights(H, S, 14)
    scales = None
    if qmode >= 2:
        amax = np.zeros(8 + S)
        O.gnn(cart, src, dst, W, H, S, amax=amax)
        scales = np.array([_pow2_at_or_above(a) if qmode == 2 else a / 127.0 for a in amax])
    got = O.gnn(cart, src, dst, W, H, S, qmode, scales, compact=compact)
    ref = _dense_gnn_quantised(cart, src, dst, W, H, S, qmode, scales, compact)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)
    # the two state formats differ, and both stay near the unquantised network
    other = O.gnn(cart, src, dst, W, H, S, qmode, scales, compact=not compact)
    full = O.gnn(cart, src, dst, W, H, S)
    assert np.abs(got - other).max() > 1e-6
    assert np.abs(got - full).max() < (2.0 if qmode == 2 else 0.5)


def test_gnn_permutation_equivariance():
    rng = np.random.default_rng(5)
    n, E, H, S = 50, 200, 32, 3
    cart = rng.uniform(-1, 1, (n, 3))
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    W = _random_gnn_weights(H, S, 12)
    base = O.gnn(cart, src, dst, W, H, S)
    pn = rng.permutation(n)        # new index of old node i is inv[i]
    inv = np.argsort(pn)
    pe = rng.permutation(E)
    got = O.gnn(cart[pn], inv[src[pe]].astype(np.int32), inv[dst[pe]].astype(np.int32), W, H, S)
    np.testing.assert_allclose(got, base[pe], rtol=1e-12, atol=1e-12)


def test_gnn_single_edge_and_isolated_direction():
    # one edge a->b: the out-sum of a and the in-sum of b equal e; reversing the
    # edge must change the logit unless the node and edge nets are symmetric
    H, S = 32, 2
    W = _random_gnn_weights(H, S, 13)
    cart = np.array([[0.1, 0.2, 0.3], [0.4, -0.1, 0.6]])
    fwd = O.gnn(cart, np.array([0], np.int32), np.array([1], np.int32), W, H, S)
    bwd = O.gnn(cart, np.array([1], np.int32), np.array([0], np.int32), W, H, S)
    ref = _dense_gnn(cart, np.array([0]), np.array([1]), W, H, S)
    np.testing.assert_allclose(fwd, ref, rtol=1e-12, atol=1e-12)
    assert abs(fwd[0] - bwd[0]) > 1e-6
    assert O.gnn(cart, np.zeros(0, np.int32), np.zeros(0, np.int32), W, H, S).shape == (0,)


# ---------------------------------------------------------------------------
# components (ch. 9 WCC: DFS over the purified graph, smallest label)
# ---------------------------------------------------------------------------

def _closure_labels(n, edges):
    reach = np.eye(n, dtype=bool)
    for a, b in edges:
        reach[a, b] = reach[b, a] = True
    for k in range(n):                       # Warshall transitive closure
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    return np.array([int(np.nonzero(reach[i])[0].min()) for i in range(n)])


def test_components_all_graphs_up_to_5_nodes():
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            edges = [pairs[t] for t in range(len(pairs)) if mask >> t & 1]
            src = np.array([a for a, b in edges], np.int32)
            dst = np.array([b for a, b in edges], np.int32)
            lab = O.components(n, src, dst, np.ones(len(edges), np.uint8))
            assert lab.tolist() == _closure_labels(n, edges).tolist()


def test_components_match_scipy_and_respect_keep():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(9)
    n, E = 3000, 2500
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    keep = rng.uniform(0, 1, E) < 0.7
    lab = O.components(n, src, dst, keep)
    A = coo_matrix((np.ones(keep.sum()), (src[keep], dst[keep])), shape=(n, n))
    ncomp, cc = connected_components(A, directed=True, connection="weak")
    assert len(np.unique(lab)) == ncomp
    # same partition, and the label is the minimum index of its part
    for c in range(ncomp):
        members = np.nonzero(cc == c)[0]
        assert np.all(lab[members] == members.min())


# ---------------------------------------------------------------------------
# quantisers (ch. 4 "Quantization": x = S x_q, x_q = clip(round(x / S)))
# ---------------------------------------------------------------------------

def _e4m3_table():
    """All 256 OCP E4M3 (FN) codes decoded from the format: bias 7, 3 mantissa
    bits, subnormals at exponent 0, S.1111.111 = NaN, no infinities."""
    vals = []
    for code in range(256):
        s, e, m = code >> 7, (code >> 3) & 15, code & 7
        if e == 15 and m == 7:
            vals.append(math.nan)
            continue
        v = (m / 8) * 2.0 ** -6 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
        vals.append(-v if s else v)
    return np.array(vals)


def test_e4m3_exhaustive_codes_and_midpoints():
    tab = _e4m3_table()
    finite = np.sort(np.unique(tab[np.isfinite(tab)]))
    assert finite.max() == 448.0 and finite.min() == -448.0 and len(finite) == 253  # +-0 merge
    for v in finite:
        assert O.round_e4m3(v) == v
    pos = finite[finite >= 0]
    for a, b in zip(pos[:-1], pos[1:]):
        mid = 0.5 * (a + b)
        # ties go to the code with an even mantissa
        ca = int(np.nonzero(tab == a)[0][0]); cb = int(np.nonzero(tab == b)[0][0])
        want = a if (ca & 1) == 0 else b
        assert O.round_e4m3(mid) == want
        assert O.round_e4m3(-mid) == -want
        assert O.round_e4m3(np.nextafter(mid, 0)) == a
        assert O.round_e4m3(np.nextafter(mid, 1e9)) == b
    assert O.round_e4m3(1e6) == 448.0 and O.round_e4m3(-500.0) == -448.0


def test_e4m3_matches_torch_cast_in_range():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 30, 5000), rng.normal(0, 0.01, 2000)])
    x = x[np.abs(x) < 440]
    ref = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([O.round_e4m3(float(np.float32(v))) for v in x])
    np.testing.assert_array_equal(got, ref)


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-30, 500), rng.normal(0, 1e30, 500)]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.round_bf16(float(v)) for v in x])
    np.testing.assert_array_equal(got, ref)


def test_int8_symmetric_example_from_thesis():
    """The thesis's worked INT8 example (ch. 4 "Quantization", calibration):
    range [-10.8, 10.8] gives S = 10.8/127, values outside clip to +-127."""
    with open(os.path.join(HERE, "golden", "quant_int8_example.json")) as f:
        g = json.load(f)
    S = g["alpha"] / g["qmax"]
    assert S == pytest.approx(10.8 / 127)
    for x, xq in g["cases"]:
        q = O.round_int8(x / S)            # the oracle's INT8 quantiser (qmode 3)
        assert q == xq
        assert abs(S * q - x) <= S / 2 or abs(x) > g["alpha"]
    # ties go to the even code
    assert [O.round_int8(v) for v in (0.5, 1.5, 2.5, -0.5, -1.5, 126.5, 127.5)] == [0, 2, 2, 0, -2, 126, 127]


# ---------------------------------------------------------------------------
# prefilter gradient and Adam
# ---------------------------------------------------------------------------

def _pf_layers(seed=3):
    layers = synth.xavier_prefilter(seed)
    rng = np.random.default_rng(seed)
    return [(W.astype(np.float64), rng.normal(0, 0.1, b.shape)) for W, b in layers]


def test_prefilter_grad_central_differences_and_torch():
    rng = np.random.default_rng(4)
    f = rng.normal(0, 1, (64, 6))
    lab = (rng.uniform(0, 1, 64) < 0.3).astype(np.uint8)
    L = _pf_layers()
    loss, g = O.prefilter_loss_grad(f, lab, L, 3.0)
    flat = O._flat(L)
    # torch autograd on the same function
    ps = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for Wb in L for a in Wb]
    x = torch.tensor(f)
    a1 = F.relu(x @ ps[0] + ps[1]); a2 = F.relu(a1 @ ps[2] + ps[3]); z = (a2 @ ps[4] + ps[5])[:, 0]
    y = torch.tensor(lab, dtype=torch.float64)
    wts = torch.where(y > 0, torch.tensor(3.0, dtype=torch.float64), torch.tensor(1.0, dtype=torch.float64))
    tl = (wts * F.binary_cross_entropy_with_logits(z, y, reduction="none")).mean()
    tl.backward()
    tg = torch.cat([p.grad.reshape(-1) for p in ps]).numpy()
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    np.testing.assert_allclose(g, tg, rtol=1e-9, atol=1e-12)
    # central differences on a sample of coordinates
    def lossof(p):
        Ls, o = [], 0
        for W, b in L:
            Wn = p[o:o + W.size].reshape(W.shape); o += W.size
            bn = p[o:o + b.size]; o += b.size
            Ls.append((Wn, bn))
        return O.prefilter_loss_grad(f, lab, Ls, 3.0)[0]
    for i in rng.choice(len(flat), 40, replace=False):
        hh = 1e-6
        p1 = flat.copy(); p1[i] += hh
        p2 = flat.copy(); p2[i] -= hh
        fd = (lossof(p1) - lossof(p2)) / (2 * hh)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i])


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(6)
    p = rng.normal(0, 1, 50); m = np.zeros(50); v = np.zeros(50)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(0, 1, 50)
        O.adam(p, m, v, g, 0.01, t=t)
        opt.zero_grad(); tp.grad = torch.tensor(g); opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# the assembled pipeline on the one-event workload
# ---------------------------------------------------------------------------

def test_pipeline_c1_invariants():
    w = synth.C1
    ev = synth.generate_event(w, 0)
    W = synth.xavier_weights(w)
    r = O.run_event(ev, w, W)
    n = len(ev["x"])
    src, dst, lab = r["src"], r["dst"], r["labels"]
    assert np.all(ev["plane"][dst] - ev["plane"][src] >= 1) and np.all(ev["plane"][dst] - ev["plane"][src] <= 2)
    assert np.all(np.bincount(src, minlength=n) <= w.k_max)
    assert np.all(lab <= np.arange(n)) and np.all(lab[lab] == lab)
    k = r["keep"]
    assert np.all(lab[src[k]] == lab[dst[k]])
    assert np.all((r["score"] >= 0.5) == k)
