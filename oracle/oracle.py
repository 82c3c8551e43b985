"""Python driver of the FP64 CPU oracle (``etx_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It marshals numpy arrays
into the C oracle and strings its steps together per event, exactly in the
order of the thesis's pipeline (ch. 8 "The ETX4VELO Pipeline"; ch. 9 runs
it on GPU without the triplet stage):

    features -> embedding MLP -> radius graph (k_max cap) -> interaction
    network -> sigmoid score -> score cut (s >= threshold) -> components,

and the triplet stage after the score cut (``run_event_triplets``):
triplets of the purified graph -> triplet classifiers -> track building.

Events are independent, so ``run_batch`` spreads them over a thread pool
(ctypes releases the GIL during each C call).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "etx_oracle.c")
_SRC_TRIPLETS = os.path.join(_HERE, "triplets.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc -O2 (no BLAS, no SIMD intrinsics)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    srcs = [_SRC, _SRC_TRIPLETS]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in srcs):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               *srcs, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.oracle_features.argtypes = [i64, P, P, P, dbl, dbl, P, P]
        L.oracle_embed.argtypes = [i64, P, i32, P, P, P, i32, P, P, i32]
        L.oracle_radius.argtypes = [i64, P, P, i32, dbl, i32, i32, P, P, i64]
        L.oracle_radius.restype = i64
        L.oracle_radius_margins.argtypes = [i64, P, P, i32, dbl, i32, i32, P, P]
        L.oracle_gnn.argtypes = [i64, P, i64, P, P, i32, i32, P, P, i32, P, P, i32, i32, P]
        L.oracle_pow2_scale.argtypes = [dbl]
        L.oracle_pow2_scale.restype = dbl
        L.oracle_components.argtypes = [i64, i64, P, P, P, P]
        L.oracle_round_bf16.argtypes = [dbl]
        L.oracle_round_bf16.restype = dbl
        L.oracle_round_e4m3.argtypes = [dbl]
        L.oracle_round_e4m3.restype = dbl
        L.oracle_round_int8.argtypes = [dbl]
        L.oracle_round_int8.restype = dbl
        L.oracle_prefilter_features.argtypes = [i64, P, P, P, P, P, P, i32, dbl, dbl, P]
        L.oracle_prefilter_forward.argtypes = [i64, P, i32, P, P, i32]
        L.oracle_prefilter_loss_grad.argtypes = [i64, P, P, i32, P, dbl, P, i32]
        L.oracle_prefilter_loss_grad.restype = dbl
        L.oracle_adam.argtypes = [i64, P, P, P, P, dbl, dbl, dbl, dbl, i64]
        L.oracle_embed_hinge_loss_grad.argtypes = [i64, P, i32, P, P, i64, P, P, i64, P, P, dbl, dbl, P]
        L.oracle_embed_hinge_loss_grad.restype = dbl
        L.oracle_gnn_focal_loss_grad.argtypes = [i64, P, i64, P, P, i32, i32, P, P, dbl, dbl, P]
        L.oracle_gnn_focal_loss_grad.restype = dbl
        L.oracle_gnn_triplet_loss_grad.argtypes = [i64, P, i64, P, P, i32, i32, P, P, i64, P, P, P, P, P, dbl, dbl,
                                                   P, P]
        L.oracle_gnn_triplet_loss_grad.restype = dbl
        L.oracle_triplets.argtypes = [i64, i64, P, P, P, P, P, P, P, i64]
        L.oracle_triplets.restype = i64
        L.oracle_triplet_head_size.argtypes = [i32]
        L.oracle_triplet_head_size.restype = i64
        L.oracle_triplet_logits.argtypes = [i64, P, P, P, P, i32, P, P]
        L.oracle_build_tracks.argtypes = [i64, i64, P, P, P, P, i64, P, P, P, P, P, P, P, P, P, P, i64, i64, P]
        L.oracle_build_tracks.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# single steps
# ---------------------------------------------------------------------------

def features(x, y, z, r_scale: float, z_scale: float) -> Tuple[np.ndarray, np.ndarray]:
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    n = len(x)
    cyl = np.zeros((n, 3)); cart = np.zeros((n, 3))
    lib().oracle_features(n, _p(x), _p(y), _p(z), float(r_scale), float(z_scale), _p(cyl), _p(cart))
    return cyl, cart


def _flat(layers) -> np.ndarray:
    parts = []
    for W, b in layers:
        parts.append(np.asarray(W, np.float64).ravel())
        parts.append(np.asarray(b, np.float64).ravel())
    return np.concatenate(parts) if parts else np.zeros(0)


def embed(cyl: np.ndarray, layers, qmode: int = 0, act_scale=None, amax=None, f32: bool = False) -> np.ndarray:
    """Embedding MLP.  qmode 1/2 quantise the GEMM operands of layers >= 1
    (act_scale[l]: scale of layer l's input in FP8); amax (float64 array of
    len(layers)) receives the running max |input| of each layer.  f32: every
    arithmetic result rounded to FP32 (an FP32 evaluation of the same network,
    used to size low-precision tolerances; not the oracle)."""
    cyl = _c(cyl, np.float64)
    dims = np.array([layers[0][0].shape[0]] + [W.shape[1] for W, _ in layers], dtype=np.int32)
    n = len(cyl)
    out = np.zeros((n, int(dims[-1])))
    params = _flat(layers)
    qs = None if act_scale is None else _c(act_scale, np.float64)
    lib().oracle_embed(n, _p(cyl), len(layers), _p(dims), _p(params), _p(out), qmode,
                       _p(qs) if qs is not None else None, _p(amax) if amax is not None else None, int(f32))
    return out


def radius_graph(plane, emb, radius: float, k_max: int, window: int) -> Tuple[np.ndarray, np.ndarray]:
    plane = _c(plane, np.int32)
    emb = _c(emb, np.float64)
    n, D = emb.shape if emb.ndim == 2 else (0, 1)
    cap = max(1, n * k_max)
    src = np.zeros(cap, np.int32); dst = np.zeros(cap, np.int32)
    E = lib().oracle_radius(n, _p(plane), _p(emb), D, float(radius), k_max, window, _p(src), _p(dst), cap)
    assert E <= cap
    return src[:E].copy(), dst[:E].copy()


def radius_margins(plane, emb, radius: float, k_max: int, window: int) -> Tuple[np.ndarray, np.ndarray]:
    plane = _c(plane, np.int32)
    emb = _c(emb, np.float64)
    n, D = emb.shape
    rm = np.zeros(n); kg = np.zeros(n)
    lib().oracle_radius_margins(n, _p(plane), _p(emb), D, float(radius), k_max, window, _p(rm), _p(kg))
    return rm, kg


def gnn_param_blocks(weights) -> list:
    """The interaction-network layers in the oracle's parameter order."""
    S = sum(1 for k in weights if k.startswith("node") and k[4:].isdigit())
    blocks = list(weights["node_enc"]) + list(weights["edge_enc"])
    for k in range(S):
        blocks += list(weights[f"node{k}"]) + list(weights[f"edge{k}"])
    blocks += list(weights["cls"])
    return blocks


def gnn(cart, src, dst, weights, H: int, S: int, qmode: int = 0, act_scale=None, amax=None,
        compact: bool = False, f32: bool = False, return_e: bool = False):
    """Interaction-network logits.  act_scale / amax: the 8 + S activation
    slots documented in etx_oracle.c (qmode 2 / observers).  compact (qmode
    1, 2): node and edge encodings stored in low precision between layers
    instead of full-precision masters.  f32: FP32 evaluation (see embed).
    return_e: also return the final edge encodings e_S ([E][H])."""
    cart = _c(cart, np.float64)
    src = _c(src, np.int32); dst = _c(dst, np.int32)
    params = _flat(gnn_param_blocks(weights))
    E = len(src)
    logit = np.zeros(max(E, 1))
    e = np.zeros((max(E, 1), H)) if return_e else None
    qs = None if act_scale is None else _c(act_scale, np.float64)
    lib().oracle_gnn(len(cart), _p(cart), E, _p(src), _p(dst), H, S, _p(params), _p(logit), qmode,
                     _p(qs) if qs is not None else None, _p(amax) if amax is not None else None, int(compact),
                     int(f32), _p(e) if e is not None else None)
    if return_e:
        return logit[:E].copy(), e[:E].copy()
    return logit[:E].copy()


def pow2_scale(amax: float) -> float:
    return lib().oracle_pow2_scale(float(amax))


def calibrate(events, w, weights):
    """Static calibration in FP64: run the unquantised pipeline on `events`
    (list of dicts with x, y, z, plane), record the absolute maximum of every
    quantised tensor, and return the power-of-two scales
    (embedding layer-input scales, interaction-network slot scales)."""
    n_emb = len(weights["emb"])
    am_e = np.zeros(n_emb)
    am_g = np.zeros(8 + w.gnn_steps)
    r32 = float(np.float32(w.radius))
    for ev in events:
        cyl, cart = features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
        emb = embed(cyl, weights["emb"], amax=am_e)
        src, dst = radius_graph(ev["plane"], emb, r32, w.k_max, w.plane_window)
        gnn(cart, src, dst, weights, w.gnn_hidden, w.gnn_steps, amax=am_g)
    return (np.array([pow2_scale(a) for a in am_e]), np.array([pow2_scale(a) for a in am_g]), am_e, am_g)


def components(n: int, src, dst, keep) -> np.ndarray:
    src = _c(src, np.int32); dst = _c(dst, np.int32)
    keep = _c(keep, np.uint8)
    lab = np.zeros(max(n, 1), np.int32)
    lib().oracle_components(n, len(src), _p(src), _p(dst), _p(keep), _p(lab))
    return lab[:n].copy()


def sigmoid(z: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-z))


def round_bf16(x: float) -> float:
    return lib().oracle_round_bf16(float(x))


def round_e4m3(x: float) -> float:
    return lib().oracle_round_e4m3(float(x))


def round_int8(v: float) -> float:
    """Symmetric INT8 code of v = x / S: nearest integer (ties to even) in [-127, 127]."""
    return lib().oracle_round_int8(float(v))


def int8_scales(amax: np.ndarray) -> np.ndarray:
    """INT8 per-tensor scales S = amax / 127 (thesis ch. 4 "Quantization",
    symmetric range); 1 where a tensor is all zero."""
    amax = np.asarray(amax, np.float64)
    return np.where(amax > 0, amax / 127.0, 1.0)


# ---------------------------------------------------------------------------
# whole pipeline
# ---------------------------------------------------------------------------

def run_event(ev: Dict[str, np.ndarray], w, weights, with_margins: bool = False, qmode: int = 0,
              scales=None, emb_qmode: Optional[int] = None, compact: bool = False,
              f32: bool = False) -> Dict[str, np.ndarray]:
    """The full hot path on one event.  ``w`` carries the workload constants
    (r_scale, z_scale, radius, k_max, plane_window, gnn_hidden, gnn_steps,
    threshold); ``weights`` the network parameters.  qmode 1 (BF16), 2 (FP8,
    ``scales`` from ``calibrate``) or 3 (INT8, ``scales`` from ``int8_scales``
    of calibrate's maxima) quantises the GEMM operands; ``emb_qmode``
    gives the embedding its own mode (default: qmode); ``compact`` stores the
    network's node and edge state in low precision (see ``gnn``); ``f32``
    evaluates the embedding and the network in FP32 arithmetic (see ``embed``;
    a tolerance instrument, not the oracle)."""
    cyl, cart = features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    es, gs = (scales[0], scales[1]) if scales is not None else (None, None)
    emb = embed(cyl, weights["emb"], qmode if emb_qmode is None else emb_qmode, es, f32=f32)
    r32 = float(np.float32(w.radius))
    src, dst = radius_graph(ev["plane"], emb, r32, w.k_max, w.plane_window)
    logit = gnn(cart, src, dst, weights, w.gnn_hidden, w.gnn_steps, qmode, gs, compact=compact, f32=f32)
    score = sigmoid(logit)
    keep = score >= w.threshold
    labels = components(len(cyl), src, dst, keep)
    out = dict(emb=emb, src=src, dst=dst, logit=logit, score=score, keep=keep, labels=labels)
    if with_margins:
        rm, kg = radius_margins(ev["plane"], emb, r32, w.k_max, w.plane_window)
        out["r_margin"], out["k_gap"] = rm, kg
    return out


def run_batch(batch: Dict[str, np.ndarray], w, weights, events: Optional[Sequence[int]] = None,
              threads: Optional[int] = None, with_margins: bool = False, qmode: int = 0,
              scales=None, emb_qmode: Optional[int] = None, compact: bool = False) -> List[Dict[str, np.ndarray]]:
    hit_off = batch["hit_off"]
    idx = list(range(len(hit_off) - 1)) if events is None else list(events)

    def one(i):
        a, b = int(hit_off[i]), int(hit_off[i + 1])
        ev = {k: batch[k][a:b] for k in ("x", "y", "z", "plane")}
        return run_event(ev, w, weights, with_margins, qmode, scales, emb_qmode, compact)

    nt = threads or os.cpu_count() or 1
    if nt <= 1 or len(idx) <= 1:
        return [one(i) for i in idx]
    with ThreadPoolExecutor(max_workers=nt) as ex:
        return list(ex.map(one, idx))


# ---------------------------------------------------------------------------
# learned prefilter (forward / loss / gradient / Adam)
# ---------------------------------------------------------------------------

def prefilter_features(src, dst, x, y, z, emb, r_scale, z_scale) -> np.ndarray:
    src = _c(src, np.int32); dst = _c(dst, np.int32)
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    emb = _c(emb, np.float64)
    E = len(src)
    f = np.zeros((max(E, 1), 6))
    lib().oracle_prefilter_features(E, _p(src), _p(dst), _p(x), _p(y), _p(z), _p(emb),
                                    emb.shape[1], float(r_scale), float(z_scale), _p(f))
    return f[:E].copy()


def prefilter_forward(f, layers, qmode: int = 0) -> np.ndarray:
    f = _c(f, np.float64)
    P = layers[0][0].shape[1]
    params = _flat(layers)
    out = np.zeros(max(len(f), 1))
    lib().oracle_prefilter_forward(len(f), _p(f), P, _p(params), _p(out), qmode)
    return out[:len(f)].copy()


def prefilter_loss_grad(f, labels, layers, pos_weight: float, qmode: int = 0) -> Tuple[float, np.ndarray]:
    f = _c(f, np.float64)
    lab = _c(labels, np.uint8)
    P = layers[0][0].shape[1]
    params = _flat(layers)
    g = np.zeros_like(params)
    loss = lib().oracle_prefilter_loss_grad(len(f), _p(f), _p(lab), P, _p(params), float(pos_weight), _p(g), qmode)
    return loss, g


def adam(p, m, v, g, lr, b1=0.9, b2=0.999, eps=1e-8, t=1):
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().oracle_adam(len(p), _p(p), _p(m), _p(v), _p(g), float(lr), float(b1), float(b2), float(eps), int(t))


# ---------------------------------------------------------------------------
# training losses and gradients (embedding and interaction network)
# ---------------------------------------------------------------------------

def embed_hinge_loss_grad(cyl, layers, gen_pairs, fake_pairs, margin: float, w_gen: float):
    """Pairwise hinge embedding loss (thesis ch. 8, eqs. loss1-loss3) over the
    genuine and fake pairs ((src, dst) arrays) and its gradient in the layout
    of the embedding parameters (W row-major [fan_in][fan_out], then b, per
    layer)."""
    cyl = _c(cyl, np.float64)
    dims = np.array([layers[0][0].shape[0]] + [W.shape[1] for W, _ in layers], dtype=np.int32)
    params = _flat(layers)
    g = np.zeros_like(params)
    gs, gd = _c(gen_pairs[0], np.int32), _c(gen_pairs[1], np.int32)
    fs, fd = _c(fake_pairs[0], np.int32), _c(fake_pairs[1], np.int32)
    loss = lib().oracle_embed_hinge_loss_grad(len(cyl), _p(cyl), len(layers), _p(dims), _p(params), len(gs), _p(gs),
                                              _p(gd), len(fs), _p(fs), _p(fd), float(margin), float(w_gen), _p(g))
    return loss, g


def gnn_focal_loss_grad(cart, src, dst, weights, H: int, S: int, labels, alpha: float = 0.25,
                        gamma: float = 2.0):
    """Mean sigmoid focal loss of the edge scores (thesis ch. 8, eq. gnn-loss
    without the triplet term) and its gradient in the layout of
    ``gnn_param_blocks`` (flattened)."""
    cart = _c(cart, np.float64)
    src = _c(src, np.int32); dst = _c(dst, np.int32)
    lab = _c(labels, np.uint8)
    params = _flat(gnn_param_blocks(weights))
    g = np.zeros_like(params)
    loss = lib().oracle_gnn_focal_loss_grad(len(cart), _p(cart), len(src), _p(src), _p(dst), H, S, _p(params),
                                            _p(lab), float(alpha), float(gamma), _p(g))
    return loss, g


# ---------------------------------------------------------------------------
# triplet stage (thesis ch. 8 "Triplet Building" and "Track Building"; the
# readings are listed at the top of triplets.c)
# ---------------------------------------------------------------------------

def triplets(n: int, src, dst, plane, keep) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Triplets of the purified graph: (ta, tb, kind), kind 0 articulation,
    1 left elbow, 2 right elbow; articulations first, then elbows."""
    src = _c(src, np.int32); dst = _c(dst, np.int32); plane = _c(plane, np.int32)
    keep = _c(keep, np.uint8)
    z = np.zeros(1, np.int32)
    cnt = lib().oracle_triplets(n, len(src), _p(src), _p(dst), _p(plane), _p(keep), _p(z), _p(z),
                                _p(np.zeros(1, np.uint8)), 0)
    ta = np.zeros(max(cnt, 1), np.int32); tb = np.zeros(max(cnt, 1), np.int32); kind = np.zeros(max(cnt, 1), np.uint8)
    lib().oracle_triplets(n, len(src), _p(src), _p(dst), _p(plane), _p(keep), _p(ta), _p(tb), _p(kind), cnt)
    return ta[:cnt].copy(), tb[:cnt].copy(), kind[:cnt].copy()


def triplet_head_size(H: int) -> int:
    return int(lib().oracle_triplet_head_size(H))


def triplet_params(heads) -> np.ndarray:
    """Flat float64 parameters of the two triplet classifiers: heads["art"],
    heads["elb"], each [(W1[2H][H], b1), (W2[H][H], b2), (w3[H][1], b3)]."""
    return np.concatenate([_flat(heads["art"]), _flat(heads["elb"])])


def triplet_logits(ta, tb, kind, e, heads) -> np.ndarray:
    ta = _c(ta, np.int32); tb = _c(tb, np.int32); kind = _c(kind, np.uint8)
    e = _c(e, np.float64)
    H = e.shape[1] if e.ndim == 2 else heads["art"][1][0].shape[0]
    params = triplet_params(heads)
    assert len(params) == 2 * triplet_head_size(H)
    out = np.zeros(max(len(ta), 1))
    lib().oracle_triplet_logits(len(ta), _p(ta), _p(tb), _p(kind), _p(e), H, _p(params), _p(out))
    return out[:len(ta)].copy()


def build_tracks(n: int, src, dst, plane, keep, ta, tb, kind, tkeep) -> Dict[str, object]:
    """Track building from the purified edge graph.  Returns dup, comp (per
    edge), tracks (list of ascending hit arrays) and each track's components
    (c1, c2; c2 = -1 for an untouched component)."""
    src = _c(src, np.int32); dst = _c(dst, np.int32); plane = _c(plane, np.int32)
    keep = _c(keep, np.uint8)
    ta = _c(ta, np.int32); tb = _c(tb, np.int32); kind = _c(kind, np.uint8); tkeep = _c(tkeep, np.uint8)
    E, T = len(src), len(ta)
    dup = np.zeros(max(E, 1), np.uint8); comp = np.zeros(max(E, 1), np.int32)
    tcap = E + T + 1                     # tracks <= components + shared links
    off = np.zeros(tcap + 1, np.int64)
    c1 = np.zeros(tcap, np.int32); c2 = np.zeros(tcap, np.int32)
    nh = C.c_int64(0)
    hcap = 4 * E + 2
    while True:
        hits = np.zeros(hcap, np.int32)
        nt = lib().oracle_build_tracks(n, E, _p(src), _p(dst), _p(plane), _p(keep), T, _p(ta), _p(tb), _p(kind),
                                       _p(tkeep), _p(dup), _p(comp), _p(off), _p(hits), _p(c1), _p(c2), tcap, hcap,
                                       C.byref(nh))
        if nh.value <= hcap:
            break
        hcap = nh.value
    assert nt <= tcap
    tracks = [hits[off[k]:off[k + 1]].copy() for k in range(nt)]
    return dict(dup=dup[:E].copy(), comp=comp[:E].copy(), tracks=tracks, c1=c1[:nt].copy(), c2=c2[:nt].copy())


def gnn_triplet_loss_grad(cart, src, dst, weights, H: int, S: int, labels, ta, tb, kind, tlabels, heads,
                          alpha: float = 0.25, gamma: float = 2.0):
    """eq. gnn-loss with its triplet term: the edge classifier's mean focal
    loss plus each triplet classifier's mean focal loss over its triplets, and
    the gradients (network parameters in the layout of ``gnn_param_blocks``;
    both triplet classifiers in the layout of ``triplet_params``)."""
    cart = _c(cart, np.float64)
    src = _c(src, np.int32); dst = _c(dst, np.int32)
    lab = _c(labels, np.uint8)
    ta = _c(ta, np.int32); tb = _c(tb, np.int32); kind = _c(kind, np.uint8); tlab = _c(tlabels, np.uint8)
    params = _flat(gnn_param_blocks(weights))
    tp = triplet_params(heads)
    g = np.zeros_like(params)
    tg = np.zeros_like(tp)
    loss = lib().oracle_gnn_triplet_loss_grad(len(cart), _p(cart), len(src), _p(src), _p(dst), H, S, _p(params),
                                              _p(lab), len(ta), _p(ta), _p(tb), _p(kind), _p(tlab), _p(tp),
                                              float(alpha), float(gamma), _p(g), _p(tg))
    return loss, g, tg


def run_event_triplets(ev: Dict[str, np.ndarray], w, weights, heads) -> Dict[str, np.ndarray]:
    """The pipeline of run_event followed by the triplet stage: triplets of
    the purified graph, their classifier scores, and the tracks."""
    cyl, cart = features(ev["x"], ev["y"], ev["z"], w.r_scale, w.z_scale)
    emb = embed(cyl, weights["emb"])
    src, dst = radius_graph(ev["plane"], emb, float(np.float32(w.radius)), w.k_max, w.plane_window)
    logit, e = gnn(cart, src, dst, weights, w.gnn_hidden, w.gnn_steps, return_e=True)
    score = sigmoid(logit)
    keep = score >= w.threshold
    n = len(cyl)
    ta, tb, kind = triplets(n, src, dst, ev["plane"], keep)
    tlogit = triplet_logits(ta, tb, kind, e, heads)
    tscore = sigmoid(tlogit)
    tkeep = tscore >= w.threshold
    tr = build_tracks(n, src, dst, ev["plane"], keep, ta, tb, kind, tkeep)
    out = dict(emb=emb, src=src, dst=dst, logit=logit, score=score, keep=keep, e=e,
               labels=components(n, src, dst, keep), ta=ta, tb=tb, kind=kind, tlogit=tlogit, tscore=tscore,
               tkeep=tkeep)
    out.update(tr)
    return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)
