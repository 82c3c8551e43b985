"""ctypes binding of ``libetx.so`` (C ABI in ``include/etx.h``).

Argument marshalling only: every step of the track-finding path runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  The
library must be built (``paper_2508_07423_amd/build.py``); importing this
module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetx.so")

ETX_OK, ETX_ERR_INVALID_ARG, ETX_ERR_CAPACITY, ETX_ERR_INPUT, ETX_ERR_WEIGHTS, ETX_ERR_UNSUPPORTED, ETX_ERR_HIP = range(7)
ETX_FP32, ETX_BF16, ETX_FP8_E4M3, ETX_INT8 = 0, 1, 2, 3
SC_I8 = 256                      # first slot of the INT8 scale set (etx_get_scales)
ETX_MAX_EVENT_HITS = 16384
ETX_N_CALIB = 64
ETX_PF_HIDDEN = 32
ETX_PF_NPARAM = 6 * 32 + 32 + 32 * 32 + 32 + 32 + 1
(ETX_VIEW_EMBEDDING, ETX_VIEW_BUCKET, ETX_VIEW_PLANE_OFF, ETX_VIEW_ROW_PTR, ETX_VIEW_COL_PTR, ETX_VIEW_CSC_EDGE,
 ETX_VIEW_NODE_H, ETX_VIEW_KEPT_EDGE, ETX_VIEW_KEPT_COUNT, ETX_VIEW_CALIB, ETX_VIEW_PF_KEEP, ETX_VIEW_PF_GRAD,
 ETX_VIEW_PF_PROB, ETX_VIEW_PF_FEAT, ETX_VIEW_PF_FALLBACK) = range(15)
(ETX_OPT_USE_GRAPH, ETX_OPT_EDGE_WG_PER_CU, ETX_OPT_NODE_WG_PER_CU, ETX_OPT_RADIUS_LDS,
 ETX_OPT_SEGSUM_UNROLL, ETX_OPT_PROFILE, ETX_OPT_EDGE_PIPELINE, ETX_OPT_EDGE_WG_SIZE,
 ETX_OPT_EDGE_WREG, ETX_OPT_EMBED_PRECISION, ETX_OPT_OUTSUM_LDS, ETX_OPT_F32_SPLIT,
 ETX_OPT_RADIUS_SINGLE_PASS, ETX_OPT_RADIUS_SORT_MIN, ETX_OPT_FUSE_MESSAGES, ETX_OPT_RADIUS_FAST,
 ETX_OPT_XCD_MAP, ETX_OPT_EDGE_PRODUCTS, ETX_OPT_CSC_PLACE, ETX_OPT_COMPACT_STATE,
 ETX_OPT_PROFILE_STAGES, ETX_OPT_PF_FEATURES, ETX_OPT_RADIUS_SPLIT) = range(23)
N_STAGES = 20


def ETX_TRIPLET_NPARAM(H: int) -> int:
    return 2 * (3 * H * H + 3 * H + 1)


class etx_config(C.Structure):
    _fields_ = [("n_planes", C.c_int32), ("r_scale_mm", C.c_float), ("z_scale_mm", C.c_float),
                ("emb_hidden", C.c_int32), ("emb_layers", C.c_int32), ("emb_dim", C.c_int32),
                ("radius", C.c_float), ("k_max", C.c_int32), ("plane_window", C.c_int32),
                ("gnn_hidden", C.c_int32), ("gnn_steps", C.c_int32), ("edge_threshold", C.c_float),
                ("precision", C.c_int32), ("prefilter", C.c_int32), ("prefilter_tau", C.c_float)]


class etx_hits(C.Structure):
    _fields_ = [("n_events", C.c_int64), ("n_hits", C.c_int64), ("hit_off", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("z", C.c_void_p), ("plane", C.c_void_p)]


class etx_out(C.Structure):
    _fields_ = [("edge_capacity", C.c_int64), ("src", C.c_void_p), ("dst", C.c_void_p), ("score", C.c_void_p),
                ("edge_off", C.c_void_p), ("labels", C.c_void_p), ("status", C.c_void_p)]


class etx_truth(C.Structure):
    _fields_ = [("particle", C.c_void_p), ("succ", C.c_void_p), ("pred", C.c_void_p), ("query", C.c_void_p),
                ("rnd", C.c_void_p), ("rnd_ptr", C.c_void_p), ("rnd_src", C.c_void_p), ("particle2", C.c_void_p),
                ("succ2", C.c_void_p)]


class etx_tracks(C.Structure):
    _fields_ = [("triplet_capacity", C.c_int64), ("tri_a", C.c_void_p), ("tri_b", C.c_void_p),
                ("tri_score", C.c_void_p), ("tri_kind", C.c_void_p), ("art_off", C.c_void_p),
                ("elb_off", C.c_void_p), ("track_capacity", C.c_int64), ("event_track_off", C.c_void_p),
                ("track_off", C.c_void_p), ("hit_capacity", C.c_int64), ("track_hits", C.c_void_p),
                ("status", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2508_07423_amd/build.py (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "etx_create": [C.POINTER(etx_config), P, sz, C.c_int, C.POINTER(P)],
            "etx_destroy": [P],
            "etx_weight_blob_size": [C.POINTER(etx_config), C.POINTER(sz)],
            "etx_workspace_size": [P, i64, i64, i64, C.POINTER(sz)],
            "etx_run": [P, C.POINTER(etx_hits), C.POINTER(etx_out), P, sz, P],
            "etx_workspace_view": [P, i64, i64, i64, i32, C.POINTER(sz), C.POINTER(sz)],
            "etx_set_option": [P, i32, i64],
            "etx_get_option": [P, i32, C.POINTER(i64)],
            "etx_autotune": [P, C.POINTER(etx_hits), C.POINTER(etx_out), P, sz, P, C.c_char_p],
            "etx_calibrate": [P, C.POINTER(etx_hits), C.POINTER(etx_out), P, sz, P],
            "etx_set_precision": [P, i32],
            "etx_prefilter_set": [P, P, i64],
            "etx_prefilter_get": [P, P, i64],
            "etx_prefilter_train_step": [P, C.POINTER(etx_hits), C.POINTER(etx_out), P, C.c_float, C.c_float, i64, P,
                                         P, sz, P],
            "etx_prefilter_state": [P, P, i64, i32],
            "etx_profile_read": [P, i32, P, P],
            "etx_get_scales": [P, P, i32],
            "etx_prefilter_config": [P, i32, C.c_float],
            "etx_quantize": [i32, P, P, i64, C.c_float, P],
            "etx_profile_reset": [P],
            "etx_save": [P, P, C.POINTER(sz)],
            "etx_load": [P, sz, C.c_int, C.POINTER(P)],
            "etx_tuning_save": [P, C.c_char_p],
            "etx_prefilter_band": [P, C.c_float, C.c_float],
            "etx_run_noalloc": [P, C.POINTER(etx_hits), C.POINTER(etx_out), P],
            "etx_train_begin": [P],
            "etx_train_params": [P, P, i64, i32],
            "etx_train_apply": [P],
            "etx_train_workspace_size": [P, i64, i64, i64, C.POINTER(sz)],
            "etx_train_view": [P, i64, i64, i64, i32, C.POINTER(sz), C.POINTER(sz)],
            "etx_train_embed_step": [P, C.POINTER(etx_hits), C.POINTER(etx_out), C.POINTER(etx_truth), C.c_float,
                                     C.c_float, C.c_float, C.c_float, i64, P, P, sz, P],
            "etx_train_gnn_step": [P, C.POINTER(etx_hits), C.POINTER(etx_out), C.POINTER(etx_truth), C.c_float,
                                   C.c_float, C.c_float, i64, P, P, sz, P],
            "etx_tuning_load": [P, C.c_char_p],
            "etx_triplet_set": [P, P, i64],
            "etx_triplet_get": [P, P, i64],
            "etx_tracks_workspace_size": [P, i64, i64, i64, i64, i64, C.POINTER(sz)],
            "etx_run_tracks": [P, C.POINTER(etx_hits), C.POINTER(etx_out), C.POINTER(etx_tracks), P, sz, P],
            "etx_train_triplet_workspace_size": [P, i64, i64, i64, i64, C.POINTER(sz)],
            "etx_train_triplet_step": [P, C.POINTER(etx_hits), C.POINTER(etx_out), C.POINTER(etx_truth), C.c_float,
                                       C.c_float, C.c_float, i64, i64, C.POINTER(i64), P, P, sz, P],
            "etx_train_triplet_view": [P, i64, i64, i64, i64, i32, C.POINTER(sz), C.POINTER(sz)],
            "etx_train_triplet_params": [P, P, i64, i32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.etx_status_str.argtypes = [C.c_int]
        L.etx_status_str.restype = C.c_char_p
        L.etx_stage_name.argtypes = [C.c_int32]
        L.etx_stage_name.restype = C.c_char_p
        L.etx_last_error.argtypes = []
        L.etx_last_error.restype = C.c_char_p
        _lib = L
    return _lib


EXPORTED = ["etx_create", "etx_destroy", "etx_weight_blob_size", "etx_workspace_size", "etx_run",
            "etx_workspace_view", "etx_set_option", "etx_get_option", "etx_autotune", "etx_calibrate",
            "etx_set_precision", "etx_prefilter_set", "etx_prefilter_get", "etx_prefilter_train_step",
            "etx_prefilter_state", "etx_status_str", "etx_last_error", "etx_profile_read", "etx_profile_reset",
            "etx_stage_name", "etx_get_scales", "etx_quantize", "etx_prefilter_config", "etx_save", "etx_load",
            "etx_tuning_save", "etx_tuning_load", "etx_prefilter_band", "etx_run_noalloc",
            "etx_train_begin", "etx_train_params", "etx_train_apply", "etx_train_workspace_size", "etx_train_view",
            "etx_train_embed_step", "etx_train_gnn_step", "etx_triplet_set", "etx_triplet_get",
            "etx_tracks_workspace_size", "etx_run_tracks", "etx_train_triplet_workspace_size",
            "etx_train_triplet_step", "etx_train_triplet_view", "etx_train_triplet_params"]


class EtxError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        detail = lib().etx_last_error().decode() if code == ETX_ERR_HIP else ""
        super().__init__(f"{what}: {etx_status_str(code)} ({code}) {detail}".rstrip())


def etx_status_str(code: int) -> str:
    return lib().etx_status_str(int(code)).decode()


def _check(code: int, what: str):
    if code != ETX_OK:
        raise EtxError(code, what)


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def etx_weight_blob_size(cfg: etx_config) -> int:
    n = C.c_size_t()
    _check(lib().etx_weight_blob_size(C.byref(cfg), C.byref(n)), "etx_weight_blob_size")
    return n.value


def etx_create(cfg: etx_config, blob: bytes, device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().etx_create(C.byref(cfg), buf, len(blob), device, C.byref(h)), "etx_create")
    return h


def etx_destroy(ctx) -> None:
    _check(lib().etx_destroy(ctx), "etx_destroy")


def etx_workspace_size(ctx, n_events: int, n_hits: int, edge_capacity: int) -> int:
    n = C.c_size_t()
    _check(lib().etx_workspace_size(ctx, n_events, n_hits, edge_capacity, C.byref(n)), "etx_workspace_size")
    return n.value


def etx_workspace_view(ctx, n_events: int, n_hits: int, edge_capacity: int, which: int):
    o, b = C.c_size_t(), C.c_size_t()
    _check(lib().etx_workspace_view(ctx, n_events, n_hits, edge_capacity, which, C.byref(o), C.byref(b)),
           "etx_workspace_view")
    return o.value, b.value


def etx_run(ctx, hits: etx_hits, out: etx_out, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _check(lib().etx_run(ctx, C.byref(hits), C.byref(out), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)),
           "etx_run")


def etx_set_option(ctx, key: int, value: int) -> None:
    _check(lib().etx_set_option(ctx, key, value), "etx_set_option")


def etx_get_option(ctx, key: int) -> int:
    v = C.c_int64()
    _check(lib().etx_get_option(ctx, key, C.byref(v)), "etx_get_option")
    return v.value


def etx_autotune(ctx, hits, out, ws_ptr, ws_bytes, stream, json_path: Optional[str] = None) -> None:
    _check(lib().etx_autotune(ctx, C.byref(hits), C.byref(out), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream),
                              json_path.encode() if json_path else None), "etx_autotune")


def etx_tuning_save(ctx, path: str) -> None:
    _check(lib().etx_tuning_save(ctx, path.encode()), "etx_tuning_save")


def etx_tuning_load(ctx, path: str) -> None:
    _check(lib().etx_tuning_load(ctx, path.encode()), "etx_tuning_load")


def etx_calibrate(ctx, hits, out, ws_ptr, ws_bytes, stream) -> None:
    _check(lib().etx_calibrate(ctx, C.byref(hits), C.byref(out), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)),
           "etx_calibrate")


def etx_set_precision(ctx, precision: int) -> None:
    _check(lib().etx_set_precision(ctx, precision), "etx_set_precision")


def etx_get_scales(ctx, n: int = 256) -> np.ndarray:
    s = np.zeros(n, np.float32)
    _check(lib().etx_get_scales(ctx, s.ctypes.data_as(C.c_void_p), n), "etx_get_scales")
    return s


def etx_quantize(precision: int, in_ptr: int, out_ptr: int, n: int, scale: float, stream: int) -> None:
    _check(lib().etx_quantize(precision, C.c_void_p(in_ptr), C.c_void_p(out_ptr), n, scale, C.c_void_p(stream)),
           "etx_quantize")


def etx_prefilter_set(ctx, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().etx_prefilter_set(ctx, p.ctypes.data_as(C.c_void_p), p.size), "etx_prefilter_set")


def etx_prefilter_config(ctx, enabled: int, tau: float) -> None:
    _check(lib().etx_prefilter_config(ctx, enabled, tau), "etx_prefilter_config")


def etx_run_noalloc(ctx, hits, out, stream) -> None:
    _check(lib().etx_run_noalloc(ctx, C.byref(hits), C.byref(out), C.c_void_p(stream)), "etx_run_noalloc")


ETX_SCRATCH_BYTES = 128 << 20


def etx_train_begin(ctx) -> None:
    _check(lib().etx_train_begin(ctx), "etx_train_begin")


def etx_train_params(ctx, host: Optional[np.ndarray] = None, n: Optional[int] = None) -> np.ndarray:
    """The training state (params, Adam m, Adam v in blob payload order): read the
    first n floats, or replace them with ``host``."""
    if host is not None:
        h = np.ascontiguousarray(host, np.float32)
        _check(lib().etx_train_params(ctx, h.ctypes.data_as(C.c_void_p), h.size, 1), "etx_train_params")
        return h
    out = np.zeros(int(n), np.float32)
    _check(lib().etx_train_params(ctx, out.ctypes.data_as(C.c_void_p), out.size, 0), "etx_train_params")
    return out


def etx_train_apply(ctx) -> None:
    _check(lib().etx_train_apply(ctx), "etx_train_apply")


def etx_train_workspace_size(ctx, n_events: int, n_hits: int, edge_capacity: int) -> int:
    b = C.c_size_t()
    _check(lib().etx_train_workspace_size(ctx, n_events, n_hits, edge_capacity, C.byref(b)),
           "etx_train_workspace_size")
    return b.value


def etx_train_view(ctx, n_events: int, n_hits: int, edge_capacity: int, which: int):
    off, nb = C.c_size_t(), C.c_size_t()
    _check(lib().etx_train_view(ctx, n_events, n_hits, edge_capacity, which, C.byref(off), C.byref(nb)),
           "etx_train_view")
    return off.value, nb.value


def etx_prefilter_band(ctx, lo: float, hi: float) -> None:
    _check(lib().etx_prefilter_band(ctx, lo, hi), "etx_prefilter_band")


def etx_prefilter_get(ctx) -> np.ndarray:
    p = np.zeros(ETX_PF_NPARAM, np.float32)
    _check(lib().etx_prefilter_get(ctx, p.ctypes.data_as(C.c_void_p), p.size), "etx_prefilter_get")
    return p


def etx_save(ctx) -> bytes:
    """Checkpoint of a context (configuration, weights, scales, prefilter state, options)."""
    n = C.c_size_t()
    _check(lib().etx_save(ctx, None, C.byref(n)), "etx_save")
    buf = C.create_string_buffer(n.value)
    _check(lib().etx_save(ctx, buf, C.byref(n)), "etx_save")
    return buf.raw[:n.value]


def etx_load(data: bytes, device: int = 0):
    """A new context from an etx_save checkpoint."""
    ctx = C.c_void_p()
    buf = C.create_string_buffer(bytes(data), len(data))
    _check(lib().etx_load(buf, len(data), device, C.byref(ctx)), "etx_load")
    return ctx


def etx_prefilter_state(ctx, state: Optional[np.ndarray] = None) -> np.ndarray:
    if state is None:
        s = np.zeros(3 * ETX_PF_NPARAM, np.float32)
        _check(lib().etx_prefilter_state(ctx, s.ctypes.data_as(C.c_void_p), s.size, 0), "etx_prefilter_state")
        return s
    s = np.ascontiguousarray(state, dtype=np.float32)
    _check(lib().etx_prefilter_state(ctx, s.ctypes.data_as(C.c_void_p), s.size, 1), "etx_prefilter_state")
    return s


def etx_prefilter_train_step(ctx, hits, out, labels_ptr: int, lr: float, pos_weight: float, step: int,
                             loss_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _check(lib().etx_prefilter_train_step(ctx, C.byref(hits), C.byref(out), C.c_void_p(labels_ptr), lr, pos_weight,
                                          step, C.c_void_p(loss_ptr), C.c_void_p(ws_ptr), ws_bytes,
                                          C.c_void_p(stream)), "etx_prefilter_train_step")


def etx_triplet_set(ctx, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().etx_triplet_set(ctx, p.ctypes.data_as(C.c_void_p), p.size), "etx_triplet_set")


def etx_triplet_get(ctx, n: int) -> np.ndarray:
    p = np.zeros(n, np.float32)
    _check(lib().etx_triplet_get(ctx, p.ctypes.data_as(C.c_void_p), n), "etx_triplet_get")
    return p


def etx_tracks_workspace_size(ctx, n_events: int, n_hits: int, edge_capacity: int, triplet_capacity: int,
                              track_capacity: int) -> int:
    b = C.c_size_t()
    _check(lib().etx_tracks_workspace_size(ctx, n_events, n_hits, edge_capacity, triplet_capacity, track_capacity,
                                           C.byref(b)), "etx_tracks_workspace_size")
    return b.value


def etx_run_tracks(ctx, hits, out, tracks, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _check(lib().etx_run_tracks(ctx, C.byref(hits), C.byref(out), C.byref(tracks), C.c_void_p(ws_ptr), ws_bytes,
                                C.c_void_p(stream)), "etx_run_tracks")


def etx_train_triplet_workspace_size(ctx, n_events: int, n_hits: int, edge_capacity: int,
                                     triplet_capacity: int) -> int:
    b = C.c_size_t()
    _check(lib().etx_train_triplet_workspace_size(ctx, n_events, n_hits, edge_capacity, triplet_capacity,
                                                  C.byref(b)), "etx_train_triplet_workspace_size")
    return b.value


def etx_train_triplet_view(ctx, n_events: int, n_hits: int, edge_capacity: int, triplet_capacity: int, which: int):
    off, nb = C.c_size_t(), C.c_size_t()
    _check(lib().etx_train_triplet_view(ctx, n_events, n_hits, edge_capacity, triplet_capacity, which,
                                        C.byref(off), C.byref(nb)), "etx_train_triplet_view")
    return off.value, nb.value


def etx_train_triplet_params(ctx, host: Optional[np.ndarray] = None, n: Optional[int] = None) -> np.ndarray:
    """The triplet classifiers' training state (params, Adam m, Adam v): read the first n floats, or replace
    them with ``host``."""
    if host is not None:
        h = np.ascontiguousarray(host, np.float32)
        _check(lib().etx_train_triplet_params(ctx, h.ctypes.data_as(C.c_void_p), h.size, 1),
               "etx_train_triplet_params")
        return h
    out = np.zeros(int(n), np.float32)
    _check(lib().etx_train_triplet_params(ctx, out.ctypes.data_as(C.c_void_p), out.size, 0),
           "etx_train_triplet_params")
    return out


def unpack_triplets(p: np.ndarray, H: int) -> Dict:
    """Inverse of pack_triplets."""
    out, o = {}, 0
    for h in ("art", "elb"):
        out[h] = []
        for K, M in [(2 * H, H), (H, H), (H, 1)]:
            W = np.asarray(p[o:o + K * M], np.float32).reshape(K, M).copy()
            o += K * M
            b = np.asarray(p[o:o + M], np.float32).copy()
            o += M
            out[h].append((W, b))
    return out


def pack_triplets(heads: Dict) -> np.ndarray:
    """The triplet classifiers' parameters in the etx.h order (articulation head, then elbow head; each
    W1[2H][H] b1 W2[H][H] b2 W3[H][1] b3)."""
    parts = []
    for h in ("art", "elb"):
        for W, b in heads[h]:
            parts.append(np.ascontiguousarray(W, np.float32).ravel())
            parts.append(np.ascontiguousarray(b, np.float32).ravel())
    return np.concatenate(parts)


def etx_stage_name(stage: int) -> str:
    return lib().etx_stage_name(stage).decode()


def etx_profile_read(ctx) -> Dict[str, tuple]:
    ms = np.zeros(N_STAGES, np.float64)
    n = np.zeros(N_STAGES, np.int64)
    _check(lib().etx_profile_read(ctx, N_STAGES, ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)),
           "etx_profile_read")
    return {etx_stage_name(i): (float(ms[i]), int(n[i])) for i in range(N_STAGES)}


def etx_profile_reset(ctx) -> None:
    _check(lib().etx_profile_reset(ctx), "etx_profile_reset")


# ---------------------------------------------------------------------------
# configuration and weight blob
# ---------------------------------------------------------------------------

def make_config(w, precision: int = ETX_FP32, prefilter: int = 0, prefilter_tau: float = 0.0) -> etx_config:
    return etx_config(w.n_planes, w.r_scale, w.z_scale, w.emb_hidden, w.emb_layers, w.emb_dim, w.radius, w.k_max,
                      w.plane_window, w.gnn_hidden, w.gnn_steps, w.threshold, precision, prefilter, prefilter_tau)


def pack_weights(w, weights: Dict) -> bytes:
    """The etx.h weight blob: header then float32 layers in the documented order."""
    hdr = np.array([0x57585445, 1, 3, w.emb_hidden, w.emb_layers, w.emb_dim, w.gnn_hidden, w.gnn_steps], np.int32)
    order = ["emb", "node_enc", "edge_enc"]
    for k in range(w.gnn_steps):
        order += [f"node{k}", f"edge{k}"]
    order.append("cls")
    parts = [hdr.tobytes()]
    for net in order:
        for W, b in weights[net]:
            parts.append(np.ascontiguousarray(W, np.float32).tobytes())
            parts.append(np.ascontiguousarray(b, np.float32).tobytes())
    return b"".join(parts)


# ---------------------------------------------------------------------------
# torch-owned buffers around one context
# ---------------------------------------------------------------------------

@dataclass
class Batch:
    n_events: int
    n_hits: int
    hit_off: "object"
    x: "object"
    y: "object"
    z: "object"
    plane: "object"


def to_device(batch: Dict[str, np.ndarray], device="cuda") -> Batch:
    import torch
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
    return Batch(len(batch["hit_off"]) - 1, int(batch["hit_off"][-1]), t(batch["hit_off"], torch.int64),
                 t(batch["x"], torch.float32), t(batch["y"], torch.float32), t(batch["z"], torch.float32),
                 t(batch["plane"], torch.int32))


class Pipeline:
    """One context plus torch-allocated outputs and workspace for a batch shape."""

    def __init__(self, w, weights: Dict, device: int = 0, precision: int = ETX_FP32, prefilter: int = 0,
                 prefilter_tau: float = 0.0):
        self.w = w
        self.cfg = make_config(w, precision, prefilter, prefilter_tau)
        self.ctx = etx_create(self.cfg, pack_weights(w, weights), device)
        self.device = device
        self._shape = None

    def close(self):
        if self.ctx:
            etx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hits_struct(self, b: Batch) -> etx_hits:
        return etx_hits(b.n_events, b.n_hits, b.hit_off.data_ptr(), b.x.data_ptr(), b.y.data_ptr(), b.z.data_ptr(),
                        b.plane.data_ptr())

    def allocate(self, b: Batch, edge_capacity: Optional[int] = None, tri_caps: Optional[tuple] = None):
        """Outputs and workspace for batch ``b``; ``tri_caps`` = (triplets, tracks) sizes the workspace for
        etx_run_tracks as well (its first part is the etx_run workspace, so the views stay valid)."""
        import torch
        cap = b.n_hits * self.w.k_max if edge_capacity is None else edge_capacity
        shape = (b.n_events, b.n_hits, cap, tri_caps)
        if self._shape != shape:
            dev = torch.device("cuda", self.device)
            self.src = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            self.dst = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            self.score = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
            self.edge_off = torch.empty(b.n_events + 1, dtype=torch.int64, device=dev)
            self.labels = torch.empty(max(b.n_hits, 1), dtype=torch.int32, device=dev)
            self.status = torch.zeros(2, dtype=torch.int64, device=dev)
            nbytes = etx_workspace_size(self.ctx, b.n_events, b.n_hits, cap) if tri_caps is None else \
                etx_tracks_workspace_size(self.ctx, b.n_events, b.n_hits, cap, tri_caps[0], tri_caps[1])
            self.ws = None
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
            self.ws_bytes = nbytes
            self.cap = cap
            self._shape = shape
        return etx_out(self.cap, self.src.data_ptr(), self.dst.data_ptr(), self.score.data_ptr(),
                       self.edge_off.data_ptr(), self.labels.data_ptr(), self.status.data_ptr())

    def calibrate(self, b: Batch, stream=None):
        """Static calibration of the per-tensor scales on batch ``b`` (etx_calibrate)."""
        import torch
        out = self.allocate(b)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        etx_calibrate(self.ctx, self.hits_struct(b), out, self.ws_ptr, self.ws_bytes, s.cuda_stream)

    def prefilter_train_step(self, b: Batch, labels, lr: float, pos_weight: float, step: int, stream=None):
        """One on-device training step of the prefilter on the candidate edges
        of ``b`` (labels: uint8 device tensor in candidate order); returns the
        device loss tensor."""
        import torch
        out = self.allocate(b)
        if not hasattr(self, "_loss"):
            self._loss = torch.zeros(1, dtype=torch.float32, device=torch.device("cuda", self.device))
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        etx_prefilter_train_step(self.ctx, self.hits_struct(b), out, labels.data_ptr(), lr, pos_weight, step,
                                 self._loss.data_ptr(), self.ws_ptr, self.ws_bytes, s.cuda_stream)
        return self._loss

    def run(self, b: Batch, edge_capacity: Optional[int] = None, stream=None):
        import torch
        out = self.allocate(b, edge_capacity)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        etx_run(self.ctx, self.hits_struct(b), out, self.ws_ptr, self.ws_bytes, s.cuda_stream)
        return out

    def view(self, b: Batch, which: int, dtype, shape=None):
        """A tensor over one internal workspace buffer (etx_workspace_view)."""
        import torch
        off, nbytes = etx_workspace_view(self.ctx, b.n_events, b.n_hits, self.cap, which)
        base = self.ws_ptr - self.ws.data_ptr()
        t = self.ws[base + off: base + off + nbytes].view(dtype)
        return t if shape is None else t.reshape(shape)

    def results(self, b: Batch) -> Dict[str, np.ndarray]:
        """Synchronise and copy the outputs of the last run to the host."""
        import torch
        torch.cuda.synchronize(self.device)
        st = self.status.cpu().numpy()
        if st[0] != ETX_OK:
            raise EtxError(int(st[0]), f"device status (edges needed {int(st[1])})")
        eo = self.edge_off.cpu().numpy()
        E = int(eo[-1])
        return dict(edge_off=eo, src=self.src[:E].cpu().numpy(), dst=self.dst[:E].cpu().numpy(),
                    score=self.score[:E].cpu().numpy(), labels=self.labels[:b.n_hits].cpu().numpy())

    # ---- triplet stage ----------------------------------------------------

    def set_triplets(self, heads: Dict) -> None:
        etx_triplet_set(self.ctx, pack_triplets(heads))

    def allocate_tracks(self, b: Batch, triplet_capacity: int, track_capacity: int, hit_capacity: int):
        import torch
        caps = (triplet_capacity, track_capacity, hit_capacity, b.n_events)
        if getattr(self, "_trk_shape", None) != caps:
            dev = torch.device("cuda", self.device)
            T = max(triplet_capacity, 1)
            self.tri_a = torch.empty(T, dtype=torch.int32, device=dev)
            self.tri_b = torch.empty(T, dtype=torch.int32, device=dev)
            self.tri_score = torch.empty(T, dtype=torch.float32, device=dev)
            self.tri_kind = torch.empty(T, dtype=torch.uint8, device=dev)
            self.art_off = torch.empty(b.n_events + 1, dtype=torch.int64, device=dev)
            self.elb_off = torch.empty(b.n_events + 1, dtype=torch.int64, device=dev)
            self.event_track_off = torch.empty(b.n_events + 1, dtype=torch.int64, device=dev)
            self.track_off = torch.empty(track_capacity + 1, dtype=torch.int64, device=dev)
            self.track_hits = torch.empty(max(hit_capacity, 1), dtype=torch.int32, device=dev)
            self.tstatus = torch.zeros(4, dtype=torch.int64, device=dev)
            self._trk_shape = caps
        return etx_tracks(triplet_capacity, self.tri_a.data_ptr(), self.tri_b.data_ptr(), self.tri_score.data_ptr(),
                          self.tri_kind.data_ptr(), self.art_off.data_ptr(), self.elb_off.data_ptr(), track_capacity,
                          self.event_track_off.data_ptr(), self.track_off.data_ptr(), hit_capacity,
                          self.track_hits.data_ptr(), self.tstatus.data_ptr())

    def run_tracks(self, b: Batch, triplet_capacity: Optional[int] = None, track_capacity: Optional[int] = None,
                   hit_capacity: Optional[int] = None, edge_capacity: Optional[int] = None, stream=None):
        """etx_run_tracks on ``b`` (default capacities: 4 triplets, 1 track, 4 track hits per hit)."""
        import torch
        tc = 4 * b.n_hits + 1024 if triplet_capacity is None else triplet_capacity
        kc = b.n_hits + 1024 if track_capacity is None else track_capacity
        hc = 4 * b.n_hits + 1024 if hit_capacity is None else hit_capacity
        out = self.allocate(b, edge_capacity, tri_caps=(tc, kc))
        tr = self.allocate_tracks(b, tc, kc, hc)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        etx_run_tracks(self.ctx, self.hits_struct(b), out, tr, self.ws_ptr, self.ws_bytes, s.cuda_stream)
        return out, tr

    def track_status(self) -> np.ndarray:
        import torch
        torch.cuda.synchronize(self.device)
        return self.tstatus.cpu().numpy()

    def run_tracks_sized(self, b: Batch, stream=None, **caps):
        """run_tracks, run again with the capacities the device asked for while one was too small."""
        self.run_tracks(b, stream=stream, **caps)
        for _ in range(3):
            st = self.track_status()
            if st[0] != ETX_ERR_CAPACITY:
                break
            tc, kc, hc = self._trk_shape[:3]
            caps = dict(triplet_capacity=max(tc, int(st[1])), track_capacity=max(kc, int(st[2])),
                        hit_capacity=max(hc, int(st[3])), edge_capacity=caps.get("edge_capacity"))
            self.run_tracks(b, stream=stream, **caps)

    def track_results(self, b: Batch) -> Dict[str, object]:
        """Synchronise; the triplets and tracks of the last etx_run_tracks (tracks per event as hit arrays)."""
        import torch
        torch.cuda.synchronize(self.device)
        st = self.tstatus.cpu().numpy()
        if st[0] != ETX_OK:
            raise EtxError(int(st[0]), f"triplet stage status (needed: triplets {int(st[1])}, tracks {int(st[2])}, "
                                       f"hits {int(st[3])})")
        ao = self.art_off.cpu().numpy()
        eo = self.elb_off.cpu().numpy()
        T = int(eo[-1])
        eto = self.event_track_off.cpu().numpy()
        nt = int(eto[-1])
        to = self.track_off[:nt + 1].cpu().numpy()
        hits = self.track_hits[:int(to[-1]) if nt else 0].cpu().numpy()
        return dict(art_off=ao, elb_off=eo, tri_a=self.tri_a[:T].cpu().numpy(), tri_b=self.tri_b[:T].cpu().numpy(),
                    tri_score=self.tri_score[:T].cpu().numpy(), tri_kind=self.tri_kind[:T].cpu().numpy(),
                    event_track_off=eto, track_off=to, track_hits=hits,
                    tracks=[hits[to[k]:to[k + 1]] for k in range(nt)])
