"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and rejects bad configurations and weight blobs on the host
before touching the device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2508_07423_amd import etx, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etx.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:etx_status|const char\*)\s+(etx_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", etx.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = set(re.findall(r" T (etx_\w+)$", out, re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = etx.lib()
    for n in names:
        assert getattr(L, n) is not None
    assert set(etx.EXPORTED) <= set(names)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_weight_blob_size_matches_packer(name):
    w = synth.WORKLOADS[name]
    cfg = etx.make_config(w)
    assert etx.etx_weight_blob_size(cfg) == len(etx.pack_weights(w, synth.xavier_weights(w)))


@pytest.mark.parametrize("field,value,code", [
    ("n_planes", 0, etx.ETX_ERR_INVALID_ARG), ("n_planes", 65, etx.ETX_ERR_INVALID_ARG),
    ("r_scale_mm", 0.0, etx.ETX_ERR_INVALID_ARG), ("emb_hidden", 96, etx.ETX_ERR_UNSUPPORTED),
    ("emb_dim", 17, etx.ETX_ERR_UNSUPPORTED), ("k_max", 65, etx.ETX_ERR_UNSUPPORTED),
    ("k_max", 0, etx.ETX_ERR_UNSUPPORTED), ("gnn_hidden", 48, etx.ETX_ERR_UNSUPPORTED),
    ("gnn_steps", 0, etx.ETX_ERR_UNSUPPORTED), ("radius", float("nan"), etx.ETX_ERR_INVALID_ARG),
    ("precision", 4, etx.ETX_ERR_INVALID_ARG), ("plane_window", 5, etx.ETX_ERR_UNSUPPORTED)])
def test_bad_config_rejected_on_host(field, value, code):
    w = synth.C1
    cfg = etx.make_config(w)
    setattr(cfg, field, value)
    blob = etx.pack_weights(w, synth.xavier_weights(w))
    with pytest.raises(etx.EtxError) as e:
        etx.etx_create(cfg, blob)
    assert e.value.code == code


def test_bad_blob_rejected_on_host():
    w = synth.C1
    cfg = etx.make_config(w)
    W = synth.xavier_weights(w)
    blob = bytearray(etx.pack_weights(w, W))
    for bad in (bytes(blob[:-4]), bytes(blob) + b"\0\0\0\0", b"XXXX" + bytes(blob[4:])):
        with pytest.raises(etx.EtxError) as e:
            etx.etx_create(cfg, bad)
        assert e.value.code == etx.ETX_ERR_WEIGHTS
    nan = bytearray(blob)
    nan[40:44] = np.array([np.nan], np.float32).tobytes()
    with pytest.raises(etx.EtxError) as e:
        etx.etx_create(cfg, bytes(nan))
    assert e.value.code == etx.ETX_ERR_WEIGHTS


def test_status_strings_and_null_handles():
    for code in range(7):
        assert etx.etx_status_str(code)
    assert etx.etx_status_str(99) == "unknown status"
    L = etx.lib()
    n = C.c_size_t()
    assert L.etx_workspace_size(None, 1, 1, 1, C.byref(n)) == etx.ETX_ERR_INVALID_ARG
    assert L.etx_run(None, None, None, None, 0, None) == etx.ETX_ERR_INVALID_ARG
    assert L.etx_destroy(None) == etx.ETX_ERR_INVALID_ARG
    assert etx.etx_stage_name(0) == "init" and etx.etx_stage_name(999) == ""


def test_checkpoint_load_rejects_foreign_buffers_on_host():
    """etx_load validates the checkpoint header before touching a device."""
    L = etx.lib()
    ctx = C.c_void_p()
    for bad in (b"", b"ETXS", b"\0" * 64, b"XXXX" + b"\0" * 200):
        buf = C.create_string_buffer(bad, max(len(bad), 1))
        assert L.etx_load(buf, len(bad), 0, C.byref(ctx)) == etx.ETX_ERR_INVALID_ARG
    n = C.c_size_t()
    assert L.etx_save(None, None, C.byref(n)) == etx.ETX_ERR_INVALID_ARG
    assert L.etx_load(None, 0, 0, C.byref(ctx)) == etx.ETX_ERR_INVALID_ARG


def test_binding_constants_match_the_header():
    """Every enumerator of the header (statuses, precisions, options, views,
    stages) exists in the binding with the same value, and so do the numeric
    macros the binding mirrors."""
    src = open(HEADER).read()
    enums = re.findall(r"^\s*(ETX_[A-Z0-9_]+)\s*=\s*(-?\d+)", src, re.M)
    assert len(enums) > 40
    for name, value in enums:
        assert getattr(etx, name, None) == int(value), name
    for name, expr in re.findall(r"^#define\s+(ETX_[A-Z0-9_]+)\s+(\(?[0-9u <()*+-]+\)?)\s*$", src, re.M):
        if hasattr(etx, name):
            assert getattr(etx, name) == eval(expr.replace("u", "")), name
    body = re.search(r"#define\s+ETX_TRIPLET_NPARAM\(H\)\s+(.+)", src).group(1)
    for h in (32, 64):
        assert etx.ETX_TRIPLET_NPARAM(h) == eval(body.replace("(H)", f"({h})")), h
