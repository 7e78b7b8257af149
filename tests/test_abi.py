"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, agrees with the binding's constants, and rejects
bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1112_0059_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lnbnn.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lnbnn_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    names = _declared()
    assert "lnbnn_classify" in names and "lnbnn_build_index" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_constants_match_header():
    src = open(HEADER).read()
    for name in ["LNBNN_OK", "LNBNN_EINVAL", "LNBNN_ENOMEM", "LNBNN_EDEVICE", "LNBNN_EAGAIN",
                 "LNBNN_ENOENT", "LNBNN_EBUSY", "LNBNN_U8", "LNBNN_F32", "LNBNN_EXACT_F16",
                 "LNBNN_EXACT_BF16", "LNBNN_FP8_RERANK", "LNBNN_EXACT_I8", "LNBNN_DEVICE_PTRS",
                 "LNBNN_PER_IMAGE_LAUNCH", "LNBNN_NO_GRAPH", "LNBNN_TIMING"]:
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", src)
        assert m, name
        assert int(m.group(1)) == getattr(L, name), name
    assert f"#define LNBNN_DIM {L.LNBNN_DIM}" in src
    assert f"#define LNBNN_DIM_LOC {L.LNBNN_DIM_LOC}" in src
    assert f"#define LNBNN_MAX_K {L.LNBNN_MAX_K}" in src


def test_struct_layouts():
    assert ctypes.sizeof(L.lnbnn_timing) == 8 + 8 + 4 * 3 + 4   # padded to 8
    assert ctypes.sizeof(L.lnbnn_req_stats) == 5 * 8 + 2 * 4


def _err(fn, *a, **kw):
    with pytest.raises(L.LnbnnError) as e:
        fn(*a, **kw)
    return e.value.code


def test_build_index_rejects_bad_arguments():
    R = np.zeros((64, 128), np.uint8)
    lab = np.zeros(64, np.int32)
    bit = L.LNBNN_MODE_BIT
    assert _err(L.lnbnn_build_index, R, lab, 0, bit(0)) == L.LNBNN_EINVAL          # no class
    assert _err(L.lnbnn_build_index, R, lab, 2, 0) == L.LNBNN_EINVAL               # no mode
    assert _err(L.lnbnn_build_index, R, lab, 2, bit(L.LNBNN_FP8_RERANK)) == L.LNBNN_EINVAL
    assert _err(L.lnbnn_build_index, R, lab + 2, 2, bit(0)) == L.LNBNN_EINVAL      # label range
    assert _err(L.lnbnn_build_index, R, lab - 1, 2, bit(0)) == L.LNBNN_EINVAL
    assert _err(L.lnbnn_build_index, np.zeros((64, 64), np.uint8), lab, 2, bit(0)) == L.LNBNN_EINVAL
    assert "label" in L.lnbnn_last_error() or "dim" in L.lnbnn_last_error()
    lib = L.load()
    out = ctypes.c_void_p()
    rc = lib.lnbnn_build_index(None, 0, 64, 128, None, 2, 1, 0, 0, None, ctypes.byref(out))
    assert rc == L.LNBNN_EINVAL
    rc = lib.lnbnn_build_index(R.ctypes.data, 0, 0, 128, lab.ctypes.data, 2, 1, 0, 0, None,
                               ctypes.byref(out))
    assert rc == L.LNBNN_EINVAL


def test_null_index_is_rejected():
    lib = L.load()
    off = np.array([0, 1], np.int64)
    cls = np.zeros(1, np.int32)
    assert lib.lnbnn_classify(None, None, 0, off.ctypes.data, 1, 10, 0, 0, cls.ctypes.data,
                              None, None, None, None) == L.LNBNN_EINVAL
    assert lib.lnbnn_index_free(None) == L.LNBNN_OK
    assert lib.lnbnn_index_info(None, None, None, None, None) == L.LNBNN_EINVAL
    assert lib.lnbnn_last_timing(None, None) == L.LNBNN_EINVAL


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="checks the no-device error path")
def test_no_device_is_a_device_error():
    R = np.zeros((64, 128), np.uint8)
    lab = np.zeros(64, np.int32)
    assert _err(L.lnbnn_build_index, R, lab, 2, 1) == L.LNBNN_EDEVICE


def test_variants_listed():
    n = L.lnbnn_num_variants()
    assert n >= 4
    names = [L.lnbnn_variant_name(v) for v in range(n)]
    assert len(set(names)) == n and "?" not in names
    assert L.lnbnn_variant_name(n) == "?"


def test_tuning_cache_entries_decode():
    """Every committed tuning-cache value decodes to a built variant and a
    chunk length the kernel accepts (a multiple of 8 tiles, 0 = whole
    slice); 160-byte rows use a 5 KB-tile stage shape."""
    import json
    with open(os.path.join(ROOT, "paper_1112_0059_amd", "tuning_cache.json")) as f:
        cache = json.load(f)
    assert cache
    n = L.lnbnn_num_variants()
    loc_shapes = {"w4_nt2_mt4_nb2", "w4_nt2_mt4_nb3", "w8_nt2_mt8_nb3", "w8_nt1_mt8_nb3", "pl_w8_nt2_mt8_nb3"}
    for key, val in cache.items():
        fields = dict(kv.split("=") for kv in key.split(","))
        assert set(fields) == {"arch", "n_refs", "dim", "kp", "mode"}, key
        v, chunk = val & 0xFF, val >> 8
        assert 0 <= v < n and chunk >= 0 and chunk % 8 == 0, key
        if fields["dim"] == str(L.LNBNN_DIM_LOC):
            assert fields["mode"] == str(L.LNBNN_EXACT_I8) and L.lnbnn_variant_name(v) in loc_shapes, key


def test_query_width_checked_before_any_call():
    """The binding rejects queries whose width is not the index's before it
    calls into the library (no device needed)."""
    ix = L.Index(None, 100, 3, 0, L.LNBNN_DIM_LOC)
    off = np.array([0, 3], np.int64)
    with pytest.raises(L.LnbnnError):
        L.lnbnn_classify(ix, np.zeros((3, 128), np.uint8), off, 5, L.LNBNN_EXACT_I8)
    with pytest.raises(L.LnbnnError):
        L.lnbnn_submit(ix, np.zeros((3, 128), np.uint8), 5, L.LNBNN_EXACT_I8)
    ix.handle = None


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
