"""The C-ABI library loads, exports every entry point include/latentam.h
declares, and rejects invalid arguments on the host before any GPU work
(these calls never reach the HIP runtime, so they run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2602_12314_amd import _lib, scenes

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "latentam.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lam_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblatentam.so not built")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version(L):
    assert L.lam_version() == 2
    for code in (0, -1, -2, -3, -4):
        assert _lib.status_string(code)


def _ws_size(n, d, cams, tw=16, th=16, cap=1000):
    out = C.c_uint64()
    cams = np.ascontiguousarray(cams, np.float32)
    st = _lib.lib().lam_render_workspace_size(None, n, d, cams.ctypes.data_as(C.c_void_p), cams.shape[0],
                                              tw, th, cap, C.byref(out))
    return st, out.value


def test_render_workspace_validation(L):
    cams = np.stack([scenes.pinhole(640, 480, 525.0).packed()])
    st, nbytes = _ws_size(1000, 16, cams)
    assert st == 0 and nbytes > 1000 * 80
    assert _ws_size(1000, 8, cams)[0] == _lib.LAM_ERR_UNSUPPORTED          # d
    assert _ws_size(1000, 16, cams, 16, 32)[0] == _lib.LAM_ERR_UNSUPPORTED  # 512-pixel tiles
    assert _ws_size(1000, 16, cams, 12, 12)[0] == _lib.LAM_ERR_UNSUPPORTED  # not powers of two
    assert _ws_size(-1, 16, cams)[0] == _lib.LAM_ERR_INVALID_ARG
    bad = cams.copy()
    bad[0, 0] = 0
    assert _ws_size(10, 16, bad)[0] == _lib.LAM_ERR_INVALID_ARG
    bad = cams.copy()
    bad[0, 2] = np.nan
    assert _ws_size(10, 16, bad)[0] == _lib.LAM_ERR_INVALID_ARG
    many = np.repeat(cams, 17, axis=0)
    assert _ws_size(10, 16, many)[0] == _lib.LAM_ERR_UNSUPPORTED
    # workspace grows with the capacity, 16 bytes per pair (two key/value buffers)
    a, b = _ws_size(1000, 16, cams, cap=0)[1], _ws_size(1000, 16, cams, cap=1 << 20)[1]
    assert b - a >= 16 * (1 << 20)


def test_render_forward_rejects_null_inputs(L):
    cams = np.ascontiguousarray(np.stack([scenes.pinhole(64, 48, 50.0).packed()]), np.float32)
    st = L.lam_render_forward(None, None, None, None, None, None, 10, 16, cams.ctypes.data_as(C.c_void_p), 1,
                              16, 16, None, None, None, 0, 0, None)
    assert st == _lib.LAM_ERR_INVALID_ARG


def test_decode_workspace_validation(L):
    ok = C.c_uint64()
    assert L.lam_decode_workspace_size(None, 1, 1000, 16, 256, 512, C.byref(ok)) == 0 and ok.value > 0
    assert L.lam_decode_workspace_size(None, 0, 1000, 16, 256, 512, C.byref(ok)) == 0
    for args in [(1, 1000, 8, 256, 512), (1, 1000, 16, 0, 512), (1, 1000, 16, 256, 100),
                 (1, 1000, 16, 256, 2048), (1, 1000, 16, 4096, 512), (7, 10, 16, 64, 128)]:
        assert L.lam_decode_workspace_size(None, *args, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED, args
    assert L.lam_decode_workspace_size(None, 1, -1, 16, 64, 128, C.byref(ok)) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_decode_workspace_size(None, 1, 10, 16, 64, 128, None) == _lib.LAM_ERR_INVALID_ARG


def test_context_options_are_validated_before_the_device(L):
    # lam_create parses its options before it touches the device, so a bad
    # option is INVALID_ARG with or without a GPU; NULL out is rejected
    out = C.c_void_p()
    for bad in (b'{"raster_schedule": 3}', b'{"decode_shape": -1}', b'{"decode_splits": 12}',
                b'{"decode_splits": 8192}', b'{"tile": 16}', b'{"decode_shape": 1.5}', b'[1]',
                b'{"decode_shape": 1', b'{"decode_shape": 1} x', b'{decode_shape: 1}'):
        assert L.lam_create(0, bad, C.byref(out)) == _lib.LAM_ERR_INVALID_ARG, bad
        assert not out.value
    assert L.lam_create(0, None, None) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_create(-1, b'{}', C.byref(out)) in (_lib.LAM_ERR_INVALID_ARG, _lib.LAM_ERR_HIP)
    L.lam_destroy(None)  # a no-op
    v = C.c_int()
    assert L.lam_ctx_get(None, b"decode_shape", C.byref(v)) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_ctx_configure(None, b"{}") == _lib.LAM_ERR_INVALID_ARG


def test_launching_calls_need_a_context(L):
    # the host-only size queries take NULL (the default options); calls that
    # launch work reject it before touching the device
    p = C.c_void_p(256)
    big = C.c_uint64(1 << 40)
    assert L.lam_decode_forward(None, 1, p, 10, 16, p, p, 64, 128, p, p, big, None) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_render_counters(None, p, None, C.byref(C.c_uint64()), C.byref(C.c_int())) == \
        _lib.LAM_ERR_INVALID_ARG
    assert L.lam_profile_enable(None, 1) == _lib.LAM_ERR_INVALID_ARG


def test_decode_lds_limit_of_fp32(L):
    # the FP32 per-pixel kernel holds 32 rows of max(atoms, D) + 8 FP32 values in LDS
    ok = C.c_uint64()
    assert L.lam_decode_workspace_size(None, 0, 100, 16, 1024, 1024, C.byref(ok)) == 0
    assert L.lam_decode_workspace_size(None, 0, 100, 16, 2048, 512, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED
    assert L.lam_decode_workspace_size(None, 1, 100, 16, 2048, 512, C.byref(ok)) == 0


def test_decode_rejects_small_workspace(L):
    st = L.lam_decode_loss(None, 1, C.c_void_p(16), 10, 16, C.c_void_p(16), C.c_void_p(16), 64, 128,
                           C.c_void_p(16), C.c_void_p(16), C.c_float(0.1), C.c_void_p(16), None,
                           C.c_void_p(16), C.c_void_p(16), None, C.c_void_p(16), 8, None)
    assert st == _lib.LAM_ERR_INVALID_ARG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()


def test_tied_decode_validation(L):
    ok = C.c_uint64()
    assert L.lam_decode_tied_workspace_size(None, 1, 1000, 16, 256, 512, C.byref(ok)) == 0 and ok.value > 0
    base = ok.value
    assert L.lam_decode_workspace_size(None, 1, 1000, 16, 256, 512, C.byref(ok)) == 0 and ok.value < base
    assert L.lam_decode_tied_workspace_size(None, 1, 1000, 8, 256, 512, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED
    assert L.lam_decode_tied_workspace_size(None, 0, 1000, 16, 256, 512, C.byref(ok)) == 0
    # E4M3 is not offered for the tied decode (its dQ misses the E4M3 bound)
    assert L.lam_decode_tied_workspace_size(None, 2, 1000, 16, 256, 512, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED
    assert L.lam_decode_tied_workspace_size(None, 1, -1, 16, 256, 512, C.byref(ok)) == _lib.LAM_ERR_INVALID_ARG
    bad = _lib.TiedParams(0.0, 0.5, 0.5, 0.2, 0.1)  # tau must be positive
    p = C.c_void_p(16)
    st = L.lam_decode_tied_loss(None, 1, p, 10, 16, p, p, 64, 128, p, p, C.byref(bad), p, None, p, p, p,
                                C.c_uint64(1 << 30), None)
    assert st == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_decode_tied_loss(None, 1, p, 10, 16, p, p, 64, 128, p, p, None, p, None, p, p, p,
                                  C.c_uint64(1 << 30), None) == _lib.LAM_ERR_INVALID_ARG
    good = _lib.TiedParams(0.1, 0.5, 0.5, 0.2, 0.1)
    # a launching call without a context is rejected first
    assert L.lam_decode_tied_loss(None, 1, p, 10, 16, p, p, 64, 128, p, p, C.byref(good), p, None, p, p, p,
                                  C.c_uint64(1 << 30), None) == _lib.LAM_ERR_INVALID_ARG


def test_kmeans_validation(L):
    ok = C.c_uint64()
    assert L.lam_kmeans_workspace_size(None, 1, 307200, 512, 1280, C.byref(ok)) == 0 and ok.value > 0
    assert L.lam_kmeans_workspace_size(None, 0, 100, 1024, 10, C.byref(ok)) == 0       # FP32 up to D = 1024
    assert L.lam_kmeans_workspace_size(None, 0, 100, 2048, 10, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED
    assert L.lam_kmeans_workspace_size(None, 1, 100, 2048, 10, C.byref(ok)) == 0       # BF16 up to 2048
    assert L.lam_kmeans_workspace_size(None, 1, 100, 48, 10, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED
    assert L.lam_kmeans_workspace_size(None, 2, 100, 512, 10, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED  # no FP8
    assert L.lam_kmeans_workspace_size(None, 1, 100, 512, 0, C.byref(ok)) == _lib.LAM_ERR_UNSUPPORTED
    assert L.lam_kmeans_workspace_size(None, 1, -1, 512, 10, C.byref(ok)) == _lib.LAM_ERR_INVALID_ARG
    p = C.c_void_p(256)
    big = C.c_uint64(1 << 40)
    # iters must be >= 1; misaligned rows are rejected
    assert L.lam_kmeans_lloyd(None, 1, p, None, 10, 64, p, 4, 0, p, None, None, p, big, None) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_kmeans_assign(None, 1, C.c_void_p(260), 10, 64, p, 4, p, None, p, big, None) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_kmeans_assign(None, 1, p, 10, 64, p, 4, p, None, p, C.c_uint64(16), None) == _lib.LAM_ERR_INVALID_ARG
    # stream: m <= n, Kp <= K, m >= K - Kp, seeds inside [0, n)
    for n, Kp, K, m in ((10, 0, 4, 11), (10, 5, 4, 3), (10, 0, 4, 3)):
        assert L.lam_stream_kmeans_workspace_size(None, 1, n, 64, Kp, K, m, C.byref(ok)) == _lib.LAM_ERR_INVALID_ARG
    assert L.lam_stream_kmeans_workspace_size(None, 1, 10, 64, 2, 4, 3, C.byref(ok)) == 0
    seeds = np.array([0, 3, 10], dtype=np.int32)  # 10 is out of range for n = 10
    st = L.lam_stream_kmeans(None, 1, p, 10, 64, None, None, 0, 3, seeds.ctypes.data_as(C.c_void_p), 3, 2, 2, p, p, p,
                             big, None)
    assert st == _lib.LAM_ERR_INVALID_ARG
    seeds[2] = -1
    st = L.lam_stream_kmeans(None, 1, p, 10, 64, None, None, 0, 3, seeds.ctypes.data_as(C.c_void_p), 3, 2, 2, p, p, p,
                             big, None)
    assert st == _lib.LAM_ERR_INVALID_ARG
