"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2305_03284_amd as ddh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddh.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s+(ddh_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = ddh.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # the binding covers exactly the declared surface
    assert set(ddh.SIGNATURES) == set(names)


def test_error_strings_and_version():
    L = ddh.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.ddh_error_string(code)
    assert b"gfx950" in L.ddh_version()


@pytest.mark.parametrize("N", [0, 32, 100, 1024])
def test_default_params_rejects_bad_N(N):
    p = ddh.Params()
    assert ddh.lib().ddh_default_params(N, ctypes.byref(p)) == ddh.DDH_EINVAL


@pytest.mark.parametrize("field,value", [
    ("N", 96), ("pupil_diameter", 0.0), ("pupil_diameter", 1e9), ("pupil_diameter", float("nan")),
    ("lambda_", -0.1), ("lambda_", 1.5), ("alpha", 2.0), ("n_k", 0), ("sigma_w2", 0.0),
    ("sigma_w2", float("inf")), ("qg_p", 1.5), ("qg_q", 0.5), ("qg_q", 2.5), ("qg_T", 0.0),
    ("qg_sigma", -1.0), ("beta_phi", -0.5), ("r_floor", 0.0),
])
def test_init_stream_validates_before_device_work(field, value):
    p = ddh.default_params(256)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    assert ddh.lib().ddh_init_stream(ctypes.byref(p), None, None, ctypes.byref(h)) == ddh.DDH_EINVAL
    assert h.value is None


def test_null_handles_are_rejected():
    L = ddh.lib()
    y = ctypes.c_void_p(1)
    assert L.ddh_step(None, y, None) == ddh.DDH_EINVAL
    assert L.ddh_em(None, y, None) == ddh.DDH_EINVAL
    assert L.ddh_get_phase(None, y, None) == ddh.DDH_EINVAL
    assert L.ddh_destroy_stream(None) == ddh.DDH_EINVAL
    assert L.ddh_init_stream(None, None, None, None) == ddh.DDH_EINVAL
    assert L.ddh_step_batch(None, None, 1, None) == ddh.DDH_EINVAL
    assert L.ddh_step_batch(None, None, -1, None) == ddh.DDH_EINVAL
    assert L.ddh_step_batch(None, None, 0, None) == ddh.DDH_OK
    assert L.ddh_step_batch_noalloc(None, None, 1, None) == ddh.DDH_EINVAL
    assert L.ddh_step_batch_noalloc(None, None, -1, None) == ddh.DDH_EINVAL
    assert L.ddh_step_batch_noalloc(None, None, 4097, None) == ddh.DDH_EINVAL
    assert L.ddh_step_batch_noalloc(None, None, 0, None) == ddh.DDH_OK
    assert L.ddh_batch_create(None, 0, 0, None) == ddh.DDH_EINVAL
    assert L.ddh_batch_step(None, None, None) == ddh.DDH_EINVAL
    assert L.ddh_batch_destroy(None) == ddh.DDH_EINVAL
    assert L.ddh_server_destroy(None) == ddh.DDH_EINVAL
    assert L.ddh_server_step(None, None, None, 0, None) == ddh.DDH_EINVAL
    assert L.ddh_server_create(0, None) == ddh.DDH_EINVAL
    n = ctypes.c_longlong()
    assert L.ddh_frame_count(None, ctypes.byref(n)) == ddh.DDH_EINVAL


@pytest.mark.parametrize("N,count,inv", [(100, 1, 0), (256, 0, 0), (256, 1, 2)])
def test_fft2_validates(N, count, inv):
    one = ctypes.c_void_p(16)
    assert ddh.lib().ddh_fft2(N, count, one, one, one, inv, None) == ddh.DDH_EINVAL


def test_stream_bytes_without_a_device():
    D = ddh
    b = ctypes.c_ulonglong()
    sizes = []
    for N in (64, 128, 256, 512):
        assert D.lib().ddh_stream_bytes(N, ctypes.byref(b)) == 0
        # state (2 r + 2 phi), T, U and |b|^2 buffers at least, 256-byte aligned pieces
        assert b.value >= 36 * N * N and b.value % 256 == 0
        sizes.append(b.value)
    assert sizes == sorted(sizes)
    assert D.lib().ddh_stream_bytes(100, ctypes.byref(b)) == D.DDH_EINVAL
    assert D.lib().ddh_stream_bytes(64, None) == D.DDH_EINVAL
    assert D.stream_bytes(256) == sizes[2]


def test_mbir_and_gradient_calls_validate_before_device_work():
    L = ddh.lib()
    one = ctypes.c_void_p(16)
    assert L.ddh_mbir(None, one, 10, 5, None) == ddh.DDH_EINVAL
    p64 = ddh.make_params(64)
    out = ddh.GradOut()
    ys = (ctypes.c_void_p * 3)(16, 16, 16)
    # single stream: null parameters, K = 0, ckpt = 0, n_k != 1
    assert L.ddh_unrolled_grad(None, 3, ys, one, one, 2, one, ctypes.byref(out), None) == ddh.DDH_EINVAL
    assert L.ddh_unrolled_grad(ctypes.byref(p64), 0, ys, one, one, 2, one, ctypes.byref(out), None) == ddh.DDH_EINVAL
    assert L.ddh_unrolled_grad(ctypes.byref(p64), 3, ys, one, one, 0, one, ctypes.byref(out), None) == ddh.DDH_EINVAL
    p2 = ddh.make_params(64, n_k=2)
    assert L.ddh_unrolled_grad(ctypes.byref(p2), 3, ys, one, one, 2, one, ctypes.byref(out), None) == ddh.DDH_EINVAL
    nul = (ctypes.c_void_p * 3)(16, None, 16)
    assert L.ddh_unrolled_grad(ctypes.byref(p64), 3, nul, one, one, 2, one, ctypes.byref(out), None) == ddh.DDH_EINVAL
    # batch: no streams, mixed N, a null per-stream pointer
    prm = (ddh.Params * 2)(ddh.make_params(64), ddh.make_params(128))
    ptr2 = (ctypes.c_void_p * 2)(16, 16)
    ys2 = (ctypes.c_void_p * 6)(16, 16, 16, 16, 16, 16)
    outs = (ddh.GradOut * 2)()
    B = L.ddh_unrolled_grad_batch
    assert B(prm, 0, 3, ys2, ptr2, ptr2, 2, ptr2, outs, None) == ddh.DDH_EINVAL
    assert B(prm, 2, 3, ys2, ptr2, ptr2, 2, ptr2, outs, None) == ddh.DDH_EINVAL
    same = (ddh.Params * 2)(ddh.make_params(64), ddh.make_params(64))
    half = (ctypes.c_void_p * 2)(16, None)
    assert B(same, 2, 3, ys2, ptr2, half, 2, ptr2, outs, None) == ddh.DDH_EINVAL


def test_autotune_mix_validates_before_device_work():
    L = ddh.lib()
    ns = (ctypes.c_int * 3)(64, 128, 100)
    assert L.ddh_autotune_mix(None, 3, None, None) == ddh.DDH_EINVAL
    assert L.ddh_autotune_mix(ns, 0, None, None) == ddh.DDH_EINVAL
    assert L.ddh_autotune_mix(ns, 3, None, None) == ddh.DDH_EINVAL  # 100 is not a supported size


def _annulus(N, outer, inner):
    import numpy as np
    c = (N - 1) / 2.0
    ii, jj = np.mgrid[0:N, 0:N]
    d2 = (2 * ii - N + 1) ** 2 + (2 * jj - N + 1) ** 2
    return ((d2 <= outer ** 2) & (d2 > inner ** 2)).astype(np.float32)


@pytest.mark.parametrize("case", ["non_binary", "nan", "empty", "one_line"])
def test_init_stream_rejects_bad_aperture_arrays_before_device_work(case):
    """The aperture array (host memory here) is validated before any device
    work: values must be 0 or 1, at least one pixel, and not all on one line
    (the RemoveTipTilt plane would not be determined)."""
    import numpy as np
    N = 64
    a = _annulus(N, N, N // 2)
    if case == "non_binary":
        a[10, 10] = 0.5
    elif case == "nan":
        a[20, 20] = np.nan
    elif case == "empty":
        a[:] = 0
    else:
        a[:] = 0
        a[5, 3:40] = 1  # one row
    p = ddh.default_params(N)
    h = ctypes.c_void_p()
    rc = ddh.lib().ddh_init_stream(ctypes.byref(p), ctypes.c_void_p(a.ctypes.data), None, ctypes.byref(h))
    assert rc == ddh.DDH_EINVAL and h.value is None


def test_aperture_array_skips_the_diameter_check():
    """With an aperture array the diameter is not used, so a zero diameter
    does not fail validation (the call then needs a device; without one it
    stops at the first device call, not at the parameters)."""
    N = 64
    a = _annulus(N, N, N // 2)
    p = ddh.default_params(N)
    p.pupil_diameter = 0.0
    h = ctypes.c_void_p()
    rc = ddh.lib().ddh_init_stream(ctypes.byref(p), ctypes.c_void_p(a.ctypes.data), None, ctypes.byref(h))
    assert rc != ddh.DDH_EINVAL


def test_stale_handles_are_rejected_without_reading_them():
    """A pointer that the library never handed out (or has destroyed) is
    reported as a dead handle: handles are checked by membership in the
    library's set of live handles, not by reading through the pointer."""
    import numpy as np
    L = ddh.lib()
    junk = np.zeros(64, dtype=np.uint8)       # readable memory that is not a handle
    h = ctypes.c_void_p(junk.ctypes.data)
    y = ctypes.c_void_p(16)
    assert L.ddh_step(h, y, None) == ddh.DDH_ESTATE
    assert L.ddh_destroy_stream(h) == ddh.DDH_ESTATE
    assert L.ddh_batch_destroy(h) == ddh.DDH_ESTATE
    assert L.ddh_server_destroy(h) == ddh.DDH_ESTATE
    arr = (ctypes.c_void_p * 1)(junk.ctypes.data)
    ys = (ctypes.c_void_p * 1)(16)
    assert L.ddh_step_batch(arr, ys, 1, None) == ddh.DDH_ESTATE
    b = ctypes.c_void_p()
    assert L.ddh_batch_create(arr, 1, 0, ctypes.byref(b)) == ddh.DDH_ESTATE
