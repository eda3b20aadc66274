"""Dynamic DH-MBIR (arXiv 2305.03284) per-frame EM step on AMD MI355X.

Thin Python binding of the C ABI in ``include/ddh.h`` (``libddh.so``, built
in-tree by ``paper_2305_03284_amd.build``).  Only argument marshalling lives
here: every step of the path runs in the library's HIP kernels.  PyTorch is
used for device memory and streams only.  There is no fallback: if the
library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddh.so")

DDH_OK = 0
DDH_EINVAL = -1
DDH_ENOMEM = -2
DDH_EDEVICE = -3
DDH_EDATA = -4
DDH_ESTATE = -5
DDH_BATCH_GRAPH = 1
DDH_BATCH_WORKLIST = 2
DDH_BATCH_TEST_GIVEUP = 4

# every function the header declares, with its ctypes signature
_c_int, _c_void_p, _c_double, _c_ll = ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_longlong


class Params(ctypes.Structure):
    """Mirror of ``ddh_params``."""
    _fields_ = [("N", ctypes.c_int), ("pupil_diameter", ctypes.c_float), ("lambda_", ctypes.c_float),
                ("alpha", ctypes.c_float), ("n_k", ctypes.c_int), ("sigma_w2", ctypes.c_float),
                ("qg_p", ctypes.c_float), ("qg_q", ctypes.c_float), ("qg_T", ctypes.c_float),
                ("qg_sigma", ctypes.c_float), ("beta_phi", ctypes.c_float), ("r_floor", ctypes.c_float)]


class GradOut(ctypes.Structure):
    """ddh_grad_out: loss and its derivatives w.r.t. sigma_w, qg_sigma, beta_phi."""
    _fields_ = [("loss", ctypes.c_double), ("d_sigma_w", ctypes.c_double), ("d_sigma_r", ctypes.c_double),
                ("d_beta", ctypes.c_double)]


SIGNATURES = {
    "ddh_default_params": (_c_int, [_c_int, ctypes.POINTER(Params)]),
    "ddh_init_stream": (_c_int, [ctypes.POINTER(Params), _c_void_p, _c_void_p, ctypes.POINTER(_c_void_p)]),
    "ddh_destroy_stream": (_c_int, [_c_void_p]),
    "ddh_step": (_c_int, [_c_void_p, _c_void_p, _c_void_p]),
    "ddh_em": (_c_int, [_c_void_p, _c_void_p, _c_void_p]),
    "ddh_mbir": (_c_int, [_c_void_p, _c_void_p, _c_int, _c_int, _c_void_p]),
    "ddh_get_phase": (_c_int, [_c_void_p, _c_void_p, _c_void_p]),
    "ddh_get_reflectance": (_c_int, [_c_void_p, _c_void_p, _c_void_p]),
    "ddh_set_state": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_ll, _c_void_p]),
    "ddh_frame_count": (_c_int, [_c_void_p, ctypes.POINTER(_c_ll)]),
    "ddh_status": (_c_int, [_c_void_p, _c_void_p]),
    "ddh_get_params": (_c_int, [_c_void_p, ctypes.POINTER(Params)]),
    "ddh_cost": (_c_int, [_c_void_p, _c_void_p, ctypes.POINTER(_c_double), _c_void_p]),
    "ddh_strehl": (_c_int, [_c_void_p, _c_void_p, ctypes.POINTER(_c_double), _c_void_p]),
    "ddh_batch_create": (_c_int, [ctypes.POINTER(_c_void_p), _c_int, _c_int, ctypes.POINTER(_c_void_p)]),
    "ddh_batch_destroy": (_c_int, [_c_void_p]),
    "ddh_batch_step": (_c_int, [_c_void_p, ctypes.POINTER(_c_void_p), _c_void_p]),
    "ddh_batch_set_timing": (_c_int, [_c_void_p, _c_int]),
    "ddh_batch_stage_times": (_c_int, [_c_void_p, ctypes.POINTER(_c_double), ctypes.POINTER(_c_ll),
                                       ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_c_int)]),
    "ddh_server_create": (_c_int, [_c_int, ctypes.POINTER(_c_void_p)]),
    "ddh_stream_bytes": (_c_int, [_c_int, ctypes.POINTER(ctypes.c_ulonglong)]),
    "ddh_server_destroy": (_c_int, [_c_void_p]),
    "ddh_server_step": (_c_int, [_c_void_p, ctypes.POINTER(_c_void_p), ctypes.POINTER(_c_void_p), _c_int,
                                 _c_void_p]),
    "ddh_step_batch": (_c_int, [ctypes.POINTER(_c_void_p), ctypes.POINTER(_c_void_p), _c_int, _c_void_p]),
    "ddh_step_batch_noalloc": (_c_int, [ctypes.POINTER(_c_void_p), ctypes.POINTER(_c_void_p), _c_int, _c_void_p]),
    "ddh_unrolled_grad": (_c_int, [ctypes.POINTER(Params), _c_int, ctypes.POINTER(_c_void_p), _c_void_p, _c_void_p,
                                   _c_int, _c_void_p, ctypes.POINTER(GradOut), _c_void_p]),
    "ddh_unrolled_grad_batch": (_c_int, [ctypes.POINTER(Params), _c_int, _c_int, ctypes.POINTER(_c_void_p),
                                         ctypes.POINTER(_c_void_p), ctypes.POINTER(_c_void_p), _c_int,
                                         ctypes.POINTER(_c_void_p), ctypes.POINTER(GradOut), _c_void_p]),
    "ddh_fft2": (_c_int, [_c_int, _c_int, _c_void_p, _c_void_p, _c_void_p, _c_int, _c_void_p]),
    "ddh_set_tiles": (_c_int, [_c_int, ctypes.POINTER(_c_int)]),
    "ddh_get_tiles": (_c_int, [_c_int, ctypes.POINTER(_c_int)]),
    "ddh_autotune": (_c_int, [_c_int, _c_int, ctypes.POINTER(_c_int), ctypes.POINTER(_c_double)]),
    "ddh_autotune_mix": (_c_int, [ctypes.POINTER(_c_int), _c_int, ctypes.POINTER(_c_int), ctypes.POINTER(_c_double)]),
    "ddh_error_string": (ctypes.c_char_p, [_c_int]),
    "ddh_last_error_message": (ctypes.c_char_p, []),
    "ddh_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libddh.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_03284_amd.build`")
        # torch first: the library's HIP runtime dependency then resolves to
        # the runtime torch has already loaded, so the process holds one HIP
        # runtime (loaded the other way round there are two, and the second
        # to initialise finds no device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DDHError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.ddh_error_string(code).decode()
        detail = L.ddh_last_error_message().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f" [{detail}]" if detail and code == DDH_EDEVICE else ""))
        self.code = code


def _check(rc: int, where: str) -> None:
    if rc != DDH_OK:
        raise DDHError(rc, where)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def default_params(N: int) -> Params:
    p = Params()
    _check(lib().ddh_default_params(N, ctypes.byref(p)), "ddh_default_params")
    return p


def make_params(N: int, **kw) -> Params:
    """Params for grid N with keyword overrides (``lam`` for lambda)."""
    p = default_params(N)
    for k, v in kw.items():
        k = "lambda_" if k in ("lam", "lambda") else k
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _check_frame(y, N):
    torch = _torch()
    if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == torch.complex64
            and tuple(y.shape) == (N, N) and y.is_contiguous()):
        raise ValueError(f"frame must be a contiguous complex64 CUDA tensor of shape ({N}, {N})")


def _aperture_ptr(aperture, N):
    """(pointer, keep-alive object) of an N x N float32 aperture given as a
    numpy array (host) or a torch tensor (host or CUDA); (None, None) for the
    circle of the parameters' diameter."""
    if aperture is None:
        return None, None
    torch = _torch()
    if isinstance(aperture, torch.Tensor):
        a = aperture.detach().to(torch.float32).contiguous()
        if tuple(a.shape) != (N, N):
            raise ValueError(f"aperture must have shape ({N}, {N})")
        return ctypes.c_void_p(a.data_ptr()), a
    import numpy as np
    a = np.ascontiguousarray(aperture, dtype=np.float32)
    if a.shape != (N, N):
        raise ValueError(f"aperture must have shape ({N}, {N})")
    return ctypes.c_void_p(a.ctypes.data), a


class Stream:
    """One DDH-MBIR stream with device-resident state (r, phi, n).
    ``aperture``: optional N x N binary array (numpy or torch, host or CUDA),
    the diagonal of D_a; default the circle of ``pupil_diameter``."""

    def __init__(self, N: int, params: Params | None = None, aperture=None, **kw):
        self.N = N
        self.params = params if params is not None else make_params(N, **kw)
        h = ctypes.c_void_p()
        ap, keep = _aperture_ptr(aperture, N)
        if keep is not None and hasattr(keep, "is_cuda") and keep.is_cuda:
            _torch().cuda.current_stream().synchronize()  # the library reads the array synchronously
        _check(lib().ddh_init_stream(ctypes.byref(self.params), ap, _stream_ptr(), ctypes.byref(h)),
               "ddh_init_stream")
        del keep
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise DDHError(DDH_ESTATE, "stream destroyed")
        return self._h

    def step(self, y) -> None:
        """One DDH frame (Fig. 1 body) on the current torch stream."""
        _check_frame(y, self.N)
        _check(lib().ddh_step(self.handle, ctypes.c_void_p(y.data_ptr()), _stream_ptr()), "ddh_step")

    def em(self, y) -> None:
        """One plain EM(r, phi; y) iteration."""
        _check_frame(y, self.N)
        _check(lib().ddh_em(self.handle, ctypes.c_void_p(y.data_ptr()), _stream_ptr()), "ddh_em")

    def mbir(self, y, iters: int, reset_every: int = 200) -> None:
        """Conventional DH-MBIR on one frame: iters EM iterations with a
        bootstrap reset every reset_every iterations (ddh_mbir)."""
        _check_frame(y, self.N)
        _check(lib().ddh_mbir(self.handle, ctypes.c_void_p(y.data_ptr()), int(iters), int(reset_every),
                              _stream_ptr()), "ddh_mbir")

    def phase(self):
        torch = _torch()
        out = torch.empty((self.N, self.N), dtype=torch.float32, device="cuda")
        _check(lib().ddh_get_phase(self.handle, ctypes.c_void_p(out.data_ptr()), _stream_ptr()), "ddh_get_phase")
        return out

    def reflectance(self):
        torch = _torch()
        out = torch.empty((self.N, self.N), dtype=torch.float32, device="cuda")
        _check(lib().ddh_get_reflectance(self.handle, ctypes.c_void_p(out.data_ptr()), _stream_ptr()),
               "ddh_get_reflectance")
        return out

    def set_state(self, r, phi, n: int = 0) -> None:
        torch = _torch()
        for x in (r, phi):
            if not (x.is_cuda and x.dtype == torch.float32 and tuple(x.shape) == (self.N, self.N) and x.is_contiguous()):
                raise ValueError("state arrays must be contiguous float32 CUDA tensors of shape (N, N)")
        _check(lib().ddh_set_state(self.handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                   int(n), _stream_ptr()), "ddh_set_state")

    def frame_count(self) -> int:
        n = ctypes.c_longlong()
        _check(lib().ddh_frame_count(self.handle, ctypes.byref(n)), "ddh_frame_count")
        return n.value

    def status(self) -> int:
        """DDH_OK or DDH_EDATA for the last submitted frame, or DDH_EDEVICE if a
        wait of a work-list batch gave up on this stream (synchronises)."""
        rc = lib().ddh_status(self.handle, _stream_ptr())
        if rc not in (DDH_OK, DDH_EDATA, DDH_EDEVICE):
            _check(rc, "ddh_status")
        return rc

    def cost(self, y) -> float:
        _check_frame(y, self.N)
        U = ctypes.c_double()
        _check(lib().ddh_cost(self.handle, ctypes.c_void_p(y.data_ptr()), ctypes.byref(U), _stream_ptr()), "ddh_cost")
        return U.value

    def strehl(self, phi_true) -> float:
        torch = _torch()
        if not (phi_true.is_cuda and phi_true.dtype == torch.float32 and phi_true.is_contiguous()
                and tuple(phi_true.shape) == (self.N, self.N)):
            raise ValueError("phi_true must be a contiguous float32 CUDA tensor of shape (N, N)")
        S = ctypes.c_double()
        _check(lib().ddh_strehl(self.handle, ctypes.c_void_p(phi_true.data_ptr()), ctypes.byref(S), _stream_ptr()),
               "ddh_strehl")
        return S.value

    def close(self) -> None:
        if self._h is not None:
            _check(lib().ddh_destroy_stream(self._h), "ddh_destroy_stream")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several streams advanced together by one call per frame."""

    def __init__(self, streams, graph: bool = True, lanes: int = 0, worklist: bool = False,
                 test_giveup: bool = False):
        self.streams = list(streams)
        arr = (ctypes.c_void_p * len(self.streams))(*[s.handle.value for s in self.streams])
        h = ctypes.c_void_p()
        flags = (DDH_BATCH_GRAPH if graph else 0) | ((int(lanes) & 0xff) << 8)  # lanes 0: one per distinct N
        if worklist:
            flags |= DDH_BATCH_WORKLIST | (DDH_BATCH_TEST_GIVEUP if test_giveup else 0)
        _check(lib().ddh_batch_create(arr, len(self.streams), flags, ctypes.byref(h)), "ddh_batch_create")
        self._h = h
        self._ptrs = (ctypes.c_void_p * len(self.streams))()

    def step(self, ys) -> None:
        if len(ys) != len(self.streams):
            raise ValueError("one frame per stream")
        for i, (y, s) in enumerate(zip(ys, self.streams)):
            _check_frame(y, s.N)
            self._ptrs[i] = y.data_ptr()
        _check(lib().ddh_batch_step(self._h, self._ptrs, _stream_ptr()), "ddh_batch_step")

    def step_ptrs(self, ptrs) -> None:
        """Like step() with raw device pointers (already validated by the caller)."""
        for i, p in enumerate(ptrs):
            self._ptrs[i] = p
        _check(lib().ddh_batch_step(self._h, self._ptrs, _stream_ptr()), "ddh_batch_step")

    def set_timing(self, enable: bool) -> None:
        _check(lib().ddh_batch_set_timing(self._h, 1 if enable else 0), "ddh_batch_set_timing")

    def stage_times(self) -> dict:
        n = ctypes.c_int(16)
        ms = (ctypes.c_double * 16)()
        calls = (ctypes.c_longlong * 16)()
        names = (ctypes.c_char_p * 16)()
        _check(lib().ddh_batch_stage_times(self._h, ms, calls, names, ctypes.byref(n)), "ddh_batch_stage_times")
        return {names[k].decode(): (ms[k], calls[k]) for k in range(n.value)}

    def close(self) -> None:
        if self._h is not None:
            _check(lib().ddh_batch_destroy(self._h), "ddh_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(streams, ys) -> None:
    """One frame on each of several distinct streams (any mix of N), without a
    handle (ddh_step_batch), on the current torch stream."""
    if len(ys) != len(streams):
        raise ValueError("one frame per stream")
    for y, s in zip(ys, streams):
        _check_frame(y, s.N)
    n = len(streams)
    hs = (ctypes.c_void_p * max(n, 1))(*[s.handle.value for s in streams])
    ps = (ctypes.c_void_p * max(n, 1))(*[y.data_ptr() for y in ys])
    _check(lib().ddh_step_batch(hs, ps, n, _stream_ptr()), "ddh_step_batch")


def stream_bytes(N: int) -> int:
    """Device bytes one stream of grid size N holds (ddh_stream_bytes)."""
    b = ctypes.c_ulonglong()
    _check(lib().ddh_stream_bytes(int(N), ctypes.byref(b)), "ddh_stream_bytes")
    return int(b.value)


class Server:
    """Continuous batching: each call advances whichever distinct streams have
    a frame ready, the set changing from call to call (``ddh_server_step``)."""

    def __init__(self, max_streams: int):
        h = ctypes.c_void_p()
        _check(lib().ddh_server_create(int(max_streams), ctypes.byref(h)), "ddh_server_create")
        self._h = h
        self.max_streams = int(max_streams)
        self._s = (ctypes.c_void_p * self.max_streams)()
        self._y = (ctypes.c_void_p * self.max_streams)()

    def step(self, streams, ys) -> None:
        if len(ys) != len(streams):
            raise ValueError("one frame per stream")
        if len(streams) > self.max_streams:
            raise ValueError("more streams than the server holds")
        for i, (y, s) in enumerate(zip(ys, streams)):
            _check_frame(y, s.N)
            self._s[i] = s.handle.value
            self._y[i] = y.data_ptr()
        _check(lib().ddh_server_step(self._h, self._s, self._y, len(streams), _stream_ptr()), "ddh_server_step")

    def step_ptrs(self, streams, ptrs) -> None:
        """Like step() with raw device pointers (already validated by the caller)."""
        for i, (s, p) in enumerate(zip(streams, ptrs)):
            self._s[i] = s.handle.value
            self._y[i] = p
        _check(lib().ddh_server_step(self._h, self._s, self._y, len(streams), _stream_ptr()), "ddh_server_step")

    def close(self) -> None:
        if self._h is not None:
            _check(lib().ddh_server_destroy(self._h), "ddh_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unrolled_grad(params: Params, frames, phi0, phi_true, ckpt: int = 2):
    """Loss of len(frames) unrolled DDH frames from r = 0, phi = phi0 (the
    piston-removed RMS phase error against phi_true after the last frame)
    and its gradient: (loss, d/dphi0 tensor, d/dsigma_w, d/dqg_sigma,
    d/dbeta_phi), by the hand-written adjoint (ddh_unrolled_grad)."""
    torch = _torch()
    N = params.N
    for y in frames:
        _check_frame(y, N)
    for x in (phi0, phi_true):
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and tuple(x.shape) == (N, N)):
            raise ValueError("phi0 and phi_true must be contiguous float32 CUDA tensors of shape (N, N)")
    ys = (ctypes.c_void_p * len(frames))(*[y.data_ptr() for y in frames])
    g = torch.empty((N, N), dtype=torch.float32, device=phi0.device)
    out = GradOut()
    _check(lib().ddh_unrolled_grad(ctypes.byref(params), len(frames), ys, ctypes.c_void_p(phi0.data_ptr()),
                                   ctypes.c_void_p(phi_true.data_ptr()), int(ckpt), ctypes.c_void_p(g.data_ptr()),
                                   ctypes.byref(out), _stream_ptr()), "ddh_unrolled_grad")
    return out.loss, g, out.d_sigma_w, out.d_sigma_r, out.d_beta


def unrolled_grad_batch(params, frames, phi0, phi_true, ckpt: int = 2):
    """unrolled_grad for several streams of one N in one pass
    (ddh_unrolled_grad_batch).  params, frames (a list of K frames per
    stream), phi0, phi_true: one entry per stream.  Returns a list of
    (loss, d/dphi0, d/dsigma_w, d/dqg_sigma, d/dbeta_phi) per stream."""
    torch = _torch()
    B = len(params)
    if not (B >= 1 and len(frames) == B and len(phi0) == B and len(phi_true) == B):
        raise ValueError("params, frames, phi0 and phi_true need one entry per stream")
    K = len(frames[0])
    N = params[0].N
    for b in range(B):
        if params[b].N != N or len(frames[b]) != K:
            raise ValueError("all streams need the same N and the same number of frames")
        for y in frames[b]:
            _check_frame(y, N)
        for x in (phi0[b], phi_true[b]):
            if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and tuple(x.shape) == (N, N)):
                raise ValueError("phi0 and phi_true must be contiguous float32 CUDA tensors of shape (N, N)")
    prm = (Params * B)(*params)
    ys = (ctypes.c_void_p * (B * K))(*[y.data_ptr() for fr in frames for y in fr])
    grads = [torch.empty((N, N), dtype=torch.float32, device=phi0[0].device) for _ in range(B)]
    p0 = (ctypes.c_void_p * B)(*[x.data_ptr() for x in phi0])
    pt = (ctypes.c_void_p * B)(*[x.data_ptr() for x in phi_true])
    gp = (ctypes.c_void_p * B)(*[x.data_ptr() for x in grads])
    outs = (GradOut * B)()
    _check(lib().ddh_unrolled_grad_batch(prm, B, K, ys, p0, pt, int(ckpt), gp, outs, _stream_ptr()),
           "ddh_unrolled_grad_batch")
    return [(o.loss, g, o.d_sigma_w, o.d_sigma_r, o.d_beta) for o, g in zip(outs, grads)]


def unrolled_loss_fn():
    """torch.autograd.Function over unrolled_grad: forward(phi0, sigma_w,
    sigma_r, beta, frames, phi_true, base_params, ckpt) -> loss; backward
    returns the hand-written adjoint's gradients for phi0, sigma_w, sigma_r
    and beta."""
    torch = _torch()

    class UnrolledEM(torch.autograd.Function):
        @staticmethod
        def forward(ctx, phi0, sigma_w, sigma_r, beta, frames, phi_true, base, ckpt=2):
            prm = Params.from_buffer_copy(base)
            prm.sigma_w2 = float(sigma_w) ** 2
            prm.qg_sigma = float(sigma_r)
            prm.beta_phi = float(beta)
            prm.n_k = 1
            L, g, gw, gr, gb = unrolled_grad(prm, frames, phi0.detach().contiguous(), phi_true, ckpt)
            ctx.save_for_backward(g)
            ctx.scal = (gw, gr, gb)
            return torch.tensor(L, dtype=torch.float64, device=phi0.device)

        @staticmethod
        def backward(ctx, gL):
            (g,) = ctx.saved_tensors
            gw, gr, gb = ctx.scal
            s = gL.to(torch.float64)
            return ((s * g.double()).to(g.dtype), s * gw, s * gr, s * gb, None, None, None, None)

    return UnrolledEM


def fft2(x, inverse: bool = False):
    """Batched unitary 2-D DFT of a contiguous complex64 CUDA tensor (..., N, N)."""
    torch = _torch()
    if not (x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous() and x.shape[-1] == x.shape[-2]):
        raise ValueError("fft2 needs a contiguous complex64 CUDA tensor (..., N, N)")
    N = x.shape[-1]
    count = x.numel() // (N * N)
    out = torch.empty_like(x)
    work = torch.empty_like(x)
    _check(lib().ddh_fft2(N, count, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(work.data_ptr()), 1 if inverse else 0, _stream_ptr()), "ddh_fft2")
    return out


def set_tiles(N: int, cfg) -> None:
    """Tiling for grid size N: (row lines, column width, M-step tile h, w)."""
    arr = (ctypes.c_int * 4)(*cfg)
    _check(lib().ddh_set_tiles(N, arr), "ddh_set_tiles")


def get_tiles(N: int):
    arr = (ctypes.c_int * 4)()
    _check(lib().ddh_get_tiles(N, arr), "ddh_get_tiles")
    return tuple(arr)


def autotune(N: int, count: int):
    """Time every tiling candidate on `count` temporary streams of size N,
    install the fastest; returns (cfg, winner times in microseconds)."""
    cfg = (ctypes.c_int * 4)()
    us = (ctypes.c_double * 4)()
    _check(lib().ddh_autotune(N, count, cfg, us), "ddh_autotune")
    return tuple(cfg), tuple(us)


def autotune_mix(sizes):
    """Tune the tilings of a mix of stream sizes together by timing the whole
    batched step (ddh_autotune_mix); installs them and returns
    ({N: cfg}, step time in microseconds)."""
    sizes = [int(n) for n in sizes]
    ns = (_c_int * len(sizes))(*sizes)
    distinct = sorted(set(sizes))
    cfgs = (_c_int * (4 * len(distinct)))()
    us = _c_double()
    _check(lib().ddh_autotune_mix(ns, len(sizes), cfgs, ctypes.byref(us)), "ddh_autotune_mix")
    return {n: tuple(cfgs[4 * k:4 * k + 4]) for k, n in enumerate(distinct)}, us.value


__all__ = ["step_batch", "set_tiles", "get_tiles", "autotune", "autotune_mix", "Stream", "Batch", "Server", "stream_bytes", "unrolled_grad", "unrolled_grad_batch", "unrolled_loss_fn", "GradOut", "Params", "make_params", "default_params", "fft2", "lib", "DDHError",
           "SIGNATURES", "LIB_PATH"]
