"""The no-allocation batched step (ddh_step_batch_noalloc) against the
allocating one (ddh_step_batch), through the C ABI: two calls in a row, the
second with fewer streams, each bit-identical to the same streams stepped by
ddh_step_batch.  Collected last so that a failure here hides no other test."""
import ctypes

import numpy as np
import pytest

import ddh_synth as synth

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_03284_amd as D
    return torch, D


def _params(D, N, s2):
    return D.make_params(N, sigma_w2=float(np.float32(s2)))


def _state(torch, s):
    torch.cuda.synchronize()
    return s.reflectance().cpu().numpy(), s.phase().cpu().numpy()


def _call(D, fn, streams, ys):
    n = len(streams)
    hs = (ctypes.c_void_p * n)(*[s.handle.value for s in streams])
    ps = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
    rc = fn(hs, ps, n, D._stream_ptr())
    assert rc == D.DDH_OK, D.lib().ddh_error_string(rc)


def test_noalloc_batched_step_equals_allocating_one():
    torch, D = _setup()
    L = D.lib()
    Ns = [256, 64, 128, 256, 512, 128]
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0 + i, snr=4.0 + i, speed=0.5, config_id=25,
                                          stream_id=i)) for i, N in enumerate(Ns)]
    prms = [_params(D, N, sm.sigma_w2) for N, sm in zip(Ns, sims)]
    frames = [[torch.from_numpy(sm.frame(n)).cuda() for n in range(2)] for sm in sims]
    ref = [D.Stream(N, p) for N, p in zip(Ns, prms)]
    new = [D.Stream(N, p) for N, p in zip(Ns, prms)]
    # call 1: all six streams; call 2: three of them (a smaller input)
    subsets = [list(range(6)), [4, 0, 2]]
    for call, idx in enumerate(subsets):
        print(f"no-alloc call {call}: streams {idx} (N {[Ns[i] for i in idx]})", flush=True)
        _call(D, L.ddh_step_batch, [ref[i] for i in idx], [frames[i][call] for i in idx])
        _call(D, L.ddh_step_batch_noalloc, [new[i] for i in idx], [frames[i][call] for i in idx])
        for i in range(6):
            r0, p0 = _state(torch, ref[i])
            r1, p1 = _state(torch, new[i])
            np.testing.assert_array_equal(r1, r0)
            np.testing.assert_array_equal(p1, p0)
            assert new[i].frame_count() == ref[i].frame_count()
    assert [s.frame_count() for s in new] == [2, 1, 2, 1, 2, 1]
    # sizes beyond the fixed list are refused before any work
    assert L.ddh_step_batch_noalloc(None, None, 4097, None) == D.DDH_EINVAL
    for s in ref + new:
        s.close()
