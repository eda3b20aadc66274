"""Continuous batching on the GPU: a stream's result is the same alone and in
any mix (bit for bit: per-stream numerics do not depend on the other streams
of a launch), through ddh_server_step directly and through the request loop
with admission by memory budget."""
import sys

import numpy as np
import pytest

import ddh_synth as synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(D, N, sigma_w2):
    v = synth.DEFAULT_PARAMS
    return D.make_params(N, pupil_diameter=float(N), lam=v["lam"], alpha=v["alpha"], n_k=v["n_k"],
                         sigma_w2=sigma_w2, qg_q=v["qg_q"], qg_T=v["qg_T"], qg_sigma=v["qg_sigma"],
                         beta_phi=v["beta_phi"], r_floor=v["r_floor"])


def _setup(sizes, n_frames, config_id):
    torch = _torch()
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0 + 2 * i, snr=5.0 + i, config_id=config_id, stream_id=i))
            for i, N in enumerate(sizes)]
    frames = [[torch.from_numpy(sm.frame(n)).cuda() for n in range(n_frames)] for sm in sims]
    return sims, frames


def _alone(D, sims, frames, counts):
    out = []
    for i, sm in enumerate(sims):
        N = sm.frame(0).shape[0]
        s = D.Stream(N, _params(D, N, sm.sigma_w2))
        for n in range(counts[i]):
            s.step(frames[i][n])
        out.append((s.reflectance().cpu().numpy(), s.phase().cpu().numpy()))
        s.close()
    return out


def test_server_step_mixes_match_alone():
    torch = _torch()
    import paper_2305_03284_amd as D
    sizes = [64, 128, 64, 256, 128, 64]
    sims, frames = _setup(sizes, 6, config_id=31)
    streams = [D.Stream(N, _params(D, N, sm.sigma_w2)) for N, sm in zip(sizes, sims)]
    srv = D.Server(8)
    rng = np.random.default_rng(7)
    done = [0] * len(sizes)
    calls = 0
    while min(done) < 6:
        # a random subset of the streams that still have frames, in random order
        live = [i for i in range(len(sizes)) if done[i] < 6]
        pick = [i for i in live if rng.random() < 0.6] or live[:1]
        rng.shuffle(pick)
        say(f"call {calls}: streams {pick}")
        srv.step([streams[i] for i in pick], [frames[i][done[i]] for i in pick])
        for i in pick:
            done[i] += 1
        calls += 1
    torch.cuda.synchronize()
    ref = _alone(D, sims, frames, done)
    for i, s in enumerate(streams):
        np.testing.assert_array_equal(s.reflectance().cpu().numpy(), ref[i][0])
        np.testing.assert_array_equal(s.phase().cpu().numpy(), ref[i][1])
        s.close()
    srv.close()


def test_server_call_with_more_streams_than_one_launch_takes():
    """70 streams in one server call (the frame-start launch carries at most
    64 streams' arguments, so the call needs two), mixed N: each equals the
    stream stepped alone."""
    torch = _torch()
    import paper_2305_03284_amd as D
    sizes = [64] * 66 + [128] * 4
    sims, frames = _setup(sizes, 2, config_id=33)
    streams = [D.Stream(N, _params(D, N, sm.sigma_w2)) for N, sm in zip(sizes, sims)]
    srv = D.Server(len(sizes))
    order = list(range(len(sizes)))
    np.random.default_rng(3).shuffle(order)
    for n in range(2):
        say(f"server call {n}: {len(order)} streams")
        srv.step([streams[i] for i in order], [frames[i][n] for i in order])
    torch.cuda.synchronize()
    ref = _alone(D, sims, frames, [2] * len(sizes))
    for i, s in enumerate(streams):
        np.testing.assert_array_equal(s.reflectance().cpu().numpy(), ref[i][0])
        np.testing.assert_array_equal(s.phase().cpu().numpy(), ref[i][1])
        s.close()
    srv.close()


def test_server_rejects_bad_calls():
    torch = _torch()
    import paper_2305_03284_amd as D
    sims, frames = _setup([64, 64], 1, config_id=32)
    a = D.Stream(64, _params(D, 64, sims[0].sigma_w2))
    b = D.Stream(64, _params(D, 64, sims[1].sigma_w2))
    srv = D.Server(2)
    with pytest.raises(D.DDHError):
        srv.step([a, a], [frames[0][0], frames[1][0]])        # repeated stream
    with pytest.raises(ValueError):
        srv.step([a, b, a], [frames[0][0]] * 3)                # more than max_streams
    srv.step([a], [frames[0][0]])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with pytest.raises(D.DDHError):
            srv.step([b], [frames[1][0]])                      # not the server's HIP stream
    torch.cuda.synchronize()
    # the rejected calls changed nothing: a ran one frame, b none
    ref = _alone(D, sims[:1], frames[:1], [1])
    np.testing.assert_array_equal(a.reflectance().cpu().numpy(), ref[0][0])
    assert b.frame_count() == 0 and a.frame_count() == 1
    for x in (a, b, srv):
        x.close()


def test_request_loop_same_alone_and_in_mix():
    torch = _torch()
    import paper_2305_03284_amd as D
    from paper_2305_03284_amd.serve import ServeLoop, latency_stats, poisson_requests
    sizes = [64, 128, 64, 128, 64, 128, 64, 64]
    n_frames = 5
    sims, frames = _setup(sizes, n_frames, config_id=33)
    keys = list(range(len(sizes)))
    reqs = poisson_requests(keys, rate_hz=4000.0, frames_per_stream=n_frames, seed=11, start_spread_s=0.002)
    for r in reqs:
        r.payload = frames[r.key][r.index]
    nbytes = {k: D.stream_bytes(sizes[k]) for k in keys}
    budget = nbytes[1] * 2 + nbytes[0]  # room for about three streams: the others wait for admission
    finals = {}

    def make_stream(k):
        return D.Stream(sizes[k], _params(D, sizes[k], sims[k].sigma_w2))

    def on_retire(k, s):
        finals[k] = (s.reflectance().cpu().numpy(), s.phase().cpu().numpy())

    for plain in (False, True):
        finals.clear()
        out = ServeLoop(budget, max_batch=8, depth=2, plain=plain).run(reqs, make_stream, nbytes.__getitem__,
                                                                       on_retire)
        st = latency_stats(out)
        say(f"plain={plain}: {st}")
        assert all(r.t_done is not None and r.t_done >= r.t_arrival for r in out)
        assert sorted(finals) == keys
        ref = _alone(D, sims, frames, [n_frames] * len(sizes))
        for k in keys:
            np.testing.assert_array_equal(finals[k][0], ref[k][0])
            np.testing.assert_array_equal(finals[k][1], ref[k][1])
        for r in reqs:
            r.t_done = None
    torch.cuda.synchronize()
