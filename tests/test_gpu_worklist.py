"""The work-list batched step (DDH_BATCH_WORKLIST: one persistent launch per
EM iteration and N group for the stats, row and column passes of all the
group's streams, then the M-step) against the default launches, through the
C ABI: every stream's state must be bit-identical, in any mix of sizes, with
several EM iterations per frame, more streams than one launch's frame
arguments hold, the whole-image M-step, HIP-graph replay and timing mode.
Also the failure path: with every dependency wait forced to give up, each
launch still ends and the streams report the error."""
import numpy as np
import pytest

import ddh_synth as synth

from test_gpu_parity import _ddh, _torch, dev, make_pair, say, state

pytestmark = pytest.mark.gpu


def _run(D, cases, frames, nfr, **batch_kw):
    streams = [D.Stream(N, gp) for (N, gp) in cases]
    b = D.Batch(streams, **batch_kw)
    for n in range(nfr):
        b.step([frames[i][n] for i in range(len(cases))])
    out = [state(s) for s in streams]
    b.close()
    for s in streams:
        s.close()
    return out


def _cases(Ns, config_id, n_k=1):
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=5.0 + i % 11, snr=3.0 + i % 7, speed=0.5,
                                          config_id=config_id, stream_id=i)) for i, N in enumerate(Ns)]
    cases = [(N, make_pair(N, sm.sigma_w2, n_k=n_k)[1]) for N, sm in zip(Ns, sims)]
    return sims, cases


@pytest.mark.parametrize("variant", ["mixed", "mixed_graph", "n_k2", "many_streams", "whole_image_mstep",
                                     "timing"])
def test_worklist_batch_equals_default_launches(variant):
    D = _ddh()
    torch = _torch()
    if variant == "many_streams":
        Ns = [64] * 70 + [128] * 3           # more than the 64 frame arguments of one launch
    elif variant in ("n_k2", "whole_image_mstep"):
        Ns = [256, 128, 256, 64]
    else:
        Ns = [128, 256, 64, 256, 512, 128, 64, 256]
    n_k = 2 if variant == "n_k2" else 1
    sims, cases = _cases(Ns, 31, n_k)
    nfr = 3
    frames = [[dev(sm.frame(n)) for n in range(nfr)] for sm in sims]
    saved = {}
    if variant == "whole_image_mstep":
        for N in set(Ns):
            saved[N] = D.get_tiles(N)
            D.set_tiles(N, (saved[N][0], saved[N][1], 0, 0))
    try:
        say(f"work list variant {variant}: {len(Ns)} streams")
        ref = _run(D, cases, frames, nfr, graph=False)
        graph = variant == "mixed_graph"
        if variant == "timing":
            streams = [D.Stream(N, gp) for (N, gp) in cases]
            b = D.Batch(streams, graph=False, worklist=True)
            b.set_timing(True)
            for n in range(nfr):
                b.step([frames[i][n] for i in range(len(cases))])
            times = b.stage_times()
            b.close()
            got = [state(s) for s in streams]
            for s in streams:
                s.close()
            assert times["frame_worklist"][1] == nfr * len(set(Ns))
            assert times["m_step"][1] == nfr * len(set(Ns))
            assert times["stats"][1] == 0 and times["col_fused"][1] == 0
        else:
            got = _run(D, cases, frames, nfr, graph=graph, worklist=True)
    finally:
        for N, t in saved.items():
            D.set_tiles(N, t)
    torch.cuda.synchronize()
    for i, ((r0, p0), (r1, p1)) in enumerate(zip(ref, got)):
        np.testing.assert_array_equal(r1, r0, err_msg=f"stream {i} N={Ns[i]}")
        np.testing.assert_array_equal(p1, p0, err_msg=f"stream {i} N={Ns[i]}")


def test_worklist_gives_up_and_every_launch_ends():
    """Every dependency wait of the work list forced to give up at once: the
    launches still end (the step and a device synchronisation return), every
    stream whose items waited reports DDH_EDEVICE once, and after its state is
    restored a normal work-list batch gives the default launches' result."""
    D = _ddh()
    torch = _torch()
    Ns = [256, 128, 256, 512]
    sims, cases = _cases(Ns, 32)
    frames = [[dev(sm.frame(n)) for n in range(2)] for sm in sims]
    streams = [D.Stream(N, gp) for (N, gp) in cases]
    b = D.Batch(streams, graph=False, worklist=True, test_giveup=True)
    say("work list with every wait giving up")
    b.step([frames[i][0] for i in range(len(Ns))])
    torch.cuda.synchronize()
    b.close()
    assert [s.status() for s in streams] == [D.DDH_EDEVICE] * len(Ns)
    # reported once (the frame's own statistics were computed from whatever the
    # items that gave up saw, so the frame may also read as rejected)
    assert all(s.status() in (D.DDH_OK, D.DDH_EDATA) for s in streams)
    # restore the zero state, then a normal work-list step equals the default one
    for s, (N, _) in zip(streams, cases):
        z = torch.zeros((N, N), dtype=torch.float32, device="cuda")
        s.set_state(z, z, 0)
    b = D.Batch(streams, graph=False, worklist=True)
    b.step([frames[i][1] for i in range(len(Ns))])
    got = [state(s) for s in streams]
    b.close()
    for s in streams:
        s.close()
    ref_streams = [D.Stream(N, gp) for (N, gp) in cases]
    rb = D.Batch(ref_streams, graph=False)
    rb.step([frames[i][1] for i in range(len(Ns))])
    ref = [state(s) for s in ref_streams]
    rb.close()
    for (r0, p0), (r1, p1) in zip(ref, got):
        np.testing.assert_array_equal(r1, r0)
        np.testing.assert_array_equal(p1, p0)


@pytest.mark.parametrize("graph", [False, True])
def test_worklist_stays_identical_over_repeated_concurrent_groups(graph):
    """Four N groups whose work-list launches run at once (one lane each),
    repeated: every repetition must give the default launches' result bit for
    bit and no wait may give up.  (Waves of one workgroup once read different
    tickets when the loop-top barrier was not preceded by a wait for the
    ticket's LDS store; under this load that showed in about a fifth of the
    runs.)"""
    D = _ddh()
    torch = _torch()
    Ns = [128, 256, 64, 256, 512, 128, 64, 256]
    sims, cases = _cases(Ns, 33)
    nfr, reps = 3, 40
    frames = [[dev(sm.frame(n)) for n in range(nfr)] for sm in sims]
    ref = _run(D, cases, frames, nfr, graph=False)
    streams = [D.Stream(N, gp) for (N, gp) in cases]
    b = D.Batch(streams, graph=graph, worklist=True)
    zs = {N: torch.zeros((N, N), dtype=torch.float32, device="cuda") for N in set(Ns)}
    say(f"work list, four concurrent groups, graph={graph}: {reps} repetitions of {nfr} frames")
    bad = []
    try:
        for rep in range(reps):
            for s, N in zip(streams, Ns):
                s.set_state(zs[N], zs[N], 0)
            for n in range(nfr):
                b.step([frames[i][n] for i in range(len(Ns))])
            got = [state(s) for s in streams]
            assert [s.status() for s in streams] == [D.DDH_OK] * len(Ns)
            bad += [(rep, i) for i, ((r0, p0), (r1, p1)) in enumerate(zip(ref, got))
                    if not (np.array_equal(r0, r1) and np.array_equal(p0, p1))]
    finally:
        b.close()
        for s in streams:
            s.close()
    assert not bad, bad[:10]
