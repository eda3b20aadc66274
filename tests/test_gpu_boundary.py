"""GPU checks of the boundary calls that take an aperture array and step many
streams without a handle (the Forward Model's D_a; Fig. 1's ReadData /
WriteData for several streams at once), through the C ABI."""
import numpy as np
import pytest

import ddh_synth as synth
from oracle import ddh as O
from oracle import metrics as M

from test_gpu_parity import TOL_PHI, TOL_R, _ddh, _torch, compare, dev, make_pair, say, state

pytestmark = pytest.mark.gpu


def annulus(N, outer, inner):
    """Binary annulus centred on the grid: outer and inner diameters in px."""
    ii, jj = np.mgrid[0:N, 0:N]
    d2 = (2 * ii - N + 1) ** 2 + (2 * jj - N + 1) ** 2
    return ((d2 <= outer ** 2) & (d2 > inner ** 2)).astype(np.float64)


class ApertureStream:
    """Frames y = a exp(j phi) F g + w drawn with a given aperture a."""

    def __init__(self, N, a, snr=10.0, d_over_r0=8.0, stream_id=0):
        self.sim = synth.Stream(synth.StreamSpec(N=N, d_over_r0=d_over_r0, snr=snr, speed=0.5, config_id=21,
                                                 stream_id=stream_id))
        self.a, self.snr = a, snr
        self.sigma_w2 = synth.sigma_w2_normalized(float(a.sum()) / (N * N), snr)

    def phase(self, n):
        return self.sim.phase(n)

    def frame(self, n):
        rng = synth.rng_for(21, self.sim.spec.stream_id, synth.PURPOSE_FRAME, n)
        return synth.hologram(self.sim.r, self.phase(n), self.a, self.snr, rng).astype(np.complex64)


@pytest.mark.parametrize("N", [64, 256])
def test_annulus_aperture_frames_cost_and_strehl_match_oracle(N):
    D = _ddh()
    a = annulus(N, N, N // 3)
    st = ApertureStream(N, a, stream_id=N)
    prm, gp = make_pair(N, st.sigma_w2)
    s = D.Stream(N, gp, aperture=a)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        say(f"annulus N={N} frame {n}")
        y = st.frame(n)
        r_o, p_o = O.ddh_frame(r_o, p_o, y.astype(np.complex128), a, prm)
        s.step(dev(y))
        assert s.status() == D.DDH_OK
        r_g, p_g = state(s)
        compare(f"frame {n}", r_g, p_g, r_o, p_o, a)
    # diagnostics read the same aperture
    y = st.frame(3)
    u_gpu = s.cost(dev(y))
    u_orc = M.cost_U(r_g, p_g, O.normalize(y.astype(np.complex128)), a, prm)
    assert abs(u_gpu - u_orc) < 1e-5 * abs(u_orc), (u_gpu, u_orc)
    truth = st.phase(2).astype(np.float32)
    S_gpu = s.strehl(dev(truth))
    S_orc = M.strehl(p_g, truth.astype(np.float64), a)
    assert abs(S_gpu - S_orc) < 1e-5, (S_gpu, S_orc)
    s.close()


def test_aperture_array_host_device_and_circle_agree():
    """The circle passed as an array (host, or device memory) gives the same
    bits as the circle given by its diameter; a resumed state keeps the phase
    zero off the aperture."""
    D = _ddh()
    torch = _torch()
    N = 128
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0, snr=10.0, speed=0.5, config_id=22))
    prm, gp = make_pair(N, st.sigma_w2)
    circ = O.aperture(N)
    frames = [dev(st.frame(n)) for n in range(3)]
    outs = []
    for ap in (None, circ, torch.from_numpy(circ.astype(np.float32)).cuda()):
        s = D.Stream(N, gp, aperture=ap)
        for y in frames:
            s.step(y)
        outs.append(state(s))
        s.close()
    for r, p in outs[1:]:
        np.testing.assert_array_equal(r, outs[0][0])
        np.testing.assert_array_equal(p, outs[0][1])
    a = annulus(N, N, N // 2)
    s = D.Stream(N, gp, aperture=a)
    rng = np.random.default_rng(3)
    s.set_state(dev(rng.uniform(0.1, 1.0, (N, N)), np.float32), dev(rng.uniform(-1, 1, (N, N)), np.float32), 5)
    _, p = state(s)
    assert np.all(p[a == 0] == 0.0) and np.all(p[a > 0] != 0.0)
    s.close()


def _streams_mixed(D):
    """Seven streams of mixed N; one has an annulus aperture."""
    Ns = [128, 256, 64, 256, 512, 128, 64]
    out = []
    for i, N in enumerate(Ns):
        if i == 5:
            a = annulus(N, N, N // 2)
            sm = ApertureStream(N, a, snr=6.0, stream_id=100 + i)
        else:
            a = None
            sm = synth.Stream(synth.StreamSpec(N=N, d_over_r0=5.0 + 2 * i, snr=3.0 + i, speed=0.5, config_id=23,
                                               stream_id=i))
        out.append((N, a, sm, make_pair(N, sm.sigma_w2)))
    return out


def test_step_batch_equals_streams_alone():
    """ddh_step_batch over streams of mixed N (one with an annulus) gives each
    stream the bits of stepping it alone, frame after frame; a later call with
    more streams than the first call's list held (70 N=64 streams) grows the
    list and still equals the streams alone."""
    D = _ddh()
    cases = _streams_mixed(D)
    frames = [[dev(sm.frame(n)) for n in range(3)] for (_, _, sm, _) in cases]
    alone = []
    for i, (N, a, sm, (prm, gp)) in enumerate(cases):
        s = D.Stream(N, gp, aperture=a)
        for y in frames[i]:
            s.step(y)
        alone.append(state(s))
        s.close()
    streams = [D.Stream(N, gp, aperture=a) for (N, a, sm, (prm, gp)) in cases]
    for n in range(3):
        say(f"step_batch frame {n}")
        D.step_batch(streams, [frames[i][n] for i in range(len(cases))])
    for i, s in enumerate(streams):
        r, p = state(s)
        np.testing.assert_array_equal(r, alone[i][0])
        np.testing.assert_array_equal(p, alone[i][1])
        assert s.frame_count() == 3
    # the annulus member against the oracle
    N, a, sm, (prm, gp) = cases[5]
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        r_o, p_o = O.ddh_frame(r_o, p_o, sm.frame(n).astype(np.complex128), a, prm)
    compare("annulus member vs oracle", *alone[5], r_o, p_o, a)
    for s in streams:
        s.close()
    # growth: 70 streams on the same HIP stream after the 7-stream calls
    S, N = 70, 64
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0, snr=10.0, speed=0.5, config_id=24, stream_id=k))
            for k in range(S)]
    pairs = [make_pair(N, sm.sigma_w2) for sm in sims]
    ys = [dev(sm.frame(0)) for sm in sims]
    ref = []
    for i in range(S):
        s = D.Stream(N, pairs[i][1])
        s.step(ys[i])
        ref.append(state(s))
        s.close()
    say(f"step_batch {S} streams")
    streams = [D.Stream(N, pairs[i][1]) for i in range(S)]
    D.step_batch(streams, ys)
    for i, s in enumerate(streams):
        r, p = state(s)
        np.testing.assert_array_equal(r, ref[i][0])
        np.testing.assert_array_equal(p, ref[i][1])
        s.close()
