"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (per frame): phase RMS over the pupil of the piston-removed
difference < 1e-4 rad; relative L2 error of r < 1e-4; Strehl within 0.005.
Batching, graphs, tiling and resume are checked bit for bit against the plain
single-stream path.
"""
import math
import sys

import numpy as np
import pytest

import ddh_synth as synth
from oracle import ddh as O
from oracle import metrics as M

pytestmark = pytest.mark.gpu

TOL_PHI = 1e-4
TOL_R = 1e-4
TOL_S = 0.005


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ddh():
    import paper_2305_03284_amd as D
    return D


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32(x):
    return float(np.float32(x))


def make_pair(N, sigma_w2, diameter=None, **over):
    """Oracle Params and GPU Params holding the same (float32) values."""
    D = _ddh()
    vals = dict(synth.DEFAULT_PARAMS)
    vals.update(over)
    prm = O.Params(sigma_w2=f32(sigma_w2), lam=f32(vals["lam"]), alpha=f32(vals["alpha"]), n_k=int(vals["n_k"]),
                   qg_p=2.0, qg_q=f32(vals["qg_q"]), qg_T=f32(vals["qg_T"]), qg_sigma=f32(vals["qg_sigma"]),
                   beta_phi=f32(vals["beta_phi"]), r_floor=f32(vals["r_floor"]))
    gp = D.make_params(N, pupil_diameter=float(N if diameter is None else diameter), lam=prm.lam, alpha=prm.alpha,
                       n_k=prm.n_k, sigma_w2=prm.sigma_w2, qg_q=prm.qg_q, qg_T=prm.qg_T, qg_sigma=prm.qg_sigma,
                       beta_phi=prm.beta_phi, r_floor=prm.r_floor)
    return prm, gp


def dev(x, dtype=None):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x if dtype is None else x.astype(dtype))).cuda()


def state(s):
    torch = _torch()
    torch.cuda.synchronize()
    return s.reflectance().cpu().numpy().astype(np.float64), s.phase().cpu().numpy().astype(np.float64)


def compare(tag, r_g, p_g, r_o, p_o, a):
    er = M.rel_l2(r_g, r_o)
    ep = M.phase_rms_diff(p_g, p_o, a)
    say(f"  {tag}: e_r={er:.2e} e_phi={ep:.2e}")
    assert er < TOL_R, (tag, er)
    assert ep < TOL_PHI, (tag, ep)
    assert np.all(p_g[a == 0] == 0.0)
    return er, ep


# ----------------------------------------------------------------------------- FFT

@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_fft2_matches_oracle(N):
    D = _ddh()
    say(f"fft2 N={N}")
    rng = np.random.default_rng(N)
    x = (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))).astype(np.complex64)
    xg = dev(x)
    for inv in (False, True):
        out = D.fft2(xg, inverse=inv).cpu().numpy()
        for b in range(3):
            ref = (O.FH if inv else O.F)(x[b].astype(np.complex128))
            err = np.linalg.norm(out[b] - ref) / np.linalg.norm(ref)
            assert err < 2e-6, (N, inv, b, err)
            assert abs(np.linalg.norm(out[b]) / np.linalg.norm(x[b]) - 1.0) < 2e-6


def test_fft2_delta_and_roundtrip():
    D = _ddh()
    torch = _torch()
    N = 256
    d = np.zeros((N, N), np.complex64)
    d[3, 5] = 1.0
    out = D.fft2(dev(d)).cpu().numpy()
    k1, k2 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    np.testing.assert_allclose(out, np.exp(-2j * np.pi * (3 * k1 + 5 * k2) / N) / N, atol=2e-7)
    x = dev((np.random.default_rng(1).standard_normal((N, N)) + 0j).astype(np.complex64))
    back = D.fft2(D.fft2(x), inverse=True)
    assert torch.max(torch.abs(back - x)).item() < 2e-6


# ----------------------------------------------------------------------------- frames

@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_first_frame_from_zero_state(N):
    D = _ddh()
    say(f"first frame N={N}")
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=10.0, snr=10.0, speed=0.5, config_id=11, stream_id=N))
    prm, gp = make_pair(N, st.sigma_w2)
    a = O.aperture(N)
    y = st.frame(0)
    r_o, p_o = O.ddh_frame(np.zeros((N, N)), np.zeros((N, N)), y.astype(np.complex128), a, prm)
    s = D.Stream(N, gp)
    s.step(dev(y))
    assert s.status() == D.DDH_OK
    compare(f"N={N}", *state(s), r_o, p_o, a)


def test_free_running_frames_and_strehl():
    """Free-running: strict parity on the first frames, Strehl within 0.005 on
    every frame.  The frame recursion itself amplifies a 1e-7 perturbation of
    its state by about 1.5-2x per frame (the oracle run against itself shows
    the same growth), so per-frame parity over long runs is pinned by the
    teacher-forced test instead."""
    D = _ddh()
    N, nf, strict = 128, 12, 6
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0, snr=8.0, speed=0.5, config_id=12, stream_id=0))
    prm, gp = make_pair(N, st.sigma_w2)
    a = O.aperture(N)
    s = D.Stream(N, gp)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(nf):
        say(f"free-running N={N} frame {n}")
        y = st.frame(n)
        r_o, p_o = O.ddh_frame(r_o, p_o, y.astype(np.complex128), a, prm)
        s.step(dev(y))
        r_g, p_g = state(s)
        if n < strict:
            compare(f"frame {n}", r_g, p_g, r_o, p_o, a)
        else:
            say(f"  frame {n}: e_r={M.rel_l2(r_g, r_o):.2e} e_phi={M.phase_rms_diff(p_g, p_o, a):.2e} (drift)")
        truth = st.phase(n)
        S_gpu = s.strehl(dev(truth, np.float32))
        S_orc_on_gpu = M.strehl(p_g, truth.astype(np.float32), a)
        S_orc = M.strehl(p_o, truth, a)
        assert abs(S_gpu - S_orc_on_gpu) < 1e-5, (S_gpu, S_orc_on_gpu)
        assert abs(S_gpu - S_orc) < TOL_S, (S_gpu, S_orc)
    assert s.frame_count() == nf


def test_teacher_forced_config1_frames():
    """N=256 streaming stand-in: each GPU frame starts from the oracle's state."""
    D = _ddh()
    torch = _torch()
    st = synth.config1_stream()
    N = 256
    prm, gp = make_pair(N, st.sigma_w2)
    a = O.aperture(N)
    s = D.Stream(N, gp)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(8):
        say(f"teacher-forced N=256 frame {n}")
        y = st.frame(n)
        s.set_state(dev(r_o, np.float32), dev(p_o, np.float32), n)
        # the oracle continues from the same float32-rounded state
        r_in, p_in = r_o.astype(np.float32).astype(np.float64), p_o.astype(np.float32).astype(np.float64)
        r_o, p_o = O.ddh_frame(r_in, p_in, y.astype(np.complex128), a, prm)
        s.step(dev(y))
        compare(f"frame {n}", *state(s), r_o, p_o, a)
    torch.cuda.synchronize()


def test_config1_150_frames_teacher_forced_and_free_running():
    """The streaming workload at full size (N = 256, D/r0 = 15, SNR 5,
    0.5 px per frame) over 150 frames, the horizon of the paper's Strehl
    claim.  Teacher-forced: every GPU frame starts from the oracle's previous
    state and must land within 1e-4 (e_r, e_phi) of the oracle's next state.
    Free-running: a second GPU stream runs all frames on its own, and its
    peak Strehl must stay within 0.005 of the free-running oracle's at every
    frame (the end-to-end pin of the streaming loop)."""
    D = _ddh()
    st = synth.config1_stream()
    N, nf = 256, 150
    prm, gp = make_pair(N, st.sigma_w2)
    a = O.aperture(N)
    tf = D.Stream(N, gp)      # teacher-forced
    fr = D.Stream(N, gp)      # free-running
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))      # oracle, re-rounded to FP32 each frame (teacher)
    r_f, p_f = np.zeros((N, N)), np.zeros((N, N))      # oracle, free-running in FP64
    worst_r = worst_p = worst_s = 0.0
    for n in range(nf):
        y = st.frame(n)
        yd = dev(y)
        yc = y.astype(np.complex128)
        tf.set_state(dev(r_o, np.float32), dev(p_o, np.float32), n)
        r_in, p_in = r_o.astype(np.float32).astype(np.float64), p_o.astype(np.float32).astype(np.float64)
        r_o, p_o = O.ddh_frame(r_in, p_in, yc, a, prm)
        r_f, p_f = O.ddh_frame(r_f, p_f, yc, a, prm)
        tf.step(yd)
        fr.step(yd)
        r_g, p_g = state(tf)
        er, ep = M.rel_l2(r_g, r_o), M.phase_rms_diff(p_g, p_o, a)
        truth = st.phase(n)
        s_gpu = fr.strehl(dev(truth, np.float32))
        s_orc = M.strehl(p_f, truth, a)
        worst_r, worst_p, worst_s = max(worst_r, er), max(worst_p, ep), max(worst_s, abs(s_gpu - s_orc))
        if n % 25 == 0 or n == nf - 1:
            say(f"config-1 frame {n}: e_r={er:.2e} e_phi={ep:.2e} S gpu {s_gpu:.4f} oracle {s_orc:.4f}")
        assert er < TOL_R and ep < TOL_PHI, (n, er, ep)
        assert np.all(p_g[a == 0] == 0.0)
        assert abs(s_gpu - s_orc) <= TOL_S, (n, s_gpu, s_orc)
    say(f"config-1 over {nf} frames: worst e_r {worst_r:.2e}, e_phi {worst_p:.2e}, |dS| {worst_s:.2e}")
    tf.close()
    fr.close()


def test_config0_em_iterations_and_cost():
    """Plain loop on one frame: DDH prologue then EM iterations; GPU FP64 cost
    is non-increasing (up to FP32 rounding of the state) and equals the
    oracle's cost at the GPU state."""
    D = _ddh()
    st = synth.config0_stream()
    N = 64
    prm, gp = make_pair(N, st.sigma_w2)
    a = O.aperture(N)
    y = st.frame(0)
    yc = y.astype(np.complex128)
    yh = O.normalize(yc)
    yd = dev(y)
    s = D.Stream(N, gp)
    r_o, p_o = O.ddh_frame(np.zeros((N, N)), np.zeros((N, N)), yc, a, prm)
    s.step(yd)
    U = [s.cost(yd)]
    errs = []
    for it in range(1, 200):
        r_o, p_o = O.em(r_o, p_o, yc, a, prm)
        s.em(yd)
        U.append(s.cost(yd))
        if it % 20 == 0 or it == 199:
            r_g, p_g = state(s)
            errs.append((it, M.rel_l2(r_g, r_o), M.phase_rms_diff(p_g, p_o, a)))
            u_orc = M.cost_U(r_g, p_g, yh, a, prm)
            assert abs(U[-1] - u_orc) < 1e-5 * abs(u_orc), (U[-1], u_orc)
    say("  (iter, e_r, e_phi):", [(i, f"{x:.1e}", f"{z:.1e}") for i, x, z in errs])
    U = np.array(U)
    inc = np.diff(U) / np.abs(U[1:])
    say(f"  U {U[0]:.3f} -> {U[-1]:.3f}, max relative increase {inc.max():.2e}")
    assert np.all(inc < 1e-6)
    for it, er, ep in errs:
        assert er < TOL_R and ep < TOL_PHI, (it, er, ep)


def test_cost_matches_oracle_on_random_state():
    D = _ddh()
    N = 128
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=10.0, snr=10.0, config_id=13))
    prm, gp = make_pair(N, st.sigma_w2)
    a = O.aperture(N)
    rng = np.random.default_rng(5)
    r = rng.uniform(0.05, 2.0, (N, N)).astype(np.float32)
    p = (a * rng.uniform(-3, 3, (N, N))).astype(np.float32)
    y = st.frame(0)
    s = D.Stream(N, gp)
    s.set_state(dev(r), dev(p), 0)
    u_gpu = s.cost(dev(y))
    u_orc = M.cost_U(r.astype(np.float64), p.astype(np.float64), O.normalize(y.astype(np.complex128)), a, prm)
    say(f"  U gpu {u_gpu:.6f} oracle {u_orc:.6f}")
    assert abs(u_gpu - u_orc) < 1e-5 * abs(u_orc)


# ----------------------------------------------------------------------------- variants and edges

def test_two_em_iterations_per_frame_and_smaller_pupil():
    D = _ddh()
    N = 128
    diam = 96.0
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0, snr=12.0, config_id=14))
    prm, gp = make_pair(N, st.sigma_w2, diameter=diam, n_k=2, beta_phi=1.5)
    a = O.aperture(N, diam)
    s = D.Stream(N, gp)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        say(f"n_k=2 pupil {diam} frame {n}")
        y = st.frame(n)
        r_o, p_o = O.ddh_frame(r_o, p_o, y.astype(np.complex128), a, prm)
        s.step(dev(y))
        compare(f"frame {n}", *state(s), r_o, p_o, a)


def test_conventional_dh_mbir_with_bootstrap_resets():
    """Conventional single-shot DH-MBIR (ddh_mbir), 50 EM iterations on one
    frame with a full (lambda = 1) bootstrap reset every 20, from r = phi = 0.

    * The loop's schedule: bit for bit the same as the explicit sequence of
      single calls (a one-iteration ddh_mbir is a reset, ddh_em a plain step).
    * Every iteration against the oracle's iteration from the same (float32)
      state (teacher forcing).  Free-running chains are not compared element
      by element: the cubic's choice among its roots is a floating-point
      decision, and at a near-tie FP32 and FP64 pick different roots at a
      pixel (measured: 1e-6 agreement right after each reset, a jump of 2e-2
      at one pixel by iteration 50), after which the chains part.
    * The free-running end state's Strehl against the oracle's within 0.005."""
    torch = _torch()
    D = _ddh()
    N = 64
    st = synth.config0_stream()
    prm, gp = make_pair(N, st.sigma_w2, lam=1.0)
    a = O.aperture(N)
    y = st.frame(0)
    yc, yd = y.astype(np.complex128), dev(y)
    z = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    s = D.Stream(N, gp)
    s.set_state(z, z, 0)
    s.mbir(yd, 50, 20)
    r_loop, p_loop = state(s)
    assert s.frame_count() == 1
    s.set_state(z, z, 0)
    worst = (0.0, 0.0)
    for it in range(50):
        r_in, p_in = state(s)
        if it % 20 == 0:
            s.mbir(yd, 1, 1)
            r_o, p_o = O.dh_mbir(yc, a, prm, iters=1, reset_every=1, r0=r_in, phi0=p_in)
        else:
            s.em(yd)
            r_o, p_o = O.em(r_in, p_in, yc, a, prm)
        r_g, p_g = state(s)
        er, ep = M.rel_l2(r_g, r_o), M.phase_rms_diff(p_g, p_o, a)
        worst = (max(worst[0], er), max(worst[1], ep))
        assert er < TOL_R and ep < TOL_PHI, (it, er, ep)
        assert np.all(p_g[a == 0] == 0.0)
    say(f"  teacher-forced worst e_r={worst[0]:.2e} e_phi={worst[1]:.2e}")
    np.testing.assert_array_equal(r_g, r_loop)
    np.testing.assert_array_equal(p_g, p_loop)
    r_o, p_o = O.dh_mbir(yc, a, prm, iters=50, reset_every=20)
    S_g = M.strehl(p_loop, st.phase(0), a)
    S_o = M.strehl(p_o, st.phase(0), a)
    say(f"  Strehl after 50 iterations: GPU {S_g:.4f} oracle {S_o:.4f}")
    assert abs(S_g - S_o) < TOL_S


def test_full_bootstrap_reset_makes_the_run_independent_of_r0():
    torch = _torch()
    D = _ddh()
    N = 64
    st = synth.config0_stream()
    _, gp = make_pair(N, st.sigma_w2, lam=1.0)
    y = dev(st.frame(0))
    rng = np.random.default_rng(4)
    phi0 = dev(O.remove_tiptilt(0.2 * rng.standard_normal((N, N)), O.aperture(N)), np.float32)
    outs = []
    for r0 in (np.zeros((N, N)), rng.uniform(0.1, 2.0, (N, N))):
        s = D.Stream(N, gp)
        s.set_state(dev(r0, np.float32), phi0, 0)
        s.mbir(y, 7, 3)
        outs.append(state(s))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    with pytest.raises(D.DDHError):
        s.mbir(y, -1, 3)
    with pytest.raises(D.DDHError):
        s.mbir(y, 5, 0)


def test_zero_phase_prior_weight():
    D = _ddh()
    N = 64
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=5.0, snr=20.0, config_id=15))
    prm, gp = make_pair(N, st.sigma_w2, beta_phi=0.0)
    a = O.aperture(N)
    s = D.Stream(N, gp)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        y = st.frame(n)
        r_o, p_o = O.ddh_frame(r_o, p_o, y.astype(np.complex128), a, prm)
        s.step(dev(y))
    r_g, p_g = state(s)
    assert M.rel_l2(r_g, r_o) < TOL_R
    # without the prior each phase lands on its own theta: compare modulo 2 pi
    d = O.wrap(p_g - p_o)[a > 0]
    d = d - d.mean()
    assert np.sqrt(np.mean(d * d)) < TOL_PHI


def test_quadratic_reflectance_prior():
    """q = p = 2 (the quadratic prior, edge weight independent of d): frames
    from the zero state, then one EM iteration from a state whose left half is
    constant (many neighbour differences exactly zero) against the oracle."""
    D = _ddh()
    torch = _torch()
    N = 64
    say("q = 2 frames and a flat-state EM iteration")
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=10.0, snr=10.0, speed=0.5, config_id=16))
    prm, gp = make_pair(N, st.sigma_w2, qg_q=2.0)
    a = O.aperture(N)
    s = D.Stream(N, gp)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        y = st.frame(n)
        r_o, p_o = O.ddh_frame(r_o, p_o, y.astype(np.complex128), a, prm)
        s.step(dev(y))
        compare(f"q=2 frame {n}", *state(s), r_o, p_o, a)
    rng = np.random.default_rng(16)
    r0 = np.full((N, N), 0.3, dtype=np.float32)
    r0[:, N // 2:] = rng.uniform(0.1, 1.0, (N, N - N // 2)).astype(np.float32)
    p0 = np.where(a > 0, rng.normal(0.0, 0.3, (N, N)), 0.0).astype(np.float32)
    s.set_state(dev(r0), dev(p0))
    y = st.frame(3)
    s.em(dev(y))
    r_o, p_o = O.em(r0.astype(np.float64), p0.astype(np.float64), y.astype(np.complex128), a, prm)
    compare("q=2 flat-state EM", *state(s), r_o, p_o, a)
    s.close()


def test_rejected_frame_leaves_state_unchanged():
    D = _ddh()
    torch = _torch()
    N = 64
    st = synth.config0_stream()
    prm, gp = make_pair(N, st.sigma_w2)
    s = D.Stream(N, gp)
    s.step(dev(st.frame(0)))
    assert s.status() == D.DDH_OK
    r0, p0 = state(s)
    const = dev(np.full((N, N), 3 - 2j, np.complex64))
    s.step(const)
    assert s.status() == D.DDH_EDATA
    r1, p1 = state(s)
    np.testing.assert_array_equal(r0, r1)
    np.testing.assert_array_equal(p0, p1)
    bad = st.frame(1)
    bad[5, 7] = np.nan
    s.step(dev(bad))
    assert s.status() == D.DDH_EDATA
    np.testing.assert_array_equal(state(s)[0], r0)
    s.step(dev(st.frame(2)))
    assert s.status() == D.DDH_OK
    torch.cuda.synchronize()


def test_resume_from_checkpoint_is_bitwise():
    D = _ddh()
    N = 128
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=10.0, snr=5.0, config_id=16))
    prm, gp = make_pair(N, st.sigma_w2)
    frames = [dev(st.frame(n)) for n in range(6)]
    a = D.Stream(N, gp)
    for y in frames:
        a.step(y)
    b = D.Stream(N, gp)
    for y in frames[:3]:
        b.step(y)
    r, p = b.reflectance(), b.phase()
    c = D.Stream(N, gp)
    c.set_state(r, p, 3)
    for y in frames[3:]:
        c.step(y)
    ra, pa = state(a)
    rc, pc = state(c)
    np.testing.assert_array_equal(ra, rc)
    np.testing.assert_array_equal(pa, pc)
    assert c.frame_count() == 6


def test_repeat_runs_are_bitwise_identical():
    D = _ddh()
    N = 256
    st = synth.config1_stream()
    prm, gp = make_pair(N, st.sigma_w2)
    frames = [dev(st.frame(n)) for n in range(3)]
    outs = []
    for _ in range(2):
        s = D.Stream(N, gp)
        for y in frames:
            s.step(y)
        outs.append(state(s))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


# ----------------------------------------------------------------------------- batches

def _mixed_specs():
    Ns = [128, 256, 64, 256, 512, 128, 64]
    return [synth.StreamSpec(N=N, d_over_r0=5.0 + 2 * i, snr=3.0 + i, speed=0.5, config_id=17, stream_id=i)
            for i, N in enumerate(Ns)]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_of_mixed_sizes_equals_streams_alone(graph):
    D = _ddh()
    specs = _mixed_specs()
    sims = [synth.Stream(sp) for sp in specs]
    pairs = [make_pair(sp.N, sm.sigma_w2) for sp, sm in zip(specs, sims)]
    frames = [[dev(sm.frame(n)) for n in range(3)] for sm in sims]
    alone = []
    for i, sp in enumerate(specs):
        s = D.Stream(sp.N, pairs[i][1])
        for y in frames[i]:
            s.step(y)
        alone.append(state(s))
    streams = [D.Stream(sp.N, pairs[i][1]) for i, sp in enumerate(specs)]
    b = D.Batch(streams, graph=graph)
    for n in range(3):
        say(f"batch graph={graph} frame {n}")
        b.step([frames[i][n] for i in range(len(specs))])
    for i, s in enumerate(streams):
        r, p = state(s)
        np.testing.assert_array_equal(r, alone[i][0])
        np.testing.assert_array_equal(p, alone[i][1])
        assert s.frame_count() == 3
    # and one member against the oracle
    i = 1
    N = specs[i].N
    a = O.aperture(N)
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        r_o, p_o = O.ddh_frame(r_o, p_o, sims[i].frame(n).astype(np.complex128), a, pairs[i][0])
    compare("batch member vs oracle", *alone[i], r_o, p_o, a)
    b.close()


def test_batch_of_mixed_pupil_diameters():
    """Streams of one N with different pupil diameters in one batch (each
    shape has its own pupil geometry table): equal to each stream alone, and
    the smaller pupil against the oracle."""
    D = _ddh()
    N = 128
    diams = [128, 96, 128, 96]
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0, snr=10.0, speed=0.5, config_id=17, stream_id=k))
            for k in range(len(diams))]
    pairs = [make_pair(N, sm.sigma_w2, diameter=d) for sm, d in zip(sims, diams)]
    frames = [[dev(sm.frame(n)) for n in range(3)] for sm in sims]
    alone = []
    for i in range(len(diams)):
        s = D.Stream(N, pairs[i][1])
        for y in frames[i]:
            s.step(y)
        alone.append(state(s))
        s.close()
    streams = [D.Stream(N, pairs[i][1]) for i in range(len(diams))]
    b = D.Batch(streams, graph=False)
    for n in range(3):
        say(f"mixed pupils frame {n}")
        b.step([frames[i][n] for i in range(len(diams))])
    for i, s in enumerate(streams):
        r, p = state(s)
        np.testing.assert_array_equal(r, alone[i][0])
        np.testing.assert_array_equal(p, alone[i][1])
    i = 1
    a = O.aperture(N, float(diams[i]))
    r_o, p_o = np.zeros((N, N)), np.zeros((N, N))
    for n in range(3):
        r_o, p_o = O.ddh_frame(r_o, p_o, sims[i].frame(n).astype(np.complex128), a, pairs[i][0])
    compare("96-px pupil in the batch vs oracle", *alone[i], r_o, p_o, a)
    b.close()
    for s in streams:
        s.close()


def test_batch_of_more_streams_than_one_launch_takes():
    """72 streams of N = 64 in one batch: the frame-start launch carries at
    most 64 streams' frame arguments, so the batch needs two of them; every
    stream equals the same stream stepped alone (eager and graph)."""
    D = _ddh()
    N, S = 64, 72
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0, snr=10.0, speed=0.5, config_id=18, stream_id=k))
            for k in range(S)]
    pairs = [make_pair(N, sm.sigma_w2) for sm in sims]
    frames = [[dev(sm.frame(n)) for n in range(2)] for sm in sims]
    alone = []
    for i in range(S):
        s = D.Stream(N, pairs[i][1])
        for y in frames[i]:
            s.step(y)
        alone.append(state(s))
        s.close()
    for graph in (False, True):
        say(f"{S} streams, graph={graph}")
        streams = [D.Stream(N, pairs[i][1]) for i in range(S)]
        b = D.Batch(streams, graph=graph)
        for n in range(2):
            b.step([frames[i][n] for i in range(S)])
        for i, s in enumerate(streams):
            r, p = state(s)
            np.testing.assert_array_equal(r, alone[i][0])
            np.testing.assert_array_equal(p, alone[i][1])
        b.close()
        for s in streams:
            s.close()


@pytest.mark.parametrize("N,S,F", [(64, 64, 24), (256, 64, 3), (512, 16, 3)])
def test_fused_statistics_pass_identical_over_many_frames(N, S, F):
    """The fused statistics + first row pass synchronises the blocks of each
    stream through device memory (XCD-local when the streams are a multiple
    of 8, device-coherent for a single stream): S streams over F frames in one
    batch (eager and HIP graph) equal every stream stepped alone, bit for bit,
    and no stream reports a wait that gave up."""
    D = _ddh()
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0, snr=8.0, speed=0.5, config_id=21, stream_id=k))
            for k in range(S)]
    pairs = [make_pair(N, sm.sigma_w2) for sm in sims]
    frames = [[dev(sm.frame(n)) for n in range(F)] for sm in sims]
    alone = []
    for i in range(S):
        s = D.Stream(N, pairs[i][1])
        for y in frames[i]:
            s.step(y)
        alone.append(state(s))
        s.close()
    for graph in (False, True):
        say(f"{S} streams x {F} frames, graph={graph}")
        streams = [D.Stream(N, pairs[i][1]) for i in range(S)]
        b = D.Batch(streams, graph=graph)
        for n in range(F):
            b.step([frames[i][n] for i in range(S)])
        for i, s in enumerate(streams):
            r, p = state(s)
            np.testing.assert_array_equal(r, alone[i][0], err_msg=f"stream {i}")
            np.testing.assert_array_equal(p, alone[i][1], err_msg=f"stream {i}")
        for i, s in enumerate(streams):
            assert s.status() == 0, f"stream {i}"
        b.close()
        for s in streams:
            s.close()


def test_batch_timing_mode_matches_graph():
    D = _ddh()
    specs = _mixed_specs()[:4]
    sims = [synth.Stream(sp) for sp in specs]
    pairs = [make_pair(sp.N, sm.sigma_w2) for sp, sm in zip(specs, sims)]
    frames = [[dev(sm.frame(n)) for n in range(2)] for sm in sims]
    res = []
    for timing in (False, True):
        streams = [D.Stream(sp.N, pairs[i][1]) for i, sp in enumerate(specs)]
        b = D.Batch(streams, graph=True)
        b.set_timing(timing)
        for n in range(2):
            b.step([frames[i][n] for i in range(len(specs))])
        if timing:
            t = b.stage_times()
            say("  stage times:", {k: round(v[0], 4) for k, v in t.items()})
            groups = len({sp.N for sp in specs})  # one launch per grid size per frame
            assert t["m_step"][1] == 2 * groups and t["col_fused"][1] == 2 * groups
        res.append([state(s) for s in streams])
        b.close()
    for (r0, p0), (r1, p1) in zip(*res):
        np.testing.assert_array_equal(r0, r1)
        np.testing.assert_array_equal(p0, p1)


def test_stage_times_are_kernel_durations_within_the_step():
    """Timing mode: each launch records its own kernel's start and end, so
    every launched kind has a positive time, and the timed kernels of a step
    add up to no more than the step's wall time on the device (they run one
    after another) and to most of it."""
    import torch
    D = _ddh()
    N, S = 256, 16
    sims = [synth.Stream(synth.StreamSpec(N=N, d_over_r0=8.0, snr=10.0, speed=0.5, config_id=19, stream_id=k))
            for k in range(S)]
    pairs = [make_pair(N, sm.sigma_w2) for sm in sims]
    frames = [[dev(sm.frame(n)) for n in range(2)] for sm in sims]
    streams = [D.Stream(N, pairs[i][1]) for i in range(S)]
    b = D.Batch(streams, graph=False)
    b.set_timing(True)
    for n in range(2):  # warm-up
        b.step([frames[i][n % 2] for i in range(S)])
    b.stage_times()
    b.set_timing(True)  # clears the sums
    steps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for n in range(steps):
        b.step([frames[i][n % 2] for i in range(S)])
    e1.record()
    torch.cuda.synchronize()
    wall = e0.elapsed_time(e1)
    t = b.stage_times()
    b.close()
    for s in streams:
        s.close()
    launched = {k: v for k, v in t.items() if v[1]}
    say("  stage times (ms):", {k: round(v[0], 4) for k, v in launched.items()}, "wall", round(wall, 4))
    assert {"stats_row_ifft", "col_fused", "row_fft", "m_step"} <= set(launched)
    assert all(v[1] == steps for v in launched.values())
    assert all(v[0] > 0.0 for v in launched.values())
    total = sum(v[0] for v in launched.values())
    assert total <= wall * 1.02, (total, wall)
    assert total >= 0.3 * wall, (total, wall)


def test_statistics_form_follows_the_lane_rule():
    """Timing mode shows which form of the frame statistics a batch uses:
    one lane forms them in the first row pass (stats_row_ifft); several
    lanes launched eagerly use a statistics launch before the first row
    pass (stats, row_ifft).  Both give the same states."""
    D = _ddh()
    specs = _mixed_specs()[:4]
    sims = [synth.Stream(sp) for sp in specs]
    pairs = [make_pair(sp.N, sm.sigma_w2) for sp, sm in zip(specs, sims)]
    frames = [[dev(sm.frame(n)) for n in range(2)] for sm in sims]
    res, kinds = [], []
    for lanes in (1, 0):
        streams = [D.Stream(sp.N, pairs[i][1]) for i, sp in enumerate(specs)]
        b = D.Batch(streams, graph=False, lanes=lanes)
        b.set_timing(True)
        for n in range(2):
            b.step([frames[i][n] for i in range(len(specs))])
        t = b.stage_times()
        kinds.append({k for k, v in t.items() if v[1]})
        res.append([state(s) for s in streams])
        b.close()
        for s in streams:
            s.close()
    say("  launched kinds:", kinds)
    assert "stats_row_ifft" in kinds[0] and "stats" not in kinds[0]
    assert "stats" in kinds[1] and "stats_row_ifft" not in kinds[1]
    for (r0, p0), (r1, p1) in zip(*res):
        np.testing.assert_array_equal(r0, r1)
        np.testing.assert_array_equal(p0, p1)


def test_full_size_batch_sampled_against_oracle():
    """64 streams x N=256 batched, as timed by the benchmark; two sampled
    streams are checked against the oracle frame by frame."""
    D = _ddh()
    specs = synth.batch_specs(uniform_N=256, count=64, config_id=2)
    sims = [synth.Stream(sp) for sp in specs]
    pairs = [make_pair(sp.N, sm.sigma_w2) for sp, sm in zip(specs, sims)]
    streams = [D.Stream(sp.N, pairs[i][1]) for i, sp in enumerate(specs)]
    b = D.Batch(streams, graph=True)
    sample = [0, 37]
    a = O.aperture(256)
    orc = {i: (np.zeros((256, 256)), np.zeros((256, 256))) for i in sample}
    for n in range(3):
        say(f"full-size batch frame {n}")
        ys = [dev(sm.frame(n)) for sm in sims]
        b.step(ys)
        for i in sample:
            orc[i] = O.ddh_frame(*orc[i], sims[i].frame(n).astype(np.complex128), a, pairs[i][0])
            compare(f"stream {i} frame {n}", *state(streams[i]), *orc[i], a)
    b.close()


def test_full_size_mixed_batch_sampled_against_oracle():
    """The uneven batch as timed by the benchmark's mixed workload (64 streams,
    N in {128, 256, 512} at 2:5:1, one lane per N, eager): one sampled stream
    of each size against the oracle frame by frame."""
    D = _ddh()
    specs = synth.batch_specs(count=64, config_id=2)
    sims = [synth.Stream(sp) for sp in specs]
    pairs = [make_pair(sp.N, sm.sigma_w2) for sp, sm in zip(specs, sims)]
    streams = [D.Stream(sp.N, pairs[i][1]) for i, sp in enumerate(specs)]
    b = D.Batch(streams, graph=False)
    sample = [next(i for i, sp in enumerate(specs) if sp.N == n) for n in (128, 256, 512)]
    orc = {i: (np.zeros((specs[i].N,) * 2), np.zeros((specs[i].N,) * 2)) for i in sample}
    for n in range(2):
        say(f"full-size mixed batch frame {n}")
        b.step([dev(sm.frame(n)) for sm in sims])
        for i in sample:
            a = O.aperture(specs[i].N)
            orc[i] = O.ddh_frame(*orc[i], sims[i].frame(n).astype(np.complex128), a, pairs[i][0])
            compare(f"stream {i} N={specs[i].N} frame {n}", *state(streams[i]), *orc[i], a)
    b.close()


# ----------------------------------------------------------------------------- tiling

def _run_frames(D, N, gp, frames):
    s = D.Stream(N, gp)
    for y in frames:
        s.step(y)
    return state(s)


@pytest.mark.parametrize("N", [64, 256, 512])
def test_tilings_give_bitwise_identical_results(N):
    D = _ddh()
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=10.0, snr=6.0, config_id=18))
    _, gp = make_pair(N, st.sigma_w2)
    frames = [dev(st.frame(n)) for n in range(3)]
    saved = D.get_tiles(N)
    cfgs = [(4, 4, 16, 16), (8, 32, 16, 64), (32, 8, 32, 32), (16, 16, 32, 64), (4, 8, 64, 64), (8, 8, 32, 128),
            (16, 16, 0, 0)]
    ref = None
    try:
        for cfg in cfgs:
            if cfg[2] > N or cfg[3] > N:
                continue
            say(f"tiles N={N} cfg={cfg}")
            D.set_tiles(N, cfg)
            out = _run_frames(D, N, gp, frames)
            if ref is None:
                ref = out
            else:
                np.testing.assert_array_equal(out[0], ref[0])
                np.testing.assert_array_equal(out[1], ref[1])
    finally:
        D.set_tiles(N, saved)


def test_autotune_installs_a_valid_tiling():
    D = _ddh()
    N = 128
    cfg, us = D.autotune(N, 8)
    say(f"  autotune N={N}: cfg={cfg} us={us}")
    assert D.get_tiles(N) == cfg
    assert all(u > 0 for u in (us[0], us[1], us[3]))
    with pytest.raises(D.DDHError):
        D.set_tiles(N, (3, 8, 16, 16))


def test_autotune_mix_installs_valid_tilings():
    D = _ddh()
    sizes = [64] * 4 + [128] * 2
    before = {n: D.get_tiles(n) for n in (64, 128)}
    cfgs, us = D.autotune_mix(sizes)
    say(f"  autotune_mix: {cfgs} step {us:.1f} us")
    try:
        assert sorted(cfgs) == [64, 128] and us > 0
        for n, c in cfgs.items():
            assert D.get_tiles(n) == c
    finally:
        for n, c in before.items():
            D.set_tiles(n, c)


@pytest.mark.parametrize("lanes,graph", [(0, False), (0, True), (2, False), (3, True), (4, True)])
def test_batch_lanes_equal_single_lane(lanes, graph):
    """lanes 0 is one lane per distinct N (the default), n >= 1 pixel-balanced"""
    D = _ddh()
    specs = _mixed_specs()
    sims = [synth.Stream(sp) for sp in specs]
    pairs = [make_pair(sp.N, sm.sigma_w2) for sp, sm in zip(specs, sims)]
    frames = [[dev(sm.frame(n)) for n in range(3)] for sm in sims]
    res = []
    for nl in (1, lanes):
        say(f"lanes={nl} graph={graph}")
        streams = [D.Stream(sp.N, pairs[i][1]) for i, sp in enumerate(specs)]
        b = D.Batch(streams, graph=graph, lanes=nl)
        for n in range(3):
            b.step([frames[i][n] for i in range(len(specs))])
        res.append([state(s) for s in streams])
        b.close()
    for (r0, p0), (r1, p1) in zip(*res):
        np.testing.assert_array_equal(r0, r1)
        np.testing.assert_array_equal(p0, p1)
