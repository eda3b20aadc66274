"""Seeded synthetic inputs for Dynamic DH-MBIR (arXiv 2305.03284).

This module only *simulates data*: reflectance targets, frozen-flow phase
screens, speckle and noise, and the digital-holography frames built from them
(Forward Model section, Eq. (1); Experimental Results, Data Simulation).  It
holds none of the reconstruction arithmetic (no Normalize, no back-projection,
no EM), and it is the one module that both the FP64 oracle tests and the GPU
path's tests/benchmarks draw inputs from.

Stand-ins (the paper's own inputs are not available):
  * reflectance: seeded ellipses/rectangles on a 0.1 background, blurred with a
    1-px Gaussian, in place of the 1951 USAF chart (Data Simulation);
  * phase: a Kolmogorov FFT screen of size 2N x 2N translated by a Fourier
    shift each frame ("frozen flow", Data Simulation), with piston, tip and
    tilt removed over the pupil as the paper does for its ground truth.

Seeds: ``Generator(PCG64(SeedSequence([config_id, stream_id, purpose])))`` with
purpose 0 = screen, 1 = flow direction, 2 = reflectance, 3 = speckle/noise
(frame n uses SeedSequence([config_id, stream_id, 3, n])), 4 = per-stream
draws (D/r0, SNR).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PURPOSE_SCREEN = 0
PURPOSE_FLOW = 1
PURPOSE_REFLECTANCE = 2
PURPOSE_FRAME = 3
PURPOSE_DRAWS = 4


def rng_for(config_id: int, stream_id: int, purpose: int, *extra: int) -> np.random.Generator:
    """Counter-style seeded generator: one independent stream per purpose."""
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([config_id, stream_id, purpose, *extra])))


def aperture(N: int, diameter: float | None = None) -> np.ndarray:
    """Binary circular camera aperture (the diagonal of D_a, Forward Model).

    Pixel (i, j) is inside when its distance from the grid centre
    ((N-1)/2, (N-1)/2) is at most diameter/2.  Default diameter: N.
    """
    d = float(N if diameter is None else diameter)
    c = 0.5 * (N - 1)
    ii = np.arange(N, dtype=np.float64)[:, None] - c
    jj = np.arange(N, dtype=np.float64)[None, :] - c
    return ((ii * ii + jj * jj) <= 0.25 * d * d).astype(np.float64)


def flow_speed(f_g: float, f_s: float, N: int, d_over_r0: float) -> float:
    """Frozen-flow displacement in pixels per sample (Data Simulation):
    ||v|| = (1/0.43) * (f_g/f_s) * N / (D/r0)."""
    return (1.0 / 0.43) * (f_g / f_s) * N / d_over_r0


def _remove_plane_truth(phi: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Remove piston, tip and tilt of the ground-truth phase over the pupil by
    unweighted least squares (Data Simulation: only higher-order aberrations
    are kept).  Off-pupil values are set to zero."""
    N = phi.shape[0]
    c = 0.5 * (N - 1)
    ii, jj = np.nonzero(a > 0)
    basis = np.stack([np.ones(ii.size), ii - c, jj - c], axis=1)
    coef, *_ = np.linalg.lstsq(basis, phi[ii, jj], rcond=None)
    out = np.zeros_like(phi)
    out[ii, jj] = phi[ii, jj] - basis @ coef
    return out


def kolmogorov_spectrum(S: int, r0_px: float, rng: np.random.Generator) -> np.ndarray:
    """Spectrum of a periodic S x S Kolmogorov phase screen (radians).

    Seeded circular complex white noise filtered by sqrt(PSD), with the
    Kolmogorov phase PSD 0.023 r0^(-5/3) f^(-11/3) (f in cycles/px, DC zeroed).
    The screen is Re(sum_k W_k sqrt(PSD_k) df exp(2 pi i k.x / S)).
    """
    f = np.fft.fftfreq(S)  # cycles per pixel
    fx, fy = np.meshgrid(f, f, indexing="ij")
    fr = np.sqrt(fx * fx + fy * fy)
    psd = np.zeros_like(fr)
    nz = fr > 0
    psd[nz] = 0.023 * r0_px ** (-5.0 / 3.0) * fr[nz] ** (-11.0 / 3.0)
    df = 1.0 / S
    w = (rng.standard_normal((S, S)) + 1j * rng.standard_normal((S, S)))
    return w * np.sqrt(psd) * df


def screen_from_spectrum(spec: np.ndarray, shift=(0.0, 0.0)) -> np.ndarray:
    """Real phase screen from its spectrum, translated by ``shift`` pixels
    (row, col) with a Fourier shift (exact for the periodic screen)."""
    S = spec.shape[0]
    f = np.fft.fftfreq(S)
    ramp = np.exp(-2j * np.pi * (f[:, None] * shift[0] + f[None, :] * shift[1]))
    return np.real(np.fft.ifft2(spec * ramp) * (S * S))


def reflectance(N: int, rng: np.random.Generator, n_shapes: int | None = None) -> np.ndarray:
    """Stand-in target reflectance r in [0.1, 1] (Data Simulation uses the
    USAF chart, which is not available).

    Background 0.1; 3-5 shapes (ellipse or rotated rectangle) with centres in
    U[0.15N, 0.85N], half-sizes U[0.05N, 0.25N], angle U[0, pi), value
    U[0.1, 1], later shapes painted over earlier ones; periodic Gaussian blur
    with sigma = 1 px; clipped to [0.1, 1].
    """
    k = int(rng.integers(3, 6)) if n_shapes is None else int(n_shapes)
    img = np.full((N, N), 0.1)
    ii, jj = np.mgrid[0:N, 0:N].astype(np.float64)
    for _ in range(k):
        kind = int(rng.integers(0, 2))
        ci, cj = rng.uniform(0.15 * N, 0.85 * N, size=2)
        hi, hj = rng.uniform(0.05 * N, 0.25 * N, size=2)
        ang = rng.uniform(0.0, np.pi)
        val = rng.uniform(0.1, 1.0)
        ca, sa = math.cos(ang), math.sin(ang)
        u = (ii - ci) * ca + (jj - cj) * sa
        v = -(ii - ci) * sa + (jj - cj) * ca
        if kind == 0:
            m = (u / hi) ** 2 + (v / hj) ** 2 <= 1.0
        else:
            m = (np.abs(u) <= hi) & (np.abs(v) <= hj)
        img[m] = val
    f = np.fft.fftfreq(N)
    g = np.exp(-2.0 * (np.pi ** 2) * (f[:, None] ** 2 + f[None, :] ** 2))  # sigma = 1 px
    img = np.real(np.fft.ifft2(np.fft.fft2(img) * g))
    return np.clip(img, 0.1, 1.0)


def sigma_w2_normalized(fill: float, snr: float) -> float:
    """Noise variance after Normalize (Eq. (4)) for the simulator's SNR.

    SNR (linear) = expected pupil signal power / raw noise variance; the noise
    covers the whole N x N grid, so the mean power of y is
    sigma_raw^2 (fill*SNR + 1) and Normalize makes it 1.
    """
    return 1.0 / (fill * snr + 1.0)


def hologram(r: np.ndarray, phi: np.ndarray, a: np.ndarray, snr: float,
             rng: np.random.Generator, noise_rng: np.random.Generator | None = None) -> np.ndarray:
    """One DH frame y = a * exp(j phi) * F g + w (Eq. (1) with the isoplanatic
    operator, Fresnel factor taken as identity).

    g ~ CN(0, diag r) (Forward Model: reflection coefficients are circular
    Gaussians with variance r); F is the unitary 2D DFT; w ~ CN(0, s2 I) on the
    whole grid with s2 = mean(r)/SNR, the expected per-pixel pupil signal power
    divided by the (linear) SNR.  ``noise_rng`` (default: ``rng``) draws w.
    """
    N = r.shape[0]
    noise_rng = rng if noise_rng is None else noise_rng
    g = np.sqrt(r / 2.0) * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    field = a * np.exp(1j * phi) * np.fft.fft2(g, norm="ortho")
    s2 = float(np.mean(r)) / snr
    w = np.sqrt(s2 / 2.0) * (noise_rng.standard_normal((N, N)) + 1j * noise_rng.standard_normal((N, N)))
    return field + w


@dataclasses.dataclass
class StreamSpec:
    """One synthetic stream: grid size, turbulence, SNR and flow."""
    N: int
    d_over_r0: float
    snr: float
    speed: float = 0.5           # px per timestep
    direction: float | None = None  # radians; None = seeded
    config_id: int = 1
    stream_id: int = 0
    frozen_speckle: bool = False


class Stream:
    """Frozen-flow stream: truth phase per frame, static reflectance, frames.

    The 2N x 2N screen is drawn once; frame n crops its top-left N x N corner
    after translating it by n * v, then removes piston/tip/tilt over the pupil.
    Speckle and noise are redrawn every frame (or frozen when requested).
    """

    def __init__(self, spec: StreamSpec):
        self.spec = spec
        N = spec.N
        self.a = aperture(N)
        self.fill = float(self.a.sum()) / (N * N)
        S = 2 * N
        r0_px = N / spec.d_over_r0
        self._spec_screen = kolmogorov_spectrum(
            S, r0_px, rng_for(spec.config_id, spec.stream_id, PURPOSE_SCREEN))
        ang = spec.direction
        if ang is None:
            ang = float(rng_for(spec.config_id, spec.stream_id, PURPOSE_FLOW).uniform(0, 2 * np.pi))
        self.v = (spec.speed * math.cos(ang), spec.speed * math.sin(ang))
        self.r = reflectance(N, rng_for(spec.config_id, spec.stream_id, PURPOSE_REFLECTANCE))
        self.sigma_w2 = sigma_w2_normalized(self.fill, spec.snr)

    def phase(self, n: int) -> np.ndarray:
        N = self.spec.N
        scr = screen_from_spectrum(self._spec_screen, (n * self.v[0], n * self.v[1]))
        return _remove_plane_truth(scr[:N, :N], self.a)

    def frame(self, n: int, phi: np.ndarray | None = None) -> np.ndarray:
        """complex64-rounded frame n (the GPU's input precision); the oracle
        reads the same rounded values upcast to complex128."""
        if phi is None:
            phi = self.phase(n)
        rng = rng_for(self.spec.config_id, self.spec.stream_id, PURPOSE_FRAME, n)
        if self.spec.frozen_speckle:
            # speckle drawn once (counter 0), noise fresh per frame
            speck = rng_for(self.spec.config_id, self.spec.stream_id, PURPOSE_FRAME, 0, 0)
            y = hologram(self.r, phi, self.a, self.spec.snr, speck, noise_rng=rng)
        else:
            y = hologram(self.r, phi, self.a, self.spec.snr, rng)
        return y.astype(np.complex64)


def config0_stream() -> Stream:
    """Single-frame correctness case: N=64, pupil 64 px, D/r0=10, SNR=10."""
    return Stream(StreamSpec(N=64, d_over_r0=10.0, snr=10.0, speed=0.0, direction=0.0,
                             config_id=0, stream_id=0))


def config1_stream(N: int = 256, stream_id: int = 0) -> Stream:
    """Streaming case: N=256 (default), D/r0=15, 0.5 px/step, SNR=5."""
    return Stream(StreamSpec(N=N, d_over_r0=15.0, snr=5.0, speed=0.5, config_id=1,
                             stream_id=stream_id))


def batch_specs(sizes_ratio=((128, 2), (256, 5), (512, 1)), count: int = 64,
                config_id: int = 2, uniform_N: int | None = None) -> list[StreamSpec]:
    """Batched case: ``count`` independent streams, D/r0 ~ U[5,20] and
    SNR ~ U[2,20] per stream, 0.5 px/step.  With ``uniform_N`` all streams
    share one size; otherwise sizes follow ``sizes_ratio`` and are shuffled
    by seed."""
    if uniform_N is not None:
        Ns = [uniform_N] * count
    else:
        tot = sum(w for _, w in sizes_ratio)
        Ns = []
        for n, w in sizes_ratio:
            Ns += [n] * (count * w // tot)
        Ns += [sizes_ratio[1][0]] * (count - len(Ns))
        perm = rng_for(config_id, 0, PURPOSE_DRAWS, 999).permutation(len(Ns))
        Ns = [Ns[i] for i in perm]
    specs = []
    for sid, N in enumerate(Ns):
        d = rng_for(config_id, sid, PURPOSE_DRAWS)
        specs.append(StreamSpec(N=N, d_over_r0=float(d.uniform(5, 20)),
                                snr=float(d.uniform(2, 20)), speed=0.5,
                                config_id=config_id, stream_id=sid))
    return specs


DEFAULT_PARAMS = dict(
    lam=0.45, alpha=0.025, n_k=1,            # Eq. (3) and Fig. 1; values from the paper
    qg_p=2.0, qg_q=1.2, qg_T=0.1, qg_sigma=0.2,  # QGGMRF on r
    beta_phi=0.5,                             # GMRF weight on phi
    r_floor=1e-8,
)
