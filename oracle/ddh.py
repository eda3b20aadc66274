"""FP64 CPU oracle of the Dynamic DH-MBIR per-frame step (arXiv 2305.03284).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU path
(no kernels, headers, tables or helpers) and the GPU path never calls it.

Plain NumPy in float64.  Every operation is written the way the paper (or the
reading recorded next to it) defines it, with no blocking, fusion or
reordering: a colour pass updates all pixels of one colour at once, which is
exactly the sequential coordinate-descent sweep because no two pixels of one
colour are 8-neighbours.

Model (Forward Model section, Eq. (1)):  y = A_phi g + w,
  A_phi = D_a D(exp(j phi)) F Gamma,   g ~ CN(0, diag r),   w ~ CN(0, s2 I),
with F the unitary ("normalized") 2D DFT and Gamma = I (a diagonal unimodular
factor does not change the law of the circular g, so r and phi estimates do
not depend on it).

EM (DH-MBIR section: EM by iterative surrogate minimisation of the joint MAP
cost Eq. (2)).  The E-step uses the diagonal approximation A^H A ~ I, which
makes it exact EM for the model b(phi) = A_phi^H y = g + w~, w~ ~ CN(0, s2 I):
  E-step:   w = r/(r+s2),  mu = w b,  C = s2 w,  s = C + |mu|^2
  r M-step: one 4-colour ICD sweep on log r + s/r + QGGMRF prior, with the
            symmetric-bound quadratic surrogate of the prior at each pass;
  phi M-step: one 4-colour sweep on -sum c cos(phi - theta) + GMRF prior,
            with the quadratic majoriser of -cos.
The cost this EM does not increase is ``cost_U`` below.

Readings where the paper is silent (each also listed in the design notes):
  * colours: colour(i, j) = (i mod 2) + 2 (j mod 2), i = row, order 0,1,2,3;
  * 8-neighbour weights 1/6 (edges) and 1/12 (diagonals); r uses a free
    boundary (no wrap), phi only counts neighbours inside the pupil;
  * QGGMRF rho(d) = |d|^p / (p sig^p) / (1 + |d/(T sig)|^(p-q));
  * r update = global minimiser of the 1-D surrogate among the positive roots
    of its stationarity cubic; exact ties take the smaller root; floor r_floor;
  * RemoveTipTilt = unweighted least-squares plane over pupil pixels
    (piston included), off-pupil phase = 0;
  * Normalize uses p = N^2 entries (noise lives on the whole grid).
"""
from __future__ import annotations

import dataclasses

import numpy as np

# 8-neighbourhood: (di, dj, weight).  Edge neighbours 1/6, diagonals 1/12.
NEIGHBOURS = (
    (-1, 0, 1.0 / 6.0), (1, 0, 1.0 / 6.0), (0, -1, 1.0 / 6.0), (0, 1, 1.0 / 6.0),
    (-1, -1, 1.0 / 12.0), (-1, 1, 1.0 / 12.0), (1, -1, 1.0 / 12.0), (1, 1, 1.0 / 12.0),
)
# each unordered neighbour pair once
HALF_NEIGHBOURS = ((0, 1, 1.0 / 6.0), (1, 0, 1.0 / 6.0), (1, 1, 1.0 / 12.0), (1, -1, 1.0 / 12.0))


@dataclasses.dataclass
class Params:
    """Algorithm parameters.  lam, alpha: Eq. (3) (paper values 0.45, 0.025);
    n_k: EM iterations per frame (Fig. 1); sigma_w2: noise variance in
    Normalize units; QGGMRF (p, q, T, sigma) on r; beta_phi: GMRF weight on
    phi; r_floor: positivity floor on r."""
    sigma_w2: float
    lam: float = 0.45
    alpha: float = 0.025
    n_k: int = 1
    qg_p: float = 2.0
    qg_q: float = 1.2
    qg_T: float = 0.1
    qg_sigma: float = 0.2
    beta_phi: float = 0.5
    r_floor: float = 1e-8


# ----------------------------------------------------------------------------
# Operators (Forward Model section)
# ----------------------------------------------------------------------------

def aperture(N: int, diameter: float | None = None) -> np.ndarray:
    """Circular pupil a: 1 where the distance to ((N-1)/2, (N-1)/2) is at most
    diameter/2 (default diameter N)."""
    d = float(N if diameter is None else diameter)
    c = (N - 1) / 2.0
    i, j = np.meshgrid(np.arange(N) - c, np.arange(N) - c, indexing="ij")
    return (i ** 2 + j ** 2 <= (d / 2.0) ** 2).astype(np.float64)


def F(x: np.ndarray) -> np.ndarray:
    """Unitary forward 2D DFT, kernel exp(-2 pi i k.n / N), scale 1/N."""
    return np.fft.fft2(x, norm="ortho")


def FH(x: np.ndarray) -> np.ndarray:
    """Adjoint (= inverse) of F."""
    return np.fft.ifft2(x, norm="ortho")


def back_project(yhat: np.ndarray, phi: np.ndarray, a: np.ndarray) -> np.ndarray:
    """b = A_phi^H yhat = F^H (a exp(-j phi) yhat) (Gamma = I, a real)."""
    return FH(a * np.exp(-1j * phi) * yhat)


# ----------------------------------------------------------------------------
# Frame prologue (Dynamic DH-MBIR section, Fig. 1, Eq. (3), Eq. (4))
# ----------------------------------------------------------------------------

def normalize(y: np.ndarray) -> np.ndarray:
    """Eq. (4): sqrt(p) (y - mu)/||y - mu||, mu = mean of y, p = number of
    entries.  Raises ValueError when ||y - mu|| is zero or not finite."""
    d = y - y.mean()
    nrm = np.linalg.norm(d)
    if not np.isfinite(nrm) or nrm == 0.0:
        raise ValueError("Normalize undefined: ||y - mean(y)|| is zero or not finite")
    return np.sqrt(y.size) * d / nrm


def remove_tiptilt(phi: np.ndarray, a: np.ndarray) -> np.ndarray:
    """RemoveTipTilt: subtract the least-squares plane c0 + c1 x + c2 y fitted
    over the pupil pixels (coordinates centred on the grid centre); phase
    off the pupil is zero."""
    N = phi.shape[0]
    c = (N - 1) / 2.0
    ii, jj = np.nonzero(a > 0)
    X = np.column_stack([np.ones(ii.size), ii - c, jj - c])
    coef = np.linalg.lstsq(X, phi[ii, jj], rcond=None)[0]
    out = np.zeros_like(phi, dtype=np.float64)
    out[ii, jj] = phi[ii, jj] - X @ coef
    return out


def r_init(r_prev: np.ndarray, b: np.ndarray, lam: float, alpha: float,
           r_floor: float) -> np.ndarray:
    """Eq. (3): (1 - lam) r_prev + lam alpha |A^H y|^2, floored at r_floor."""
    return np.maximum((1.0 - lam) * r_prev + lam * alpha * np.abs(b) ** 2, r_floor)


# ----------------------------------------------------------------------------
# E-step
# ----------------------------------------------------------------------------

def e_step(r: np.ndarray, b: np.ndarray, s2: float):
    """Posterior of g given b = g + w~: mean mu, variance C and second moment
    s = E|g|^2 (pointwise under A^H A ~ I)."""
    w = r / (r + s2)
    mu = w * b
    C = s2 * w
    s = C + np.abs(mu) ** 2
    return mu, C, s


# ----------------------------------------------------------------------------
# QGGMRF prior on r
# ----------------------------------------------------------------------------

def qggmrf_rho(d, p, q, T, sig):
    """rho(d) = |d|^p / (p sig^p) * 1 / (1 + |d/(T sig)|^(p-q))."""
    ad = np.abs(d)
    return ad ** p / (p * sig ** p) / (1.0 + (ad / (T * sig)) ** (p - q))


def qggmrf_weight(d, p, q, T, sig):
    """rho'(d)/d = |d|^(p-2)/sig^p * (1 + (q/p) v)/(1 + v)^2, v = |d/(T sig)|^(p-q).
    (derivative of qggmrf_rho; equals 1/sig^2 at d = 0 when p = 2)."""
    ad = np.abs(d)
    v = (ad / (T * sig)) ** (p - q)
    return ad ** (p - 2.0) / sig ** p * (1.0 + (q / p) * v) / (1.0 + v) ** 2


def colour_map(N: int) -> np.ndarray:
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return (i % 2) + 2 * (j % 2)


def _neighbour(x: np.ndarray, di: int, dj: int):
    """Value of the (di, dj) neighbour of every pixel and whether it exists
    (free boundary: no wrap)."""
    N0, N1 = x.shape
    out = np.zeros_like(x)
    ok = np.zeros(x.shape, dtype=bool)
    i0, i1 = max(0, -di), min(N0, N0 - di)
    j0, j1 = max(0, -dj), min(N1, N1 - dj)
    out[i0:i1, j0:j1] = x[i0 + di:i1 + di, j0 + dj:j1 + dj]
    ok[i0:i1, j0:j1] = True
    return out, ok


def surrogate_h(rho, s, A, B):
    """1-D surrogate of the r M-step for one pixel, up to a constant:
    log rho + s/rho + sum_j (w_j/2)(rho - r_j)^2
      = log rho + s/rho + (A/2) rho^2 - B rho + const,
    A = sum_j w_j, B = sum_j w_j r_j."""
    return np.log(rho) + s / rho + 0.5 * A * rho ** 2 - B * rho


def solve_pixel_r(s: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Global minimiser on (0, inf) of surrogate_h, for arrays of pixels.

    Stationarity: h'(rho) rho^2 = A rho^3 - B rho^2 + rho - s = 0.  The roots
    are the eigenvalues of the companion matrix (a library primitive).  The
    global minimum is a positive real root, so taking the minimum of h over the
    positive real parts of all three eigenvalues returns it; exact ties take the
    smaller root.  A = 0 (no prior) gives rho = s.
    """
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    noprior = A <= 0
    out[noprior] = s[noprior]
    m = ~noprior
    if np.any(m):
        a3, b3, s3 = A[m], B[m], s[m]
        comp = np.zeros((a3.size, 3, 3))
        comp[:, 0, 0] = b3 / a3
        comp[:, 0, 1] = -1.0 / a3
        comp[:, 0, 2] = s3 / a3
        comp[:, 1, 0] = 1.0
        comp[:, 2, 1] = 1.0
        roots = np.linalg.eigvals(comp).real          # (n, 3)
        # two guarded Newton polishes on the cubic (reduce eigen-solver error)
        for _ in range(2):
            f = ((a3[:, None] * roots - b3[:, None]) * roots + 1.0) * roots - s3[:, None]
            fp = (3.0 * a3[:, None] * roots - 2.0 * b3[:, None]) * roots + 1.0
            step = np.where(fp != 0, f / np.where(fp != 0, fp, 1.0), 0.0)
            cand = roots - step
            fc = ((a3[:, None] * cand - b3[:, None]) * cand + 1.0) * cand - s3[:, None]
            roots = np.where(np.abs(fc) < np.abs(f), cand, roots)
        roots = np.sort(roots, axis=1)
        h = np.where(roots > 0,
                     surrogate_h(np.where(roots > 0, roots, 1.0), s3[:, None], a3[:, None], b3[:, None]),
                     np.inf)
        k = np.argmin(h, axis=1)                      # first minimum = smaller root
        out[m] = roots[np.arange(roots.shape[0]), k]
    return out


def r_m_step(r: np.ndarray, s: np.ndarray, prm: Params) -> np.ndarray:
    """One 4-colour ICD sweep of the r M-step.

    Pass k updates every colour-k pixel from the current r: edge weights
    w_ij = b_ij rho'(r_i - r_j)/(r_i - r_j) (symmetric bound of the QGGMRF
    prior at the current values), then the global minimiser of
    log rho + s_i/rho + sum_j (w_ij/2)(rho - r_j)^2, floored at r_floor.
    """
    r = r.astype(np.float64, copy=True)
    col = colour_map(r.shape[0])
    for k in range(4):
        A = np.zeros_like(r)
        B = np.zeros_like(r)
        for di, dj, bij in NEIGHBOURS:
            rj, ok = _neighbour(r, di, dj)
            w = np.where(ok, bij * qggmrf_weight(r - rj, prm.qg_p, prm.qg_q, prm.qg_T, prm.qg_sigma), 0.0)
            A += w
            B += w * rj
        sel = col == k
        new = solve_pixel_r(s[sel], A[sel], B[sel])
        r[sel] = np.maximum(new, prm.r_floor)
    return r


# ----------------------------------------------------------------------------
# phi M-step
# ----------------------------------------------------------------------------

def wrap(x):
    """Wrap to [-pi, pi)."""
    return np.mod(x + np.pi, 2.0 * np.pi) - np.pi


def phi_data_terms(yhat: np.ndarray, z: np.ndarray, a: np.ndarray, s2: float):
    """Per-pixel data term of the phi M-step.  The expected complete-data
    log-likelihood depends on phi only through -2 Re(yhat^H A_phi mu)/s2, i.e.
    -sum_i c_i cos(phi_i - theta_i) with c = (2/s2) a |yhat| |z|,
    theta = arg(yhat conj(z)), z = F mu."""
    c = (2.0 / s2) * a * np.abs(yhat) * np.abs(z)
    theta = np.angle(yhat * np.conj(z))
    return c, theta


def phi_m_step(phi: np.ndarray, yhat: np.ndarray, z: np.ndarray, a: np.ndarray,
               prm: Params) -> np.ndarray:
    """One 4-colour MM sweep of the phi M-step over pupil pixels.

    -cos(x) is majorised at x0 = wrap(phi_i - theta_i) by
    -cos(x0) + (sinc(x0)/2)(x^2 - x0^2), so pixel i minimises
    (kappa/2)(phi - theta~)^2 + beta sum_j b_ij (phi - phi_j)^2 with
    kappa = c_i sinc(x0), theta~ = phi_i - x0, sum over pupil neighbours:
    phi_i = (kappa theta~ + 2 beta Phi)/(kappa + 2 beta P).
    A zero denominator leaves phi_i unchanged.
    """
    phi = phi.astype(np.float64, copy=True)
    c, theta = phi_data_terms(yhat, z, a, prm.sigma_w2)
    col = colour_map(phi.shape[0])
    pup = a > 0
    beta = prm.beta_phi
    for k in range(4):
        P = np.zeros_like(phi)
        Ph = np.zeros_like(phi)
        for di, dj, bij in NEIGHBOURS:
            pj, ok = _neighbour(phi, di, dj)
            aj, _ = _neighbour(pup.astype(np.float64), di, dj)
            wgt = np.where(ok & (aj > 0), bij, 0.0)
            P += wgt
            Ph += wgt * pj
        x0 = wrap(phi - theta)
        kappa = c * np.sinc(x0 / np.pi)            # numpy sinc is sin(pi t)/(pi t)
        tt = phi - x0
        den = kappa + 2.0 * beta * P
        num = kappa * tt + 2.0 * beta * Ph
        new = np.where(den > 0, num / np.where(den > 0, den, 1.0), phi)
        sel = (col == k) & pup
        phi[sel] = new[sel]
    return phi


# ----------------------------------------------------------------------------
# EM iteration and the DDH-MBIR frame loop
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class EMTrace:
    b: np.ndarray
    mu: np.ndarray
    s: np.ndarray
    z: np.ndarray


def em_core(r, phi, b, yhat, a, prm: Params, trace: list | None = None):
    """One EM iteration given b = A_phi^H yhat for the current phi."""
    mu, _C, s = e_step(r, b, prm.sigma_w2)
    z = F(mu)
    r_new = r_m_step(r, s, prm)
    phi_new = phi_m_step(phi, yhat, z, a, prm)
    if trace is not None:
        trace.append(EMTrace(b=b, mu=mu, s=s, z=z))
    return r_new, phi_new


def em(r, phi, y, a, prm: Params, trace: list | None = None):
    """EM(r, phi; y) of the plain DH-MBIR loop: one iteration on the
    normalised frame, no frame prologue."""
    yhat = normalize(np.asarray(y, dtype=np.complex128))
    b = back_project(yhat, phi, a)
    return em_core(r, phi, b, yhat, a, prm, trace)


def ddh_frame(r, phi, y, a, prm: Params, trace: list | None = None):
    """One pass of the DDH-MBIR loop body (Fig. 1): Normalize, RemoveTipTilt,
    the r initialisation of Eq. (3), then n_k EM iterations.  Returns the new
    (r, phi), i.e. what WriteData receives."""
    yhat = normalize(np.asarray(y, dtype=np.complex128))
    phi = remove_tiptilt(phi, a)
    b = back_project(yhat, phi, a)
    r = r_init(r, b, prm.lam, prm.alpha, prm.r_floor)
    for k in range(prm.n_k):
        if k > 0:
            b = back_project(yhat, phi, a)
        r, phi = em_core(r, phi, b, yhat, a, prm, trace)
    return r, phi


def dh_mbir(y, a, prm: Params, iters: int, reset_every: int, r0=None, phi0=None):
    """Conventional single-shot DH-MBIR with periodic bootstrap resets (the
    DH-MBIR Algorithm section: hundreds of EM iterations on one frame, with r
    reset to a back-projected estimate every 200 iterations).

    Reading: the reset is the Eq. (3) initialisation, whose second term is
    the bootstrap's |back-projection|^2 estimate, applied with the stream's
    lambda (lambda = 1 discards the previous r, as the bootstrap does), on the
    frame prologue (Normalize, RemoveTipTilt); it is followed by one EM
    iteration.  Iteration it (0-based) is such a reset when it % reset_every
    == 0, and otherwise one plain EM(r, phi; y).  Starts from r = phi = 0
    unless r0 / phi0 are given."""
    if iters < 0 or reset_every < 1:
        raise ValueError("iters >= 0 and reset_every >= 1")
    N = a.shape[0]
    r = np.zeros((N, N)) if r0 is None else np.array(r0, dtype=np.float64)
    phi = np.zeros((N, N)) if phi0 is None else np.array(phi0, dtype=np.float64)
    one = dataclasses.replace(prm, n_k=1)
    for it in range(iters):
        if it % reset_every == 0:
            r, phi = ddh_frame(r, phi, y, a, one)
        else:
            r, phi = em(r, phi, y, a, one)
    return r, phi


def run_stream(frames, a, prm: Params, r0=None, phi0=None):
    """DDH_MBIR over a sequence of frames starting from r = 0, phi = 0
    (Fig. 1); yields (r, phi) after each frame."""
    N = a.shape[0]
    r = np.zeros((N, N)) if r0 is None else np.array(r0, dtype=np.float64)
    phi = np.zeros((N, N)) if phi0 is None else np.array(phi0, dtype=np.float64)
    for y in frames:
        r, phi = ddh_frame(r, phi, y, a, prm)
        yield r, phi
