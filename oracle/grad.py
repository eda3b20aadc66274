"""FP64 reference gradient of K unrolled DDH-MBIR frames (CPU, PyTorch autograd).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the GPU path never
imports it.  It re-expresses ``oracle.ddh``'s frame (Fig. 1 body: Normalize,
RemoveTipTilt, Eq. (3), one EM iteration per frame) in float64 torch ops so
that autograd differentiates it; each function follows its ``oracle.ddh``
counterpart operation for operation (same order, same readings), and
a test checks that the two forwards agree to rounding.

Differentiated inputs: the initial phase phi0, the noise standard deviation
sigma_w (sigma_w2 = sigma_w^2), the QGGMRF scale sigma_r (the prior weight is
1/sigma_r^2 and the threshold T sigma_r) and the phase-prior weight beta.
The loss is the piston-removed RMS phase error over the pupil after the last
frame.

Two places need care to be differentiable:
  * the r update is a root of A rho^3 - B rho^2 + rho - s chosen by comparing
    surrogate values: the root is found with ``oracle.ddh.solve_pixel_r`` (no
    gradient) and re-entered through one Newton step in torch, whose
    derivative at the root is the implicit-function derivative
    -(df/d(A,B,s))/f'(rho);
  * |d|^(2-q) at d = 0 has an infinite derivative; there the weight is flat
    in the forward (both sides of the edge are usually floored) and the
    gradient of the power is taken as zero.
Everywhere else (wrap, floors, the choice among roots) autograd takes the
derivative of the branch the forward took.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ddh as O

_T = torch.float64


def _t(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.complex128 if np.iscomplexobj(x) else _T)


def neighbour_t(x: torch.Tensor, di: int, dj: int):
    """(value, exists) of the (di, dj) neighbour of every pixel, free boundary."""
    N0, N1 = x.shape
    out = torch.zeros_like(x)
    ok = torch.zeros(x.shape, dtype=torch.bool)
    i0, i1 = max(0, -di), min(N0, N0 - di)
    j0, j1 = max(0, -dj), min(N1, N1 - dj)
    out[i0:i1, j0:j1] = x[i0 + di:i1 + di, j0 + dj:j1 + dj]
    ok[i0:i1, j0:j1] = True
    return out, ok


def remove_tiptilt_t(phi: torch.Tensor, a: np.ndarray) -> torch.Tensor:
    N = phi.shape[0]
    c = (N - 1) / 2.0
    ii, jj = np.nonzero(a > 0)
    X = torch.as_tensor(np.column_stack([np.ones(ii.size), ii - c, jj - c]), dtype=_T)
    v = phi[ii, jj]
    coef = torch.linalg.solve(X.T @ X, X.T @ v)   # the least-squares plane (normal equations)
    out = torch.zeros_like(phi)
    out[ii, jj] = v - X @ coef
    return out


def qggmrf_weight_t(d: torch.Tensor, p: float, q: float, T, sig) -> torch.Tensor:
    ad = torch.abs(d)
    pos = ad > 0
    safe = torch.where(pos, ad, torch.ones_like(ad))
    if p - q > 0:
        v = torch.where(pos, (safe / (T * sig)) ** (p - q), torch.zeros_like(ad))
    else:
        v = torch.ones_like(ad)
    base = torch.where(pos, safe ** (p - 2.0), torch.ones_like(ad)) if p != 2.0 else torch.ones_like(ad)
    return base / sig ** p * (1.0 + (q / p) * v) / (1.0 + v) ** 2


def solve_pixel_r_t(s: torch.Tensor, A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    rho0 = torch.as_tensor(O.solve_pixel_r(s.detach().numpy(), A.detach().numpy(), B.detach().numpy()), dtype=_T)
    f = ((A * rho0 - B) * rho0 + 1.0) * rho0 - s
    fp = (3.0 * A * rho0 - 2.0 * B) * rho0 + 1.0
    newton = rho0 - f / torch.where(fp != 0, fp, torch.ones_like(fp))
    return torch.where(A <= 0, s, newton)


def r_m_step_t(r: torch.Tensor, s: torch.Tensor, prm: O.Params, sig_r) -> torch.Tensor:
    col = torch.as_tensor(O.colour_map(r.shape[0]))
    for k in range(4):
        A = torch.zeros_like(r)
        B = torch.zeros_like(r)
        for di, dj, bij in O.NEIGHBOURS:
            rj, ok = neighbour_t(r, di, dj)
            w = torch.where(ok, bij * qggmrf_weight_t(r - rj, prm.qg_p, prm.qg_q, prm.qg_T, sig_r),
                            torch.zeros_like(r))
            A = A + w
            B = B + w * rj
        sel = col == k
        new = solve_pixel_r_t(s, A, B)
        r = torch.where(sel, torch.clamp_min(new, prm.r_floor), r)
    return r


def phi_m_step_t(phi: torch.Tensor, yhat: torch.Tensor, z: torch.Tensor, a: np.ndarray, s2, beta) -> torch.Tensor:
    at = torch.as_tensor(a, dtype=_T)
    c = (2.0 / s2) * at * torch.abs(yhat) * torch.abs(z)
    theta = torch.angle(yhat * torch.conj(z))
    col = torch.as_tensor(O.colour_map(phi.shape[0]))
    pup = at > 0
    for k in range(4):
        P = torch.zeros_like(phi)
        Ph = torch.zeros_like(phi)
        for di, dj, bij in O.NEIGHBOURS:
            pj, ok = neighbour_t(phi, di, dj)
            aj, _ = neighbour_t(at, di, dj)
            wgt = torch.where(ok & (aj > 0), torch.full_like(phi, bij), torch.zeros_like(phi))
            P = P + wgt
            Ph = Ph + wgt * pj
        x0 = torch.remainder(phi - theta + math.pi, 2.0 * math.pi) - math.pi
        kappa = c * torch.sinc(x0 / math.pi)
        tt = phi - x0
        den = kappa + 2.0 * beta * P
        num = kappa * tt + 2.0 * beta * Ph
        new = torch.where(den > 0, num / torch.where(den > 0, den, torch.ones_like(den)), phi)
        sel = (col == k) & pup
        phi = torch.where(sel, new, phi)
    return phi


def ddh_frame_t(r, phi, yhat: torch.Tensor, a: np.ndarray, prm: O.Params, s2, sig_r, beta):
    """oracle.ddh.ddh_frame with N_k = 1 on a normalised frame yhat."""
    at = torch.as_tensor(a, dtype=_T)
    phi = remove_tiptilt_t(phi, a)
    b = torch.fft.ifft2(at * torch.exp(-1j * phi) * yhat, norm="ortho")
    r = torch.clamp_min((1.0 - prm.lam) * r + prm.lam * prm.alpha * torch.abs(b) ** 2, prm.r_floor)
    w = r / (r + s2)
    mu = w * b
    s = s2 * w + torch.abs(mu) ** 2
    z = torch.fft.fft2(mu, norm="ortho")
    r_new = r_m_step_t(r, s, prm, sig_r)
    phi_new = phi_m_step_t(phi, yhat, z, a, s2, beta)
    return r_new, phi_new


def phase_rmse_t(phi, phi_true, a):
    """Piston-removed RMS phase error over the pupil."""
    m = torch.as_tensor(a > 0)
    d = (phi - phi_true)[m]
    d = d - d.mean()
    return torch.sqrt(torch.mean(d * d))


def unrolled_loss(phi0, sigma_w, sigma_r, beta, frames, phi_true, a, prm: O.Params):
    """Loss after len(frames) DDH frames (N_k = 1) from r = 0, phi = phi0."""
    N = a.shape[0]
    r = torch.zeros((N, N), dtype=_T)
    phi = phi0
    s2 = sigma_w * sigma_w
    for y in frames:
        yhat = _t(O.normalize(np.asarray(y, dtype=np.complex128)))
        r, phi = ddh_frame_t(r, phi, yhat, a, prm, s2, sigma_r, beta)
    return phase_rmse_t(phi, _t(phi_true), a)


def reference_gradient(phi0: np.ndarray, sigma_w: float, sigma_r: float, beta: float, frames, phi_true, a,
                       prm: O.Params):
    """(loss, d/d phi0 (N x N), d/d sigma_w, d/d sigma_r, d/d beta) in FP64."""
    p0 = torch.tensor(np.asarray(phi0, dtype=np.float64), requires_grad=True)
    sw = torch.tensor(float(sigma_w), dtype=_T, requires_grad=True)
    sr = torch.tensor(float(sigma_r), dtype=_T, requires_grad=True)
    bt = torch.tensor(float(beta), dtype=_T, requires_grad=True)
    L = unrolled_loss(p0, sw, sr, bt, frames, phi_true, a, prm)
    L.backward()
    # a parameter the loss does not reach (sigma_r with one frame: the phase
    # step of a frame uses the Eq. (3) reflectance, not the r M-step's) has
    # derivative zero; autograd leaves its grad unset
    d = [float(x.grad) if x.grad is not None else 0.0 for x in (sw, sr, bt)]
    return float(L.detach()), p0.grad.numpy().copy(), d[0], d[1], d[2]


def oracle_loss(phi0: np.ndarray, sigma_w: float, sigma_r: float, beta: float, frames, phi_true, a,
                prm: O.Params) -> float:
    """The same loss through the NumPy oracle (for finite differences)."""
    import dataclasses
    p = dataclasses.replace(prm, sigma_w2=sigma_w * sigma_w, qg_sigma=sigma_r, beta_phi=beta, n_k=1)
    N = a.shape[0]
    r = np.zeros((N, N))
    phi = np.asarray(phi0, dtype=np.float64)
    for y in frames:
        r, phi = O.ddh_frame(r, phi, np.asarray(y, dtype=np.complex128), a, p)
    m = a > 0
    d = (phi - phi_true)[m]
    d = d - d.mean()
    return float(np.sqrt(np.mean(d * d)))
