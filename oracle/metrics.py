"""FP64 metrics of the oracle: the monitored MAP cost and the peak Strehl ratio.

TEST INFRASTRUCTURE ONLY (see oracle/ddh.py): imported by tests, the smoke
check and the benchmark's CPU-baseline leg, never by the GPU path.
"""
from __future__ import annotations

import numpy as np

from .ddh import (F, FH, HALF_NEIGHBOURS, Params, back_project, normalize,
                  qggmrf_rho, remove_tiptilt)


def _pairs(x: np.ndarray, di: int, dj: int):
    """(x_i, x_j) for every unordered neighbour pair at offset (di, dj) that
    lies inside the grid."""
    N0, N1 = x.shape
    i0, i1 = 0, N0 - di
    j0, j1 = max(0, -dj), min(N1, N1 - dj)
    return x[i0:i1, j0:j1], x[i0 + di:i1 + di, j0 + dj:j1 + dj]


def cost_U(r: np.ndarray, phi: np.ndarray, yhat: np.ndarray, a: np.ndarray,
           prm: Params) -> float:
    """Cost that one EM iteration does not increase (MAP cost of the
    back-projected model b(phi) = g + w~, Eq. (2) with A^H A ~ I):

      U = sum_i |b_i(phi)|^2/(r_i + s2) + log(r_i + s2)
        + sum_{8-nbr pairs} b_ij rho(r_i - r_j)
        + beta sum_{pupil pairs} b_ij (phi_i - phi_j)^2,
      b(phi) = F^H(a exp(-j phi) yhat).

    With a = 1 everywhere the data term equals -log p(yhat | r, phi) of Eq. (2)
    up to a constant.
    """
    s2 = prm.sigma_w2
    b = back_project(yhat, phi, a)
    U = float(np.sum(np.abs(b) ** 2 / (r + s2) + np.log(r + s2)))
    pup = (a > 0).astype(np.float64)
    for di, dj, bij in HALF_NEIGHBOURS:
        ri, rj = _pairs(r, di, dj)
        U += bij * float(np.sum(qggmrf_rho(ri - rj, prm.qg_p, prm.qg_q, prm.qg_T, prm.qg_sigma)))
        pi_, pj = _pairs(phi, di, dj)
        ai, aj = _pairs(pup, di, dj)
        U += prm.beta_phi * bij * float(np.sum(ai * aj * (pi_ - pj) ** 2))
    return U


def cost_U_frame(r, phi, y, a, prm: Params) -> float:
    """cost_U on the normalised frame y."""
    return cost_U(r, phi, normalize(np.asarray(y, dtype=np.complex128)), a, prm)


def strehl(phi_hat: np.ndarray, phi_true: np.ndarray, a: np.ndarray) -> float:
    """Peak Strehl ratio (Algorithm Parameters and Metrics):
    S = max |F^H(a exp(j psi))|^2 / max |F^H a|^2 on the N x N grid,
    psi = phi_hat - phi_true with piston, tip and tilt removed over the pupil
    (the paper scores only higher-order error)."""
    psi = remove_tiptilt(np.asarray(phi_hat, np.float64) - np.asarray(phi_true, np.float64), a)
    num = np.max(np.abs(FH(a * np.exp(1j * psi))) ** 2)
    den = np.max(np.abs(FH(a.astype(np.complex128))) ** 2)
    return float(num / den)


def phase_rms_diff(phi1, phi2, a) -> float:
    """RMS over the pupil of (phi1 - phi2) with its pupil mean removed."""
    m = a > 0
    d = (np.asarray(phi1, np.float64) - np.asarray(phi2, np.float64))[m]
    d = d - d.mean()
    return float(np.sqrt(np.mean(d * d)))


def rel_l2(x, ref) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


__all__ = ["cost_U", "cost_U_frame", "strehl", "phase_rms_diff", "rel_l2", "F", "FH"]
