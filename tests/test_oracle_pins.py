"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: explicit
sums, dense linear algebra, brute force, closed forms and invariants, chosen
so that a dropped term, a wrong sign or index, or a transposed operand fails
one of them.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

import ddh_synth as synth
from oracle import ddh, metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(20230503)


def crandn(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def dft_matrix(N):
    """Unitary 2D DFT acting on row-major vectors, written from its sum."""
    W = np.empty((N * N, N * N), dtype=np.complex128)
    for k1 in range(N):
        for k2 in range(N):
            for n1 in range(N):
                for n2 in range(N):
                    W[k1 * N + k2, n1 * N + n2] = np.exp(-2j * np.pi * (k1 * n1 + k2 * n2) / N) / N
    return W


# ---------------------------------------------------------------- operators

def test_F_is_the_explicit_unitary_dft():
    N = 4
    x = crandn(N, N)
    W = dft_matrix(N)
    np.testing.assert_allclose(ddh.F(x).ravel(), W @ x.ravel(), atol=1e-13)
    np.testing.assert_allclose(ddh.FH(x).ravel(), W.conj().T @ x.ravel(), atol=1e-13)


@pytest.mark.parametrize("N", [8, 64])
def test_F_parseval_inverse_delta(N):
    x = crandn(N, N)
    assert abs(np.linalg.norm(ddh.F(x)) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    np.testing.assert_allclose(ddh.FH(ddh.F(x)), x, atol=1e-12)
    d = np.zeros((N, N), complex)
    d[0, 0] = 1
    np.testing.assert_allclose(ddh.F(d), np.full((N, N), 1.0 / N), atol=1e-15)


def test_back_project_is_adjoint_of_dense_forward_model():
    """<A x, v> = <x, A^H v> with A = D_a D(exp(j phi)) W built densely."""
    N = 6
    a = ddh.aperture(N)
    phi = RNG.uniform(-3, 3, (N, N))
    A = (a.ravel() * np.exp(1j * phi.ravel()))[:, None] * dft_matrix(N)
    v = crandn(N, N)
    np.testing.assert_allclose(ddh.back_project(v, phi, a).ravel(), A.conj().T @ v.ravel(), atol=1e-13)
    x = crandn(N, N)
    lhs = np.vdot(v.ravel(), A @ x.ravel())
    rhs = np.vdot(ddh.back_project(v, phi, a).ravel(), x.ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_aperture_counts_by_integer_arithmetic(N):
    # (i - c)^2 + (j - c)^2 <= (N/2)^2 with c = (N-1)/2, multiplied by 4
    cnt = 0
    for i in range(N):
        di = (2 * i - (N - 1)) ** 2
        for j in range(N):
            if di + (2 * j - (N - 1)) ** 2 <= N * N:
                cnt += 1
    assert int(ddh.aperture(N).sum()) == cnt
    np.testing.assert_array_equal(ddh.aperture(N), synth.aperture(N))


# ---------------------------------------------------------------- Normalize

def test_normalize_mean_norm_and_affine_invariance():
    y = crandn(32, 32) * 3 + (2 - 1j)
    yh = ddh.normalize(y)
    assert abs(yh.mean()) < 1e-13
    assert abs(np.linalg.norm(yh) - 32.0) < 1e-12
    c, d = 0.3 - 2.1j, 7 + 4j
    np.testing.assert_allclose(ddh.normalize(c * y + d), (c / abs(c)) * yh, atol=1e-12)


@pytest.mark.parametrize("bad", ["const", "nan"])
def test_normalize_undefined_inputs_raise(bad):
    y = np.full((8, 8), 1 + 1j)
    if bad == "nan":
        y = crandn(8, 8)
        y[3, 3] = np.nan
    with pytest.raises(ValueError):
        ddh.normalize(y)


# ---------------------------------------------------------------- RemoveTipTilt

def test_remove_tiptilt_plane_orthogonality_idempotence():
    N = 64
    a = ddh.aperture(N)
    c = (N - 1) / 2
    i, j = np.meshgrid(np.arange(N) - c, np.arange(N) - c, indexing="ij")
    plane = 0.7 - 0.05 * i + 0.11 * j
    np.testing.assert_allclose(ddh.remove_tiptilt(plane, a), 0.0, atol=1e-12)
    phi = RNG.standard_normal((N, N))
    res = ddh.remove_tiptilt(phi, a)
    m = a > 0
    for basis in (np.ones_like(i), i, j):
        assert abs(np.sum(res[m] * basis[m])) < 1e-9
    assert np.all(res[~m] == 0)
    np.testing.assert_allclose(ddh.remove_tiptilt(res, a), res, atol=1e-12)
    # the centred disk is symmetric, so the normal equations are diagonal
    c0 = phi[m].mean()
    c1 = np.sum(i[m] * phi[m]) / np.sum(i[m] ** 2)
    c2 = np.sum(j[m] * phi[m]) / np.sum(j[m] ** 2)
    np.testing.assert_allclose(res[m], phi[m] - c0 - c1 * i[m] - c2 * j[m], atol=1e-12)


# ---------------------------------------------------------------- Eq. (3)

def test_r_init_hand_values():
    r_prev = np.array([[0.5, 0.0]])
    b = np.array([[2.0 + 0j, 0.0]])
    out = ddh.r_init(r_prev, b, 0.45, 0.025, 1e-8)
    # (1-0.45)*0.5 + 0.45*0.025*4 = 0.32 ; second pixel hits the floor
    np.testing.assert_allclose(out, [[0.32, 1e-8]], rtol=1e-15)


def test_paper_parameter_defaults():
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    prm = ddh.Params(sigma_w2=0.1)
    assert prm.alpha == g["params"]["alpha"] and prm.lam == g["params"]["lambda"]
    assert synth.DEFAULT_PARAMS["alpha"] == g["params"]["alpha"]
    assert synth.DEFAULT_PARAMS["lam"] == g["params"]["lambda"]


def test_flow_speed_matches_paper_worked_value():
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["flow"]
    v = synth.flow_speed(g["f_g"], g["f_s"], g["N"], g["D_over_r0"]) / math.sqrt(2.0)
    assert round(v, g["digits"]) == g["v_component"]


# ---------------------------------------------------------------- E-step

def _dense_posterior(yh, phi, a, r, s2):
    N = a.shape[0]
    A = (a.ravel() * np.exp(1j * phi.ravel()))[:, None] * dft_matrix(N)
    C = np.linalg.inv(A.conj().T @ A / s2 + np.diag(1.0 / r.ravel()))
    mu = C @ (A.conj().T @ yh.ravel()) / s2
    return mu, C


def test_e_step_equals_dense_posterior_full_aperture():
    N, s2 = 8, 0.13
    a = np.ones((N, N))
    phi = RNG.uniform(-2, 2, (N, N))
    r = RNG.uniform(0.05, 2.0, (N, N))
    yh = ddh.normalize(crandn(N, N))
    mu_d, C_d = _dense_posterior(yh, phi, a, r, s2)
    mu, C, s = ddh.e_step(r, ddh.back_project(yh, phi, a), s2)
    np.testing.assert_allclose(mu.ravel(), mu_d, atol=1e-12)
    np.testing.assert_allclose(C.ravel(), np.real(np.diag(C_d)), atol=1e-12)
    np.testing.assert_allclose(s.ravel(), np.real(np.diag(C_d)) + np.abs(mu_d) ** 2, atol=1e-12)


def test_e_step_gap_with_circular_pupil_is_reported():
    """With a circular pupil A^H A != I; the pointwise E-step is then the
    exact posterior of the back-projected model only.  Report the gap."""
    N, s2 = 8, 0.13
    a = ddh.aperture(N)
    phi = RNG.uniform(-2, 2, (N, N))
    r = RNG.uniform(0.05, 2.0, (N, N))
    yh = ddh.normalize(crandn(N, N))
    mu_d, _ = _dense_posterior(yh, phi, a, r, s2)
    mu, _, _ = ddh.e_step(r, ddh.back_project(yh, phi, a), s2)
    gap = np.linalg.norm(mu.ravel() - mu_d) / np.linalg.norm(mu_d)
    print(f"E-step gap with circular pupil at N=8: rel-L2 {gap:.3f}")
    assert np.isfinite(gap)


# ---------------------------------------------------------------- QGGMRF

QG = dict(p=2.0, q=1.2, T=0.1, sig=0.2)


def test_qggmrf_weight_is_derivative_over_delta():
    d = np.concatenate([RNG.uniform(-3, 3, 200), [1e-3, -2e-3, 0.02, 5.0]])
    h = 1e-6
    fd = (ddh.qggmrf_rho(d + h, **QG) - ddh.qggmrf_rho(d - h, **QG)) / (2 * h)
    np.testing.assert_allclose(ddh.qggmrf_weight(d, **QG), fd / d, rtol=1e-6)
    assert abs(ddh.qggmrf_weight(np.array(0.0), **QG) - 1.0 / QG["sig"] ** 2) < 1e-12
    # quadratic near 0, |d|^q growth far away
    d0 = 1e-12
    assert abs(ddh.qggmrf_rho(np.array(d0), **QG) / (d0 ** 2 / (2 * 0.04)) - 1.0) < 1e-7
    big = np.array([1e3, 1e4])
    ratio = ddh.qggmrf_rho(big[1:], **QG) / ddh.qggmrf_rho(big[:1], **QG)
    assert abs(np.log10(ratio[0]) - QG["q"]) < 1e-3


def test_symmetric_bound_majorises_qggmrf():
    grid = np.linspace(-4, 4, 4001)
    for d0 in RNG.uniform(-3, 3, 50):
        q = ddh.qggmrf_rho(np.array(d0), **QG) + 0.5 * ddh.qggmrf_weight(np.array(d0), **QG) * (grid ** 2 - d0 ** 2)
        assert np.all(q - ddh.qggmrf_rho(grid, **QG) >= -1e-12)


# ---------------------------------------------------------------- r update

def test_pixel_solver_is_the_global_minimiser():
    n = 400
    s = np.exp(RNG.uniform(np.log(1e-3), np.log(5.0), n))
    A = np.exp(RNG.uniform(np.log(1e-2), np.log(100.0), n))
    B = A * np.exp(RNG.uniform(np.log(1e-2), np.log(3.0), n))
    rho = ddh.solve_pixel_r(s, A, B)
    grid = np.exp(np.linspace(np.log(1e-5), np.log(50.0), 200001))
    n_multi = 0
    for k in range(n):
        h = np.log(grid) + s[k] / grid + 0.5 * A[k] * grid ** 2 - B[k] * grid
        g = grid[np.argmin(h)]
        hk = np.log(rho[k]) + s[k] / rho[k] + 0.5 * A[k] * rho[k] ** 2 - B[k] * rho[k]
        assert hk <= h.min() + 1e-12
        assert abs(rho[k] - g) <= 2e-4 * g
        dh = np.diff(h)
        n_multi += int(np.sum((dh[:-1] < 0) & (dh[1:] >= 0)) > 1)
    assert n_multi > 0, "instances should include two-minimum cases"


def test_pixel_solver_without_prior_returns_s():
    s = np.array([0.3, 2.0])
    np.testing.assert_array_equal(ddh.solve_pixel_r(s, np.zeros(2), np.zeros(2)), s)
    prm = ddh.Params(sigma_w2=0.1, qg_sigma=1e150)
    r = RNG.uniform(0.1, 1.0, (8, 8))
    s = RNG.uniform(0.1, 1.0, (8, 8))
    np.testing.assert_allclose(ddh.r_m_step(r, s, prm), s, rtol=1e-12)


def _sequential_r_sweep(r, s, prm):
    """Pixel-by-pixel ICD in colour order, neighbours by explicit bounds."""
    r = r.copy()
    N = r.shape[0]
    for colour in range(4):
        for i in range(N):
            for j in range(N):
                if (i % 2) + 2 * (j % 2) != colour:
                    continue
                A = B = 0.0
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        if di == 0 and dj == 0:
                            continue
                        ii, jj = i + di, j + dj
                        if not (0 <= ii < N and 0 <= jj < N):
                            continue
                        bij = 1 / 6 if (di == 0 or dj == 0) else 1 / 12
                        d = r[i, j] - r[ii, jj]
                        v = (abs(d) / (prm.qg_T * prm.qg_sigma)) ** (prm.qg_p - prm.qg_q)
                        w = bij * abs(d) ** (prm.qg_p - 2) / prm.qg_sigma ** prm.qg_p * (1 + prm.qg_q / prm.qg_p * v) / (1 + v) ** 2
                        A += w
                        B += w * r[ii, jj]
                rho = ddh.solve_pixel_r(np.array([s[i, j]]), np.array([A]), np.array([B]))[0]
                r[i, j] = max(rho, prm.r_floor)
    return r


def test_r_sweep_matches_sequential_icd():
    prm = ddh.Params(sigma_w2=0.1)
    r = RNG.uniform(0.05, 1.5, (8, 8))
    s = RNG.uniform(0.01, 2.0, (8, 8))
    np.testing.assert_allclose(ddh.r_m_step(r, s, prm), _sequential_r_sweep(r, s, prm), rtol=1e-12)


def _G_r(r, s, prm):
    v = float(np.sum(np.log(r) + s / r))
    for di, dj, bij in ddh.HALF_NEIGHBOURS:
        a, b = metrics._pairs(r, di, dj)
        v += bij * float(np.sum(ddh.qggmrf_rho(a - b, prm.qg_p, prm.qg_q, prm.qg_T, prm.qg_sigma)))
    return v


def test_r_sweep_decreases_its_objective():
    prm = ddh.Params(sigma_w2=0.1)
    for _ in range(5):
        r = RNG.uniform(0.05, 1.5, (32, 32))
        s = RNG.uniform(0.01, 2.0, (32, 32))
        assert _G_r(ddh.r_m_step(r, s, prm), s, prm) <= _G_r(r, s, prm) + 1e-12


# ---------------------------------------------------------------- phi update

def test_cos_majoriser_bound_on_grid():
    xs = np.linspace(-12, 12, 24001)
    for x0 in np.concatenate([np.linspace(-np.pi, np.pi, 101), RNG.uniform(-np.pi, np.pi, 50)]):
        k = np.sinc(x0 / np.pi)
        q = -np.cos(x0) + 0.5 * k * (xs ** 2 - x0 ** 2)
        assert np.all(q + np.cos(xs) >= -1e-12)


def test_phi_step_without_prior_lands_on_theta():
    N = 16
    a = ddh.aperture(N)
    yh = crandn(N, N)
    z = crandn(N, N)
    phi = a * RNG.uniform(-6, 6, (N, N))
    prm = ddh.Params(sigma_w2=0.2, beta_phi=0.0)
    out = ddh.phi_m_step(phi, yh, z, a, prm)
    theta = np.angle(yh * np.conj(z))
    m = a > 0
    np.testing.assert_allclose(ddh.wrap(out[m] - theta[m]), 0.0, atol=1e-12)
    # the nearest 2 pi translate of theta is taken: |out - phi| <= pi
    assert np.all(np.abs(out[m] - phi[m]) <= np.pi + 1e-12)
    assert np.all(out[~m] == 0)


def _sequential_phi_sweep(phi, yh, z, a, prm):
    phi = phi.copy()
    N = phi.shape[0]
    for colour in range(4):
        for i in range(N):
            for j in range(N):
                if (i % 2) + 2 * (j % 2) != colour or a[i, j] == 0:
                    continue
                c = 2.0 / prm.sigma_w2 * abs(yh[i, j]) * abs(z[i, j])
                th = math.atan2((yh[i, j] * np.conj(z[i, j])).imag, (yh[i, j] * np.conj(z[i, j])).real)
                x0 = (phi[i, j] - th + math.pi) % (2 * math.pi) - math.pi
                kap = c * (math.sin(x0) / x0 if x0 != 0 else 1.0)
                P = Ph = 0.0
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        ii, jj = i + di, j + dj
                        if (di, dj) == (0, 0) or not (0 <= ii < N and 0 <= jj < N) or a[ii, jj] == 0:
                            continue
                        bij = 1 / 6 if (di == 0 or dj == 0) else 1 / 12
                        P += bij
                        Ph += bij * phi[ii, jj]
                den = kap + 2 * prm.beta_phi * P
                if den > 0:
                    phi[i, j] = (kap * (phi[i, j] - x0) + 2 * prm.beta_phi * Ph) / den
    return phi


def test_phi_sweep_matches_sequential_mm():
    N = 10
    a = ddh.aperture(N)
    yh, z = crandn(N, N), crandn(N, N)
    phi = a * RNG.uniform(-4, 4, (N, N))
    prm = ddh.Params(sigma_w2=0.3, beta_phi=0.7)
    np.testing.assert_allclose(ddh.phi_m_step(phi, yh, z, a, prm),
                               _sequential_phi_sweep(phi, yh, z, a, prm), atol=1e-12)


def test_phi_sweep_decreases_its_objective():
    N = 32
    a = ddh.aperture(N)
    prm = ddh.Params(sigma_w2=0.3, beta_phi=0.7)
    pup = (a > 0).astype(float)
    for _ in range(5):
        yh, z = crandn(N, N), crandn(N, N)
        phi = a * RNG.uniform(-4, 4, (N, N))
        c, th = ddh.phi_data_terms(yh, z, a, prm.sigma_w2)

        def G(p):
            v = -float(np.sum(c * np.cos(p - th)))
            for di, dj, bij in ddh.HALF_NEIGHBOURS:
                x1, x2 = metrics._pairs(p, di, dj)
                m1, m2 = metrics._pairs(pup, di, dj)
                v += prm.beta_phi * bij * float(np.sum(m1 * m2 * (x1 - x2) ** 2))
            return v
        assert G(ddh.phi_m_step(phi, yh, z, a, prm)) <= G(phi) + 1e-12


# ---------------------------------------------------------------- cost and EM

def test_cost_data_term_equals_dense_gaussian_likelihood():
    """a = 1: U (priors off) = yh^H S^-1 yh + log det S, S = A D(r) A^H + s2 I."""
    N, s2 = 8, 0.21
    a = np.ones((N, N))
    phi = RNG.uniform(-2, 2, (N, N))
    r = RNG.uniform(0.05, 2.0, (N, N))
    yh = ddh.normalize(crandn(N, N))
    prm = ddh.Params(sigma_w2=s2, beta_phi=0.0, qg_sigma=1e150)
    A = np.exp(1j * phi.ravel())[:, None] * dft_matrix(N)
    Sg = A @ np.diag(r.ravel()) @ A.conj().T + s2 * np.eye(N * N)
    dense = np.real(np.vdot(yh.ravel(), np.linalg.solve(Sg, yh.ravel()))) + np.linalg.slogdet(Sg)[1]
    assert abs(metrics.cost_U(r, phi, yh, a, prm) - dense) < 1e-9 * abs(dense)


def test_cost_prior_terms_by_pair_loops():
    N = 7
    a = ddh.aperture(N)
    r = RNG.uniform(0.05, 2.0, (N, N))
    phi = a * RNG.uniform(-2, 2, (N, N))
    prm = ddh.Params(sigma_w2=0.2, beta_phi=0.8)
    yh = ddh.normalize(crandn(N, N))
    b = ddh.back_project(yh, phi, a)
    ref = float(np.sum(np.abs(b) ** 2 / (r + 0.2) + np.log(r + 0.2)))
    for i in range(N):
        for j in range(N):
            for ii in range(N):
                for jj in range(N):
                    if (ii, jj) <= (i, j) or max(abs(ii - i), abs(jj - j)) != 1:
                        continue
                    bij = 1 / 6 if (ii == i or jj == j) else 1 / 12
                    ref += bij * float(ddh.qggmrf_rho(np.array(r[i, j] - r[ii, jj]), 2.0, 1.2, 0.1, 0.2))
                    if a[i, j] and a[ii, jj]:
                        ref += 0.8 * bij * (phi[i, j] - phi[ii, jj]) ** 2
    assert abs(metrics.cost_U(r, phi, yh, a, prm) - ref) < 1e-10 * abs(ref)


def test_em_cost_is_non_increasing_config0():
    st = synth.config0_stream()
    a = ddh.aperture(64)
    y = st.frame(0).astype(np.complex128)
    prm = ddh.Params(sigma_w2=st.sigma_w2)
    yh = ddh.normalize(y)
    r, phi = ddh.ddh_frame(np.zeros((64, 64)), np.zeros((64, 64)), y, a, prm)
    U = [metrics.cost_U(r, phi, yh, a, prm)]
    for _ in range(199):
        r, phi = ddh.em(r, phi, y, a, prm)
        U.append(metrics.cost_U(r, phi, yh, a, prm))
    U = np.array(U)
    assert np.all(np.diff(U) <= 1e-12 * np.abs(U[1:]))
    assert U[-1] < U[0]


def test_piston_invariance_of_frame_and_cost():
    st = synth.config0_stream()
    a = ddh.aperture(64)
    y = st.frame(0).astype(np.complex128)
    prm = ddh.Params(sigma_w2=st.sigma_w2)
    phi = st.phase(0)
    r = RNG.uniform(0.1, 1.0, (64, 64))
    r1, p1 = ddh.ddh_frame(r, phi, y, a, prm)
    r2, p2 = ddh.ddh_frame(r, phi + 2.5 * a, y, a, prm)
    np.testing.assert_allclose(r1, r2, rtol=1e-10)
    np.testing.assert_allclose(p1, p2, atol=1e-10)
    yh = ddh.normalize(y)
    assert abs(metrics.cost_U(r, phi, yh, a, prm) - metrics.cost_U(r, phi + 1.3 * a, yh, a, prm)) < 1e-9 * abs(metrics.cost_U(r, phi, yh, a, prm))


def test_integer_cycle_tilt_is_a_circular_shift_of_b():
    N = 32
    a = ddh.aperture(N)
    yh = ddh.normalize(crandn(N, N))
    phi = a * RNG.uniform(-1, 1, (N, N))
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    tilt = 2 * np.pi * (3 * i + 5 * j) / N
    b0 = ddh.back_project(yh, phi, a)
    b1 = ddh.back_project(yh, phi + tilt, a)
    np.testing.assert_allclose(np.abs(b1), np.abs(np.roll(b0, (3, 5), axis=(0, 1))), atol=1e-12)


# ---------------------------------------------------------------- Strehl

def test_strehl_one_for_piston_and_tilt_residual():
    N = 64
    a = ddh.aperture(N)
    tr = RNG.standard_normal((N, N))
    c = (N - 1) / 2
    i, j = np.meshgrid(np.arange(N) - c, np.arange(N) - c, indexing="ij")
    assert abs(metrics.strehl(tr + 3.0, tr, a) - 1.0) < 1e-12
    assert abs(metrics.strehl(tr + 0.3 * i - 0.2 * j + 1, tr, a) - 1.0) < 1e-12


def test_strehl_marechal_small_residual():
    N = 128
    a = ddh.aperture(N)
    f = np.fft.fftfreq(N)
    filt = np.exp(-(f[:, None] ** 2 + f[None, :] ** 2) / (2 * 0.03 ** 2))
    psi = np.real(np.fft.ifft2(np.fft.fft2(RNG.standard_normal((N, N))) * filt))
    psi = ddh.remove_tiptilt(psi, a)
    psi *= 0.2 / np.sqrt(np.mean(psi[a > 0] ** 2))
    S = metrics.strehl(psi, np.zeros((N, N)), a)
    assert abs(S - np.exp(-0.04)) < 0.01
    # on-axis intensity is a lower bound of the peak
    onaxis = abs(np.sum(a * np.exp(1j * psi))) ** 2 / np.sum(a) ** 2
    assert S >= onaxis - 1e-12


# ---------------------------------------------------------------- simulator

def test_screen_structure_function_kolmogorov():
    """D(r) ~ 6.88 (r/r0)^(5/3) for separations well inside the screen
    (loose statistical check; FFT screens without subharmonics run low at
    large separations)."""
    S, r0 = 256, 8.0
    acc = {2: [], 4: [], 8: []}
    for seed in range(8):
        scr = np.real(synth.screen_from_spectrum(synth.kolmogorov_spectrum(S, r0, np.random.default_rng(seed))))
        for d in acc:
            acc[d].append(np.mean((scr[:, d:] - scr[:, :-d]) ** 2))
    for d, v in acc.items():
        ratio = np.mean(v) / (6.88 * (d / r0) ** (5 / 3))
        assert 0.6 < ratio < 1.4, (d, ratio)


def test_frames_are_seeded_and_complex64():
    st1 = synth.config0_stream()
    st2 = synth.config0_stream()
    y1, y2 = st1.frame(3), st2.frame(3)
    assert y1.dtype == np.complex64
    np.testing.assert_array_equal(y1, y2)
    assert not np.array_equal(st1.frame(4), y1)


def test_phase_step_conventions_with_unit_wiener_weight():
    """Noise-free frame y = a exp(j phi0) F g and a signal variance far above
    the noise (w -> 1): the E-step returns mu = b, so z = F mu = a exp(-j phi)
    yhat on the pupil and theta = arg(yhat conj z) is the phase phi used in b.
    This pins the sign and conjugate conventions of A_phi, A_phi^H and theta (a
    wrong sign or a missing conjugate moves theta by 2 phi or more).  It is not
    a recovery check: with w = 1 every phase is a fixed point of the phase
    step, so the phase is not identifiable in this limit (the recovery pins
    below use an object with a dark surround)."""
    N = 16
    rng = np.random.default_rng(5)
    a = ddh.aperture(N)
    phi0 = ddh.remove_tiptilt(rng.uniform(-2.5, 2.5, (N, N)), a)
    g = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(2)
    y = a * np.exp(1j * phi0) * ddh.F(g)
    yhat = ddh.normalize(y)
    b = ddh.back_project(yhat, phi0, a)
    mu, _, _ = ddh.e_step(np.full((N, N), 1e12), b, 1e-9)
    z = ddh.F(mu)
    prm = ddh.Params(sigma_w2=1e-9, beta_phi=0.0)
    phi1 = ddh.phi_m_step(phi0, yhat, z, a, prm)
    m = a > 0
    np.testing.assert_allclose(phi1[m], phi0[m], atol=1e-9)
    # any other phase used in b is returned as theta too (w = 1: no information)
    phi_off = ddh.remove_tiptilt(phi0 + 0.3 * rng.standard_normal((N, N)) * m, a)
    z_off = ddh.F(ddh.e_step(np.full((N, N), 1e12), ddh.back_project(yhat, phi_off, a), 1e-9)[0])
    theta = np.angle(yhat * np.conj(z_off))
    np.testing.assert_allclose(np.angle(np.exp(1j * (theta[m] - phi_off[m]))), 0.0, atol=1e-9)


# ------------------------------------------------- noise-free phase recovery
#
# A case where the reading of the E-step is exact and the phase identifiable:
# the aperture is the whole grid (A_phi unitary, so the pointwise E-step is the
# exact posterior), the frame is noise-free, and the object is dark outside a
# centred disc (g = 0 there), so the Wiener weight w = r/(r + s2) is ~1 on the
# object and ~0 around it.  The phase step is then the Fourier-magnitude /
# object-support projection pair of phase retrieval, and the true phase is a
# fixed point.

def _support_case(N=16, seed=1, a=None, s2=1e-6, r_floor=1e-8):
    a = np.ones((N, N)) if a is None else a
    c = (N - 1) / 2.0
    ii, jj = np.mgrid[0:N, 0:N]
    support = ((ii - c) ** 2 + (jj - c) ** 2) <= (N / 4.0) ** 2
    r = np.where(support, synth.reflectance(N, synth.rng_for(9, seed, synth.PURPOSE_REFLECTANCE)), 0.0)
    spec = synth.kolmogorov_spectrum(2 * N, N / 6.0, synth.rng_for(9, seed, synth.PURPOSE_SCREEN))
    ptrue = synth._remove_plane_truth(synth.screen_from_spectrum(spec)[:N, :N], a)
    y = synth.hologram(r, ptrue, a, np.inf, synth.rng_for(9, seed, synth.PURPOSE_FRAME))
    # the phase step's input is the field scaled to unit mean power; Normalize
    # would also remove the mean of y, which adds mean(y) F^H(a exp(-j phi))
    # to b, a term that is not zero around the object
    scale2 = N * N / np.linalg.norm(y) ** 2
    yhat = y * np.sqrt(scale2)
    prm = ddh.Params(sigma_w2=s2, beta_phi=0.0, r_floor=r_floor)
    r_n = np.maximum(r * scale2, r_floor)
    pert = ddh.remove_tiptilt(
        synth.screen_from_spectrum(synth.kolmogorov_spectrum(
            2 * N, N / 4.0, synth.rng_for(9, seed + 100, synth.PURPOSE_SCREEN)))[:N, :N], a)
    pert *= 0.5 / np.sqrt(np.mean(pert[a > 0] ** 2))      # 0.5 rad RMS, smooth
    return a, yhat, r_n, ptrue, ddh.remove_tiptilt(ptrue + pert, a), prm


def _phase_only_em(phi, yhat, r, a, prm, iters):
    """EM iterations with r held fixed: E-step, z = F mu, phase M-step."""
    for _ in range(iters):
        mu, _, _ = ddh.e_step(r, ddh.back_project(yhat, phi, a), prm.sigma_w2)
        phi = ddh.phi_m_step(phi, yhat, ddh.F(mu), a, prm)
    return phi


def _wrapped_rms(phi, ptrue, a):
    """RMS over the pupil of the phase difference taken modulo 2 pi, with its
    circular mean (piston) removed."""
    z = np.exp(1j * (phi - ptrue))[a > 0]
    return float(np.sqrt(np.mean(np.angle(z * np.exp(-1j * np.angle(z.sum()))) ** 2)))


def test_true_phase_is_a_fixed_point_and_an_attractor_noise_free():
    """Full aperture, noise-free, dark surround, reflectance known: one phase
    step from the true phase moves it by less than 1e-6 rad, one step from a
    0.5 rad (smooth) perturbation moves it by more than 1e-2, and 300 steps
    bring the perturbed phase back to the truth (residual < 1e-3 rad modulo
    2 pi, Strehl > 0.999).  Like every error-reduction phase retrieval the
    iteration can stall at other fixed points, so over seven more objects and
    0.3 rad starts at least six must return below 1e-2 rad.  A sign error in
    the phase of A_phi or A_phi^H, a conjugate missing in theta, or a
    transposed F fails this."""
    a, yhat, r, ptrue, phi_p, prm = _support_case(seed=3)
    m = a > 0
    one = _phase_only_em(ptrue, yhat, r, a, prm, 1)
    assert _wrapped_rms(one, ptrue, a) < 1e-6
    step = _phase_only_em(phi_p, yhat, r, a, prm, 1)
    assert np.sqrt(np.mean((step - phi_p)[m] ** 2)) > 1e-2
    assert _wrapped_rms(phi_p, ptrue, a) > 0.45
    back = _phase_only_em(phi_p, yhat, r, a, prm, 300)
    assert _wrapped_rms(back, ptrue, a) < 1e-3
    assert metrics.strehl(back, ptrue, a) > 0.999
    converged = 0
    for seed in range(2, 9):
        a, yhat, r, ptrue, phi_p, prm = _support_case(seed=seed)
        phi_p = ddh.remove_tiptilt(ptrue + 0.6 * (phi_p - ptrue), a)
        converged += _wrapped_rms(_phase_only_em(phi_p, yhat, r, a, prm, 300), ptrue, a) < 1e-2
    assert converged >= 6, converged


@pytest.mark.xfail(strict=True, reason="joint EM (r re-estimated each iteration) from a perturbed phase: the r M-step "
                   "explains the energy that the wrong phase leaks outside the object by raising r there, which "
                   "removes the dark surround that identifies the phase; the phase then stays where it started")
def test_joint_em_recovers_the_phase_noise_free():
    a, yhat, r, ptrue, phi, prm = _support_case()
    for _ in range(300):
        r, phi = ddh.em_core(r, phi, ddh.back_project(yhat, phi, a), yhat, a, prm)
    assert _wrapped_rms(phi, ptrue, a) < 1e-2


def test_circular_pupil_moves_the_fixed_point_is_reported():
    """With the circular pupil the pointwise E-step is not the exact posterior
    (A^H A is the pupil's low-pass projection, not I): the back-projection of
    the true field leaks outside the object, so the true phase is no longer a
    fixed point of the phase step even in the noise-free case above.  Report
    the size of one step from the truth (the quality gap of this reading)."""
    N = 16
    a, yhat, r, ptrue, _, prm = _support_case(N=N, a=ddh.aperture(N))
    one = _phase_only_em(ptrue, yhat, r, a, prm, 1)
    move = _wrapped_rms(one, ptrue, a)
    print(f"circular pupil: one phase step from the true phase moves it by {move:.3f} rad RMS")
    assert move > 1e-3


# ---------------------------------------------------------------- metrics

def test_phase_rms_diff_hand_values_and_piston_invariance():
    """RMS over the pupil of the difference with its pupil mean removed:
    differences (1, 2, 3) on a three-pixel pupil give sqrt(2/3); values off the
    pupil do not count; a constant added on the pupil (piston) changes nothing;
    the arguments commute."""
    a = np.array([[1.0, 1.0], [1.0, 0.0]])
    p1 = np.array([[1.5, 2.5], [3.5, 100.0]])
    p2 = np.array([[0.5, 0.5], [0.5, -7.0]])
    assert abs(metrics.phase_rms_diff(p1, p2, a) - math.sqrt(2.0 / 3.0)) < 1e-15
    assert abs(metrics.phase_rms_diff(p2, p1, a) - math.sqrt(2.0 / 3.0)) < 1e-15
    assert abs(metrics.phase_rms_diff(p1 + 4.25 * a, p2, a) - math.sqrt(2.0 / 3.0)) < 1e-14
    assert metrics.phase_rms_diff(p1, p1 + 0.7, a) < 1e-15
    # a pure piston difference over a real pupil is zero; a unit step on half of it is 1/2
    N = 8
    ap = ddh.aperture(N)
    step = np.where(np.arange(N)[:, None] < N // 2, 1.0, 0.0) * np.ones((N, N))
    assert abs(metrics.phase_rms_diff(step, np.zeros((N, N)), ap) - 0.5) < 1e-15


def test_rel_l2_hand_values():
    """||x - ref|| / ||ref||, normalised by the reference (not symmetric)."""
    ref = np.array([[1.0, 0.0], [0.0, 0.0]])
    x = np.array([[1.0, 2.0], [2.0, 0.0]])
    assert abs(metrics.rel_l2(x, ref) - math.sqrt(8.0)) < 1e-15
    assert metrics.rel_l2(ref, ref) == 0.0
    assert abs(metrics.rel_l2(2.0 * ref, ref) - 1.0) < 1e-15
    assert abs(metrics.rel_l2(ref, 2.0 * ref) - 0.5) < 1e-15
    assert abs(metrics.rel_l2(np.array([3.0, 4.0]), np.array([0.0, 5.0])) - math.sqrt(10.0) / 5.0) < 1e-15


def test_reference_gradient_against_central_differences():
    """FP64 autograd of the unrolled frames against central differences of the
    NumPy oracle's loss (the forwards agree exactly first)."""
    from oracle import grad as G
    N, K = 16, 3
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0, snr=20.0, speed=0.5, config_id=3, stream_id=0))
    a = ddh.aperture(N)
    frames = [st.frame(n) for n in range(K)]
    ptrue = st.phase(K - 1)
    prm = ddh.Params(sigma_w2=st.sigma_w2)
    sw, sr, bt = float(np.sqrt(st.sigma_w2)), 0.2, 0.5
    rng = np.random.default_rng(0)
    phi0 = ddh.remove_tiptilt(0.3 * rng.standard_normal((N, N)), a)
    L, g0, gsw, gsr, gbt = G.reference_gradient(phi0, sw, sr, bt, frames, ptrue, a, prm)
    assert abs(L - G.oracle_loss(phi0, sw, sr, bt, frames, ptrue, a, prm)) <= 1e-12 * L
    args = [sw, sr, bt]
    for idx, g, h in ((0, gsw, 1e-6), (1, gsr, 1e-3), (1, gsr, 1e-5), (2, gbt, 1e-3), (2, gbt, 1e-5)):
        up, dn = list(args), list(args)
        up[idx] += h
        dn[idx] -= h
        fd = (G.oracle_loss(phi0, *up, frames, ptrue, a, prm) - G.oracle_loss(phi0, *dn, frames, ptrue, a, prm)) / (2 * h)
        assert abs(fd - g) <= 2e-3 * abs(g), (idx, h, fd, g)
    d = ddh.remove_tiptilt(rng.standard_normal((N, N)), a)
    d /= np.sqrt(np.mean(d[a > 0] ** 2))
    h = 1e-6
    fd = (G.oracle_loss(phi0 + h * d, sw, sr, bt, frames, ptrue, a, prm)
          - G.oracle_loss(phi0 - h * d, sw, sr, bt, frames, ptrue, a, prm)) / (2 * h)
    assert abs(fd - np.sum(g0 * d)) <= 2e-3 * abs(fd)


def test_reference_gradient_against_central_differences_eight_frames():
    """The same at N = 32 over K = 8 frames (the unroll depth of the
    differentiation workload): the FP64 autograd gradient against central
    differences of the NumPy oracle's loss with respect to sigma_w, sigma_r,
    beta_phi and phi0 along a random tip/tilt-free direction.  The loss over
    eight frames is strongly curved (wrapped phases, the reflectance floor,
    the choice of the cubic's root), so a step of 1e-3 is dominated by
    curvature (up to 20 % off at these parameters); steps of 1e-6 (1e-5 for
    the prior weights) agree to within 1e-4."""
    from oracle import grad as G
    N, K = 32, 8
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0, snr=20.0, speed=0.5, config_id=3, stream_id=1))
    a = ddh.aperture(N)
    frames = [st.frame(n) for n in range(K)]
    ptrue = st.phase(K - 1)
    prm = ddh.Params(sigma_w2=st.sigma_w2)
    sw, sr, bt = float(np.sqrt(st.sigma_w2)), 0.2, 0.5
    rng = np.random.default_rng(1)
    phi0 = ddh.remove_tiptilt(0.3 * rng.standard_normal((N, N)), a)
    L, g0, gsw, gsr, gbt = G.reference_gradient(phi0, sw, sr, bt, frames, ptrue, a, prm)
    assert abs(L - G.oracle_loss(phi0, sw, sr, bt, frames, ptrue, a, prm)) <= 1e-12 * L
    args = [sw, sr, bt]
    for idx, g, h in ((0, gsw, 1e-6), (1, gsr, 1e-5), (2, gbt, 1e-5)):
        up, dn = list(args), list(args)
        up[idx] += h
        dn[idx] -= h
        fd = (G.oracle_loss(phi0, *up, frames, ptrue, a, prm) - G.oracle_loss(phi0, *dn, frames, ptrue, a, prm)) / (2 * h)
        assert abs(fd - g) <= 1e-4 * abs(g), (idx, h, fd, g)
    d = ddh.remove_tiptilt(rng.standard_normal((N, N)), a)
    d /= np.sqrt(np.mean(d[a > 0] ** 2))
    h = 1e-6
    fd = (G.oracle_loss(phi0 + h * d, sw, sr, bt, frames, ptrue, a, prm)
          - G.oracle_loss(phi0 - h * d, sw, sr, bt, frames, ptrue, a, prm)) / (2 * h)
    assert abs(fd - np.sum(g0 * d)) <= 1e-4 * abs(fd)


def _mbir_case(N=16):
    st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0, snr=20.0, speed=0.5, config_id=5, stream_id=0))
    return st, ddh.aperture(N), st.frame(0).astype(np.complex128)


def test_plain_loop_without_bootstrap_stays_at_r_zero():
    """r = 0 is a fixed point of EM up to the floor (w = 0, so s = 0 and the
    cubic's root is 0): twenty plain EM iterations from r = 0 leave r within
    0.1 % of the floor, which is why the conventional loop starts with a
    reset.  Zero iterations return the start state."""
    st, a, y = _mbir_case()
    prm = ddh.Params(sigma_w2=st.sigma_w2)
    r, phi = np.zeros((16, 16)), np.zeros((16, 16))
    for _ in range(20):
        r, phi = ddh.em(r, phi, y, a, prm)
    assert r.max() < 1.001 * prm.r_floor
    assert np.abs(phi).max() < 1e-6
    r, phi = ddh.dh_mbir(y, a, prm, iters=0, reset_every=1, r0=np.ones((16, 16)), phi0=np.full((16, 16), 0.5))
    assert np.all(r == 1.0) and np.all(phi == 0.5)
    r, _ = ddh.dh_mbir(y, a, prm, iters=1, reset_every=1)
    assert r.max() > 1e3 * prm.r_floor


def test_full_bootstrap_reset_discards_the_previous_r():
    """With lambda = 1 a reset replaces r by the back-projection estimate, so
    the result of a run that starts with a reset does not depend on r0; with
    lambda < 1 it does."""
    import dataclasses
    st, a, y = _mbir_case()
    rng = np.random.default_rng(3)
    phi0 = 0.2 * rng.standard_normal((16, 16))
    full = dataclasses.replace(ddh.Params(sigma_w2=st.sigma_w2), lam=1.0)
    outs = [ddh.dh_mbir(y, a, full, iters=7, reset_every=3, r0=r0, phi0=phi0)
            for r0 in (np.zeros((16, 16)), rng.uniform(0.1, 2.0, (16, 16)))]
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    part = dataclasses.replace(full, lam=0.45)
    outs = [ddh.dh_mbir(y, a, part, iters=2, reset_every=3, r0=r0, phi0=phi0)
            for r0 in (np.zeros((16, 16)), np.ones((16, 16)))]
    assert not np.array_equal(outs[0][0], outs[1][0])


def test_conventional_loop_cost_decreases_between_resets():
    """Between two resets the iterations are plain EM steps, each of which
    does not increase the MAP surrogate cost U."""
    import dataclasses
    from oracle import metrics as M
    st, a, y = _mbir_case()
    prm = dataclasses.replace(ddh.Params(sigma_w2=st.sigma_w2), lam=1.0)
    yh = ddh.normalize(y)
    r, phi = ddh.dh_mbir(y, a, prm, iters=1, reset_every=50)
    U = [M.cost_U(r, phi, yh, a, prm)]
    for _ in range(10):
        r, phi = ddh.em(r, phi, y, a, prm)
        U.append(M.cost_U(r, phi, yh, a, prm))
    r2, phi2 = ddh.dh_mbir(y, a, prm, iters=11, reset_every=50)
    np.testing.assert_array_equal(r2, r)
    np.testing.assert_array_equal(phi2, phi)
    assert np.all(np.diff(U) <= 1e-12 * np.abs(U[1:]))
