"""Pins for the oracle's K, K^T and normal operator.

* K^T is the exact transpose of K; K annihilates constants; the spectrum of
  K^T K is the closed form of the Neumann grid Laplacian (DCT-II modes):
  4 sin^2(pi p / 2N) + 4 sin^2(pi q / 2N);
* A = alpha R^T M^T M R + lambda K^T K + sigma I (the operator of eq:KKT,
  eq:PD_resolve, eq:SB_solve, Section 2) is symmetric and positive and
  matches the dense composition of its parts;
* the point-spread function of R^T R around the centre pixel falls off like
  n_meas / (pi rho), the continuum behaviour of backprojected projections.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_K_transpose_and_constants(n):
    rng = np.random.default_rng(n)
    u = rng.standard_normal(n * n)
    vx, vy = rng.standard_normal(n * n), rng.standard_normal(n * n)
    gx, gy = oracle.grad(n, u)
    lhs = np.dot(gx, vx) + np.dot(gy, vy)
    rhs = np.dot(u, oracle.gradT(n, vx, vy))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    cx, cy = oracle.grad(n, np.full(n * n, 3.25))
    assert not cx.any() and not cy.any()


@pytest.mark.parametrize("n", [4, 7, 8])
def test_KtK_spectrum_closed_form(n):
    M = np.zeros((n * n, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        M[:, j] = oracle.gradT(n, *oracle.grad(n, e))
    assert np.array_equal(M, M.T)
    ev = np.sort(np.linalg.eigvalsh(M))
    p = np.arange(n)
    lam = (4 * np.sin(np.pi * p / (2 * n)) ** 2)[:, None] + (4 * np.sin(np.pi * p / (2 * n)) ** 2)[None, :]
    np.testing.assert_allclose(ev, np.sort(lam.reshape(-1)), atol=1e-12)


def test_K_values_on_a_ramp():
    # u = ix gives D_x u = 1 except the last column, D_y u = 0
    n = 6
    u = np.tile(np.arange(n, dtype=float), n)
    gx, gy = oracle.grad(n, u)
    want = np.tile(np.r_[np.ones(n - 1), 0.0], n)
    np.testing.assert_array_equal(gx, want)
    assert not gy.any()


def test_normal_operator_dense_composition_and_spd():
    n, na = 8, 9
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, 2)
    op = oracle.OracleOp(n, na, nb, mask)
    R = op.MR.to_dense()
    KtK = np.zeros((n * n, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        KtK[:, j] = oracle.gradT(n, *oracle.grad(n, e))
    alpha, lam, sigma = 10.0, 1.0, 0.5
    A = alpha * R.T @ R + lam * KtK + sigma * np.eye(n * n)
    rng = np.random.default_rng(0)
    for _ in range(3):
        x = rng.standard_normal(n * n)
        np.testing.assert_allclose(op.normal(x, alpha, lam, sigma), A @ x, rtol=1e-12, atol=1e-10)
    x, y = rng.standard_normal(n * n), rng.standard_normal(n * n)
    a, b = np.dot(op.normal(x, alpha, lam), y), np.dot(x, op.normal(y, alpha, lam))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.dot(x, op.normal(x, alpha, lam)) > 0
    # the measured rows are exactly the rows of the full R at measured angles
    full = oracle.build_R(n, na, nb).to_dense()
    sel = np.concatenate([np.arange(k * nb, (k + 1) * nb) for k in range(na) if mask[k]])
    np.testing.assert_array_equal(full[sel], R)


def test_point_spread_function_decay():
    n, na = 128, 90
    op = oracle.OracleOp(n, na, W.n_bins_for(n))
    c = (n // 2) * n + n // 2
    d = np.zeros(op.nn)
    d[c] = 1.0
    alpha = 10.0
    psf = op.normal(d, alpha, 0.0, 0.0).reshape(n, n)
    iy, ix = np.mgrid[0:n, 0:n]
    rho = np.hypot(ix - n // 2, iy - n // 2)
    for r in (4, 8, 16, 24):
        ring = (rho >= r - 0.5) & (rho < r + 0.5)
        got = psf[ring].mean()
        want = alpha * na / (math.pi * r)
        assert abs(got / want - 1) < 0.1, (r, got, want)


def test_single_precision_values_option():
    """values="f32": every entry is the FP64 entry rounded once to binary32, in
    both the matrix and its transpose, and products move by at most the
    binary32 unit roundoff relative to the FP64 operator."""
    n, na = 24, 13
    nb = W.n_bins_for(n)
    a = oracle.OracleOp(n, na, nb)
    b = oracle.OracleOp(n, na, nb, values="f32")
    np.testing.assert_array_equal(b.MR.rp, a.MR.rp)
    np.testing.assert_array_equal(b.MR.ci, a.MR.ci)
    np.testing.assert_array_equal(b.MR.v, a.MR.v.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(b.MRT.v, a.MRT.v.astype(np.float32).astype(np.float64))
    assert np.any(b.MR.v != a.MR.v)
    x = np.abs(np.random.default_rng(0).standard_normal(n * n))
    ya, yb = a.fwd(x), b.fwd(x)
    assert np.max(np.abs(ya - yb) / np.maximum(ya, 1e-300)) <= 2.0 ** -24
    with pytest.raises(ValueError):
        oracle.OracleOp(n, na, nb, values="f16")
