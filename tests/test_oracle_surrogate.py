"""Pins for the oracle's surrogate operator T (Section 3.2, eq:def_sparse_surr).

T is the sum over pixels q of the centre pixel's point-spread function
P = R^T M^T M R e_c moved to q and cut to the disc of radius r, entries
outside the image dropped.  The pins check it through routes independent of
the stencil loop:

* its weights are the exact operator's column for the centre pixel (read off
  ora_normal applied to e_c), symmetrised; for odd N that column is already
  point-symmetric;
* T e_q is that window moved to q, for interior q, and clipped (not wrapped)
  at the image edge;
* r = 0 gives P_cc times the identity;
* T is exactly symmetric, and for r = 2 on a small geometry positive definite,
  where split Bregman on eq:surr_SBupd with exact inner solves must reach the
  unique minimiser of alpha/2 u^T T u - alpha u^T (MR)^T f + ||K u||_1, found
  independently by a primal-dual (Chambolle-Pock) iteration.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def make(n, na, every=1):
    return oracle.OracleOp(n, na, W.n_bins_for(n), W.angle_mask(na, every))


def psf(op):
    n = op.n
    e = np.zeros(op.nn)
    e[(n // 2) * n + n // 2] = 1.0
    return op.normal(e, 1.0, 0.0, 0.0).reshape(n, n)


@pytest.mark.parametrize("n,na,r", [(16, 12, 1), (16, 12, 3), (15, 30, 2), (20, 9, 4)])
def test_weights_are_the_symmetrised_centre_column(n, na, r):
    op = make(n, na)
    P = psf(op)
    c = n // 2
    w = op.surrogate_weights(r)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            want = 0.5 * (P[c + dy, c + dx] + P[c - dy, c - dx]) if dy * dy + dx * dx <= r * r else 0.0
            assert w[dy + r, dx + r] == pytest.approx(want, rel=1e-13, abs=1e-13)


def test_odd_n_column_is_already_point_symmetric():
    op = make(15, 30)
    P = psf(op)
    r, c = 3, 7
    win = P[c - r:c + r + 1, c - r:c + r + 1]
    np.testing.assert_allclose(win, win[::-1, ::-1], rtol=0, atol=1e-12 * np.abs(win).max())
    w = op.surrogate_weights(r)
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    inside = yy ** 2 + xx ** 2 <= r * r
    np.testing.assert_allclose(w[inside], win[inside], rtol=1e-13)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_translation_and_edge_clipping(r):
    n = 14
    op = make(n, 11)
    w = op.surrogate_weights(r)
    sur = op.with_surrogate(r)
    for qy, qx in ((6, 5), (3, 9), (0, 0), (n - 1, 2), (1, n - 1)):
        e = np.zeros(op.nn)
        e[qy * n + qx] = 1.0
        Te = sur.normal(e, 1.0, 0.0, 0.0).reshape(n, n)
        want = np.zeros((n, n))
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                py, px = qy + dy, qx + dx
                if 0 <= py < n and 0 <= px < n:
                    want[py, px] = w[dy + r, dx + r]
        np.testing.assert_allclose(Te, want, rtol=0, atol=1e-13 * np.abs(w).max())
        # nothing wraps to the opposite edge
        if qy == 0:
            assert not Te[n - r:, :].any()


def test_radius_zero_is_a_scaled_identity():
    op = make(12, 10)
    P = psf(op)
    sur = op.with_surrogate(0)
    x = np.random.default_rng(1).standard_normal(op.nn)
    got = sur.normal(x, 2.0, 0.5, 0.25)
    from oracle import grad, gradT
    gx, gy = grad(op.n, x)
    want = 2.0 * P[6, 6] * x + 0.5 * gradT(op.n, gx, gy) + 0.25 * x
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def dense(fn, m):
    return np.column_stack([fn(np.eye(m)[j]) for j in range(m)])


def test_symmetric_and_positive_at_radius_two():
    op = make(9, 16)
    sur = op.with_surrogate(2)
    T = dense(lambda e: sur.normal(e, 1.0, 0.0, 0.0), op.nn)
    assert np.array_equal(T, T.T)
    assert np.linalg.eigvalsh(T).min() > 1.0


def solve_quadratic_tv_pdhg(Q, b, Kd, alpha, iters=60000):
    """Chambolle-Pock on min_u ||K u||_1 + alpha/2 u^T Q u - alpha b^T u."""
    n = Q.shape[0]
    L = np.linalg.norm(Kd, 2)
    tau = sigma = 0.99 / L
    Minv = np.linalg.inv(np.eye(n) + tau * alpha * Q)
    u = np.zeros(n)
    ub = u.copy()
    y = np.zeros(Kd.shape[0])
    for _ in range(iters):
        y = np.clip(y + sigma * (Kd @ ub), -1.0, 1.0)
        un = Minv @ (u - tau * (Kd.T @ y) + tau * alpha * b)
        ub = 2 * un - u
        u = un
    return u


def test_surrogate_split_bregman_reaches_its_minimiser():
    n, na, r = 9, 16, 2
    op = make(n, na)
    sur = op.with_surrogate(r)
    T = dense(lambda e: sur.normal(e, 1.0, 0.0, 0.0), op.nn)
    Kd = np.vstack([dense(lambda e: oracle.grad(n, e)[0], op.nn),
                    dense(lambda e: oracle.grad(n, e)[1], op.nn)])
    mu = W.phantom(n, 3, seed=4)
    f = op.fwd(mu) + 0.05 * np.random.default_rng(4).standard_normal(op.rows)
    alpha, lam = 0.5, 1.0
    u_sb = sur.sb(f, alpha, lam, n_outer=3000, n_cg=200)[0]
    u_pd = solve_quadratic_tv_pdhg(T, op.adj(f), Kd, alpha)
    assert np.linalg.norm(u_sb - u_pd) <= 1e-6 * np.linalg.norm(u_pd), np.linalg.norm(u_sb - u_pd)


def test_disc_must_fit():
    with pytest.raises(ValueError):
        make(6, 5).surrogate_weights(3)
