"""Pins for the oracle's CG, split Bregman and gradients.

* CG on a 64-unknown system converges to numpy's dense solve; its residual
  recurrence matches the true residual and successive residuals are
  orthogonal (textbook CG properties);
* split Bregman with exact inner solves converges to the unique minimiser of
  alpha/2 ||MRu - f||^2 + ||Ku||_1 (eq:objmin with p = 1, K = grad), checked
  against an independent primal-dual (Chambolle-Pock) solve;
* the primal-dual (Chambolle-Pock) iteration with CG resolvents of
  eq:PD_resolve equals the same iteration with a dense inverse, and with
  inexact resolvents reaches the split-Bregman minimiser;
* split Bregman resume is bitwise, the carried residual stays consistent with
  the right-hand side of eq:SB_solve, and truncated inner solves still reduce
  the error (the error-forgetting behaviour of Section 3.2);
* loss gradients match central finite differences of the oracle's own
  forward pass and complex-step derivatives of an independent complex
  evaluation of the unrolled loss, and the unrolled-CG gradient reduces to a
  closed form when tau = 0.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def small_op(n=8, na=16, every=1):
    return oracle.OracleOp(n, na, W.n_bins_for(n), W.angle_mask(na, every))


def dense_A(op, alpha, lam, sigma):
    A = np.zeros((op.nn, op.nn))
    for j in range(op.nn):
        e = np.zeros(op.nn)
        e[j] = 1.0
        A[:, j] = op.normal(e, alpha, lam, sigma)
    return A


def test_cg_matches_dense_solve():
    op = small_op(8, 7, 1)
    alpha, lam, sigma = 10.0, 1.0, 0.0
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal(op.nn)
    A = dense_A(op, alpha, lam, sigma)
    want = np.linalg.solve(A, rhs)
    x, r, hist, it, bd = op.cg(alpha, lam, sigma, rhs=rhs, n_iter=400, rtol=1e-14)
    assert bd == 0
    assert np.linalg.norm(x - want) <= 1e-9 * np.linalg.norm(want)


def test_cg_recurrence_and_orthogonality():
    op = small_op(8, 12, 2)
    alpha, lam, sigma = 10.0, 1.0, 0.1
    rng = np.random.default_rng(2)
    rhs = rng.standard_normal(op.nn)
    rs = []
    for k in range(1, 7):
        x, r, hist, it, bd = op.cg(alpha, lam, sigma, rhs=rhs, n_iter=k)
        true_r = rhs - op.normal(x, alpha, lam, sigma)
        assert np.linalg.norm(r - true_r) <= 1e-10 * np.linalg.norm(rhs)
        assert abs(hist[-1] - np.dot(r, r)) <= 1e-12 * hist[0]
        rs.append(r)
    for i in range(len(rs)):
        for j in range(i):
            c = np.dot(rs[i], rs[j]) / (np.linalg.norm(rs[i]) * np.linalg.norm(rs[j]))
            assert abs(c) < 1e-8


def test_cg_guards():
    op = small_op(8, 6)
    x, r, hist, it, bd = op.cg(1.0, 1.0, 0.0, rhs=np.zeros(op.nn), n_iter=5)
    assert it == 0 and bd == 0 and not x.any() and np.all(hist == 0)
    # lambda = sigma = 0 with only theta = 0 measured: A = R^T R is singular, and an
    # image whose column sums vanish (row 0 = +1, row 1 = -1) lies in its null space,
    # so the first step finds <p, Ap> = 0 and CG reports a breakdown at iteration 1
    op1 = oracle.OracleOp(8, 4, W.n_bins_for(8), np.array([1, 0, 0, 0], np.uint8))
    rhs = np.zeros(op1.nn)
    rhs[:8] = 1.0
    rhs[8:16] = -1.0
    x, r, hist, it, bd = op1.cg(1.0, 0.0, 0.0, r0=rhs, n_iter=3)
    assert bd == 1 and it == 0


def solve_tv_pdhg(A, Kd, f, alpha, iters=60000):
    """Chambolle-Pock on min_u ||K u||_1 + alpha/2 ||A u - f||^2, quadratic in G."""
    n = A.shape[1]
    AtA, Atf = A.T @ A, A.T @ f
    L = np.linalg.norm(Kd, 2)
    tau = sigma = 0.99 / L
    M = np.linalg.inv(np.eye(n) + tau * alpha * AtA)
    u = np.zeros(n)
    ub = u.copy()
    y = np.zeros(Kd.shape[0])
    for _ in range(iters):
        y = np.clip(y + sigma * (Kd @ ub), -1.0, 1.0)
        un = M @ (u - tau * (Kd.T @ y) + tau * alpha * Atf)
        ub = 2 * un - u
        u = un
    return u


def test_split_bregman_reaches_tv_minimiser():
    n, na = 8, 12
    op = small_op(n, na, 1)
    A = op.MR.to_dense()
    Kd = np.zeros((2 * op.nn, op.nn))
    for j in range(op.nn):
        e = np.zeros(op.nn)
        e[j] = 1.0
        gx, gy = oracle.grad(n, e)
        Kd[:op.nn, j], Kd[op.nn:, j] = gx, gy
    mu = W.phantom(n, 3, seed=5)
    rng = np.random.default_rng(5)
    f = A @ mu + 0.05 * rng.standard_normal(A.shape[0])
    alpha, lam = 2.0, 1.0
    u_sb, ub, uu, k, _ = op.sb(f, alpha, lam, n_outer=3000, n_cg=200)
    u_pd = solve_tv_pdhg(A, Kd, f, alpha)
    assert np.linalg.norm(u_sb - u_pd) <= 1e-6 * np.linalg.norm(u_pd), np.linalg.norm(u_sb - u_pd)
    # and it is a minimiser: the objective does not drop along random perturbations
    E = lambda u: alpha / 2 * np.sum((A @ u - f) ** 2) + np.abs(Kd @ u).sum()
    for d in np.random.default_rng(9).standard_normal((20, op.nn)):
        assert E(u_sb + 1e-4 * d) >= E(u_sb) - 1e-12


def test_split_bregman_resume_is_bitwise():
    w = W.WORKLOADS["small_64_f64"]
    op = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    mu, eps = W.phantom_and_noise(w.n, w.n_ellipses, op.rows, seed=0)
    y = op.fwd(mu)
    f = y + w.noise * np.sqrt(np.mean(y ** 2)) * eps
    u20, b20, _, _, st20 = op.sb(f, w.alpha, w.lam, 20, 5)
    u10, b10, _, _, st10 = op.sb(f, w.alpha, w.lam, 10, 5)
    u, b2, _, _, st = op.sb(f, w.alpha, w.lam, 10, 5, u0=u10, state=st10)
    np.testing.assert_array_equal(u, u20)
    np.testing.assert_array_equal(st, st20)
    np.testing.assert_array_equal(np.r_[b10, b2], b20)


def test_split_bregman_carried_residual_and_error_forgetting():
    w = W.WORKLOADS["small_64_f64"]
    op = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    mu, eps = W.phantom_and_noise(w.n, w.n_ellipses, op.rows, seed=0)
    y = op.fwd(mu)
    f = y + w.noise * np.sqrt(np.mean(y ** 2)) * eps
    u, ub, uu, k, st = op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg)
    nn = op.nn
    dx, dy, bx, by, r = (st[i * nn:(i + 1) * nn] for i in range(5))
    # r is the residual of the *next* solve: alpha R^T f + lambda K^T (d - b) - A u
    rhs = w.alpha * op.adj(f) + w.lam * oracle.gradT(w.n, dx - bx, dy - by)
    true_r = rhs - op.normal(u, w.alpha, w.lam)
    assert np.linalg.norm(r - true_r) <= 1e-9 * np.linalg.norm(rhs)
    # truncated (10-step) inner solves still drive the error down over outer iterations
    errs = []
    for outer in (1, 5, 20):
        uo = op.sb(f, w.alpha, w.lam, outer, w.n_cg)[0]
        errs.append(np.abs(uo - mu).sum() / np.abs(mu).sum())
    assert errs[0] > errs[1] > errs[2], errs
    # Bregman updates shrink
    assert ub[-1] < ub[0]
    # tolerance stop: stops once the update falls below tol * first update
    u_t, ub_t, _, k_t, _ = op.sb(f, w.alpha, w.lam, 200, 5, tol=0.3)
    assert 1 < k_t < 200 and ub_t[-1] < 0.3 * ub_t[0] and np.all(ub_t[1:-1] >= 0.3 * ub_t[0])


def test_loss1_gradient_matches_finite_differences():
    op = small_op(8, 10, 1)
    rng = np.random.default_rng(4)
    mu, f = rng.standard_normal(op.nn), rng.standard_normal(op.rows)
    L, gm, gf = op.loss1(mu, f)
    r = op.fwd(mu) - f
    assert abs(L - 0.5 * np.dot(r, r)) <= 1e-12 * L
    for d_mu, d_f in zip(rng.standard_normal((4, op.nn)), rng.standard_normal((4, op.rows))):
        h = 1e-5
        Lp = op.loss1(mu + h * d_mu, f + h * d_f)[0]
        Lm = op.loss1(mu - h * d_mu, f - h * d_f)[0]
        fd = (Lp - Lm) / (2 * h)
        an = np.dot(gm, d_mu) + np.dot(gf, d_f)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


@pytest.mark.parametrize("n_iter", [1, 3, 10])
def test_loss2_gradient_matches_finite_differences(n_iter):
    op = small_op(8, 10, 1)
    rng = np.random.default_rng(10 + n_iter)
    mu, f = rng.uniform(0, 1, op.nn), rng.standard_normal(op.rows)
    ta = 0.1 * 10.0
    L, gm, gf, un = op.loss2(mu, f, ta, n_iter)
    # forward agrees with the oracle's own CG on (I + ta R^T R) u = mu + ta R^T f
    rhs = mu + ta * op.adj(f)
    u_cg = op.cg(ta, 0.0, 1.0, rhs=rhs, n_iter=n_iter)[0]
    np.testing.assert_allclose(un, u_cg, rtol=0, atol=1e-12 * np.abs(u_cg).max())
    def fd(h, d_mu, d_f):
        Lp = op.loss2(mu + h * d_mu, f + h * d_f, ta, n_iter)[0]
        Lm = op.loss2(mu - h * d_mu, f - h * d_f, ta, n_iter)[0]
        return (Lp - Lm) / (2 * h)

    # central differences at h = 1e-3 (error O(h^2)); smaller h is swamped by the
    # rounding noise of the nearly converged forward solve, so the tighter check
    # uses Richardson extrapolation of h = 2e-3 and 1e-3 instead
    for d_mu, d_f in zip(rng.standard_normal((4, op.nn)), rng.standard_normal((4, op.rows))):
        an = np.dot(gm, d_mu) + np.dot(gf, d_f)
        d1, d2 = fd(1e-3, d_mu, d_f), fd(2e-3, d_mu, d_f)
        assert abs(d1 - an) <= 1e-5 * max(1.0, abs(an)), (d1, an)
        assert abs((4 * d1 - d2) / 3 - an) <= 2e-6 * max(1.0, abs(an)), (d1, d2, an)


def test_loss2_at_tau_zero_is_closed_form():
    op = small_op(8, 10, 1)
    rng = np.random.default_rng(6)
    mu, f = rng.uniform(0, 1, op.nn), rng.standard_normal(op.rows)
    L, gm, gf, un = op.loss2(mu, f, 0.0, 10)
    # A = I: the first step returns u = mu, the residual is exactly zero, the rest are skipped
    np.testing.assert_array_equal(un, mu)
    L1, gm1, gf1 = op.loss1(mu, f)
    assert L == L1
    np.testing.assert_allclose(gm, gm1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gf, gf1, rtol=1e-12, atol=1e-12)


def _loss2_complex(op, mu, f, ta, n_iter):
    """The unrolled-CG loss evaluated in complex arithmetic with bilinear
    (non-conjugating) dots: the forward map of the loss, independent of the
    oracle's reverse sweep.  Products use the oracle's matrix entries through
    scipy, applied to real and imaginary parts separately."""
    import scipy.sparse as sp
    R = sp.csr_matrix((op.MR.v, op.MR.ci, op.MR.rp), shape=(op.rows, op.nn))
    RT = R.T.tocsr()

    def mv(M, z):
        return M @ z.real + 1j * (M @ z.imag)

    def A(z):
        return ta * mv(RT, mv(R, z)) + z

    dot = lambda a, b: np.sum(a * b)
    r = mu + ta * mv(RT, f)
    p, u, rho = r.copy(), np.zeros_like(r), dot(r, r)
    for _ in range(n_iter):
        if rho == 0:
            break
        q = A(p)
        a = rho / dot(p, q)
        u = u + a * p
        r = r - a * q
        rho_n = dot(r, r)
        p = r + (rho_n / rho) * p
        rho = rho_n
    res = mv(R, u) - f
    return 0.5 * dot(res, res)


@pytest.mark.parametrize("n_iter,tol", [(4, 1e-10), (10, 1e-6)])
def test_loss2_gradient_matches_complex_step(n_iter, tol):
    """Complex-step derivative (Squire & Trapp 1998): Im L(x + i h v) / h is
    the directional derivative to rounding, with no cancellation, for h tiny.
    After 10 steps two FP64 evaluations of the same map already differ at the
    1e-7 level (loss of orthogonality amplifies rounding), hence the looser
    bound there."""
    op = small_op(10, 12, 1)
    rng = np.random.default_rng(20 + n_iter)
    mu, f = rng.uniform(0, 1, op.nn), rng.standard_normal(op.rows)
    ta = 1.0
    L, gm, gf, _ = op.loss2(mu, f, ta, n_iter)
    h = 1e-30
    for _ in range(3):
        d_mu, d_f = rng.standard_normal(op.nn), rng.standard_normal(op.rows)
        cs = _loss2_complex(op, mu + 1j * h * d_mu, f + 1j * h * d_f, ta, n_iter).imag / h
        an = np.dot(gm, d_mu) + np.dot(gf, d_f)
        assert abs(cs - an) <= tol * abs(an), (cs, an)
    # the real part reproduces the loss (to the same rounding spread)
    assert abs(_loss2_complex(op, mu + 0j, f + 0j, ta, n_iter).real - L) <= tol * 1e-2 * L


def _dense_K(n):
    m = n * n
    Kd = np.zeros((2 * m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        gx, gy = oracle.grad(n, e)
        Kd[:m, j], Kd[m:, j] = gx, gy
    return Kd


def test_primal_dual_with_exact_resolvent_is_dense_chambolle_pock():
    """With the resolvent of eq:PD_resolve solved to convergence by CG, the
    oracle's primal-dual iterates are those of the same iteration with the
    resolvent applied as a dense inverse (numpy), after every outer step."""
    n, na = 8, 12
    op = small_op(n, na, 1)
    A = op.MR.to_dense()
    Kd = _dense_K(n)
    mu = W.phantom(n, 3, seed=7)
    f = A @ mu + 0.05 * np.random.default_rng(7).standard_normal(A.shape[0])
    alpha = 2.0
    L = np.linalg.norm(Kd, 2)
    tau = sigma = 0.99 / L
    for iters in (1, 7, 60):
        u_cg = op.pd(f, alpha, tau, sigma, n_outer=iters, n_cg=200)
        u_dense = solve_tv_pdhg(A, Kd, f, alpha, iters=iters)
        assert np.linalg.norm(u_cg - u_dense) <= 1e-10 * max(1.0, np.linalg.norm(u_dense)), iters


def test_primal_dual_reaches_tv_minimiser_and_warm_start():
    """Inexact resolvents (10 CG steps from the previous iterate) still reach
    the unique minimiser that split Bregman reaches (to the 5e-7 floor those
    inexact steps leave); a warm start begins at the given image."""
    n, na = 8, 12
    op = small_op(n, na, 1)
    A = op.MR.to_dense()
    Kd = _dense_K(n)
    mu = W.phantom(n, 3, seed=5)
    f = A @ mu + 0.05 * np.random.default_rng(5).standard_normal(A.shape[0])
    alpha, lam = 2.0, 1.0
    tau = sigma = 0.99 / np.sqrt(8.0)
    u_pd = op.pd(f, alpha, tau, sigma, n_outer=20000, n_cg=10)
    u_sb = op.sb(f, alpha, lam, n_outer=3000, n_cg=200)[0]
    assert np.linalg.norm(u_pd - u_sb) <= 1e-6 * np.linalg.norm(u_sb)
    # the warm start is the given image (the dual variable starts at 0)
    assert np.array_equal(op.pd(f, alpha, tau, sigma, n_outer=0, n_cg=10, u0=u_sb), u_sb)
    assert not np.array_equal(op.pd(f, alpha, tau, sigma, 3, 10, u0=u_sb),
                              op.pd(f, alpha, tau, sigma, 3, 10))


def test_results_do_not_depend_on_thread_count():
    """The oracle's parallel loops only split independent rows, pixels and
    rays; every sum runs in one thread in a fixed order.  So the build, the
    products and whole solves are bitwise the same on 1 and 4 threads."""
    n, na, nb = 48, 30, W.n_bins_for(48)
    mask = W.angle_mask(na, 2)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n * n)
    prev = oracle.set_threads(0)
    try:
        out = []
        for t in (1, 4):
            oracle.set_threads(t)
            op = oracle.OracleOp(n, na, nb, mask)
            f = op.fwd(x)
            out.append((op.MR.ci.copy(), op.MR.v.copy(), f, op.adj(f), op.normal(x, 0.3, 1.0, 0.1),
                        op.cg(0.3, 1.0, 0.1, rhs=x, n_iter=15)[0],
                        op.sb(f, 0.3, 1.0, 4, 5)[0]))
    finally:
        oracle.set_threads(prev)
    for a, b in zip(*out):
        assert np.array_equal(a, b)
