"""Pins for the Fourier-domain oracle (Sections 2 and 3.1: eq:four_obj,
eq:SBFFT, eq:fusedop).

* the dense definition H = Re(F_nu F_nu^*) against closed forms: at one angle
  theta = 0 (or pi/2) H is the Dirichlet kernel of the radial frequencies
  along x (or y) and constant along the other axis; its diagonal is the number
  of sample points; it is symmetric and positive semi-definite, and real
  because the sample set is closed under xi -> -xi;
* the deconvolution A against a quadrature of the periodic heat kernel's
  Fourier coefficients (its inverse);
* the gridded transforms against the dense definition within Greengard-Lee's
  accuracy (6 digits for M_sp = 6, tau = 6/N^2; about 12 for M_sp = 12) in
  their native measure, max error over ||input||_1; the gridded pair is an
  exact adjoint pair;
* eq:fusedop with B B^* as one sparse matrix equals the unfused B B^*
  product to rounding, and is close to H;
* CG on a dense SPD system against a direct solve, and split Bregman on the
  fused system against an independent primal-dual iteration on the same
  objective.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fourier as F


def dense(fn, m):
    return np.column_stack([fn(np.eye(m)[j]) for j in range(m)])


def dirichlet(Q, n_bins, d):
    """sum_{q=-Q..Q} cos(2 pi q d / n_bins) in closed form."""
    t = np.pi * np.asarray(d, dtype=float) / n_bins
    out = np.full(t.shape, 2.0 * Q + 1.0)
    nz = np.abs(np.sin(t)) > 1e-12
    out[nz] = np.sin((2 * Q + 1) * t[nz]) / np.sin(t[nz])
    return out


def test_points_closed_under_negation():
    for nb in (23, 24):
        xi = F.points(10, nb)
        Q = (nb - 1) // 2
        assert len(xi) == 10 * (2 * Q + 1)
        per = xi.reshape(10, 2 * Q + 1, 2)
        np.testing.assert_array_equal(per, -per[:, ::-1, :])
        assert np.abs(xi).max() < np.pi


@pytest.mark.parametrize("n,nb", [(12, 17), (9, 13), (10, 14)])
def test_single_angle_is_a_dirichlet_kernel(n, nb):
    na = 8
    Q = (nb - 1) // 2
    iy, ix = np.divmod(np.arange(n * n), n)
    for k, axis in ((0, ix), (na // 2, iy)):   # theta = 0 and theta = pi/2
        mask = np.zeros(na, dtype=np.uint8)
        mask[k] = 1
        xi = F.points(na, nb, mask)
        for j in (0, n * n // 2 + 3, n * n - 1):
            e = np.zeros(n * n)
            e[j] = 1.0
            got = F.nudft_normal(n, xi, e)
            want = dirichlet(Q, nb, axis - axis[j])
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * (2 * Q + 1))


def test_definition_is_real_symmetric_psd_with_trace():
    n, na, nb = 6, 7, 9
    xi = F.points(na, nb, W.angle_mask(na, 1))
    H = dense(lambda e: F.nudft_normal(n, xi, e), n * n)
    np.testing.assert_allclose(np.diag(H), len(xi), rtol=1e-13)
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-11 * len(xi))
    assert np.linalg.eigvalsh(H).min() > -1e-10 * len(xi)
    mu = np.random.default_rng(0).standard_normal(n * n)
    z = F.nudft_adj(n, xi, F.nudft_fwd(n, xi, mu))
    assert np.abs(z.imag).max() <= 1e-11 * np.abs(z.real).max()


@pytest.mark.parametrize("n,grid,m_sp", [(16, 32, 6), (24, 64, 12), (33, 128, 6)])
def test_deconvolution_inverts_the_heat_kernel_coefficients(n, grid, m_sp):
    g = F.Gridding(n, F.points(3, 5), m_sp, grid=grid)
    tau = g.tau
    L = 4096
    x = 2 * np.pi * np.arange(L) / L
    ell = np.arange(-4, 5)
    kern = np.exp(-((x[:, None] - 2 * np.pi * ell[None, :]) ** 2) / (4 * tau)).sum(axis=1)
    m = F.modes(n)
    coef = np.array([(kern * np.exp(-1j * k * x)).mean() for k in m]).real
    a = g.a_diag()
    np.testing.assert_allclose(1.0 / a[n // 2, :] / (1.0 / a[n // 2, n // 2]), coef / coef[n // 2],
                               rtol=1e-12)
    np.testing.assert_allclose(1.0 / a[n // 2, n // 2], coef[n // 2] ** 2, rtol=1e-12)


CASES = [(16, 12, 23, 1), (24, 20, 35, 1), (32, 25, 47, 2)]


@pytest.mark.parametrize("n,na,nb,ev", CASES)
@pytest.mark.parametrize("m_sp,eps", [(6, 1e-6), (12, 1e-11)])
def test_gridded_transforms_match_the_definition(n, na, nb, ev, m_sp, eps):
    rng = np.random.default_rng(n + m_sp)
    xi = F.points(na, nb, W.angle_mask(na, ev))
    g = F.Gridding(n, xi, m_sp)
    mu = rng.standard_normal(n * n)
    fh = rng.standard_normal(len(xi)) + 1j * rng.standard_normal(len(xi))
    assert np.abs(g.nufft_fwd(mu) - F.nudft_fwd(n, xi, mu)).max() <= eps * np.abs(mu).sum()
    assert np.abs(g.nufft_adj(fh) - F.nudft_adj(n, xi, fh)).max() <= eps * np.abs(fh).sum()


@pytest.mark.parametrize("n,na,nb,ev", CASES)
def test_gridded_pair_is_adjoint(n, na, nb, ev):
    rng = np.random.default_rng(7)
    xi = F.points(na, nb, W.angle_mask(na, ev))
    g = F.Gridding(n, xi, 6)
    mu = rng.standard_normal(n * n)
    fh = rng.standard_normal(len(xi)) + 1j * rng.standard_normal(len(xi))
    lhs = np.vdot(g.nufft_fwd(mu), fh)
    rhs = np.vdot(mu, g.nufft_adj(fh))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(g.nufft_fwd(mu)) * np.linalg.norm(fh)


@pytest.mark.parametrize("n,na,nb,ev", CASES)
@pytest.mark.parametrize("m_sp,tol", [(6, 1e-5), (12, 1e-10)])
def test_fused_operator(n, na, nb, ev, m_sp, tol):
    rng = np.random.default_rng(3)
    xi = F.points(na, nb, W.angle_mask(na, ev))
    g = F.Gridding(n, xi, m_sp)
    mu = rng.standard_normal(n * n)
    fused = g.fused_normal(mu)
    unfused = g.nufft_adj(g.nufft_fwd(mu)).real
    np.testing.assert_allclose(fused, unfused, rtol=0, atol=1e-12 * np.abs(unfused).max())
    H = F.nudft_normal(n, xi, mu)
    assert np.linalg.norm(fused - H) <= tol * np.linalg.norm(H)


def test_fused_matrix_symmetric_and_operator_psd():
    n = 8
    xi = F.points(9, 13)
    g = F.Gridding(n, xi, 4)
    BB = g.fused_matrix()
    assert abs(BB - BB.T).max() == 0.0
    Ht = dense(g.fused_normal, n * n)
    np.testing.assert_allclose(Ht, Ht.T, rtol=0, atol=1e-12 * np.abs(Ht).max())
    assert np.linalg.eigvalsh(0.5 * (Ht + Ht.T)).min() > -1e-10 * np.abs(Ht).max()


def test_cg_against_a_direct_solve():
    rng = np.random.default_rng(5)
    m = 40
    G = rng.standard_normal((m, m))
    A = G @ G.T + m * np.eye(m)
    b = rng.standard_normal(m)
    x, r = np.zeros(m), b.copy()
    it, bd = F.cg(lambda v: A @ v, x, r, m)
    assert bd == 0 and it == m
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r, b - A @ x, atol=1e-9 * np.linalg.norm(b))


def pdhg(Q, b, Kd, alpha, iters=40000):
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


def test_split_bregman_on_the_fused_system_reaches_its_minimiser():
    n = 8
    xi = F.points(10, 13)
    g = F.Gridding(n, xi, 6)
    mu = W.phantom(n, 3, seed=2)
    fh = g.nufft_fwd(mu) + 0.05 * np.random.default_rng(2).standard_normal(len(xi))
    alpha, lam = 0.05, 1.0
    b = g.nufft_adj(fh).real
    BB = g.fused_matrix()
    H = lambda v: g.fused_normal(v, BB)
    u_sb, upd = F.sb(H, n, alpha * b, alpha, lam, n_outer=2000, n_cg=32)
    Q = dense(H, n * n)
    Q = 0.5 * (Q + Q.T)
    Kd = np.vstack([dense(lambda e: F.grad(n, e)[0], n * n), dense(lambda e: F.grad(n, e)[1], n * n)])
    u_pd = pdhg(Q, b, Kd, alpha)
    assert np.linalg.norm(u_sb - u_pd) <= 1e-6 * np.linalg.norm(u_pd)
    assert upd[-1] < 1e-8 * upd[0]


def test_f32_tables_are_rounded_once():
    n = 16
    xi = F.points(12, 23)
    g64 = F.Gridding(n, xi, 6)
    g32 = F.Gridding(n, xi, 6, values="f32")
    np.testing.assert_array_equal(g32.S_used.data, g64.S.data.astype(np.float32))
    BB64, BB32 = g64.fused_matrix(), g32.fused_matrix()
    scale = float(g64.M) ** 4
    np.testing.assert_array_equal((BB32 * scale).data, (BB64 * scale).data.astype(np.float32))
    mu = np.random.default_rng(1).standard_normal(n * n)
    a, b = g64.fused_normal(mu, BB64), g32.fused_normal(mu, BB32)
    assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)


def test_fused_operator_psf_is_spread_and_its_truncation_indefinite():
    """Section 3.2 builds the surrogate T from the point-spread function of
    A F_D (B B^*) F_D^* A at the centre pixel.  At 64 x 64 (50 angles, 91 bins)
    that PSF is not concentrated (the r = 3 disc holds under 10% of its
    absolute mass: the DC samples add a constant, the polar density a 1/rho
    tail), and the symmetric stencil cut to the disc has an indefinite symbol,
    so alpha T + lambda K^T K is not SPD."""
    n = 64
    xi = F.points(50, W.n_bins_for(n))
    g = F.Gridding(n, xi, 6)
    e = np.zeros(n * n)
    c = n // 2
    e[c * n + c] = 1.0
    P = g.fused_normal(e).reshape(n, n)
    yy, xx = np.mgrid[-c:n - c, -c:n - c]
    r = 3
    disc = yy ** 2 + xx ** 2 <= r * r
    assert np.abs(P[disc]).sum() < 0.1 * np.abs(P).sum()
    G = np.zeros((128, 128))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dy * dy + dx * dx <= r * r:
                G[dy % 128, dx % 128] = 0.5 * (P[c + dy, c + dx] + P[c - dy, c - dx])
    sym = np.fft.fft2(G).real
    assert sym.min() < -0.05 * sym.max()
