"""FP64 CPU oracle for the Fourier-domain operators of Sections 2 and 3.1
(test infrastructure only: tests, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` may use it; the GPU library never does).

The Fourier form of the problem (eq:four_obj) replaces each measured
projection by its one-dimensional DFT over the detector bins.  By the Fourier
slice theorem, the DFT of the projection at angle theta_k and radial frequency
rho_q samples the two-dimensional Fourier transform of the image at
xi = rho_q (cos theta_k, sin theta_k).  With pixel modes m (integer offsets from
the image centre) the forward map is the nonuniform DFT

    (F_nu^* mu)_p = sum_m mu_m exp(-i xi_p . m),

its adjoint (F_nu fhat)_m = sum_p fhat_p exp(+i xi_p . m), and the split
Bregman system eq:SBFFT needs the normal operator H = Re(F_nu F_nu^*): the
dense "plain definition" here (``nudft_*``).

Section 3.1 evaluates H through Gaussian gridding (the NUFFT of Greengard and
Lee): F_nu F_nu^* ~ A F_D B B^* F_D^* A (eq:fusedop), with

* A: the diagonal deconvolution sqrt(pi/tau) exp(k^2 tau) per dimension,
* F_D^*: the DFT (sign -) of the zero-padded, scaled image onto an M x M grid
  of frequencies eta_l = 2 pi l / M, F_D its adjoint (sign +),
* B^*: interpolation of the grid at each xi_p with the periodic heat kernel
  exp(-|xi_p - eta_l|^2 / (4 tau)) over the 2 M_sp nearest grid points per
  dimension, scaled by 1/M^2 (the trapezoid rule of the convolution), and
  B its adjoint (spreading),
* B B^*: the precomputed sparse grid-to-grid matrix that fuses the two
  convolutions into one product.

``nufft_fwd``/``nufft_adj`` are the gridded F_nu^* and F_nu (the paper's NUFFT
baseline), ``fused_normal`` is eq:fusedop with B B^* formed as one sparse
matrix.  The pins in tests/test_oracle_fourier.py tie the dense definition to
closed forms (Dirichlet kernels at one angle, the trace) and the gridded
operators to the dense definition within Greengard-Lee's accuracy.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# sample points and the plain definition
# ---------------------------------------------------------------------------

def points(n_angles: int, n_bins: int, measured=None) -> np.ndarray:
    """Frequencies xi_p = rho_q (cos theta_k, sin theta_k), angle-major over
    the measured angles theta_k = pi k / n_angles and, within an angle,
    q = -Q .. Q ascending with rho_q = 2 pi q / n_bins and Q = (n_bins-1)//2
    (the DFT frequencies of a projection of n_bins unit-spaced bins; for an
    even bin count the unpaired Nyquist frequency is left out so that the set
    is closed under xi -> -xi)."""
    ks = np.arange(n_angles) if measured is None else np.flatnonzero(np.asarray(measured))
    Q = (n_bins - 1) // 2
    rho = 2.0 * np.pi * np.arange(-Q, Q + 1) / n_bins
    th = np.pi * ks / n_angles
    xi = np.empty((len(ks) * len(rho), 2))
    xi[:, 0] = (np.cos(th)[:, None] * rho[None, :]).ravel()
    xi[:, 1] = (np.sin(th)[:, None] * rho[None, :]).ravel()
    return xi


def modes(n: int) -> np.ndarray:
    """Pixel index ix -> mode ix - n//2 (the same along y)."""
    return np.arange(n) - n // 2


def _phases(n, xi):
    m = modes(n)
    return np.exp(-1j * np.outer(xi[:, 0], m)), np.exp(-1j * np.outer(xi[:, 1], m))


def nudft_fwd(n: int, xi: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """(F_nu^* mu)_p = sum over pixels of mu exp(-i xi_p . m), mu as [iy][ix]."""
    ex, ey = _phases(n, xi)
    img = np.asarray(mu, dtype=float).reshape(n, n)
    return np.einsum("py,yx,px->p", ey, img, ex)


def nudft_adj(n: int, xi: np.ndarray, fh: np.ndarray) -> np.ndarray:
    """(F_nu fhat)_m = sum_p fhat_p exp(+i xi_p . m), complex image [iy][ix]."""
    ex, ey = _phases(n, xi)
    return np.einsum("p,py,px->yx", np.asarray(fh, dtype=complex), ey.conj(), ex.conj()).ravel()


def nudft_normal(n: int, xi: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """H mu = Re(F_nu F_nu^* mu) by the dense definition."""
    return nudft_adj(n, xi, nudft_fwd(n, xi, mu)).real


# ---------------------------------------------------------------------------
# Gaussian gridding (Section 3.1)
# ---------------------------------------------------------------------------

def default_grid(n: int) -> int:
    """Oversampled grid: the smallest power of two >= 2n (the paper's 2N
    points per dimension, rounded up to a power of two)."""
    m = 1
    while m < 2 * n:
        m *= 2
    return m


def default_tau(grid: int, m_sp: int) -> float:
    """tau = 4 M_sp / M^2 on an M-point grid: the pairing (M_sp, tau) =
    (6, 6/N^2), (12, 12/N^2) that Section 3.1 quotes for 6 and 12 digits on
    the 2N-point grid, kept at the same width in grid spacings when M > 2N."""
    return 4.0 * m_sp / float(grid * grid)


class Gridding:
    """The pieces A, F_D, B of eq:fusedop for one image size and point set."""

    def __init__(self, n: int, xi: np.ndarray, m_sp: int = 6, tau: float | None = None,
                 grid: int | None = None, values: str = "f64"):
        """values="f32" rounds the stored tables as a library that keeps them
        in FP32 does: every entry of S (each window product g_y g_x) and every
        entry of S S^T (formed from the unrounded S), each rounded once; the
        rest stays FP64."""
        self.n, self.xi = n, np.asarray(xi, dtype=float)
        self.values = values
        self.m_sp = m_sp
        self.M = default_grid(n) if grid is None else int(grid)
        self.tau = default_tau(self.M, m_sp) if tau is None else float(tau)
        if self.M < 2 * n:
            raise ValueError("grid must be at least 2n")
        self.S = self._spread_matrix()
        self.S_used = self.S if values == "f64" else self._round32(self.S)

    @staticmethod
    def _round32(A):
        A = A.copy()
        A.data = A.data.astype(np.float32).astype(np.float64)
        return A

    def a_diag(self) -> np.ndarray:
        """A on the image: product over the two dimensions of
        sqrt(pi/tau) exp(k^2 tau) (the inverse Fourier coefficient of the
        periodic heat kernel)."""
        m = modes(self.n).astype(float)
        a1 = np.sqrt(np.pi / self.tau) * np.exp(m * m * self.tau)
        return np.outer(a1, a1)

    def window(self, c: np.ndarray):
        """For coordinates c (one dimension): the 2 M_sp nearest grid indices
        l = floor(c/h) - M_sp + 1 .. floor(c/h) + M_sp (unwrapped, h = 2 pi/M)
        and the heat-kernel weights exp(-(c - l h)^2 / (4 tau))."""
        h = 2.0 * np.pi / self.M
        base = np.floor(c / h).astype(np.int64)
        ls = base[:, None] + np.arange(-self.m_sp + 1, self.m_sp + 1)[None, :]
        w = np.exp(-((c[:, None] - ls * h) ** 2) / (4.0 * self.tau))
        return ls, w

    def _spread_matrix(self):
        """S[l, p] = g(xi_p - eta_l) for the grid points l in p's window
        (grid index l_y * M + l_x, periodic), as a sparse M^2 x P matrix; the
        spreading B is S / M^2 and the interpolation B^* is S^T / M^2."""
        M, P = self.M, len(self.xi)
        lx, wx = self.window(self.xi[:, 0])
        ly, wy = self.window(self.xi[:, 1])
        k = 2 * self.m_sp
        rows = ((ly[:, :, None] % M) * M + (lx[:, None, :] % M)).reshape(P, k * k)
        vals = (wy[:, :, None] * wx[:, None, :]).reshape(P, k * k)
        cols = np.repeat(np.arange(P), k * k).reshape(P, k * k)
        return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(M * M, P))

    def _pad(self, img: np.ndarray) -> np.ndarray:
        """Zero-padded M x M array with mode m at index m mod M."""
        M, n = self.M, self.n
        G = np.zeros((M, M), dtype=complex)
        idx = modes(n) % M
        G[np.ix_(idx, idx)] = img.reshape(n, n)
        return G

    def _crop(self, G: np.ndarray) -> np.ndarray:
        idx = modes(self.n) % self.M
        return G[np.ix_(idx, idx)]

    # F_D^* A: scaled image -> grid values h(eta_l) = sum_m c_m exp(-i m . eta_l)
    def grid_of_image(self, mu: np.ndarray) -> np.ndarray:
        c = self.a_diag() * np.asarray(mu, dtype=float).reshape(self.n, self.n)
        return np.fft.fft2(self._pad(c))

    # A F_D: grid values s(eta_l) -> A_m sum_l s_l exp(+i m . eta_l)
    def image_of_grid(self, s: np.ndarray) -> np.ndarray:
        t = np.fft.ifft2(s.reshape(self.M, self.M)) * (self.M * self.M)
        return (self.a_diag() * self._crop(t)).ravel()

    def nufft_fwd(self, mu: np.ndarray) -> np.ndarray:
        """Gridded F_nu^* mu = B^* F_D^* A mu (type-2 NUFFT)."""
        h = self.grid_of_image(mu).ravel()
        return (self.S_used.T @ h) / (self.M * self.M)

    def nufft_adj(self, fh: np.ndarray) -> np.ndarray:
        """Gridded F_nu fhat = A F_D B fhat (type-1 NUFFT), complex image."""
        s = (self.S_used @ np.asarray(fh, dtype=complex)) / (self.M * self.M)
        return self.image_of_grid(s)

    def fused_matrix(self):
        """B B^* = S S^T / M^4: the grid-to-grid matrix of eq:fusedop."""
        SS = (self.S @ self.S.T).tocsr()
        if self.values != "f64":
            SS = self._round32(SS)
        return SS / float(self.M) ** 4

    def fused_normal(self, mu: np.ndarray, BB=None) -> np.ndarray:
        """Re(A F_D (B B^*) F_D^* A mu), eq:fusedop with B B^* precomputed."""
        BB = self.fused_matrix() if BB is None else BB
        h = self.grid_of_image(mu).ravel()
        return self.image_of_grid(BB @ h).real


# ---------------------------------------------------------------------------
# the solvers of Section 2 on the Fourier system (eq:SBFFT)
# ---------------------------------------------------------------------------

def grad(n, u):
    u = u.reshape(n, n)
    gx = np.zeros((n, n))
    gy = np.zeros((n, n))
    gx[:, :-1] = u[:, 1:] - u[:, :-1]
    gy[:-1, :] = u[1:, :] - u[:-1, :]
    return gx.ravel(), gy.ravel()


def gradT(n, vx, vy):
    vx, vy = vx.reshape(n, n), vy.reshape(n, n)
    out = np.zeros((n, n))
    out[:, 1:] += vx[:, :-1]
    out[:, :-1] -= vx[:, :-1]
    out[1:, :] += vy[:-1, :]
    out[:-1, :] -= vy[:-1, :]
    return out.ravel()


def normal(H, n, x, alpha, lam, sigma=0.0):
    """alpha H x + lambda K^T K x + sigma x for a callable H."""
    gx, gy = grad(n, x)
    return alpha * H(x) + lam * gradT(n, gx, gy) + sigma * x


def cg(A, x, r, n_iter):
    """Hestenes-Stiefel CG on A (callable), x and r updated in place; the
    guards of the library's solver (stop at rho = 0, breakdown when
    <p, Ap> <= 0 or not finite).  Returns (iterations, breakdown)."""
    p = r.copy()
    rho = float(r @ r)
    for it in range(n_iter):
        if rho == 0.0:
            return it, 0
        q = A(p)
        gamma = float(p @ q)
        if not (gamma > 0.0) or not math.isfinite(gamma):
            return it, it + 1
        a = rho / gamma
        x += a * p
        r -= a * q
        rho_new = float(r @ r)
        p = r + (rho_new / rho) * p
        rho = rho_new
    return n_iter, 0


def sb(H, n, g_f, alpha, lam, n_outer, n_cg, tol=0.0):
    """Anisotropic-TV split Bregman on (alpha H + lambda K^T K) u =
    g_f + lambda K^T (d - b) (eq:SBFFT with g_f = alpha Re(F_nu fhat)): the
    same steps as the sparse-matrix solver (warm-started CG of n_cg steps with
    the carried residual, shrink by 1/lambda, Bregman update).  Returns
    (u, upd_b list)."""
    nn = n * n
    u = np.zeros(nn)
    dx, dy, bx, by = (np.zeros(nn) for _ in range(4))
    r = np.asarray(g_f, dtype=float).copy()
    A = lambda v: normal(H, n, v, alpha, lam)
    upd = []
    for k in range(n_outer):
        wx, wy = dx - bx, dy - by
        cg(A, u, r, n_cg)
        gx, gy = grad(n, u)
        t = 1.0 / lam
        ndx = np.sign(gx + bx) * np.maximum(np.abs(gx + bx) - t, 0.0)
        ndy = np.sign(gy + by) * np.maximum(np.abs(gy + by) - t, 0.0)
        nbx, nby = bx + gx - ndx, by + gy - ndy
        upd.append(float(np.abs(nbx - bx).sum() + np.abs(nby - by).sum()))
        r += lam * gradT(n, (ndx - nbx) - wx, (ndy - nby) - wy)
        dx, dy, bx, by = ndx, ndy, nbx, nby
        if tol > 0.0 and k > 0 and upd[-1] < tol * upd[0]:
            break
    return u, upd
