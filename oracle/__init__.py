"""FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_1705_07497_amd``: the arithmetic lives in ``oracle.c`` (plain C, FP64,
OpenMP over rows, sequential sums) and this file only marshals numpy arrays.

Every function follows the paper (Barnard & Archibald, arXiv 1705.07497):
the objective eq:objmin (Section 1), the normal operator of eq:KKT,
eq:PD_resolve and eq:SB_solve (Section 2), conjugate gradients for those
systems (Section 2) and anisotropic-TV split Bregman (Section 4), with the
Radon transform as an exact Siddon intersection-length matrix.  The Fourier
form of the problem (eq:four_obj, eq:SBFFT) and its convolution-fused normal
operator (eq:fusedop) live in ``oracle/fourier.py`` (numpy, FP64).

Parity: pinned by tests/test_oracle_*.py (brute-force clipping, closed forms,
invariants, dense solves, an independent primal-dual solver, finite and
complex-step derivatives).  The only parts with no pin beyond the oracle
itself are full-size CG/SB trajectories ("parity unpinned" there: the paper
prints no values for this operator).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (strict IEEE: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-std=gnu11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OraOp(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("rp", _i64p), ("ci", _i32p), ("v", _dp),
                ("trp", _i64p), ("tci", _i32p), ("tv", _dp),
                ("sur_r", ctypes.c_int32), ("sur_w", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.ora_trig.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.ora_ray.argtypes = [ctypes.c_int] * 5 + [_i32p, _dp]
        L.ora_ray.restype = ctypes.c_int
        L.ora_build.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p,
                                _i64p, _i32p, _dp]
        L.ora_transpose.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _dp,
                                    _i64p, _i32p, _dp]
        L.ora_spmv.argtypes = [ctypes.c_int64, _i64p, _i32p, _dp, _dp, _dp]
        L.ora_grad.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.ora_gradT.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        P = ctypes.POINTER(_OraOp)
        L.ora_normal.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.ora_cg.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp,
                             ctypes.c_int, ctypes.c_double, _dp, ctypes.POINTER(ctypes.c_int)]
        L.ora_cg.restype = ctypes.c_int
        L.ora_sb.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                             ctypes.c_double, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
        L.ora_sb.restype = ctypes.c_int
        L.ora_loss1.argtypes = [P, _dp, _dp, _dp, _dp]
        L.ora_loss1.restype = ctypes.c_double
        L.ora_loss2.argtypes = [P, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.ora_loss2.restype = ctypes.c_double
        L.ora_stencil.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.ora_pd.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.ora_pd.restype = ctypes.c_int
        L.ora_surrogate_weights.argtypes = [P, ctypes.c_int, _dp]
        L.ora_surrogate_weights.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n > 0) and return the count in
    effect.  Timing only: results do not depend on it."""
    return int(lib().ora_set_threads(int(n)))


def _p(a, typ=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def trig(k: int, n_angles: int) -> tuple[float, float]:
    c, s = ctypes.c_double(), ctypes.c_double()
    lib().ora_trig(k, n_angles, ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def ray(n: int, n_angles: int, n_bins: int, k: int, b: int) -> tuple[np.ndarray, np.ndarray]:
    """Entries (pixel index, length) of ray (k, b), sorted by pixel."""
    cols = np.zeros(2 * n + 4, dtype=np.int32)
    vals = np.zeros(2 * n + 4, dtype=np.float64)
    m = lib().ora_ray(n, n_angles, n_bins, k, b, _p(cols, _i32p), _p(vals))
    return cols[:m].copy(), vals[:m].copy()


@dataclass
class CSR:
    rows: int
    cols: int
    rp: np.ndarray   # int64[rows+1]
    ci: np.ndarray   # int32[nnz]
    v: np.ndarray    # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = _f64(x)
        assert x.shape == (self.cols,)
        y = np.empty(self.rows, dtype=np.float64)
        lib().ora_spmv(self.rows, _p(self.rp, _i64p), _p(self.ci, _i32p), _p(self.v), _p(x), _p(y))
        return y

    def transpose(self) -> "CSR":
        trp = np.empty(self.cols + 1, dtype=np.int64)
        tci = np.empty(self.nnz, dtype=np.int32)
        tv = np.empty(self.nnz, dtype=np.float64)
        lib().ora_transpose(self.rows, self.cols, _p(self.rp, _i64p), _p(self.ci, _i32p),
                            _p(self.v), _p(trp, _i64p), _p(tci, _i32p), _p(tv))
        return CSR(self.cols, self.rows, trp, tci, tv)

    def row(self, i: int) -> tuple[np.ndarray, np.ndarray]:
        a, b = self.rp[i], self.rp[i + 1]
        return self.ci[a:b], self.v[a:b]

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.rows, self.cols))
        for i in range(self.rows):
            c, v = self.row(i)
            d[i, c] += v
        return d


def build_R(n: int, n_angles: int, n_bins: int, angles=None) -> CSR:
    """CSR of R over the listed angle indices (default all), rows (angle, bin)."""
    if angles is None:
        angles = np.arange(n_angles, dtype=np.int32)
    angles = np.ascontiguousarray(angles, dtype=np.int32)
    rows = len(angles) * n_bins
    rp = np.zeros(rows + 1, dtype=np.int64)
    L = lib()
    L.ora_build(n, n_angles, n_bins, len(angles), _p(angles, _i32p), _p(rp, _i64p), None, None)
    nnz = int(rp[-1])
    ci = np.empty(nnz, dtype=np.int32)
    v = np.empty(nnz, dtype=np.float64)
    L.ora_build(n, n_angles, n_bins, len(angles), _p(angles, _i32p), _p(rp, _i64p),
                _p(ci, _i32p), _p(v))
    return CSR(rows, n * n, rp, ci, v)


def grad(n: int, u: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    u = _f64(u)
    gx = np.empty(n * n)
    gy = np.empty(n * n)
    lib().ora_grad(n, _p(u), _p(gx), _p(gy))
    return gx, gy


def gradT(n: int, vx: np.ndarray, vy: np.ndarray) -> np.ndarray:
    vx, vy = _f64(vx), _f64(vy)
    out = np.empty(n * n)
    lib().ora_gradT(n, _p(vx), _p(vy), _p(out))
    return out


class OracleOp:
    """MR and (MR)^T for one geometry; measured rays in ascending angle order."""

    def __init__(self, n: int, n_angles: int, n_bins: int, measured=None, values: str = "f64"):
        """values="f32" rounds every matrix entry once to binary32 (and back to
        float64): the matrix of an operator that stores its values in single
        precision, everything else still FP64."""
        self.n, self.n_angles, self.n_bins = n, n_angles, n_bins
        if measured is None:
            measured = np.ones(n_angles, dtype=np.uint8)
        self.measured = np.asarray(measured, dtype=np.uint8)
        self.angles = np.nonzero(self.measured)[0].astype(np.int32)
        self.MR = build_R(n, n_angles, n_bins, self.angles)
        if values == "f32":
            self.MR.v = self.MR.v.astype(np.float32).astype(np.float64)
        elif values != "f64":
            raise ValueError("values must be 'f64' or 'f32'")
        self.MRT = self.MR.transpose()
        self.rows = self.MR.rows
        self._s = _OraOp(n, self.rows, _p(self.MR.rp, _i64p), _p(self.MR.ci, _i32p),
                         _p(self.MR.v), _p(self.MRT.rp, _i64p), _p(self.MRT.ci, _i32p),
                         _p(self.MRT.v), -1, None)

    @property
    def nn(self) -> int:
        return self.n * self.n

    def fwd(self, x) -> np.ndarray:
        return self.MR.matvec(x)

    def adj(self, y) -> np.ndarray:
        return self.MRT.matvec(y)

    def normal(self, x, alpha: float, lam: float, sigma: float = 0.0) -> np.ndarray:
        x = _f64(x)
        out = np.empty(self.nn)
        lib().ora_normal(ctypes.byref(self._s), alpha, lam, sigma, _p(x), _p(out))
        return out

    def cg(self, alpha, lam, sigma, rhs=None, x0=None, r0=None, n_iter=10, rtol=0.0):
        """CG on A(alpha, lam, sigma).  Give rhs (r0 = rhs - A x0) or r0 directly.
        Returns (x, r, rho_hist, iterations, breakdown)."""
        x = np.zeros(self.nn) if x0 is None else _f64(x0).copy()
        if r0 is None:
            r = _f64(rhs).copy()
            if x0 is not None:
                r -= self.normal(x, alpha, lam, sigma)
        else:
            r = _f64(r0).copy()
        hist = np.zeros(n_iter + 1)
        bd = ctypes.c_int(0)
        it = lib().ora_cg(ctypes.byref(self._s), alpha, lam, sigma, _p(x), _p(r), n_iter, rtol,
                          _p(hist), ctypes.byref(bd))
        return x, r, hist, it, bd.value

    def sb(self, f, alpha, lam, n_outer, n_cg, tol=0.0, u0=None, state=None):
        """Split Bregman.  Returns (u, upd_b, upd_u, outer_iterations, state)."""
        f = _f64(f)
        assert f.shape == (self.rows,)
        u = np.zeros(self.nn) if u0 is None else _f64(u0).copy()
        resume = state is not None
        st = np.zeros(5 * self.nn) if state is None else _f64(state).copy()
        ub = np.zeros(max(n_outer, 1))
        uu = np.zeros(max(n_outer, 1))
        k = lib().ora_sb(ctypes.byref(self._s), alpha, lam, n_outer, n_cg, tol, _p(f), _p(u),
                         int(u0 is not None), _p(st), int(resume), _p(ub), _p(uu))
        return u, ub[:k], uu[:k], k, st

    def pd(self, f, alpha, tau, sigma, n_outer, n_cg, u0=None):
        """Chambolle-Pock TV with inexact resolvent solves (n_cg CG steps of
        eq:PD_resolve per outer step).  Returns u."""
        f = _f64(f)
        u = np.zeros(self.nn) if u0 is None else _f64(u0).copy()
        lib().ora_pd(ctypes.byref(self._s), float(alpha), float(tau), float(sigma), int(n_outer),
                     int(n_cg), _p(f), _p(u), int(u0 is not None))
        return u

    def loss1(self, mu, f):
        mu, f = _f64(mu), _f64(f)
        gm = np.empty(self.nn)
        gf = np.empty(self.rows)
        L = lib().ora_loss1(ctypes.byref(self._s), _p(mu), _p(f), _p(gm), _p(gf))
        return L, gm, gf

    def surrogate_weights(self, radius: int) -> np.ndarray:
        """Weights of the surrogate T of Section 3.2 (eq:def_sparse_surr) for
        truncation radius r: (2r+1) x (2r+1), w[dy + r, dx + r] = the symmetric
        part of the centre pixel's point-spread function at offset (dy, dx)
        inside the disc |d| <= r, zero outside."""
        k = 2 * radius + 1
        w = np.zeros(k * k)
        if lib().ora_surrogate_weights(ctypes.byref(self._s), int(radius), _p(w)) != 0:
            raise ValueError("the disc of radius %d does not fit in the image" % radius)
        return w.reshape(k, k)

    def with_surrogate(self, radius: int) -> "OracleOp":
        """A copy whose normal operator uses T in place of R^T M^T M R (the
        data right-hand side of split Bregman keeps the exact (MR)^T), as in
        eq:surr_SBupd."""
        import copy
        o = copy.copy(self)
        o.sur_w = np.ascontiguousarray(self.surrogate_weights(radius).reshape(-1))
        o._s = _OraOp(self.n, self.rows, _p(self.MR.rp, _i64p), _p(self.MR.ci, _i32p),
                      _p(self.MR.v), _p(self.MRT.rp, _i64p), _p(self.MRT.ci, _i32p),
                      _p(self.MRT.v), int(radius), _p(o.sur_w))
        return o

    def stencil(self, radius: int, w, x) -> np.ndarray:
        """(T x) for weights w of radius r (plain loops)."""
        x = _f64(x)
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
        out = np.empty(self.nn)
        lib().ora_stencil(self.n, int(radius), _p(w), _p(x), _p(out))
        return out

    def loss2(self, mu, f, tau_alpha: float, n_iter: int):
        """Loss through n_iter unrolled CG steps; returns (L, g_mu, g_f, u_n)."""
        mu, f = _f64(mu), _f64(f)
        gm = np.empty(self.nn)
        gf = np.empty(self.rows)
        un = np.empty(self.nn)
        L = lib().ora_loss2(ctypes.byref(self._s), tau_alpha, n_iter, _p(mu), _p(f), _p(gm),
                            _p(gf), _p(un))
        return L, gm, gf, un
