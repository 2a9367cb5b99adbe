"""Fourier-domain operator (Sections 2 and 3.1: eq:four_obj, eq:SBFFT,
eq:fusedop) on the GPU against the oracle.

* the point set, grid and tau agree with the oracle's;
* the gridded transforms F^* and F match the oracle's (on the tables the kind
  stores) for several sizes, ragged image sides (n not a power of two, odd n,
  grid above 2n), an even bin count and half-window widths;
* the normal operator through the fused B B^* and through the two transforms
  matches the oracle's, with the K^T K and sigma terms and <x, out>;
* split Bregman on eq:SBFFT matches the oracle's split Bregman; a batch of
  images and a resumed run equal single and uninterrupted runs bitwise;
* at 512 x 512 (180 of 360 angles, 725 bins): sampled outputs of F^* and F
  against the dense definition within the gridding accuracy, the adjoint
  identity, and the fused and unfused normal operators agreeing;
* argument errors.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import host, need_gpu, rel_l2, rounded, say, to_dev, torch
from oracle import fourier as F

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

MODES = {"f64": (torch.float64, torch.float64), "mixed": (torch.float32, torch.float64),
         "f32": (torch.float32, torch.float32)}
# FP64 arithmetic reaches the oracle to rounding (FFT and summation orders);
# the FP32 kind carries FP32 grids and transforms
TOL = {"f64": 1e-11, "mixed": 1e-9, "f32": 2e-4}

CASES = [(8, 7, 13, 1), (16, 12, 23, 1), (24, 20, 35, 1), (32, 25, 47, 2), (33, 19, 48, 1)]


def setup(case, mode, m_sp):
    n, na, nb, ev = case
    mat, vec = MODES[mode]
    mask = W.angle_mask(na, ev)
    op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec)
    fo = sct.RadonFourier(op, m_sp)
    g = F.Gridding(n, F.points(na, nb, mask), m_sp, values="f64" if mode == "f64" else "f32")
    return op, fo, g


def cplx(t):
    a = host(t)
    return a[..., 0] + 1j * a[..., 1]


def as_pairs(z, dtype):
    return to_dev(np.stack([z.real, z.imag], axis=-1), dtype)


@pytest.mark.parametrize("mode", ["f64", "mixed", "f32"])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("m_sp", [2, 6])
def test_transforms_match_oracle(mode, case, m_sp):
    need_gpu()
    op, fo, g = setup(case, mode, m_sp)
    assert fo.P == len(g.xi) and fo.grid == g.M and fo.tau == g.tau
    dt = MODES[mode][1]
    rng = np.random.default_rng(case[0] + m_sp)
    mu = rounded(rng.standard_normal((2, op.nn)), dt)
    fh = rounded(rng.standard_normal((2, fo.P, 2)), dt)
    got = cplx(fo.fwd(to_dev(mu, dt)))
    fz = fh[..., 0] + 1j * fh[..., 1]
    x = host(fo.adj(to_dev(fh, dt), alpha=0.7))
    for b in range(2):
        want = g.nufft_fwd(mu[b])
        assert np.linalg.norm(got[b] - want) <= TOL[mode] * np.linalg.norm(want)
        wa = 0.7 * g.nufft_adj(fz[b]).real
        assert rel_l2(x[b], wa) <= TOL[mode]


@pytest.mark.parametrize("mode", ["f64", "mixed", "f32"])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("path", ["fused", "nufft"])
def test_normal_operator_matches_oracle(mode, case, path):
    need_gpu()
    op, fo, g = setup(case, mode, 6)
    dt = MODES[mode][1]
    rng = np.random.default_rng(11)
    x = rounded(rng.standard_normal((2, op.nn)), dt)
    BB = g.fused_matrix()
    n = case[0]
    for alpha, lam, sigma in ((1.0, 0.0, 0.0), (0.05, 1.0, 0.0), (2.0, 0.5, 0.25)):
        out, dot = fo.normal(to_dev(x, dt), alpha, lam, sigma, path=path, dot=True)
        out, dot = host(out), host(dot)
        for b in range(2):
            if path == "fused":
                H = lambda v: g.fused_normal(v, BB)
            else:
                H = lambda v: g.nufft_adj(g.nufft_fwd(v)).real
            want = F.normal(H, n, x[b], alpha, lam, sigma)
            assert rel_l2(out[b], want) <= TOL[mode], (alpha, lam, sigma)
            assert abs(dot[b] - x[b] @ want) <= 10 * TOL[mode] * np.abs(x[b]).dot(np.abs(want))


@pytest.mark.parametrize("mode", ["f64", "mixed"])
@pytest.mark.parametrize("case", [(16, 12, 23, 1), (32, 25, 47, 2)])
def test_wide_window_m_sp_12(mode, case):
    """M_sp = 12 (about 12 digits): 47 x 48 stencil coefficients per grid
    point, wider than the 32-point grid at n = 16 (the stencil wraps), and
    the two-image stencil's LDS above 64 KB."""
    need_gpu()
    op, fo, g = setup(case, mode, 12)
    dt = MODES[mode][1]
    rng = np.random.default_rng(12)
    x = rounded(rng.standard_normal((3, op.nn)), dt)
    BB = g.fused_matrix()
    for path, H in (("fused", lambda v: g.fused_normal(v, BB)),
                    ("nufft", lambda v: g.nufft_adj(g.nufft_fwd(v)).real)):
        out = host(fo.normal(to_dev(x, dt), 1.5, 0.5, 0.0, path=path))
        for b in range(3):
            assert rel_l2(out[b], F.normal(H, case[0], x[b], 1.5, 0.5)) <= TOL[mode], (path, b)


@pytest.mark.parametrize("mode,tol", [("f64", 1e-9), ("mixed", 1e-8), ("f32", 5e-2)])
@pytest.mark.parametrize("path", ["fused", "nufft"])
def test_split_bregman_matches_oracle(mode, tol, path):
    need_gpu()
    case = (32, 25, 47, 1)
    op, fo, g = setup(case, mode, 6)
    n = case[0]
    dt = MODES[mode][1]
    mu = W.phantom(n, 5, seed=3)
    rng = np.random.default_rng(3)
    fz = g.nufft_fwd(mu)
    fz = fz + 0.01 * np.sqrt(np.mean(np.abs(fz) ** 2)) * (rng.standard_normal(len(fz))
                                                          + 1j * rng.standard_normal(len(fz)))
    fh = rounded(np.stack([fz.real, fz.imag], axis=-1), dt)
    fz = fh[..., 0] + 1j * fh[..., 1]
    alpha, lam = 0.02, 1.0
    say(f"Fourier split Bregman {mode} {path}")
    u, info = fo.sb(to_dev(fh[None], dt), alpha, lam, 20, 10, path=path)
    BB = g.fused_matrix()
    H = (lambda v: g.fused_normal(v, BB)) if path == "fused" else \
        (lambda v: g.nufft_adj(g.nufft_fwd(v)).real)
    uo, upd = F.sb(H, n, alpha * g.nufft_adj(fz).real, alpha, lam, 20, 10)
    assert rel_l2(host(u), uo) <= tol
    inf = sct.decode_sb_info(info)[0]
    assert inf["outer"] == 20 and inf["breakdowns"] == 0
    if mode != "f32":
        assert inf["upd_b"] == pytest.approx(upd[-1], rel=1e-6)


def test_batch_and_resume_are_bitwise():
    """Three images in one call equal three single calls, and 10 + resumed 10
    Bregman steps equal 20, bitwise (per-image arithmetic and state)."""
    need_gpu()
    case = (24, 20, 35, 1)
    op, fo, g = setup(case, "mixed", 6)
    rng = np.random.default_rng(8)
    fh = to_dev(rng.standard_normal((3, fo.P, 2)), torch.float64)
    for path in ("fused", "nufft"):
        U, _ = fo.sb(fh, 0.05, 1.0, 6, 8, path=path)
        for b in range(3):
            u, _ = fo.sb(fh[b:b + 1].contiguous(), 0.05, 1.0, 6, 8, path=path)
            assert torch.equal(u[0], U[b])
        u20, _ = fo.sb(fh[:1].contiguous(), 0.05, 1.0, 20, 8, path=path)
        u10, _ = fo.sb(fh[:1].contiguous(), 0.05, 1.0, 10, 8, path=path)
        u10b, _ = fo.sb(fh[:1].contiguous(), 0.05, 1.0, 10, 8, path=path, resume=True, out=u10)
        assert torch.equal(u10b, u20)


def test_full_size_sampled_against_the_definition():
    """512 x 512, 180 of 360 angles, 725 bins, mixed kind, m_sp = 6."""
    need_gpu()
    n, na, nb = 512, 360, 725
    mask = W.angle_mask(na, 2)
    op = sct.RadonOp(n, na, nb, mask, dtype=torch.float32, vec_dtype=torch.float64)
    say("building the 512 x 512 Fourier operator")
    fo = sct.RadonFourier(op, 6)
    xi = F.points(na, nb, mask)
    assert fo.P == len(xi) and fo.grid == 1024
    rng = np.random.default_rng(21)
    mu = W.phantom(n, 10, seed=0)
    MU = to_dev(mu[None], torch.float64)
    fh = cplx(fo.fwd(MU))[0]
    m = F.modes(n)
    my, mx = np.meshgrid(m, m, indexing="ij")
    img = mu.reshape(n, n)
    l1 = np.abs(mu).sum()
    for p in rng.choice(fo.P, 48, replace=False):
        want = (img * np.exp(-1j * (xi[p, 0] * mx + xi[p, 1] * my))).sum()
        assert abs(fh[p] - want) <= 2e-6 * l1, p
    # F at sampled pixels from random samples
    z = rng.standard_normal(fo.P) + 1j * rng.standard_normal(fo.P)
    x = host(fo.adj(as_pairs(z[None], torch.float64)))[0]
    for j in rng.choice(op.nn, 16, replace=False):
        iy, ix = divmod(int(j), n)
        want = (z * np.exp(1j * (xi[:, 0] * m[ix] + xi[:, 1] * m[iy]))).sum().real
        assert abs(x[j] - want) <= 2e-6 * np.abs(z).sum(), j
    # <F^* mu, z> = <mu, F z> (the same stored weights on both sides)
    lhs = np.vdot(fh, z).real
    assert abs(lhs - mu @ x) <= 1e-10 * np.linalg.norm(fh) * np.linalg.norm(z)
    # fused and unfused H, and symmetry
    X = to_dev(rng.standard_normal((2, op.nn)), torch.float64)
    a = host(fo.normal(X, 1.0, path="fused"))
    b = host(fo.normal(X, 1.0, path="nufft"))
    assert rel_l2(a, b) <= 1e-6
    xh = host(X)
    assert abs(xh[0] @ a[1] - xh[1] @ a[0]) <= 1e-9 * np.linalg.norm(a[0]) * np.linalg.norm(xh[1])


def test_errors():
    need_gpu()
    op = sct.RadonOp(16, 12, 23, dtype=torch.float64)
    with pytest.raises(sct.SparsectError, match="m_sp"):
        sct.RadonFourier(op, 0)
    with pytest.raises(sct.SparsectError, match="m_sp"):
        sct.RadonFourier(op, 13)
    with pytest.raises(sct.SparsectError, match="power of two"):
        sct.RadonFourier(op, 6, grid=48)
    with pytest.raises(sct.SparsectError, match="power of two"):
        sct.RadonFourier(op, 6, grid=16)
    with pytest.raises(sct.SparsectError, match="tau"):
        sct.RadonFourier(op, 6, tau=20.0)
    fo = sct.RadonFourier(op, 2)
    L = sct.lib()
    x = torch.zeros((1, op.nn), dtype=torch.float64, device="cuda")
    assert L.fourier_normal(fo._h, 5, 1.0, 0.0, 0.0, sct._vp(x.data_ptr()), sct._vp(x.data_ptr() + 8),
                            None, 1, None, 0, None) == -1
    assert "path" in L.radon_last_error().decode()
    with pytest.raises(sct.SparsectError, match="2 P"):
        fo.adj(torch.zeros(3, dtype=torch.float64, device="cuda"))
