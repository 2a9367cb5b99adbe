"""Full-size parity of the two largest workloads with the FP64 oracle.

* 2048 x 2048, 90 angles (every one measured), 2897 bins, 30 ellipses, 1%
  noise: the under-resolved case whose inner solves are truncated (Section
  3.2 relies on the outer Bregman iteration forgetting the inner error).  The
  normal operator is compared element by element, then the whole split
  Bregman 30 x 10 in the launch configuration the benchmark times (FP32
  matrix, FP64 vectors, line-banded forward).
* 64 slices of 1024 x 1024, 360 angles, 1449 bins sharing one operator: the
  fused multi-image normal operator (every matrix load shared by a chunk of
  images, line-banded forward with per-image band partials) over all 64
  slices, with three slices (first, middle, last chunk) compared element by
  element against the oracle's per-slice products; for the default chunking
  (4 images per forward chunk, 8 per adjoint chunk), for 16-image chunks,
  and for the compact forward layout of 32 rays over 2 angles gathering from
  pixel-major chunk copies.
* Both large workloads also run with the compact forward layout (one stored
  length per ray and line, the second derived from the ray's chord).

The oracle is the plain FP64 one (exact Siddon entries), so the tolerance
1e-5 covers the single rounding of the GPU's FP32 matrix entries as well as
the summation order.  Each test builds an oracle of ~4.9e8 nonzeros (about
12 GB of host memory and a minute of host time) and needs a GPU.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

F64 = torch.float64


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_large_2048_normal_and_split_bregman_30x10():
    w = W.WORKLOADS["large_2048_f32"]
    say("large_2048: oracle build (FP64 entries)")
    ref = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    mu, eps = W.phantom_and_noise(w.n, w.n_ellipses, ref.rows, seed=0)
    y = ref.fwd(mu)
    f = y + w.noise * np.sqrt(np.mean(y ** 2)) * eps
    say("large_2048: gpu build")
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=F64)
    assert op.info.nnz == ref.MR.nnz
    say("large_2048: normal operator")
    want = ref.normal(mu, w.alpha, w.lam)
    got = host(op.normal(to_dev(mu[None], F64), w.alpha, w.lam))[0]
    err_n = rel_l2(got, want)
    say(f"large_2048: normal operator rel L2 = {err_n:.3e}")
    assert err_n <= 1e-5
    # and with the compact forward layout, 64 rays over 2 angles
    opc = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=F64,
                      tuning="default", bundle=64, bundle_angles=2, compact=True)
    got_c = host(opc.normal(to_dev(mu[None], F64), w.alpha, w.lam))[0]
    err_nc = rel_l2(got_c, want)
    say(f"large_2048: normal operator, compact layout, rel L2 = {err_nc:.3e}")
    assert err_nc <= 1e-5
    # stored by symmetry too (the 90 measured angles are closed under the maps)
    ops = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=F64,
                      tuning="default", bundle=64, bundle_angles=2, compact=True, symmetric=True)
    err_ns = rel_l2(host(ops.normal(to_dev(mu[None], F64), w.alpha, w.lam))[0], want)
    say(f"large_2048: normal operator, compact and symmetric, rel L2 = {err_ns:.3e}")
    assert err_ns <= 1e-5
    us = host(ops.sb(to_dev(f[None], F64), w.alpha, w.lam, w.n_outer, w.n_cg)[0])[0]
    del ops
    say("large_2048: split Bregman 30x10 on the GPU")
    u, info = op.sb(to_dev(f[None], F64), w.alpha, w.lam, w.n_outer, w.n_cg)
    uh = host(u)[0]
    assert sct.decode_sb_info(info)[0]["outer"] == w.n_outer
    uc, _ = opc.sb(to_dev(f[None], F64), w.alpha, w.lam, w.n_outer, w.n_cg)
    uch = host(uc)[0]
    del opc
    # the oracle runs the 30 outer iterations as three resumed runs of 10
    # (resuming is bitwise the same as one run), printing between them
    uo, st, done = None, None, 0
    while done < w.n_outer:
        k = min(10, w.n_outer - done)
        say(f"large_2048: split Bregman on the oracle, outer {done}..{done + k}")
        uo, _, _, _, st = ref.sb(f, w.alpha, w.lam, k, w.n_cg, u0=uo, state=st)
        done += k
    err = rel_l2(uh, uo)
    err_c = rel_l2(uch, uo)
    err_s = rel_l2(us, uo)
    say(f"large_2048: split Bregman rel L2 = {err:.3e}, compact layout {err_c:.3e}, "
        f"compact and symmetric {err_s:.3e}")
    assert err <= 1e-5
    assert err_c <= 1e-5
    assert err_s <= 1e-5


@pytest.mark.parametrize("chunks,bundle,vec", [(None, 16, "f64"), ((16, 16), 16, "f64"),
                                               ((16, 16), 64, "f32"), ((8, 8), 32, "f32"),
                                               ((16, 16), (32, 2, True), "f32")],
                         ids=["default_chunks", "chunks16", "f32_chunks16_bundle64",
                              "f32_chunks8_bundle32", "f32_chunks16_compact_32x2_pixel_major"])
def test_volume_64x1024_fused_normal_slices(chunks, bundle, vec):
    """FP64 vectors (the mixed kind) and FP32 vectors (the pure FP32 kind the
    benchmark's volume leg times); the FP32 kind's inputs are the phantoms
    rounded to FP32, which the oracle receives too."""
    w = W.WORKLOADS["volume_64x1024_f32"]
    vdt = F64 if vec == "f64" else torch.float32
    say(f"volume_64x1024 {chunks} {bundle} {vec}: oracle build (FP64 entries)")
    ref = _volume_oracle(w)
    say(f"volume_64x1024 {chunks} {bundle} {vec}: gpu build and {w.batch} phantoms")
    if isinstance(bundle, tuple):   # (rays, angles, compact), gathering from pixel-major chunks
        op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                         tuning="default", bundle=bundle[0], bundle_angles=bundle[1], compact=bundle[2])
        op.tuning = {"fwd_rhs": chunks[0], "adj_rhs": chunks[1], "fwd_layout": 1, "adj_layout": 1}
    else:
        op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                         tuning="default", bundle=bundle)
        if chunks is not None:
            op.tuning = {"fwd_rhs": chunks[0], "adj_rhs": chunks[1]}
    X = np.stack([W.phantom(w.n, w.n_ellipses, seed=0, index=i) for i in range(w.batch)])
    if vec == "f32":
        X = X.astype(np.float32).astype(np.float64)
    got = host(op.normal(to_dev(X, vdt), w.alpha, w.lam))
    for i in (0, 37, w.batch - 1):
        want = ref.normal(X[i], w.alpha, w.lam)
        err = rel_l2(got[i], want)
        say(f"volume_64x1024 {chunks} {bundle} {vec}: slice {i} rel L2 = {err:.3e}")
        assert err <= 1e-5, i


_VOLUME_ORACLE = {}


def _volume_oracle(w):
    """One oracle build serves both chunkings (module-level cache)."""
    if "op" not in _VOLUME_ORACLE:
        _VOLUME_ORACLE["op"] = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    return _VOLUME_ORACLE["op"]


def teardown_module(module):
    _VOLUME_ORACLE.clear()
