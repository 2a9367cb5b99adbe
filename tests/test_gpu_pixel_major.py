"""The fused forward from a pixel-major copy of each chunk (fwd_layout 1) and
the band height knob (fwd_lines).

* every operator kind, bundle width, chunk size (4, 8, 16), band height and
  ragged batch (a last chunk with fewer images) matches the FP64 oracle's
  forward and normal operator, image by image;
* it equals the per-image gather layout to rounding;
* the normal operator and CG through it agree with the oracle on a
  banded operator (1024 pixels) with rays on both gather classes.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, rounded, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
MODES = {"f64": (F64, F64), "f32": (F32, F32), "mixed": (F32, F64)}


@pytest.mark.parametrize("mode", ["mixed", "f32", "f64"])
@pytest.mark.parametrize("bw", [16, 32, 64])
def test_pixel_major_matches_oracle(mode, bw):
    need_gpu()
    n, na, ev, batch = 300, 24, 2, 11
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, ev)
    say(f"pixel-major forward {mode} bundle {bw} n={n} batch={batch}")
    ref = oracle.OracleOp(n, na, nb, mask)
    mat, vec = MODES[mode]
    tol = 1e-12 if mode == "f64" else 1e-5
    rng = np.random.default_rng(bw)
    x = rounded(rng.standard_normal((batch, n * n)), vec)
    want_y = [ref.fwd(x[b]) for b in range(batch)]
    want_a = [ref.normal(x[b], 0.7, 0.3, 0.05) for b in range(batch)]
    op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", bundle=bw)
    assert op.needs_transpose
    X = to_dev(x, vec)
    op.tuning = {"fwd_rhs": 16, "fwd_layout": 0, "fwd_lines": 0}
    y_img = op.fwd(X)
    for fr in (4, 8, 16):
        for lines in (0, 16, 128):
            op.tuning = {"fwd_rhs": fr, "adj_rhs": 4, "fwd_layout": 1, "fwd_lines": lines}
            y = op.fwd(X)
            a = host(op.normal(X, 0.7, 0.3, 0.05))
            assert rel_l2(host(y), host(y_img)) <= (1e-13 if vec == F64 else 1e-6), (fr, lines)
            yh = host(y)
            for b in range(batch):
                assert rel_l2(yh[b], want_y[b]) <= tol, (fr, lines, b)
                assert rel_l2(a[b], want_a[b]) <= tol, (fr, lines, b)


def test_pixel_major_banded_normal_and_cg():
    need_gpu()
    n, na = 1024, 8
    nb = W.n_bins_for(n)
    say(f"pixel-major banded n={n} angles={na}")
    ref = oracle.OracleOp(n, na, nb)
    op = sct.RadonOp(n, na, nb, None, dtype=F64, tuning="default")
    op.tuning = {"fwd_rhs": 4, "adj_rhs": 4, "fwd_layout": 1, "fwd_lines": 32}
    rng = np.random.default_rng(12)
    x = rng.standard_normal((5, n * n))
    out = host(op.normal(to_dev(x, F64), 0.5, 1.0, 0.25))
    for b in (0, 4):
        assert rel_l2(out[b], ref.normal(x[b], 0.5, 1.0, 0.25)) <= 1e-12, b
    rhs = rng.standard_normal((5, n * n))
    xs, _ = op.cg(to_dev(rhs, F64), 0.5, 1.0, 0.0, n_iter=4)
    xo = ref.cg(0.5, 1.0, 0.0, rhs=rhs[3], n_iter=4)[0]
    assert rel_l2(host(xs)[3], xo) <= 1e-10


def test_band_height_knob_matches_default():
    """Every band height gives the forward of the default choice to
    rounding, for one image and for a fused chunk."""
    need_gpu()
    n, na = 512, 12
    op = sct.RadonOp(n, na, W.n_bins_for(n), None, dtype=F32, vec_dtype=F64, tuning="default")
    rng = np.random.default_rng(2)
    X = to_dev(rng.standard_normal((6, n * n)), F64)
    base = host(op.fwd(X))
    for lines in (16, 32, 64, 128):
        for fr in (1, 4):
            op.tuning = {"fwd_rhs": fr, "fwd_lines": lines}
            assert rel_l2(host(op.fwd(X)), base) <= 1e-13, (lines, fr)


@pytest.mark.parametrize("mode", ["mixed", "f32", "f64"])
def test_adjoint_pixel_major_equals_per_image_staging(mode):
    """adj_layout 1 stages a chunk's bands from a pixel-major copy of its
    sinograms; each image's sum runs in the same order as with per-image
    staging, so adjoint, normal operator (with <x, out>) and CG agree bitwise,
    and match the oracle."""
    need_gpu()
    n, na, batch = 90, 30, 11
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, 2)
    mat, vec = MODES[mode]
    say(f"pixel-major adjoint {mode} batch={batch}")
    ref = oracle.OracleOp(n, na, nb, mask)
    op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default")
    rng = np.random.default_rng(21)
    y = rounded(rng.standard_normal((batch, op.rows)), vec)
    x = rounded(rng.standard_normal((batch, op.nn)), vec)
    Y, X = to_dev(y, vec), to_dev(x, vec)
    tol = 1e-12 if mode == "f64" else 1e-5
    for ar in (4, 8, 16):
        op.tuning = {"adj_rhs": ar, "adj_layout": 0}
        a0 = op.adj(Y)
        n0, d0 = op.normal(X, 0.7, 0.3, 0.05, dot=True)
        c0, _ = op.cg(X, 0.7, 0.3, 0.05, n_iter=3)
        op.tuning = {"adj_rhs": ar, "adj_layout": 1}
        assert op.workspace(sct.WS_ADJ, batch)[1] > 0
        a1 = op.adj(Y)
        n1, d1 = op.normal(X, 0.7, 0.3, 0.05, dot=True)
        c1, _ = op.cg(X, 0.7, 0.3, 0.05, n_iter=3)
        assert torch.equal(a1, a0), ar
        assert torch.equal(n1, n0) and torch.equal(d1, d0), ar
        assert torch.equal(c1, c0), ar
        ah = host(a1)
        for b in (0, batch - 1):
            assert rel_l2(ah[b], ref.adj(y[b])) <= tol, (ar, b)
    # radon_adj without a workspace stages per image (the same result)
    L = sct.lib()
    out = torch.empty_like(X)
    rc = L.radon_adj(op._h, sct._vp(Y.data_ptr()), sct._vp(out.data_ptr()), batch, 0, None, 0, op._stream())
    assert rc == 0, L.radon_last_error()
    assert torch.equal(out, a1)
