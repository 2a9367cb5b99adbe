"""The compact forward layout (fwd_compact): one stored length per (ray,
line), the second derived as the ray's chord minus the first on the lines it
crosses from side to side, stored per ray on its first and last lines.

In exact arithmetic the two lengths of a fully crossed line add up to the
chord, so the derived operator is the stored one; in floating point a derived
FP32 length differs from the stored (rounded once) one by about one rounding
relative to the chord.  So:

* the forward and the normal operator match the FP64 oracle at the bar of
  their kind (1e-12 for FP64, 1e-5 for the FP32 matrix kinds) for every
  bundle layout, gather path (per image, pixel-major chunks, line bands,
  groups) and geometry, including rays that run along the image boundary
  (their lines hold half the chord, which the build takes from the ray's own
  lengths);
* the forward differs from the stored layout's by at most about 1e-7
  relative for the FP32 matrix (rounding), 1e-13 for FP64;
* the adjoint is the stored layout's, bitwise, and the operator holds no
  second-length array.
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
LAYOUTS = [(16, 1), (64, 2), (32, 2), (64, 4)]


@pytest.mark.parametrize("mode", ["mixed", "f32", "f64"])
@pytest.mark.parametrize("geom", [(70, 36, 2), (61, 45, 1), (33, 7, 1), (8, 4, 1)])
def test_compact_matches_oracle_and_stored_layout(mode, geom):
    need_gpu()
    n, na, ev = geom
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, ev)
    say(f"compact {mode} n={n} angles={na} every {ev}")
    ref = oracle.OracleOp(n, na, nb, mask)
    mat, vec = MODES[mode]
    tol = 1e-12 if mode == "f64" else 1e-5
    rng = np.random.default_rng(n * na)
    x = rounded(rng.standard_normal((5, n * n)), vec)
    y = rounded(rng.standard_normal((5, ref.rows)), vec)
    X, Y = to_dev(x, vec), to_dev(y, vec)
    for bw, ang in LAYOUTS:
        if bw // ang < 16:
            continue
        full = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", bundle=bw,
                           bundle_angles=ang)
        op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", bundle=bw,
                         bundle_angles=ang, compact=True)
        assert op.compact and not full.compact
        assert op.info.nnz == full.info.nnz == ref.MR.nnz
        assert op.info.device_bytes < full.info.device_bytes
        assert torch.equal(op.adj(Y), full.adj(Y))
        for fr in (1, 4):
            op.tuning = {"fwd_rhs": fr, "adj_rhs": 4}
            full.tuning = {"fwd_rhs": fr, "adj_rhs": 4}
            yc = host(op.fwd(X))
            assert rel_l2(yc, host(full.fwd(X))) <= (1e-13 if mode == "f64" else 5e-7), (bw, ang, fr)
            a = host(op.normal(X, 0.7, 0.3, 0.05))
            for b in range(5):
                assert rel_l2(yc[b], ref.fwd(x[b])) <= tol, (bw, ang, fr, b)
                assert rel_l2(a[b], ref.normal(x[b], 0.7, 0.3, 0.05)) <= tol, (bw, ang, fr, b)
        # <R x, y> against <x, R^T y>: the derived entries keep the pair
        # adjoint to rounding
        rx = host(op.fwd(X[:1]))[0]
        rty = host(op.adj(Y[:1]))[0]
        lhs, rhs = float(rx @ y[0]), float(x[0] @ rty)
        scale = np.linalg.norm(rx) * np.linalg.norm(y[0])
        assert abs(lhs - rhs) <= {"f64": 1e-12, "mixed": 1e-6, "f32": 1e-5}[mode] * scale


@pytest.mark.parametrize("bw,ang", [(64, 2), (32, 2)])
def test_compact_pixel_major_chunks(bw, ang):
    need_gpu()
    n, na = 90, 30
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, 2)
    say(f"compact pixel-major {bw}x{ang}")
    ref = oracle.OracleOp(n, na, nb, mask)
    op = sct.RadonOp(n, na, nb, mask, dtype=F32, vec_dtype=F64, tuning="default", bundle=bw,
                     bundle_angles=ang, compact=True)
    x = np.random.default_rng(bw).standard_normal((11, n * n))
    X = to_dev(x, F64)
    for fr in (4, 8, 16):
        op.tuning = {"fwd_rhs": fr, "fwd_layout": 1}
        yy = host(op.fwd(X))
        for b in (0, 5, 10):
            assert rel_l2(yy[b], ref.fwd(x[b])) <= 1e-5, (fr, b)


def test_compact_banded_normal_cg_and_group():
    """Line-banded forward (1024 pixels, FP64: the derived lengths are exact
    to FP64 rounding), CG against the oracle, and a group mixing compact and
    stored-layout instances."""
    need_gpu()
    n, na = 1024, 10
    nb = W.n_bins_for(n)
    say(f"compact banded n={n}")
    ref = oracle.OracleOp(n, na, nb)
    op = sct.RadonOp(n, na, nb, None, dtype=F64, tuning="default", bundle=64, bundle_angles=2, compact=True)
    x = np.random.default_rng(4).standard_normal((3, n * n))
    for fr, lay in ((1, 0), (4, 1)):
        op.tuning = {"fwd_rhs": fr, "fwd_layout": lay}
        out = host(op.normal(to_dev(x, F64), 0.5, 1.0, 0.25))
        for b in (0, 2):
            assert rel_l2(out[b], ref.normal(x[b], 0.5, 1.0, 0.25)) <= 1e-12, (fr, b)
    xs, _ = op.cg(to_dev(x, F64), 0.5, 1.0, 0.0, n_iter=3)
    xo = ref.cg(0.5, 1.0, 0.0, rhs=x[1], n_iter=3)[0]
    assert rel_l2(host(xs)[1], xo) <= 1e-10
    specs = [(64, 12, True), (96, 20, False), (1024, 6, True)]
    ops = [sct.RadonOp(m, a, W.n_bins_for(m), None, dtype=F64, tuning="default", bundle=64, bundle_angles=2,
                       compact=c) for m, a, c in specs]
    g = sct.RadonMulti(ops, 1.0, 0.5, 0.0)
    xs = [to_dev(np.random.default_rng(i).standard_normal(o.nn), F64) for i, o in enumerate(ops)]
    A = g.apply(2, g.pack_images(xs))
    for i, o in enumerate(ops):
        r = oracle.OracleOp(o.n, o.n_angles, o.n_bins)
        assert rel_l2(host(g.image(A, i)), r.normal(host(xs[i]), 1.0, 0.5, 0.0)) <= 1e-12, i
