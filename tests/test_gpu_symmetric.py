"""The forward layout stored by the symmetries of the square (fwd_symmetric):
bundles only for the measured angles in [0, pi/4], each ray also serving the
rays of pi - theta, pi/2 - theta and pi/2 + theta with the same bin (their
images under x -> -x, the transpose and both).

Those rays meet the mirrored pixels with the same lengths in exact
arithmetic, so the forward matches the FP64 oracle (which traces every ray
itself) at the bar of its kind and the stored layout to rounding, for angle
sets that are closed under the maps (every angle, every second angle, the
axis-aligned and 45-degree angles whose images coincide), with both lengths
stored or compact, one or two angles per bundle, and several images per
call.  Angle sets that are not closed are refused by the build (host checks
in test_abi.py); a group does not take such an operator.

With n a multiple of 8 the adjoint layout is stored the same way (pixel
(px, py) meets the rays of the three partner angles as (n-1-px, py),
(py, px) and (py, n-1-px) meet those of the stored angle, and 8x8 tiles map
onto tiles): the adjoint, with one workgroup per tile or per tile orbit
(adj_layout 0 or 1) at each wave count, matches the oracle at the bar of
its kind and the full layout to rounding, and the exported per-(pixel, angle) records, read
through the maps, hold the full layout's bins exactly and its lengths to
rounding.  Otherwise the adjoint is the full layout's, bitwise.
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
@pytest.mark.parametrize("geom", [(70, 36, 2), (61, 44, 1), (33, 8, 1), (8, 4, 1), (64, 36, 2), (40, 20, 1),
                                  (24, 180, 2), (32, 256, 1)])   # the last: 17 quads of stored angles
def test_symmetric_matches_oracle_and_stored_layout(mode, geom):
    need_gpu()
    n, na, ev = geom
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, ev)
    say(f"symmetric {mode} n={n} angles={na} every {ev}")
    ref = oracle.OracleOp(n, na, nb, mask)
    mat, vec = MODES[mode]
    tol = 1e-12 if mode == "f64" else 1e-5
    rng = np.random.default_rng(n + 7 * na)
    x = rounded(rng.standard_normal((3, n * n)), vec)
    y = rounded(rng.standard_normal((3, ref.rows)), vec)
    X, Y = to_dev(x, vec), to_dev(y, vec)
    for bw, ang, compact in ((16, 1, False), (64, 2, False), (64, 2, True), (32, 2, True)):
        full = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", bundle=bw,
                           bundle_angles=ang)
        op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", bundle=bw,
                         bundle_angles=ang, compact=compact, symmetric=True)
        assert op.symmetric and op.compact == compact
        assert op.info.fwd_slots < full.info.fwd_slots
        assert op.adj_symmetric == (n % 8 == 0)
        if op.adj_symmetric:
            assert op.info.adj_slots <= full.info.adj_slots   # equal when both fit one quad
            for aw in (1, 2, 4):
                for al in (0, 1):   # one workgroup per tile, or per tile orbit
                    op.tuning = {"adj_waves": aw, "adj_layout": al}
                    xa = host(op.adj(Y))
                    assert rel_l2(xa, host(full.adj(Y))) <= (1e-13 if mode == "f64" else 5e-7), (bw, ang, aw, al)
                    for b in range(3):
                        assert rel_l2(xa[b], ref.adj(y[b])) <= tol, (bw, ang, aw, al, b)
                    a = host(op.normal(X, 0.7, 0.3, 0.05))
                    for b in range(3):
                        assert rel_l2(a[b], ref.normal(x[b], 0.7, 0.3, 0.05)) <= tol, (bw, ang, aw, al, b)
            op.tuning = {"adj_waves": 0, "adj_layout": 0}
        else:
            assert torch.equal(op.adj(Y), full.adj(Y))
        for waves in (2, 4):
            op.tuning = {"fwd_waves": waves}
            yy = host(op.fwd(X))
            bound = 1e-13 if mode == "f64" else 5e-7
            assert rel_l2(yy, host(full.fwd(X))) <= bound, (bw, ang, compact, waves)
            a = host(op.normal(X, 0.7, 0.3, 0.05))
            for b in range(3):
                assert rel_l2(yy[b], ref.fwd(x[b])) <= tol, (bw, ang, compact, waves, b)
                assert rel_l2(a[b], ref.normal(x[b], 0.7, 0.3, 0.05)) <= tol, (bw, ang, compact, waves, b)


def test_symmetric_cg_and_group_refusal():
    need_gpu()
    na = 44
    nb = W.n_bins_for(64)
    ref = oracle.OracleOp(64, na, nb)
    op = sct.RadonOp(64, na, nb, None, dtype=F64, tuning="default", bundle=64, bundle_angles=2,
                     compact=True, symmetric=True)
    rhs = np.random.default_rng(9).standard_normal((2, op.nn))
    xs, _ = op.cg(to_dev(rhs, F64), 0.5, 1.0, 0.1, n_iter=6)
    xo = ref.cg(0.5, 1.0, 0.1, rhs=rhs[1], n_iter=6)[0]
    assert rel_l2(host(xs)[1], xo) <= 1e-7
    with pytest.raises(sct.SparsectError, match="symmetry"):
        sct.RadonMulti([op])


@pytest.mark.parametrize("mode", ["mixed", "f64"])
def test_symmetric_adjoint_records(mode):
    """The adjoint records exported through the maps: bins equal the full
    layout's, lengths equal them to the rounding of the matrix type."""
    need_gpu()
    n, na = 48, 40
    nb = W.n_bins_for(n)
    mat, vec = MODES[mode]
    say(f"symmetric adjoint records {mode}")
    full = sct.RadonOp(n, na, nb, None, dtype=mat, vec_dtype=vec, tuning="default", bundle=32)
    op = sct.RadonOp(n, na, nb, None, dtype=mat, vec_dtype=vec, tuning="default", bundle=32, symmetric=True)
    assert op.adj_symmetric
    bf, v0f, v1f = full.export_adj()
    bs, v0s, v1s = op.export_adj()
    np.testing.assert_array_equal(bs, bf)
    bound = 1e-14 if mode == "f64" else 1e-6
    assert np.max(np.abs(v0s - v0f)) <= bound * max(1.0, np.max(np.abs(v0f)))
    assert np.max(np.abs(v1s - v1f)) <= bound * max(1.0, np.max(np.abs(v1f)))


def test_symmetric_adjoint_batched_normal_and_partials():
    """Several images per call through every entry that runs the adjoint:
    radon_normal with its FP64 <x, Ax> partials (CG's dot), and image
    batches of each size the multi-image paths chunk by."""
    need_gpu()
    n, na = 96, 60
    nb = W.n_bins_for(n)
    say("symmetric adjoint batched")
    ref = oracle.OracleOp(n, na, nb)
    op = sct.RadonOp(n, na, nb, None, dtype=F32, vec_dtype=F64, tuning="default", bundle=64, bundle_angles=2,
                     compact=True, symmetric=True)
    assert op.adj_symmetric
    rng = np.random.default_rng(5)
    for batch in (1, 5, 16):
        x = rng.standard_normal((batch, n * n))
        y = rng.standard_normal((batch, ref.rows))
        for rhs, al in ((1, 0), (4, 1), (16, 0), (16, 1)):
            op.tuning = {"adj_rhs": rhs, "fwd_rhs": rhs, "adj_layout": al}
            xa = host(op.adj(to_dev(y, F64)))
            a = host(op.normal(to_dev(x, F64), 0.5, 1.0, 0.1))
            for b in range(batch):
                assert rel_l2(xa[b], ref.adj(y[b])) <= 1e-5, (batch, rhs, b)
                assert rel_l2(a[b], ref.normal(x[b], 0.5, 1.0, 0.1)) <= 1e-5, (batch, rhs, b)
    # CG through the <x, Ax> partials of both adjoint kernels
    rhs = rng.standard_normal((3, n * n))
    xo = ref.cg(0.5, 1.0, 0.1, rhs=rhs[2], n_iter=4)[0]
    for al in (0, 1):
        op.tuning = {"adj_layout": al}
        xs, _ = op.cg(to_dev(rhs, F64), 0.5, 1.0, 0.1, n_iter=4)
        assert rel_l2(host(xs)[2], xo) <= 1e-5, al


def test_symmetric_adjoint_kernels_agree_and_autotune():
    """At 512^2 each map's quads fit one staging chunk, so the per-tile and
    the per-orbit kernels form the same sums in the same order: bitwise
    equal.  The autotuner keeps the per-tile kernel here (528 orbits, fewer
    than 4 per CU)."""
    need_gpu()
    w = W.WORKLOADS["gpu_512_f32"]
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64, tuning="default", bundle=32,
                     bundle_angles=2, symmetric=True)
    y = to_dev(np.random.default_rng(8).standard_normal((2, op.rows)), F64)
    op.tuning = {"adj_layout": 0}
    a0 = op.adj(y)
    op.tuning = {"adj_layout": 1}
    assert torch.equal(op.adj(y), a0)
    from paper_1705_07497_amd import autotune
    autotune.autotune(op, batch=1, save=False)
    assert op.tuning["adj_layout"] == 0
    assert rel_l2(host(op.adj(y)), host(a0)) <= 1e-13
