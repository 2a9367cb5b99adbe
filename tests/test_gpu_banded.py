"""The line-banded forward product (images from 1024 pixels on).

* radon_fwd (banded, with a workspace) equals radon_fwd_xt (bundle order) to
  rounding, for image sides that are and are not multiples of the 128-line
  band, with subsampled angles, for one image and for fused chunks of 4 and
  16 images;
* the normal operator and a CG solve through it match the oracle on an
  operator small enough for the oracle (few angles);
* in a group, a banded instance's products equal the single operator's
  bitwise (same items, same partial order).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,na,ev", [(1024, 24, 1), (1100, 30, 3), (1030, 7, 1)])
@pytest.mark.parametrize("batch", [1, 4, 16])
def test_banded_equals_bundle_order(n, na, ev, batch):
    need_gpu()
    say(f"banded forward n={n} angles={na} every={ev} batch={batch}")
    op = sct.RadonOp(n, na, W.n_bins_for(n), W.angle_mask(na, ev), dtype=torch.float32,
                     vec_dtype=torch.float64)
    op.tuning = {"fwd_rhs": 16}
    rng = np.random.default_rng(n + batch)
    X = to_dev(rng.standard_normal((batch, op.nn)), torch.float64)
    XT = X.reshape(batch, n, n).transpose(1, 2).contiguous().reshape(batch, -1)
    yb = host(op.fwd(X))
    yo = host(op.fwd_xt(X, XT))
    for b in range(batch):
        assert rel_l2(yb[b], yo[b]) <= 1e-13, b


def test_banded_normal_and_cg_match_oracle():
    need_gpu()
    n, na, nb = 1024, 6, W.n_bins_for(1024)
    op = sct.RadonOp(n, na, nb, None, dtype=torch.float64)
    ref = oracle.OracleOp(n, na, nb)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(n * n)
    out = host(op.normal(to_dev(x[None], torch.float64), 0.5, 1.0, 0.25))[0]
    assert rel_l2(out, ref.normal(x, 0.5, 1.0, 0.25)) <= 1e-12
    rhs = rng.standard_normal(n * n)
    xs, _ = op.cg(to_dev(rhs[None], torch.float64), 0.5, 1.0, 0.0, n_iter=5)
    xo = ref.cg(0.5, 1.0, 0.0, rhs=rhs, n_iter=5)[0]
    assert rel_l2(host(xs)[0], xo) <= 1e-10


def test_group_with_banded_instance_equals_single():
    need_gpu()
    specs = [(1024, 8, W.n_bins_for(1024)), (64, 45, 91), (1100, 5, W.n_bins_for(1100))]
    ops = [sct.RadonOp(n, na, nb, dtype=torch.float32, vec_dtype=torch.float64, tuning="default")
           for n, na, nb in specs]
    g = sct.RadonMulti(ops, 1.0, 0.5, 0.0)
    for o in ops:
        o.tuning = {"fwd_waves": g.fwd_waves, "adj_waves": g.adj_waves}
    rng = np.random.default_rng(6)
    xs = [to_dev(rng.standard_normal(o.nn), torch.float64) for o in ops]
    X = g.pack_images(xs)
    F, A = g.apply(0, X), g.apply(2, X)
    for i, o in enumerate(ops):
        assert torch.equal(g.sinogram(F, i), o.fwd(xs[i][None])[0]), i
        assert torch.equal(g.image(A, i), o.normal(xs[i][None], 1.0, 0.5, 0.0)[0]), i


@pytest.mark.parametrize("n,na,ev,batch,rhs,vec", [
    (512, 12, 1, 6, 4, "f64"),     # 4-image chunks of 512^2 FP64 overflow the band budget: 128-line bands
    (600, 10, 2, 19, 16, "f64"),   # ragged side and chunk tail: 16-line bands
    (1024, 8, 1, 10, 8, "f32"),    # FP32, 8-image chunks: 64-line bands
    (300, 9, 1, 5, 4, "f32"),      # 4 x 300^2 FP32 fits the budget whole: no bands
])
def test_fused_chunks_band_to_their_chunk(n, na, ev, batch, rhs, vec):
    """Fused multi-image products: the forward runs its chunks one after
    another, each line-banded to the height the chunk's images fit (or not at
    all when they fit whole), and the adjoint visits tiles in the XCD-compact
    order.  Every image matches the oracle and its own single-image product."""
    need_gpu()
    say(f"fused chunks n={n} angles={na} batch={batch} rhs={rhs} {vec}")
    vdt = torch.float64 if vec == "f64" else torch.float32
    mat = torch.float64 if vec == "f64" else torch.float32
    mask = W.angle_mask(na, ev)
    nb = W.n_bins_for(n)
    op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vdt, tuning="default")
    op.tuning = {"fwd_rhs": rhs, "adj_rhs": rhs}
    ref = oracle.OracleOp(n, na, nb, mask)
    rng = np.random.default_rng(n + batch)
    X = rng.standard_normal((batch, n * n))
    if vec == "f32":
        X = X.astype(np.float32).astype(np.float64)
    Xd = to_dev(X, vdt)
    y = host(op.fwd(Xd))
    o = host(op.normal(Xd, 0.5, 1.0, 0.25))
    tol = 1e-12 if vec == "f64" else 1e-5
    for b in (0, batch // 2, batch - 1):
        assert rel_l2(y[b], ref.fwd(X[b])) <= tol, b
        assert rel_l2(o[b], ref.normal(X[b], 0.5, 1.0, 0.25)) <= tol, b
    op.tuning = {"fwd_rhs": 1, "adj_rhs": 1}
    y1 = host(op.fwd(Xd))
    o1 = host(op.normal(Xd, 0.5, 1.0, 0.25))
    assert np.max(np.abs(y - y1)) <= (1e-12 if vec == "f64" else 1e-4) * np.max(np.abs(y1))
    assert np.max(np.abs(o - o1)) <= (1e-12 if vec == "f64" else 1e-4) * np.max(np.abs(o1))
