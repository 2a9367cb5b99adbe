"""Pixel-major vectors at the C ABI (RADON_LAYOUT_PIXEL: element i of image b
at i*batch + b).

Every call that takes a layout computes exactly what the image-major call
computes (the inputs and outputs are relaid, the products are the same), so
the results are compared bitwise with the image-major results, and one of
them with the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
PIX = sct.LAYOUT_PIXEL


def pm(t):
    """[b, count] -> pixel-major [count, b]."""
    return t.t().contiguous()


@pytest.mark.parametrize("mode,batch", [("mixed", 5), ("f32", 3), ("mixed", 1), ("f64", 37)])
def test_pixel_layout_products_equal_image_layout(mode, batch):
    need_gpu()
    n, na = 70, 36
    mat, vec = {"mixed": (F32, F64), "f32": (F32, F32), "f64": (F64, F64)}[mode]
    say(f"pixel layout products {mode} batch={batch}")
    op = sct.RadonOp(n, na, W.n_bins_for(n), W.angle_mask(na, 2), dtype=mat, vec_dtype=vec)
    rng = np.random.default_rng(batch)
    X = to_dev(rng.standard_normal((batch, op.nn)), vec)
    Y = to_dev(rng.standard_normal((batch, op.rows)), vec)
    assert torch.equal(op.fwd(pm(X), layout=PIX), pm(op.fwd(X)))
    assert torch.equal(op.adj(pm(Y), layout=PIX), pm(op.adj(Y)))
    a0, d0 = op.normal(X, 0.7, 0.3, 0.05, dot=True)
    a1, d1 = op.normal(pm(X), 0.7, 0.3, 0.05, dot=True, layout=PIX)
    assert torch.equal(a1, pm(a0)) and torch.equal(d1, d0)
    x0, i0 = op.cg(X, 0.7, 0.3, 0.05, n_iter=6)
    x1, i1 = op.cg(pm(X), 0.7, 0.3, 0.05, n_iter=6, layout=PIX)
    assert torch.equal(x1, pm(x0)) and torch.equal(i1, i0)
    X0 = X * 0.5 + 0.25
    x0, _ = op.cg(X, 0.7, 0.3, 0.05, x0=X0, n_iter=4)
    x1, _ = op.cg(pm(X), 0.7, 0.3, 0.05, x0=pm(X0), n_iter=4, layout=PIX)
    assert torch.equal(x1, pm(x0))


def test_pixel_layout_split_bregman_and_resume_match_oracle():
    need_gpu()
    w = W.WORKLOADS["small_64_f64"]
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64)
    ref = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    rng = np.random.default_rng(8)
    F = rng.standard_normal((4, op.rows))
    Fd = to_dev(F, F64)
    u0, i0 = op.sb(Fd, w.alpha, w.lam, 3, 5, ws_key="img")
    u1, i1 = op.sb(pm(Fd), w.alpha, w.lam, 3, 5, ws_key="pix", layout=PIX)
    assert torch.equal(u1, pm(u0)) and torch.equal(i1, i0)
    u0, _ = op.sb(Fd, w.alpha, w.lam, 2, 5, resume=True, out=u0, ws_key="img")
    u1, _ = op.sb(pm(Fd), w.alpha, w.lam, 2, 5, resume=True, out=u1, ws_key="pix", layout=PIX)
    assert torch.equal(u1, pm(u0))
    # a warm start given pixel-major
    u0, _ = op.sb(Fd, w.alpha, w.lam, 2, 5, mu0=u0, ws_key="img")
    u1, _ = op.sb(pm(Fd), w.alpha, w.lam, 2, 5, mu0=u1, ws_key="pix", layout=PIX)
    assert torch.equal(u1, pm(u0))
    want = ref.sb(F[2], w.alpha, w.lam, 5, 5)[0]
    got, _ = op.sb(pm(Fd), w.alpha, w.lam, 5, 5, ws_key="pix2", layout=PIX)
    assert rel_l2(host(got)[:, 2], want) <= 1e-5


def test_pixel_layout_argument_and_workspace_errors():
    need_gpu()
    op = sct.RadonOp(16, 8, W.n_bins_for(16), dtype=F32)
    L = sct.lib()
    b = 3
    x = torch.zeros((op.nn, b), dtype=F32, device="cuda")
    out = torch.zeros_like(x)
    ws, nbytes = op.workspace(sct.WS_NORMAL, b)          # the image-major size
    need = L.radon_workspace_bytes(op._h, sct.WS_NORMAL | sct.WS_PIXEL_LAYOUT, b)
    assert need > nbytes
    rc = L.normal_apply(op._h, 1.0, 1.0, 0.0, sct._vp(x.data_ptr()), sct._vp(out.data_ptr()), None, b,
                        PIX, sct._vp(ws.data_ptr()), nbytes, None)
    assert rc == -4 and "workspace" in L.radon_last_error().decode()
    rc = L.normal_apply(op._h, 1.0, 1.0, 0.0, sct._vp(x.data_ptr()), sct._vp(out.data_ptr()), None, b,
                        2, sct._vp(ws.data_ptr()), nbytes, None)
    assert rc == -1 and "layout" in L.radon_last_error().decode()
    assert L.radon_workspace_bytes(op._h, sct.WS_PD | sct.WS_PIXEL_LAYOUT, b) == -1
    # one image: both layouts are the same and need no relay
    assert L.radon_workspace_bytes(op._h, sct.WS_ADJ | sct.WS_PIXEL_LAYOUT, 1) == 0
    with pytest.raises(sct.SparsectError):
        op.fwd(x, layout=2)
