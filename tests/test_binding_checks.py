"""Host-side checks of the Python binding that need no GPU.

* Every wrapper rejects a caller's buffer whose image or sinogram count differs
  from the input batch before anything reaches the library (an undersized
  out= would otherwise be written past its end on the device).
* The autograd Functions return gradients in the shape of their inputs.

The operators here are stubs: a RadonOp whose handle is never built, on the
CPU device, so any call that got as far as the library would fail loudly.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1705_07497_amd as sct
from paper_1705_07497_amd import autograd as AG


def stub_op(n=4, rows=6, dtype=torch.float64):
    op = object.__new__(sct.RadonOp)
    op.n, op.nn, op.rows = n, n * n, rows
    op.dtype = dtype
    op.device = torch.device("cpu")
    op._ws = {}
    op._h = None
    return op


def imgs(b, op):
    return torch.zeros((b, op.nn), dtype=op.dtype)


def sinos(b, op):
    return torch.zeros((b, op.rows), dtype=op.dtype)


@pytest.mark.parametrize("call", [
    lambda op: op.fwd(imgs(2, op), out=sinos(1, op)),
    lambda op: op.fwd(imgs(1, op), out=sinos(2, op)),
    lambda op: op.fwd_xt(imgs(2, op), imgs(2, op), out=sinos(1, op)),
    lambda op: op.adj(sinos(2, op), out=imgs(1, op)),
    lambda op: op.normal(imgs(3, op), 1.0, 1.0, out=imgs(2, op)),
    lambda op: op.cg(imgs(2, op), 1.0, 1.0, out=imgs(1, op)),
    lambda op: op.cg(imgs(2, op), 1.0, 1.0, x0=imgs(1, op)),
    lambda op: op.cg(imgs(2, op), 1.0, 1.0, x0=imgs(2, op), out=imgs(1, op)),
    lambda op: op.sb(sinos(2, op), 1.0, 1.0, 1, 1, out=imgs(1, op)),
    lambda op: op.sb(sinos(2, op), 1.0, 1.0, 1, 1, mu0=imgs(3, op)),
    lambda op: op.sb(sinos(1, op), 1.0, 1.0, 1, 1, resume=True, out=imgs(2, op)),
    lambda op: op.pd(sinos(2, op), 1.0, 1, 1, out=imgs(1, op)),
    lambda op: op.pd(sinos(2, op), 1.0, 1, 1, mu0=imgs(1, op)),
])
def test_wrappers_reject_wrong_sized_buffers(call):
    op = stub_op()
    with pytest.raises(sct.SparsectError, match="holds"):
        call(op)


def test_wrong_dtype_and_layout_rejected():
    op = stub_op()
    with pytest.raises(sct.SparsectError):
        op.fwd(torch.zeros((1, op.nn), dtype=torch.float32))
    with pytest.raises(sct.SparsectError):
        op.fwd(torch.zeros((op.nn, 2), dtype=op.dtype).t())
    with pytest.raises(sct.SparsectError):
        op.adj(torch.zeros(op.rows + 1, dtype=op.dtype))


class DenseStub:
    """fwd/adj/normal by a dense matrix, in the binding's flat output shapes."""

    def __init__(self, n=3, rows=5, seed=0):
        g = torch.Generator().manual_seed(seed)
        self.n, self.nn, self.rows = n, n * n, rows
        self.A = torch.randn(rows, n * n, generator=g, dtype=torch.float64)

    def fwd(self, x):
        return x.reshape(-1, self.nn) @ self.A.t()

    def adj(self, y):
        return y.reshape(-1, self.rows) @ self.A

    def normal(self, x, alpha, lam, sigma):
        xf = x.reshape(-1, self.nn)
        return alpha * (xf @ self.A.t()) @ self.A + sigma * xf


def test_autograd_gradients_keep_the_input_shape():
    op = DenseStub()
    mu = torch.randn(2, op.n, op.n, dtype=torch.float64, requires_grad=True)
    f = torch.randn(2, op.rows, dtype=torch.float64)
    AG.loss_data(op, mu, f).sum().backward()
    assert mu.grad.shape == mu.shape
    want = ((mu.detach().reshape(2, -1) @ op.A.t() - f) @ op.A).reshape(mu.shape)
    assert torch.allclose(mu.grad, want)
    y = torch.randn(2, 1, op.rows, dtype=torch.float64, requires_grad=True)
    AG.RadonAdj.apply(op, y).sum().backward()
    assert y.grad.shape == y.shape
    x = torch.randn(2, op.n, op.n, dtype=torch.float64, requires_grad=True)
    AG.NormalOp.apply(op, x, 2.0, 0.0, 1.0).sum().backward()
    assert x.grad.shape == x.shape
    assert torch.autograd.gradcheck(lambda t: AG.NormalOp.apply(op, t, 2.0, 0.0, 1.0),
                                    (x.detach().clone().requires_grad_(True),))
    assert torch.autograd.gradcheck(lambda t: AG.RadonFwd.apply(op, t),
                                    (x.detach().clone().requires_grad_(True),))


@pytest.mark.parametrize("call", [
    lambda op: op.fwd(imgs(3, op), layout=sct.LAYOUT_PIXEL),
    lambda op: op.fwd(imgs(3, op).t().contiguous(), layout=sct.LAYOUT_IMAGE),
    lambda op: op.adj(sinos(3, op), layout=sct.LAYOUT_PIXEL),
    lambda op: op.normal(imgs(3, op), 1.0, 1.0, layout=sct.LAYOUT_PIXEL),
    lambda op: op.cg(imgs(3, op), 1.0, 1.0, layout=sct.LAYOUT_PIXEL),
    lambda op: op.sb(sinos(3, op), 1.0, 1.0, 1, 1, layout=sct.LAYOUT_PIXEL),
    lambda op: op.fwd(imgs(3, op), layout=2),
])
def test_layout_and_tensor_shape_must_agree(call):
    """A 2-D tensor of several vectors is [batch, count] image-major and
    [count, batch] pixel-major; a contradiction is refused before any launch."""
    op = stub_op()
    with pytest.raises(sct.SparsectError, match="shape|layout"):
        call(op)
