"""normal_apply_noalloc: the workspace-free normal operator, through the C ABI.

Its output must equal normal_apply's (same kernels, same summation order:
bitwise) on consecutive calls that share the library's fixed per-GPU scratch
array, the later call with a smaller input than the earlier one, for the
default layout and for both products stored by symmetry, and match the FP64
oracle; a size beyond the fixed array is refused before anything is
enqueued.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
_vp = sct._vp


def _abi_pair(op, x, alpha, lam, sigma):
    """(normal_apply with a workspace, normal_apply_noalloc) outputs and dots."""
    L = sct.lib()
    b = x.shape[0]
    o_ws = torch.empty_like(x)
    o_na = torch.full_like(x, float("nan"))
    d_ws = torch.empty(b, dtype=F64, device=x.device)
    d_na = torch.full((b,), float("nan"), dtype=F64, device=x.device)
    ws, nb = op.workspace(sct.WS_NORMAL, b)
    s = op._stream()
    rc = L.normal_apply(op._h, alpha, lam, sigma, _vp(x.data_ptr()), _vp(o_ws.data_ptr()),
                        _vp(d_ws.data_ptr()), b, 0, _vp(ws.data_ptr()), nb, s)
    assert rc == 0, L.radon_last_error()
    rc = L.normal_apply_noalloc(op._h, alpha, lam, sigma, _vp(x.data_ptr()), _vp(o_na.data_ptr()),
                                _vp(d_na.data_ptr()), b, s)
    assert rc == 0, L.radon_last_error()
    torch.cuda.synchronize()
    return o_ws, o_na, d_ws, d_na


def test_noalloc_equals_normal_apply_on_consecutive_calls():
    need_gpu()
    rng = np.random.default_rng(77)
    # call 1: the benchmark's operator (FP32 matrix, FP64 vectors), 3 images
    w = W.WORKLOADS["gpu_512_f32"]
    say("noalloc: 512^2 / 180 angles, batch 3")
    big = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64)
    x1 = to_dev(rng.standard_normal((3, big.nn)), F64)
    o_ws, o_na, d_ws, d_na = _abi_pair(big, x1, w.alpha, w.lam, 0.0)
    assert torch.equal(o_ws, o_na) and torch.equal(d_ws, d_na)
    # call 2: a smaller input on the same operator (one image)
    say("noalloc: 512^2, batch 1")
    o_ws, o_na, d_ws, d_na = _abi_pair(big, x1[1:2].contiguous(), 0.5, 2.0, 0.25)
    assert torch.equal(o_ws, o_na) and torch.equal(d_ws, d_na)
    # call 3: a smaller operator (FP64, odd size, every angle), checked against the oracle too
    say("noalloc: 45^2 / 30 angles FP64, batch 2")
    n, na = 45, 30
    nb = W.n_bins_for(n)
    small = sct.RadonOp(n, na, nb, None, dtype=F64)
    xs = rng.standard_normal((2, n * n))
    o_ws, o_na, d_ws, d_na = _abi_pair(small, to_dev(xs, F64), 1.5, 0.5, 0.1)
    assert torch.equal(o_ws, o_na) and torch.equal(d_ws, d_na)
    ref = oracle.OracleOp(n, na, nb)
    got = host(o_na)
    for b in range(2):
        want = ref.normal(xs[b], 1.5, 0.5, 0.1)
        assert rel_l2(got[b], want) <= 1e-12
        assert abs(float(host(d_na)[b]) - float(np.dot(xs[b], want))) <= 1e-10 * abs(np.dot(xs[b], want))
    # call 4: the benchmark's layout (32-ray bundles over 2 angles, both
    # products stored by symmetry) on the 512^2 operator, then on a 64^2
    # FP64 one against the oracle
    say("noalloc: 512^2 stored by symmetry, batch 2")
    sym = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64, tuning="default",
                      bundle=32, bundle_angles=2, symmetric=True)
    assert sym.adj_symmetric
    o_ws, o_na, d_ws, d_na = _abi_pair(sym, x1[:2].contiguous(), w.alpha, w.lam, 0.0)
    assert torch.equal(o_ws, o_na) and torch.equal(d_ws, d_na)
    say("noalloc: 64^2 / 44 angles FP64 stored by symmetry, batch 2")
    n, na = 64, 44
    nb = W.n_bins_for(n)
    sym = sct.RadonOp(n, na, nb, None, dtype=F64, tuning="default", bundle=32, bundle_angles=2, symmetric=True)
    xs = rng.standard_normal((2, n * n))
    o_ws, o_na, d_ws, d_na = _abi_pair(sym, to_dev(xs, F64), 1.5, 0.5, 0.1)
    assert torch.equal(o_ws, o_na) and torch.equal(d_ws, d_na)
    ref = oracle.OracleOp(n, na, nb)
    got = host(o_na)
    for b in range(2):
        assert rel_l2(got[b], ref.normal(xs[b], 1.5, 0.5, 0.1)) <= 1e-12


def test_noalloc_refuses_sizes_beyond_its_scratch():
    need_gpu()
    w = W.WORKLOADS["gpu_512_f32"]
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64)
    L = sct.lib()
    limit = 64 << 20
    b = 1
    while L.radon_workspace_bytes(op._h, sct.WS_NORMAL, b) <= limit:
        b += 1
    x = torch.zeros((b, op.nn), dtype=F64, device="cuda")
    o = torch.full_like(x, 7.0)
    rc = L.normal_apply_noalloc(op._h, 1.0, 1.0, 0.0, _vp(x.data_ptr()), _vp(o.data_ptr()), None, b,
                                op._stream())
    assert rc == -4 and "scratch" in L.radon_last_error().decode()
    torch.cuda.synchronize()
    assert bool((o == 7.0).all())   # nothing was enqueued
    # one image fewer fits and runs
    x1 = to_dev(np.random.default_rng(3).standard_normal((b - 1, op.nn)), F64)
    o_ws, o_na, _, _ = _abi_pair(op, x1, 1.0, 1.0, 0.0)
    assert torch.equal(o_ws, o_na)
