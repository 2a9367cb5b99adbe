"""split_bregman_tv captured as one HIP graph: every replay equals the eager
solve bitwise, three replays in a row with new data and unrelated GPU work
between them; a warm start cannot be resumed through a graph."""
import numpy as np
import pytest

import workloads as W
from gpu_common import need_gpu, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,vdt", [(torch.float64, torch.float64), (torch.float32, torch.float64),
                                       (torch.float32, torch.float32)])
def test_graph_replays_equal_eager(dtype, vdt):
    need_gpu()
    n, na, nb = 48, 36, W.n_bins_for(48)
    mask = W.angle_mask(na, 2)
    op = sct.RadonOp(n, na, nb, mask, dtype=dtype, vec_dtype=vdt)
    rng = np.random.default_rng(9)
    f0 = to_dev(rng.standard_normal((2, op.rows)), vdt)
    g = op.sb_graph(f0, 0.05, 1.0, 6, 5)
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):
        say(f"SB graph replay {rep}")
        f = to_dev(rng.standard_normal((2, op.rows)), vdt)
        g.f.copy_(f)
        g.launch()
        torch.cuda.synchronize()
        mu_g, info_g = g.mu.clone(), g.info.clone()
        scratch.add_(1.0)                                    # unrelated eager work
        op.normal(to_dev(rng.standard_normal((1, op.nn)), vdt), 1.0, 1.0)
        mu_e, info_e = op.sb(f, 0.05, 1.0, 6, 5)
        torch.cuda.synchronize()
        assert torch.equal(mu_g, mu_e)
        assert torch.equal(info_g, info_e)


def test_graph_rejects_resume():
    need_gpu()
    op = sct.RadonOp(16, 12, W.n_bins_for(16), dtype=torch.float64)
    L = sct.lib()
    f = torch.zeros((1, op.rows), dtype=torch.float64, device="cuda")
    mu = torch.zeros((1, op.nn), dtype=torch.float64, device="cuda")
    nbytes = L.radon_workspace_bytes(op._h, sct.WS_SB, 1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    P = sct.SbParams(1.0, 1.0, 0.0, 2, 2, sct.SB_RESUME, 0)
    import ctypes
    h = ctypes.c_void_p()
    assert L.split_bregman_tv_graph(op._h, ctypes.byref(P), sct._vp(f.data_ptr()), sct._vp(mu.data_ptr()),
                                    1, sct._vp(ws.data_ptr()), nbytes, None, ctypes.byref(h)) == -1
    assert "captured" in L.radon_last_error().decode()
