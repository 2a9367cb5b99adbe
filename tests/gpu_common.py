"""Shared helpers for the GPU tests: seeded inputs, oracle comparisons."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    want = np.asarray(want, dtype=np.float64).reshape(-1)
    den = np.linalg.norm(want)
    return float(np.linalg.norm(got - want) / (den if den > 0 else 1.0))


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rounded(a, dtype):
    """The values the GPU receives: the oracle runs on exactly these."""
    return np.asarray(a, dtype=np.float64).astype(
        np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def workload_problem(name, seed=0):
    """Oracle operator, phantom and noisy measured data of a named workload."""
    w = W.WORKLOADS[name]
    op = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    mu, eps = W.phantom_and_noise(w.n, w.n_ellipses, op.rows, seed=seed)
    y = op.fwd(mu)
    f = y + w.noise * np.sqrt(np.mean(y ** 2)) * eps
    return w, op, mu, f


def say(msg):
    print(msg, flush=True)
