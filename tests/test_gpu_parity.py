"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Operator kinds: "f64" (FP64 matrix and vectors), "f32" (FP32 matrix and
vectors) and "mixed" (FP32 matrix values, FP64 vectors and multiply-adds).

Tolerances (relative L2 against the FP64 oracle):
* single products: 1e-12 for f64, 1e-5 for f32 and mixed (FP32 matrix values);
* CG and split-Bregman trajectories: 1e-7 for f64 (a different summation
  order is amplified by the conditioning of the normal operator), 1e-5 for
  mixed (the accuracy the workloads are measured at).  Pure f32 trajectories
  drift by ~1e-2 from exact arithmetic within ten CG steps on these
  operators (FP32 rounding of the iterates times the conditioning; the same
  drift shows in a CPU emulation of FP32 CG), so f32 solves are only checked
  loosely and are not used for accuracy claims.
Matrix entries are compared exactly: the builder evaluates the same
crossing-parameter formulas in plain IEEE double, so FP64 entries are bitwise
equal to the oracle's and FP32 entries are the oracle's rounded once.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, rounded, say, to_dev, torch, workload_problem

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
MODES = {"f64": (F64, F64), "f32": (F32, F32), "mixed": (F32, F64)}


def make_op(n, na, nb, mask, mode):
    mat, vec = MODES[mode]
    return sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec)

# (n, n_angles, n_bins, measured-every): ragged sizes, odd N, even bin counts
# (half-integer offsets), bins narrower than the image, subsampled angles
SMALL = [
    (8, 8, 13, 1), (8, 7, 13, 1), (7, 8, 11, 1), (8, 12, 16, 1), (8, 6, 5, 1),
    (33, 10, 47, 2), (64, 45, 91, 1), (100, 30, 143, 3), (1, 4, 3, 1), (2, 1, 3, 1),
]


def _ids(c):
    return "n%d_a%d_b%d_e%d" % c


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def oracle_rows_sorted(op_o):
    return op_o.MR


@pytest.mark.parametrize("geom", SMALL, ids=_ids)
@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_builder_matches_oracle_entries(geom, mode):
    n, na, nb, every = geom
    say(f"builder {geom} {mode}")
    mask = W.angle_mask(na, every)
    ref = oracle.OracleOp(n, na, nb, mask)
    op = make_op(n, na, nb, mask, mode)
    dtype = MODES[mode][0]
    assert op.info.nnz == ref.MR.nnz
    rp, col, val = op.export_csr()
    np.testing.assert_array_equal(rp, ref.MR.rp)
    conv = (lambda v: v) if dtype == F64 else (lambda v: v.astype(np.float32).astype(np.float64))
    for i in range(ref.rows):
        a, b = rp[i], rp[i + 1]
        o = np.argsort(col[a:b], kind="stable")
        np.testing.assert_array_equal(col[a:b][o], ref.MR.ci[a:b])
        np.testing.assert_array_equal(val[a:b][o], conv(ref.MR.v[a:b]))
    # the adjoint layout holds exactly the transpose's entries
    bins, v0, v1 = op.export_adj()
    nm = ref.angles.size
    T = ref.MRT
    for j in range(n * n):
        want = dict(zip(T.ci[T.rp[j]:T.rp[j + 1]].tolist(), conv(T.v[T.rp[j]:T.rp[j + 1]]).tolist()))
        got = {}
        for a in range(nm):
            bb = bins[j * nm + a]
            if bb < 0:
                continue
            if v0[j * nm + a] != 0:
                got[a * nb + bb] = v0[j * nm + a]
            if v1[j * nm + a] != 0:
                got[a * nb + bb + 1] = v1[j * nm + a]
        assert got == want, j


@pytest.mark.parametrize("geom", SMALL, ids=_ids)
@pytest.mark.parametrize("mode", ["f64", "f32", "mixed"])
def test_products_match_oracle(geom, mode):
    n, na, nb, every = geom
    say(f"products {geom} {mode}")
    mask = W.angle_mask(na, every)
    ref = oracle.OracleOp(n, na, nb, mask)
    op = make_op(n, na, nb, mask, mode)
    dtype = MODES[mode][1]
    tol = 1e-12 if mode == "f64" else 1e-5
    rng = np.random.default_rng(n * 1000 + na)
    x = rounded(rng.standard_normal(n * n), dtype)
    y = rounded(rng.standard_normal(ref.rows), dtype)
    assert rel_l2(host(op.fwd(to_dev(x, dtype))), ref.fwd(x)) <= tol
    assert rel_l2(host(op.adj(to_dev(y, dtype))), ref.adj(y)) <= tol
    for alpha, lam, sigma in ((10.0, 1.0, 0.0), (1.0, 0.0, 1.0), (2.5, 0.3, 0.7)):
        out, dot = op.normal(to_dev(x, dtype), alpha, lam, sigma, dot=True)
        want = ref.normal(x, alpha, lam, sigma)
        assert rel_l2(host(out), want) <= tol, (alpha, lam, sigma)
        d = float(host(dot)[0])
        assert abs(d - np.dot(x, want)) <= 10 * tol * np.abs(x).dot(np.abs(want))


def test_adjoint_identity_fp64():
    w = W.WORKLOADS["small_64_f64"]
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F64)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(op.nn), rng.standard_normal(op.rows)
    Rx = host(op.fwd(to_dev(x, F64)))[0]
    Rty = host(op.adj(to_dev(y, F64)))[0]
    assert abs(Rx @ y - x @ Rty) <= 1e-12 * np.linalg.norm(Rx) * np.linalg.norm(y)


@pytest.mark.parametrize("geom", [(64, 45, 91, 1), (33, 10, 47, 2), (8, 1, 13, 1)], ids=_ids)
def test_forward_kernel_with_caller_transpose(geom):
    """radon_fwd_xt (the caller holds the transposed image) equals radon_fwd
    bitwise; without xT it is refused where some angle needs it."""
    n, na, nb, ev = geom
    op = make_op(n, na, nb, W.angle_mask(na, ev), "mixed")
    rng = np.random.default_rng(6)
    X = to_dev(rng.standard_normal((3, n * n)), F64)
    XT = X.reshape(3, n, n).transpose(1, 2).contiguous().reshape(3, -1)
    assert torch.equal(op.fwd_xt(X, XT), op.fwd(X))
    if op.needs_transpose:
        with pytest.raises(sct.SparsectError, match="transposed"):
            op.fwd_xt(X, None)
    else:
        assert torch.equal(op.fwd_xt(X, None), op.fwd(X))


@pytest.mark.parametrize("batch", [4, 8, 16, 21])
@pytest.mark.parametrize("mode", ["mixed", "f32"])
def test_fused_batch_products_equal_single_image(batch, mode):
    """Chunks of 4/8/16 right-hand sides share every matrix load; each image's
    result must be bitwise the single-image result (same summation order)."""
    n, na = 40, 30
    op = make_op(n, na, W.n_bins_for(n), W.angle_mask(na, 2), mode)
    dt = MODES[mode][1]
    rng = np.random.default_rng(batch)
    X = to_dev(rng.standard_normal((batch, n * n)), dt)
    Yb = op.fwd(X)
    Ab, Db = op.normal(X, 2.0, 0.5, 0.25, dot=True)
    Tb = op.adj(Yb)
    for b in (0, batch // 2, batch - 1):
        xb = X[b:b + 1].contiguous()
        assert torch.equal(op.fwd(xb)[0], Yb[b])
        a1, d1 = op.normal(xb, 2.0, 0.5, 0.25, dot=True)
        assert torch.equal(a1[0], Ab[b]) and torch.equal(d1[0], Db[b])
        assert torch.equal(op.adj(Yb[b:b + 1].contiguous())[0], Tb[b])


def test_fused_batch_split_bregman_and_cg():
    w, ref, mu, f = workload_problem("small_64_f64")
    op = make_op(w.n, w.n_angles, w.n_bins, w.mask, "mixed")
    rng = np.random.default_rng(3)
    F = np.stack([f * (1 + 0.1 * k) + rng.standard_normal(f.size) for k in range(6)])
    Fd = to_dev(F, F64)
    U, info = op.sb(Fd, w.alpha, w.lam, 5, 5)
    X, cinfo = op.cg(Fd[:, :0].new_zeros((6, op.nn)) + 1.0, w.alpha, w.lam, 0.5, n_iter=7)
    for b in (0, 5):
        u1, _ = op.sb(Fd[b:b + 1].contiguous(), w.alpha, w.lam, 5, 5, ws_key="single")
        assert torch.equal(u1[0], U[b])
    uo = ref.sb(F[5], w.alpha, w.lam, 5, 5)[0]
    assert rel_l2(host(U[5]), uo) <= 1e-5
    assert [d["outer"] for d in sct.decode_sb_info(info)] == [5] * 6
    x1, _ = op.cg(torch.ones((1, op.nn), dtype=F64, device="cuda"), w.alpha, w.lam, 0.5, n_iter=7)
    assert torch.equal(x1[0], X[3])


def test_batch_equals_per_slice_and_is_deterministic():
    n, na, nb = 48, 20, W.n_bins_for(48)
    op = sct.RadonOp(n, na, nb, W.angle_mask(na, 2), dtype=F32)
    rng = np.random.default_rng(11)
    X = to_dev(rng.standard_normal((3, n * n)), F32)
    Y = op.normal(X, 10.0, 1.0)
    for b in range(3):
        yb = op.normal(X[b:b + 1].contiguous(), 10.0, 1.0)
        assert torch.equal(yb[0], Y[b])
    Y2 = op.normal(X, 10.0, 1.0)
    assert torch.equal(Y, Y2)
    S = op.fwd(X)
    assert torch.equal(op.fwd(X[1:2].contiguous())[0], S[1])


@pytest.mark.parametrize("mode,tol", [("f64", 1e-7), ("mixed", 1e-5), ("f32", 5e-2)])
def test_cg_matches_oracle(mode, tol):
    w, ref, mu, f = workload_problem("small_64_f64")
    op = make_op(w.n, w.n_angles, w.n_bins, w.mask, mode)
    dtype = MODES[mode][1]
    rhs = rounded(w.alpha * ref.adj(f), dtype)
    for sigma, x0 in ((0.0, None), (0.5, rounded(mu, dtype))):
        x, info = op.cg(to_dev(rhs, dtype), w.alpha, w.lam, sigma,
                        x0=None if x0 is None else to_dev(x0, dtype), n_iter=10)
        xo, ro, hist, it, bd = ref.cg(w.alpha, w.lam, sigma, rhs=rhs, x0=x0, n_iter=10)
        assert rel_l2(host(x), xo) <= tol
        inf = sct.decode_cg_info(info)[0]
        assert inf["iterations"] == it == 10 and inf["breakdown"] == bd == 0
        # r_0 = rhs - A x_0 cancels, so rho_0 carries the matrix/vector rounding
        assert abs(inf["rho0"] - hist[0]) <= {"f64": 1e-9, "mixed": 1e-4, "f32": 1e-3}[mode] * hist[0]
        # the final residual norm is more sensitive than the iterate itself; in pure
        # FP32 the recurred residual norm drifts by a factor ~2 within ten steps
        if mode != "f32":
            assert abs(inf["rho"] - hist[-1]) <= {"f64": 1e-6, "mixed": 1e-4}[mode] * hist[-1]


@pytest.mark.parametrize("geom", [(100, 30, 143, 3), (33, 10, 47, 2), (64, 45, 91, 1)], ids=_ids)
@pytest.mark.parametrize("mode,tol", [("f64", 1e-7), ("mixed", 1e-5)])
def test_cg_matches_oracle_ragged_batch(geom, mode, tol):
    """CG on three right-hand sides at once.  At 100 and 33 pixels the vector
    kernels' last blocks and tiles are partial (the path with per-element
    tests); at 64 every block is whole.  Each image must match its own
    oracle solve."""
    n, na, nb, every = geom
    mask = W.angle_mask(na, every)
    say(f"cg ragged batch {geom} {mode}")
    op = make_op(n, na, nb, mask, mode)
    ref = oracle.OracleOp(n, na, nb, mask, values="f32" if mode == "mixed" else "f64")
    dtype = MODES[mode][1]
    rng = np.random.default_rng([3, n])
    rhs = rounded(rng.standard_normal((3, n * n)), dtype)
    x, info = op.cg(to_dev(rhs, dtype), 0.5, 1.0, 0.1, n_iter=12)
    got = host(x)
    for b in range(3):
        xo = ref.cg(0.5, 1.0, 0.1, rhs=rhs[b], n_iter=12)[0]
        assert rel_l2(got[b], xo) <= tol, (geom, mode, b)
    infos = sct.decode_cg_info(info)
    assert all(i["iterations"] == 12 and i["breakdown"] == 0 for i in infos)


def test_cg_guards_on_gpu():
    n = 8
    op = sct.RadonOp(n, 4, W.n_bins_for(n), np.array([1, 0, 0, 0], np.uint8), dtype=F64)
    # zero right-hand side: nothing to do
    x, info = op.cg(torch.zeros((1, n * n), dtype=F64, device="cuda"), 1.0, 1.0, n_iter=5)
    inf = sct.decode_cg_info(info)[0]
    assert inf["iterations"] == 0 and inf["breakdown"] == 0 and not host(x).any()
    # a null-space direction of R^T R (theta = 0 only, lambda = sigma = 0): breakdown at step 1
    rhs = np.zeros(n * n)
    rhs[:8], rhs[8:16] = 1.0, -1.0
    x, info = op.cg(to_dev(rhs, F64), 1.0, 0.0, 0.0, n_iter=3)
    inf = sct.decode_cg_info(info)[0]
    assert inf["breakdown"] == 1 and inf["iterations"] == 0
    # relative tolerance stops early, like the oracle (sigma = 1 keeps the system well
    # conditioned, so the iterates of the two implementations stay close)
    ref = oracle.OracleOp(16, 12, W.n_bins_for(16))
    op2 = sct.RadonOp(16, 12, W.n_bins_for(16), dtype=F64)
    rhs = np.random.default_rng(0).standard_normal(256)
    xo, ro, hist, it, bd = ref.cg(0.1, 1.0, 1.0, rhs=rhs, n_iter=200, rtol=1e-6)
    x, info = op2.cg(to_dev(rhs, F64), 0.1, 1.0, 1.0, n_iter=200, rtol=1e-6)
    assert sct.decode_cg_info(info)[0]["iterations"] == it < 200
    assert rel_l2(host(x), xo) <= 1e-9


@pytest.mark.parametrize("mode,tol", [("f64", 1e-7), ("mixed", 1e-5), ("f32", 5e-2)])
def test_split_bregman_small_workload(mode, tol):
    w, ref, mu, f = workload_problem("small_64_f64")
    dtype = MODES[mode][1]
    fr = rounded(f, dtype)
    say(f"sb small {mode}")
    u, info = make_op(w.n, w.n_angles, w.n_bins, w.mask, mode).sb(
        to_dev(fr, dtype), w.alpha, w.lam, w.n_outer, w.n_cg)
    uo, ub, uu, k, st = ref.sb(fr, w.alpha, w.lam, w.n_outer, w.n_cg)
    assert rel_l2(host(u), uo) <= tol
    inf = sct.decode_sb_info(info)[0]
    assert inf["outer"] == w.n_outer and inf["breakdowns"] == 0
    t_last, t_first = {"f64": (1e-6, 1e-6), "mixed": (1e-3, 1e-4), "f32": (0.2, 0.2)}[mode]
    assert abs(inf["upd_b"] - ub[-1]) <= t_last * ub[-1]
    assert abs(inf["upd_b_first"] - ub[0]) <= t_first * ub[0]


def test_split_bregman_resume_warm_and_tol():
    w, ref, mu, f = workload_problem("small_64_f64")
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F64)
    fd = to_dev(f, F64)
    u20, _ = op.sb(fd, w.alpha, w.lam, 20, 5, ws_key="a")
    u10, _ = op.sb(fd, w.alpha, w.lam, 10, 5, ws_key="b")
    u10b, _ = op.sb(fd, w.alpha, w.lam, 10, 5, resume=True, out=u10, ws_key="b")
    assert torch.equal(u10b, u20)
    # warm start from an image, like the oracle
    u0 = rounded(0.5 * mu, F64)
    uw, _ = op.sb(fd, w.alpha, w.lam, 5, 5, mu0=to_dev(u0, F64))
    uo = ref.sb(f, w.alpha, w.lam, 5, 5, u0=u0)[0]
    assert rel_l2(host(uw), uo) <= 1e-7
    # tolerance stop after the same number of outer iterations
    ut, info = op.sb(fd, w.alpha, w.lam, 200, 5, tol=0.3)
    uo, ub, uu, k, st = ref.sb(f, w.alpha, w.lam, 200, 5, tol=0.3)
    assert sct.decode_sb_info(info)[0]["outer"] == k < 200
    assert rel_l2(host(ut), uo) <= 1e-6      # a longer FP64 trajectory: more amplification


def test_main_workload_normal_and_split_bregman():
    """The 512^2 workload (FP32 matrix, 180 of 360 angles, 725 bins) in the
    launch configuration the benchmark times: full-size parity."""
    say("gpu_512_f32: oracle build")
    w, ref, mu, f = workload_problem("gpu_512_f32")
    say("gpu_512_f32: gpu build")
    op = make_op(w.n, w.n_angles, w.n_bins, w.mask, "mixed")
    op32 = make_op(w.n, w.n_angles, w.n_bins, w.mask, "f32")
    assert op.info.nnz == ref.MR.nnz
    x = rounded(mu, F32)
    say("gpu_512_f32: normal")
    want = ref.normal(x, w.alpha, w.lam)
    assert rel_l2(host(op.normal(to_dev(x, F64), w.alpha, w.lam)), want) <= 1e-5
    assert rel_l2(host(op32.normal(to_dev(x, F32), w.alpha, w.lam)), want) <= 1e-5
    # the compact forward layout of 64 rays over 2 angles at 4 waves per
    # bundle, as the benchmark's tuned operator
    opc = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64, tuning="default",
                      bundle=64, bundle_angles=2, compact=True)
    opc.tuning = {"fwd_waves": 4}
    assert rel_l2(host(opc.normal(to_dev(x, F64), w.alpha, w.lam)), want) <= 1e-5
    # and also stored by the symmetries of the square, compact or with both
    # lengths (32 rays over 2 angles: the layout the benchmark's chooser
    # picked on this operator)
    ops = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64, tuning="default",
                      bundle=64, bundle_angles=2, compact=True, symmetric=True)
    ops.tuning = {"fwd_waves": 4}
    assert rel_l2(host(ops.normal(to_dev(x, F64), w.alpha, w.lam)), want) <= 1e-5
    opy = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=F32, vec_dtype=F64, tuning="default",
                      bundle=32, bundle_angles=2, symmetric=True)
    opy.tuning = {"fwd_waves": 4, "adj_waves": 2}
    assert rel_l2(host(opy.normal(to_dev(x, F64), w.alpha, w.lam)), want) <= 1e-5
    fr = rounded(f, F32)
    say("gpu_512_f32: split Bregman 50x20 on the GPU")
    u, info = op.sb(to_dev(fr, F64), w.alpha, w.lam, w.n_outer, w.n_cg)
    uc, _ = opc.sb(to_dev(fr, F64), w.alpha, w.lam, w.n_outer, w.n_cg)
    us, _ = ops.sb(to_dev(fr, F64), w.alpha, w.lam, w.n_outer, w.n_cg)
    uy, _ = opy.sb(to_dev(fr, F64), w.alpha, w.lam, w.n_outer, w.n_cg)
    say("gpu_512_f32: split Bregman 50x20 on the oracle")
    uo = ref.sb(fr, w.alpha, w.lam, w.n_outer, w.n_cg)[0]
    err = rel_l2(host(u), uo)
    err_c = rel_l2(host(uc), uo)
    err_s = rel_l2(host(us), uo)
    err_y = rel_l2(host(uy), uo)
    say(f"gpu_512_f32: split Bregman rel L2 = {err:.3e}, compact layout {err_c:.3e}, "
        f"compact and symmetric {err_s:.3e}, symmetric {err_y:.3e}")
    assert err <= 1e-5
    assert err_c <= 1e-5
    assert err_s <= 1e-5
    assert err_y <= 1e-5


def test_large_workload_sampled_and_invariants():
    """The 2048^2 FP32 workload (90 angles, 2897 bins): sampled rows and columns
    against the oracle ray by ray, plus size-independent invariants."""
    w = W.WORKLOADS["large_2048_f32"]
    say("large_2048_f32: gpu build")
    op = make_op(w.n, w.n_angles, w.n_bins, w.mask, "f32")
    n, nb = w.n, w.n_bins
    rng = np.random.default_rng(21)
    mu = rounded(W.phantom(n, w.n_ellipses, seed=0), F32)
    xd = to_dev(mu, F32)
    y = host(op.fwd(xd))[0]
    say("large_2048_f32: sampled rays")
    for i in rng.integers(0, op.rows, 40):
        k, b = divmod(int(i), nb)
        cols, vals = oracle.ray(n, w.n_angles, nb, k, b)
        want = float(np.dot(vals, mu[cols]))
        assert abs(y[i] - want) <= 1e-5 * max(1.0, np.abs(vals).dot(np.abs(mu[cols])))
    # adjoint columns: pixel j gathers the (<= 2 per angle) rays crossing it
    g = rng.standard_normal(op.rows).astype(np.float32).astype(np.float64)
    xt = host(op.adj(to_dev(g, F32)))[0]
    say("large_2048_f32: sampled pixels")
    for j in rng.integers(0, n * n, 12):
        iy, ix = divmod(int(j), n)
        want, scale = 0.0, 0.0
        for k in range(w.n_angles):
            c, s = oracle.trig(k, w.n_angles)
            sc = (ix - n / 2 + 0.5) * c + (iy - n / 2 + 0.5) * s + (nb - 1) / 2
            for b in range(int(np.floor(sc)) - 1, int(np.floor(sc)) + 3):
                if 0 <= b < nb:
                    cols, vals = oracle.ray(n, w.n_angles, nb, k, b)
                    hit = vals[cols == j]
                    if hit.size:
                        want += hit[0] * g[k * nb + b]
                        scale += abs(hit[0] * g[k * nb + b])
        assert abs(xt[j] - want) <= 1e-5 * max(1.0, scale), j
    # invariants at full size: adjoint identity and symmetry of the normal operator
    v = to_dev(rng.standard_normal(n * n), F32)
    # (random-sign sums: tolerances scale with the Cauchy-Schwarz bound)
    vh = host(v).reshape(-1)
    Rv = host(op.fwd(v))[0]
    a1, a2 = float(np.dot(Rv, g)), float(np.dot(vh, xt))
    assert abs(a1 - a2) <= 1e-5 * np.linalg.norm(Rv) * np.linalg.norm(g)
    Av = host(op.normal(v, w.alpha, w.lam))[0]
    Ax = host(op.normal(xd, w.alpha, w.lam))[0]
    s1, s2 = np.dot(mu, Av), np.dot(vh, Ax)
    assert abs(s1 - s2) <= 1e-5 * np.linalg.norm(mu) * np.linalg.norm(Av)


def test_workspace_and_argument_errors_on_gpu():
    op = sct.RadonOp(16, 8, W.n_bins_for(16), dtype=F32)
    L = sct.lib()
    x = torch.zeros(256, dtype=F32, device="cuda")
    out = torch.zeros(256, dtype=F32, device="cuda")
    ws, nbytes = op.workspace(sct.WS_NORMAL, 1)
    rc = L.normal_apply(op._h, 1.0, 1.0, 0.0, sct._vp(x.data_ptr()), sct._vp(out.data_ptr()), None, 1, 0,
                        sct._vp(ws.data_ptr()), nbytes - 1, None)
    assert rc == -4 and "workspace" in L.radon_last_error().decode()
    rc = L.normal_apply(op._h, 1.0, 1.0, 0.0, sct._vp(x.data_ptr()), sct._vp(x.data_ptr()), None, 1, 0,
                        sct._vp(ws.data_ptr()), nbytes, None)
    assert rc == -1 and "alias" in L.radon_last_error().decode()
    with pytest.raises(sct.SparsectError):
        op.fwd(torch.zeros(255, dtype=F32, device="cuda"))
    with pytest.raises(sct.SparsectError):
        op.fwd(torch.zeros(256, dtype=F64, device="cuda"))


def test_tuning_setter_autotune_and_parity(tmp_path, monkeypatch):
    monkeypatch.setenv("SPARSECT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_1705_07497_amd import autotune
    n, na = 48, 30
    mask = W.angle_mask(na, 2)
    ref = oracle.OracleOp(n, na, W.n_bins_for(n), mask)
    op = make_op(n, na, W.n_bins_for(n), mask, "mixed")
    assert op.tuning == {"fwd_waves": 2, "adj_waves": 0, "fwd_rhs": 4, "adj_rhs": 8, "fwd_layout": 0,
                         "fwd_lines": 0, "adj_layout": 0, "reserved": 0}
    with pytest.raises(sct.SparsectError):
        op.tuning = {"fwd_waves": 3}
    with pytest.raises(sct.SparsectError):
        op.tuning = {"adj_rhs": 5}
    with pytest.raises(sct.SparsectError):
        op.tuning = {"fwd_layout": 2}
    with pytest.raises(sct.SparsectError):
        op.tuning = {"adj_layout": -1}
    with pytest.raises(sct.SparsectError):
        op.tuning = {"reserved": 1}
    with pytest.raises(sct.SparsectError):
        op.tuning = {"fwd_lines": 32}     # no band sets below 256 pixels
    with pytest.raises(sct.SparsectError):
        op.tuning = {"fwd_rhs_typo": 4}
    x = rounded(np.random.default_rng(1).standard_normal((6, n * n)), F64)
    want = [ref.normal(x[b], 1.0, 0.5, 0.1) for b in range(6)]
    for fw in (2, 4):
        for aw in (1, 2, 4):
            for fr, ar, lay in ((1, 1, 0), (4, 8, 0), (8, 4, 0), (4, 8, 1), (8, 4, 1), (4, 16, 1)):
                op.tuning = {"fwd_waves": fw, "adj_waves": aw, "fwd_rhs": fr, "adj_rhs": ar, "fwd_layout": lay,
                             "adj_layout": lay}
                got = host(op.normal(to_dev(x, F64), 1.0, 0.5, 0.1))
                for b in range(6):
                    assert rel_l2(got[b], want[b]) <= 1e-5, (fw, aw, fr, ar, lay, b)
    entry = autotune.autotune(op, batch=8)
    assert entry["source"] == "timed"
    assert set(entry["tuning"]) == set(autotune.DEFAULT)
    assert op.tuning == entry["tuning"]
    got = host(op.normal(to_dev(x, F64), 1.0, 0.5, 0.1))
    for b in range(6):
        assert rel_l2(got[b], want[b]) <= 1e-5, b
    # a second operator of the same geometry picks the cached entry up
    op2 = sct.RadonOp(n, na, W.n_bins_for(n), mask, dtype=F32, vec_dtype=F64, tune_batch=8)
    assert op2.tuning == entry["tuning"]
    assert autotune.autotune(op2, batch=8)["source"] == "cache"


@pytest.mark.parametrize("mode", ["mixed", "f32", "f64"])
def test_bundle_widths_match_oracle_and_each_other(mode):
    """The forward layout's bundle width (16, 32, 64 rays) changes only how
    each ray's sum is split: every width matches the oracle, and the layouts
    hold the same entries as the CSR."""
    n, na, ev = 70, 36, 2
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, ev)
    ref = oracle.OracleOp(n, na, nb, mask)
    mat, vec = MODES[mode]
    rng = np.random.default_rng(5)
    x = rounded(rng.standard_normal((5, n * n)), vec)
    tol = 1e-12 if mode == "f64" else 1e-5
    outs = {}
    for bw in (16, 32, 64):
        op = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", bundle=bw)
        assert op.bundle == bw
        op.tuning = {"fwd_rhs": 4, "adj_rhs": 4}
        y = host(op.fwd(to_dev(x, vec)))
        o = host(op.normal(to_dev(x, vec), 0.7, 0.3, 0.05))
        for b in range(5):
            assert rel_l2(y[b], ref.fwd(x[b])) <= tol, (bw, b)
            assert rel_l2(o[b], ref.normal(x[b], 0.7, 0.3, 0.05)) <= tol, (bw, b)
        outs[bw] = y
        rp, col, val = op.export_csr()
        np.testing.assert_array_equal(rp, ref.MR.rp)
    for bw in (32, 64):
        assert np.max(np.abs(outs[bw] - outs[16])) <= 1e-4 * np.max(np.abs(outs[16])) + 1e-300


def test_bundle_width_in_banded_volume_and_group():
    """Bundle widths through the line-banded forward (1024 pixels) and a group."""
    n, na = 1024, 8
    nb = W.n_bins_for(n)
    ref = oracle.OracleOp(n, na, nb)
    x = np.random.default_rng(8).standard_normal((3, n * n))
    for bw in (32, 64):
        op = sct.RadonOp(n, na, nb, None, dtype=F64, tuning="default", bundle=bw)
        op.tuning = {"fwd_rhs": 1}
        y = host(op.fwd(to_dev(x, F64)))
        for b in range(3):
            assert rel_l2(y[b], ref.fwd(x[b])) <= 1e-12, (bw, b)
    ops = [sct.RadonOp(m, a, W.n_bins_for(m), None, dtype=F64, tuning="default", bundle=32)
           for m, a in ((64, 12), (96, 20))]
    g = sct.RadonMulti(ops, 1.0, 0.5, 0.0)
    xs = [to_dev(np.random.default_rng(i).standard_normal(o.nn), F64) for i, o in enumerate(ops)]
    A = g.apply(2, g.pack_images(xs))
    for i, o in enumerate(ops):
        r = oracle.OracleOp(o.n, o.n_angles, o.n_bins)
        assert rel_l2(host(g.image(A, i)), r.normal(host(xs[i]), 1.0, 0.5, 0.0)) <= 1e-12
    with pytest.raises(sct.SparsectError, match="bundle width"):
        sct.RadonMulti([ops[0], sct.RadonOp(64, 12, W.n_bins_for(64), None, dtype=F64,
                                            tuning="default", bundle=16)])


@pytest.mark.parametrize("compact", [False, True])
def test_caller_buffer_build_symmetric(compact):
    """The caller-buffer build of operators stored by symmetry (forward and,
    with n a multiple of 8, adjoint): the same sizes, records and products,
    bitwise, as the library build."""
    n, na = 120, 48
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, 2)
    kw = dict(dtype=F32, vec_dtype=F64, tuning="default", bundle=32, bundle_angles=2, compact=compact,
              symmetric=True)
    a = sct.RadonOp(n, na, nb, mask, **kw)
    b = sct.RadonOp(n, na, nb, mask, storage="torch", **kw)
    assert a.adj_symmetric and b.adj_symmetric
    assert b.sizes["fwd_slots"] == a.info.fwd_slots and b.sizes["adj_slots"] == a.info.adj_slots
    for u, v in zip(a.export_adj(), b.export_adj()):
        np.testing.assert_array_equal(u, v)
    x = to_dev(np.random.default_rng(3).standard_normal((2, n * n)), F64)
    y = to_dev(np.random.default_rng(4).standard_normal((2, a.rows)), F64)
    assert torch.equal(a.fwd(x), b.fwd(x))
    assert torch.equal(a.adj(y), b.adj(y))
    assert torch.equal(a.normal(x, 1.0, 0.5), b.normal(x, 1.0, 0.5))


@pytest.mark.parametrize("mode", ["mixed", "f64"])
def test_caller_buffer_build_equals_library_build(mode):
    """radon_csr_sizes + build_radon_csr_into (every array a torch tensor)
    produce bitwise the operator build_radon_csr produces."""
    n, na, ev = 120, 50, 2
    nb = W.n_bins_for(n)
    mask = W.angle_mask(na, ev)
    mat, vec = MODES[mode]
    a = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default")
    b = sct.RadonOp(n, na, nb, mask, dtype=mat, vec_dtype=vec, tuning="default", storage="torch")
    assert b.sizes["nnz"] == a.info.nnz and b.sizes["fwd_slots"] == a.info.fwd_slots
    assert b.sizes["adj_slots"] == a.info.adj_slots
    ea, eb = a.export_csr(), b.export_csr()
    for u, v in zip(ea, eb):
        np.testing.assert_array_equal(u, v)
    for u, v in zip(a.export_adj(), b.export_adj()):
        np.testing.assert_array_equal(u, v)
    rp, col, val = b.csr()
    np.testing.assert_array_equal(rp.cpu().numpy(), ea[0])
    np.testing.assert_array_equal(col.cpu().numpy(), ea[1])
    np.testing.assert_array_equal(val.double().cpu().numpy(), ea[2])
    x = to_dev(np.random.default_rng(2).standard_normal((3, n * n)), vec)
    assert torch.equal(a.normal(x, 1.0, 0.5), b.normal(x, 1.0, 0.5))
    assert torch.equal(a.fwd(x), b.fwd(x))
    # short buffers are refused before any device work
    L = sct.lib()
    g = sct._Geom(n, na, nb, a.kind, a.measured.ctypes.data_as(sct.ctypes.POINTER(sct.ctypes.c_uint8)))
    sz = sct.RadonSizes()
    assert L.radon_csr_sizes(sct.ctypes.byref(g), None, 0, None, sct.ctypes.byref(sz)) == 0
    assert sz.nnz == -1 and sz.ws_bytes > 0
    ws = torch.empty(sz.ws_bytes, dtype=torch.uint8, device="cuda")
    assert L.radon_csr_sizes(sct.ctypes.byref(g), sct._vp(ws.data_ptr()), sz.ws_bytes - 1, None,
                             sct.ctypes.byref(sz)) == -4
    # a layout block too small for even the bundle table: refused before the count kernels run
    rp2 = torch.empty_like(rp)
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    bufs = sct.RadonBuffers(rp2.data_ptr(), small.data_ptr(), small.data_ptr(), small.data_ptr(),
                            ws.data_ptr(), rp2.numel() * 8, 256, 256, 256, ws.numel())
    h = sct._vp()
    assert L.build_radon_csr_into(sct.ctypes.byref(g), sct.ctypes.byref(bufs), None,
                                  sct.ctypes.byref(h)) == -4
    assert not h.value


@pytest.mark.parametrize("mode", ["mixed", "f64"])
def test_nan_in_data_breaks_down_like_the_oracle(mode):
    """A NaN in the measured data (the central ray of the first angle) makes
    <p, Ap> non-finite at the first step of every inner solve: CG reports a
    breakdown at iteration 1 and leaves x at zero, split Bregman never moves
    u from zero and counts one breakdown per outer iteration -- on the GPU
    exactly as in the oracle."""
    n, na = 16, 12
    nb = W.n_bins_for(n)
    ref = oracle.OracleOp(n, na, nb)
    op = make_op(n, na, nb, None, mode)
    mat, vec = MODES[mode]
    f = rounded(np.random.default_rng(3).standard_normal(ref.rows), vec)
    f[nb // 2] = np.nan
    rhs = ref.adj(f)
    assert np.isnan(rhs).any()
    x_o, _, _, it_o, bd_o = ref.cg(1.0, 1.0, 0.0, rhs=rhs, n_iter=5)
    assert bd_o == 1 and it_o == 0 and not x_o.any()
    x, info = op.cg(to_dev(rhs[None], vec), 1.0, 1.0, 0.0, n_iter=5)
    ci = sct.decode_cg_info(info)[0]
    assert ci["breakdown"] == bd_o and ci["iterations"] == it_o
    assert not host(x).any()
    u_o = ref.sb(f, 1.0, 1.0, 3, 4)[0]
    assert not u_o.any()
    u, sinfo = op.sb(to_dev(f[None], vec), 1.0, 1.0, 3, 4)
    si = sct.decode_sb_info(sinfo)[0]
    assert si["breakdowns"] == 3 and si["outer"] == 3
    assert not host(u).any()
