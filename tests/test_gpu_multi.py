"""Mixed batches: several operators of different geometry in one group.

* each instance's forward, adjoint and normal product equals the single
  operator's product bitwise (same per-bundle and per-tile code, same waves);
* CG over the group matches the oracle per instance (on the matrix values the
  kind stores) and starts from the same rho_0 bitwise as cg_solve;
* a captured CG graph replays bitwise like the eager group CG, also with new
  right-hand sides and with other GPU work between replays;
* the full uneven batch (32 instances, N in {256, 512, 1024}, 60-180 angles)
  against per-instance cg_solve, plus the smallest instances against the
  oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import host, need_gpu, rel_l2, rounded, say, to_dev, torch

import paper_1705_07497_amd as sct

pytestmark = pytest.mark.gpu

MODES = {"f64": (torch.float64, torch.float64), "mixed": (torch.float32, torch.float64),
         "f32": (torch.float32, torch.float32)}

# (n, n_angles, n_bins, measured-every): odd and tiny sizes, even bin counts,
# subsampled angles, an instance that needs no transposed image (one angle)
SMALL_GROUP = [(8, 7, 13, 1), (13, 10, 19, 2), (16, 12, 23, 1), (24, 9, 35, 3), (33, 20, 47, 1),
               (40, 1, 57, 1), (64, 45, 91, 1)]


def _group(specs, mode, alpha, lam, sigma):
    mat, vec = MODES[mode]
    ops = [sct.RadonOp(n, na, nb, W.angle_mask(na, ev), dtype=mat, vec_dtype=vec, tuning="default")
           for n, na, nb, ev in specs]
    return ops, sct.RadonMulti(ops, alpha, lam, sigma)


def _oracle(spec, mode):
    n, na, nb, ev = spec
    return oracle.OracleOp(n, na, nb, W.angle_mask(na, ev), values="f64" if mode == "f64" else "f32")


@pytest.mark.parametrize("mode", ["f64", "mixed", "f32"])
def test_group_products_equal_single_products(mode):
    need_gpu()
    dt = MODES[mode][1]
    alpha = [2.0, 1.0, 0.5, 3.0, 1.5, 1.0, 10.0]
    lam = [0.5, 0.0, 1.0, 0.25, 0.0, 2.0, 1.0]
    sigma = [0.0, 1.0, 0.25, 0.0, 0.5, 0.0, 0.0]
    ops, g = _group(SMALL_GROUP, mode, alpha, lam, sigma)
    for o in ops:
        o.tuning = {"fwd_waves": g.fwd_waves, "adj_waves": g.adj_waves}
    rng = np.random.default_rng(1)
    xs = [to_dev(rng.standard_normal(o.nn), dt) for o in ops]
    ys = [to_dev(rng.standard_normal(o.rows), dt) for o in ops]
    X, Y = g.pack_images(xs), g.pack_sinograms(ys)
    F, B, A = g.apply(0, X), g.apply(1, Y), g.apply(2, X)
    for i, o in enumerate(ops):
        say(f"instance {i}: n={o.n} rows={o.rows}")
        assert torch.equal(g.sinogram(F, i), o.fwd(xs[i][None])[0])
        assert torch.equal(g.image(B, i), o.adj(ys[i][None])[0])
        assert torch.equal(g.image(A, i), o.normal(xs[i][None], alpha[i], lam[i], sigma[i])[0])


@pytest.mark.parametrize("mode,tol", [("f64", 1e-7), ("mixed", 1e-7), ("f32", 5e-2)])
def test_group_cg_matches_oracle(mode, tol):
    need_gpu()
    dt = MODES[mode][1]
    alpha, lam = 10.0, 1.0
    ops, g = _group(SMALL_GROUP, mode, alpha, lam, 0.0)
    rng = np.random.default_rng(2)
    rhs = [rounded(rng.standard_normal(o.nn), dt) for o in ops]
    X, info = g.cg(g.pack_images([to_dev(r, dt) for r in rhs]), n_iter=10)
    infos = sct.decode_cg_info(info)
    for i, (spec, o) in enumerate(zip(SMALL_GROUP, ops)):
        ref = _oracle(spec, mode)
        xo, ro, hist, it, bd = ref.cg(alpha, lam, 0.0, rhs=rhs[i], n_iter=10)
        assert rel_l2(host(g.image(X, i)), xo) <= tol, i
        assert infos[i]["iterations"] == it and infos[i]["breakdown"] == bd
        # rho_0 = <rhs, rhs> with the single solver's tile partials: bitwise
        xs, ins = o.cg(to_dev(rhs[i][None], dt), alpha, lam, 0.0, n_iter=10)
        assert infos[i]["rho0"] == sct.decode_cg_info(ins)[0]["rho0"]


def test_group_cg_guards():
    """An all-zero right-hand side stops its instance at once; a null-space
    direction of R^T R (one angle, lambda = sigma = 0) breaks down at step 1;
    the other instances are unaffected."""
    need_gpu()
    specs = [(8, 4, 13, 4), (16, 12, 23, 1), (8, 4, 13, 4)]
    ops, g = _group(specs, "f64", [1.0, 1.0, 1.0], [0.0, 1.0, 1.0], 0.0)
    rhs0 = np.zeros(64)
    rhs0[:8], rhs0[8:16] = 1.0, -1.0   # null space of the theta = 0 projection
    rng = np.random.default_rng(3)
    r1 = rng.standard_normal(256)
    R = g.pack_images([to_dev(rhs0, torch.float64), to_dev(r1, torch.float64),
                       torch.zeros(64, dtype=torch.float64, device="cuda")])
    X, info = g.cg(R, n_iter=6)
    inf = sct.decode_cg_info(info)
    assert inf[0]["breakdown"] == 1 and inf[0]["iterations"] == 0
    assert inf[1]["breakdown"] == 0 and inf[1]["iterations"] == 6
    assert inf[2]["iterations"] == 0 and not host(g.image(X, 2)).any()
    xs, _ = ops[1].cg(to_dev(r1[None], torch.float64), 1.0, 1.0, 0.0, n_iter=6)
    assert rel_l2(host(g.image(X, 1)), host(xs)) <= 1e-12


def test_group_cg_graph_replays():
    """A captured solve replays like the eager one, bitwise, three times in a
    row with eager GPU work and new right-hand sides between the replays."""
    need_gpu()
    ops, g = _group(SMALL_GROUP, "mixed", 10.0, 1.0, 0.0)
    graph = g.cg_graph(n_iter=8)
    rng = np.random.default_rng(4)
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):
        say(f"graph replay {rep}")
        R = g.pack_images([to_dev(rng.standard_normal(o.nn), torch.float64) for o in ops])
        graph.rhs.copy_(R)
        graph.launch()
        torch.cuda.synchronize()
        gx, ginfo = graph.x.clone(), graph.info.clone()
        scratch.add_(1.0)                          # unrelated eager work
        ops[3].normal(to_dev(rng.standard_normal((2, ops[3].nn)), torch.float64), 1.0, 1.0)
        X, info = g.cg(R, n_iter=8)
        torch.cuda.synchronize()
        assert torch.equal(gx, X)
        assert torch.equal(ginfo, info)


def test_group_errors():
    need_gpu()
    a = sct.RadonOp(8, 4, 13, dtype=torch.float64)
    b = sct.RadonOp(8, 4, 13, dtype=torch.float32)
    with pytest.raises(sct.SparsectError, match="dtype"):
        sct.RadonMulti([a, b])
    g = sct.RadonMulti([a])
    with pytest.raises(sct.SparsectError):
        g.apply(0, torch.zeros(3, dtype=torch.float64, device="cuda"))
    L = sct.lib()
    X = g.empty_images()
    assert L.radon_multi_apply(g._h, 7, sct._vp(X.data_ptr()), sct._vp(X.data_ptr() + 8), None, 0,
                               None) == -1
    assert L.radon_multi_cg(g._h, sct._vp(X.data_ptr()), sct._vp(X.data_ptr()), 3, 0.0, None, 0,
                            None, None) == -1


def test_uneven_batch_full_size():
    """32 instances of the uneven mixed batch (mixed kind, SB inner operator
    alpha = 0.01, lambda = 1), CG(10) in one group against cg_solve per
    instance, and the two smallest instances against the oracle."""
    need_gpu()
    specs = [(n, na, W.n_bins_for(n), 1) for n, na in W.mixed_batch_specs(32)]
    alpha, lam = 0.01, 1.0
    say("building 32 operators")
    ops, g = _group(specs, "mixed", alpha, lam, 0.0)
    rng = np.random.default_rng(5)
    rhs = [to_dev(rng.standard_normal(o.nn), torch.float64) for o in ops]
    say("group CG")
    X, info = g.cg(g.pack_images(rhs), n_iter=10)
    infos = sct.decode_cg_info(info)
    for i, o in enumerate(ops):
        xs, ins = o.cg(rhs[i][None], alpha, lam, 0.0, n_iter=10)
        si = sct.decode_cg_info(ins)[0]
        assert infos[i]["rho0"] == si["rho0"] and infos[i]["iterations"] == si["iterations"] == 10
        # only the summation order of gamma differs (per-instance partials)
        assert rel_l2(host(g.image(X, i)), host(xs)) <= 1e-10, i
    order = np.argsort([o.nn * o.n_meas for o in ops], kind="stable")[:2]
    for i in order:
        say(f"oracle check of instance {i}: n={specs[i][0]} angles={specs[i][1]}")
        ref = _oracle(specs[i], "mixed")
        xo = ref.cg(alpha, lam, 0.0, rhs=host(rhs[i]), n_iter=10)[0]
        assert rel_l2(host(g.image(X, i)), xo) <= 1e-7


def test_group_tables_in_caller_storage():
    """radon_multi_create_into: the group's device tables in a torch tensor
    (the library allocates nothing) give bitwise the products and the CG of
    the self-allocating group; too small or misaligned storage is refused."""
    need_gpu()
    import ctypes
    ops = [sct.RadonOp(n, na, nb, W.angle_mask(na, ev), dtype=torch.float32, vec_dtype=torch.float64,
                       tuning="default") for n, na, nb, ev in SMALL_GROUP]
    g_lib = sct.RadonMulti(ops, 1.5, 0.5, 0.25)
    g_torch = sct.RadonMulti(ops, 1.5, 0.5, 0.25, storage="torch")
    assert g_torch._tables is not None and g_lib._tables is None
    rng = np.random.default_rng(7)
    X = g_lib.pack_images([to_dev(rng.standard_normal(o.nn), torch.float64) for o in ops])
    for which in (0, 2):
        assert torch.equal(g_torch.apply(which, X), g_lib.apply(which, X)), which
    x1, i1 = g_lib.cg(X, n_iter=6)
    x2, i2 = g_torch.cg(X, n_iter=6)
    assert torch.equal(x1, x2) and torch.equal(i1, i2)
    L = sct.lib()
    k = len(ops)
    handles = (sct._vp * k)(*[o._h for o in ops])
    nb = ctypes.c_int64()
    assert L.radon_multi_table_bytes(handles, k, ctypes.byref(nb)) == 0 and nb.value > 0
    buf = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device="cuda")
    h = sct._vp()
    rc = L.radon_multi_create_into(handles, k, None, None, None, sct._vp(buf.data_ptr()), nb.value - 1,
                                   ctypes.byref(h))
    assert rc == -4 and not h.value
    rc = L.radon_multi_create_into(handles, k, None, None, None, sct._vp(buf.data_ptr() + 16), nb.value,
                                   ctypes.byref(h))
    assert rc == -1 and "aligned" in L.radon_last_error().decode()
