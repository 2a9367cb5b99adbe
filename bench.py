#!/usr/bin/env python3
"""Benchmark of the sparse-Radon split-Bregman hot path on one MI355X.

Workload: the 512 x 512 random-ellipse phantom (10 ellipses), 360 angles on
[0, pi) of which every second one is measured (180), 725 bins, 2% noise,
split Bregman with alpha = 0.01, lambda = 1, 50 outer x 20 CG iterations.  The
operator streams its matrix in FP32 and keeps vectors and multiply-adds in
FP64 (the FP32-matrix / FP64-vector operator kind): with FP32 vectors the CG
iterates drift ~1e-2 from exact arithmetic, far outside the 1e-5 the
reconstruction is checked at.

One step = one full split-Bregman reconstruction (every stage of the path:
the forward product, the adjoint product with the fused normal-operator
epilogue, the CG updates and the Bregman shrink/update steps).  It performs
exactly 50 x 20 = 1000 normal-operator applies, so

  value      = normal-operator applies per second inside the solver
               (1000 * steps / timed seconds, the whole job),
  recon_per_s = reconstructions per second.

The JSON line also carries the standalone back-to-back normal_apply rate,
the roofline of the dominant kernel (algorithmic CSR bytes per launch over
its HIP-event-timed average duration, against the 8 TB/s HBM peak) and the
FP64 CPU oracle timed on the host cores as a reported baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "normal-operator applies/s + HBM GB/s (% peak); split-Bregman recon/s at 1e-5 rel"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "gpu_512_f32"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed split-Bregman reconstructions")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--applies", type=int, default=200, help="timed standalone kernel calls")
    ap.add_argument("--no-verify", action="store_true", help="skip the oracle accuracy check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-applies", type=int, default=0,
                    help="oracle normal applies to time (0: sized to ~15 s)")
    ap.add_argument("--no-batched", action="store_true", help="skip the fused multi-image legs")
    ap.add_argument("--profile", action="store_true",
                    help="profiler mode: 100 forward kernels at each bundle width (16, 32, 64), 100 "
                         "adj, 20 normal applies, one CG(20) solve and the stream copy / read kernels "
                         "over 1 GiB (counter calibration), then exit")
    ap.add_argument("--profile-multi", action="store_true",
                    help="profiler mode for the uneven 32-instance batch: one captured-graph CG(10), "
                         "one eager group CG(10) and the 32 per-instance CG(10) solves, then exit")
    ap.add_argument("--profile-volume", action="store_true",
                    help="profiler mode for the 64 x 1024^2 volume (FP32 kind): 3 fused normal "
                         "applies with 16-image chunks gathering per image, 3 from pixel-major chunk "
                         "copies and 4 single-image applies, then exit")
    ap.add_argument("--bundle", type=int, default=0,
                    help="forward bundle width for the profiler modes (0: 16)")
    ap.add_argument("--profile-fourier", action="store_true",
                    help="profiler mode for the Fourier-domain operator: its build, 20 fused and 20 "
                         "NUFFT normal applies and a plain 1 GiB device copy, then exit")
    return ap.parse_args()


PROFILE = os.path.join(ROOT, "profiles", "k_fwd_k_adj1_512x512_180angles.md")
# forward bundle layouts (rays, angles per bundle, compact storage, stored by
# symmetry) of the --profile sequence, in launch order
PROFILE_LAYOUTS = ((16, 1, 0, 0), (32, 1, 0, 0), (64, 1, 0, 0), (32, 2, 0, 0), (64, 2, 0, 0), (64, 4, 0, 0),
                   (16, 1, 1, 0), (32, 2, 1, 0), (64, 2, 1, 0), (64, 4, 1, 0),
                   (32, 2, 1, 1), (64, 2, 1, 1), (64, 4, 1, 1), (32, 2, 0, 1))


def traffic_from_profile(kernel, bundle=None, angles=1, waves=None, compact=False, symmetric=False):
    """HBM bytes per launch of `kernel` (the forward: of the given bundle
    layout, rays and angles per bundle, compact storage or not, stored by
    symmetry or not, and waves per bundle) from the committed counter record (FETCH_SIZE and WRITE_SIZE
    scaled by the copy-kernel calibration), or None when the record is
    missing or the kernel's sources changed since."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    for line in text.splitlines():
        if not line.startswith("traffic-record ") or f"kernel={kernel} " not in line:
            continue
        kv = dict(tok.split("=", 1) for tok in line.split()[1:])
        if bundle is not None and (kv.get("bundle") != str(bundle) or kv.get("angles", "1") != str(angles)):
            continue
        if waves is not None and kv.get("waves", str(waves)) != str(waves):
            continue
        if bundle is not None and kv.get("compact", "0") != ("1" if compact else "0"):
            continue
        if bundle is not None and kv.get("symmetric", "0") != ("1" if symmetric else "0"):
            continue
        h = hashlib.sha256()
        for f in kv["sources"].split(","):
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != kv["sha256"]:
            return None
        return int(1024 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"])
                           + float(kv["write_kib"]) * float(kv["write_scale"])))
    return None


def host_cpu():
    """CPU model, socket count and OMP_NUM_THREADS of the host the oracle runs on."""
    model, sockets = "unknown", set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    sockets.add(v)
    except OSError:
        pass
    return {"cpu_model": model, "sockets": max(1, len(sockets)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS", "unset")}


def bandwidth_ceiling(sct, torch, dev, nbytes=1 << 30, reps=20):
    """The practical HBM ceiling: the project's own stream copy and read-only
    stream kernels over 1 GiB (HIP events on the current stream)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    src.fill_(1)
    dst = torch.empty_like(src)
    part = torch.empty(4096, dtype=torch.int32, device=dev)
    t_copy = event_time(torch, lambda: sct.bandwidth_probe(sct.PROBE_COPY, src, dst), reps)
    t_read = event_time(torch, lambda: sct.bandwidth_probe(sct.PROBE_READ, src, part), reps)
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_gbs": round(2 * nbytes / t_copy / 1e9, 1), "read_gbs": round(nbytes / t_read / 1e9, 1),
            "bytes": nbytes, "kernels": "k_stream_copy, k_stream_read"}


def event_time(torch, fn, reps):
    """Seconds per call of fn (one untimed call first), HIP events on the
    current stream, which every library call here is enqueued on."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def bench_batched(sct, W, torch, dev, vdt, verify=True):
    """Fused multi-image normal_apply (every matrix load shared by a chunk of up
    to 16 images) against the same images applied one at a time."""
    out = {}
    vdt_main = vdt

    def t(fn, reps):
        return event_time(torch, fn, reps)

    from paper_1705_07497_amd import autotune
    for name in ("grad_16x512_f32", "volume_64x1024_f32"):
        w = W.WORKLOADS[name]
        B = w.batch
        # the volume is the FP32 SpMM of 64 slices (FP32 matrix and vectors, its
        # normal operator within 1e-5 of the FP64 oracle); the gradient batch
        # keeps FP64 vectors for its unrolled CG
        vdt = torch.float32 if name == "volume_64x1024_f32" else vdt_main
        op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                         device=dev, tuning="default")
        X = torch.randn((B, op.nn), dtype=vdt, device=dev)
        O = torch.empty_like(X)
        o1 = torch.empty((1, op.nn), dtype=vdt, device=dev)
        singles = [X[b:b + 1] for b in range(B)]
        alpha, lam = (w.alpha, w.lam) if w.lam > 0 else (w.extra["tau"] * w.alpha, 0.0)
        sigma = 0.0 if w.lam > 0 else 1.0

        def fused(o):
            return lambda: o.normal(X, alpha, lam, sigma, out=O)

        def looped():
            for xb in singles:
                op.normal(xb, alpha, lam, sigma, out=o1)

        # library defaults (16-ray bundles of one angle), then the autotuned
        # operator for this batch: bundle layout chosen over the candidates of
        # choose_bundle, launch settings timed
        tf_def, tl = t(fused(op), 5), t(looped, 2)
        ch = autotune.choose_bundle(w.n, w.n_angles, w.n_bins, w.mask, torch.float32, vdt, dev,
                                    batch=B, reps=3, save=False)
        opt = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                          device=dev, tuning="default", bundle=ch["bundle"], bundle_angles=ch["angles"])
        autotune.autotune(opt, batch=B, save=False)
        tf = t(fused(opt), 5)
        # the fairest one-image-at-a-time baseline: the best single-image
        # operator (bundle layout chosen at one image, both products stored by
        # symmetry where the angle set allows it, launch settings tuned)
        try:
            ch1 = autotune.choose_bundle(w.n, w.n_angles, w.n_bins, w.mask, torch.float32, vdt, dev,
                                         batch=1, reps=3, save=False, symmetric=True)
            sym1 = True
        except sct.SparsectError:
            ch1 = autotune.choose_bundle(w.n, w.n_angles, w.n_bins, w.mask, torch.float32, vdt, dev,
                                         batch=1, reps=3, save=False)
            sym1 = False
        op1 = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                          device=dev, tuning="default", bundle=ch1["bundle"], bundle_angles=ch1["angles"],
                          symmetric=sym1)
        autotune.autotune(op1, batch=1, save=False)

        def looped_best():
            for xb in singles:
                op1.normal(xb, alpha, lam, sigma, out=o1)

        tlb = t(looped_best, 2)
        out[name] = {"batch": B, "n": w.n, "measured_angles": w.n_meas, "bins": w.n_bins,
                     "nnz": op.info.nnz, "vectors": str(vdt).replace("torch.", ""),
                     "fused_ms": round(tf * 1e3, 3),
                     "fused_default_ms": round(tf_def * 1e3, 3),
                     "tuned": {"bundle": opt.bundle, "bundle_angles": opt.bundle_angles, **opt.tuning},
                     "per_image_loop_ms": round(tl * 1e3, 3), "speedup": round(tl / tf, 2),
                     "speedup_default": round(tl / tf_def, 2),
                     "per_image_loop_best_ms": round(tlb * 1e3, 3),
                     "loop_best_layout": {"bundle": op1.bundle, "bundle_angles": op1.bundle_angles,
                                          "symmetric": op1.symmetric, **op1.tuning},
                     "speedup_vs_best_loop": round(tlb / tf, 2),
                     "image_applies_per_s": round(B / tf, 1)}
        print(f"# batched {name}: fused {tf * 1e3:.2f} ms tuned (bundle {opt.bundle}x{opt.bundle_angles}, "
              f"{opt.tuning}), "
              f"{tf_def * 1e3:.2f} ms default, loop {tl * 1e3:.2f} ms ({tl / tf:.2f}x), loop on the best "
              f"single-image operator ({op1.bundle}x{op1.bundle_angles}{' symmetric' if op1.symmetric else ''}) "
              f"{tlb * 1e3:.2f} ms ({tlb / tf:.2f}x)",
              file=sys.stderr, flush=True)
        if name == "grad_16x512_f32":
            out["grad_16x512_f32_autograd"] = bench_autograd(opt, w, torch, dev, vdt, t, op1)
        del op, opt, op1
        torch.cuda.empty_cache()
    vdt = vdt_main
    out["mixed_batch_32"] = bench_mixed_batch(sct, W, torch, dev, vdt, t)
    out["small_batch_64"] = bench_mixed_batch(
        sct, W, torch, dev, vdt, t,
        specs=[(n, na, W.n_bins_for(n)) for n, na in W.small_batch_specs(64)], label="small batch")
    out["large_2048_f32"] = bench_large(sct, W, torch, dev, vdt, t, verify)
    return out


def bench_mixed_batch(sct, W, torch, dev, vdt, t, specs=None, label="mixed batch"):
    """The uneven batch: 32 instances (N in {256, 512, 1024}, 60-180 angles),
    CG(10) on each instance's split-Bregman inner operator (alpha = 0.01,
    lambda = 1): one captured graph replay (one launch per phase over all
    instances, 6 phases per iteration) against the eager group call and
    against 32 separate cg_solve calls.  `specs` replaces the instance list."""
    if specs is None:
        specs = [(n, na, W.n_bins_for(n)) for n, na in W.mixed_batch_specs(32)]
    ops = [sct.RadonOp(n, na, nb, None, dtype=torch.float32, vec_dtype=vdt, device=dev)
           for n, na, nb in specs]
    g = sct.RadonMulti(ops, 0.01, 1.0, 0.0)
    rhs = [torch.randn((1, o.nn), dtype=vdt, device=dev) for o in ops]
    R = g.pack_images(rhs)
    graph = g.cg_graph(n_iter=10)
    graph.rhs.copy_(R)
    xs = [torch.empty_like(r) for r in rhs]

    def replay():
        graph.launch()

    def eager():
        g.cg(R, n_iter=10)

    def looped():
        for o, r, x in zip(ops, rhs, xs):
            o.cg(r, 0.01, 1.0, 0.0, n_iter=10, out=x)

    tg, te, tl = t(replay, 5), t(eager, 5), t(looped, 2)
    nnz = sum(o.info.nnz for o in ops)
    print(f"# {label} {len(ops)} instances: graph {tg * 1e3:.2f} ms, eager group {te * 1e3:.2f} ms, "
          f"per-instance loop {tl * 1e3:.2f} ms", file=sys.stderr, flush=True)
    out = {"instances": len(ops), "sizes": sorted({s[0] for s in specs}),
           "angles": [min(s[1] for s in specs), max(s[1] for s in specs)], "nnz_total": nnz,
           "cg_iterations": 10, "graph_ms": round(tg * 1e3, 3), "eager_group_ms": round(te * 1e3, 3),
           "per_instance_loop_ms": round(tl * 1e3, 3), "speedup_vs_loop": round(tl / tg, 2),
           "instance_applies_per_s": round(len(ops) * 10 / tg, 1)}
    del graph, g, ops
    torch.cuda.empty_cache()
    return out


def bench_surrogate(sct, op, w, f, mu, u_exact, torch, timed, stream):
    """Split Bregman with the surrogate T of Section 3.2 (radius 1, the paper's
    timing setting) in every inner solve, same workload and iteration counts;
    both reconstructions' relative L2 error to the phantom."""
    sur = sct.RadonSurrogate(op, 1)
    op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg, surrogate=sur)
    reps = 10
    t = timed(lambda: op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg, surrogate=sur), reps) / reps
    us, info = op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg, surrogate=sur)
    nrm = torch.linalg.vector_norm(mu)
    e_sur = float(torch.linalg.vector_norm(us - mu) / nrm)
    e_ex = float(torch.linalg.vector_norm(u_exact - mu) / nrm)
    print(f"# surrogate split Bregman (r=1): {t * 1e3:.2f} ms per reconstruction, error to phantom "
          f"{e_sur:.4f} (exact {e_ex:.4f})", file=sys.stderr, flush=True)
    return {"radius": 1, "ms_per_recon": round(t * 1e3, 3), "recon_per_s": round(1.0 / t, 1),
            "rel_err_to_phantom": round(e_sur, 4), "exact_rel_err_to_phantom": round(e_ex, 4)}


def bench_pd(op, w, f, mu, torch, timed):
    """Chambolle-Pock TV on the same workload: 50 primal-dual steps, each a
    10-step CG resolvent of eq:PD_resolve from the current iterate (11
    normal-operator applies per step)."""
    n_outer, n_cg = 50, 10
    op.pd(f, w.alpha, n_outer, n_cg)
    reps = 3
    t = timed(lambda: op.pd(f, w.alpha, n_outer, n_cg), reps) / reps
    u = op.pd(f, w.alpha, n_outer, n_cg)
    err = float(torch.linalg.vector_norm(u - mu) / torch.linalg.vector_norm(mu))
    print(f"# Chambolle-Pock {n_outer} x {n_cg}: {t * 1e3:.1f} ms per reconstruction, error to "
          f"phantom {err:.4f}", file=sys.stderr, flush=True)
    return {"n_outer": n_outer, "n_cg": n_cg, "ms_per_recon": round(t * 1e3, 2),
            "applies_per_s": round(n_outer * (n_cg + 1) / t, 1), "rel_err_to_phantom": round(err, 4)}


def bench_fourier(sct, op, w, mu, torch, timed, profile=False):
    """The Fourier-domain problem of eq:four_obj / eq:SBFFT on the same
    geometry: gridded transforms with m_sp = 6 (about 6 digits), the normal
    operator through the precomputed B B^* of eq:fusedop and through the two
    transforms (the paper's fusing and NUFFT rows), and split Bregman 50 x 20
    on both, with 1% complex noise on F^* mu."""
    t0 = time.perf_counter()
    fo = sct.RadonFourier(op, 6)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    x = torch.randn((1, op.nn), dtype=mu.dtype, device=mu.device)
    out = torch.empty_like(x)
    if profile:
        for path in ("fused", "nufft"):
            for _ in range(20):
                fo.normal(x, w.alpha, w.lam, path=path, out=out)
        # counter calibration: the project's copy kernel over 1 GiB, 5 times
        src = torch.ones(1 << 30, dtype=torch.uint8, device=mu.device)
        dst = torch.empty_like(src)
        for _ in range(5):
            sct.bandwidth_probe(sct.PROBE_COPY, src, dst)
        torch.cuda.synchronize()
        return None
    reps = 50
    res = {"m_sp": fo.m_sp, "grid": fo.grid, "points": fo.P, "build_s": round(build_s, 3),
           "fused_tiles": fo.info["fused_tiles"], "fused_bytes": fo.info["fused_bytes"],
           "spread_nnz": fo.info["spread_nnz"]}
    for path in ("fused", "nufft"):
        fo.normal(x, w.alpha, w.lam, path=path, out=out)
        t = timed(lambda: fo.normal(x, w.alpha, w.lam, path=path, out=out), reps) / reps
        res[f"{path}_normal_us"] = round(t * 1e6, 1)
    # four images per call: the fused path shares each B B^* coefficient
    # load between two grids
    x4 = torch.randn((4, op.nn), dtype=mu.dtype, device=mu.device)
    out4 = torch.empty_like(x4)
    for path in ("fused", "nufft"):
        fo.normal(x4, w.alpha, w.lam, path=path, out=out4)
        t = timed(lambda: fo.normal(x4, w.alpha, w.lam, path=path, out=out4), 20) / 20
        res[f"{path}_normal_batch4_us_per_image"] = round(t / 4 * 1e6, 1)
    fh = fo.fwd(mu)
    g = torch.Generator(device=mu.device).manual_seed(0)
    noise = torch.randn(fh.shape, dtype=fh.dtype, device=fh.device, generator=g)
    fh = (fh + 0.01 * torch.sqrt(torch.mean(fh ** 2)) * noise).contiguous()
    # the unscaled DFT of a projection carries n_bins times its energy
    # (Parseval): alpha / n_bins weights the data term as alpha does on the
    # sinogram
    alpha_f = w.alpha / w.n_bins
    res["alpha"] = alpha_f
    for path in ("fused", "nufft"):
        fo.sb(fh, alpha_f, w.lam, w.n_outer, w.n_cg, path=path)
        t_sb = timed(lambda: fo.sb(fh, alpha_f, w.lam, w.n_outer, w.n_cg, path=path), 3) / 3
        u, _ = fo.sb(fh, alpha_f, w.lam, w.n_outer, w.n_cg, path=path)
        err = float(torch.linalg.vector_norm(u - mu) / torch.linalg.vector_norm(mu))
        res.update({f"sb_{path}_ms_per_recon": round(t_sb * 1e3, 2),
                    f"sb_{path}_applies_per_s": round(w.n_outer * w.n_cg / t_sb, 1),
                    f"sb_{path}_rel_err_to_phantom": round(err, 4)})
    # algorithmic bytes of one fused apply: the stored coefficients once, the
    # image in and out, and the grid passes (two M x M complex grids written
    # and read by the transforms and the stencil)
    grid_bytes = 16 * fo.grid * fo.grid
    fused_alg = fo.info["fused_bytes"] + 2 * 8 * op.nn + 6 * grid_bytes
    res["fused_normal_gbs"] = round(fused_alg / (res["fused_normal_us"] * 1e-6) / 1e9, 1)
    print(f"# Fourier (m_sp 6, grid {fo.grid}, {fo.P} points): build {build_s:.2f} s, "
          f"B B^* {fo.info['fused_bytes'] / 1e9:.2f} GB; normal fused {res['fused_normal_us']:.0f} us, "
          f"NUFFT {res['nufft_normal_us']:.0f} us (4 images: {res['fused_normal_batch4_us_per_image']:.0f} and "
          f"{res['nufft_normal_batch4_us_per_image']:.0f} us per image); split Bregman fused "
          f"{res['sb_fused_ms_per_recon']:.1f} ms, "
          f"NUFFT {res['sb_nufft_ms_per_recon']:.1f} ms, error to phantom "
          f"{res['sb_fused_rel_err_to_phantom']:.4f}", file=sys.stderr, flush=True)
    return res


def bench_large(sct, W, torch, dev, vdt, t, verify=True):
    """The large under-resolved workload: 2048 x 2048, 90 angles, 2897 bins
    (4.8e8 nonzeros), split Bregman 30 outer x 10 CG on a random-ellipse
    phantom; the normal operator alone and whole reconstructions."""
    w = W.WORKLOADS["large_2048_f32"]
    from paper_1705_07497_amd import autotune
    # the layout: the library default (line-banded forward, 16 rays of one
    # angle) or a layout stored by the symmetries of the square (the 90
    # angles are closed under the maps, 2048 is a multiple of 8), each with
    # its launch settings tuned, whichever applies the normal operator faster
    x0 = torch.randn((1, w.n * w.n), dtype=vdt, device=dev)
    o0 = torch.empty_like(x0)
    op, t_best, by_layout = None, None, {}
    for bw, ang, cmp, sym in ((16, 1, False, False), (64, 2, True, True), (32, 2, True, True),
                              (32, 2, False, True)):
        cand = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                           device=dev, tuning="default", bundle=bw, bundle_angles=ang, compact=cmp,
                           symmetric=sym)
        autotune.autotune(cand, batch=1, save=False)
        tc = t(lambda: cand.normal(x0, w.alpha, w.lam, out=o0), 10)
        by_layout[f"{bw}x{ang}{'c' if cmp else ''}{'s' if sym else ''}"] = round(tc * 1e3, 3)
        if t_best is None or tc < t_best:
            op, t_best = cand, tc
        else:
            del cand
        torch.cuda.empty_cache()
    del x0, o0
    mu_np, eps_np = W.phantom_and_noise(w.n, w.n_ellipses, op.rows, seed=0)
    mu = torch.as_tensor(mu_np, dtype=vdt, device=dev).reshape(1, -1)
    y = op.fwd(mu)
    f = (y + w.noise * torch.sqrt(torch.mean(y ** 2)).item()
         * torch.as_tensor(eps_np, dtype=vdt, device=dev)).contiguous()
    out = torch.empty_like(mu)
    t_normal = t(lambda: op.normal(mu, w.alpha, w.lam, out=out), 20)
    t_sb = t(lambda: op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg), 2)
    u, _ = op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg)
    err = float(torch.linalg.vector_norm(u.reshape(-1) - mu.reshape(-1))
                / torch.linalg.vector_norm(mu))
    nnz = op.info.nnz
    bytes_normal = 2 * 8 * nnz + 4 * (op.rows + 1) + 4 * (op.nn + 1) + 8 * (3 * op.nn + 2 * op.rows)
    print(f"# large 2048x2048/90 angles: layout {op.bundle}x{op.bundle_angles}"
          f"{' compact' if op.compact else ''}{' symmetric' if op.symmetric else ''} "
          f"(normal ms by layout {by_layout}): normal {t_normal * 1e3:.3f} ms, split Bregman "
          f"{t_sb * 1e3:.1f} ms", file=sys.stderr, flush=True)
    out_d = {"n": w.n, "angles": w.n_angles, "bins": w.n_bins, "nnz": nnz, "bundle": op.bundle,
             "bundle_angles": op.bundle_angles, "fwd_compact": op.compact, "fwd_symmetric": op.symmetric,
             "adj_symmetric": op.adj_symmetric, "tuning": dict(op.tuning),
             "normal_ms_by_layout": by_layout,
             "normal_apply_ms": round(t_normal * 1e3, 3),
             "normal_apply_gbs": round(bytes_normal / t_normal / 1e9, 1),
             "sb_ms": round(t_sb * 1e3, 1), "sb_applies": w.n_outer * w.n_cg,
             "recon_per_s": round(1.0 / t_sb, 3), "rel_err_to_phantom": round(err, 4)}
    if verify:
        # the reconstruction checked against the FP64 oracle, from data the
        # oracle makes itself (its own forward of the phantom plus the same
        # noise draw: no oracle input comes from the GPU); 30 outer iterations
        # run as three resumed runs of 10, bitwise one run
        import oracle
        t0 = time.perf_counter()
        ref = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
        y_ref = ref.fwd(mu_np)
        fr = y_ref + w.noise * np.sqrt(np.mean(y_ref ** 2)) * eps_np
        u_chk, _ = op.sb(torch.as_tensor(fr, dtype=vdt, device=dev).reshape(1, -1), w.alpha, w.lam,
                         w.n_outer, w.n_cg)
        ug = u_chk.double().cpu().numpy().reshape(-1)
    del op
    torch.cuda.empty_cache()
    if verify:
        uo, st = None, None
        for _ in range(w.n_outer // 10):
            uo, _, _, _, st = ref.sb(fr, w.alpha, w.lam, 10, w.n_cg, u0=uo, state=st)
            print("# large: oracle split Bregman, 10 more outer iterations", file=sys.stderr, flush=True)
        out_d["sb_rel_l2_vs_oracle"] = float(np.linalg.norm(ug - uo) / np.linalg.norm(uo))
        out_d["oracle_s"] = round(time.perf_counter() - t0, 1)
        print(f"# large: split Bregman rel L2 vs FP64 oracle {out_d['sb_rel_l2_vs_oracle']:.3e}",
              file=sys.stderr, flush=True)
        del ref
    return out_d


def profile_volume(sct, W, torch, dev, bundle):
    """Kernel sequence of the 64-slice 1024^2 volume (FP32 kind, as the volume
    leg times it) for rocprofv3: the fused normal operator over all 64 slices
    with 16-image chunks, first gathering and staging per image, then from
    pixel-major chunk copies (fwd_layout = adj_layout = 1), then single-slice
    applies."""
    w = W.WORKLOADS["volume_64x1024_f32"]
    op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=torch.float32,
                     device=dev, tuning="default", bundle=bundle)
    X = torch.randn((w.batch, op.nn), dtype=torch.float32, device=dev)
    O = torch.empty_like(X)
    for lay in (0, 1):
        op.tuning = {"fwd_rhs": 16, "adj_rhs": 16, "fwd_layout": lay, "adj_layout": lay, "fwd_lines": 0}
        for _ in range(3):
            op.normal(X, w.alpha, w.lam, out=O)
        torch.cuda.synchronize()
        print(f"# volume: 3 fused applies, 16-image chunks, layout {lay}", file=sys.stderr, flush=True)
    op.tuning = {"fwd_rhs": 1, "adj_rhs": 1, "fwd_layout": 0, "adj_layout": 0}
    for b in range(4):
        op.normal(X[b:b + 1], w.alpha, w.lam, out=O[b:b + 1])
    torch.cuda.synchronize()
    print("# profile sequence done (volume)", file=sys.stderr, flush=True)


def bench_autograd(op, w, torch, dev, vdt, t, op1=None):
    """Loss and gradient through 10 unrolled CG iterations checkpointed every 5
    (forward 10 applies, reverse 10 replayed + 10 adjoint applies), the 16
    images fused against one image at a time, on the same operator and on
    op1 (the best single-image operator) when given."""
    from paper_1705_07497_amd import autograd as AG
    ta = w.extra["tau"] * w.alpha
    B, ck = w.batch, w.extra["ckpt"]
    M = torch.randn((B, op.nn), dtype=vdt, device=dev, requires_grad=True)
    F = torch.randn((B, op.rows), dtype=vdt, device=dev, requires_grad=True)
    singles = [(M[b:b + 1].detach().clone().requires_grad_(True),
                F[b:b + 1].detach().clone().requires_grad_(True)) for b in range(B)]

    def fused():
        AG.loss_unrolled(op, M, F, ta, w.n_cg, ck).sum().backward()

    def looped(o):
        def run():
            for m, f in singles:
                AG.loss_unrolled(o, m, f, ta, w.n_cg, ck).sum().backward()
        return run

    tf, tl = t(fused, 3), t(looped(op), 1)
    res = {"batch": B, "cg_iterations": w.n_cg, "ckpt": ck, "fused_ms": round(tf * 1e3, 3),
           "per_image_loop_ms": round(tl * 1e3, 3), "speedup": round(tl / tf, 2),
           "image_grads_per_s": round(B / tf, 1)}
    msg = f"# autograd {w.name}: fused {tf * 1e3:.2f} ms vs loop {tl * 1e3:.2f} ms ({tl / tf:.2f}x)"
    if op1 is not None:
        tlb = t(looped(op1), 1)
        res["per_image_loop_best_ms"] = round(tlb * 1e3, 3)
        res["speedup_vs_best_loop"] = round(tlb / tf, 2)
        msg += f", loop on the best single-image operator {tlb * 1e3:.2f} ms ({tlb / tf:.2f}x)"
    print(msg, file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (got --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1705_07497_amd as sct

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    w = W.WORKLOADS[WORKLOAD]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.profile_volume:
        profile_volume(sct, W, torch, dev, args.bundle)
        return
    t0 = time.perf_counter()
    vdt = torch.float64
    op_def = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                         device=dev, tuning="default")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    print(f"# built operator: nnz={op_def.info.nnz} rows={op_def.rows} in {build_s:.2f} s",
          file=sys.stderr, flush=True)
    # the autotuned operator the timed steps run: the forward layout stored by
    # the symmetries of the square (the measured angles in [0, pi/4] serve
    # their mirror and transpose partners), with both lengths per ray and line
    # or compact (the second from the ray's chord), and its bundle layout
    # (rays and angles per bundle) chosen by the normal operator's time, then
    # the launch settings timed
    from paper_1705_07497_amd import autotune
    if args.profile or args.profile_fourier or args.profile_multi:
        op = op_def
        tuning_info = None
    else:
        t0 = time.perf_counter()
        # both storages of the second length: with a quarter of the slots
        # streamed, deriving it can cost more than loading it
        chs = {cmp: autotune.choose_bundle(w.n, w.n_angles, w.n_bins, w.mask, torch.float32, vdt, dev, batch=1,
                                           save=False, compact=cmp, symmetric=True) for cmp in (False, True)}
        cmp = min(chs, key=lambda c: min(chs[c]["normal_s"].values()))
        ch = chs[cmp]
        op = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt,
                         device=dev, tuning="default", bundle=ch["bundle"], bundle_angles=ch["angles"],
                         compact=cmp, symmetric=True)
        autotune.autotune(op, batch=1, save=False)
        tuning_info = {"bundle": op.bundle, "bundle_angles": op.bundle_angles, "fwd_compact": op.compact,
                       "fwd_symmetric": op.symmetric,
                       **op.tuning,
                       "tune_s": round(time.perf_counter() - t0, 2),
                       "normal_us_by_bundle": {("compact " if c else "") + str(k): round(v * 1e6, 1)
                                               for c in chs for k, v in chs[c]["normal_s"].items()}}
        print(f"# autotuned: bundle {op.bundle}x{op.bundle_angles}{' compact' if op.compact else ''}"
              f"{' symmetric' if op.symmetric else ''}, "
              f"{op.tuning}", file=sys.stderr, flush=True)

    mu_np, eps_np = W.phantom_and_noise(w.n, w.n_ellipses, op.rows, seed=0)
    mu = torch.as_tensor(mu_np, dtype=vdt, device=dev).reshape(1, -1)
    y_clean = op.fwd(mu)
    sigma = w.noise * torch.sqrt(torch.mean(y_clean.double() ** 2)).item()
    f = (y_clean + sigma * torch.as_tensor(eps_np, dtype=vdt, device=dev)).contiguous()

    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    # warmup
    x = torch.randn((1, op.nn), dtype=vdt, device=dev)
    out = torch.empty_like(x)
    ysb = torch.empty((1, op.rows), dtype=vdt, device=dev)
    xT = x.reshape(w.n, w.n).t().contiguous().reshape(1, -1)
    if args.profile_fourier:
        bench_fourier(sct, op, w, mu, torch, timed, profile=True)
        print("# profile sequence done (Fourier normal operator, fused and NUFFT; k_stream_copy over "
              "1073741824 bytes)", file=sys.stderr,
              flush=True)
        return
    if args.profile_multi:
        bench_mixed_batch(sct, W, torch, dev, vdt, lambda fn, reps: event_time(torch, fn, 1))
        print("# profile sequence done (mixed batch)", file=sys.stderr, flush=True)
        return
    if args.profile:
        # the forward kernel of each bundle layout (the benchmark times the
        # layout choose_bundle picks) at 2 and 4 waves per bundle, 100
        # launches each, layouts in the order of PROFILE_LAYOUTS (layouts of
        # one width and wave count share a kernel name and are told apart by
        # that order; the adjoint stored by symmetry, 100 launches per tile and
        # 100 per tile orbit, after the forwards of the symmetric layout with
        # both lengths), then the
        # adjoint, the normal operator and CG of the default operator
        for bw, ang, cmp, sym in PROFILE_LAYOUTS:
            same = (bw, ang, cmp, sym) == (op.bundle, op.bundle_angles, int(op.compact), int(op.symmetric))
            op_b = op if same else sct.RadonOp(
                w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, vec_dtype=vdt, device=dev,
                tuning="default", bundle=bw, bundle_angles=ang, compact=bool(cmp), symmetric=bool(sym))
            for waves in (2, 4):
                op_b.tuning = {"fwd_waves": waves}
                for _ in range(100):
                    op_b.fwd_xt(x, xT, out=ysb)
            if sym and not cmp:
                # the adjoint stored by symmetry (the same pixel-group layout
                # for every forward layout): one workgroup per tile
                # (k_adj1_sym), then per tile orbit (k_adj1_orb)
                for al in (0, 1):
                    op_b.tuning = {"adj_layout": al}
                    for _ in range(100):
                        op_b.adj(ysb, out=out)
                op_b.tuning = {"adj_layout": 0}
            op_b.tuning = {"fwd_waves": 2}
            torch.cuda.synchronize()
            del op_b
        for _ in range(100):
            op.adj(ysb, out=out)
        for _ in range(20):
            op.normal(x, w.alpha, w.lam, out=out)
        op.cg(x, w.alpha, w.lam, n_iter=20)
        # counter calibration: the project's stream kernels over 1 GiB, 5 times each
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        part = torch.empty(4096, dtype=torch.int32, device=dev)
        for _ in range(5):
            sct.bandwidth_probe(sct.PROBE_COPY, src, dst)
        for _ in range(5):
            sct.bandwidth_probe(sct.PROBE_READ, src, part)
        torch.cuda.synchronize()
        print("# profile sequence done (k_stream_copy and k_stream_read over 1073741824 bytes)",
              file=sys.stderr, flush=True)
        return
    for _ in range(10):
        op.normal(x, w.alpha, w.lam, out=out)
    for _ in range(args.warmup):
        op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg)
    torch.cuda.synchronize()

    # standalone kernels
    t_normal = timed(lambda: op.normal(x, w.alpha, w.lam, out=out), args.applies)
    t_fwd = timed(lambda: op.fwd_xt(x, xT, out=ysb), args.applies)
    t_adj = timed(lambda: op.adj(ysb, out=out), args.applies)
    print(f"# normal {t_normal / args.applies * 1e6:.1f} us, fwd {t_fwd / args.applies * 1e6:.1f} us, "
          f"adj {t_adj / args.applies * 1e6:.1f} us", file=sys.stderr, flush=True)

    x_def_out = torch.empty_like(x)
    t_normal_def = timed(lambda: op_def.normal(x, w.alpha, w.lam, out=x_def_out), args.applies)
    del op_def
    ceiling = bandwidth_ceiling(sct, torch, dev)
    print(f"# stream ceiling: copy {ceiling['copy_gbs']:.0f} GB/s, read {ceiling['read_gbs']:.0f} GB/s",
          file=sys.stderr, flush=True)

    # timed split-Bregman reconstructions (the step)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        u, info = op.sb(f, w.alpha, w.lam, w.n_outer, w.n_cg)
    e1.record(stream)
    torch.cuda.synchronize()
    t_sb_eager = e0.elapsed_time(e1) / 1e3
    # the same reconstruction captured once as a HIP graph (one launch per
    # reconstruction, no host work between its ~4,000 kernels); it must equal
    # the eager result bitwise
    sbg = op.sb_graph(f, w.alpha, w.lam, w.n_outer, w.n_cg)
    for _ in range(args.warmup):
        sbg.launch()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        sbg.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    t_sb_graph = e0.elapsed_time(e1) / 1e3
    if not torch.equal(sbg.mu, u):
        raise RuntimeError("the captured split-Bregman graph differs from the eager solve")
    t_sb = min(t_sb_eager, t_sb_graph)
    applies_per_recon = w.n_outer * w.n_cg
    recon_per_s = args.steps / t_sb
    value = applies_per_recon * recon_per_s
    print(f"# split Bregman: eager {t_sb_eager / args.steps * 1e3:.2f} ms, graph "
          f"{t_sb_graph / args.steps * 1e3:.2f} ms per reconstruction", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (algorithmic CSR bytes: 4 B FP32 value + 4 B
    # index per nonzero, int32 row pointers, FP64 vectors read and written once)
    nnz, rows, nn = op.info.nnz, op.rows, op.nn
    vb = 8
    bytes_fwd = 8 * nnz + 4 * (rows + 1) + vb * nn + vb * rows
    bytes_adj = 8 * nnz + 4 * (nn + 1) + vb * rows + vb * nn
    avg_fwd, avg_adj = t_fwd / args.applies, t_adj / args.applies
    if avg_adj >= avg_fwd:
        kname = ("k_adj_orb" if op.tuning["adj_layout"] == 1 else "k_adj_sym") if op.adj_symmetric else "k_adj"
        kbytes, kavg = bytes_adj, avg_adj
    else:
        kname, kbytes, kavg = "k_fwd", bytes_fwd, avg_fwd
    achieved = kbytes / kavg / 1e9
    normal_bytes = bytes_fwd + bytes_adj
    if kname == "k_fwd":
        traffic = traffic_from_profile(kname, op.bundle, op.bundle_angles, op.tuning["fwd_waves"], op.compact,
                                       op.symmetric)
    else:
        traffic = traffic_from_profile(kname)
    # the kernel's own name (the traffic records are keyed by product and layout)
    kernel_name = {"k_fwd": "k_fwd_sym" if op.symmetric else "k_fwd",
                   "k_adj": "k_adj1", "k_adj_sym": "k_adj1_sym", "k_adj_orb": "k_adj1_orb"}[kname]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_name, "avg_us": round(kavg * 1e6, 2), "algorithmic_bytes": kbytes,
                "ceiling_gbs": ceiling["read_gbs"],
                "frac_of_ceiling": round(achieved / ceiling["read_gbs"], 4), "ceiling": ceiling}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "normal applies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_sb / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "matrix_storage": "f32",
        "data": "synthetic",
        "config": {"workload": "split-Bregman TV, 512x512 FP32 ellipse phantom, 180 of 360 angles, "
                               "725 bins, 50 outer x 20 CG", "n": w.n, "angles": w.n_angles,
                   "measured_angles": w.n_meas, "bins": w.n_bins, "n_outer": w.n_outer,
                   "n_cg": w.n_cg, "nnz": nnz, "batch": 1},
        "recon_per_s": round(recon_per_s, 3),
        "sb_eager_ms": round(t_sb_eager / args.steps * 1e3, 3),
        "sb_graph_ms": round(t_sb_graph / args.steps * 1e3, 3),
        "normal_apply_per_s": round(args.applies / t_normal, 1),
        "normal_apply_gbs": round(normal_bytes / (t_normal / args.applies) / 1e9, 1),
        "fwd_us": round(avg_fwd * 1e6, 2), "adj_us": round(avg_adj * 1e6, 2),
        "build_s": round(build_s, 3),
        "tuning": tuning_info,
        "normal_apply_default_per_s": round(args.applies / t_normal_def, 1),
        "roofline": roofline,
    }

    # the same normal operator in the pure FP32 kind (FP32 vectors too): its
    # split Bregman drifts from exact arithmetic by ~1e-2, so it is a
    # throughput figure only (the timed operator's bundle layout, launch
    # settings tuned for this kind)
    op32 = sct.RadonOp(w.n, w.n_angles, w.n_bins, w.mask, dtype=torch.float32, device=dev, tuning="default",
                       bundle=op.bundle, bundle_angles=op.bundle_angles, compact=op.compact,
                       symmetric=op.symmetric)
    if tuning_info is not None:
        autotune.autotune(op32, batch=1, save=False)
    x32 = x.float()
    out32 = torch.empty_like(x32)
    for _ in range(10):
        op32.normal(x32, w.alpha, w.lam, out=out32)
    t32 = timed(lambda: op32.normal(x32, w.alpha, w.lam, out=out32), args.applies) / args.applies
    bytes32 = 2 * 8 * nnz + 4 * (rows + 1) + 4 * (nn + 1) + 4 * (2 * nn + 2 * rows)
    result["normal_apply_f32_kind"] = {"us": round(t32 * 1e6, 1), "per_s": round(1.0 / t32, 1),
                                       "gbs": round(bytes32 / t32 / 1e9, 1),
                                       "frac": round(bytes32 / t32 / 1e9 / HBM_PEAK_GBS, 4),
                                       "bundle": op32.bundle, "bundle_angles": op32.bundle_angles,
                                       "fwd_compact": op32.compact, "fwd_symmetric": op32.symmetric,
                                       "tuning": op32.tuning}
    print(f"# normal operator, FP32 kind: {t32 * 1e6:.1f} us, {bytes32 / t32 / 1e9:.0f} GB/s",
          file=sys.stderr, flush=True)
    del op32

    result["surrogate"] = bench_surrogate(sct, op, w, f, mu, u, torch, timed, stream)
    result["primal_dual"] = bench_pd(op, w, f, mu, torch, timed)
    result["fourier"] = bench_fourier(sct, op, w, mu, torch, timed)

    if not args.no_batched:
        result["batched"] = bench_batched(sct, W, torch, dev, vdt, not args.no_verify)

    if not args.no_verify or not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
        oracle_build_s = time.perf_counter() - t0
        if not args.no_cpu:
            xr = np.random.default_rng(0).standard_normal(op.nn)
            ref.normal(xr, w.alpha, w.lam)
            t0 = time.perf_counter()
            ref.normal(xr, w.alpha, w.lam)
            one = time.perf_counter() - t0
            reps = args.cpu_applies or max(3, min(5000, int(15.0 / max(one, 1e-4))))
            t0 = time.perf_counter()
            for _ in range(reps):
                ref.normal(xr, w.alpha, w.lam)
            tc = time.perf_counter() - t0
            cores = oracle.set_threads()
            result["cpu_baseline"] = {
                "value": round(reps / tc, 2), "unit": "normal applies/s", "cores": cores,
                "kind": "oracle",
                "sample": f"{reps} FP64 normal applies of the same 512x512 / 180-angle operator "
                          f"({tc:.1f} s); oracle CSR build {oracle_build_s:.1f} s not included",
                **host_cpu(),
            }
            print(f"# cpu oracle: {reps / tc:.2f} applies/s on {cores} threads", file=sys.stderr,
                  flush=True)
            # the same on one thread, a ~5 s sample
            oracle.set_threads(1)
            t0 = time.perf_counter()
            ref.normal(xr, w.alpha, w.lam)
            one1 = time.perf_counter() - t0
            reps1 = max(2, min(500, int(5.0 / max(one1, 1e-4))))
            t0 = time.perf_counter()
            for _ in range(reps1):
                ref.normal(xr, w.alpha, w.lam)
            tc1 = time.perf_counter() - t0
            oracle.set_threads(cores)
            result["cpu_baseline_1thread"] = {
                "value": round(reps1 / tc1, 2), "unit": "normal applies/s", "cores": 1, "kind": "oracle",
                "sample": f"{reps1} FP64 normal applies of the same operator ({tc1:.1f} s)"}
            print(f"# cpu oracle: {reps1 / tc1:.2f} applies/s on 1 thread", file=sys.stderr, flush=True)
        if not args.no_verify:
            # the reconstruction checked against the FP64 oracle, from data
            # the oracle makes itself (its own forward of the phantom plus the
            # same noise draw: no oracle input comes from the GPU), solved once
            # more by the timed operator
            t0 = time.perf_counter()
            y_ref = ref.fwd(mu_np)
            f_ref = y_ref + w.noise * np.sqrt(np.mean(y_ref ** 2)) * eps_np
            uo = ref.sb(f_ref, w.alpha, w.lam, w.n_outer, w.n_cg)[0]
            u_chk, _ = op.sb(torch.as_tensor(f_ref, dtype=vdt, device=dev).reshape(1, -1), w.alpha, w.lam,
                             w.n_outer, w.n_cg)
            ug = u_chk.double().cpu().numpy().reshape(-1)
            err = float(np.linalg.norm(ug - uo) / np.linalg.norm(uo))
            result["sb_rel_l2_vs_oracle"] = err
            result["oracle_sb_s"] = round(time.perf_counter() - t0, 2)
            print(f"# reconstruction rel L2 vs FP64 oracle: {err:.3e}", file=sys.stderr, flush=True)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
