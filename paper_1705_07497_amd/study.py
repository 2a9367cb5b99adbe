"""Convergence-to-tolerance study of split Bregman (the protocol of Section 4,
Tables 3-5) on this library's operators.

For N = 512 and 512 pi / (4 d) evenly spaced angles (d = 1, 2, 4), split
Bregman with at most 5 CG steps per Bregman update runs until the L1 norm of
an update falls below 1e-8 of the first update or 6000 updates.  For each
threshold 1e-2, 1e-4, 1e-6, 1e-8 the table lists the updates and GPU time
needed to get below it and the relative L1 error of the image at that point.
Solvers: the exact sparse operator and the surrogate T of radius 3 on the
sinogram problem, and convolution fusing (the Fourier-domain problem
eq:SBFFT through the precomputed B B^* of eq:fusedop, m_sp = 6) on the
gridded Fourier samples of the same phantom with 1% complex noise and the
data weight alpha / n_bins.

The phantom is a random-ellipse image (the workload generator's recipe), the
data carry 1% noise, and the weights are alpha = 0.01, lambda = 1 (the
reading used for the 512 x 512 workloads).  Run:
    python -m paper_1705_07497_amd.study [--max-updates 6000] [--d 1 2 4]
                                          [--solvers exact surrogate fusing]
    python -m paper_1705_07497_amd.study --table1
    python -m paper_1705_07497_amd.study --warm-start [K ...] [--d 1 2 4]
"""
from __future__ import annotations

import argparse
import math
import sys

THRESHOLDS = (1e-2, 1e-4, 1e-6, 1e-8)


def run_case(sct, W, torch, d: int, max_updates: int, surrogate_radius: int | None,
             alpha: float = 0.01, lam: float = 1.0, n_cg: int = 5, seed: int = 0,
             fourier: bool = False):
    n = 512
    na = int(round(n * math.pi / (4 * d)))
    nb = W.n_bins_for(n)
    dev = torch.device("cuda", 0)
    op = sct.RadonOp(n, na, nb, None, dtype=torch.float32, vec_dtype=torch.float64, device=dev)
    sur = sct.RadonSurrogate(op, surrogate_radius) if surrogate_radius is not None else None
    mu_np, eps = W.phantom_and_noise(n, 10, op.rows, seed=seed)
    mu = torch.as_tensor(mu_np, dtype=torch.float64, device=dev).reshape(1, -1)
    if fourier:
        # eq:SBFFT with the fused B B^* of eq:fusedop: the data are the gridded
        # Fourier samples of the phantom with 1% complex noise
        fo = sct.RadonFourier(op, 6)
        y = fo.fwd(mu)
        g = torch.Generator(device=dev).manual_seed(seed)
        noise = torch.randn(y.shape, dtype=y.dtype, device=dev, generator=g)
        f = (y + 0.01 * torch.sqrt(torch.mean(y ** 2)).item() * noise).contiguous()
        # the unscaled DFT of a projection carries n_bins times its energy
        # (Parseval), so alpha / n_bins weights the data term as alpha does in
        # the sinogram problem
        alpha_f = alpha / nb
        step = lambda k, u: fo.sb(f, alpha_f, lam, 1, n_cg, resume=k > 0, out=u, path="fused")
        label = "convolution fusing"
    else:
        y = op.fwd(mu)
        f = (y + 0.01 * torch.sqrt(torch.mean(y ** 2)).item()
             * torch.as_tensor(eps, dtype=torch.float64, device=dev)).contiguous()
        step = lambda k, u: op.sb(f, alpha, lam, 1, n_cg, resume=k > 0, out=u, ws_key=("study", d),
                                  surrogate=sur)
        label = "exact" if sur is None else f"surrogate r={surrogate_radius}"
    mu_l1 = float(mu.abs().sum())
    u = torch.empty_like(mu)
    first = None
    elapsed = 0.0
    found = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k = 0
    while k < max_updates and len(found) < len(THRESHOLDS):
        e0.record()
        _, info = step(k, u)
        e1.record()
        torch.cuda.synchronize()
        elapsed += e0.elapsed_time(e1) / 1e3
        k += 1
        upd = sct.decode_sb_info(info)[0]["upd_b"]
        if first is None:
            first = upd
        rel = upd / first if first > 0 else 0.0
        for t in THRESHOLDS:
            if t not in found and rel < t:
                err = float((u - mu).abs().sum()) / mu_l1
                found[t] = (k, elapsed, err)
    return {"d": d, "angles": na, "updates": k, "time_s": elapsed, "found": found, "solver": label}


def run_warm_start(sct, W, torch, d: int, k_sur: int, max_updates: int, radius: int = 3,
                   alpha: float = 0.01, lam: float = 1.0, n_cg: int = 5, seed: int = 0,
                   thresholds=(1e-2, 1e-4)):
    """The surrogate as a warm start for the exact solver (Section 3.2 relies
    on the outer iteration forgetting inner errors): k_sur surrogate updates,
    then exact updates from that image (fresh d and b), against exact updates
    from zero.  Update sizes are measured relative to the first update of the
    cold exact run, so both variants stop at the same absolute size."""
    n = 512
    na = int(round(n * math.pi / (4 * d)))
    nb = W.n_bins_for(n)
    dev = torch.device("cuda", 0)
    op = sct.RadonOp(n, na, nb, None, dtype=torch.float32, vec_dtype=torch.float64, device=dev)
    sur = sct.RadonSurrogate(op, radius)
    mu_np, eps = W.phantom_and_noise(n, 10, op.rows, seed=seed)
    mu = torch.as_tensor(mu_np, dtype=torch.float64, device=dev).reshape(1, -1)
    y = op.fwd(mu)
    f = (y + 0.01 * torch.sqrt(torch.mean(y ** 2)).item()
         * torch.as_tensor(eps, dtype=torch.float64, device=dev)).contiguous()
    mu_l1 = float(mu.abs().sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1) / 1e3

    def exact_until(u, warm, first, elapsed, key):
        found, k = {}, 0
        while k < max_updates and len(found) < len(thresholds):
            if k == 0 and warm:
                (_, info), dt = timed(lambda: op.sb(f, alpha, lam, 1, n_cg, mu0=u.clone(), out=u,
                                                    ws_key=key))
            else:
                (_, info), dt = timed(lambda: op.sb(f, alpha, lam, 1, n_cg, resume=k > 0, out=u,
                                                    ws_key=key))
            elapsed += dt
            k += 1
            upd = sct.decode_sb_info(info)[0]["upd_b"]
            first = upd if first is None else first
            for t in thresholds:
                if t not in found and upd / first < t:
                    found[t] = (k, elapsed, float((u - mu).abs().sum()) / mu_l1)
        return found, first, k

    u = torch.empty_like(mu)
    cold, first, _ = exact_until(u, False, None, 0.0, ("cold", d))
    u = torch.empty_like(mu)
    t_sur = 0.0
    for k in range(k_sur):
        _, dt = timed(lambda: op.sb(f, alpha, lam, 1, n_cg, resume=k > 0, out=u, ws_key=("sur", d),
                                    surrogate=sur))
        t_sur += dt
    err_sur = float((u - mu).abs().sum()) / mu_l1
    warm, _, _ = exact_until(u, True, first, t_sur, ("warm", d))
    return {"d": d, "angles": na, "k_sur": k_sur, "sur_s": t_sur, "sur_err": err_sur, "cold": cold,
            "warm": warm, "thresholds": thresholds}


def warm_table(rows) -> str:
    ts = rows[0]["thresholds"]
    out = ["| d (angles) | surrogate updates (time, L1 err) | " +
           " | ".join(f"{t:.0e}: exact alone | {t:.0e}: after surrogate" for t in ts) + " |",
           "|---|---|" + "---|---|" * len(ts)]
    for r in rows:
        cells = []
        for t in ts:
            for v in (r["cold"], r["warm"]):
                if t in v:
                    k, s, e = v[t]
                    cells.append(f"{k} upd, {s:.2f} s, err {e:.4g}")
                else:
                    cells.append("(*)")
        out.append(f"| {r['d']} ({r['angles']}) | {r['k_sur']} ({r['sur_s']:.3f} s, {r['sur_err']:.3g}) | "
                   + " | ".join(cells) + " |")
    return "\n".join(out)


def table(rows) -> str:
    out = ["| d (angles) | solver | " + " | ".join(f"{t:.0e}" for t in THRESHOLDS) + " |",
           "|---|---|" + "---|" * len(THRESHOLDS)]
    for r in rows:
        cells = []
        for t in THRESHOLDS:
            if t in r["found"]:
                k, s, e = r["found"][t]
                cells.append(f"{k} upd, {s:.2f} s, L1 err {e:.4g}")
            else:
                cells.append(f"(*) {r['updates']} upd, {r['time_s']:.2f} s")
        out.append(f"| {r['d']} ({r['angles']}) | {r['solver']} | " + " | ".join(cells) + " |")
    return "\n".join(out)


def table1(sct, W, torch, sizes=(128, 256, 512), m_sps=(2, 6, 12)) -> str:
    """Per-evaluation time of the normal operator in the configurations of
    Table 1 (N, N pi / 4 evenly spaced angles, M_sp): the Fourier-domain
    operator through the fused B B^* and through the two gridded transforms,
    and the sparse Siddon operator of the same geometry (mixed kind)."""
    dev = torch.device("cuda", 0)

    def timed(fn, reps=50):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = ["| N | angles | M_sp | fused B B^* (ms) | two transforms (ms) | sparse Siddon (ms) | B B^* GB |",
            "|---|---|---|---|---|---|---|"]
    for n in sizes:
        na = int(round(n * math.pi / 4))
        op = sct.RadonOp(n, na, W.n_bins_for(n), None, dtype=torch.float32, vec_dtype=torch.float64,
                         device=dev)
        x = torch.randn((1, op.nn), dtype=torch.float64, device=dev)
        out = torch.empty_like(x)
        t_sp = timed(lambda: op.normal(x, 1.0, 1.0, out=out))
        for m_sp in m_sps:
            fo = sct.RadonFourier(op, m_sp)
            t_f = timed(lambda: fo.normal(x, 1.0, 1.0, path="fused", out=out))
            t_u = timed(lambda: fo.normal(x, 1.0, 1.0, path="nufft", out=out))
            rows.append(f"| {n} | {na} | {m_sp} | {t_f:.3f} | {t_u:.3f} | {t_sp:.3f} | "
                        f"{fo.info['fused_bytes'] / 1e9:.2f} |")
            print(f"# table 1: n={n} m_sp={m_sp} done", file=sys.stderr, flush=True)
            del fo
            torch.cuda.empty_cache()
        del op
    return "\n".join(rows)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-updates", type=int, default=6000)
    ap.add_argument("--d", type=int, nargs="+", default=[1, 2, 4])
    ap.add_argument("--surrogate-radius", type=int, default=3)
    ap.add_argument("--solvers", nargs="+", default=["exact", "surrogate", "fusing"],
                    choices=["exact", "surrogate", "fusing"])
    ap.add_argument("--table1", action="store_true",
                    help="per-evaluation times in the configurations of Table 1 instead")
    ap.add_argument("--warm-start", type=int, nargs="*", default=None, metavar="K",
                    help="the surrogate as a warm start: K surrogate updates, then exact updates to "
                         "1e-2 and 1e-4 of the cold run's first update, against exact alone")
    args = ap.parse_args(argv)
    import torch
    import workloads as W
    import paper_1705_07497_amd as sct
    if args.table1:
        print(table1(sct, W, torch))
        return
    if args.warm_start is not None:
        rows = []
        for d in args.d:
            for k in args.warm_start or [10, 30, 100]:
                r = run_warm_start(sct, W, torch, d, k, min(args.max_updates, 3000),
                                   args.surrogate_radius)
                rows.append(r)
                print(f"# warm start d={d} k={k} done", file=sys.stderr, flush=True)
        print(warm_table(rows))
        return
    rows = []
    for d in args.d:
        cases = {"exact": (None, False), "surrogate": (args.surrogate_radius, False),
                 "fusing": (None, True)}
        for name in args.solvers:
            radius, fourier = cases[name]
            r = run_case(sct, W, torch, d, args.max_updates, radius, fourier=fourier)
            rows.append(r)
            print(f"# d={d} {r['solver']}: {r['updates']} updates, {r['time_s']:.2f} s", file=sys.stderr,
                  flush=True)
    print(table(rows))


if __name__ == "__main__":
    main()
