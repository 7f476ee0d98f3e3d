"""Benchmark: HSS compress + factor + solve of the symmetric Muller-like system on one GPU.

A step is one pass of the whole path over one boundary: proxy-method
compression (kernel blocks + IDs), factorisation (kernel blocks + LU) and one
solve, with the boundary geometry and right-hand side already in HBM.

    python bench.py [--steps K] [--warmup W] [--config 2] [--no-base] [--no-cpu]

Prints one JSON line.  Workload (default): star r = 1 + 0.3 cos 5t,
N = 32768 nodes (65536 unknowns), k = 50 / 75, leaf 128, tol 1e-10.

--config 3: a batch of 64 seeded random stars (3-8 arms, amplitude
U[0.1, 0.3], N log-uniform in [4096, 65536], k_out U[5, 80], k_in = 1.5 k_out)
solved together in one context: per-level shared launches, autotuned launch
variants, factorisation and solve replayed as HIP graphs.  Also reports the
sum of the same boundaries solved one at a time.

--config 4: star r = 1 + 0.25 cos 7t, N = 262144, k = 200 / 300, solved by
the FP64 path and by the mixed-precision path (FP32 factorisation and
sweeps, refined against the FP64 HSS product to 1e-10).

--config 6: the paper's fixed-rank schedule (k_L = 30, growth a per level)
on the five-arm star at N = 8192 ... 131072: time and factorisation flops
against N, with fitted exponents (O(N) for a < 2^(1/3)).

--config 7: the paper's speedup experiment on one GPU: kite, eps = 1 / 3,
omega = 2, fixed ranks k_L = 30, a = 1.15, 6400 ... 1638400 DOF, symmetric
one-sided form and Burton-Miller against the unscaled two-sided Base.

--config 5: the same batch with proxy circles sized by the rank predictor,
trained on the GPU from ranks the solver measures on one random star per
seed 1000-1099 (ID tolerances 1e-6 ... 1e-12); compared with the same batch
without the predictor.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_FP64_TFLOPS = 78.6
MI355X_HBM_TBS = 8.0

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs of
# this script (star5-n32768-k50-75, one step), scaled by the same counters read
# on a plain 512 MiB copy (fetch x2.0, write x1.0).  Valid only while the
# kernels' sources are the ones profiled: keyed by the SHA-256 prefixes of
# their files.  An ID launch is the blocked QR and the pivoted QR of its
# triangle (k_id_qr + k_id_sq) for many matrices, or k_cpqr for few; its
# figure is the mean over the five ID launches of a step.
MEASURED_TRAFFIC = {
    "id": {"sources": {"idqr.hip": "7e597cd35c9ff6a3", "cpqr.hip": "5a4bcc5299aacbf7"}, "bytes": 7.733e+08,
           "profile": "profiles/id_star5-n32768.md"},
    "k_lu_fused": {"sources": {"dense_body.inc": "deeda13ca7b2dbdf"}, "bytes": 7.483e+08,
                   "profile": "profiles/k_lu_fused_star5-n32768.md"},
    "k_kblock": {"sources": {"kblock.hip": "b8965c325ada25df"}, "bytes": 7.427e+07,
                 "profile": "profiles/k_kblock_star5-n32768.md"},
}


def _traffic(kernel: str, workload: str):
    import hashlib
    t = MEASURED_TRAFFIC.get(kernel)
    if t is None or workload != "star5-n32768-k50-75":
        return None
    for name, sha in t["sources"].items():
        src = os.path.join(ROOT, "paper_2609_33216_amd", "csrc", name)
        try:
            if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != sha:
                return None
        except OSError:
            return None
    return t["bytes"]


def _workload(cfg: int):
    import workloads
    if cfg == 1:
        return workloads.config1()
    if cfg == 2:
        return workloads.config2()
    if cfg == 4:
        return workloads.config4()
    raise SystemExit(f"unknown config {cfg}")


def _run_form(s, wl, form, steps, warmup, b, x, torch, root_max=0, fused=True):
    x_, dx_, ddx_ = wl.boundary()
    s.assemble(x_, dx_, ddx_, wl.k0, wl.k1, wl.eps0, wl.eps1, leaf=wl.leaf, tol=wl.tol, form=form,
               n_proxy=wl.n_proxy if wl.n_proxy > 0 else 64, proxy_ratio=wl.proxy_ratio, root_max=root_max)
    s.rhs_plane_wave_device(wl.angle, b.data_ptr())
    def factor_and_solve():
        # one call (the solve's sweep up the levels beside the top-level LU),
        # or the two calls one after the other
        if fused:
            s.factor_solve_device(b.data_ptr(), x.data_ptr())
        else:
            s.factor()
            s.solve_device(b.data_ptr(), x.data_ptr())

    for _ in range(warmup):
        s.compress()
        factor_and_solve()
    torch.cuda.synchronize()
    per = []
    phases = {"t_compress": [], "t_factor": [], "t_solve": []}
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        s.compress()
        factor_and_solve()
        torch.cuda.synchronize()
        per.append(time.perf_counter() - ts)
        st = s.stats()
        for k in phases:
            phases[k].append(st[k])
    t1 = time.perf_counter()
    st = s.stats()
    # phase times: the mean over the timed steps (the last step's kernel timings stay in st)
    for k, v in phases.items():
        st[k] = sum(v) / max(len(v), 1)
    return (t1 - t0) / max(steps, 1), st, per


def _cpu_baseline(wl):
    """The oracle on the host: dense assembly rows and dense LU on samples,
    scaled to one dense solve of the full 2N system."""
    import numpy as np
    from oracle import dense, geometry, kernels
    from oracle.kernels import Medium, PointSet
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    x, dx, ddx = wl.boundary()
    g = geometry.discretize(x, dx, ddx)
    med = Medium(wl.k0, wl.k1, wl.eps0, wl.eps1)
    n = g.n
    rows = 256
    ps = PointSet.boundary(g)
    t0 = time.perf_counter()
    kernels.muller_blocks(ps.take(np.arange(rows)), ps, med, True)
    t_rows = time.perf_counter() - t0
    t_assembly = t_rows * n / rows  # all 2N x 2N entries (4 per node pair)
    m = 3072
    rng = np.random.default_rng(0)
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    bb = rng.standard_normal(m) + 0j
    t0 = time.perf_counter()
    dense.solve_dense(A, bb)
    t_lu = time.perf_counter() - t0
    t_lu_full = t_lu * (2 * n / m) ** 3
    total = t_assembly + t_lu_full
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": round(total, 3), "unit": "s/solve", "cores": int(cores), "kind": "oracle",
        "extrapolated": True, "cpu_model": model,
        "sample": (f"extrapolated from samples: oracle dense assembly of {rows} of {n} node rows "
                   f"(x{n / rows:.0f}) plus scipy LU of a {m}x{m} complex system (x{(2 * n / m) ** 3:.0f} "
                   f"by n^3) to the dense {2 * n}-unknown solve; assembly {t_assembly:.1f} s, "
                   f"LU {t_lu_full:.1f} s"),
        "gentries_per_s": round(4.0 * rows * n / t_rows / 1e9, 5),
    }


def _run_batch(args):
    import numpy as np
    import torch
    import workloads
    from paper_2609_33216_amd import binding

    wls = workloads.config3_batch(seed=3, count=64)
    ntot = sum(w.n for w in wls)
    dev = torch.device("cuda:0")
    b = torch.zeros(2 * ntot, dtype=torch.complex128, device=dev)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    s = binding.Solver(0)
    s.configure(graphs=not args.no_graphs, autotune=True)
    s.assemble_batch([w.boundary() for w in wls], [(w.k0, w.k1, w.eps0, w.eps1) for w in wls], leaf=128,
                     tol=1e-10, form=binding.MULLER_SYM)
    s.rhs_plane_wave_batch_device([w.angle for w in wls], b.data_ptr())
    print(f"batch: {len(wls)} boundaries, {ntot} nodes; warmup", file=sys.stderr, flush=True)
    for _ in range(max(args.warmup, 2)):  # tuning, then capture
        s.compress()
        s.factor()
        s.solve_device(b.data_ptr(), x.data_ptr())
    torch.cuda.synchronize()
    per = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        s.compress()
        s.factor()
        s.solve_device(b.data_ptr(), x.data_ptr())
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t0)
    st = s.stats()
    t_batch = sum(per) / len(per)
    print(f"batch: {1e3 * t_batch:.1f} ms per batch solve; residual", file=sys.stderr, flush=True)
    y = torch.zeros_like(x)
    s.lib.symhss_matvec_direct(s.h, binding.ctypes.c_void_p(x.data_ptr()), binding.ctypes.c_void_p(y.data_ptr()),
                               binding.DEVICE_PTRS)
    torch.cuda.synchronize()
    res = []
    o = 0
    for w in wls:
        r = torch.linalg.vector_norm(y[o:o + 2 * w.n] - b[o:o + 2 * w.n]) / torch.linalg.vector_norm(b[o:o + 2 * w.n])
        res.append(float(r))
        o += 2 * w.n
    # the same boundaries one at a time (same options, one warm-up each)
    t_single = 0.0
    ent_single = 0
    if not args.no_single:
        for i, w in enumerate(wls):
            s1 = binding.Solver(0)
            s1.configure(graphs=not args.no_graphs, autotune=True)
            xw, dxw, ddxw = w.boundary()
            s1.assemble(xw, dxw, ddxw, w.k0, w.k1, w.eps0, w.eps1, leaf=128, tol=1e-10)
            b1 = torch.zeros(2 * w.n, dtype=torch.complex128, device=dev)
            x1 = torch.zeros_like(b1)
            torch.cuda.synchronize()
            s1.rhs_plane_wave_device(w.angle, b1.data_ptr())
            for _ in range(2):
                s1.compress()
                s1.factor()
                s1.solve_device(b1.data_ptr(), x1.data_ptr())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1.compress()
            s1.factor()
            s1.solve_device(b1.data_ptr(), x1.data_ptr())
            torch.cuda.synchronize()
            t_single += time.perf_counter() - t0
            s1st = s1.stats()
            ent_single += s1st["entries_compress"] + s1st["entries_factor"]
            s1.close()
    ent = st["entries_compress"] + st["entries_factor"]
    out = {
        "metric": "HSS compress+factor s/solve & Gentries/s, sym vs nonsym, at 1e-8 rel err",
        "value": round(t_batch, 6),
        "unit": "s/solve (whole 64-boundary batch)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t_batch, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "batch64-stars-seed3", "boundaries": len(wls), "n_nodes_total": ntot,
                   "n_range": [min(w.n for w in wls), max(w.n for w in wls)], "leaf": 128, "tol": 1e-10,
                   "form": "symmetric one-sided ID", "graphs": not args.no_graphs, "autotune": True,
                   "parallelism": "1 GPU"},
        "boundaries_per_s": round(len(wls) / t_batch, 3),
        "step_times": [round(v, 6) for v in per],
        "t_compress": round(st["t_compress"], 6), "t_factor": round(st["t_factor"], 6),
        "t_compress_host": round(st["t_compress"] - st["t_compress_wait"], 6),
        "host_seconds": {k: round(st["t_host_" + k], 6) for k in ("plan", "ids", "post", "factor")},
        "kernel_seconds": {"kblock": round(st["t_kblock_compress"] + st["t_kblock_factor"], 6),
                           "id": round(st["t_id"], 6), "lu": round(st["t_lu"], 6)},
        "t_solve": round(st["t_solve"], 6),
        "entries": int(ent),
        "gentries_per_s_whole_step": round(ent / t_batch / 1e9, 3),
        "graph_replays": st["graph_replays"], "tuned_buckets": st["tuned_buckets"],
        "residual_fp64_direct_max": max(res),
        "unbatched_sum_s": round(t_single, 6) if not args.no_single else None,
        "speedup_batched_vs_unbatched": round(t_single / t_batch, 3) if not args.no_single else None,
    }
    print(json.dumps(out))


def _run_predictor(args):
    """Batch workload with and without predictor-sized proxy circles."""
    import torch
    import workloads
    from paper_2609_33216_amd import binding, predictor

    t0 = time.perf_counter()
    feat, rank = predictor.training_set(seeds=range(1000, 1100))
    t_data = time.perf_counter() - t0
    print(f"predictor: {len(rank)} training boxes in {t_data:.1f} s", file=sys.stderr, flush=True)
    wls = workloads.config3_batch(seed=3, count=64)
    ntot = sum(w.n for w in wls)
    dev = torch.device("cuda:0")
    b = torch.zeros(2 * ntot, dtype=torch.complex128, device=dev)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    s = binding.Solver(0)
    t0 = time.perf_counter()
    hist = s.predictor_train(feat, rank, epochs=args.epochs, batch=1024, lr=2e-3, alpha=4.0, seed=0)
    t_train = time.perf_counter() - t0
    print(f"predictor: trained {args.epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3g} -> {hist[-1]:.3g}",
          file=sys.stderr, flush=True)
    s.configure(graphs=not args.no_graphs, autotune=True)
    s.assemble_batch([w.boundary() for w in wls], [(w.k0, w.k1, w.eps0, w.eps1) for w in wls], leaf=128,
                     tol=1e-10, form=binding.MULLER_SYM)
    s.rhs_plane_wave_batch_device([w.angle for w in wls], b.data_ptr())

    def timed(use_pred):
        s.configure(predictor=use_pred, proxy_margin=args.proxy_margin)
        for _ in range(max(args.warmup, 2)):
            s.compress()
            s.factor()
            s.solve_device(b.data_ptr(), x.data_ptr())
        torch.cuda.synchronize()
        per, tc = [], []
        for _ in range(args.steps):
            t1 = time.perf_counter()
            s.compress()
            tc.append(time.perf_counter() - t1)
            s.factor()
            s.solve_device(b.data_ptr(), x.data_ptr())
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t1)
        st = s.stats()
        y = torch.zeros_like(x)
        s.lib.symhss_matvec_direct(s.h, binding.ctypes.c_void_p(x.data_ptr()),
                                   binding.ctypes.c_void_p(y.data_ptr()), binding.DEVICE_PTRS)
        torch.cuda.synchronize()
        res, o = [], 0
        for w in wls:
            res.append(float(torch.linalg.vector_norm(y[o:o + 2 * w.n] - b[o:o + 2 * w.n]) /
                             torch.linalg.vector_norm(b[o:o + 2 * w.n])))
            o += 2 * w.n
        return sum(per) / len(per), sum(tc) / len(tc), st, max(res), x.clone()

    t_base, tc_base, st_base, res_base, x_base = timed(False)
    print(f"predictor: without {1e3 * t_base:.1f} ms", file=sys.stderr, flush=True)
    t_pred, tc_pred, st_pred, res_pred, x_pred = timed(True)
    print(f"predictor: with {1e3 * t_pred:.1f} ms", file=sys.stderr, flush=True)
    diff = float(torch.linalg.vector_norm(x_pred - x_base) / torch.linalg.vector_norm(x_base))
    out = {
        "metric": "HSS compress+factor s/solve & Gentries/s, sym vs nonsym, at 1e-8 rel err",
        "value": round(t_pred, 6),
        "unit": "s/solve (whole 64-boundary batch, predictor-sized)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t_pred, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "batch64-stars-seed3+rank-predictor", "boundaries": len(wls), "n_nodes_total": ntot,
                   "train_seeds": "1000-1099", "train_tols": [1e-6, 1e-8, 1e-10, 1e-12], "leaf": 128,
                   "tol": 1e-10, "graphs": not args.no_graphs, "parallelism": "1 GPU"},
        "train_boxes": int(len(rank)), "train_data_s": round(t_data, 3), "train_s": round(t_train, 3),
        "train_epochs": args.epochs, "train_loss": [float(hist[0]), float(hist[-1])],
        "without": {"s_per_solve": round(t_base, 6), "t_compress": round(tc_base, 6),
                    "residual_fp64_direct_max": res_base, "proxy_rows": st_base["proxy_rows"],
                    "proxy_bytes": st_base["proxy_bytes"]},
        "with": {"s_per_solve": round(t_pred, 6), "t_compress": round(tc_pred, 6),
                 "residual_fp64_direct_max": res_pred, "proxy_rows": st_pred["proxy_rows"],
                 "proxy_bytes": st_pred["proxy_bytes"], "predicted_boxes": st_pred["pred_boxes"],
                 "fallbacks": st_pred["pred_fallbacks"]},
        "compress_speedup": round(tc_base / tc_pred, 3),
        "total_speedup": round(t_base / t_pred, 3),
        "fallback_rate": round(st_pred["pred_fallbacks"] / max(st_pred["pred_boxes"], 1), 4),
        "proxy_bytes_saved": st_base["proxy_bytes"] - st_pred["proxy_bytes"],
        "solution_rel_diff_with_vs_without": diff,
    }
    print(json.dumps(out))


def _run_mixed(args):
    """Star r = 1 + 0.25 cos 7t, N = 262144, k = 200 / 300: FP64 path and the
    mixed-precision path (FP32 factorisation, FP64 HSS refinement to 1e-10)."""
    import torch
    import workloads
    from paper_2609_33216_amd import binding

    wl = workloads.config4() if args.n4 is None else workloads.scaled_config(workloads.config4(), args.n4)
    n = wl.n
    dev = torch.device("cuda:0")
    b = torch.zeros(2 * n, dtype=torch.complex128, device=dev)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    s = binding.Solver(0)
    xw, dxw, ddxw = wl.boundary()
    s.assemble(xw, dxw, ddxw, wl.k0, wl.k1, wl.eps0, wl.eps1, leaf=wl.leaf, tol=wl.tol, root_max=args.root_max)
    s.rhs_plane_wave_device(wl.angle, b.data_ptr())

    def run(mixed):
        s.configure(mixed=mixed)
        per = []
        for it in range(args.warmup + args.steps):
            t0 = time.perf_counter()
            s.compress()
            t1 = time.perf_counter()
            s.factor()
            t2 = time.perf_counter()
            s.solve_device(b.data_ptr(), x.data_ptr())
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            st = s.stats()
            print(f"  {'mixed' if mixed else 'fp64'} step {it}: compress {t1 - t0:.3f} factor {t2 - t1:.3f} "
                  f"solve {t3 - t2:.3f} s; ranks {st['rank_max']} root {st['root_size']}", file=sys.stderr,
                  flush=True)
            if it >= args.warmup:
                per.append(t3 - t0)
        return sum(per) / len(per), s.stats(), x.clone()

    print(f"mixed: N={n}; FP64 path", file=sys.stderr, flush=True)
    t64, st64, x64 = run(False)
    print(f"mixed: FP64 {1e3 * t64:.1f} ms; mixed path", file=sys.stderr, flush=True)
    t32, st32, x32 = run(True)
    print(f"mixed: mixed {1e3 * t32:.1f} ms; residuals", file=sys.stderr, flush=True)
    # FP32-only iterate (one refinement step: reported as not converged)
    s.configure(refine_maxit=1)
    st1 = s.lib.symhss_solve(s.h, binding.ctypes.c_void_p(b.data_ptr()), binding.ctypes.c_void_p(x.data_ptr()), 1,
                             binding.DEVICE_PTRS)
    if st1 not in (binding.OK, binding.ENOTCONV):
        raise binding.SymhssError(st1, s.lib.symhss_last_error(s.h).decode())
    torch.cuda.synchronize()
    x1 = x.clone()
    s.configure(refine_maxit=10)

    def resid(v):
        y = torch.zeros_like(v)
        s.lib.symhss_matvec_direct(s.h, binding.ctypes.c_void_p(v.data_ptr()), binding.ctypes.c_void_p(y.data_ptr()),
                                   binding.DEVICE_PTRS)
        torch.cuda.synchronize()
        return float(torch.linalg.vector_norm(y - b) / torch.linalg.vector_norm(b))

    def rdiff(a, c):
        return float(torch.linalg.vector_norm(a - c) / torch.linalg.vector_norm(c))

    r64 = resid(x64) if not args.no_residual else None
    r32 = resid(x32) if not args.no_residual else None
    out = {
        "metric": "HSS compress+factor s/solve & Gentries/s, sym vs nonsym, at 1e-8 rel err",
        "value": round(t32, 6),
        "unit": "s/solve (mixed precision, refined to 1e-10)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t32, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128", "data": "synthetic",
        "config": {"workload": wl.name, "n_nodes": n, "unknowns": 2 * n, "k_out": wl.k0, "k_in": wl.k1,
                   "leaf": wl.leaf, "tol": wl.tol, "form": "symmetric one-sided ID", "parallelism": "1 GPU"},
        "fp64": {"s_per_solve": round(t64, 6), "t_compress": round(st64["t_compress"], 6),
                 "t_factor": round(st64["t_factor"], 6), "t_solve": round(st64["t_solve"], 6),
                 "residual_fp64_direct": r64},
        "mixed": {"s_per_solve": round(t32, 6), "t_compress": round(st32["t_compress"], 6),
                  "t_factor": round(st32["t_factor"], 6), "t_solve": round(st32["t_solve"], 6),
                  "refine_iters": st32["refine_iters"], "hss_residual_first_fp32_solve": st32["fp32_residual"],
                  "hss_residual_refined": st32["refine_residual"], "residual_fp64_direct": r32},
        "err_fp32_only_vs_fp64_hss": rdiff(x1, x64),
        "err_refined_vs_fp64_hss": rdiff(x32, x64),
        "speedup_mixed_vs_fp64": round(t64 / t32, 3),
        "ranks_max_per_level": st32["rank_max"], "root_size": st32["root_size"],
        "device_bytes_fp64": st64["device_bytes"], "device_bytes_mixed": st32["device_bytes"],
    }
    print(json.dumps(out))


def _run_scaling(args):
    """Fixed-rank schedule k_l = a^(L - l) k_L (Section 4.3, Theorem 1): time and
    factorisation flops against N on the five-arm star, k = 50 / 75."""
    import numpy as np
    import torch
    import workloads
    from paper_2609_33216_amd import binding

    ns = [8192, 16384, 32768, 65536, 131072]
    dev = torch.device("cuda:0")
    res = {}
    for a in (1.0, 1.15, 1.3):
        rows = []
        for n in ns:
            wl = workloads.scaled_config(workloads.config2(), n)
            b = torch.zeros(2 * n, dtype=torch.complex128, device=dev)
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            s = binding.Solver(0)
            xw, dxw, ddxw = wl.boundary()
            s.assemble(xw, dxw, ddxw, wl.k0, wl.k1, wl.eps0, wl.eps1, leaf=128, tol=1e-10, root_max=-1)
            s.configure(rank_leaf=30, rank_scale=a)
            s.rhs_plane_wave_device(wl.angle, b.data_ptr())
            per = []
            for it in range(args.warmup + args.steps):
                t0 = time.perf_counter()
                s.compress()
                s.factor()
                s.solve_device(b.data_ptr(), x.data_ptr())
                torch.cuda.synchronize()
                if it >= args.warmup:
                    per.append(time.perf_counter() - t0)
            st = s.stats()
            rows.append({"n": n, "s_per_solve": round(sum(per) / len(per), 6), "t_factor": round(st["t_factor"], 6),
                         "flops_lu": st["flops_lu_batched"] + st["flops_lu_multi"], "root_size": st["root_size"]})
            print(f"scaling: a={a} N={n} {1e3 * rows[-1]['s_per_solve']:.1f} ms", file=sys.stderr, flush=True)
            s.close()
        lx = np.log([r["n"] for r in rows])
        res[str(a)] = {"runs": rows,
                       "exponent_time": round(float(np.polyfit(lx, np.log([r["s_per_solve"] for r in rows]), 1)[0]), 3),
                       "exponent_flops": round(float(np.polyfit(lx, np.log([r["flops_lu"] for r in rows]), 1)[0]), 3),
                       "theorem_exponent": 1.0 if a < 2 ** (1 / 3) else round(3 * np.log2(a), 3)}
    big = res["1.15"]["runs"][-1]
    out = {
        "metric": "HSS compress+factor s/solve & Gentries/s, sym vs nonsym, at 1e-8 rel err",
        "value": big["s_per_solve"], "unit": "s/solve (fixed ranks k_L = 30, a = 1.15, N = 131072)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * big["s_per_solve"], 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "star5-k50-75 fixed-rank sweep", "n": ns, "leaf": 128, "k_L": 30,
                   "a": [1.0, 1.15, 1.3], "parallelism": "1 GPU"},
        "scaling_by_a": res,
    }
    print(json.dumps(out))


def _run_kite(args):
    """The paper's speedup experiment on one GPU: kite, eps0 = 1, eps1 = 3, plane
    wave along x1, fixed ranks k_L = 30, a = 1.15, 6400 ... 1638400 DOF; the
    symmetric one-sided form and Burton-Miller (two-sided) against the
    unscaled two-sided Base (Table 4's three columns)."""
    import math
    import numpy as np
    import torch
    from workloads.curves import sample_curve
    from paper_2609_33216_amd import binding

    omega = 2.0
    k0, k1 = omega, omega * math.sqrt(3.0)
    dofs = [6400 * 2 ** i for i in range(9)] if args.kite_max is None else \
        [d for d in (6400 * 2 ** i for i in range(9)) if d <= args.kite_max]
    dev = torch.device("cuda:0")
    rows = []
    for dof in dofs:
        n = dof // 2
        x, dx, ddx = sample_curve("kite", n)
        b = torch.zeros(2 * n, dtype=torch.complex128, device=dev)
        xv = torch.zeros_like(b)
        torch.cuda.synchronize()
        rec = {"dof": dof}
        sols = {}
        forms = [("sym", binding.MULLER_SYM), ("base", binding.MULLER_BASE)]
        if not args.no_bm:
            forms.append(("bm", binding.BURTON_MILLER))
        for name, form in forms:
            s = binding.Solver(0)
            s.assemble(x, dx, ddx, k0, k1, 1.0, 3.0, leaf=128, tol=1e-10, form=form)
            s.configure(rank_leaf=30, rank_scale=1.15)
            s.rhs_plane_wave_device(0.0, b.data_ptr())
            per = []
            for it in range(args.warmup + args.steps):
                t0 = time.perf_counter()
                s.compress()
                s.factor()
                s.solve_device(b.data_ptr(), xv.data_ptr())
                torch.cuda.synchronize()
                if it >= args.warmup:
                    per.append(time.perf_counter() - t0)
            st = s.stats()
            rec[name] = {"s_per_solve": round(float(np.median(per)), 6), "t_compress": round(st["t_compress"], 6),
                         "t_factor": round(st["t_factor"], 6), "t_solve": round(st["t_solve"], 6),
                         "entries": int(st["entries_compress"] + st["entries_factor"])}
            sols[name] = xv.clone()
            s.close()
        rec["speedup_sym_vs_base"] = round(rec["base"]["s_per_solve"] / rec["sym"]["s_per_solve"], 3)
        rec["speedup_compress"] = round(rec["base"]["t_compress"] / rec["sym"]["t_compress"], 3)
        rec["rel_diff_sym_base"] = float(torch.linalg.vector_norm(sols["sym"] - sols["base"]) /
                                         torch.linalg.vector_norm(sols["base"]))
        if "bm" in rec:
            rec["speedup_bm_vs_base"] = round(rec["base"]["s_per_solve"] / rec["bm"]["s_per_solve"], 3)
            # Burton-Miller's hypersingular N_k0 converges at O(h): its
            # solution differs from the Muller-like one by that error
            rec["rel_diff_bm_base"] = float(torch.linalg.vector_norm(sols["bm"] - sols["base"]) /
                                            torch.linalg.vector_norm(sols["base"]))
        rows.append(rec)
        print(f"kite: DOF {dof}: sym {1e3 * rec['sym']['s_per_solve']:.1f} ms, base "
              f"{1e3 * rec['base']['s_per_solve']:.1f} ms, x{rec['speedup_sym_vs_base']}"
              + (f"; bm {1e3 * rec['bm']['s_per_solve']:.1f} ms, x{rec['speedup_bm_vs_base']}" if "bm" in rec else ""),
              file=sys.stderr, flush=True)
    mean = float(np.mean([r["speedup_sym_vs_base"] for r in rows]))
    mean_bm = float(np.mean([r["speedup_bm_vs_base"] for r in rows])) if not args.no_bm else None
    big = rows[-1]
    out = {
        "metric": "HSS compress+factor s/solve & Gentries/s, sym vs nonsym, at 1e-8 rel err",
        "value": big["sym"]["s_per_solve"], "unit": f"s/solve (kite, {big['dof']} DOF, symmetric)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * big["sym"]["s_per_solve"], 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "kite DOF sweep", "curve": "kite x = (cos t + 0.65 cos 2t - 0.65, 1.5 sin t)",
                   "omega": omega, "eps": [1.0, 3.0], "k_L": 30, "a": 1.15, "leaf": 128, "dof": dofs,
                   "parallelism": "1 GPU"},
        "runs": rows,
        "mean_speedup_sym_vs_base": round(mean, 3),
        "mean_speedup_bm_vs_base": round(mean_bm, 3) if mean_bm is not None else None,
        "paper_context": "M-sym 1.436, BM 1.234 mean over 9 sizes on one 192-core CPU node (Table 4)",
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-base", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-residual", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the untimed relative-error check against the stored dense-LU solution")
    ap.add_argument("--no-graphs", action="store_true", help="batch mode: no HIP-graph replay")
    ap.add_argument("--no-single", action="store_true", help="batch mode: skip the one-at-a-time sum")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="factor each level after compress instead of on a second stream during it")
    ap.add_argument("--epochs", type=int, default=300, help="predictor mode: training epochs")
    ap.add_argument("--proxy-margin", type=int, default=16,
                    help="predictor mode: proxy points added to the predicted rank")
    ap.add_argument("--autotune", action="store_true", help="single-boundary mode: autotuned launch variants")
    ap.add_argument("--graphs", action="store_true", help="single-boundary mode: solves replayed as HIP graphs")
    ap.add_argument("--separate-calls", action="store_true",
                    help="single-boundary mode: symhss_factor then symhss_solve instead of symhss_factor_solve")
    ap.add_argument("--n4", type=int, default=None, help="mixed mode: another N for the seven-arm star")
    ap.add_argument("--kite-max", type=int, default=None, help="kite sweep: largest DOF")
    ap.add_argument("--no-bm", action="store_true", help="kite sweep: without the Burton-Miller column")
    ap.add_argument("--root-max", type=int, default=None,
                    help="largest dense top-level system (sum of ranks); default 2048, 8192 for --config 4")
    args = ap.parse_args()
    args.root_max_given = args.root_max is not None
    if args.root_max is None:
        args.root_max = 8192 if args.config == 4 else 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this path has no multi-GPU mode); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    if args.config == 3:
        _run_batch(args)
        return
    if args.config == 5:
        _run_predictor(args)
        return
    if args.config == 4:
        _run_mixed(args)
        return
    if args.config == 6:
        _run_scaling(args)
        return
    if args.config == 7:
        _run_kite(args)
        return

    import numpy as np
    import torch
    from paper_2609_33216_amd import binding

    wl = _workload(args.config)
    n = wl.n
    dev = torch.device("cuda:0")
    b = torch.zeros(2 * n, dtype=torch.complex128, device=dev)
    x = torch.zeros(2 * n, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()  # the solver queues on its own stream
    s = binding.Solver(0)
    s.configure(pipeline=not args.no_pipeline, autotune=args.autotune, graphs=args.graphs)

    rm = args.root_max if args.root_max_given else 0
    fused = not args.separate_calls
    t_sym, st, per = _run_form(s, wl, binding.MULLER_SYM, args.steps, args.warmup, b, x, torch, rm, fused)
    resid = None
    if not args.no_residual:
        y = torch.zeros_like(x)
        torch.cuda.synchronize()
        s.lib.symhss_matvec_direct(s.h, binding.ctypes.c_void_p(x.data_ptr()), binding.ctypes.c_void_p(y.data_ptr()),
                                   binding.DEVICE_PTRS)
        torch.cuda.synchronize()
        resid = float(torch.linalg.vector_norm(y - b) / torch.linalg.vector_norm(b))

    ent = st["entries_compress"] + st["entries_factor"]
    t_kb = st["t_kblock_compress"] + st["t_kblock_factor"]
    kernels_t = {"kblock": t_kb, "id": st["t_id"], "lu": st["t_lu"]}
    out = {
        "metric": "HSS compress+factor s/solve & Gentries/s, sym vs nonsym, at 1e-8 rel err",
        "value": round(t_sym, 6),
        "unit": "s/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_sym, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wl.name, "curve": f"{wl.curve} {dict(wl.curve_params)}", "n_nodes": n,
                   "unknowns": 2 * n, "k_out": wl.k0, "k_in": wl.k1, "leaf": wl.leaf, "tol": wl.tol,
                   "form": "symmetric one-sided ID", "pipelined_factor": not args.no_pipeline,
                   "autotune": args.autotune, "graphs": args.graphs,
                   "factor_solve": not args.separate_calls, "parallelism": "1 GPU"},
        # with factor_solve, t_factor is the time to queue the top-level LU; its
        # GPU time, beside the solve's sweep up the levels, falls in t_solve
        "t_compress": round(st["t_compress"], 6),
        "t_compress_host": round(st["t_compress"] - st["t_compress_wait"], 6),
        "host_seconds": {k: round(st["t_host_" + k], 6) for k in ("plan", "ids", "post", "factor")},
        "t_factor": round(st["t_factor"], 6),
        "t_solve": round(st["t_solve"], 6),
        "step_times": [round(v, 6) for v in per],
        "entries": int(ent),
        "gentries_per_s": round(ent / t_kb / 1e9, 3) if t_kb > 0 else None,
        "kernel_seconds": {k: round(v, 6) for k, v in kernels_t.items()},
        "ranks_max_per_level": st["rank_max"],
        "root_size": st["root_size"],
        "residual_fp64_direct": resid,
    }
    # Rooflines.  achieved = algorithmic work of the timed launches / their
    # summed duration (HIP events on the solver's stream), i.e. the mean work
    # per launch over the mean launch time.  The kernel-block generator is
    # priced by the bytes of the entries it writes (16 B each) against HBM;
    # the ID and LU kernels by FP64 flops against the FP64 peak.
    rl = {}
    if t_kb > 0:
        a = st["bytes_kblock"] / t_kb / 1e9
        rl["k_kblock"] = {"bound": "hbm", "achieved": a, "peak": MI355X_HBM_TBS * 1e3, "unit": "GB/s",
                          "seconds": t_kb, "launches": st["n_kblock"]}
    for name, t, f, nl in (("id", st["t_id"], st["flops_id"], st["n_id"]),
                           ("k_lu_fused", st["t_lu_batched"], st["flops_lu_batched"], st["n_lu_batched"]),
                           ("lu_multi (several kernels)", st["t_lu_multi"], st["flops_lu_multi"], st["n_lu_multi"])):
        if t > 0:
            rl[name] = {"bound": "alu", "achieved": f / t / 1e12, "peak": MI355X_FP64_TFLOPS, "unit": "TFLOP/s",
                        "seconds": t, "launches": nl}
    for v in rl.values():
        v["frac"] = round(v["achieved"] / v["peak"], 4)
        v["achieved"] = round(v["achieved"], 3)
        v["seconds"] = round(v["seconds"], 6)
    single = [k for k in ("k_kblock", "id", "k_lu_fused") if k in rl]
    if single:
        # The batched LU when it ran: the single kernel with the most GPU time
        # per step in the kernel trace (profiles/kernel_trace_star5-n32768.md).
        # Event times do not rank the kernels here: with the factorisation
        # pipelined, a compress-stream launch (an ID, a kernel-block batch)
        # can wait for compute units that the leaf-level LU on the factor
        # stream holds, and its events count that wait.
        dom = "k_lu_fused" if "k_lu_fused" in rl else max(single, key=lambda k: rl[k]["seconds"])
        d = rl[dom]
        out["roofline"] = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                           "unit": d["unit"], "frac": d["frac"], "traffic": _traffic(dom, wl.name),
                           "avg_launch_us": round(1e6 * d["seconds"] / max(d["launches"], 1), 1)}
        out["kernel_rooflines"] = rl
    lm = rl.get("lu_multi (several kernels)")
    if lm:
        # beside the single-kernel roofline: the multi-workgroup LU sequences
        # (dense top-level system and the top levels' blocks), whose time per
        # step exceeds any single kernel's
        out["roofline_lu_multi"] = {"kernels": "k_calu_* sequence per call", "bound": "alu",
                                    "achieved": lm["achieved"], "peak": lm["peak"], "unit": lm["unit"],
                                    "frac": lm["frac"], "calls": lm["launches"],
                                    "avg_call_us": round(1e6 * lm["seconds"] / max(lm["launches"], 1), 1)}

    if not args.no_base:
        # the unscaled two-sided baseline over the same steps and warm-up
        t_base, stb, _ = _run_form(s, wl, binding.MULLER_BASE, args.steps, args.warmup, b, x, torch, rm, fused)
        out["nonsym"] = {"s_per_solve": round(t_base, 6), "t_compress": round(stb["t_compress"], 6),
                         "t_factor": round(stb["t_factor"], 6), "t_solve": round(stb["t_solve"], 6),
                         "t_compress_host": round(stb["t_compress"] - stb["t_compress_wait"], 6),
                         "kernel_seconds": {"kblock": round(stb["t_kblock_compress"] + stb["t_kblock_factor"], 6),
                                            "id": round(stb["t_id"], 6), "lu": round(stb["t_lu"], 6)},
                         "entries": int(stb["entries_compress"] + stb["entries_factor"]),
                         "steps": args.steps}
        out["speedup_sym_vs_nonsym"] = {"compress": round(stb["t_compress"] / st["t_compress"], 3),
                                        "total": round(t_base / t_sym, 3),
                                        "id_kernels": round(stb["t_id"] / st["t_id"], 3) if st["t_id"] > 0 else None,
                                        "entries": round(out["nonsym"]["entries"] / max(out["entries"], 1), 3)}
    if not args.no_parity:
        out["rel_err_vs_dense_oracle"] = _parity_vs_golden(s, wl, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(wl)
    print(json.dumps(out))


def _parity_vs_golden(s, wl, torch):
    """Untimed: the same path on the same curve and wavenumbers at a size whose
    dense-LU solution the oracle stored (tests/golden), relative 2-norm error."""
    import numpy as np
    import workloads
    from paper_2609_33216_amd import binding
    out = {}
    for n in (16384,):
        path = os.path.join(ROOT, "tests", "golden", f"star5_k50-75_n{n}_dense_x.npy")
        if wl.name != "star5-n32768-k50-75" or not os.path.exists(path):
            return None
        xd = np.load(path, allow_pickle=False)
        w = workloads.config2_reduced(n)
        x_, dx_, ddx_ = w.boundary()
        s.assemble(x_, dx_, ddx_, w.k0, w.k1, w.eps0, w.eps1, leaf=w.leaf, tol=w.tol, form=binding.MULLER_SYM)
        b = s.rhs_plane_wave(w.angle)
        s.compress()
        s.factor()
        xg = s.solve(b)
        out[f"n{n}"] = float(np.linalg.norm(xg - xd) / np.linalg.norm(xd))
    return out


if __name__ == "__main__":
    main()
