#!/usr/bin/env python3
"""Benchmark: BKS solves on one MI355X.

One step = one mixed-precision block Krylov-Schur solve (Algorithm 5,
BKS(2,4; k1, k3), rank (5,5,5)) of the C2 law as printed (20000 x 20000 x
2000, 2e6 stored, Zipf(1.3) modes 1-2, uniform mode 3, |N(0,1)| FP32) run
to its stopping rule -- the tolerance or the outer-iteration cap -- from a
fixed seeded start, with the tensor already resident in HBM.  `value` =
solves/s over the K timed steps; p50/p99 are per-solve latencies.  Beside
them: whether the solve converged, its angle to the plain FP64 GPU solve
of the same start, and the relative S-value gaps that condition the
subspaces.  The roofline object reports the dominant tensor-product kernel
class, timed live with HIP events on the stream it runs on
(`roofline_narrow` the dominant narrow product).  The `c2p` key reports the
same shape with a planted rank-(5,5,5) part.  The CPU baseline is the FP64
NumPy oracle's own BKS solve of the same workload and start, stopped after
3 outer iterations and scaled by the GPU's outer-iteration count.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --workload c5 --steps 1 --warmup 0   # the 2e8-entry tensor, rank 20
    python bench.py --ttmc-sweep      # C3-shaped product sweep (one JSON line per product)
    python bench.py --ablation        # block vs repeated one-column products
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

from paper_2012_07595_amd import bks, workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def dist(Ua, Ub):
    Qa = np.linalg.qr(Ua)[0]
    Qb = np.linalg.qr(Ub)[0]
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))


WORKLOAD_TEXT = {
    "c2p": "C2-shaped (1,2)-symmetric 20000x20000x2000, 2e6 stored, Zipf(1.3) modes 1-2, "
           "uniform mode 3, |N(0,1)| FP32 + planted rank-(5,5,5)",
    "c2": "C2-shaped (1,2)-symmetric 20000x20000x2000, 2e6 stored, Zipf(1.3) modes 1-2, "
          "uniform mode 3, |N(0,1)| FP32",
    "c3": "C3-shaped (1,2)-symmetric 200000x200000x10000, 5e7 stored, Zipf(1.5) modes 1-2, "
          "uniform mode 3, |N(0,1)| FP32",
    "c3p": "C3-shaped (1,2)-symmetric 200000x200000x10000, 5e7 stored, Zipf(1.5) modes 1-2, "
           "uniform mode 3, |N(0,1)| FP32 + planted rank-(10,10,10)",
    "p_princeton": "Princeton-shaped stand-in 6593x6593x29: Zipf(1.0) friendship pairs in their "
                   "endpoints' flag slices, 6.1e5 stored (1.2e6 full), values 1",
    "p_reuters": "Reuters-shaped stand-in 13332x13332x66: 2.4e5 stored (4.9e5 full), Zipf(1.0) "
                 "indices, Zipf(2) integer weights",
    "p_darpa": "DARPA-shaped stand-in 8891x8891x371: 1e6 stored, Zipf(1.2) indices, binary, "
               "slices scaled to Frobenius norm 1",
    "c5": "C5-shaped (1,2)-symmetric 1000000x1000000x500, 2e8 stored, Zipf(1.6) mode-1/2 degrees "
          "(Chung-Lu law), uniform mode 3, |N(0,1)| FP32",
}
WORKLOAD_GEN = {"c2p": "c2_planted", "c2": "c2", "c3": "c3", "c3p": "c3_planted",
                "p_princeton": "p_princeton", "p_reuters": "p_reuters", "p_darpa": "p_darpa",
                "c5": "c5"}
# the paper's ranks for its data sets (section "Experiments")
DEFAULT_RANK = {"c2p": 5, "c2": 5, "c3": 10, "c3p": 10, "p_princeton": 3, "p_reuters": 2,
                "p_darpa": 2, "c5": 20}


def load_traffic(kernel_class, workload):
    """HBM traffic per launch of `kernel_class` on `workload` from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by a
    plain copy of known size), or None if there is none for this kernel."""
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(root, "profiles", "traffic.json")) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    # counters taken on another revision of the kernels do not count
    for rel, sha in tab.get("_kernel_sources_sha1", {}).items():
        if file_sha1(os.path.join(root, rel)) != sha:
            return None
    ent = tab.get(f"{workload}/{kernel_class}")
    return None if ent is None else ent.get("bytes_per_launch")


def file_sha1(path):
    """git's blob id of a file (sha1 of 'blob <size>\\0' + content)."""
    import hashlib
    try:
        with open(path, "rb") as f:
            data = f.read()
    except OSError:
        return None
    return hashlib.sha1(b"blob %d\0" % len(data) + data).hexdigest()


def roofline_of(stats, workload=None):
    """Dominant kernel (by total event time of its main kernel) and its
    roofline.  `<class>_call` entries time whole calls (packing, fixups and
    reductions included) and are reported beside it."""
    if not stats:
        return None
    main = {k: v for k, v in stats.items() if not k.endswith("_call")}
    name, (calls, ms, by, fl) = max(main.items(), key=lambda kv: kv[1][1])
    call = stats.get(name + "_call")
    extra = {"call_avg_us": round(call[1] / call[0] * 1e3, 2)} if call else {}
    traffic = load_traffic(name, workload) if workload else None
    avg_s = ms / calls / 1e3
    if name.startswith("free3_sym_wide"):
        # FP32: a dense contraction on the matrix cores (FP32 MFMA peak);
        # FP64: vector FMA (FP64 peak)
        peak = FP32_PEAK_TFLOPS if name.endswith("_f32") else FP64_PEAK_TFLOPS
        bound = "mfma" if name.endswith("_f32") else "alu"
        ach = fl / calls / avg_s / 1e12
        return {"kernel": "ttmc_" + name, "bound": bound, "achieved": round(ach, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": traffic,
                "launches": calls, "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_flops_per_launch": fl / calls, **extra}
    alu_peak = FP32_PEAK_TFLOPS if name.endswith("_f32") else FP64_PEAK_TFLOPS
    if fl / (alu_peak * 1e12) > by / (HBM_PEAK_GBS * 1e9):
        # more time at the vector ALU peak than at the HBM peak: ALU-bound
        ach = fl / calls / avg_s / 1e12
        return {"kernel": "ttmc_" + name, "bound": "alu", "achieved": round(ach, 3),
                "peak": alu_peak, "unit": "TFLOP/s", "frac": round(ach / alu_peak, 4),
                "traffic": traffic, "launches": calls, "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_flops_per_launch": fl / calls,
                "hbm_GBs": round(by / calls / avg_s / 1e9, 1), **extra}
    ach = by / calls / avg_s / 1e9
    return {"kernel": "ttmc_" + name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "launches": calls, "avg_launch_us": round(avg_s * 1e6, 2),
            "algorithmic_bytes_per_launch": by / calls, **extra}


def host_cpu():
    """(logical CPUs, model name) of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline_b(coo, r, U0, W0, gpu_iters, outer=3):
    """Baseline B: the oracle's BKS algorithm with C++/OpenMP FP64 products
    and numpy's BLAS/LAPACK on all host cores, stopped after `outer` outer
    iterations, scaled to a whole solve by the GPU solve's iterations."""
    from baseline import cpu
    from oracle import sptensor
    T = sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))
    cpu.layouts(T)  # the sorted layouts are built once, outside the timing
    t0 = time.perf_counter()
    res = cpu.bks_solve(T, r, r, U0, W0, p=4, s=2, tol=1e-11, max_outer=outer)
    dt = time.perf_counter() - t0
    per_iter = dt / max(res["outer_iters"], 1)
    ncpu, model = host_cpu()
    return {"value": round(1.0 / (per_iter * max(gpu_iters, 1)), 6), "unit": "solves/s",
            "cores": cpu.threads(), "kind": "cpp-openmp", "host_cpus": ncpu, "host_model": model,
            "sample": f"the oracle's BKS(2,4) algorithm with C++/OpenMP FP64 products on "
                      f"{cpu.threads()} threads, same workload and start, {res['outer_iters']} "
                      f"outer iterations ({dt:.1f} s), scaled by the GPU solve's {gpu_iters} "
                      f"outer iterations"}


def cpu_baseline(coo, r, U0, W0, gpu_iters, outer=3):
    """The FP64 oracle's BKS solve on the same workload and start, stopped
    after `outer` outer iterations (about 10 s on one thread), scaled to a
    whole solve by the GPU solve's outer-iteration count."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import bks as obks, sptensor
    T = sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))
    ctxm = threadpool_limits(limits=1) if threadpool_limits else None
    t0 = time.perf_counter()
    res = obks.bks_solve(T, r, r, U0, W0, p=4, s=2, tol=1e-11, max_outer=outer)
    dt = time.perf_counter() - t0
    if ctxm is not None:
        ctxm.unregister() if hasattr(ctxm, "unregister") else None
    per_iter = dt / max(res["outer_iters"], 1)
    ncpu, model = host_cpu()
    return {"value": round(1.0 / (per_iter * max(gpu_iters, 1)), 6), "unit": "solves/s",
            "cores": 1, "kind": "oracle", "host_cpus": ncpu, "host_model": model,
            "sample": f"the FP64 NumPy oracle's BKS(2,4) solve of the same workload and start, "
                      f"{res['outer_iters']} outer iterations ({dt:.1f} s, 1 BLAS thread), "
                      f"scaled by the GPU solve's {gpu_iters} outer iterations"}


def narrow_roofline(stats, workload):
    """Roofline of the narrow product class (FREE3, FREE1, MODE3) that took
    the most kernel time."""
    narrow = {k: v for k, v in stats.items()
              if not k.endswith("_call") and not k.startswith("free3_sym_wide")}
    if not narrow:
        return None
    return roofline_of(narrow | {k + "_call": stats[k + "_call"] for k in narrow
                                 if k + "_call" in stats}, workload)


def s_gaps(info, r, r3):
    """Relative S-value gaps (s_r - s_{r+1}) / s_1 of modes 1 and 3 (the
    conditioning of the subspaces, section "Conditioning of the best
    approximation problem")."""
    s1, s3 = list(info.svals1[:r + 1]), list(info.svals3[:r3 + 1])
    g1 = (s1[r - 1] - s1[r]) / s1[0] if s1[0] > 0 else 0.0
    g3 = (s3[r3 - 1] - s3[r3]) / s3[0] if s3[0] > 0 else 0.0
    return g1, g3


def timed_solves(ctx, t, rank, precision, steps, kw):
    import torch
    lat, results = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        results.append(ctx.solve(t, rank, rank, precision=precision, **kw))
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat, results


def solve_summary(elapsed, lat, results, ref, rank):
    U, W, F, info, rc = results[0]
    Ur, Wr, Fr, info_r, rc_r = ref
    g1, g3 = s_gaps(info_r, rank, rank)
    au, aw = dist(Ur, U), dist(Wr, W)
    conv = bool(info.converged) and bool(info_r.converged)
    return {
        "value": round(len(lat) / elapsed, 4),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
        "converged": bool(info.converged), "outer_iters": info.outer_iters,
        "rel_grad": info.rel_grad,
        "angle_U_vs_fp64": au, "angle_W_vs_fp64": aw,
        "fp64_converged": bool(info_r.converged), "fp64_outer_iters": info_r.outer_iters,
        "fp64_rel_grad": info_r.rel_grad,
        "rel_gap_mode1": g1, "rel_gap_mode3": g3,
        # a reading of the section "Conditioning of the best approximation
        # problem": parity is claimed for converged solves on subspaces whose
        # relative S-value gap is at least 1e-3; otherwise the gaps are
        # reported beside the angle
        "parity": ("pinned" if conv and max(au, aw) <= 1e-8 and min(g1, g3) >= 1e-3 else
                   "not converged in max_outer" if not conv else
                   "unpinned (ill-conditioned)" if min(g1, g3) < 1e-3 else "angle above 1e-8"),
    }


def run_bks(args):
    import torch
    rank = args.rank if args.rank else DEFAULT_RANK[args.workload]
    t_gen = time.perf_counter()
    coo = getattr(workloads, WORKLOAD_GEN[args.workload])()
    U0, W0 = workloads.random_start(coo.m, coo.n, rank, rank, 2024)
    t_gen = time.perf_counter() - t_gen
    big = args.workload == "c5"
    stage = (lambda s: print(f"[bench] {s}", file=sys.stderr, flush=True)) if big else (lambda s: None)
    stage(f"generated {coo.nnz} stored entries in {t_gen:.1f} s")
    assert torch.cuda.is_available(), "bench needs a GPU"
    ctx = bks.Ctx(0)
    t_up = time.perf_counter()
    t = ctx.upload_coo(coo)
    t_up = time.perf_counter() - t_up
    stage(f"uploaded in {t_up:.1f} s")
    max_outer = args.max_outer if args.max_outer else (4 if big else 200)
    kw = dict(U0=U0, W0=W0, p=4, s=2, max_outer=max_outer, tol=1e-11)
    # plain FP64 GPU solve: the accuracy reference, then the comparison
    # throughput from warm FP64 solves
    a = time.perf_counter()
    ref = ctx.solve(t, rank, rank, precision=bks.PREC_FP64, **kw)
    torch.cuda.synchronize()
    ref_s = time.perf_counter() - a
    stage(f"FP64 reference solve: {ref_s:.1f} s, {ref[3].outer_iters} outer iterations")
    n64 = 0 if big else max(1, min(args.steps, 2))
    fp64_s = ref_s
    if n64:
        el, _, _ = timed_solves(ctx, t, rank, bks.PREC_FP64, n64, kw)
        fp64_s = el / n64
    for _ in range(args.warmup):
        ctx.solve(t, rank, rank, precision=bks.PREC_MIXED, **kw)
    torch.cuda.synchronize()
    ctx.profile(True)
    elapsed, lat, results = timed_solves(ctx, t, rank, bks.PREC_MIXED, args.steps, kw)
    stats = ctx.profile_read()
    ctx.profile(False)
    summ = solve_summary(elapsed, lat, results, ref, rank)
    U, W, F, info, rc = results[0]
    out = {
        "metric": "BKS solves/s + p50/p99 latency at 1e-8 subspace angle; TTMc HBM GB/s vs peak",
        "value": summ.pop("value"),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "dtype_detail": "f32 tensor-times-block products (the core product on FP32 MFMA); "
                        "f64 orthogonalisation, gradient and inner solve",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT[args.workload],
            "rank": [rank, rank, rank], "method": f"BKS(2,4;{info.k1},{info.k3})",
            "precision": "mixed", "tol": 1e-11, "max_outer": max_outer,
        },
        **summ,
        "fp64_solves_per_s": round(1.0 / fp64_s, 4),
        "phase_s": {"expand": round(info.t_expand, 4), "core": round(info.t_core, 4),
                    "inner_host": round(info.t_inner, 4), "bk_step": round(info.t_step, 4)},
        "svals1": list(np.round(info.svals1[:rank + 1], 4)),
        "svals3": list(np.round(info.svals3[:rank + 1], 4)),
        "kernels": {k: {"calls": v[0], "ms": round(v[1], 3)} for k, v in stats.items()},
        "roofline": roofline_of(stats, workload=args.workload),
        "roofline_narrow": narrow_roofline(stats, args.workload),
        "gen_s": round(t_gen, 2),
        "upload_s": round(t_up, 2),
    }
    if args.workload == "c2" and not args.no_extra:
        # the same law with a planted rank-(5,5,5) part: a well-conditioned
        # solve of the C2 shape (reported beside the headline, not as it)
        cp = workloads.c2_planted()
        tp = ctx.upload_coo(cp)
        refp = ctx.solve(tp, rank, rank, precision=bks.PREC_FP64, **kw)
        ctx.solve(tp, rank, rank, precision=bks.PREC_MIXED, **kw)
        el, latp, resp = timed_solves(ctx, tp, rank, bks.PREC_MIXED, max(args.steps, 5), kw)
        out["c2p"] = {"workload": WORKLOAD_TEXT["c2p"], **solve_summary(el, latp, resp, refp, rank)}
        tp.free()
    if big and not args.no_extra:
        # the comparison method on the same tensor and start (the C5
        # configuration names it): mixed-precision HOOI for as many
        # iterations as fit in the BKS solve's time, ||F|| beside BKS's
        stage("HOOI, same start")
        a = time.perf_counter()
        Uh, Wh, Fh, ih, _ = ctx.hooi(t, rank, rank, U0=U0, W0=W0, precision=bks.PREC_MIXED,
                                     max_iter=args.hooi_iters, grad_every=5)
        torch.cuda.synchronize()
        out["hooi"] = {"precision": "mixed", "iters": ih.outer_iters,
                       "seconds": round(time.perf_counter() - a, 2),
                       "normF": float(np.linalg.norm(Fh)), "rel_grad": ih.rel_grad,
                       "bks_normF": info.normF}
    if args.copy_ref_mb:
        copy_reference(args.copy_ref_mb)
    if not args.no_cpu and not big:
        out["cpu_baseline"] = cpu_baseline(coo, rank, U0, W0, info.outer_iters)
        out["cpu_baseline_b"] = cpu_baseline_b(coo, rank, U0, W0, info.outer_iters)
    print(json.dumps(out), flush=True)


def copy_reference(mb):
    """A plain device copy of `mb` MiB (outside any timed region): the
    reference that scales the FETCH_SIZE / WRITE_SIZE counters of a profiled
    run to bytes, and the measured stream-copy bandwidth (bytes read plus
    written per second, HIP events over 5 copies after 3)."""
    import torch
    nb = mb << 20
    a = torch.ones(nb // 4, device="cuda:0", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nb * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    print(json.dumps({"copy_ref_bytes": nb, "copy_GBs": round(gbs, 1)}), file=sys.stderr,
          flush=True)
    return gbs


def ttmc_sweep(args):
    """C3-shaped standalone products (one JSON line each)."""
    import torch
    t_gen = time.perf_counter()
    coo = workloads.c3()
    print(json.dumps({"stage": "generated", "seconds": round(time.perf_counter() - t_gen, 1)}), flush=True)
    ctx = bks.Ctx(0)
    t0 = time.perf_counter()
    t = ctx.upload_coo(coo)
    print(json.dumps({"stage": "uploaded", "seconds": round(time.perf_counter() - t0, 1),
                      "dev_bytes": t.dev_bytes, "pairs": t.npairs}), flush=True)
    del coo
    # measured stream-copy bandwidth: the attainable HBM rate beside the 8 TB/s
    copy_gbs = copy_reference(args.copy_ref_mb or 1024)
    dev = "cuda:0"
    cases = []
    for p in args.widths:
        cases += [("free3_sym", p, p), ("free3", p, p), ("free1", p, p), ("mode3", 0, p)]
    if args.ops:
        cases = [c for c in cases if c[0] in args.ops]
    for name, p1, p2 in cases:
        X = torch.randn(t.m, max(p1, 1), device=dev, dtype=torch.float32)
        Y = torch.randn(t.m, max(p1, 1), device=dev, dtype=torch.float32)
        Z = torch.randn(t.n, p2, device=dev, dtype=torch.float32)
        if name == "free3_sym":
            out = torch.empty(t.n, p1 * (p1 + 1) // 2, device=dev)
            call = lambda: ctx.ttmc(t, bks.FREE3, X, None, out, sym_half=True)
        elif name == "free3":
            Y2 = torch.randn(t.m, p2, device=dev)
            out = torch.empty(t.n, p1 * p2, device=dev)
            call = lambda: ctx.ttmc(t, bks.FREE3, X, Y2, out)
        elif name == "free1":
            out = torch.empty(t.m, p1 * p2, device=dev)
            call = lambda: ctx.ttmc(t, bks.FREE1, Y, Z, out)
        else:
            out = torch.empty(t.npairs, p2, device=dev)
            call = lambda: ctx.ttmc(t, bks.MODE3, None, Z, out)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(args.steps):
            call()
        torch.cuda.synchronize()
        st = ctx.profile_read()
        ctx.profile(False)
        rl = roofline_of(st, workload=f"c3/{name}{p2}")
        if rl.get("unit") == "GB/s":
            rl["copy_GBs"] = round(copy_gbs, 1)
            rl["frac_of_copy"] = round(rl["achieved"] / copy_gbs, 4)
        print(json.dumps({"op": name, "p": p2, "roofline": rl}), flush=True)


def ablation(args):
    """Block products against repeated single-vector products (the paper's
    3-9x claim for 6 vectors, section "Block-Krylov methods"): on two tensors of the paper's
    stated sizes, each block product and the equivalent sequence of
    one-column products, timed with HIP events (one JSON line each)."""
    import torch
    dev = "cuda:0"
    ctx = bks.Ctx(0)
    shapes = [("500x500x500", 500, 500), ("3600x3600x60", 3600, 60)]
    for label, m, n in shapes:
        coo = workloads.sparse_sym(m, n, 1_000_000, zipf=0.0, values="abs", seed=1020 + n)
        t = ctx.upload_coo(coo)
        X = torch.randn(m, 6, device=dev)
        Y = torch.randn(m, 2, device=dev)
        Z = torch.randn(n, 6, device=dev)
        o3 = torch.empty(n, 21, device=dev)
        o3v = torch.empty(n, 1, device=dev)
        o1 = torch.empty(m, 6, device=dev)
        o1v = torch.empty(m, 1, device=dev)
        om = torch.empty(t.npairs, 6, device=dev)
        omv = torch.empty(t.npairs, 1, device=dev)
        cols = [X[:, a:a + 1].contiguous() for a in range(6)]
        ycols = [Y[:, a:a + 1].contiguous() for a in range(2)]
        zcols = [Z[:, c:c + 1].contiguous() for c in range(6)]
        cases = {
            # A.(X, X)_{1,2}, 6 columns (21 distinct column pairs)
            "free3_sym": (lambda: ctx.ttmc(t, bks.FREE3, X, None, o3, sym_half=True),
                          lambda: [ctx.ttmc(t, bks.FREE3, cols[a], cols[b], o3v)
                                   for b in range(6) for a in range(b + 1)]),
            # A.(Y, Z)_{2,3}, 2 x 3 columns (6 column pairs)
            "free1": (lambda: ctx.ttmc(t, bks.FREE1, Y, Z[:, :3], o1),
                      lambda: [ctx.ttmc(t, bks.FREE1, ycols[b], zcols[c], o1v)
                               for c in range(3) for b in range(2)]),
            # A.(Z)_3, 6 columns
            "mode3": (lambda: ctx.ttmc(t, bks.MODE3, None, Z, om),
                      lambda: [ctx.ttmc(t, bks.MODE3, None, zcols[c], omv) for c in range(6)]),
        }
        for name, (blk, vec) in cases.items():
            res = {}
            for kind, fn in (("block", blk), ("vectors", vec)):
                for _ in range(3):
                    fn()
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(args.steps):
                    fn()
                b.record()
                torch.cuda.synchronize()
                res[kind] = a.elapsed_time(b) * 1e3 / args.steps
            print(json.dumps({"ablation": name, "tensor": label, "stored": coo.nnz,
                              "block_us": round(res["block"], 1),
                              "vectors_us": round(res["vectors"], 1),
                              "ratio": round(res["vectors"] / res["block"], 2)}), flush=True)
        t.free()
    ctx.close()


def serving(args):
    """C4-shaped serving trace (one JSON line): requests of different sizes and
    ranks, uploaded by the server after admission; closed-loop throughput, then
    Poisson arrivals at 0.7x that rate for the mixed-precision server and the
    plain FP64 server on the same trace."""
    import threading
    import torch
    from concurrent.futures import ThreadPoolExecutor
    reqs = workloads.c4_requests(count=args.requests, rate_per_s=1.0, nnz_range=(10_000, args.max_nnz))
    t0 = time.perf_counter()
    coos = []
    with ThreadPoolExecutor(max_workers=4) as ex:
        for q, coo in enumerate(ex.map(workloads.request_tensor, reqs)):
            coos.append(coo)
            print(f"[serving] generated request {q}", file=sys.stderr, flush=True)
    gen_s = time.perf_counter() - t0
    starts = [workloads.random_start(q.m, q.n, q.r, q.r, q.seed + 1) for q in reqs]
    assert torch.cuda.is_available()
    ctx = bks.Ctx(0)

    def run(precision, arrivals):
        srv = bks.Server(ctx, max_active=args.slots, host_workers=args.slots)
        ids = [None] * len(reqs)
        t_begin = srv.now()

        def submitter():
            for q, req in enumerate(reqs):
                if arrivals is not None:
                    delay = t_begin + arrivals[q] - srv.now()
                    if delay > 0:
                        time.sleep(delay)
                ids[q] = srv.submit(None, req.r, req.r, precision=precision, U0=starts[q][0],
                                    W0=starts[q][1], coo=coos[q], tol=1e-11, max_outer=args.max_outer)
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        pending = set(range(len(reqs)))
        while pending:
            for q in sorted(pending):
                res = srv.poll(ids[q])
                if res.done:
                    pending.discard(q)
                    print(f"[serving] prec {precision} request {q} m={reqs[q].m} n={reqs[q].n} "
                          f"nnz={reqs[q].nnz} r={reqs[q].r} status {res.status} "
                          f"iters {res.info.outer_iters} latency {res.t_end - res.t_submit:.3f}s",
                          file=sys.stderr, flush=True)
            time.sleep(0.05)
        out = []
        for q in range(len(reqs)):
            U, W, F, res = srv.wait(ids[q])
            out.append((U, W, res))
        makespan = max(r.t_end for _, _, r in out) - t_begin
        srv.close()
        lat = np.array([r.t_end - r.t_submit for _, _, r in out])
        return out, makespan, lat

    closed, mk_closed, _ = run(bks.PREC_MIXED, None)

    def summary(res, mk, lat):
        return {"solves_per_s": round(len(reqs) / mk, 3),
                "p50_ms": round(1e3 * np.percentile(lat, 50), 1),
                "p99_ms": round(1e3 * np.percentile(lat, 99), 1),
                "converged": sum(int(r.info.converged) for _, _, r in res)}

    # Poisson arrivals at fixed fractions of the closed-loop rate, the same
    # arrival trace for the mixed and the FP64 server
    sweep = []
    for f in args.rate_factors:
        rate_f = f * len(reqs) / mk_closed
        arr = np.cumsum(np.random.default_rng(1003).exponential(1.0 / rate_f, size=len(reqs)))
        arr -= arr[0]
        m_res = run(bks.PREC_MIXED, arr)
        f_res = run(bks.PREC_FP64, arr)
        a_f = max(max(dist(a[0], b[0]), dist(a[1], b[1])) for a, b in zip(m_res[0], f_res[0]))
        sweep.append({"factor": f, "arrival_rate_per_s": round(rate_f, 3),
                      "mixed": summary(*m_res), "fp64": summary(*f_res),
                      "max_angle_mixed_vs_fp64": a_f, "_res": (m_res, f_res)})
    main_ = min(sweep, key=lambda e: abs(e["factor"] - 0.7))
    (mixed, mk_m, lat_m), (fp64, mk_f, lat_f) = main_["_res"]
    rate = main_["arrival_rate_per_s"]
    for e in sweep:
        del e["_res"]
    ang = main_["max_angle_mixed_vs_fp64"]
    conv = sum(int(r.info.converged) for _, _, r in mixed)
    out = {
        "metric": "BKS solves/s + p50/p99 latency (serving, Poisson arrivals)",
        "requests": len(reqs), "slots": args.slots, "arrival_rate_per_s": round(rate, 3),
        "closed_loop_solves_per_s": round(len(reqs) / mk_closed, 3),
        "mixed": {"solves_per_s": round(len(reqs) / mk_m, 3), "p50_ms": round(1e3 * np.percentile(lat_m, 50), 1),
                  "p99_ms": round(1e3 * np.percentile(lat_m, 99), 1), "converged": conv},
        "fp64": {"solves_per_s": round(len(reqs) / mk_f, 3), "p50_ms": round(1e3 * np.percentile(lat_f, 50), 1),
                 "p99_ms": round(1e3 * np.percentile(lat_f, 99), 1),
                 "converged": sum(int(r.info.converged) for _, _, r in fp64)},
        "max_angle_mixed_vs_fp64": ang,
        "rate_sweep": sweep,
        "config": {"workload": f"C4-shaped: I~U[1e3,1e5], K~U[100,5000], nnz~U[1e4,{args.max_nnz:.0e}] "
                               "Zipf(1.3)/uniform |N(0,1)| FP32 + planted rank-r, r in {2,3,5,8,10}",
                   "latency": "upload + solve + result"},
        "gen_s": round(gen_s, 1),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOAD_TEXT), default="c2")
    ap.add_argument("--rank", type=int, default=0)
    ap.add_argument("--max-outer", type=int, default=0,
                    help="outer iteration cap (default 200; 4 for c5)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--hooi-iters", type=int, default=10,
                    help="HOOI iterations of the c5 comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the planted C2 variant reported beside the C2 line")
    ap.add_argument("--ttmc-sweep", action="store_true")
    ap.add_argument("--widths", type=int, nargs="*", default=[5, 10, 20])
    ap.add_argument("--ops", nargs="*", default=None,
                    choices=["free3_sym", "free3", "free1", "mode3"])
    ap.add_argument("--copy-ref-mb", type=int, default=0)
    ap.add_argument("--serving", action="store_true")
    ap.add_argument("--ablation", action="store_true",
                    help="block products against repeated one-column products")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--max-nnz", type=int, default=5_000_000)
    ap.add_argument("--rate-factors", type=float, nargs="*", default=[0.7],
                    help="Poisson arrival rates as fractions of the closed-loop rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path "
              "runs on one GPU; sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving(args)
    elif args.ablation:
        ablation(args)
    elif args.ttmc_sweep:
        ttmc_sweep(args)
    else:
        run_bks(args)


if __name__ == "__main__":
    main()
