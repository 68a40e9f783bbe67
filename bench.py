"""Benchmark: time to rtol 1e-8 for the 20-group block system, FP32 batched
AMG V-cycles inside FP64 FGMRES vs the plain FP64 form.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload g20_3d64]

One step is one complete preconditioned GMRES(30) solve to rtol 1e-8 of the
synthetic system (preconditioner built beforehand; setup is timed and
reported separately).  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def sources_digest() -> str:
    """SHA-256 (first 16 hex digits) over the library sources, sorted by name,
    each as its relative path, a NUL byte and its bytes."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2002_04958_amd", "csrc", "*.hip"))
                   + glob.glob(os.path.join(ROOT, "paper_2002_04958_amd", "csrc", "*.hpp")))
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, calibrated), or None when there is no
    record for it or the library sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "solve_kernels_g20_3d64.md")
    if not os.path.exists(path):
        return None
    want = sources_digest()
    for line in open(path):
        m = re.match(r"traffic-record: kernel=(.+) bytes_per_launch=(\d+) sources=([0-9a-f]+)\s*$",
                     line)
        if m and m.group(1) == kernel and m.group(3) == want:
            return int(m.group(2))
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(name: str, budget_s: float = 20.0):
    """The oracle (numpy/scipy FP64) on a bounded sample: the same generator,
    group count and preconditioner on a smaller mesh, scaled linearly in the
    number of unknowns to the full workload."""
    import numpy as np

    import synth_inputs as si
    from oracle import amg as oamg
    from oracle import assemble as oasm
    from oracle import krylov as okry
    from oracle import precond as opc

    w = si.WORKLOADS[name]
    n_sample = {3: 28, 2: 192}[w.dim]
    inp = si.generate(w.G, w.dim, n_sample, w.seed)
    t0 = time.perf_counter()
    sysm = oasm.assemble(inp)
    M = opc.BlockPreconditioner(sysm, opc.BlockParams(kind="schur2", amg=oamg.AMGParams(seed=w.seed)))
    t1 = time.perf_counter()
    A = sysm.monolithic()
    x, info = okry.gmres(sysm.matvec, M, inp.b, rtol=1e-8)
    t2 = time.perf_counter()
    scale = w.n_unknowns / sysm.n
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    return {
        "value": (t2 - t1) * scale, "unit": "s", "cores": cores, "kind": "oracle",
        "sample": (f"G={w.G} {w.dim}D {n_sample}^{w.dim} ({sysm.n} unknowns): setup {t1 - t0:.2f}s, "
                   f"solve {t2 - t1:.2f}s in {info.iters} iterations; solve time scaled x{scale:.0f} "
                   "by unknowns"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="g20_3d64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--no-inner", action="store_true")
    ap.add_argument("--no-option4", action="store_true")
    ap.add_argument("--no-aggressive", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate layouts of every level once and keep the fastest "
                         "(cached per process, or in MGD_AUTOTUNE_CACHE)")
    ap.add_argument("--counters-run", action="store_true",
                    help="short run for hardware-counter passes: a streaming calibration "
                         "kernel (torch mul reading 1 GiB and writing 1 GiB, its input pushed "
                         "out of the last-level cache first), then the FP32 batched setup and "
                         "--steps solves; no timing lines")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; sharding across GPUs is designed "
                                   "but not implemented", "n_gpus": a.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth_inputs as si
    from paper_2002_04958_amd import api

    w = si.WORKLOADS[a.workload]
    log(f"[bench] workload {w.name}: G={w.G} {w.dim}D {w.n}^{w.dim}, {w.n_unknowns} unknowns")
    inp = si.generate_workload(w.name)
    ctx = api.Context(0)
    co = api.Coeffs.from_inputs(ctx, inp)
    sysg = api.BlockSystem.assemble(ctx, co)
    b = torch.as_tensor(inp.b, device=ctx.device)
    bnorm = float(torch.linalg.vector_norm(b))

    def build(batched, fp32, graph, adaptive=False, inner_tol=0.0, option4=0, aggressive=0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = api.BlockPreconditioner(ctx, sysg, "schur2", amg_seed=w.seed,
                                    amg_precision=1 if fp32 else 0, batched=int(batched),
                                    use_graph=int(graph), adaptive=int(adaptive),
                                    inner_tol=inner_tol, option4_steps=option4,
                                    amg_aggressive_levels=aggressive,
                                    amg_autotune=int(a.autotune))
        torch.cuda.synchronize()
        return M, time.perf_counter() - t0

    def solve(M):
        x = torch.zeros_like(b)
        x, r = api.gmres(ctx, sysg, M, b, x, rtol=1e-8, flexible=1)
        return x, r

    if a.counters_run:
        src = torch.ones(256 << 20, dtype=torch.float32, device=ctx.device)
        flush = torch.ones(512 << 20, dtype=torch.float32, device=ctx.device)  # 2 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst, flush
        M32, _ = build(True, True, True)
        for _ in range(max(1, a.steps)):
            x, r = solve(M32)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "counters", "workload": w.name, "iters": r.iters,
                          "calibration_bytes": {"read": 1 << 30, "written": 1 << 30}}))
        return

    # headline form: FP32 hierarchies, batched V-cycles, graph replay
    M32, setup32 = build(True, True, True)
    log(f"[bench] fp32 batched setup {setup32:.2f}s")
    for idx, label in ((0, "group 1"), (w.G, "E"), (w.G + 1, "I")):
        hi = M32.hierarchy(idx).info()
        log(f"[bench] hierarchy {label}: rows per level {hi['n']}, nnz {hi['nnz']}")
    for _ in range(a.warmup):
        solve(M32)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    t0 = time.perf_counter()
    iters = []
    for _ in range(a.steps):
        x, r = solve(M32)
        iters.append(r.iters)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / a.steps
    relres = float(torch.linalg.vector_norm(b - sysg.matvec(x))) / bnorm
    log(f"[bench] fp32 batched: {ms_step:.1f} ms/solve, iters {iters}, relres {relres:.2e}")

    # the adaptive variant of the same preconditioner (alpha-Schur2, Section 3.5)
    alpha = None
    if not a.no_adaptive:
        Ma, setup_a = build(True, True, True, adaptive=True)
        ia = Ma.info()
        solve(Ma)
        torch.cuda.synchronize()
        ea0, ea1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea0.record()
        iters_a = []
        for _ in range(a.steps):
            xa, ra = solve(Ma)
            iters_a.append(ra.iters)
        ea1.record()
        torch.cuda.synchronize()
        ms_a = ea0.elapsed_time(ea1) / a.steps
        relres_a = float(torch.linalg.vector_norm(b - sysg.matvec(xa))) / bnorm
        weak = ia["weak"]
        alpha = {"s": ms_a / 1e3, "iters": iters_a, "relres": relres_a, "setup_s": setup_a,
                 "neglected": {"gE": [g for g, v in enumerate(weak["gE"]) if v],
                               "Eg": [g for g, v in enumerate(weak["Eg"]) if v],
                               "EI": weak["EI"], "IE": weak["IE"]},
                 "jacobi_roles": [r for r, v in enumerate(ia["jacobi"]) if v],
                 "inverses_per_apply": ia["inverses_per_apply"]}
        log(f"[bench] alpha-schur2 fp32 batched: {ms_a:.1f} ms/solve, iters {iters_a}, "
            f"relres {relres_a:.2e}, neglected {alpha['neglected']}, "
            f"jacobi roles {alpha['jacobi_roles']}")
        del Ma, xa

    # option #4: S_I by two fixed-point steps on A_I and A_E instead of the hat
    opt4 = None
    if not a.no_option4:
        M4, setup_4 = build(True, True, True, option4=2)
        solve(M4)
        torch.cuda.synchronize()
        e40, e41 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e40.record()
        iters_4 = []
        for _ in range(a.steps):
            x4, r4 = solve(M4)
            iters_4.append(r4.iters)
        e41.record()
        torch.cuda.synchronize()
        ms_4 = e40.elapsed_time(e41) / a.steps
        relres_4 = float(torch.linalg.vector_norm(b - sysg.matvec(x4))) / bnorm
        opt4 = {"s": ms_4 / 1e3, "iters": iters_4, "relres": relres_4, "setup_s": setup_4,
                "steps": 2}
        log(f"[bench] schur2 option #4 (2 steps) fp32 batched: {ms_4:.1f} ms/solve, "
            f"iters {iters_4}, relres {relres_4:.2e}")
        del M4, x4

    # aggressive coarsening with multipass interpolation on the finest level of every inverse
    aggr = None
    if not a.no_aggressive:
        Mg_, setup_g = build(True, True, True, aggressive=1)
        solve(Mg_)
        torch.cuda.synchronize()
        eg0, eg1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        eg0.record()
        iters_g = []
        for _ in range(a.steps):
            xg_, rg_ = solve(Mg_)
            iters_g.append(rg_.iters)
        eg1.record()
        torch.cuda.synchronize()
        ms_g = eg0.elapsed_time(eg1) / a.steps
        relres_g = float(torch.linalg.vector_norm(b - sysg.matvec(xg_))) / bnorm
        hg = Mg_.hierarchy(0).info()
        aggr = {"s": ms_g / 1e3, "iters": iters_g, "relres": relres_g, "setup_s": setup_g,
                "group0_levels": hg["n"], "group0_operator_complexity": hg["operator_complexity"]}
        log(f"[bench] schur2 aggressive finest level fp32 batched: {ms_g:.1f} ms/solve, "
            f"iters {iters_g}, relres {relres_g:.2e}, setup {setup_g:.3f} s, "
            f"group-0 levels {hg['n']}")
        del Mg_, xg_

    # the inner solves of Section 4: S^_g and S^_I to a relative tolerance 1e-2
    inner = None
    if not a.no_inner:
        Mi, setup_i = build(True, True, False, inner_tol=1e-2)
        solve(Mi)
        torch.cuda.synchronize()
        t0i = time.perf_counter()
        xi, ri = solve(Mi)
        torch.cuda.synchronize()
        ti = time.perf_counter() - t0i
        relres_i = float(torch.linalg.vector_norm(b - sysg.matvec(xi))) / bnorm
        ii = Mi.info()
        inner = {"s": ti, "iters": ri.iters, "relres": relres_i, "setup_s": setup_i,
                 "inner_cycles_last_apply": ii["inner_cycles"]}
        log(f"[bench] schur2 inner tol 1e-2 fp32 batched: {ti * 1e3:.1f} ms/solve, iters {ri.iters}, "
            f"relres {relres_i:.2e}, inner cycles of the last apply {ii['inner_cycles']}")
        del Mi, xi

    # plain FP64 form: sequential launches, no graph
    plain = None
    if not a.no_plain:
        M64, setup64 = build(False, False, False)
        solve(M64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x64, r64 = solve(M64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        err32 = float(torch.linalg.vector_norm(x - x64)) / float(torch.linalg.vector_norm(x64))
        plain = {"s": t64, "iters": r64.iters, "setup_s": setup64,
                 "relres": r64.relres_true, "fp32_vs_fp64_rel_err": err32}
        log(f"[bench] fp64 plain: {t64 * 1e3:.1f} ms/solve, iters {r64.iters}")
        del M64

    # per-kernel timing pass: HIP events on the context stream around every
    # launch of one solve (no graph), algorithmic bytes from the hierarchy
    ctx.reset_kernel_stats()
    ctx.set_profiling(True)
    solve(M32)
    ctx.set_profiling(False)
    stats = ctx.kernel_stats()
    tagged = ctx.kernel_symbol_stats()  # "symbol@L<level>/<members>"
    syms = {}
    for k, v in tagged.items():
        agg = syms.setdefault(k.split("@")[0], {"launches": 0, "ms": 0.0, "bytes": 0.0})
        for f in agg:
            agg[f] += v[f]
    dom = max(syms, key=lambda k: syms[k]["ms"])
    s = syms[dom]
    achieved = (s["bytes"] / 1e9) / (s["ms"] / 1e3) if s["ms"] > 0 else 0.0
    log("[bench] kernel classes: " + ", ".join(
        f"{k}={v['ms']:.1f}ms/{v['launches']}" for k, v in stats.items() if v["launches"]))
    log("[bench] kernels: " + ", ".join(
        f"{k}={v['ms']:.1f}ms/{v['launches']}" for k, v in sorted(syms.items(), key=lambda kv: -kv[1]["ms"])))
    log("[bench] by level: " + ", ".join(
        f"{k}={v['ms']:.1f}ms/{v['launches']}({(v['bytes'] / 1e9) / (v['ms'] / 1e3) if v['ms'] else 0:.0f}GB/s)"
        for k, v in sorted(tagged.items(), key=lambda kv: -kv[1]["ms"])[:40]))

    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] oracle CPU baseline (bounded sample)...")
        cpu = cpu_baseline(w.name)

    out = {
        "metric": "time to rtol 1e-8 (s) & SpMV HBM GB/s, G=20; FP32-AMG batched vs FP64 plain",
        "value": ms_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64 (FGMRES) / f32 (V-cycles)",
        "data": "synthetic",
        "config": {"workload": f"G={w.G} {w.dim}D {w.n}^{w.dim} 7-point, {w.n_unknowns} unknowns, "
                               "Schur2, FGMRES(30) rtol 1e-8",
                   "global_batch": 1, "parallelism": "none"},
        "iters": iters,
        "relres_true": relres,
        "setup_s": setup32,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": (plain["s"] / (ms_step / 1e3)) if plain else None,
        "alpha_schur2_fp32": alpha,
        "schur2_inner_tol_1e-2_fp32": inner,
        "schur2_option4_fp32": opt4,
        "schur2_aggressive_fp32": aggr,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(dom), "traffic_unit": "bytes per launch",
                     "launches": s["launches"],
                     "avg_launch_us": 1e3 * s["ms"] / max(1, s["launches"]),
                     "bytes_per_launch": s["bytes"] / max(1, s["launches"])},
        "kernels": {k: {"ms": v["ms"], "launches": v["launches"],
                        "GB/s": (v["bytes"] / 1e9) / (v["ms"] / 1e3) if v["ms"] else 0.0}
                    for k, v in syms.items()},
        "kernels_by_level": {k: {"ms": v["ms"], "launches": v["launches"],
                                 "GB/s": (v["bytes"] / 1e9) / (v["ms"] / 1e3) if v["ms"] else 0.0}
                             for k, v in tagged.items()},
        "kernel_classes": {k: {"ms": v["ms"], "launches": v["launches"],
                               "GB/s": (v["bytes"] / 1e9) / (v["ms"] / 1e3) if v["ms"] else 0.0}
                           for k, v in stats.items() if v["launches"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
