"""Benchmark: time to rtol 1e-8 for the 20-group block system, FP32 batched
AMG V-cycles inside FP64 FGMRES vs the plain FP64 form.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload g20_3d64]

One step is one complete preconditioned FGMRES(30) solve to rtol 1e-8 of the
synthetic 20-group 3D 64^3 system (Schur2 of Section 3.3 with the Section 3.4
diagonal approximations; the preconditioner is built beforehand and its setup
is timed and reported separately).  Prints ONE JSON line: the headline, the
forms that split the FP32/FP64 ratio, the other workloads (2D 1024^2 G=1 with
five preconditioners, 2D 256^2 G=20 block-diagonal batched against
sequential, 2D 512^2 G=20 forward and adjoint), the roofline of the kernel
with the largest time and the oracle timed on the host.
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
    """HBM bytes per launch of `kernel` (symbol, with its level tag) from the
    committed counter summary (FETCH_SIZE and WRITE_SIZE passes, calibrated),
    or None when there is no record for it or the library sources changed since
    the counters were taken."""
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


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(name: str):
    """The oracle (numpy/scipy FP64, single-threaded: BLAS limited to one
    thread, scipy.sparse is serial) on the full workload: Schur2 setup, then
    FGMRES(30) to rtol 1e-8 from zero.  Returns (record, oracle solution)."""
    from threadpoolctl import threadpool_limits

    import synth_inputs as si
    from oracle import amg as oamg
    from oracle import assemble as oasm
    from oracle import krylov as okry
    from oracle import precond as opc

    w = si.WORKLOADS[name]
    inp = si.generate_workload(name)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sysm = oasm.assemble(inp)
        M = opc.BlockPreconditioner(sysm, opc.BlockParams(kind="schur2",
                                                          amg=oamg.AMGParams(seed=w.seed)))
        t1 = time.perf_counter()
        log(f"[bench] oracle setup {t1 - t0:.1f} s; FGMRES(30) to 1e-8 ...")
        x, info = okry.gmres(sysm.matvec, M, inp.b, rtol=1e-8, flexible=True)
        t2 = time.perf_counter()
    log(f"[bench] oracle solve {t2 - t1:.1f} s, {info.iters} iterations")
    rec = {
        "value": t2 - t1, "unit": "s", "cores": 1, "kind": "oracle",
        "sample": (f"the full workload (G={w.G} {w.dim}D {w.n}^{w.dim}, {w.n_unknowns} unknowns): "
                   f"oracle Schur2 setup {t1 - t0:.1f} s (not in value), FGMRES(30) to rtol 1e-8 "
                   f"in {info.iters} iterations {t2 - t1:.1f} s; one thread"),
        "setup_s": t1 - t0, "iters": info.iters, "relres_true": info.relres_true,
        "host_cpu": host_cpu(), "host_cpus_available": len(os.sched_getaffinity(0)),
    }
    return rec, x


def error_against(x, ref, G):
    """max_i |x_i - ref_i| / max_{seg(i)} |ref| over the block segments, and
    the relative 2-norm difference."""
    import numpy as np
    X = np.asarray(x).reshape(G + 2, -1)
    R = np.asarray(ref).reshape(G + 2, -1)
    seg = np.abs(R).max(axis=1, keepdims=True)
    return {"max_abs_over_segment_max": float((np.abs(X - R) / seg).max()),
            "rel_2norm": float(np.linalg.norm(X - R) / np.linalg.norm(R))}


def error_against_sample(x, name, G):
    """The same measure at the stored sample positions of the oracle's solution
    (written by tests/golden/make_fullsize.py)."""
    import numpy as np
    jpath = os.path.join(ROOT, "tests", "golden", f"fullsize_{name}.json")
    npath = os.path.join(ROOT, "tests", "golden", f"fullsize_{name}.npz")
    if not (os.path.exists(jpath) and os.path.exists(npath)):
        return None
    meta = json.load(open(jpath))
    case = meta["cases"]["schur2"]
    with np.load(npath) as z:
        pos, ref = z["pos"], z["schur2/x"]
    N = np.asarray(x).size // (G + 2)
    seg = np.asarray(case["x_norminf"])[pos // N]
    return {"max_abs_over_segment_max": float((np.abs(np.asarray(x)[pos] - ref) / seg).max()),
            "positions": int(len(pos)), "oracle_iters": case["gmres"]["iters"]}


def copy_ceiling(torch, device, reps=10):
    """Streaming copy of 1 GiB into another 1 GiB on the device (torch's copy
    kernel), timed with events: (GB/s counting bytes read + written)."""
    src = torch.ones(256 << 20, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form-steps", type=int, default=3,
                    help="solves timed for each of the other forms and workloads")
    ap.add_argument("--workload", default="g20_3d64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip Schur1, PCTL and lower Schur2 in the benchmark's form, and the "
                         "adaptive, option #4, aggressive and inner-tolerance variants of Schur2")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the 2D 1024^2, 2D 256^2 and 2D 512^2 workloads")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default layout rules instead of timing the candidate layouts "
                         "of every level at setup (the tuned choice is cached per process, or "
                         "in MGD_AUTOTUNE_CACHE)")
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

    def build(sysx, kind, seed, fp32, batched, graph, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = api.BlockPreconditioner(ctx, sysx, kind, amg_seed=seed,
                                    amg_precision=1 if fp32 else 0, batched=int(batched),
                                    use_graph=int(graph), amg_autotune=int(a.autotune), **kw)
        torch.cuda.synchronize()
        return M, time.perf_counter() - t0

    def solve(sysx, M, rhs):
        x = torch.zeros_like(rhs)
        return api.gmres(ctx, sysx, M, rhs, x, rtol=1e-8, flexible=1)

    def timed(sysx, M, rhs, steps, warmup=1):
        """Mean event-timed ms per solve over `steps` solves after `warmup`."""
        for _ in range(warmup):
            solve(sysx, M, rhs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        iters = []
        for _ in range(steps):
            x, r = solve(sysx, M, rhs)
            iters.append(r.iters)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, iters, x, r

    if a.counters_run:
        src = torch.ones(256 << 20, dtype=torch.float32, device=ctx.device)
        flush = torch.ones(512 << 20, dtype=torch.float32, device=ctx.device)  # 2 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst, flush
        M32, _ = build(sysg, "schur2", w.seed, True, True, True)
        for _ in range(max(1, a.steps)):
            x, r = solve(sysg, M32, b)
        # and the all-block matvec alone (roofline.standalone)
        xa_ = torch.rand(sysg.n, dtype=torch.float64, device=ctx.device)
        ya_ = ctx.empty(sysg.n)
        for _ in range(5):
            sysg.matvec(xa_, ya_)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "counters", "workload": w.name, "iters": r.iters,
                          "calibration_bytes": {"read": 1 << 30, "written": 1 << 30}}))
        return

    # headline form: FP32 hierarchies, batched V-cycles, graph replay
    M32, setup32 = build(sysg, "schur2", w.seed, True, True, True)
    log(f"[bench] fp32 batched setup {setup32:.2f}s")
    for idx, label in ((0, "group 1"), (w.G, "E"), (w.G + 1, "I")):
        hi = M32.hierarchy(idx).info()
        log(f"[bench] hierarchy {label}: rows per level {hi['n']}, nnz {hi['nnz']}")
    ms_step, iters, x32, r32 = timed(sysg, M32, b, a.steps, a.warmup)
    relres = float(torch.linalg.vector_norm(b - sysg.matvec(x32))) / bnorm
    x32h = x32.cpu().numpy()
    log(f"[bench] fp32 batched: {ms_step:.1f} ms/solve, iters {iters}, relres {relres:.2e}")

    # the forms that split the FP32-batched / FP64-plain ratio
    forms = {}
    if not a.no_forms:
        for key, fp32, batched, graph in (("fp64_plain", False, False, False),
                                          ("fp64_batched_graph", False, True, True),
                                          ("fp32_sequential", True, False, False)):
            M, su = build(sysg, "schur2", w.seed, fp32, batched, graph)
            ms, it, xf, rf = timed(sysg, M, b, a.form_steps)
            rr = float(torch.linalg.vector_norm(b - sysg.matvec(xf))) / bnorm
            forms[key] = {"ms": ms, "iters": it, "setup_s": su, "relres_true": rr}
            if key == "fp64_plain":
                x64h = xf.cpu().numpy()
            log(f"[bench] {key}: {ms:.1f} ms/solve, iters {it}, setup {su:.2f}s")
            del M, xf
        forms["fp32_batched_graph"] = {"ms": ms_step, "iters": iters, "setup_s": setup32,
                                       "relres_true": relres}
        p = forms["fp64_plain"]["ms"]
        forms["ratios_vs_fp64_plain"] = {k: p / v["ms"] for k, v in forms.items()
                                         if isinstance(v, dict) and "ms" in v}

    # the other block preconditioners of Sections 3.2-3.3 in the same form, and
    # the adaptive, option #4, aggressive and inner-tolerance variants of Schur2
    # (Sections 3.4, 3.5)
    variants = {}
    if not a.no_variants:
        for key, kind, kw, graph in (("schur1", "schur1", {}, True),
                                     ("pctl", "pctl", {}, True),
                                     ("schur2_lower", "schur2_lower", {}, True),
                                     ("alpha_schur2", "schur2", dict(adaptive=1), True),
                                     ("option4_2steps", "schur2", dict(option4_steps=2), True),
                                     ("aggressive_finest", "schur2", dict(amg_aggressive_levels=1),
                                      True),
                                     ("inner_tol_1e-2", "schur2", dict(inner_tol=1e-2), False)):
            M, su = build(sysg, kind, w.seed, True, True, graph, **kw)
            steps = 1 if key.startswith("inner") else a.form_steps
            ms, it, xv, rv = timed(sysg, M, b, steps)
            rr = float(torch.linalg.vector_norm(b - sysg.matvec(xv))) / bnorm
            rec = {"ms": ms, "iters": it, "setup_s": su, "relres_true": rr}
            inf = M.info()
            if key == "alpha_schur2":
                weak = inf["weak"]
                rec["neglected"] = {"gE": [g for g, v in enumerate(weak["gE"]) if v],
                                    "Eg": [g for g, v in enumerate(weak["Eg"]) if v],
                                    "EI": weak["EI"], "IE": weak["IE"]}
                rec["jacobi_roles"] = [r for r, v in enumerate(inf["jacobi"]) if v]
            if key == "aggressive_finest":
                hg = M.hierarchy(0).info()
                rec["group0_levels"] = hg["n"]
            if key.startswith("inner"):
                rec["inner_cycles_last_apply"] = inf["inner_cycles"]
            variants[key] = rec
            log(f"[bench] {key}: {ms:.1f} ms/solve, iters {it}, relres {rr:.2e}")
            del M, xv

    # per-kernel timing pass: HIP events on the context stream around every
    # launch of one FP32 batched solve (direct launches, no graph)
    M32d, _ = build(sysg, "schur2", w.seed, True, True, False)
    solve(sysg, M32d, b)
    ctx.reset_kernel_stats()
    ctx.set_profiling(True)
    solve(sysg, M32d, b)
    ctx.set_profiling(False)
    stats = ctx.kernel_stats()
    tagged = ctx.kernel_symbol_stats()  # "symbol@L<level>/<members>" for V-cycle kernels
    del M32d
    dom = max((k for k in tagged if tagged[k]["bytes"] > 0), key=lambda k: tagged[k]["ms"])
    s = tagged[dom]
    avg_us = 1e3 * s["ms"] / s["launches"]
    bpl = s["bytes"] / s["launches"]
    bpl_csr = s["bytes_csr"] / s["launches"]
    copy_gbs = copy_ceiling(torch, ctx.device)
    achieved = bpl_csr / (avg_us * 1e-6) / 1e9
    achieved_stored = bpl / (avg_us * 1e-6) / 1e9
    log("[bench] kernel classes: " + ", ".join(
        f"{k}={v['ms']:.1f}ms/{v['launches']}" for k, v in stats.items() if v["launches"]))
    log("[bench] kernels: " + ", ".join(
        f"{k}={v['ms']:.2f}ms/{v['launches']}({v['bytes_csr'] / v['ms'] / 1e6 if v['ms'] else 0:.0f}GB/s)"
        for k, v in sorted(tagged.items(), key=lambda kv: -kv[1]["ms"])[:40]))
    log(f"[bench] dominant {dom}: {avg_us:.2f} us/launch, {achieved:.0f} GB/s (CSR model), "
        f"{achieved_stored:.0f} GB/s (stored layout); copy {copy_gbs:.0f} GB/s")
    # The block matvec alone on the device: y = A x over all G+2 blocks, the
    # kernel family and storage of the split launch (which shares the device
    # with the E V-cycle in the solve), 20 launches back to back, event-timed.
    xa_ = torch.rand(sysg.n, dtype=torch.float64, device=ctx.device)
    ya_ = ctx.empty(sysg.n)
    for _ in range(3):
        sysg.matvec(xa_, ya_)
    ctx.reset_kernel_stats()
    ctx.set_profiling(True)
    for _ in range(20):
        sysg.matvec(xa_, ya_)
    ctx.set_profiling(False)
    al_stats = ctx.kernel_symbol_stats()
    alone_k = next((k for k in al_stats if k.startswith("k_block_matvec_shared<512, false, false")),
                   None)
    al = al_stats.get(alone_k) if alone_k else None
    standalone = None
    if al and al["launches"]:
        al_us = 1e3 * al["ms"] / al["launches"]
        al_b, al_bc = al["bytes"] / al["launches"], al["bytes_csr"] / al["launches"]
        al_csr, al_st = al_bc / (al_us * 1e-6) / 1e9, al_b / (al_us * 1e-6) / 1e9
        standalone = {"kernel": alone_k, "what": "y = A x over all blocks, alone on the device",
                      "launches": al["launches"], "avg_launch_us": al_us,
                      "traffic": recorded_traffic(alone_k),
                      "bytes_per_launch": al_bc, "bytes_per_launch_stored": al_b,
                      "achieved": al_csr, "frac": al_csr / HBM_PEAK_GBS,
                      "achieved_stored": al_st, "frac_stored": al_st / HBM_PEAK_GBS,
                      "frac_of_copy": al_st / copy_gbs}
        log(f"[bench] {alone_k} alone: {al_us:.2f} us/launch, {al_csr:.0f} GB/s (CSR model), "
            f"{al_st:.0f} GB/s (stored)")
    del xa_, ya_
    # the whole solve: every launch's algorithmic bytes (the same 38-step solve,
    # event-timed above) over the graph-replayed time of one solve
    # (the class totals include the few launches profiled without a symbol:
    # vector work, whose bytes are the same under both pricings)
    solve_bytes = sum(v["bytes"] for v in stats.values())
    solve_bytes_csr = (sum(v["bytes_csr"] for v in tagged.values()) + solve_bytes -
                       sum(v["bytes"] for v in tagged.values()))
    solve_gbs = solve_bytes / (ms_step * 1e-3) / 1e9

    # the other workloads: 2D 1024^2 G=1, 2D 256^2 G=20, 2D 512^2 G=20 (FP64 unless stated)
    workloads = {}
    if not a.no_workloads:
        del M32
        for wname, cases in (("g1_2d1024", [("amg", False, False), ("pctl", False, False),
                                            ("schur2_lower", False, False), ("schur1", False, False),
                                            ("schur2", False, False)]),
                             ("g20_2d256", [("bdiag", False, False), ("bdiag", True, True)]),
                             ("g20_2d512", [("schur2", True, True)])):
            ww = si.WORKLOADS[wname]
            winp = si.generate_workload(wname)
            wco = api.Coeffs.from_inputs(ctx, winp)
            wsys = api.BlockSystem.assemble(ctx, wco)
            wb = torch.as_tensor(winp.b, device=ctx.device)
            wn = float(torch.linalg.vector_norm(wb))
            out = {}
            for kind, batched, graph in cases:
                fp32 = wname == "g20_2d512"
                M, su = build(wsys, kind, ww.seed, fp32, batched, graph)
                ms, it, xw, rw = timed(wsys, M, wb, a.form_steps)
                rr = float(torch.linalg.vector_norm(wb - wsys.matvec(xw))) / wn
                key = kind + ("_batched_graph" if batched else "_sequential") + \
                    ("_fp32" if fp32 else "_fp64")
                out[key] = {"ms": ms, "iters": it, "setup_s": su, "relres_true": rr}
                log(f"[bench] {wname} {key}: {ms:.1f} ms/solve, iters {it}, setup {su:.2f}s")
                if wname == "g20_2d512":
                    # adjoint: A^T lambda = x - x_target with Schur2 built on A^T
                    g = xw - torch.as_tensor(winp.x_target, device=ctx.device)
                    MT, sut = build(wsys, kind, ww.seed, fp32, batched, graph, transpose=1)
                    api.adjoint(ctx, wco, wsys, MT, xw, g, rtol=1e-8, flexible=1)
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(a.form_steps):
                        lam, dk, dc, ra = api.adjoint(ctx, wco, wsys, MT, xw, g, rtol=1e-8,
                                                      flexible=1)
                    e1.record()
                    torch.cuda.synchronize()
                    msa = e0.elapsed_time(e1) / a.form_steps
                    out["adjoint_" + key] = {"ms": msa, "iters": ra.iters, "setup_s": sut,
                                             "relres_est": ra.relres_est,
                                             "includes": "adjoint FGMRES and the gradients"}
                    log(f"[bench] {wname} adjoint: {msa:.1f} ms, iters {ra.iters}")
                    del MT
                del M, xw
            if wname == "g20_2d256":
                out["batched_speedup"] = (out["bdiag_sequential_fp64"]["ms"]
                                          / out["bdiag_batched_graph_fp64"]["ms"])
            workloads[wname] = out
            del wsys, wco

    cpu = None
    err_oracle = None
    if not a.no_cpu_baseline:
        log("[bench] oracle CPU baseline on the full workload ...")
        cpu, x_or = cpu_baseline(w.name)
        err_oracle = {"fp32_batched": error_against(x32h, x_or, w.G)}
        if forms:
            err_oracle["fp64_plain"] = error_against(x64h, x_or, w.G)
        err_oracle["against"] = f"oracle FGMRES(30) solution to 1e-8 ({cpu['iters']} iterations)"
    else:
        e = error_against_sample(x32h, w.name, w.G)
        if e is not None:
            err_oracle = {"fp32_batched": e, "against": "stored oracle solution at sample positions"}

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
        "layouts": "autotuned at setup" if a.autotune else "default rules",
        "forms": forms or None,
        "speedup_vs_plain_fp64": (forms["fp64_plain"]["ms"] / ms_step) if forms else None,
        "error_vs_oracle": err_oracle,
        "variants": variants or None,
        "workloads": workloads or None,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(dom), "traffic_unit": "bytes per launch",
                     "bytes_model": "plain CSR: value + 4-byte column per entry, 4-byte row "
                                    "pointer per row, vectors once",
                     "bytes_per_launch": bpl_csr,
                     "bytes_per_launch_stored": bpl,
                     "achieved_stored": achieved_stored,
                     "frac_stored": achieved_stored / HBM_PEAK_GBS,
                     "copy_ceiling": copy_gbs,
                     # the bytes the launch moves as stored, against a device copy's rate
                     "frac_of_copy": achieved_stored / copy_gbs,
                     "launches": s["launches"], "avg_launch_us": avg_us,
                     "standalone": standalone},
        "solve_bandwidth": {"bytes_stored": solve_bytes, "bytes_csr": solve_bytes_csr,
                            "GB/s_stored": solve_gbs, "frac_of_peak": solve_gbs / HBM_PEAK_GBS,
                            "frac_of_copy": solve_gbs / copy_gbs,
                            "time_at_copy_rate_ms": solve_bytes / (copy_gbs * 1e9) * 1e3},
        "kernels": {k: {"ms": v["ms"], "launches": v["launches"],
                        "GB/s": (v["bytes_csr"] / 1e9) / (v["ms"] / 1e3) if v["ms"] else 0.0,
                        "GB/s_stored": (v["bytes"] / 1e9) / (v["ms"] / 1e3) if v["ms"] else 0.0}
                    for k, v in tagged.items()},
        "kernel_classes": {k: {"ms": v["ms"], "launches": v["launches"],
                               "GB/s": (v["bytes"] / 1e9) / (v["ms"] / 1e3) if v["ms"] else 0.0}
                           for k, v in stats.items() if v["launches"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
