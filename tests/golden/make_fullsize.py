"""Write the oracle's results on the full-size workloads for the GPU parity
tests.  Calls only ``oracle`` and ``synth_inputs``.

    python tests/golden/make_fullsize.py [workload ...]

For every (workload, preconditioner kind) of CASES it stores, in
fullsize_<workload>.json:
  * per inverse role and AMG level: rows, entries of A_l and P_l, PMIS rounds
    and digests of the C/F marker, A_l and P_l (byte forms in
    fullsize_format.py);
  * FGMRES(30) from x0 = 0 to rtol 1e-8 (Section 4 with the stop test of
    reading A1): iteration count, restarts, estimated and true relative
    residuals, the residual history;
  * per block segment the 2-norm and max-norm of the solution;
and in fullsize_<workload>.npz the solution at the sample positions of
fullsize_format.sample_positions.  For the adjoint case (Section 2's system
transposed) the same is stored for lambda = A^-T (x - x_target), with the
coefficient gradients at the sample positions.  Host times are recorded for
information only.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import fullsize_format as ff  # noqa: E402
import synth_inputs as si  # noqa: E402
from oracle import adjoint as oadj  # noqa: E402
from oracle import amg as oamg  # noqa: E402
from oracle import assemble as oasm  # noqa: E402
from oracle import krylov as okry  # noqa: E402
from oracle import precond as opc  # noqa: E402

# workload -> preconditioner kinds (FP64 throughout; the AMG seed is the workload seed)
CASES = {
    "g20_3d64": ["schur2", "schur1", "pctl"],
    "g20_2d256": ["bdiag"],
    "g1_2d1024": ["amg", "pctl", "schur2_lower", "schur1", "schur2"],
    "g20_2d512": ["schur2", "adjoint_schur2"],
}


def log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, file=sys.stderr, flush=True)


def role_name(key) -> str:
    return f"g{key[1]}" if isinstance(key, tuple) else key


def hierarchy_record(H: oamg.Hierarchy):
    levels = []
    for L in H.levels:
        rec = {"n": int(L.A.shape[0]), "nnz": int(L.A.nnz),
               "A": ff.digest_csr(L.A.indptr, L.A.indices, L.A.data)}
        if L.cf is not None:
            rec.update({"nnz_P": int(L.P.nnz), "rounds": int(L.pmis_rounds),
                        "cf": ff.digest_cf(L.cf),
                        "P": ff.digest_csr(L.P.indptr, L.P.indices, L.P.data)})
        levels.append(rec)
    return {"levels": levels, "coarse_kind": H.coarse_kind}


def precond_record(M: opc.BlockPreconditioner):
    out = {}
    for key, inv in M.inv.items():
        H = getattr(inv, "hierarchy", None)
        if H is not None:
            out[role_name(key)] = hierarchy_record(H)
    if M.kind == "pctl":
        out["pctl_p_cycles"] = [int(c) for c in M.setup_info["p_cycles"]]
    return out


def gmres_record(info: okry.GmresInfo, t_solve: float):
    return {"iters": info.iters, "restarts": info.restarts, "converged": bool(info.converged),
            "relres_est": info.relres_est, "relres_true": info.relres_true,
            "history": list(info.history), "host_solve_s": t_solve}


def run_case(inp, osys, kind, seed, arrays, pos, x_forward=None):
    G = inp.G
    params = opc.BlockParams(kind=kind.replace("adjoint_", ""), amg=oamg.AMGParams(seed=seed))
    if kind.startswith("adjoint_"):
        sysm = osys.transpose()
        rhs = x_forward - inp.x_target
    else:
        sysm = osys
        rhs = inp.b
    t0 = time.perf_counter()
    M = opc.BlockPreconditioner(sysm, params)
    t1 = time.perf_counter()
    log(f"  {kind}: setup {t1 - t0:.1f} s")
    x, info = okry.gmres(sysm.matvec, M, rhs, rtol=1e-8, flexible=True)
    t2 = time.perf_counter()
    log(f"  {kind}: {info.iters} iterations, relres {info.relres_true:.3e}, solve {t2 - t1:.1f} s")
    rec = {"hierarchies": precond_record(M), "gmres": gmres_record(info, t2 - t1),
           "host_setup_s": t1 - t0}
    n2, ninf = ff.segment_norms(x, G + 2)
    rec["x_norm2"], rec["x_norminf"] = n2, ninf
    arrays[f"{kind}/x"] = x[pos]
    if kind.startswith("adjoint_"):
        dk, dgE, dEg, dEI = oadj.gradients(inp, x_forward, x)
        dc = np.concatenate([dgE.reshape(-1), dEg.reshape(-1), dEI])
        arrays[f"{kind}/dL_dkappa"] = dk.reshape(-1)[pos]
        pos_c = ff.sample_positions(2 * G + 1, inp.N)
        arrays[f"{kind}/dL_dc_pos"] = pos_c
        arrays[f"{kind}/dL_dc"] = dc[pos_c]
        rec["rhs"] = "x - x_target with x the oracle's forward solution of the schur2 case"
    return rec, x


def main(argv):
    names = argv or list(CASES)
    for name in names:
        w = si.WORKLOADS[name]
        log(f"{name}: G={w.G} {w.dim}D {w.n}^{w.dim}, {w.n_unknowns} unknowns")
        inp = si.generate_workload(name)
        osys = oasm.assemble(inp)
        pos = ff.sample_positions(w.G + 2, w.N)
        arrays = {"pos": pos}
        out = {"workload": name, "G": w.G, "dim": w.dim, "n": w.n, "seed": w.seed,
               "restart": 30, "rtol": 1e-8, "flexible": True,
               "host": {"machine": platform.processor() or platform.machine(),
                        "cpus": len(os.sched_getaffinity(0))},
               "cases": {}}
        x_fwd = None
        for kind in CASES[name]:
            rec, x = run_case(inp, osys, kind, w.seed, arrays, pos, x_forward=x_fwd)
            if kind == "schur2":
                x_fwd = x
            out["cases"][kind] = rec
        jpath, npath = ff.paths(name)
        with open(jpath, "w") as f:
            json.dump(out, f, indent=1)
        np.savez_compressed(npath, **arrays)
        log(f"{name}: wrote {os.path.basename(jpath)}, {os.path.basename(npath)}")


if __name__ == "__main__":
    main(sys.argv[1:])
