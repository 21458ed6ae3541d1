#!/usr/bin/env python3
"""Write the stored reference solution of the 3D 128x64x64 SIMP cantilever
(1,635,075 dofs, 160 subdomains, seed 3) used by the full-size GPU parity
test.

Calls only the oracle (``oracle.reference.refined_solve``: FP64 CPU Schur
route with per-subdomain sparse LU, flexible CG preconditioned by inverse
Lanczos, refined in long double) and the seeded input generator.  Outputs,
next to this script:

  cantilever3d_simp_128x64x64_u_ref.npy   u (FP64, full length, node-major)
  cantilever3d_simp_128x64x64_u_ref.json  compliance, residuals, timings,
                                          host, and this script's sha256

Usage: python tests/golden/make_reference.py [--workers N] [--small]
(--small writes nothing; it runs the same pipeline on a 32x16x16 mesh.)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import fe, reference  # noqa: E402


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--tol", type=float, default=1e-13)
    ap.add_argument("--small", action="store_true")
    args = ap.parse_args()

    def log(s):
        print(f"[reference] {s}", flush=True)

    if args.small:
        w = workloads.cantilever3d_simp(32, 16, 16, ([0, 16, 32], [0, 8, 16], [0, 8, 16]),
                                        seed=3)
    else:
        w = workloads.cantilever3d_simp_128x64x64()
    t0 = time.perf_counter()
    u_ld, rec = reference.refined_solve(w, tol=args.tol, workers=args.workers, log=log)
    wall = time.perf_counter() - t0
    free = ~fe.dirichlet_dof_mask(w)
    c_ld = float(np.sum(w.f.astype(np.longdouble) * u_ld))
    u = np.asarray(u_ld, dtype=np.float64)
    res64 = fe.residual_norm(w, u)
    log(f"compliance {c_ld:.17g}; long-double rel.res {rec['rel_residual']:.3e}; "
        f"FP64 rel.res of the rounded u {res64:.3e}; {wall:.0f} s")
    if args.small:
        ud = fe.solve_direct(w)
        err = np.linalg.norm(u - ud) / np.linalg.norm(ud)
        log(f"against the sparse direct solve: {err:.3e}")
        return
    with open(os.path.abspath(__file__), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    with open(os.path.join(ROOT, "oracle", "reference.py"), "rb") as fh:
        sha_or = hashlib.sha256(fh.read()).hexdigest()
    base = os.path.join(HERE, f"{w.name}_u_ref")
    np.save(base + ".npy", u)
    meta = {
        "workload": w.name,
        "ndof": int(w.ndof),
        "free_dofs": int(free.sum()),
        "kind": "FP64 CPU Schur-PCG reference (per-subdomain sparse LU, flexible CG with "
                "inverse-Lanczos Hhat_0.5, refined with long-double residuals)",
        "compliance": c_ld,
        "rel_residual_long_double": rec["rel_residual"],
        "rel_residual_fp64_of_stored_u": res64,
        "norm_u": float(np.linalg.norm(u)),
        "rounds": rec["rounds"],
        "wall_seconds": round(wall, 1),
        "worker_processes": args.workers,
        "os_cpu_count": os.cpu_count(),
        "cpu_model": cpu_model(),
        "script_sha256": sha,
        "oracle_reference_sha256": sha_or,
    }
    with open(base + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    log(f"wrote {base}.npy and .json")


if __name__ == "__main__":
    main()
