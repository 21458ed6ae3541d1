#!/usr/bin/env python3
"""Time to relative residual 1e-8 for the 3D 128x64x64 hexahedral cantilever
(1.6M dofs, 160 uneven subdomains) on one MI355X.

A step is one pass of the whole hot path on resident inputs: set the element
moduli (assembly and band Cholesky of every interior block) and solve
K u = f by condensation, interface Krylov iteration and back-substitution
until ||f - K u|| <= 1e-8 ||f|| (checked with an FP64 K apply).  The
headline path (default: plain FP64) is timed, and beside it the mixed
path (one flexible CG whose Schur applies move from FP64 to FP32 interior
factors once the interface residual has dropped by 10x, with an FP64
restart if that phase stalls); the JSON line reports the headline as
``value`` (milliseconds per step, lower is better).

Also reported:
  roofline      the batched interior solve (the dominant byte stream; with
                dissected interiors it is five launches: forward sweeps,
                separator right-hand sides, separator solves, tail updates,
                backward sweeps, timed as one unit): algorithmic bytes per
                call (every band entry read twice, the dissection couplings
                twice, right-hand side in, solution out) over its average
                duration, from HIP events on the solver's stream during the
                timed steps, against 8 TB/s
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
                (40 subdomain factorisations + solves, one element-by-element
                K apply), scaled to the whole solve
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled
# by a 1 GiB copy calibration), keyed by kernel; valid only while the kernel
# source and the workload are the ones the counters were taken on.
MEASURED_TRAFFIC = {
    "interior_solve<double>": {
        "source": "paper_1501_06211_amd/csrc/kernels_band.hip",
        "sha256_prefix": "15cef711506d7c9f",
        "workload": "cantilever3d_simp_128x64x64",
        "bytes": 1.4705e+10,
        "profile": "profiles/hbm_counters_interior_solve_cantilever3d_simp_128x64x64.md",
    },
}


def measured_traffic(kernel, workload):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if not m or m["workload"] != workload:
        return None
    with open(os.path.join(ROOT, m["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest()[:16] != m["sha256_prefix"]:
            return None
    return m["bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="3d",
                    choices=["3d", "2d", "small", "batch", "sequence"],
                    help="batch: the 64 uneven problems solved concurrently "
                         "(solves/s and per-problem latency); sequence: a 3D "
                         "128x64x64 density sequence, network trained on the "
                         "first solves, held-out solves timed plain vs learned")
    ap.add_argument("--train", type=int, default=40, help="sequence: training solves")
    ap.add_argument("--test", type=int, default=20, help="sequence: held-out solves")
    ap.add_argument("--epochs", type=int, default=20, help="sequence: training epochs")
    ap.add_argument("--precond", default="htheta", choices=["identity", "htheta"])
    ap.add_argument("--headline", default="plain",
                    choices=["plain", "mixed", "relaxed"])
    ap.add_argument("--switch", type=float, default=0.1,
                    help="relaxed path: relative interface residual at which the "
                         "S applies move to FP32 factors")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: replay the preconditioner apply from a captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (5 launches) whose "
                         "known byte count calibrates HBM traffic counters")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip timing the plain FP64 path when it is not the headline")
    return ap.parse_args()


def make_workload(name):
    import workloads
    if name == "3d":
        return workloads.cantilever3d_simp_128x64x64()
    if name == "2d":
        return workloads.cantilever2d_simp_512x256()
    return workloads.cantilever2d_uniform_64x32()


def solve_opts(path, precond, tol, switch, graphs=0):
    from paper_1501_06211_amd import edd
    o = dict(tol=tol, maxit=5000, use_graphs=graphs,
             precond=edd.PC_HTHETA if precond == "htheta" else edd.PC_IDENTITY)
    if path == "mixed":
        o.update(precision=edd.MODE_MIXED)
    elif path == "relaxed":
        o.update(precision=edd.MODE_RELAXED, mixed_inner_tol=switch)
    return o


def time_path(prob, E, f, u, opts, steps, warmup, timing=False):
    import torch
    for k in range(warmup):
        prob.set_element_moduli(E)
        _, st = prob.solve(f, u, **opts)
        print(f"[bench]   warmup {k}: its={st['iterations']} res={st['rel_residual']:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if timing:
        prob.set_kernel_timing(True)
    stats = []
    t0 = time.perf_counter()
    for k in range(steps):
        prob.set_element_moduli(E)
        _, st = prob.solve(f, u, **opts)
        stats.append(st)
        print(f"[bench]   step {k}: its={st['iterations']} outer={st['outer_iterations']} "
              f"res={st['rel_residual']:.2e} {st['t_total_ms']:.1f} ms (solve)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = prob.kernel_times() if timing else None
    if timing:
        prob.set_kernel_timing(False)
    return (t1 - t0) * 1e3 / steps, stats, kt


def sub_problem(w, sid):
    """The element block of subdomain ``sid`` as its own problem, with every
    face that is a clamp or an internal cut held fixed: its free system is
    exactly the interior block K_{I_i I_i}."""
    import numpy as np
    import workloads
    nb = [len(c) - 1 for c in w.cuts]
    b = [sid % nb[0], (sid // nb[0]) % nb[1], sid // (nb[0] * nb[1])]
    lo = [int(w.cuts[a][b[a]]) for a in range(3)]
    hi = [int(w.cuts[a][b[a] + 1]) for a in range(3)]
    E3 = w.E.reshape(w.nel[2], w.nel[1], w.nel[0])
    Es = E3[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].reshape(-1)
    dims = [hi[a] - lo[a] for a in range(3)]
    sub = workloads.cantilever3d(*dims, cuts=([0, dims[0]], [0, dims[1]], [0, dims[2]]),
                                 E=Es)
    clamp = 0
    for a in range(3):
        if lo[a] > 0 or (w.clamp >> (2 * a)) & 1:
            clamp |= 1 << (2 * a)
        if hi[a] < w.nel[a] or (w.clamp >> (2 * a + 1)) & 1:
            clamp |= 1 << (2 * a + 1)
    sub.clamp = clamp
    return sub


def cpu_baseline(w, iterations, nsample=40):
    """Oracle timings on a sample, scaled to one whole solve."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits

    from oracle import fe
    nsub = w.n_sub
    sids = np.linspace(0, nsub - 1, nsample).round().astype(int)
    with threadpool_limits(1):
        t_fac = t_sol = 0.0
        for s in sids:
            sub = sub_problem(w, int(s))
            t0 = time.perf_counter()
            Kff, _ = fe.free_system(sub)
            lu = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A")
            t1 = time.perf_counter()
            lu.solve(np.ones(Kff.shape[0]))
            t2 = time.perf_counter()
            t_fac += t1 - t0
            t_sol += t2 - t1
        rng = np.random.default_rng(0)
        u = rng.standard_normal(w.ndof)
        t0 = time.perf_counter()
        fe.apply_K_elementwise(w, u)
        t_apply = time.perf_counter() - t0
    scale = nsub / nsample
    # per interface iteration: one interior solve of every subdomain and two
    # element sweeps; plus the factorisations, condensation and back-substitution
    total_s = scale * t_fac + (iterations + 2) * (scale * t_sol) + (iterations + 1) * 2 * t_apply
    sample_s = t_fac + t_sol + t_apply
    return {
        "value": total_s * 1e3,
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{nsample} of {nsub} subdomains: oracle assembly + SuperLU factor "
                   f"and one solve each ({t_fac + t_sol:.1f} s), one element-by-element "
                   f"K apply of the full mesh ({t_apply:.2f} s); scaled x{scale:.0f} "
                   f"over subdomains and by {iterations} interface iterations "
                   f"(sample took {sample_s:.1f} s, 1 thread)"),
    }


def run_batch(args):
    """64 independent problems (32 2D, 32 3D, uneven sizes, own moduli and
    loads) solved concurrently to 1e-8 through edd_solve_batch, each handle
    on its own stream, substitution variants autotuned per shape class."""
    import numpy as np
    import torch

    import workloads
    from paper_1501_06211_amd import edd

    torch.cuda.set_device(0)
    ws = [workloads.batch_uneven_problem(p) for p in range(64)]
    probs, fs, us = [], [], []
    for wk in ws:
        prob = edd.Problem.from_workload(wk, stream=torch.cuda.Stream())
        prob.set_element_moduli(torch.tensor(wk.E, device="cuda"))
        prob.autotune()
        probs.append(prob)
        fs.append(torch.tensor(wk.f, device="cuda"))
        us.append(torch.zeros(wk.ndof, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    opts = solve_opts(args.headline, args.precond, args.tol, args.switch, args.graphs)
    for k in range(args.warmup):
        rc, stats = edd.solve_batch(probs, fs, us, **opts)
        print(f"[bench]   warmup {k}: status {rc}", file=sys.stderr, flush=True)
    lat, its, worst = [], [], 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rc, stats = edd.solve_batch(probs, fs, us, **opts)
        lat += [s["t_total_ms"] for s in stats]
        its += [s["iterations"] for s in stats]
        worst = max(worst, max(s["rel_residual"] for s in stats))
        print(f"[bench]   step {k}: status {rc}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = {
        "metric": "batched uneven solves per second (64 problems, rel.res 1e-8)",
        "value": round(len(ws) / dt, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 2),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64" if args.headline == "plain" else "f64+f32", "data": "synthetic",
        "config": {"workload": "batch_uneven_64", "problems": len(ws), "path": args.headline,
                   "graphs": args.graphs,
                   "precond": args.precond, "tol": args.tol, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                       "p99": round(float(np.percentile(lat, 99)), 2),
                       "max": round(float(max(lat)), 2)},
        "iterations": {"p50": int(np.percentile(its, 50)), "max": int(max(its))},
        "worst_rel_residual": worst,
    }
    for prob in probs:
        prob.close()
    print(json.dumps(out))


def run_sequence(args):
    """Topology-optimisation-like sequence on the 3D 128x64x64 cantilever:
    densities blended 10% per step toward a fresh seeded field and
    thresholded (E = 1e-3 + rho^3).  The first solves (warm-started from the
    previous solution) train the correction network; on the held-out steps
    each solve is timed from the same warm start plain, with the learned
    guess, and with the learned guess plus the relaxed mixed precision."""
    import numpy as np
    import torch

    import workloads
    from paper_1501_06211_amd import edd, learned

    torch.cuda.set_device(0)
    base = workloads.cantilever3d_simp_128x64x64()
    t0 = time.perf_counter()
    seq = [torch.tensor(E, device="cuda")
           for E in workloads.to_sequence_3d(args.train + args.test, 128, 64, 64, ell=8.0)]
    print(f"[bench] sequence of {len(seq)} fields in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    prob = edd.Problem.from_workload(base)
    f = torch.tensor(base.f, device="cuda")
    prob.set_element_moduli(seq[0])
    prob.autotune()
    prob.cnn_setup(32)
    prob.cnn_set_params(learned.flatten_params(
        workloads.cnn_initial_weights(3, 4, 32, 3, seed=1)))
    opts = dict(tol=args.tol, maxit=5000)
    t0 = time.perf_counter()
    tr = learned.warm_start_solves(
        prob, f, seq[:args.train],
        log=lambda s: print("[bench]   training " + s, file=sys.stderr, flush=True), **opts)
    print(f"[bench] {args.train} training solves in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = learned.train(prob, tr, epochs=args.epochs, lr=1e-3,
                         log=lambda s: print("[bench]   " + s, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    u_prev = sum(r["e"] for r in tr)
    del tr
    rows = []
    for k, E in enumerate(seq[args.train:]):
        prob.set_element_moduli(E)
        res = {}
        for name, extra in (("plain", {}), ("learned", {"learned_guess": 1}),
                            ("learned_mixed", {"learned_guess": 1,
                                               "precision": edd.MODE_RELAXED,
                                               "mixed_inner_tol": args.switch})):
            torch.cuda.synchronize()
            t = time.perf_counter()
            u, st = prob.solve(f, u_prev.clone(), use_initial_guess=1, **opts, **extra)
            torch.cuda.synchronize()
            res[name] = (1e3 * (time.perf_counter() - t), st["iterations"], st["rel_residual"],
                         st["learned_alpha"])
            if name == "plain":
                u_next = u
        rows.append(res)
        print(f"[bench]   held-out step {k}: " + " ".join(
            f"{n}={v[0]:.0f}ms/{v[1]}its" for n, v in res.items()), file=sys.stderr, flush=True)
        u_prev = u_next
    mean = {n: float(np.mean([r[n][0] for r in rows])) for n in rows[0]}
    its = {n: float(np.mean([r[n][1] for r in rows])) for n in rows[0]}
    out = {
        "metric": "time to rel.res 1e-8 on held-out steps of a 3D 128x64x64 density sequence: "
                  "plain vs learned vs learned+mixed",
        "value": round(mean["learned_mixed"], 2), "unit": "ms", "n_gpus": 1,
        "steps": args.test, "warmup": 0, "ms_per_step": round(mean["learned_mixed"], 2),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "cantilever3d_sequence_128x64x64", "train_solves": args.train,
                   "test_solves": args.test, "epochs": args.epochs, "tol": args.tol,
                   "parallelism": "single GPU"},
        "mean_ms": {n: round(v, 2) for n, v in mean.items()},
        "mean_iterations": {n: round(v, 1) for n, v in its.items()},
        "speedup_learned_mixed_vs_plain": round(mean["plain"] / mean["learned_mixed"], 3),
        "speedup_learned_vs_plain": round(mean["plain"] / mean["learned"], 3),
        "training": {"seconds": round(t_train, 2), "loss_first_epoch": round(hist[0], 4),
                     "loss_last_epoch": round(hist[-1], 4)},
        "worst_rel_residual": max(r[n][2] for r in rows for n in r),
    }
    prob.close()
    print(json.dumps(out))


def main():
    args = parse()
    if args.workload == "sequence":
        if args.gpus != 1:
            print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                              "n_gpus": args.gpus}))
            sys.exit(2)
        run_sequence(args)
        return
    if args.workload == "batch":
        if args.gpus != 1:
            print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                              "n_gpus": args.gpus}))
            sys.exit(2)
        run_batch(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1501_06211_amd import edd

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        del src, dst
        print("[bench] copy calibration: 5 x 1 GiB device copies done",
              file=sys.stderr, flush=True)
    w = make_workload(args.workload)
    E = torch.tensor(w.E, device="cuda")
    f = torch.tensor(w.f, device="cuda")
    u = torch.zeros_like(f)

    head = args.headline
    res = {}
    other = "relaxed" if head == "plain" else "plain"
    paths = [head] if args.no_plain else [head, other]
    for path in paths:
        # each path sets up only the factor precisions it uses: the plain
        # path FP64, the mixed paths FP64 and FP32
        prec = edd.F64 if path == "plain" else edd.F64 | edd.F32
        prob = edd.Problem.from_workload(w, factor_precision=prec)
        # substitution variants: timed once per shape class, outside the
        # timed region (the choice is cached for later handles)
        prob.set_element_moduli(E)
        pv = prob.autotune()
        print(f"[bench] {path}: autotuned substitution variants (FP64, FP32): {pv}",
              file=sys.stderr, flush=True)
        ms, stats, kt = time_path(prob, E, f, u,
                                  solve_opts(path, args.precond, args.tol, args.switch, args.graphs),
                                  args.steps, args.warmup, timing=True)
        res[path] = (ms, stats, kt)
        if path == head:
            info, variants = prob.info, pv
        prob.close()
        print(f"[bench] {path}: {ms:.1f} ms/step, its={stats[-1]['iterations']} "
              f"outer={stats[-1]['outer_iterations']} res={stats[-1]['rel_residual']:.2e}",
              file=sys.stderr, flush=True)
    ms, stats, kt = res[head]
    st = stats[-1]
    if st["rel_residual"] > args.tol:
        print(f"[bench] WARNING: residual {st['rel_residual']:.2e} above {args.tol}",
              file=sys.stderr)

    # roofline of the batched substitution kernel (the dominant byte stream):
    # both triangular sweeps read every band entry once, plus the right-hand
    # side in and the solution out, FP64
    def band_roof(name, word):
        n_solve, t_solve = kt[name]
        if not n_solve:
            return None
        # the dissection couplings are read twice (separator right-hand
        # side and tail update)
        bytes_per_launch = (2 * info["factor_entries"] * word
                            + 2 * info["coupling_entries"] * word
                            + 16 * info["n_interior_dofs"])
        avg_ms = t_solve / n_solve
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        kname = "interior_solve<%s>" % ("double" if word == 8 else "float")
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname, w.name),
                "kernel": kname,
                "avg_launch_ms": round(avg_ms, 4), "launches": n_solve,
                "total_ms": round(t_solve, 2), "bytes_per_launch": bytes_per_launch}
    roofs = [r for r in (band_roof("band_solve", 8), band_roof("band_solve32", 4)) if r]
    roofs.sort(key=lambda r: -r["total_ms"])
    roof = roofs[0]

    out = {
        "metric": "time to rel.res 1e-8, 3D 1.6M dofs: plain vs learned+mixed; HBM GB/s frac",
        "value": round(ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if head == "plain" else "f64+f32",
        "data": "synthetic",
        "layout": {"band_blocks": info["band_blocks"], "band_entries": info["factor_entries"],
                   "coupling_entries": info["coupling_entries"],
                   "interior_dofs": info["n_interior_dofs"], "gamma_nodes": info["n_gamma"],
                   "substitution_variants": list(variants)},
        "config": {"workload": w.name, "ndof": int(w.ndof), "subdomains": int(w.n_sub),
                   "path": head, "precond": args.precond, "tol": args.tol,
                   "parallelism": "single GPU"},
        "solve": {"iterations": st["iterations"], "outer_iterations": st["outer_iterations"],
                  "rel_residual": st["rel_residual"], "compliance": st["compliance"],
                  "flags": st["flags"]},
        "kernels_ms": {k: (round(v[1] / v[0], 4) if v[0] else None) for k, v in kt.items()},
        "roofline": roof,
    }
    if len(roofs) > 1:
        out["roofline_second"] = roofs[1]
    if other in res:
        om, ost, _ = res[other]
        key = "plain_f64" if other == "plain" else "mixed_relaxed"
        out[key] = {"ms_per_step": round(om, 3), "iterations": ost[-1]["iterations"],
                    "rel_residual": ost[-1]["rel_residual"],
                    "compliance": ost[-1]["compliance"], "flags": ost[-1]["flags"],
                    "speedup_vs_headline": round(ms / om, 3)}
        out["compliance_rel_diff"] = abs(st["compliance"] - ost[-1]["compliance"]) / abs(ost[-1]["compliance"])
    if not args.no_cpu_baseline:
        its = res["plain"][1][-1]["iterations"] if "plain" in res else st["iterations"]
        out["cpu_baseline"] = cpu_baseline(w, its) if w.dim == 3 else None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
