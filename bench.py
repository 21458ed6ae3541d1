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
        "sha256_prefix": "4cfeff6317e33ba8",
        "workload": "cantilever3d_simp_128x64x64",
        "bytes": 1.5274e+10,
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
                    choices=["3d", "2d", "2d-thresholded", "small", "batch", "sequence",
                             "sequence2d", "topopt"],
                    help="2d-thresholded: the first field of "
                         "the 2D 1024x512 density sequence on its own; "
                         "batch: the 64 uneven problems solved concurrently "
                         "(solves/s and per-problem latency); sequence: a 3D "
                         "128x64x64 density sequence, network trained on the "
                         "first solves, held-out solves timed plain vs learned "
                         "(sequence2d: the same on the 2D 1024x512 cantilever with "
                         "2048 subdomains, the fields of to_sequence_2d); "
                         "topopt: the topology-optimisation loop (OC update, adaptive "
                         "tolerance) on the 2D 1024x512 cantilever with 2048 subdomains, "
                         "and the mesh/subdomain sweep of the paper's Table 3")
    ap.add_argument("--train", type=int, default=40, help="sequence: training solves")
    ap.add_argument("--test", type=int, default=20, help="sequence: held-out solves")
    ap.add_argument("--epochs", type=int, default=20, help="network training epochs")
    ap.add_argument("--precond", default="htheta", choices=["identity", "htheta"])
    ap.add_argument("--headline", default="plain", choices=list(LEG_OPTS),
                    help="the leg whose time is the line's value")
    ap.add_argument("--legs", default="plain,mixed,learned,learned_mixed",
                    help="comma-separated legs timed on the same workload: plain (FP64), "
                         "mixed (FP64 FCG whose S applies move to FP32 interior factors "
                         "once the interface residual has dropped by --switch), learned "
                         "(FP64 with the network's line-searched initial guess), "
                         "learned_mixed (both)")
    ap.add_argument("--switch", type=float, default=1e-2,
                    help="mixed legs: relative interface residual at which the "
                         "S applies move to FP32 factors")
    ap.add_argument("--train-fields", type=int, default=8,
                    help="learned legs: cold solves of other cfg3-shaped moduli fields "
                         "that train the network before the timed steps")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: replay the preconditioner apply from a captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="topopt: skip the Table 3 sweep")
    ap.add_argument("--pc-form", type=int, default=None,
                    help="interface norm form: 0 Htilde inverse Lanczos, 1 H inverse, "
                         "2 Htilde forward (no inner solves), 3 H forward")
    ap.add_argument("--lanczos-k", type=int, default=None, help="Lanczos steps per apply")
    ap.add_argument("--dissect", type=int, default=-1,
                    help="interior dissection rule (edd_mesh_desc.dissect): -1 auto, 0 never, "
                         "1 every interior, 2 only interiors above 1.5x the median band work")
    ap.add_argument("--inner", type=int, default=None, help="inner PCG steps per Lanczos step")
    ap.add_argument("--paper-pc", action="store_true",
                    help="topopt: the paper's adaptive preconditioner form (Lanczos to a "
                         "1e-2 change, inner PCG to 1e-3, at most 12 iterations) instead of "
                         "the fixed 3 x 4 device-resident form")
    ap.add_argument("--variants", default=None,
                    help="V64,V32: substitution variants to use after autotuning (for "
                         "counter runs, where the profiler's overhead can change the "
                         "tuner's pick; the bench line records the variants used)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (5 launches) whose "
                         "known byte count calibrates HBM traffic counters")
    return ap.parse_args()


def make_workload(name):
    import workloads
    if name == "3d":
        return workloads.cantilever3d_simp_128x64x64()
    if name == "2d":
        return workloads.cantilever2d_simp_512x256()
    if name == "2d-thresholded":
        # the first field of the 2D 1024x512 density sequence (E = 1e-3 + rho^3,
        # rho thresholded at the median), 2048 subdomains of 16x16
        w = workloads.cantilever2d(1024, 512, name="cantilever2d_thresholded_1024x512")
        w.E = next(workloads.to_sequence_2d(1, 1024, 512))
        return w
    return workloads.cantilever2d_uniform_64x32()


PC_EXTRA = {}  # preconditioner form and step counts from the command line


def solve_opts(path, precond, tol, switch, graphs=0):
    from paper_1501_06211_amd import edd
    o = dict(tol=tol, maxit=5000, use_graphs=graphs,
             precond=edd.PC_HTHETA if precond == "htheta" else edd.PC_IDENTITY)
    o.update(PC_EXTRA)
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
        ts = time.perf_counter()
        prob.set_element_moduli(E)
        _, st = prob.solve(f, u, **opts)  # synchronises before returning
        st["step_ms"] = (time.perf_counter() - ts) * 1e3
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, iterations, ref_meta=None, nsample=40):
    """The oracle timed on this host's cores on a bounded sample, scaled to
    one whole solve (a model, labelled as such), plus the oracle's full
    reference run of the same workload where one is stored."""
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
    out = {
        "value": total_s * 1e3,
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "modelled": True,
        "sample": (f"MODELLED from a timed sample: {nsample} of {nsub} subdomains "
                   f"(oracle assembly + SuperLU factor and one solve each, "
                   f"{t_fac + t_sol:.1f} s) and one element-by-element K apply of the full "
                   f"mesh ({t_apply:.2f} s), scaled x{scale:.0f} over subdomains and by "
                   f"{iterations} interface iterations; the sample took {sample_s:.1f} s "
                   f"on 1 thread"),
        "host": {"os_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
                 "threads_used": 1},
    }
    if ref_meta is not None:
        first = ref_meta["rounds"][0]
        out["full_oracle_run"] = {
            "what": "measured, not modelled: the oracle's FP64 Schur route on the whole "
                    "workload (per-subdomain sparse LU, flexible CG with inverse-Lanczos "
                    "Hhat_0.5), refined in long double to the stored reference",
            "first_solve_seconds": round(first["seconds"], 1),
            "first_solve_iterations": first["iterations"],
            "first_solve_rel_residual": ref_meta["rounds"][1]["rel_residual"],
            "total_seconds": ref_meta["wall_seconds"],
            "worker_processes": ref_meta["worker_processes"],
            "host_cpu_count": ref_meta["os_cpu_count"],
            "host_cpu_model": ref_meta["cpu_model"],
            "host": "the build container, not this host",
        }
    return out


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


def run_sequence(args, dim=3):
    """Topology-optimisation-like sequence on the 3D 128x64x64 cantilever
    (dim 3) or the 2D 1024x512 cantilever with 16x16-element subdomains
    (dim 2): densities blended 10% per step toward a fresh seeded field and
    thresholded (E = 1e-3 + rho^3).  The first solves (warm-started from the
    previous solution) train the correction network; on the held-out steps
    each solve is timed from the same warm start plain, with the learned
    guess, with the learned guess plus the relaxed mixed precision, and with
    the learned guess plus a network correction step every 4th step."""
    import numpy as np
    import torch

    import workloads
    from paper_1501_06211_amd import edd, learned

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    if dim == 3:
        base = workloads.cantilever3d_simp_128x64x64()
        fields = workloads.to_sequence_3d(args.train + args.test, 128, 64, 64, ell=8.0)
        wl_name = "cantilever3d_sequence_128x64x64"
    else:
        base = workloads.cantilever2d(1024, 512, name="cantilever2d_1024x512")
        fields = workloads.to_sequence_2d(args.train + args.test, 1024, 512)
        wl_name = "cantilever2d_sequence_1024x512"
    seq = [torch.tensor(E, device="cuda") for E in fields]
    print(f"[bench] sequence of {len(seq)} fields in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    prob = edd.Problem.from_workload(base)
    f = torch.tensor(base.f, device="cuda")
    prob.set_element_moduli(seq[0])
    prob.autotune()
    prob.cnn_setup(32)
    prob.cnn_set_params(learned.flatten_params(
        workloads.cnn_initial_weights(dim, dim + 1, 32, dim, seed=1)))
    opts = dict(tol=args.tol, maxit=5000)
    t0 = time.perf_counter()
    tr, u_prev = learned.warm_start_solves(
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
    del tr
    rows = []
    for k, E in enumerate(seq[args.train:]):
        prob.set_element_moduli(E)
        res = {}
        for name, extra in (("plain", {}), ("learned", {"learned_guess": 1}),
                            ("learned_mixed", {"learned_guess": 1,
                                               "precision": edd.MODE_RELAXED,
                                               "mixed_inner_tol": args.switch}),
                            ("learned_corr", {"learned_guess": 1, "learned_correction": 4})):
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
        "metric": "time to rel.res 1e-8 on held-out steps of a %s density sequence: "
                  "plain vs learned vs learned+mixed vs learned+correction" % (
                      "3D 128x64x64" if dim == 3 else "2D 1024x512"),
        "value": round(mean["learned_mixed"], 2), "unit": "ms", "n_gpus": 1,
        "steps": args.test, "warmup": 0, "ms_per_step": round(mean["learned_mixed"], 2),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": wl_name, "train_solves": args.train,
                   "test_solves": args.test, "epochs": args.epochs, "tol": args.tol,
                   "parallelism": "single GPU"},
        "mean_ms": {n: round(v, 2) for n, v in mean.items()},
        "mean_iterations": {n: round(v, 1) for n, v in its.items()},
        "speedup_learned_mixed_vs_plain": round(mean["plain"] / mean["learned_mixed"], 3),
        "speedup_learned_vs_plain": round(mean["plain"] / mean["learned"], 3),
        "speedup_learned_corr_vs_plain": round(mean["plain"] / mean["learned_corr"], 3),
        "training": {"seconds": round(t_train, 2), "loss_first_epoch": round(hist[0], 4),
                     "loss_last_epoch": round(hist[-1], 4)},
        "worst_rel_residual": max(r[n][2] for r in rows for n in r),
    }
    prob.close()
    print(json.dumps(out))


def run_topopt(args):
    """Section 5's fixed-point loop (FEA, OC update, convergence check; the
    Krylov tolerance follows successive compliance values) on the GPU.

    The timed run is the 2D 1024x512 cantilever (1.05M dofs, 2048 subdomains
    of 16x16, VTS, volume fraction 1/2, from a uniform design).  Beside it, the
    sweep of Table 3: meshes 2/h x 1/h for h = 1/16 ... 1/256 with 4, 16, 64
    and 256 regular subdomains (2x2 ... 16x16), theta picked per subdomain
    count as in the paper; fixed-point steps and average interface
    iterations per analysis are reported next to the paper's numbers."""
    import numpy as np
    import torch

    import workloads
    from paper_1501_06211_amd import edd

    def log(s):
        print(f"[bench] {s}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    with open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")) as fh:
        tab3 = json.load(fh)["table3"]

    pc = dict(theta=-1.0, maxit=5000)
    if args.paper_pc:
        # the paper's adaptive form: Lanczos until a 1e-2 change, inner PCG
        # to 1e-3 with at most 12 iterations
        pc.update(lanczos_kmax=20, lanczos_tol=1e-2, inner_tol=1e-3, inner_maxit=12)

    def run(nx, ny, bx, by, maxit=200):
        wk = workloads.cantilever2d(nx, ny, cuts=(workloads.even_cuts(nx, nx // bx),
                                                  workloads.even_cuts(ny, ny // by)))
        prob = edd.Problem.from_workload(wk, factor_precision=edd.F64)
        f = torch.tensor(wk.f, device="cuda")
        rho = torch.full((wk.n_el,), 0.5, dtype=torch.float64, device="cuda")
        # tile shapes and the S apply tuned once per shape class, untimed (VTS:
        # the moduli are the densities)
        prob.set_element_moduli(rho)
        prob.autotune()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho, u, st, hist = prob.topopt(f, rho, maxit=maxit, solve_opts=pc)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prob.close()
        return st, hist, dt

    sweep = []
    if not args.no_sweep:
        for hi, hs in enumerate(tab3["h"]):
            n = int(hs.split("/")[1])
            for di, N in enumerate(tab3["domains"]):
                b = int(round(N ** 0.5))
                if n // b < 2:
                    sweep.append({"h": hs, "domains": N, "mesh": f"{2 * n}x{n}",
                                  "skipped": "subdomains one element thin"})
                    continue
                try:
                    st, hist, dt = run(2 * n, n, b, b)
                except edd.EddError as exc:
                    sweep.append({"h": hs, "domains": N, "mesh": f"{2 * n}x{n}",
                                  "skipped": f"set-up refused: {exc}"})
                    log(f"h={hs} N={N}: skipped ({exc})")
                    continue
                sweep.append({"h": hs, "domains": N, "mesh": f"{2 * n}x{n}", "steps": st["steps"],
                              "avg_iterations": round(st["avg_krylov"], 1),
                              "paper_steps": tab3["steps"][hi][di],
                              "paper_avg_gmres": tab3["avg_gmres"][hi][di],
                              "compliance": st["compliance"], "seconds": round(dt, 2)})
                log(f"h={hs} N={N}: {st['steps']} steps, avg {st['avg_krylov']:.1f} its "
                    f"(paper {tab3['steps'][hi][di]} ({tab3['avg_gmres'][hi][di]})), {dt:.1f} s")
    # the timed run at the sequence configuration's size
    for k in range(args.warmup):
        run(128, 64, 8, 4, maxit=5)
    st, hist, dt = run(1024, 512, 64, 32)
    log(f"1024x512, 2048 subdomains: {st['steps']} steps, {st['krylov_iterations']} iterations "
        f"(avg {st['avg_krylov']:.1f}), {dt:.1f} s; solve {st['t_solve_ms']:.0f} ms, moduli "
        f"{st['t_moduli_ms']:.0f} ms, OC {st['t_update_ms']:.0f} ms")
    out = {
        "metric": "topology optimisation (Section 5): ms per fixed-point step, 2D 1024x512",
        "value": round(1e3 * dt / st["steps"], 3), "unit": "ms", "n_gpus": 1,
        "steps": st["steps"], "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / st["steps"], 3),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "topopt_vts_cantilever2d_1024x512", "subdomains": 2048,
                   "volfrac": 0.5, "change_tol": 1e-2, "tolerance": "adaptive 1e-2..1e-8",
                   "preconditioner": "paper adaptive form" if args.paper_pc else
                   "device-resident 3 Lanczos x 4 inner steps", "theta": "per subdomain count",
                   "parallelism": "single GPU"},
        "run": {"fixed_point_steps": st["steps"], "krylov_iterations": st["krylov_iterations"],
                "avg_iterations": round(st["avg_krylov"], 2), "compliance": st["compliance"],
                "converged": st["converged"], "seconds": round(dt, 2),
                "t_solve_ms": round(st["t_solve_ms"], 1),
                "t_moduli_ms": round(st["t_moduli_ms"], 1),
                "t_update_ms": round(st["t_update_ms"], 1),
                "compliance_history": [round(c, 6) for c in hist[:, 0].tolist()],
                "iterations_history": [int(x) for x in hist[:, 2].tolist()]},
        "table3_sweep": sweep,
    }
    print(json.dumps(out))


LEG_OPTS = {
    # leg: (factor precisions, extra solve options)
    "plain": ("f64", {}),
    "mixed": ("f64+f32", {"mixed": True}),
    "learned": ("f64", {"learned_guess": 1}),
    "learned_mixed": ("f64+f32", {"mixed": True, "learned_guess": 1}),
    # the network also as the direction of every 10th interface step
    "learned_corr": ("f64", {"learned_guess": 1, "learned_correction": 10}),
}


def leg_opts(leg, args):
    from paper_1501_06211_amd import edd
    _, extra = LEG_OPTS[leg]
    o = solve_opts("relaxed" if extra.get("mixed") else "plain", args.precond, args.tol,
                   args.switch, args.graphs)
    if extra.get("learned_guess"):
        o["learned_guess"] = 1
    if extra.get("learned_correction"):
        o["learned_correction"] = extra["learned_correction"]
    return o


def reference_solution(w):
    """The stored oracle reference for this workload, if there is one."""
    import numpy as np
    base = os.path.join(ROOT, "tests", "golden", f"{w.name}_u_ref")
    if not (os.path.exists(base + ".npy") and os.path.exists(base + ".json")):
        return None, None
    with open(base + ".json") as fh:
        meta = json.load(fh)
    return np.load(base + ".npy"), meta


def train_network(prob, args, log):
    """Train the correction network outside the timed region on cold solves
    of cfg3-shaped moduli fields that are not the timed field: pairs
    (E_k, r = f, e = u_k) formed by the library.  Returns the statistics."""
    import numpy as np
    import torch

    import workloads
    from paper_1501_06211_amd import learned
    w0 = make_workload(args.workload)
    t0 = time.perf_counter()
    fields = [torch.tensor(E, device="cuda")
              for E in workloads.simp_sequence_3d(args.train_fields, *w0.nel)]
    t_gen = time.perf_counter() - t0
    f = torch.tensor(w0.f, device="cuda")
    prob.cnn_setup(32)
    prob.cnn_set_params(learned.flatten_params(
        workloads.cnn_initial_weights(w0.dim, 1 + w0.dim, 32, w0.dim, seed=1)))
    zero = torch.zeros_like(f)
    pairs, its = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, E in enumerate(fields):
        prob.set_element_moduli(E)
        u, st = prob.solve(f, **solve_opts("plain", args.precond, args.tol, args.switch))
        r, e = prob.cnn_training_pair(f, zero, u)
        pairs.append({"E": E, "r": r, "e": e})
        its.append(st["iterations"])
    torch.cuda.synchronize()
    t_solves = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = learned.train(prob, pairs, epochs=args.epochs, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"network: {len(fields)} training solves in {t_solves:.1f} s, {args.epochs} epochs "
        f"in {t_train:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    return {"fields": len(fields), "field_kind": "simp_sequence_3d (seeds 7000+k), "
            "not the timed field", "pairs": "cold solves: r = f, e = u_k",
            "solve_iterations": its, "seconds_generate_fields": round(t_gen, 2),
            "seconds_solves": round(t_solves, 2), "epochs": args.epochs,
            "seconds_train": round(t_train, 2), "loss_first_epoch": round(hist[0], 4),
            "loss_last_epoch": round(hist[-1], 4)}


def one_gpu_guard(args):
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 "
                                   "(no multi-GPU path is built)",
                          "n_gpus": args.gpus}))
        sys.exit(2)


def main():
    args = parse()
    one_gpu_guard(args)
    if args.pc_form is not None:
        PC_EXTRA["pc_form"] = args.pc_form
    if args.lanczos_k is not None:
        PC_EXTRA["lanczos_kmax"] = args.lanczos_k
    if args.inner is not None:
        PC_EXTRA["inner_maxit"] = args.inner
    if args.workload in ("sequence", "sequence2d"):
        run_sequence(args, dim=2 if args.workload == "sequence2d" else 3)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "topopt":
        run_topopt(args)
        return
    import numpy as np
    import torch

    from paper_1501_06211_amd import edd

    def log(s):
        print(f"[bench] {s}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 5 x 1 GiB device copies done")
    w = make_workload(args.workload)
    E = torch.tensor(w.E, device="cuda")
    f = torch.tensor(w.f, device="cuda")
    legs = [l for l in args.legs.split(",") if l]
    if w.dim != 3:
        legs = [l for l in legs if not l.startswith("learned")]
    head = args.headline if args.headline in legs else legs[0]
    res, training, info, variants = {}, None, None, None
    params = None
    # one handle per factor-precision set: each path builds only the factors it uses
    for prec_name in ("f64", "f64+f32"):
        group = [l for l in legs if LEG_OPTS[l][0] == prec_name]
        if not group:
            continue
        prec = edd.F64 if prec_name == "f64" else edd.F64 | edd.F32
        prob = edd.Problem.from_workload(w, factor_precision=prec, dissect=args.dissect)
        prob.set_element_moduli(E)
        pv = prob.autotune()  # timed once per shape class, outside the timed region
        if args.variants:
            v64, v32 = (int(x) for x in args.variants.split(","))
            prob.set_solve_variants(v64, v32 if prec != edd.F64 else 0)
            pv = (v64, v32 if prec != edd.F64 else 0) + tuple(pv[2:])
        log(f"{prec_name}: autotuned (substitution FP64, FP32; element tiles all, interior, "
            f"interface): {pv}; S apply {'explicit local Schur complements' if prob.s_apply else 'through the interior factors'}")
        if info is None:
            info, variants = prob.info, list(pv) + [prob.s_apply]
        for leg in group:
            if leg.startswith("learned"):
                if params is None:
                    training = train_network(prob, args, log)
                    params = prob.cnn_get_params()
                else:
                    prob.cnn_setup(32)
                    prob.cnn_set_params(params)
            u = torch.zeros_like(f)
            ms, stats, kt = time_path(prob, E, f, u, leg_opts(leg, args), args.steps,
                                      args.warmup, timing=True)
            res[leg] = {"ms": ms, "stats": stats, "kt": kt, "u": u.cpu().numpy()}
            log(f"{leg}: {ms:.1f} ms/step, its={stats[-1]['iterations']} "
                f"res={stats[-1]['rel_residual']:.2e} flags={stats[-1]['flags']}")
        prob.close()
        del prob

    ms, stats, kt = res[head]["ms"], res[head]["stats"], res[head]["kt"]
    st = stats[-1]
    if st["rel_residual"] > args.tol:
        log(f"WARNING: residual {st['rel_residual']:.2e} above {args.tol}")

    # roofline of the batched interior solve (the dominant byte stream): both
    # triangular sweeps read every band entry once, the dissection couplings
    # twice (separator right-hand side and tail update), right-hand side in
    # and solution out
    def band_roof(kt, name, word):
        n_solve, t_solve = kt[name]
        if not n_solve:
            return None
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
    roof = band_roof(kt, "band_solve", 8)

    u_ref, ref_meta = reference_solution(w)
    u_plain = res["plain"]["u"] if "plain" in res else None

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    leg_out = {}
    for leg, r in res.items():
        s = r["stats"][-1]
        step_ms = sorted(x["step_ms"] for x in r["stats"])
        d = {"ms_per_step": round(r["ms"], 3),
             "step_ms_min_median_max": [round(step_ms[0], 2),
                                        round(float(np.median(step_ms)), 2),
                                        round(step_ms[-1], 2)],
             "solve_ms_per_step": [round(x["t_total_ms"], 2) for x in r["stats"]],
             "iterations": s["iterations"],
             "rel_residual": s["rel_residual"], "compliance": s["compliance"],
             "flags": s["flags"], "factors": LEG_OPTS[leg][0]}
        if LEG_OPTS[leg][1].get("mixed"):
            d["fp32_switch_rel_residual"] = args.switch
        if LEG_OPTS[leg][1].get("learned_guess"):
            d["learned_alpha"] = s["learned_alpha"]
        if u_plain is not None:
            d["u_err_vs_plain_f64"] = rel(r["u"], u_plain)
            d["compliance_err_vs_plain_f64"] = abs(s["compliance"] - res["plain"]["stats"][-1]
                                                   ["compliance"]) / abs(s["compliance"])
            d["speedup_vs_plain"] = round(res["plain"]["ms"] / r["ms"], 3)
        if u_ref is not None:
            d["u_err_vs_reference"] = rel(r["u"], u_ref)
            d["compliance_err_vs_reference"] = abs(s["compliance"] - ref_meta["compliance"]) \
                / abs(ref_meta["compliance"])
        leg_out[leg] = d

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
        "dtype": "f64" if LEG_OPTS[head][0] == "f64" else "f64+f32",
        "data": "synthetic",
        "layout": {"band_blocks": info["band_blocks"], "band_entries": info["factor_entries"],
                   "coupling_entries": info["coupling_entries"],
                   "interior_dofs": info["n_interior_dofs"], "gamma_nodes": info["n_gamma"],
                   "autotuned": {"substitution_fp64": variants[0],
                                 "substitution_fp32": variants[1],
                                 "element_tile_all": variants[2],
                                 "element_tile_interior": variants[3],
                                 "element_tile_interface": variants[4],
                                 "s_apply": "explicit local Schur complements" if variants[5]
                                            else "interior factors"}},
        "config": {"workload": w.name, "ndof": int(w.ndof), "subdomains": int(w.n_sub),
                   "path": head, "precond": args.precond, "tol": args.tol,
                   "step": "set_element_moduli + solve from zero",
                   "parallelism": "single GPU"},
        "solve": {"iterations": st["iterations"], "outer_iterations": st["outer_iterations"],
                  "rel_residual": st["rel_residual"], "compliance": st["compliance"],
                  "flags": st["flags"]},
        "legs": leg_out,
        "kernels_ms": {k: (round(v[1] / v[0], 4) if v[0] else None) for k, v in kt.items()},
        "roofline": roof,
    }
    if "mixed" in res:
        r2 = band_roof(res["mixed"]["kt"], "band_solve32", 4)
        if r2:
            out["roofline_fp32_factors"] = r2
    if training is not None:
        out["training"] = training
    if ref_meta is not None:
        out["reference"] = {"kind": ref_meta["kind"],
                            "rel_residual": ref_meta["rel_residual_long_double"],
                            "file": f"tests/golden/{w.name}_u_ref.npy"}
    if not args.no_cpu_baseline:
        its = res["plain"]["stats"][-1]["iterations"] if "plain" in res else st["iterations"]
        out["cpu_baseline"] = cpu_baseline(w, its, ref_meta) if w.dim == 3 else None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
