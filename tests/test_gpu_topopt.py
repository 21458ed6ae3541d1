"""The topology-optimisation loop of Section 5 on the GPU against the
oracle (oracle/topopt.py): element energies, the OC update with its volume
multiplier, and whole fixed-point runs (tight fixed tolerance against the
oracle's exact solves; adaptive tolerance against the same design)."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle import fe, topopt

from gpu_util import make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _case(dim):
    rng = np.random.default_rng(40 + dim)
    if dim == 2:
        p = w.cantilever2d(37, 21, cuts=(np.array([0, 9, 25, 37]), np.array([0, 10, 21])))
    else:
        p = w.cantilever3d(13, 9, 7, cuts=(np.array([0, 6, 13]), np.array([0, 4, 9]),
                                           np.array([0, 3, 7])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    return p


@pytest.mark.parametrize("dim", [2, 3])
def test_element_energies_parity(dim):
    require_gpu()
    p = _case(dim)
    prob = make_problem(p)
    u = np.random.default_rng(1).standard_normal(p.ndof)
    s = to_np(prob.element_energies(to_cuda(u)))
    ref = topopt.element_energies(p, u)
    err = np.abs(s - ref).max() / np.abs(ref).max()
    print(f"{dim}D element energies: max rel err {err:.2e}")
    assert err <= 1e-13
    prob.close()


@pytest.mark.parametrize("penal,emin", [(1.0, 0.0), (3.0, 1e-3)])
def test_oc_update_parity(penal, emin):
    require_gpu()
    p = _case(2)
    prob = make_problem(p)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.05, 0.95, p.n_el)
    s = 10.0 ** rng.uniform(-3, 2, p.n_el)
    s[::17] = 0.0  # elements that carry no energy
    V = 0.4 * p.n_el
    g = topopt.sensitivity_weights(rho, penal, emin) * s
    ref, lam_ref = topopt.oc_update(rho, g, V)
    new, E_new, res = prob.oc_update(to_cuda(rho), to_cuda(s), V, penal=penal, emin=emin)
    new, E_new = to_np(new), to_np(E_new)
    print(f"OC p={penal}: lambda {res['lambda']:.15e} (oracle {lam_ref:.15e}), "
          f"max |drho| {np.abs(new - ref).max():.2e}")
    assert np.abs(new - ref).max() <= 1e-10
    assert abs(res["lambda"] - lam_ref) <= 1e-9 * lam_ref
    assert abs(res["volume"] - V) <= 1e-9 * V
    assert res["max_change"] == pytest.approx(np.abs(ref - rho).max(), rel=1e-9)
    assert np.allclose(E_new, topopt.moduli(new, penal, emin), rtol=1e-14, atol=0)
    # the volume bound cannot bind / cannot be met
    hi, _, r_hi = prob.oc_update(to_cuda(rho), to_cuda(s), 1.01 * p.n_el, penal=penal, emin=emin)
    assert r_hi["lambda"] == 0.0
    assert np.array_equal(to_np(hi), np.minimum(1.0, rho + 0.2))
    lo, _, r_lo = prob.oc_update(to_cuda(rho), to_cuda(s), 1e-6, penal=penal, emin=emin)
    assert np.isinf(r_lo["lambda"])
    assert np.array_equal(to_np(lo), np.maximum(1e-3, rho - 0.2))
    prob.close()


def _loop_case(dim):
    if dim == 2:
        return w.cantilever2d(32, 16, cuts=(np.array([0, 16, 32]), np.array([0, 8, 16])))
    return w.cantilever3d(16, 8, 8, cuts=(np.array([0, 8, 16]), np.array([0, 8]),
                                          np.array([0, 4, 8])))


@pytest.mark.parametrize("dim", [2, 3])
def test_loop_parity_with_tight_solves(dim):
    """Fixed tolerance 1e-12: the GPU loop follows the oracle loop with exact
    direct solves step for step."""
    require_gpu()
    p = _loop_case(dim)
    ref = topopt.optimise(p, volfrac=0.5, change_tol=1e-2, maxit=60)
    prob = make_problem(p)
    rho = torch.full((p.n_el,), 0.5, dtype=torch.float64, device="cuda")
    rho, u, st, hist = prob.topopt(to_cuda(p.f), rho, maxit=60, adaptive_tol=0, tol_min=1e-12,
                                   solve_opts=dict(maxit=5000))
    c = hist[:, 0]
    print(f"{dim}D loop: {st['steps']} steps (oracle {ref['steps']}), avg its "
          f"{st['avg_krylov']:.1f}, compliance {c[0]:.6f} -> {c[-1]:.6f}")
    assert st["steps"] == ref["steps"]
    assert np.allclose(c, ref["compliance"], rtol=1e-8, atol=0)
    assert np.abs(to_np(rho) - ref["rho"]).max() <= 1e-7
    assert abs(st["volume"] - 0.5 * p.n_el) <= 1e-9 * p.n_el
    prob.close()


def test_loop_with_adaptive_tolerance():
    """The adaptive Krylov tolerance (from successive compliance values)
    reaches the same design as exact solves, with fewer iterations than a
    fixed tight tolerance."""
    require_gpu()
    p = w.cantilever2d(64, 32)
    ref = topopt.optimise(p, volfrac=0.5, change_tol=1e-2, maxit=80)
    prob = make_problem(p)
    f = to_cuda(p.f)
    runs = {}
    for name, kw in (("adaptive", {}), ("fixed", dict(adaptive_tol=0, tol_min=1e-10))):
        rho = torch.full((p.n_el,), 0.5, dtype=torch.float64, device="cuda")
        rho, u, st, hist = prob.topopt(f, rho, maxit=80, **kw)
        runs[name] = (to_np(rho), st, hist)
        print(f"{name}: {st['steps']} steps, {st['krylov_iterations']} iterations "
              f"(avg {st['avg_krylov']:.1f}), tolerances {np.round(np.log10(hist[:, 1]), 1).tolist()}")
    rho_a, st_a, h_a = runs["adaptive"]
    rho_f, st_f, _ = runs["fixed"]
    c_ref = ref["compliance"][-1]
    assert abs(st_a["compliance"] - c_ref) <= 1e-3 * c_ref
    assert abs(st_a["steps"] - ref["steps"]) <= 3
    assert np.abs(rho_a - ref["rho"]).max() <= 2e-2
    assert st_a["krylov_iterations"] < st_f["krylov_iterations"]
    assert h_a[0, 1] == 1e-2 and h_a[:, 1].min() >= 1e-8
    prob.close()


def test_table3_trend():
    """Section 5, Table 3, as a trend on our cantilever (the paper's load,
    clamp side and material are not fully specified): meshes 2/h x 1/h for
    h = 1/16, 1/32, 1/64 with 4 and 16 regular subdomains.  The fixed-point
    step count grows with refinement and does not depend on the subdomain
    count; with Hhat_theta the average interface iterations per analysis
    grow far less under refinement than with S~ = I."""
    require_gpu()
    import json
    import os
    from paper_1501_06211_amd import edd
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "paper_tables.json")))["table3"]
    assert all(a <= b for a, b in zip([r[0] for r in tab["steps"]], [r[0] for r in tab["steps"][1:]]))

    def run(n, b, precond):
        p = w.cantilever2d(2 * n, n, cuts=(w.even_cuts(2 * n, 2 * n // b), w.even_cuts(n, n // b)))
        prob = edd.Problem.from_workload(p, factor_precision=edd.F64)
        rho = torch.full((p.n_el,), 0.5, dtype=torch.float64, device="cuda")
        _, _, st, _ = prob.topopt(to_cuda(p.f), rho, maxit=100,
                                  solve_opts=dict(theta=-1.0, maxit=5000, precond=precond))
        prob.close()
        return st["steps"], st["avg_krylov"]

    res = {(n, b): run(n, b, edd.PC_HTHETA) for n in (16, 32, 64) for b in (2, 4)}
    for key, (steps, its) in sorted(res.items()):
        print(f"  h=1/{key[0]} N={key[1] ** 2}: {steps} steps, avg {its:.1f} iterations")
    for b in (2, 4):
        steps = [res[(n, b)][0] for n in (16, 32, 64)]
        assert steps[0] < steps[1] < steps[2]
    for n in (16, 32, 64):
        assert res[(n, 2)][0] == res[(n, 4)][0]
    ident = {n: run(n, 4, edd.PC_IDENTITY)[1] for n in (16, 64)}
    growth_h = res[(64, 4)][1] / res[(16, 4)][1]
    growth_i = ident[64] / ident[16]
    print(f"  N=16, h 1/16 -> 1/64: iterations x{growth_h:.2f} with Hhat_theta, "
          f"x{growth_i:.2f} with S~ = I")
    assert growth_h < 1.6 and growth_h < growth_i


def test_energies_and_oc_step_at_full_size():
    """One fixed-point step's kernels at the size of the Section 5 run
    (2D 1024x512, 2,048 subdomains): element energies of a solved
    displacement and the OC update with its volume multiplier, against the
    oracle on every element."""
    require_gpu()
    p = w.cantilever2d(1024, 512)  # 16 x 16-element subdomains
    prob = make_problem(p)
    rho = np.full(p.n_el, 0.5)
    prob.set_element_moduli(to_cuda(topopt.moduli(rho, 3.0, 1e-3)))
    u, st = prob.solve(to_cuda(p.f), tol=1e-8, maxit=8000)
    un = to_np(u)
    s = to_np(prob.element_energies(u))
    s_ref = topopt.element_energies(p, un)
    # a solved displacement is smooth: u_e^T K0 u_e is a small difference of
    # terms of the size of |u_e|^T |K0| |u_e|, and both sides round each of
    # the 64 products, so the bar is the forward error bound of that sum
    K0 = fe.element_stiffness(p.dim, p.nu)
    ue = np.where(fe.dirichlet_dof_mask(p), 0.0, un)[fe.element_dofs(p)]
    scale = np.einsum("ei,ij,ej->e", np.abs(ue), np.abs(K0), np.abs(ue))
    es = np.max(np.abs(s - s_ref) / (128 * np.finfo(float).eps * scale))
    V = 0.5 * p.n_el
    g = topopt.sensitivity_weights(rho, 3.0, 1e-3) * s_ref
    ref, lam_ref = topopt.oc_update(rho, g, V)
    new, _, res = prob.oc_update(to_cuda(rho), to_cuda(s_ref), V, penal=3.0, emin=1e-3)
    dr = np.abs(to_np(new) - ref).max()
    print(f"1024x512: {st['iterations']} its; energies at {es:.2f} of the rounding bound; OC lambda "
          f"{res['lambda']:.15e} (oracle {lam_ref:.15e}), max |drho| {dr:.2e}")
    assert es <= 1.0 and dr <= 1e-10
    assert abs(res["lambda"] - lam_ref) <= 1e-9 * lam_ref
    assert abs(res["volume"] - V) <= 1e-9 * V
    prob.close()
