"""Degenerate decompositions against the oracle: subdomains one element
thick (interiors empty across the cut), a single subdomain (no interface),
ragged cut spacing, in 2D and 3D, with both preconditioners."""
import numpy as np
import pytest

import workloads as w
from oracle import fe

from gpu_util import make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(21)
    c = {}
    p = w.cantilever2d(20, 12, cuts=(np.array([0, 1, 9, 10, 20]), np.array([0, 6, 12])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    c["2d_thin"] = p
    p = w.cantilever3d(9, 6, 5, cuts=(np.array([0, 1, 5, 9]), np.array([0, 6]),
                                      np.array([0, 2, 5])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    c["3d_thin"] = p
    p = w.cantilever2d(24, 8, cuts=(np.array([0, 24]), np.array([0, 8])))
    c["2d_single"] = p
    p = w.cantilever3d(10, 6, 6, cuts=(np.array([0, 10]), np.array([0, 6]), np.array([0, 6])))
    c["3d_single"] = p
    return c


CASES = _cases()


@pytest.mark.parametrize("precond", ["identity", "htheta"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_decompositions(name, precond):
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = CASES[name]
    prob = make_problem(wk)
    uref = fe.solve_direct(wk)
    cref = fe.compliance(wk.f, uref)
    pc = edd.PC_IDENTITY if precond == "identity" else edd.PC_HTHETA
    u, st = prob.solve(to_cuda(wk.f), tol=1e-12, maxit=4000, precond=pc)
    un = to_np(u)
    err = float(np.linalg.norm(un - uref) / np.linalg.norm(uref))
    cerr = abs(st["compliance"] - cref) / abs(cref)
    print(f"{name} {precond}: n_gamma={prob.n_gamma} its={st['iterations']} "
          f"res={st['rel_residual']:.2e} u_err={err:.2e} c_err={cerr:.2e}")
    assert err <= 1e-8 and cerr <= 1e-10
    prob.close()


def test_fp32_moduli_input():
    """EDD_F32 moduli: the library widens them to FP64, so K is the oracle's
    K of the FP32-rounded moduli (apply to 1e-14; solution to 1e-8)."""
    require_gpu()
    import torch
    from paper_1501_06211_amd import edd
    rng = np.random.default_rng(31)
    p = w.cantilever2d(20, 12, cuts=(np.array([0, 10, 20]), np.array([0, 6, 12])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    E32 = p.E.astype(np.float32)
    prob = edd.Problem.from_workload(p, factor_precision=edd.F64)
    prob.set_element_moduli(torch.tensor(E32, device="cuda"))
    E_widened = E32.astype(np.float64)
    v = rng.standard_normal(p.ndof)
    y = to_np(prob.apply_K(to_cuda(v)))
    ref = fe.apply_K_elementwise(p, v, E_widened)
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)
    u, st = prob.solve(to_cuda(p.f), tol=1e-12, maxit=3000)
    uref = fe.solve_direct(p, E_widened)
    assert np.linalg.norm(to_np(u) - uref) <= 1e-8 * np.linalg.norm(uref)
    prob.close()


def test_zero_network_proposal_is_dropped():
    """With all-zero network parameters the proposal is zero, its interface
    energy is zero, and the solve drops it (EDD_FLAG_LEARNED_REJECTED)
    and solves as without it."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p = w.cantilever2d(32, 16, cuts=(np.array([0, 16, 32]), np.array([0, 8, 16])))
    prob = make_problem(p)
    assert prob.cnn_setup(32) > 0  # parameters start at zero
    f = to_cuda(p.f)
    u0, s0 = prob.solve(f, tol=1e-10)
    u1, s1 = prob.solve(f, tol=1e-10, learned_guess=1)
    assert s1["flags"] & edd.FLAG_LEARNED_REJECTED
    assert s1["learned_alpha"] == 0.0
    assert s1["iterations"] == s0["iterations"]
    assert np.array_equal(to_np(u0), to_np(u1))
    prob.close()


def test_skeleton_away_from_the_clamp():
    """Two subdomains side by side along x: the one interface line has no
    cross point and does not meet the clamp, so its face block of L is the
    singular Neumann Laplacian (the face preconditioner falls back to the
    diagonal).  Set-up succeeds and S~ = I solves to the oracle's answer."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p = w.cantilever2d(32, 16, cuts=(np.array([0, 16, 32]), np.array([0, 16])))
    p.E = 1e-3 + np.random.default_rng(4).uniform(0, 1, p.n_el) ** 3
    prob = make_problem(p)
    u, st = prob.solve(to_cuda(p.f), tol=1e-12, maxit=2000, precond=edd.PC_IDENTITY)
    uref = fe.solve_direct(p)
    assert np.linalg.norm(to_np(u) - uref) <= 1e-8 * np.linalg.norm(uref)
    prob.close()


def test_wrong_length_and_device_arguments_raise_before_any_call():
    """The binding checks every tensor's length against the problem before
    it calls the library (no launch ever sees a short buffer)."""
    require_gpu()
    import torch
    from paper_1501_06211_amd import edd
    p = w.cantilever2d(16, 8, cuts=(np.array([0, 8, 16]), np.array([0, 8])))
    prob = make_problem(p)
    short = torch.zeros(p.ndof - 1, dtype=torch.float64, device="cuda")
    good = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    nG = prob.n_gamma * 2
    for call in (lambda: prob.apply_K(short),
                 lambda: prob.apply_K(good, out=short),
                 lambda: prob.solve(short),
                 lambda: prob.solve(good, short),
                 lambda: prob.apply_S(torch.zeros(nG + 1, dtype=torch.float64, device="cuda")),
                 lambda: prob.solve_interior(torch.zeros(3, dtype=torch.float64, device="cuda")),
                 lambda: prob.set_element_moduli(torch.ones(p.n_el - 1, dtype=torch.float64,
                                                            device="cuda")),
                 lambda: prob.apply_K(good.float()),
                 lambda: prob.apply_K(good.cpu())):
        with pytest.raises(ValueError):
            call()
    prob.close()
