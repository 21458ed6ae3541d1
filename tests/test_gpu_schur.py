"""Explicit local Schur complements (edd_set_s_apply mode 1): S v as the sum
over the subdomains of S_i v_i, with S_i = K^i_GG - K^i_GI (K^i_II)^{-1}
K^i_IG formed on the device from the interior factors.  Against the
oracle's dense S (built from the global blocks, a different computation),
the factor path, and the oracle's direct solve; the S_i are re-formed on
every moduli update."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle import dd, fe

from gpu_util import gamma_check, make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _case2d(seed=31):
    rng = np.random.default_rng(seed)
    p = w.cantilever2d(37, 21, cuts=(np.array([0, 9, 25, 37]), np.array([0, 10, 21])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    return p


def _case3d():
    rng = np.random.default_rng(33)
    p = w.cantilever3d(10, 8, 6, cuts=(np.array([0, 5, 10]), np.array([0, 4, 8]),
                                       np.array([0, 3, 6])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    return p


@pytest.mark.parametrize("dim", [2, 3])
def test_explicit_schur_apply_matches_the_oracle(dim):
    require_gpu()
    wk = _case2d() if dim == 2 else _case3d()
    prob = make_problem(wk, dissect=0)
    gamma_check(wk, prob)
    v = np.random.default_rng(4).standard_normal(prob.info["n_gamma"] * dim)
    y0 = to_np(prob.apply_S(to_cuda(v)))
    prob.set_s_apply(1)
    assert prob.s_apply == 1
    y1 = to_np(prob.apply_S(to_cuda(v)))
    y1b = to_np(prob.apply_S(to_cuda(v)))
    ref = dd.schur_dense(wk) @ v
    e1 = np.linalg.norm(y1 - ref) / np.linalg.norm(ref)
    e0 = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    print(f"{dim}D explicit S_i: vs oracle S {e1:.2e}, vs factor path {e0:.2e}")
    assert e1 <= 1e-12 and e0 <= 1e-12
    assert np.array_equal(y1, y1b)  # deterministic
    prob.set_s_apply(0)
    assert np.array_equal(to_np(prob.apply_S(to_cuda(v))), y0)
    prob.close()


def test_explicit_schur_reformed_on_moduli_update_and_solve():
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = _case2d()
    prob = make_problem(wk, dissect=0)
    prob.set_s_apply(1)
    # new moduli: S_i are formed again
    wk2 = _case2d(seed=32)
    prob.set_element_moduli(torch.tensor(wk2.E, device="cuda", dtype=torch.float64))
    v = np.random.default_rng(5).standard_normal(prob.info["n_gamma"] * 2)
    ref = dd.schur_dense(wk2) @ v
    y = to_np(prob.apply_S(to_cuda(v)))
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    # a whole solve with the explicit S apply against the direct solve
    uref = fe.solve_direct(wk2)
    cref = fe.compliance(wk2.f, uref)
    u, st = prob.solve(to_cuda(wk2.f), tol=1e-12, maxit=5000)
    err = np.linalg.norm(to_np(u) - uref) / np.linalg.norm(uref)
    cerr = abs(st["compliance"] - cref) / abs(cref)
    print(f"explicit S_i solve: {st['iterations']} its, u_err {err:.2e}, c_err {cerr:.2e}")
    assert err <= 1e-8 and cerr <= 1e-10
    # FP32 applies (mixed modes) keep the factor path
    y32 = to_np(prob.apply_S(to_cuda(v), precision=edd.F32))
    assert np.linalg.norm(y32 - ref) <= 1e-2 * np.linalg.norm(ref)
    prob.close()


def test_explicit_schur_refused_for_dissected_interiors():
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = w.cantilever3d(16, 12, 12, cuts=(np.array([0, 7, 16]), np.array([0, 12]),
                                          np.array([0, 5, 12])))
    prob = make_problem(wk, dissect=1)
    with pytest.raises(edd.EddError):
        prob.set_s_apply(1)
    assert prob.s_apply == 0
    prob.close()
