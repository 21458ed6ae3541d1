"""GPU (HIP, gfx950) results against the CPU oracle, called through the
C ABI.  Tolerances: apply_K 1e-14, interior solves 1e-12, S 1e-12, end to
end 1e-8 on displacements and 1e-10 on compliance (FP64 paths)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as w
from oracle import dd, fe

from gpu_util import (gamma_check, interior_perm, make_problem, require_gpu,
                      to_cuda, to_np)

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(11)
    c2 = w.cantilever2d(37, 21, cuts=(np.array([0, 9, 25, 37]), np.array([0, 10, 21])))
    c2.E = 1e-3 + rng.uniform(0, 1, c2.n_el) ** 3
    c3 = w.cantilever3d(13, 9, 7, cuts=(np.array([0, 6, 13]), np.array([0, 4, 9]),
                                        np.array([0, 3, 7])))
    c3.E = 1e-3 + rng.uniform(0, 1, c3.n_el) ** 3
    # interior half-bandwidths 137..257 (> 64): the wide-band substitution
    c3w = w.cantilever3d(16, 12, 12, cuts=(np.array([0, 7, 16]), np.array([0, 12]),
                                           np.array([0, 5, 12])))
    c3w.E = 1e-3 + rng.uniform(0, 1, c3w.n_el) ** 3
    return {"2d": c2, "3d": c3, "3d_wide": c3w, "3d_dissected": c3w,
            "cfg_small": w.cantilever2d_uniform_64x32()}


def _make(name):
    return make_problem(CASES[name], dissect=1 if name == "3d_dissected" else 0)


CASES = _cases()


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_apply_K_parity_and_determinism(name):
    require_gpu()
    wk = CASES[name]
    prob = _make(name)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(wk.ndof)
    ref = fe.apply_K_elementwise(wk, u)
    y1 = prob.apply_K(to_cuda(u))
    y2 = prob.apply_K(to_cuda(u))
    a, b = to_np(y1), to_np(y2)
    assert np.array_equal(a, b)
    assert np.linalg.norm(a - ref) <= 1e-14 * np.linalg.norm(ref)
    prob.close()


@pytest.mark.parametrize("name", ["2d", "3d", "3d_wide", "3d_dissected"])
def test_interior_solve_parity(name):
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = CASES[name]
    prob = _make(name)
    gamma_check(wk, prob)
    perm = interior_perm(wk, prob)
    KII, *_ = dd.blocks(wk)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(prob.n_interior_dofs)
    x = to_np(prob.solve_interior(to_cuda(b)))
    xr = spla.spsolve(KII.tocsc(), b[perm])
    assert np.linalg.norm(x[perm] - xr) <= 1e-12 * np.linalg.norm(xr)
    x32 = to_np(prob.solve_interior(to_cuda(b), precision=edd.F32))
    err32 = np.linalg.norm(x32[perm] - xr) / np.linalg.norm(xr)
    print(f"{name}: FP32 interior solve relative error vs FP64 oracle {err32:.2e}")
    assert err32 < 1e-2
    prob.close()


@pytest.mark.parametrize("name", ["2d", "3d", "3d_wide", "3d_dissected"])
def test_schur_apply_parity(name):
    require_gpu()
    wk = CASES[name]
    prob = _make(name)
    S = dd.schur_dense(wk)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(S.shape[0])
    y = to_np(prob.apply_S(to_cuda(v)))
    ref = S @ v
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    prob.close()


@pytest.mark.parametrize("name", ["2d", "3d", "3d_wide", "3d_dissected", "cfg_small"])
@pytest.mark.parametrize("pc", ["identity"])
def test_solve_parity(name, pc):
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = CASES[name]
    prob = _make(name)
    uref = fe.solve_direct(wk)
    cref = fe.compliance(wk.f, uref)
    u, st = prob.solve(to_cuda(wk.f), tol=1e-13, maxit=5000,
                       precond=edd.PC_IDENTITY)
    un = to_np(u)
    err = np.linalg.norm(un - uref) / np.linalg.norm(uref)
    cerr = abs(st["compliance"] - cref) / abs(cref)
    print(f"{name}: its={st['iterations']} res={st['rel_residual']:.2e} "
          f"u_err={err:.2e} c_err={cerr:.2e}")
    assert err <= 1e-8
    assert cerr <= 1e-10
    # the oracle's own residual of the GPU answer
    assert fe.residual_norm(wk, un) <= 1e-12
    prob.close()


def test_error_paths():
    require_gpu()
    import torch
    from paper_1501_06211_amd import edd
    wk = CASES["2d"]
    prob = edd.Problem.from_workload(wk)
    f = to_cuda(wk.f)
    with pytest.raises(edd.EddError) as e:
        prob.solve(f)
    assert e.value.code == edd.ESTATE
    bad = to_cuda(wk.E)
    bad[3] = -1.0
    with pytest.raises(edd.EddError) as e:
        prob.set_element_moduli(bad)
    assert e.value.code == edd.EINVAL
    bad[3] = float("nan")
    with pytest.raises(edd.EddError) as e:
        prob.set_element_moduli(bad)
    assert e.value.code == edd.EINVAL
    prob.set_element_moduli(to_cuda(wk.E))
    fn = f.clone()
    fn[5] = float("inf")
    with pytest.raises(edd.EddError) as e:
        prob.solve(fn)
    assert e.value.code == edd.EINVAL
    u, st = prob.solve(f, maxit=2, precond=edd.PC_IDENTITY)
    assert st["status"] == edd.NOT_CONVERGED and st["rel_residual"] > 1e-8
    # zero load gives zero displacement
    u0, st0 = prob.solve(torch.zeros_like(f), precond=edd.PC_IDENTITY)
    assert float(u0.abs().max()) == 0.0
    prob.close()


@pytest.mark.parametrize("mode", ["mixed", "relaxed"])
@pytest.mark.parametrize("name", ["2d", "3d", "3d_wide", "3d_dissected"])
def test_mixed_precision_solve(name, mode):
    """Reduced-precision interior factors (interface refinement, or one
    flexible CG with relaxed operator accuracy): the FP64 true residual
    reaches the tolerance and the answer matches the oracle."""
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = CASES[name]
    prob = _make(name)
    uref = fe.solve_direct(wk)
    cref = fe.compliance(wk.f, uref)
    m = edd.MODE_MIXED if mode == "mixed" else edd.MODE_RELAXED
    u, st = prob.solve(to_cuda(wk.f), tol=1e-11, maxit=4000, precision=m,
                       precond=edd.PC_HTHETA, mixed_inner_tol=1e-4)
    un = to_np(u)
    err = float(np.linalg.norm(un - uref) / np.linalg.norm(uref))
    cerr = abs(st["compliance"] - cref) / abs(cref)
    print(f"{name} {mode}: its={st['iterations']} rounds={st['outer_iterations']} "
          f"flags={st['flags']} res={st['rel_residual']:.2e} u_err={err:.2e} c_err={cerr:.2e}")
    assert st["rel_residual"] <= 1e-11
    assert err <= 1e-8 and cerr <= 1e-10
    if mode == "mixed":
        assert st["flags"] & edd.FLAG_MIXED_FALLBACK == 0
    prob.close()
