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
