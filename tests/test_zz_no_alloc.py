"""edd_apply_S_noalloc (work vector in a static device array) against
edd_apply_S (work vector in the handle's buffer), both called through the C
ABI: two calls in a row on different problems, the second one smaller, in
both factor precisions.  Same kernels in the same order, so the results
must be bitwise equal."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as w
from gpu_util import make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _case_3d():
    rng = np.random.default_rng(21)
    c = w.cantilever3d(16, 12, 12, cuts=(np.array([0, 7, 16]), np.array([0, 12]),
                                         np.array([0, 5, 12])))
    c.E = 1e-3 + rng.uniform(0, 1, c.n_el) ** 3
    return c, 1


def _case_2d():
    rng = np.random.default_rng(22)
    c = w.cantilever2d(37, 21, cuts=(np.array([0, 9, 25, 37]), np.array([0, 10, 21])))
    c.E = 1e-3 + rng.uniform(0, 1, c.n_el) ** 3
    return c, 0


def _call(fn, prob, v, y, prec):
    rc = fn(prob.h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(y.data_ptr()), prec)
    torch.cuda.synchronize()
    return rc


def test_noalloc_matches_apply_S_on_two_calls():
    require_gpu()
    from paper_1501_06211_amd import edd
    L = edd.lib()
    sizes = []
    for make in (_case_3d, _case_2d):  # the second problem is the smaller one
        wk, dissect = make()
        prob = make_problem(wk, dissect=dissect)
        sizes.append(prob.n_interior_dofs)
        nG = prob.n_gamma * wk.dim
        v = to_cuda(np.random.default_rng(5).standard_normal(nG))
        for prec in (edd.F64, edd.F32):
            y_ref = torch.full((nG,), np.nan, dtype=torch.float64, device="cuda")
            y_new = torch.full((nG,), np.nan, dtype=torch.float64, device="cuda")
            assert _call(L.edd_apply_S, prob, v, y_ref, prec) == edd.OK
            assert _call(L.edd_apply_S_noalloc, prob, v, y_new, prec) == edd.OK
            a, b = to_np(y_ref), to_np(y_new)
            assert np.isfinite(a).all()
            assert np.array_equal(a, b), (wk.name, prec, np.abs(a - b).max())
        prob.close()
    assert sizes[1] < sizes[0]


def test_noalloc_error_paths():
    require_gpu()
    from paper_1501_06211_amd import edd
    L = edd.lib()
    wk, _ = _case_2d()
    prob = edd.Problem.from_workload(wk, factor_precision=edd.F64)
    nG = prob.n_gamma * wk.dim
    v = torch.zeros(nG, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(v)
    assert _call(L.edd_apply_S_noalloc, prob, v, y, edd.F64) == edd.ESTATE  # no moduli
    prob.set_element_moduli(torch.tensor(wk.E, device="cuda"))
    assert _call(L.edd_apply_S_noalloc, prob, v, y, edd.F32) == edd.ESTATE  # no FP32 factors
    assert _call(L.edd_apply_S_noalloc, prob, v, y, 3) == edd.EINVAL
    assert L.edd_apply_S_noalloc(prob.h, None, ctypes.c_void_p(y.data_ptr()), edd.F64) == edd.EINVAL
    prob.close()
    # an interior vector longer than the static array: rejected before any launch
    big = w.cantilever2d(1280, 1024, E=np.ones(1280 * 1024))
    prob = edd.Problem.from_workload(big, factor_precision=edd.F64)
    assert prob.n_interior_dofs > edd.NOALLOC_MAX_INTERIOR_DOFS
    nG = prob.n_gamma * 2
    v = torch.zeros(nG, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(v)
    assert _call(L.edd_apply_S_noalloc, prob, v, y, edd.F64) == edd.EINVAL
    prob.close()
