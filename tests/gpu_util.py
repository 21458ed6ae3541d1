"""Helpers shared by the GPU parity tests: build a GPU problem from a
workload and translate between the library's vector orderings and the
oracle's."""
import numpy as np
import pytest
import torch

from oracle import dd


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_problem(w, factor_precision=None, dissect=-1):
    from paper_1501_06211_amd import edd
    fp = factor_precision if factor_precision is not None else (edd.F64 | edd.F32)
    p = edd.Problem.from_workload(w, factor_precision=fp, dissect=dissect)
    E = torch.tensor(w.E, device="cuda", dtype=torch.float64)
    p.set_element_moduli(E)
    return p


def interior_perm(w, prob):
    """perm such that x_oracle = x_gpu[perm] (oracle I order: subdomain,
    node id, component)."""
    I, G, cls = dd.partition(w)
    d = w.dim
    gnodes = prob.interior_nodes()
    pos = np.full(w.n_nodes, -1, dtype=np.int64)
    pos[gnodes] = np.arange(len(gnodes))
    onodes = I[::d] // d
    assert (pos[onodes] >= 0).all()
    return (d * pos[onodes][:, None] + np.arange(d)).reshape(-1)


def gamma_check(w, prob):
    I, G, cls = dd.partition(w)
    assert np.array_equal(prob.gamma_nodes(), G[::w.dim] // w.dim)


def to_cuda(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
