"""The interface preconditioner with the consistent skeleton mass matrix
(edd_solve_opts.mass_matrix = 1, Section 3's M as the FE mass matrix rather
than its row-sum lumping): the mass product and the Chebyshev M^{-1} against
the oracle's assembled M, every form of the interface norm against the
oracle's closed forms and its inverse Lanczos with the same M, the
device-resident and captured applies, and whole solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as w
from oracle import fe, iface

from gpu_util import make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _small2d():
    rng = np.random.default_rng(21)
    p = w.cantilever2d(24, 16, block=8)
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    return p


def _small3d():
    return w.cantilever3d_simp(8, 8, 6, (w.even_cuts(8, 4), w.even_cuts(8, 4),
                                         np.array([0, 3, 6])), seed=5, ell=3.0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("weighted", [0, 1])
def test_consistent_mass_product_and_solve(dim, weighted):
    require_gpu()
    p = _small2d() if dim == 2 else _small3d()
    prob = make_problem(p)
    M, _, g = iface.skeleton_matrices(p, weighted=bool(weighted))
    x = np.random.default_rng(7).standard_normal((len(g), dim))
    y = to_np(prob.skeleton_op(4, to_cuda(x.reshape(-1)), weighting=weighted)).reshape(-1, dim)
    ref = M @ x
    e4 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    z = to_np(prob.skeleton_op(5, to_cuda(x.reshape(-1)), weighting=weighted)).reshape(-1, dim)
    lu = spla.splu(M.tocsc())
    zref = np.column_stack([lu.solve(x[:, c]) for c in range(dim)])
    e5 = np.linalg.norm(z - zref) / np.linalg.norm(zref)
    print(f"{dim}D weighted={weighted}: M x {e4:.2e}, M^-1 x (Chebyshev) {e5:.2e}")
    assert e4 <= 1e-14 and e5 <= 1e-11
    prob.close()


@pytest.mark.parametrize("weighted", [0, 1])
@pytest.mark.parametrize("form", ["htilde_inv", "h_inv", "htilde_fwd", "h_fwd"])
def test_consistent_mass_forms_match_closed_forms_2d(form, weighted):
    """With as many Lanczos steps as interface nodes per component the
    process spans the space and reproduces the closed forms built from the
    generalised eigenpairs of (L, M) with the consistent M."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _small2d()
    prob = make_problem(p)
    M, L, g = iface.skeleton_matrices(p, weighted=bool(weighted))
    assert len(g) <= 64
    theta = 0.6
    A = iface.h_inv(M, L, theta) if form.startswith("h_") else iface.htilde_inv(M, L, theta)
    pcf = {"htilde_inv": edd.PCF_HTILDE_INV, "h_inv": edd.PCF_H_INV,
           "htilde_fwd": edd.PCF_HTILDE_FWD, "h_fwd": edd.PCF_H_FWD}[form]
    r = np.random.default_rng(3).standard_normal(len(g) * 2)
    zref = iface.componentwise(A, r, 2)
    z = to_np(prob.apply_precond(to_cuda(r), precond=edd.PC_HTHETA, theta=theta, pc_form=pcf,
                                 lanczos_kmax=64, lanczos_tol=0.0, inner_tol=1e-14,
                                 inner_maxit=1000, interface_weighting=weighted, mass_matrix=1))
    err = np.linalg.norm(z - zref) / np.linalg.norm(zref)
    # the lumped form is a different operator: it must not match these
    zl = to_np(prob.apply_precond(to_cuda(r), precond=edd.PC_HTHETA, theta=theta, pc_form=pcf,
                                  lanczos_kmax=64, lanczos_tol=0.0, inner_tol=1e-14,
                                  inner_maxit=1000, interface_weighting=weighted))
    el = np.linalg.norm(zl - zref) / np.linalg.norm(zref)
    print(f"2D {form} weighted={weighted}: consistent M {err:.2e} (lumped M {el:.2e})")
    assert err <= 1e-7 and el > 1e-3
    prob.close()


@pytest.mark.parametrize("weighted", [0, 1])
def test_consistent_mass_matches_oracle_lanczos_3d(weighted):
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _small3d()
    prob = make_problem(p)
    M, L, g = iface.skeleton_matrices(p, weighted=bool(weighted))
    r = np.random.default_rng(2).standard_normal(len(g) * 3)
    R = r.reshape(-1, 3)
    k = 12
    zref = np.column_stack([iface.inverse_lanczos(M, L, 0.5, R[:, c], kmax=k, tol=0.0)[0]
                            for c in range(3)]).reshape(-1)
    z = to_np(prob.apply_precond(to_cuda(r), precond=edd.PC_HTHETA, theta=0.5,
                                 lanczos_kmax=k, lanczos_tol=0.0, inner_tol=1e-14,
                                 inner_maxit=2000, interface_weighting=weighted, mass_matrix=1))
    err = np.linalg.norm(z - zref) / np.linalg.norm(zref)
    print(f"3D weighted={weighted}: consistent M vs oracle Lanczos {err:.2e}")
    assert err <= 1e-8
    prob.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_consistent_mass_device_resident_graph_and_solve(dim):
    """The fixed-step form (no host waits) against the oracle's k-step inverse
    Lanczos with exact Laplacian solves, its captured graph replayed against
    the eager launches, and a whole solve against the direct solve."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _small2d() if dim == 2 else _small3d()
    prob = make_problem(p)
    M, L, g = iface.skeleton_matrices(p, weighted=True)
    r = np.random.default_rng(3).standard_normal(len(g) * dim)
    R = r.reshape(-1, dim)
    k = 6
    zref = np.column_stack([iface.inverse_lanczos(M, L, 0.5, R[:, c], kmax=k, tol=0.0)[0]
                            for c in range(dim)]).reshape(-1)
    opts = dict(precond=edd.PC_HTHETA, theta=0.5, lanczos_kmax=k, lanczos_tol=0.0,
                inner_tol=0.0, inner_maxit=300, interface_weighting=1, mass_matrix=1)
    z = to_np(prob.apply_precond(to_cuda(r), **opts))
    err = float(np.linalg.norm(z - zref) / np.linalg.norm(zref))
    rc = to_cuda(r)
    zs = [to_np(prob.apply_precond(rc, use_graphs=1, **opts)) for _ in range(3)]
    print(f"{dim}D device-resident consistent M, k={k}: vs oracle {err:.2e}")
    assert err <= 1e-9
    for zg in zs:
        assert np.array_equal(zg, z)
    u, st = prob.solve(to_cuda(p.f), tol=1e-12, maxit=2000, lanczos_kmax=3, inner_maxit=4,
                       mass_matrix=1)
    uref = fe.solve_direct(p)
    e = float(np.linalg.norm(to_np(u) - uref) / np.linalg.norm(uref))
    print(f"{dim}D solve with consistent M: its={st['iterations']} u_err={e:.2e}")
    assert e <= 1e-8
    with pytest.raises(edd.EddError):
        prob.apply_precond(to_cuda(r), precond=edd.PC_HTHETA, mass_matrix=2)
    prob.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_consistent_mass_in_captured_iterations_and_batch(dim):
    """use_graphs = 8 (the interface iterations replayed from a captured
    graph, the Chebyshev M^{-1} inside it) against the host-driven loop, and
    the batch entry point against single solves, both with the consistent
    mass."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _small2d() if dim == 2 else _small3d()
    prob = make_problem(p)
    f = to_cuda(p.f)
    uref = fe.solve_direct(p)
    u0, s0 = prob.solve(f, tol=1e-10, maxit=3000, mass_matrix=1)
    u0 = to_np(u0)
    u1, s1 = prob.solve(f, tol=1e-10, maxit=3000, mass_matrix=1, use_graphs=8)
    u1 = to_np(u1)
    print(f"{dim}D consistent M: host loop {s0['iterations']} its, graph {s1['iterations']} its")
    assert abs(s1["iterations"] - s0["iterations"]) <= 16
    assert np.linalg.norm(u1 - u0) <= 1e-9 * np.linalg.norm(u0)
    assert np.linalg.norm(u1 - uref) <= 1e-8 * np.linalg.norm(uref)
    prob2 = make_problem(p)
    import torch
    outs = [torch.zeros_like(f), torch.zeros_like(f)]
    status, stats = edd.solve_batch([prob, prob2], [f, f], outs, tol=1e-10, maxit=3000,
                                    mass_matrix=1)
    assert status == edd.OK
    for u in outs:
        assert np.array_equal(to_np(u), u0)
    prob.close()
    prob2.close()
