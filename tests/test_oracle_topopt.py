"""Pins for oracle/topopt.py (Section 5, eq. (NumberTen)).

* Element energies: zero for rigid-body motions; for an affine field the
  constant strain gives u_e^T K0 u_e = eps^T D eps (unit element volume),
  a closed form that does not go through K0's quadrature; and
  sum_e E_e s_e = u^T K(E) u.
* OC update: the volume constraint is met; a uniform design with uniform
  sensitivities is a fixed point with Lambda equal to the sensitivity;
  Lambda agrees with a library root finder (brentq) on the volume function;
  larger sensitivity never gives a smaller density.
* The loop: the converged VTS design satisfies the optimality (KKT)
  conditions of the convex problem: g_e equals Lambda on elements strictly
  inside their bounds, g_e >= Lambda at the upper bound, g_e <= Lambda at
  the lower bound; compliance decreases.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

import workloads as w
from oracle import fe, topopt


def _mesh(dim):
    if dim == 2:
        return w.cantilever2d(6, 4, block=3)
    return w.cantilever3d(4, 3, 3, cuts=([0, 2, 4], [0, 3], [0, 3]))


@pytest.mark.parametrize("dim", [2, 3])
def test_element_energy_rigid_and_affine(dim):
    p = _mesh(dim)
    p.clamp = 0  # no clamp: keep every dof of the affine field
    X = fe.node_coords(p).astype(np.float64)
    R = fe.rigid_body_modes(X, dim)
    for j in range(R.shape[1]):
        assert np.abs(topopt.element_energies(p, R[:, j])).max() <= 1e-12
    rng = np.random.default_rng(2)
    A = rng.standard_normal((dim, dim))
    u = (X @ A.T).reshape(-1)
    eps_t = 0.5 * (A + A.T)
    if dim == 2:
        eps = np.array([eps_t[0, 0], eps_t[1, 1], 2 * eps_t[0, 1]])
    else:
        eps = np.array([eps_t[0, 0], eps_t[1, 1], eps_t[2, 2],
                        2 * eps_t[0, 1], 2 * eps_t[1, 2], 2 * eps_t[0, 2]])
    D = fe.dmatrix(dim, p.nu)
    want = eps @ D @ eps
    s = topopt.element_energies(p, u)
    assert np.allclose(s, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_energies_sum_to_the_energy(dim):
    p = _mesh(dim)
    rng = np.random.default_rng(3)
    E = 10.0 ** rng.uniform(-3, 0, p.n_el)
    u = rng.standard_normal(p.ndof) * (~fe.dirichlet_dof_mask(p))
    s = topopt.element_energies(p, u)
    assert np.isclose(E @ s, u @ fe.apply_K_elementwise(p, u, E), rtol=1e-13)


def test_oc_volume_fixed_point_and_root_finder():
    rng = np.random.default_rng(4)
    m = 500
    rho = rng.uniform(0.05, 0.95, m)
    g = 10.0 ** rng.uniform(-2, 2, m)
    V = 0.4 * m
    new, lam = topopt.oc_update(rho, g, V)
    assert abs(new.sum() - V) <= 1e-10 * V
    assert np.all(new >= np.maximum(1e-3, rho - 0.2) - 1e-15)
    assert np.all(new <= np.minimum(1.0, rho + 0.2) + 1e-15)
    # a library root finder on the volume function gives the same multiplier
    def vol(loglam):
        return topopt.oc_candidate(rho, g, np.exp(loglam), 1e-3, 1.0, 0.2, 0.5).sum() - V
    ref = np.exp(brentq(vol, np.log(lam) - 5, np.log(lam) + 5, xtol=1e-14, rtol=1e-14))
    assert abs(lam - ref) <= 1e-9 * ref
    # uniform design with uniform sensitivity: a fixed point, Lambda = g
    rho0 = np.full(m, 0.4)
    new0, lam0 = topopt.oc_update(rho0, np.full(m, 3.0), V)
    assert np.allclose(new0, rho0, rtol=1e-12) and abs(lam0 - 3.0) <= 1e-10
    # monotone in the sensitivity
    order = np.argsort(g)
    same = np.full(m, 0.5)
    upd, _ = topopt.oc_update(same, g, V)
    assert np.all(np.diff(upd[order]) >= -1e-15)


def test_adaptive_tolerance_rule():
    assert topopt.adaptive_tolerance([]) == 1e-2
    assert topopt.adaptive_tolerance([5.0]) == 1e-2
    assert topopt.adaptive_tolerance([10.0, 9.0]) == pytest.approx(1.0 / 9.0 if 1.0 / 9.0 < 1e-2 else 1e-2)
    assert topopt.adaptive_tolerance([10.0, 9.999]) == pytest.approx(0.001 / 9.999)
    assert topopt.adaptive_tolerance([10.0, 10.0]) == 1e-8


def test_vts_loop_reaches_the_kkt_point():
    p = w.cantilever2d(12, 6, block=6)
    res = topopt.optimise(p, volfrac=0.5, change_tol=1e-7, maxit=400)
    rho = res["rho"]
    c = res["compliance"]
    assert c[-1] < c[0]
    assert all(b <= a * (1 + 1e-9) for a, b in zip(c[5:], c[6:]))  # decreasing once settled
    u = fe.solve_direct(p, topopt.moduli(rho))
    g = topopt.element_energies(p, u)
    assert abs(rho.sum() - 0.5 * p.n_el) <= 1e-9 * p.n_el
    inner = (rho > 1e-3 + 1e-6) & (rho < 1.0 - 1e-6)
    assert inner.sum() > 0
    lam = np.median(g[inner])
    assert np.all(np.abs(g[inner] / lam - 1.0) <= 1e-4)
    assert np.all(g[rho >= 1.0 - 1e-6] >= lam * (1 - 1e-4))
    assert np.all(g[rho <= 1e-3 + 1e-6] <= lam * (1 + 1e-4))
