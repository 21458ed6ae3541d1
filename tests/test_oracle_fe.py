"""Pins for oracle/fe.py: constitutive law, element matrices, assembly,
direct solve.  Each pin is computed by a route other than the oracle's own
(symbolic integration, closed forms, invariants, brute force)."""
import numpy as np
import pytest
import sympy

import workloads as w
from oracle import fe


def test_lame_and_plane_stress_textbook():
    # Section 1: mu = E/(2(1+nu)), lambda = nu E/((1+nu)(1-2nu)).
    E, nu = 2.5, 0.3
    D2 = fe.dmatrix(2, nu, E)
    text = E / (1 - nu ** 2) * np.array([[1, nu, 0], [nu, 1, 0],
                                         [0, 0, (1 - nu) / 2]])
    assert np.allclose(D2, text, rtol=1e-15, atol=1e-15)
    D3 = fe.dmatrix(3, nu, E)
    c = E / ((1 + nu) * (1 - 2 * nu))
    text3 = np.zeros((6, 6))
    text3[:3, :3] = c * nu
    for i in range(3):
        text3[i, i] = c * (1 - nu)
        text3[3 + i, 3 + i] = c * (1 - 2 * nu) / 2
    assert np.allclose(D3, text3, rtol=1e-14, atol=1e-15)


def _symbolic_K0(dim, nu):
    """Exact integral of B^T D B with sympy, independent of fe.shape_grads."""
    xs = sympy.symbols("x0:%d" % dim)
    corners = fe.local_node_offsets(dim)
    N = []
    for o in corners:
        term = sympy.Integer(1)
        for k in range(dim):
            term *= xs[k] if o[k] else (1 - xs[k])
        N.append(term)
    nuq = sympy.Rational(nu).limit_denominator(1000)
    mu = sympy.Rational(1, 2) / (1 + nuq)
    lam = nuq / ((1 + nuq) * (1 - 2 * nuq))
    if dim == 2:
        lam = 2 * mu * lam / (lam + 2 * mu)
        nn, ns = 2, 1
    else:
        nn, ns = 3, 3
    D = sympy.zeros(nn + ns, nn + ns)
    for i in range(nn):
        for j in range(nn):
            D[i, j] = lam + (2 * mu if i == j else 0)
    for i in range(ns):
        D[nn + i, nn + i] = mu
    # strain rows built from the displacement gradient directly
    ndof = dim * len(N)
    B = sympy.zeros(nn + ns, ndof)
    shear_pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for a, Na in enumerate(N):
        for k in range(dim):
            B[k, dim * a + k] = sympy.diff(Na, xs[k])
        for s, (p, q) in enumerate(shear_pairs):
            B[nn + s, dim * a + p] = sympy.diff(Na, xs[q])
            B[nn + s, dim * a + q] = sympy.diff(Na, xs[p])
    integrand = B.T * D * B
    K = np.zeros((ndof, ndof))
    for i in range(ndof):
        for j in range(i, ndof):
            poly = sympy.Poly(sympy.expand(integrand[i, j]), *xs)
            val = sympy.Integer(0)
            for mon, coef in poly.terms():
                den = 1
                for e in mon:
                    den *= e + 1
                val += coef / den
            K[i, j] = K[j, i] = float(val)
    return K


@pytest.mark.parametrize("dim", [2, 3])
def test_K0_equals_symbolic_integral(dim):
    K0 = fe.element_stiffness(dim, 0.3)
    Ks = _symbolic_K0(dim, 0.3)
    assert np.abs(K0 - Ks).max() <= 1e-14 * np.abs(Ks).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_K0_rigid_modes_and_rank(dim):
    K0 = fe.element_stiffness(dim, 0.3)
    assert np.array_equal(K0, K0.T) or np.abs(K0 - K0.T).max() < 1e-15
    R = fe.rigid_body_modes(fe.local_node_offsets(dim), dim)
    assert np.abs(K0 @ R).max() < 1e-14
    ev = np.linalg.eigvalsh(K0)
    nrig = 3 if dim == 2 else 6
    assert (ev[:nrig] < 1e-13).all() and (ev[nrig:] > 1e-3).all()
    # linear in E
    assert np.allclose(fe.element_stiffness(dim, 0.3, E=2.0), 2 * K0,
                       rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_energy_of_homogeneous_strain(dim):
    # u = G x with a constant gradient G: energy u^T K0 u = eps^T D eps (unit
    # volume), with eps the Voigt strain of sym(G).
    rng = np.random.default_rng(1)
    G = rng.standard_normal((dim, dim))
    X = fe.local_node_offsets(dim).astype(float)
    u = (X @ G.T).reshape(-1)
    Esym = 0.5 * (G + G.T)
    if dim == 2:
        eps = np.array([Esym[0, 0], Esym[1, 1], 2 * Esym[0, 1]])
    else:
        eps = np.array([Esym[0, 0], Esym[1, 1], Esym[2, 2], 2 * Esym[0, 1],
                        2 * Esym[1, 2], 2 * Esym[0, 2]])
    D = fe.dmatrix(dim, 0.3)
    K0 = fe.element_stiffness(dim, 0.3)
    assert u @ K0 @ u == pytest.approx(eps @ D @ eps, rel=1e-13)


def _small(dim):
    if dim == 2:
        return w.cantilever2d(7, 5, block=3)
    return w.cantilever3d(5, 4, 3, cuts=(w.even_cuts(5, 2), w.even_cuts(4, 2),
                                         w.even_cuts(3, 2)))


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test(dim):
    prob = _small(dim)
    K = fe.assemble(prob)
    X = fe.node_coords(prob).astype(float)
    rng = np.random.default_rng(2)
    G = rng.standard_normal((dim, dim))
    a = rng.standard_normal(dim)
    u = (X @ G.T + a).reshape(-1)
    y = K @ u
    inner = np.ones(prob.n_nodes, dtype=bool)
    for ax in range(dim):
        inner &= (X[:, ax] > 0) & (X[:, ax] < prob.nel[ax])
    yi = y.reshape(-1, dim)[inner]
    assert np.abs(yi).max() <= 1e-13 * np.abs(K.data).max() * np.abs(u).max()
    # prescribe the affine field on the boundary, solve for the inside
    bnd = np.repeat(~inner, dim)
    ins = np.flatnonzero(~bnd)
    bd = np.flatnonzero(bnd)
    Kii = K[ins][:, ins].toarray()
    rhs = -K[ins][:, bd] @ u[bd]
    ui = np.linalg.solve(Kii, rhs)
    assert np.abs(ui - u[ins]).max() <= 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_assembly_symmetric_spd_linear(dim):
    prob = _small(dim)
    rng = np.random.default_rng(3)
    E1 = rng.uniform(1e-3, 1.0, prob.n_el)
    E2 = rng.uniform(1e-3, 1.0, prob.n_el)
    K1 = fe.assemble(prob, E1)
    K2 = fe.assemble(prob, E2)
    assert abs(K1 - K1.T).max() < 1e-15
    free = np.flatnonzero(~fe.dirichlet_dof_mask(prob))
    Kff = K1[free][:, free].toarray()
    np.linalg.cholesky(Kff)  # raises if not SPD
    K12 = fe.assemble(prob, 0.7 * E1 + 1.9 * E2)
    assert abs(K12 - (0.7 * K1 + 1.9 * K2)).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_elementwise_apply_matches_assembled(dim):
    prob = _small(dim)
    rng = np.random.default_rng(4)
    E = rng.uniform(1e-3, 1.0, prob.n_el)
    u = rng.standard_normal(prob.ndof)
    K = fe.assemble(prob, E)
    dm = fe.dirichlet_dof_mask(prob)
    uu = np.where(dm, 0.0, u)
    ref = np.where(dm, 0.0, K @ uu)
    y = fe.apply_K_elementwise(prob, u, E)
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)


def test_direct_solve_residual_betti_compliance():
    prob = w.cantilever2d(32, 16, block=8)
    rng = np.random.default_rng(5)
    E = rng.uniform(1e-3, 1.0, prob.n_el)
    u = fe.solve_direct(prob, E)
    K = fe.assemble(prob, E)
    # residual evaluated in long double; storing u in FP64 alone leaves a
    # floor of about eps * ||K||_inf ||u||_inf / ||f||, which refinement must
    # reach (without refinement the LU residual sits several times above it)
    free = np.flatnonzero(~fe.dirichlet_dof_mask(prob))
    Kl = K[free][:, free].astype(np.longdouble)
    rl = prob.f[free].astype(np.longdouble) - Kl @ u[free].astype(np.longdouble)
    floor = (np.finfo(float).eps * abs(K).sum(axis=1).max() * np.abs(u).max()
             / np.linalg.norm(prob.f))
    assert float(np.linalg.norm(rl.astype(float)) / np.linalg.norm(prob.f)) <= 2 * floor
    assert fe.residual_norm(prob, u, E) <= 1e-12
    assert fe.compliance(prob.f, u) == pytest.approx(u @ (K @ u), rel=1e-12)
    # Maxwell-Betti reciprocity for two independent loads
    fa = rng.standard_normal(prob.ndof)
    fb = rng.standard_normal(prob.ndof)
    dm = fe.dirichlet_dof_mask(prob)
    fa[dm] = 0
    fb[dm] = 0
    ua = fe.solve_direct(prob, E, fa)
    ub = fe.solve_direct(prob, E, fb)
    assert ua @ fb == pytest.approx(ub @ fa, rel=1e-11)


def test_cantilever_beam_sanity():
    # Loose check against beam theory (Timoshenko): tip deflection under a
    # unit tip load P for a 64 x 32 beam, E=1, nu=0.3, unit thickness:
    # P L^3 / (3 E I) + P L / (kappa G A), kappa = 5/6.  The full clamp
    # stiffens, the point load softens; agreement to ~10% is expected.
    prob = w.cantilever2d_uniform_64x32()
    u = fe.solve_direct(prob)
    c = fe.compliance(prob.f, u)
    L, h, E, nu = 64.0, 32.0, 1.0, 0.3
    I = h ** 3 / 12.0
    G = E / (2 * (1 + nu))
    est = L ** 3 / (3 * E * I) + L / (5.0 / 6.0 * G * h)
    assert abs(c - est) / est < 0.1
