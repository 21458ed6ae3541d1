"""Pins for oracle/iface.py: skeleton M and L, H_theta closed forms, inverse
Lanczos, face-block preconditioner."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as w
from oracle import dd, iface, krylov


def test_skeleton_element_matrices_closed_form():
    Me, Le = iface._segment_matrices()
    assert np.allclose(Me, np.array([[2, 1], [1, 2]]) / 6.0, rtol=0, atol=1e-16)
    assert np.allclose(Le, np.array([[1, -1], [-1, 1]]), rtol=0, atol=1e-15)
    Mq, Lq = iface._quad_matrices()
    Mt = np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]]) / 36.0
    Lt = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1],
                   [-1, -2, -1, 4]]) / 6.0
    assert np.allclose(Mq, Mt, rtol=0, atol=1e-16)
    assert np.allclose(Lq, Lt, rtol=0, atol=1e-15)


def _unclamped(dim):
    if dim == 2:
        p = w.cantilever2d(24, 16, block=8)
    else:
        p = w.cantilever3d(8, 8, 6, cuts=(w.even_cuts(8, 4), w.even_cuts(8, 4),
                                          np.array([0, 3, 6])))
    p.clamp = 0
    return p


@pytest.mark.parametrize("dim", [2, 3])
def test_skeleton_measure_and_constants(dim):
    p = _unclamped(dim)
    M, L, g = iface.skeleton_matrices(p)
    one = np.ones(M.shape[0])
    if dim == 2:
        # total length of the cut lines
        meas = (len(p.cuts[0]) - 2) * p.nel[1] + (len(p.cuts[1]) - 2) * p.nel[0]
    else:
        nx, ny, nz = p.nel
        meas = ((len(p.cuts[0]) - 2) * ny * nz + (len(p.cuts[1]) - 2) * nx * nz
                + (len(p.cuts[2]) - 2) * nx * ny)
    assert one @ (M @ one) == pytest.approx(meas, rel=1e-14)
    assert np.abs(L @ one).max() < 1e-13
    assert abs(M - M.T).max() < 1e-16 and abs(L - L.T).max() < 1e-16


@pytest.mark.parametrize("dim", [2, 3])
def test_skeleton_nodes_are_gamma_and_L_spd(dim):
    p = w.cantilever2d_uniform_64x32() if dim == 2 else \
        w.cantilever3d(8, 8, 6, cuts=(w.even_cuts(8, 4), w.even_cuts(8, 4),
                                      np.array([0, 3, 6])))
    M, L, g = iface.skeleton_matrices(p)
    els = iface.skeleton_elements(p)
    cls = dd.classify(p)
    sk = np.unique(els)
    sk = sk[cls[sk] != dd.DIRICHLET]
    assert np.array_equal(np.sort(sk), np.flatnonzero(cls == dd.GAMMA))
    assert np.linalg.eigvalsh(L.toarray()).min() > 0


def test_htilde_special_cases():
    p = w.cantilever2d(32, 16, block=8)
    for lumped in (False, True):
        M, L, _ = iface.skeleton_matrices(p, lumped=lumped)
        Md, Ld = M.toarray(), L.toarray()
        assert np.allclose(iface.htilde(M, L, 1.0), Md, atol=1e-12)
        assert np.allclose(iface.htilde(M, L, 0.0), Ld, atol=1e-11)
        H = iface.htilde(M, L, 0.5)
        X = np.linalg.solve(Md, H)
        assert np.allclose(X @ X, np.linalg.solve(Md, Ld), atol=1e-9)
        assert np.allclose(H, H.T, atol=1e-12)
        assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0
        Hi = iface.htilde_inv(M, L, 0.3)
        assert np.allclose(Hi @ iface.htilde(M, L, 0.3), np.eye(len(Md)), atol=1e-8)
        # H_theta = M + M (M^{-1} L)^{1-theta}
        Hfull = Md + iface.htilde(M, L, 0.4)
        assert np.allclose(iface.h_inv(M, L, 0.4) @ Hfull, np.eye(len(Md)), atol=1e-8)


def test_inverse_lanczos_converges_to_closed_form():
    p = w.cantilever2d(32, 16, block=8)
    M, L, _ = iface.skeleton_matrices(p, lumped=True)
    rng = np.random.default_rng(0)
    r = rng.standard_normal(M.shape[0])
    for theta in (0.5, 0.7):
        zd = iface.htilde_inv(M, L, theta) @ r
        errs = []
        for k in (4, 8, 16, 64):
            z, kk = iface.inverse_lanczos(M, L, theta, r, kmax=k, tol=0.0)
            errs.append(np.linalg.norm(z - zd) / np.linalg.norm(zd))
        assert errs[-1] < 1e-10
        assert errs[0] > errs[1] > errs[2] > errs[3]


def test_face_partition_2d_counts():
    p = w.cantilever2d_uniform_64x32()
    faces, rest = iface.face_partition(p)
    # 3 vertical lines split by the y=16 line into 2 segments each, and the
    # y=16 line split into 4 segments: 10 faces; 3 interior crossings.
    assert len(faces) == 10 and len(rest) == 3
    assert sum(len(f) for f in faces) + len(rest) == 160


@pytest.mark.parametrize("dim", [2, 3])
def test_face_block_pcg_solves_L(dim):
    p = w.cantilever2d(48, 32, block=16) if dim == 2 else \
        w.cantilever3d(12, 8, 8, cuts=(w.even_cuts(12, 4), w.even_cuts(8, 4),
                                       w.even_cuts(8, 4)))
    M, L, _ = iface.skeleton_matrices(p, lumped=True)
    B = iface.FaceBlockPreconditioner(p, L)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(L.shape[0])
    x, its, _ = krylov.pcg(lambda v: L @ v, b, B.apply, tol=1e-12, maxit=500)
    xr = spla.spsolve(L.tocsc(), b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    _, its_plain, _ = krylov.pcg(lambda v: L @ v, b, None, tol=1e-12, maxit=2000)
    assert its < its_plain


def test_weighted_skeleton_constant_modulus_and_adjacency():
    # with a constant modulus c the weighted operators are c times the
    # unweighted ones; the two neighbours of every skeleton element straddle it
    for p in (w.cantilever2d(24, 16, block=8),
              w.cantilever3d(8, 8, 6, cuts=(w.even_cuts(8, 4), w.even_cuts(8, 4),
                                            np.array([0, 3, 6])))):
        p.E = np.full(p.n_el, 2.5)
        M, L, _ = iface.skeleton_matrices(p, lumped=True)
        Mw, Lw, _ = iface.skeleton_matrices(p, lumped=True, weighted=True)
        assert abs(Mw - 2.5 * M).max() < 1e-14 and abs(Lw - 2.5 * L).max() < 1e-13
        els, adj = iface.skeleton_elements(p, adjacent=True)
        from oracle import fe
        en = fe.element_nodes(p)
        for q, (a, b) in zip(els[::7], adj[::7]):
            assert set(q) <= set(en[a]) and set(q) <= set(en[b]) and a != b


def test_weighted_htheta_helps_heterogeneous_interface():
    # contrast 1e3 (SIMP map of a smooth field): the modulus-weighted
    # interface norm is a much better preconditioner than the unweighted one
    p = w.cantilever3d_simp(16, 8, 8, (w.even_cuts(16, 4), w.even_cuts(8, 4),
                                      w.even_cuts(8, 4)), seed=3, ell=4.0)
    _, its_u, _ = krylov.schur_pcg(p, precond="htilde_lumped", theta=0.5, tol=1e-8)
    _, its_w, _ = krylov.schur_pcg(p, precond="htilde_lumped", theta=0.5, tol=1e-8,
                                   weighted=True)
    assert its_w < 0.6 * its_u


@pytest.mark.parametrize("dim", [2, 3])
def test_consistent_mass_integrates_products_exactly(dim):
    """The consistent skeleton mass is the Gram matrix of the piecewise
    (bi)linear functions on the skeleton: for the nodal values u of x and of
    x*y, which lie in that space on every cut line or plane and vanish on the
    clamped face x = 0 (so the removed rows carry zeros), u^T M u is the
    integral of u^2 over the skeleton.  The integrals here are summed over the
    cuts in closed form.  The lumped mass misses them (it is exact only for
    linear integrands)."""
    if dim == 2:
        p = w.cantilever2d(24, 16, block=8)
    else:
        p = w.cantilever3d(8, 8, 6, cuts=(w.even_cuts(8, 4), w.even_cuts(8, 4),
                                          np.array([0, 3, 6])))
    M, _, g = iface.skeleton_matrices(p)
    Ml, _, _ = iface.skeleton_matrices(p, lumped=True)
    nn = [n + 1 for n in p.nel]
    x = (g % nn[0]).astype(float)
    y = ((g // nn[0]) % nn[1]).astype(float)
    cx, cy = p.cuts[0][1:-1], p.cuts[1][1:-1]
    nx, ny = p.nel[0], p.nel[1]
    if dim == 2:
        # vertical lines x = c (0 <= y <= ny), horizontal lines y = c
        int_x2 = sum(c * c * ny for c in cx) + len(cy) * nx ** 3 / 3
        int_xy2 = sum(c * c * ny ** 3 / 3 for c in cx) + sum(c * c * nx ** 3 / 3 for c in cy)
    else:
        nz, cz = p.nel[2], p.cuts[2][1:-1]
        # planes x = c (y, z free), y = c (x, z free), z = c (x, y free)
        int_x2 = (sum(c * c * ny * nz for c in cx) + len(cy) * nx ** 3 / 3 * nz
                  + len(cz) * nx ** 3 / 3 * ny)
        int_xy2 = (sum(c * c * ny ** 3 / 3 * nz for c in cx)
                   + sum(c * c * nx ** 3 / 3 * nz for c in cy)
                   + len(cz) * (nx ** 3 / 3) * (ny ** 3 / 3))
    for u, exact in ((x, int_x2), (x * y, int_xy2)):
        assert u @ (M @ u) == pytest.approx(exact, rel=1e-13)
        assert abs(u @ (Ml @ u) - exact) > 1e-6 * exact
