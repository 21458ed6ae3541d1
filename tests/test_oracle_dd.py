"""Pins for oracle/dd.py: node classes, Schur complement, eq. (3MatSplit)."""
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import workloads as w
from oracle import dd, fe, krylov


def _brute_gamma_count(prob):
    """Count interface nodes by walking the grid: a node is on Gamma when one
    of its coordinates sits on an internal cut and it is not clamped."""
    internal = [set(int(c) for c in cuts[1:-1]) for cuts in prob.cuts]
    n = 0
    for ijk in itertools.product(*[range(m) for m in prob.nnodes_axis]):
        if ijk[0] == 0:  # clamped face x = 0
            continue
        if any(ijk[a] in internal[a] for a in range(prob.dim)):
            n += 1
    return n


@pytest.mark.parametrize("make", [
    w.cantilever2d_uniform_64x32,
    lambda: w.cantilever2d(40, 24, block=7),
    lambda: w.cantilever3d(20, 12, 9, cuts=(w.even_cuts(20, 8),
                                            w.even_cuts(12, 5),
                                            np.array([0, 4, 9])))])
def test_gamma_count_brute_force(make):
    prob = make()
    cls = dd.classify(prob)
    assert (cls == dd.GAMMA).sum() == _brute_gamma_count(prob)
    # every free non-Gamma node belongs to exactly one subdomain
    assert ((cls >= 0) | (cls < 0)).all()
    assert set(np.unique(cls[cls >= 0])) == set(range(prob.n_sub))


def test_gamma_count_small_config():
    assert (dd.classify(w.cantilever2d_uniform_64x32()) == dd.GAMMA).sum() == 160


def _problems():
    rng = np.random.default_rng(7)
    p2 = w.cantilever2d(48, 24, block=16)
    p2.E = rng.uniform(1e-3, 1.0, p2.n_el)
    p3 = w.cantilever3d(12, 8, 7, cuts=(np.array([0, 5, 12]),
                                        np.array([0, 4, 8]),
                                        np.array([0, 3, 7])))
    p3.E = 1e-3 + rng.uniform(0, 1, p3.n_el) ** 3
    return [p2, p3]


@pytest.mark.parametrize("prob", _problems(), ids=["2d", "3d"])
def test_schur_solution_equals_monolithic(prob):
    u = fe.solve_direct(prob)
    us = dd.schur_solve_dense(prob)
    assert np.linalg.norm(us - u) <= 1e-12 * np.linalg.norm(u)


@pytest.mark.parametrize("prob", _problems(), ids=["2d", "3d"])
def test_S_symmetric_spd_and_sum_of_local(prob):
    S = dd.schur_dense(prob)
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0
    # S = sum_i R_i^T S_i R_i (the Steklov-Poincare splitting, Section 1)
    cls = dd.classify(prob)
    g = np.flatnonzero(cls == dd.GAMMA)
    pos = {int(n): k for k, n in enumerate(g)}
    d = prob.dim
    acc = np.zeros_like(S)
    for s in range(prob.n_sub):
        Ss, gn = dd.local_schur(prob, s)
        idx = np.array([d * pos[int(n)] + c for n in gn for c in range(d)])
        acc[np.ix_(idx, idx)] += Ss
    assert np.abs(acc - S).max() <= 1e-11 * np.abs(S).max()


def test_floating_subdomain_rigid_modes():
    prob = w.cantilever2d(48, 32, block=16)
    fl = dd.floating_subdomains(prob)
    assert len(fl) > 0
    X = fe.node_coords(prob)
    for s in fl[:2]:
        Ks, nodes = dd.subdomain_neumann(prob, s)
        R = fe.rigid_body_modes(X[nodes], 2)
        assert np.abs(Ks @ R).max() <= 1e-13 * np.abs(Ks).max() * np.abs(R).max()
        Ss, gn = dd.local_schur(prob, s)
        Rg = fe.rigid_body_modes(X[gn], 2)
        assert np.abs(Ss @ Rg).max() <= 1e-10 * np.abs(Ss).max() * np.abs(Rg).max()
        assert np.linalg.matrix_rank(Ss, tol=1e-9 * np.abs(Ss).max()) == Ss.shape[0] - 3


def test_exact_interface_preconditioner_iteration_counts():
    # Section 3: with S~ = S, K P~^{-1} has minimal polynomial of degree 2, so
    # GMRES converges in at most 2 iterations; PCG on S with S^{-1} in 1.
    prob = _problems()[0]
    op = dd.SchurOperator(prob)
    S = dd.schur_dense(prob)
    Sinv = np.linalg.inv(S)
    g = op.rhs()
    _, its, _ = krylov.pcg(op.apply, g, lambda r: Sinv @ r, tol=1e-10)
    assert its == 1
    A = krylov.full_operator(op)
    Pinv = krylov.block_triangular_inverse(op, lambda v: Sinv @ v)
    f = prob.f[np.concatenate([op.I, op.G])]
    x, its = krylov.gmres_right(A, f, Pinv, tol=1e-10)
    assert its <= 2
    u = fe.solve_direct(prob)
    assert np.linalg.norm(x - u[np.concatenate([op.I, op.G])]) <= 1e-9 * np.linalg.norm(u)
    # with S~ = I the same GMRES needs many more iterations
    _, its_id = krylov.gmres_right(A, f, krylov.block_triangular_inverse(
        op, lambda v: v), tol=1e-6)
    assert its_id > 10


@settings(max_examples=6, deadline=None)
@given(nx=st.integers(6, 14), ny=st.integers(4, 10),
       cx=st.integers(2, 5), cy=st.integers(2, 4),
       logc=st.floats(0, 3), seed=st.integers(0, 1000))
def test_schur_property_random_meshes(nx, ny, cx, cy, logc, seed):
    rng = np.random.default_rng(seed)
    prob = w.cantilever2d(nx, ny, cuts=(w.even_cuts(nx, cx), w.even_cuts(ny, cy)),
                          load_node=(nx, int(rng.integers(0, ny + 1))))
    prob.E = 10 ** (-logc * rng.uniform(0, 1, prob.n_el))
    u = fe.solve_direct(prob)
    us = dd.schur_solve_dense(prob)
    assert np.linalg.norm(us - u) <= 1e-10 * np.linalg.norm(u)
