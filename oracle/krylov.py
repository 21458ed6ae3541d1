"""Reference Krylov solvers in FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``pcg``: preconditioned conjugate gradients (S is SPD, Section 2).
* ``fcg``: flexible CG for preconditioners that change from one iteration
  to the next (Section 3 uses a flexible Krylov method for the same
  reason): each new direction is the preconditioned residual made
  A-orthogonal to the previous directions by explicit Gram-Schmidt (all of
  them, or the last ``mmax``), then an exact line search along it.
* ``gmres_right``: GMRES on K P~^{-1} y = f, u = P~^{-1} y (Section 3,
  right preconditioning with the block-triangular P~).
* ``schur_pcg``: the whole interface solve on the CPU: condensation, Krylov
  on S u_Gamma = g, back-substitution (eq. (3MatSplit)).

Stopping rule (reading): ||r|| <= tol * ||f||, with f the full free-dof load,
so a good initial guess earns no credit.
"""
from __future__ import annotations

import numpy as np

from . import dd, fe, iface


def pcg(A, b, P=None, x0=None, tol=1e-10, maxit=1000, ref_norm=None):
    """Returns (x, iterations, residual-norm history)."""
    if P is None:
        def P(v):
            return v
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x)
    ref = np.linalg.norm(b) if ref_norm is None else ref_norm
    hist = [np.linalg.norm(r)]
    if hist[-1] <= tol * ref:
        return x, 0, hist
    z = P(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol * ref:
            return x, it, hist
        z = P(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist


def fcg(A, b, P, x0=None, tol=1e-10, maxit=1000, ref_norm=None, mmax=None):
    """Flexible CG: each new direction is made A-orthogonal to the last
    ``mmax`` directions (all of them when ``mmax`` is None), the long
    recurrence a changing preconditioner needs.  With a fixed SPD
    preconditioner it reproduces PCG in exact arithmetic."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x)
    ref = np.linalg.norm(b) if ref_norm is None else ref_norm
    hist = [np.linalg.norm(r)]
    if hist[-1] <= tol * ref:
        return x, 0, hist
    Ps, Qs, PQ = [], [], []
    for it in range(1, maxit + 1):
        z = P(r)
        p = z.copy()
        keep = len(Ps) if mmax is None else min(mmax, len(Ps))
        for j in range(len(Ps) - keep, len(Ps)):
            p -= ((z @ Qs[j]) / PQ[j]) * Ps[j]
        q = A(p)
        pq = p @ q
        alpha = (p @ r) / pq
        x += alpha * p
        r -= alpha * q
        Ps.append(p)
        Qs.append(q)
        PQ.append(pq)
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol * ref:
            return x, it, hist
    return x, maxit, hist


def gmres_right(A, b, Pinv, tol=1e-6, maxit=500):
    """Full (unrestarted) GMRES on A Pinv y = b; returns (x = Pinv y, its).

    Convergence is measured on ||b - A x|| / ||b||, which equals the GMRES
    residual of the right-preconditioned system.
    """
    n = b.size
    beta = np.linalg.norm(b)
    V = np.zeros((n, maxit + 1))
    H = np.zeros((maxit + 1, maxit))
    V[:, 0] = b / beta
    Z = []
    for j in range(maxit):
        z = Pinv(V[:, j])
        Z.append(z)
        w = A(z)
        for i in range(j + 1):
            H[i, j] = w @ V[:, i]
            w = w - H[i, j] * V[:, i]
        for i in range(j + 1):  # second Gram-Schmidt pass
            h = w @ V[:, i]
            H[i, j] += h
            w = w - h * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
        if res <= tol * beta or H[j + 1, j] <= 1e-14 * beta:
            x = np.column_stack(Z) @ y
            return x, j + 1
        V[:, j + 1] = w / H[j + 1, j]
    x = np.column_stack(Z) @ y
    return x, maxit


def block_triangular_inverse(op, Stilde_inv):
    """P~^{-1} v for P~ = [[K_II, K_IG], [0, S~]] in the factored order of
    Section 3: z_G = S~^{-1} v_G; z_I = K_II^{-1} (v_I - K_IG z_G).
    ``op`` is a dd.SchurOperator; v is ordered (I, G)."""
    nI = len(op.I)

    def apply(v):
        vI, vG = v[:nI], v[nI:]
        zG = Stilde_inv(vG)
        zI = op.solve_II(vI - op.KIG @ zG)
        return np.concatenate([zI, zG])
    return apply


def full_operator(op):
    """K v for v ordered (I, G), the block form of eq. (NumberFour)."""
    K = fe.assemble(op.prob)
    perm = np.concatenate([op.I, op.G])
    Kp = K[perm][:, perm].tocsr()

    def apply(v):
        return Kp @ v
    return apply


def schur_pcg(prob, precond="I", theta=0.5, tol=1e-10, maxit=2000,
              lanczos_tol=1e-2, kmax=20, flexible=None, E=None, weighted=False):
    """Interface solve on the CPU.  Returns (u, iterations, history).

    precond: "I" (no interface preconditioner), "htilde" (dense closed form
    of Hhat_theta with consistent M), "htilde_lumped" (dense, lumped M),
    "lanczos" (inverse Lanczos, lumped M, exact L solves).  ``weighted``
    builds M and L with the modulus weighting of iface.skeleton_matrices.
    """
    op = dd.SchurOperator(prob, E)
    g = op.rhs()
    free = ~fe.dirichlet_dof_mask(prob)
    ref = np.linalg.norm(prob.f[free])
    d = prob.dim
    if precond == "I":
        P = None
    elif precond in ("htilde", "htilde_lumped"):
        M, L, _ = iface.skeleton_matrices(prob, lumped=precond.endswith("lumped"),
                                          weighted=weighted, E=E)
        Hi = iface.htilde_inv(M, L, theta)

        def P(r):
            return iface.componentwise(Hi, r, d)
    elif precond == "lanczos":
        M, L, _ = iface.skeleton_matrices(prob, lumped=True, weighted=weighted, E=E)

        def P(r):
            R = r.reshape(-1, d)
            Z = np.column_stack([
                iface.inverse_lanczos(M, L, theta, R[:, c], kmax=kmax,
                                      tol=lanczos_tol)[0] for c in range(d)])
            return Z.reshape(-1)
    else:
        raise ValueError(precond)
    if flexible is None:
        flexible = precond == "lanczos"
    if flexible:
        uG, its, hist = fcg(op.apply, g, P, tol=tol, maxit=maxit, ref_norm=ref)
    else:
        uG, its, hist = pcg(op.apply, g, P, tol=tol, maxit=maxit, ref_norm=ref)
    return op.assemble_u(uG), its, hist
