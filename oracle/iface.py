"""Interface preconditioner H_theta (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 3 preconditions S with discrete interpolation norms built from the
mass matrix M and the Laplacian L assembled on the skeleton Gamma:

    H_theta       = M + M (M^{-1} L)^{1-theta}        (eq. (NumberEight))
    H~_theta      = M (M^{-1} L)^{1-theta}
    Hhat_theta    = H~_theta applied to each of the d displacement
                    components                        (eq. (NumberNine))

Fractional powers come either from a generalised eigendecomposition (small
interfaces) or from the inverse Lanczos process (large ones); the paper's
results use inverse Lanczos, with the Laplacian solves inside it done by PCG
preconditioned by L restricted to the interface pieces with the cross points
removed (Section 4).

Readings (the defining report is not available):
* M and L are the FE mass and stiffness matrices of the skeleton: 1D linear
  elements on interface edges for 2D problems, bilinear quadrilaterals on
  interface faces for 3D problems, assembled across cross points, with the
  rows and columns of clamped nodes removed.  ``lumped=True`` replaces M by
  the diagonal of row sums of the assembled mass taken before the clamped
  columns are removed (each node's share of the skeleton's length or area).
* Inverse Lanczos: Lanczos on C = L^{-1} M in the M inner product, started
  from b = M^{-1} r; then H~^{-1} r = C^{1-theta} b ~ |b|_M Q_k T_k^{1-theta} e1
  with T_k^{1-theta} from the eigendecomposition of the small tridiagonal.
* "Interface pieces with cross points removed": a face is the set of Gamma
  nodes shared by exactly the same two subdomains; nodes shared by three or
  more subdomains (cross points, and in 3D the wire-basket edges) are left
  to the diagonal of L.

Extension beyond the paper (its analysis is for one homogeneous material):
``weighted=True`` multiplies each skeleton element's mass and Laplacian by
the mean modulus of the two volume elements on either side of it, so the
interface norm follows the local scale of the Steklov-Poincare operator in
heterogeneous (SIMP) designs.  With a constant modulus c it is c times the
unweighted form.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dd, fe


# ---------------------------------------------------------------------------
# Skeleton element matrices (computed by quadrature, not typed in)
# ---------------------------------------------------------------------------

def _segment_matrices():
    pts, wts = fe.gauss_points_unit(2)
    Me = np.zeros((2, 2))
    Le = np.zeros((2, 2))
    for t, w in zip(pts, wts):
        N = np.array([1.0 - t, t])
        dN = np.array([-1.0, 1.0])
        Me += w * np.outer(N, N)
        Le += w * np.outer(dN, dN)
    return Me, Le


def _quad_matrices():
    pts, wts = fe.gauss_points_unit(2)
    off = fe.local_node_offsets(2)
    Me = np.zeros((4, 4))
    Le = np.zeros((4, 4))
    for i in range(2):
        for j in range(2):
            xi = (pts[i], pts[j])
            w = wts[i] * wts[j]
            N = np.array([(xi[0] if o[0] else 1 - xi[0]) *
                          (xi[1] if o[1] else 1 - xi[1]) for o in off])
            G = fe.shape_grads(2, xi)
            Me += w * np.outer(N, N)
            Le += w * (G @ G.T)
    return Me, Le


def skeleton_elements(prob, adjacent=False):
    """Node ids of every skeleton element (edges in 2D, faces in 3D) lying
    on an internal cut line/plane, each listed once.  With ``adjacent`` also
    return the ids of the two volume elements on either side."""
    nn = prob.nnodes_axis
    out, adj = [], []
    if prob.dim == 2:
        nx = prob.nel[0]

        def nid(i, j):
            return i + nn[0] * j

        def eid(i, j):
            return i + nx * j
        for c in prob.cuts[0][1:-1]:      # vertical lines x = c
            for j in range(prob.nel[1]):
                out.append((nid(c, j), nid(c, j + 1)))
                adj.append((eid(c - 1, j), eid(c, j)))
        for c in prob.cuts[1][1:-1]:      # horizontal lines y = c
            for i in range(prob.nel[0]):
                out.append((nid(i, c), nid(i + 1, c)))
                adj.append((eid(i, c - 1), eid(i, c)))
    else:
        def nid(i, j, k):
            return i + nn[0] * (j + nn[1] * k)

        def eid(i, j, k):
            return i + prob.nel[0] * (j + prob.nel[1] * k)
        for ax in range(3):
            a1, a2 = [a for a in range(3) if a != ax]
            for c in prob.cuts[ax][1:-1]:
                for p in range(prob.nel[a1]):
                    for q in range(prob.nel[a2]):
                        quad = []
                        for (dp, dq) in [(0, 0), (1, 0), (1, 1), (0, 1)]:
                            ijk = [0, 0, 0]
                            ijk[ax] = c
                            ijk[a1] = p + dp
                            ijk[a2] = q + dq
                            quad.append(nid(*ijk))
                        out.append(tuple(quad))
                        e = [0, 0, 0]
                        e[a1], e[a2] = p, q
                        e0, e1 = list(e), list(e)
                        e0[ax], e1[ax] = c - 1, c
                        adj.append((eid(*e0), eid(*e1)))
    arr = np.array(out, dtype=np.int64)
    adj = np.array(adj, dtype=np.int64)
    # an element lies on one cut line/plane only; no duplicates to drop
    if adjacent:
        return arr, adj
    return arr


def skeleton_matrices(prob, lumped=False, weighted=False, E=None):
    """(M, L, gamma node ids) on the free skeleton nodes, sparse CSR.
    ``weighted`` scales each skeleton element by the mean modulus of its two
    neighbouring volume elements (see the module docstring)."""
    els, adj = skeleton_elements(prob, adjacent=True)
    Me, Le = _segment_matrices() if prob.dim == 2 else _quad_matrices()
    if weighted:
        Ev = prob.E if E is None else E
        wts = 0.5 * (Ev[adj[:, 0]] + Ev[adj[:, 1]])
    else:
        wts = np.ones(len(els))
    m = els.shape[1]
    rows = np.repeat(els, m, axis=1).reshape(-1)
    cols = np.tile(els, (1, m)).reshape(-1)
    N = prob.n_nodes
    M = sp.coo_matrix(((wts[:, None] * Me.reshape(1, -1)).reshape(-1), (rows, cols)),
                      shape=(N, N)).tocsr()
    L = sp.coo_matrix(((wts[:, None] * Le.reshape(1, -1)).reshape(-1), (rows, cols)),
                      shape=(N, N)).tocsr()
    cls = dd.classify(prob)
    g = np.flatnonzero(cls == dd.GAMMA)
    if lumped:
        # row sums of the assembled mass, clamped columns included: each free
        # node keeps its full share of the skeleton's length/area
        Ml = sp.diags(np.asarray(M.sum(axis=1)).ravel()[g]).tocsr()
    M = M[g][:, g]
    L = L[g][:, g]
    if lumped:
        M = Ml
    return M.tocsr(), L.tocsr(), g


# ---------------------------------------------------------------------------
# Closed forms (generalised eigendecomposition, O(n_Gamma^3))
# ---------------------------------------------------------------------------

def gen_eig(M, L):
    """L V = M V diag(lam), V^T M V = I."""
    lam, V = sla.eigh(np.asarray(L.todense() if sp.issparse(L) else L),
                      np.asarray(M.todense() if sp.issparse(M) else M))
    return lam, V


def htilde(M, L, theta):
    """H~_theta = M (M^{-1} L)^{1-theta} as a dense matrix."""
    lam, V = gen_eig(M, L)
    Md = np.asarray(M.todense() if sp.issparse(M) else M)
    MV = Md @ V
    return MV @ np.diag(lam ** (1.0 - theta)) @ MV.T


def htilde_inv(M, L, theta):
    """H~_theta^{-1} = V diag(lam^{theta-1}) V^T."""
    lam, V = gen_eig(M, L)
    return V @ np.diag(lam ** (theta - 1.0)) @ V.T


def h_inv(M, L, theta):
    """H_theta^{-1} = V diag(1 / (1 + lam^{1-theta})) V^T (eq. (NumberEight))."""
    lam, V = gen_eig(M, L)
    return V @ np.diag(1.0 / (1.0 + lam ** (1.0 - theta))) @ V.T


def componentwise(Ainv, r, dim):
    """Apply a scalar interface operator to each displacement component of a
    Gamma vector in node-major interleaved layout (eq. (NumberNine))."""
    R = np.asarray(r).reshape(-1, dim)
    return (Ainv @ R).reshape(-1)


# ---------------------------------------------------------------------------
# Face blocks: L restricted to interface pieces, cross points removed
# ---------------------------------------------------------------------------

def face_partition(prob):
    """List of arrays of positions (into the Gamma node list) forming the
    faces, and the positions of the remaining (cross-point) nodes."""
    cls = dd.classify(prob)
    g = np.flatnonzero(cls == dd.GAMMA)
    en = fe.element_nodes(prob)
    sid = dd.element_subdomain(prob)
    pairs = np.unique(np.stack([en.reshape(-1),
                                np.repeat(sid, en.shape[1])], axis=1), axis=0)
    subs = {}
    for n, s in pairs:
        subs.setdefault(int(n), []).append(int(s))
    faces = {}
    rest = []
    for pos, n in enumerate(g):
        ss = tuple(sorted(subs[int(n)]))
        if len(ss) == 2:
            faces.setdefault(ss, []).append(pos)
        else:
            rest.append(pos)
    return [np.array(v, dtype=np.int64) for _, v in sorted(faces.items())], \
        np.array(rest, dtype=np.int64)


class FaceBlockPreconditioner:
    """Block Jacobi for L: exact inverse of L on each face, 1/L_ii on the
    cross-point nodes."""

    def __init__(self, prob, L):
        self.faces, self.rest = face_partition(prob)
        Ld = L.tocsr()
        self.inv = [np.linalg.inv(Ld[f][:, f].toarray()) for f in self.faces]
        self.dinv = 1.0 / Ld.diagonal()[self.rest]

    def apply(self, r):
        z = np.zeros_like(r)
        for f, A in zip(self.faces, self.inv):
            z[f] = A @ r[f]
        z[self.rest] = self.dinv * r[self.rest]
        return z


# ---------------------------------------------------------------------------
# Inverse Lanczos
# ---------------------------------------------------------------------------

def tridiag_power(alpha, beta, p):
    """f(T) e1 for the symmetric tridiagonal T (diag alpha, off-diag beta)
    and f(t) = t^p, via the eigendecomposition of T."""
    k = len(alpha)
    T = np.diag(alpha)
    if k > 1:
        T += np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    w, U = np.linalg.eigh(T)
    w = np.maximum(w, 0.0)
    return U @ (w ** p * U[0, :])


def inverse_lanczos(M, L, theta, r, solve_L=None, kmax=20, tol=1e-2,
                    reorth=True):
    """Approximate H~_theta^{-1} r by inverse Lanczos.

    Lanczos on C = L^{-1} M, self-adjoint in the M inner product, started
    from b = M^{-1} r; the answer is C^{1-theta} b.  Stops when two
    successive approximations differ by at most ``tol`` in the M norm
    (relative), or at ``kmax`` steps.  Returns (z, k).
    """
    Md = M.tocsr()
    if solve_L is None:
        luL = spla.splu(L.tocsc())
        solve_L = luL.solve
    Mlu = spla.splu(Md.tocsc())
    b = Mlu.solve(r)
    beta0 = np.sqrt(b @ (Md @ b))
    if beta0 == 0.0:
        return np.zeros_like(r), 0
    Q = [b / beta0]
    alpha, beta = [], []
    y_prev = None
    y = None
    for j in range(kmax):
        w = solve_L(Md @ Q[j])
        a = Q[j] @ (Md @ w)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[j - 1] * Q[j - 1]
        if reorth:
            for _ in range(2):
                for q in Q:
                    w = w - (q @ (Md @ w)) * q
        bnext = np.sqrt(max(w @ (Md @ w), 0.0))
        alpha.append(a)
        beta.append(bnext)
        y = beta0 * tridiag_power(np.array(alpha), np.array(beta),
                                  1.0 - theta)
        if y_prev is not None:
            diff = np.linalg.norm(y - np.append(y_prev, 0.0))
            if diff <= tol * np.linalg.norm(y):
                break
        y_prev = y
        if bnext <= 1e-14 * beta0:
            break
        Q.append(w / bnext)
    k = len(alpha)
    z = np.column_stack(Q[:k]) @ y
    return z, k
