"""Non-overlapping domain decomposition and the Schur complement (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 1 splits Omega into subdomains Omega_i with skeleton Gamma; Section 2
partitions the unknowns as (u_I, u_Gamma) (eq. (NumberFour)) with
K_II = direct sum of K_{I_i I_i} (eq. (NumberFive)) and solves

    K_II u1_I = f_I,
    S u_Gamma = f_Gamma - K_Gamma I u1_I,
    K_II u2_I = -K_I Gamma u_Gamma,         u = (u1_I + u2_I, u_Gamma)

(eq. (3MatSplit)), S = K_GammaGamma - K_Gamma I K_II^{-1} K_I Gamma.

Reading of the node classes: a node belongs to the closure of every
subdomain that owns one of its elements.  Gamma is the set of nodes that lie
in two or more closures, minus clamped nodes; every other free node is
interior to exactly one subdomain (this is what makes K_II block diagonal).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe

GAMMA = -1
DIRICHLET = -2


def element_subdomain(prob):
    """Subdomain id of every element; ids run x fastest over the blocks."""
    el_axes = [np.arange(n) for n in prob.nel]
    grids = np.meshgrid(*el_axes, indexing="ij")
    ijk = [g.transpose().reshape(-1) for g in grids]
    sid = np.zeros(prob.n_el, dtype=np.int64)
    stride = 1
    for ax in range(prob.dim):
        cuts = np.asarray(prob.cuts[ax])
        blk = np.searchsorted(cuts, ijk[ax], side="right") - 1
        sid += stride * blk
        stride *= len(cuts) - 1
    return sid


def node_closure_count(prob):
    """For every node: number of distinct subdomain closures containing it,
    and one subdomain id that contains it."""
    en = fe.element_nodes(prob)
    sid = element_subdomain(prob)
    pairs = np.unique(np.stack([en.reshape(-1),
                                np.repeat(sid, en.shape[1])], axis=1), axis=0)
    count = np.bincount(pairs[:, 0], minlength=prob.n_nodes)
    owner = np.full(prob.n_nodes, -1, dtype=np.int64)
    owner[pairs[:, 0]] = pairs[:, 1]
    return count, owner


def classify(prob):
    """Per-node class: owning subdomain (>= 0) for interior nodes, GAMMA for
    interface nodes, DIRICHLET for clamped nodes."""
    count, owner = node_closure_count(prob)
    cls = np.where(count >= 2, GAMMA, owner)
    cls[fe.dirichlet_node_mask(prob)] = DIRICHLET
    return cls


def partition(prob):
    """Dof index arrays (I, G): I ordered by subdomain then node id then
    component; G ordered by node id then component."""
    cls = classify(prob)
    d = prob.dim
    inodes = np.flatnonzero(cls >= 0)
    inodes = inodes[np.argsort(cls[inodes], kind="stable")]
    gnodes = np.flatnonzero(cls == GAMMA)
    I = (d * inodes[:, None] + np.arange(d)).reshape(-1)
    G = (d * gnodes[:, None] + np.arange(d)).reshape(-1)
    return I, G, cls


def blocks(prob, E=None):
    K = fe.assemble(prob, E)
    I, G, _ = partition(prob)
    KII = K[I][:, I].tocsc()
    KIG = K[I][:, G].tocsc()
    KGI = K[G][:, I].tocsc()
    KGG = K[G][:, G].tocsc()
    return KII, KIG, KGI, KGG, I, G


def schur_dense(prob, E=None):
    """Dense S = K_GG - K_GI K_II^{-1} K_IG."""
    KII, KIG, KGI, KGG, I, G = blocks(prob, E)
    lu = spla.splu(KII)
    W = lu.solve(KIG.toarray())
    return KGG.toarray() - KGI @ W


class SchurOperator:
    """S applied matrix-free: S v = K_GG v - K_GI K_II^{-1} K_IG v, with the
    interior solves done by one sparse LU of the block-diagonal K_II."""

    def __init__(self, prob, E=None, f=None):
        self.prob = prob
        KII, KIG, KGI, KGG, I, G = blocks(prob, E)
        self.KIG, self.KGI, self.KGG = KIG, KGI, KGG
        self.I, self.G = I, G
        self.lu = spla.splu(KII, permc_spec="MMD_AT_PLUS_A")
        self.f = prob.f if f is None else f
        self.n = len(G)

    def solve_II(self, b):
        return self.lu.solve(b)

    def apply(self, v):
        w = self.solve_II(self.KIG @ v)
        return self.KGG @ v - self.KGI @ w

    def rhs(self):
        """g = f_G - K_GI K_II^{-1} f_I (first two lines of eq. (3MatSplit))."""
        u1 = self.solve_II(self.f[self.I])
        return self.f[self.G] - self.KGI @ u1

    def assemble_u(self, uG):
        """Back-substitution (third line of eq. (3MatSplit))."""
        uI = self.solve_II(self.f[self.I] - self.KIG @ uG)
        u = np.zeros(self.prob.ndof)
        u[self.I] = uI
        u[self.G] = uG
        return u


def schur_solve_dense(prob, E=None):
    """The three steps of eq. (3MatSplit) with a dense solve on S."""
    op = SchurOperator(prob, E)
    S = schur_dense(prob, E)
    uG = np.linalg.solve(S, op.rhs())
    return op.assemble_u(uG)


# ---------------------------------------------------------------------------
# Subdomain-local quantities (eq. (3MatSplit2) and the Steklov-Poincare
# splitting S = sum_i S_i of Section 1)
# ---------------------------------------------------------------------------

def subdomain_neumann(prob, s, E=None):
    """Neumann matrix of subdomain s: its elements only, over the free dofs
    of its closure.  Returns (K_s dense, closure node ids)."""
    if E is None:
        E = prob.E
    sid = element_subdomain(prob)
    en = fe.element_nodes(prob)
    mine = np.flatnonzero(sid == s)
    nodes = np.unique(en[mine])
    dmask = fe.dirichlet_node_mask(prob)
    nodes = nodes[~dmask[nodes]]
    d = prob.dim
    dofs = (d * nodes[:, None] + np.arange(d)).reshape(-1)
    Emask = np.zeros_like(E)
    Emask[mine] = E[mine]
    K = fe.assemble(prob, Emask)
    return K[dofs][:, dofs].toarray(), nodes


def local_schur(prob, s, E=None):
    """S_s = K^s_GG - K^s_GI (K^s_II)^{-1} K^s_IG on the Gamma nodes of the
    closure of s.  Returns (S_s, Gamma node ids)."""
    Ks, nodes = subdomain_neumann(prob, s, E)
    cls = classify(prob)
    d = prob.dim
    isG = np.repeat(cls[nodes] == GAMMA, d)
    iI = np.flatnonzero(~isG)
    iG = np.flatnonzero(isG)
    KII = Ks[np.ix_(iI, iI)]
    KIG = Ks[np.ix_(iI, iG)]
    KGG = Ks[np.ix_(iG, iG)]
    Ss = KGG - KIG.T @ np.linalg.solve(KII, KIG)
    return Ss, nodes[cls[nodes] == GAMMA]


def floating_subdomains(prob):
    """Subdomains whose closure contains no clamped node."""
    sid = element_subdomain(prob)
    en = fe.element_nodes(prob)
    dmask = fe.dirichlet_node_mask(prob)
    touch = np.zeros(prob.n_sub, dtype=bool)
    np.logical_or.at(touch, sid, dmask[en].any(axis=1))
    return np.flatnonzero(~touch)
