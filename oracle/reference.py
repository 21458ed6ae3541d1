"""Reference solution of a large problem by the Schur route with
extended-precision iterative refinement (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

``fe.solve_direct`` (one sparse LU of the whole free system) does not fit a
1.6M-dof hexahedral mesh: its fill grows far past memory.  This module
reaches the same monolithic solution of Section 2, eq. (NumberFour), by the
exact reformulation of eq. (3MatSplit):

* K_II is the direct sum of the subdomain blocks K_{I_i I_i}
  (eq. (NumberFive)); each block gets its own sparse LU, so the interior
  solves are direct and exact up to rounding.  Blocks are spread over worker
  processes, which hold their factors for the whole run.
* The interface system S u_G = g is solved by flexible CG
  (``krylov.fcg``) preconditioned by Hhat_theta applied by inverse Lanczos
  (Section 3) with exact skeleton-Laplacian solves; the preconditioner only
  changes the iteration count, never the answer.
* The result is refined: r = f - K u is formed in long double from the
  assembled K, the correction K d = r is solved by the same Schur route in
  FP64, and u += d is accumulated in long double, until
  ||r|| <= tol ||f|| (free dofs).  Each round reduces the error by about the
  relative accuracy of its inner solve, so a few rounds carry u well below
  the accuracy of any single FP64 Krylov solve.

The block products K_IG v, K_GI w, K_GG v are slices of the assembled K
(eq. (NumberFour)'s partition), exactly as in ``dd.SchurOperator``.
Parity: pinned through ``dd.SchurOperator`` and ``fe.solve_direct`` on small
meshes (the two routes must agree; see tests/test_oracle_reference.py).
"""
from __future__ import annotations

import multiprocessing as mp
import time

import numpy as np
import scipy.sparse.linalg as spla

from . import dd, fe, iface, krylov


def _worker(conn, blocks):
    """Factor the given blocks, then answer solve requests until told to
    stop.  ``blocks`` is a list of CSC matrices."""
    lus = [spla.splu(B, permc_spec="MMD_AT_PLUS_A") for B in blocks]
    conn.send("ready")
    while True:
        msg = conn.recv()
        if msg is None:
            break
        conn.send([lu.solve(b) for lu, b in zip(lus, msg)])
    conn.close()


class BlockSchurOperator:
    """S v = K_GG v - K_GI K_II^{-1} K_IG v with K_II^{-1} applied block by
    block (one sparse LU per subdomain interior, eq. (NumberFive)).

    The interior ordering is that of ``dd.partition`` (subdomain, then node,
    then component), so the slices of one subdomain are contiguous."""

    def __init__(self, prob, E=None, workers=4, log=None):
        self.prob = prob
        t0 = time.perf_counter()
        K = fe.assemble(prob, E)
        I, G, cls = dd.partition(prob)
        self.I, self.G = I, G
        self.KIG = K[I][:, G].tocsr()
        self.KGI = K[G][:, I].tocsr()
        self.KGG = K[G][:, G].tocsr()
        KII = K[I][:, I].tocsr()
        del K
        # contiguous interior range of every subdomain
        owner = cls[I[::prob.dim] // prob.dim]
        starts = np.searchsorted(owner, np.arange(prob.n_sub), side="left")
        ends = np.searchsorted(owner, np.arange(prob.n_sub), side="right")
        self.ranges = [(int(a) * prob.dim, int(b) * prob.dim)
                       for a, b in zip(starts, ends) if b > a]
        blocks = [KII[a:b][:, a:b].tocsc() for a, b in self.ranges]
        del KII
        if log:
            log(f"blocks extracted in {time.perf_counter() - t0:.1f} s "
                f"({len(blocks)} interiors)")
        t0 = time.perf_counter()
        nw = max(1, min(workers, len(blocks)))
        # deal blocks round-robin by size so the workers carry similar work
        order = np.argsort([-B.shape[0] for B in blocks], kind="stable")
        self.assign = [list(order[w::nw]) for w in range(nw)]
        ctx = mp.get_context("fork")
        self.conns, self.procs = [], []
        for w in range(nw):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(b, [blocks[i] for i in self.assign[w]]))
            p.start()
            self.conns.append(a)
            self.procs.append(p)
        for c in self.conns:
            if c.recv() != "ready":
                raise RuntimeError("worker failed to factor its blocks")
        if log:
            log(f"{len(blocks)} interior blocks factored by {nw} workers in "
                f"{time.perf_counter() - t0:.1f} s")
        self.n = len(G)

    def close(self):
        for c in self.conns:
            c.send(None)
        for p in self.procs:
            p.join()
        self.conns, self.procs = [], []

    def solve_II(self, b):
        x = np.empty_like(b)
        for w, c in enumerate(self.conns):
            c.send([b[self.ranges[i][0]:self.ranges[i][1]] for i in self.assign[w]])
        for w, c in enumerate(self.conns):
            for i, xi in zip(self.assign[w], c.recv()):
                x[self.ranges[i][0]:self.ranges[i][1]] = xi
        return x

    def apply(self, v):
        w = self.solve_II(self.KIG @ v)
        return self.KGG @ v - self.KGI @ w

    def rhs(self, f):
        """g = f_G - K_GI K_II^{-1} f_I (first two lines of eq. (3MatSplit))."""
        return f[self.G] - self.KGI @ self.solve_II(f[self.I])

    def assemble_u(self, f, uG):
        """Back-substitution (third line of eq. (3MatSplit))."""
        uI = self.solve_II(f[self.I] - self.KIG @ uG)
        u = np.zeros(self.prob.ndof)
        u[self.I] = uI
        u[self.G] = uG
        return u


def lanczos_preconditioner(prob, theta=0.5, kmax=20, tol=1e-2, weighted=True, E=None):
    """z = Hhat_theta^{-1} r per displacement component by inverse Lanczos
    (Section 3) with lumped M and exact skeleton-Laplacian solves."""
    M, L, _ = iface.skeleton_matrices(prob, lumped=True, weighted=weighted, E=E)
    solve_L = spla.splu(L.tocsc()).solve
    d = prob.dim

    def P(r):
        R = r.reshape(-1, d)
        Z = np.column_stack([
            iface.inverse_lanczos(M, L, theta, np.ascontiguousarray(R[:, c]),
                                  solve_L=solve_L, kmax=kmax, tol=tol)[0]
            for c in range(d)])
        return Z.reshape(-1)
    return P


def refined_solve(prob, tol=1e-13, inner_tol=1e-8, max_rounds=6, workers=4,
                  theta=0.5, E=None, log=None, op=None):
    """Solve K u = f (free dofs) to ||f - K u|| <= tol ||f|| with the
    residual and u held in long double.

    Returns (u_longdouble_full, record) where record lists, per refinement
    round, the relative residual before the round, the interface iterations
    of its inner solve and ||d|| / ||u|| of its correction."""
    own_op = op is None
    if own_op:
        op = BlockSchurOperator(prob, E=E, workers=workers, log=log)
    try:
        P = lanczos_preconditioner(prob, theta=theta, E=E)
        Kff, free = fe.free_system(prob, E)
        Kl = Kff.astype(np.longdouble)
        del Kff
        fl = prob.f[free].astype(np.longdouble)
        nf = float(np.sqrt(np.sum(fl * fl)))
        x = np.zeros(len(free), dtype=np.longdouble)
        rounds = []
        for rnd in range(max_rounds + 1):
            r = fl - Kl @ x
            rel = float(np.sqrt(np.sum(r * r))) / nf
            if log:
                log(f"round {rnd}: relative residual {rel:.3e} (long double)")
            if rel <= tol or rnd == max_rounds:
                rounds.append({"rel_residual": rel})
                break
            rhs = np.zeros(prob.ndof)
            rhs[free] = np.asarray(r, dtype=np.float64)
            t0 = time.perf_counter()
            g = op.rhs(rhs)
            uG, its, hist = krylov.fcg(op.apply, g, P, tol=inner_tol, maxit=3000,
                                       ref_norm=np.linalg.norm(rhs[free]))
            d = op.assemble_u(rhs, uG)[free]
            x = x + d.astype(np.longdouble)
            xn = float(np.sqrt(np.sum(x * x)))
            rounds.append({"rel_residual": rel, "iterations": its,
                           "correction_rel": float(np.linalg.norm(d)) / xn,
                           "seconds": time.perf_counter() - t0})
            if log:
                log(f"round {rnd}: {its} interface iterations, "
                    f"||d||/||u|| = {rounds[-1]['correction_rel']:.3e}, "
                    f"{rounds[-1]['seconds']:.0f} s")
        u = np.zeros(prob.ndof, dtype=np.longdouble)
        u[free] = x
        return u, {"rounds": rounds, "rel_residual": rel}
    finally:
        if own_op:
            op.close()
