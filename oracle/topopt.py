"""Topology optimisation by the fixed-point loop of Section 5 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 5 minimises the compliance f^T u subject to K(rho) u = f with
K(rho) = sum_i rho_i K_i (the Variable Thickness Sheet problem,
eq. (NumberTen)), a volume bound sum_i rho_i <= V and box bounds on rho,
by repeating: (1) finite element analysis, (2) an Optimality Criteria (OC)
density update, (3) a convergence check; the Krylov tolerance of step 1
adapts to successive compliance values.

Readings where the section is silent:
* element modulus E_e = rho_e (the linear K(rho) of eq. (NumberTen)); an
  optional SIMP power p gives E_e = emin + rho_e^p (1 - emin);
* OC update (the textbook form for a compliance objective): with
  g_e = -dc/drho_e = dE_e/drho_e * u_e^T K0 u_e and Lagrange multiplier
  Lambda of the volume constraint,
      rho_e <- clamp(rho_e (g_e / Lambda)^eta, max(lo, rho_e - move),
                                               min(hi, rho_e + move)),
  eta = 1/2, move = 0.2, Lambda chosen so that sum_e rho_e = V;
* adaptive tolerance: tol_k = clamp(|c_{k-1} - c_{k-2}| / c_{k-1},
  tol_min, tol_max); the first two analyses use tol_max;
* stop when max_e |rho_new - rho_old| <= change_tol.
"""
from __future__ import annotations

import numpy as np

from . import fe


def element_energies(prob, u):
    """s_e = u_e^T K0 u_e for every element (unit modulus), the element
    strain energy (times two) whose negative is dc/dE_e.  Clamped dofs of u
    count as zero."""
    K0 = fe.element_stiffness(prob.dim, prob.nu)
    dofs = fe.element_dofs(prob)
    uu = np.where(fe.dirichlet_dof_mask(prob), 0.0, u)
    ue = uu[dofs]
    return np.einsum("ei,ij,ej->e", ue, K0, ue)


def moduli(rho, p=1.0, emin=0.0):
    """E_e from rho_e: rho itself for the Variable Thickness Sheet (p = 1,
    emin = 0), otherwise emin + rho^p (1 - emin)."""
    if p == 1.0 and emin == 0.0:
        return rho.copy()
    return emin + rho ** p * (1.0 - emin)


def sensitivity_weights(rho, p=1.0, emin=0.0):
    """dE_e/drho_e."""
    if p == 1.0 and emin == 0.0:
        return np.ones_like(rho)
    return p * rho ** (p - 1.0) * (1.0 - emin)


def oc_candidate(rho, g, lam, lo, hi, move, eta):
    """The OC update for multiplier lam (elementwise)."""
    lower = np.maximum(lo, rho - move)
    upper = np.minimum(hi, rho + move)
    return np.clip(rho * (g / lam) ** eta, lower, upper)


def oc_update(rho, g, volume, lo=1e-3, hi=1.0, move=0.2, eta=0.5, rtol=1e-13):
    """OC density update; Lambda by bisection on log(Lambda) until the
    bracket's relative width is below rtol.  Returns (rho_new, Lambda)."""
    lower = np.maximum(lo, rho - move)
    upper = np.minimum(hi, rho + move)
    if upper.sum() <= volume:  # the constraint cannot bind
        return upper.copy(), 0.0
    if lower.sum() >= volume:
        return lower.copy(), np.inf
    pos = g > 0
    # beyond these multipliers every element sits on its lower / upper bound
    lam_hi = np.max(g[pos] * (rho[pos] / lower[pos]) ** (1.0 / eta)) * 2.0
    lam_lo = np.min(g[pos] * (rho[pos] / upper[pos]) ** (1.0 / eta)) * 0.5
    a, b = np.log(lam_lo), np.log(lam_hi)
    while b - a > rtol:
        mid = 0.5 * (a + b)
        if oc_candidate(rho, g, np.exp(mid), lo, hi, move, eta).sum() > volume:
            a = mid
        else:
            b = mid
    lam = np.exp(0.5 * (a + b))
    return oc_candidate(rho, g, lam, lo, hi, move, eta), lam


def adaptive_tolerance(c_hist, tol_min=1e-8, tol_max=1e-2):
    """Krylov tolerance for the next analysis from the compliance history."""
    if len(c_hist) < 2:
        return tol_max
    d = abs(c_hist[-1] - c_hist[-2]) / abs(c_hist[-1])
    return float(min(tol_max, max(tol_min, d)))


def optimise(prob, volfrac=0.5, lo=1e-3, hi=1.0, move=0.2, eta=0.5, p=1.0, emin=0.0,
             change_tol=1e-2, maxit=100, solve=None):
    """The fixed-point loop.  ``solve(E, tol, u0)`` returns (u, krylov
    iterations); by default an exact sparse direct solve (0 iterations).
    Returns a dict with the final rho, u and the per-step history."""
    if solve is None:
        def solve(E, tol, u0):
            return fe.solve_direct(prob, E), 0
    rho = np.full(prob.n_el, volfrac)
    volume = volfrac * prob.n_el
    u = np.zeros(prob.ndof)
    c_hist, its, tols, changes = [], [], [], []
    for k in range(maxit):
        tol = adaptive_tolerance(c_hist)
        E = moduli(rho, p, emin)
        u, n = solve(E, tol, u)
        c_hist.append(fe.compliance(prob.f, u))
        its.append(n)
        tols.append(tol)
        g = sensitivity_weights(rho, p, emin) * element_energies(prob, u)
        rho_new, lam = oc_update(rho, g, volume, lo, hi, move, eta)
        change = float(np.max(np.abs(rho_new - rho)))
        changes.append(change)
        rho = rho_new
        if change <= change_tol:
            break
    return {"rho": rho, "u": u, "compliance": c_hist, "iterations": its,
            "tolerances": tols, "changes": changes, "steps": len(c_hist)}
