"""FP64 finite elements for isotropic linear elasticity (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows the paper's Section 1 (the boundary value problem, the linearised
strain tensor and Hooke's law with the Lame constants mu and lambda-hat) and
Section 2 (the discrete system K u = f of eq. (NumberFour)).  Readings of
details the paper leaves to its companion report:

* element type: bilinear quadrilaterals (2D) and trilinear hexahedra (3D) on
  unit-size elements, integrated exactly by 2x2 / 2x2x2 Gauss rules;
* 2D is plane stress with unit thickness: the 3D Lame constant lambda-hat is
  replaced by lambda* = 2 mu lambda-hat / (lambda-hat + 2 mu);
* the topology-optimisation stiffness K(rho) = sum_i rho_i K_i of eq.
  (NumberTen) is realised as K(E) = sum_e E_e P_e^T K0 P_e with K0 the
  element matrix for unit modulus.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# Constitutive law (Section 1, Hooke's law and the Lame constants)
# ---------------------------------------------------------------------------

def lame(E, nu):
    """Return (mu, lambda_hat) for Young's modulus E and Poisson ratio nu."""
    mu = E / (2.0 * (1.0 + nu))
    lam = nu * E / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def dmatrix(dim, nu, E=1.0):
    """Elasticity matrix D with sigma = D eps in Voigt notation.

    Strain vectors use engineering shear strains:
      2D: (e_xx, e_yy, g_xy)
      3D: (e_xx, e_yy, e_zz, g_xy, g_yz, g_xz)
    sigma = 2 mu eps + lambda tr(eps) I  (Section 1); with engineering shear
    the shear rows carry mu.
    """
    mu, lam = lame(E, nu)
    if dim == 2:
        lam = 2.0 * mu * lam / (lam + 2.0 * mu)  # plane stress
        nn, ns = 2, 1
    else:
        nn, ns = 3, 3
    D = np.zeros((nn + ns, nn + ns))
    D[:nn, :nn] = lam
    D[np.arange(nn), np.arange(nn)] += 2.0 * mu
    D[np.arange(nn, nn + ns), np.arange(nn, nn + ns)] = mu
    return D


# ---------------------------------------------------------------------------
# Reference element
# ---------------------------------------------------------------------------

def local_node_offsets(dim):
    """Corner offsets of the unit element, counter-clockwise; 3D: z=0 face
    then z=1 face."""
    quad = [(0, 0), (1, 0), (1, 1), (0, 1)]
    if dim == 2:
        return np.array(quad, dtype=np.int64)
    return np.array([q + (0,) for q in quad] + [q + (1,) for q in quad],
                    dtype=np.int64)


def shape_grads(dim, xi):
    """Gradients dN_a/dx of the (tri)linear shape functions at point xi in
    the unit element; returns array (n_local_nodes, dim)."""
    off = local_node_offsets(dim)
    G = np.zeros((len(off), dim))
    for a, o in enumerate(off):
        # N_a = prod_k phi(o_k, xi_k), phi(1,t)=t, phi(0,t)=1-t
        vals = [xi[k] if o[k] == 1 else 1.0 - xi[k] for k in range(dim)]
        ders = [1.0 if o[k] == 1 else -1.0 for k in range(dim)]
        for k in range(dim):
            g = ders[k]
            for m in range(dim):
                if m != k:
                    g *= vals[m]
            G[a, k] = g
    return G


def bmatrix(dim, G):
    """Strain-displacement matrix: eps = B u_e, u_e node-major interleaved."""
    n = G.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * n))
        for a in range(n):
            dx, dy = G[a]
            B[0, 2 * a] = dx
            B[1, 2 * a + 1] = dy
            B[2, 2 * a] = dy
            B[2, 2 * a + 1] = dx
        return B
    B = np.zeros((6, 3 * n))
    for a in range(n):
        dx, dy, dz = G[a]
        B[0, 3 * a] = dx
        B[1, 3 * a + 1] = dy
        B[2, 3 * a + 2] = dz
        B[3, 3 * a] = dy
        B[3, 3 * a + 1] = dx
        B[4, 3 * a + 1] = dz
        B[4, 3 * a + 2] = dy
        B[5, 3 * a] = dz
        B[5, 3 * a + 2] = dx
    return B


def gauss_points_unit(order=2):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(order)
    return 0.5 * (x + 1.0), 0.5 * w


def element_stiffness(dim, nu, E=1.0, order=2):
    """K0 = integral over the unit element of B^T D B (Gauss, exact)."""
    D = dmatrix(dim, nu, E)
    pts, wts = gauss_points_unit(order)
    nloc = 2 ** dim
    K = np.zeros((dim * nloc, dim * nloc))
    for idx in itertools.product(range(order), repeat=dim):
        xi = [pts[i] for i in idx]
        w = np.prod([wts[i] for i in idx])
        B = bmatrix(dim, shape_grads(dim, xi))
        K += w * (B.T @ D @ B)
    return K


# ---------------------------------------------------------------------------
# Mesh bookkeeping
# ---------------------------------------------------------------------------

def node_coords(prob):
    """(n_nodes, dim) integer coordinates, node id = x fastest."""
    axes = [np.arange(n) for n in prob.nnodes_axis]
    grids = np.meshgrid(*axes, indexing="ij")
    # flatten with x fastest
    return np.stack([g.transpose().reshape(-1) for g in grids], axis=1)


def element_nodes(prob):
    """(n_el, 2^dim) global node ids of every element in local order."""
    dim = prob.dim
    nn = prob.nnodes_axis
    el_axes = [np.arange(n) for n in prob.nel]
    grids = np.meshgrid(*el_axes, indexing="ij")
    base = [g.transpose().reshape(-1) for g in grids]  # element origin ijk
    off = local_node_offsets(dim)
    out = np.zeros((prob.n_el, len(off)), dtype=np.int64)
    for a, o in enumerate(off):
        if dim == 2:
            out[:, a] = (base[0] + o[0]) + nn[0] * (base[1] + o[1])
        else:
            out[:, a] = (base[0] + o[0]) + nn[0] * (
                (base[1] + o[1]) + nn[1] * (base[2] + o[2]))
    return out


def element_dofs(prob):
    en = element_nodes(prob)
    d = prob.dim
    dofs = (d * en[:, :, None] + np.arange(d)[None, None, :])
    return dofs.reshape(prob.n_el, -1)


def dirichlet_node_mask(prob):
    """True for nodes on a clamped face (u = 0 on the Dirichlet boundary)."""
    xyz = node_coords(prob)
    m = np.zeros(prob.n_nodes, dtype=bool)
    for ax in range(prob.dim):
        if prob.clamp & (1 << (2 * ax)):
            m |= xyz[:, ax] == 0
        if prob.clamp & (1 << (2 * ax + 1)):
            m |= xyz[:, ax] == prob.nel[ax]
    return m


def dirichlet_dof_mask(prob):
    return np.repeat(dirichlet_node_mask(prob), prob.dim)


# ---------------------------------------------------------------------------
# Assembly and operator application (Section 2, eq. (NumberFour); eq.
# (NumberTen) for K(rho) = sum rho_i K_i)
# ---------------------------------------------------------------------------

def assemble(prob, E=None):
    """Full K(E) (all dofs, Dirichlet rows/cols included) as CSR FP64."""
    if E is None:
        E = prob.E
    K0 = element_stiffness(prob.dim, prob.nu)
    dofs = element_dofs(prob)
    m = dofs.shape[1]
    rows = np.repeat(dofs, m, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, m)).reshape(-1)
    vals = (E[:, None] * K0.reshape(1, -1)).reshape(-1)
    K = sp.coo_matrix((vals, (rows, cols)), shape=(prob.ndof, prob.ndof))
    return K.tocsr()


def apply_K_elementwise(prob, u, E=None):
    """y = K(E) u with Dirichlet entries of u treated as 0 and of y set to 0.

    Element by element: y = sum_e E_e P_e^T K0 P_e u.  Used where assembling
    K would not fit comfortably (large 3D meshes).
    """
    if E is None:
        E = prob.E
    K0 = element_stiffness(prob.dim, prob.nu)
    dmask = dirichlet_dof_mask(prob)
    uu = np.where(dmask, 0.0, u)
    dofs = element_dofs(prob)
    y = np.zeros(prob.ndof)
    chunk = 65536
    for s in range(0, prob.n_el, chunk):
        dd = dofs[s:s + chunk]
        ue = uu[dd]
        ye = (ue @ K0.T) * E[s:s + chunk, None]
        y += np.bincount(dd.reshape(-1), weights=ye.reshape(-1),
                         minlength=prob.ndof)
    y[dmask] = 0.0
    return y


def free_system(prob, E=None):
    """(K_ff, free dof index array) after Dirichlet elimination."""
    K = assemble(prob, E)
    free = np.flatnonzero(~dirichlet_dof_mask(prob))
    return K[free][:, free].tocsc(), free


def solve_direct(prob, E=None, f=None, refine=3):
    """u solving K u = f on free dofs (u = 0 on Dirichlet dofs).

    Sparse LU (SuperLU, minimum-degree ordering on A^T + A) followed by
    iterative refinement whose residuals are accumulated in long double, so
    the reference is accurate well below the solver tolerances under test.
    Returns the full-length u.
    """
    if f is None:
        f = prob.f
    Kff, free = free_system(prob, E)
    lu = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A")
    ff = f[free]
    x = lu.solve(ff)
    Kl = Kff.astype(np.longdouble)
    fl = ff.astype(np.longdouble)
    for _ in range(refine):
        r = fl - Kl @ x.astype(np.longdouble)
        x = x + lu.solve(np.asarray(r, dtype=np.float64))
    u = np.zeros(prob.ndof)
    u[free] = x
    return u


def residual_norm(prob, u, E=None, f=None):
    """||f - K u||_2 / ||f||_2 over free dofs, matrix-free, in FP64."""
    if f is None:
        f = prob.f
    dmask = dirichlet_dof_mask(prob)
    r = np.where(dmask, 0.0, f) - apply_K_elementwise(prob, u, E)
    return np.linalg.norm(r) / np.linalg.norm(np.where(dmask, 0.0, f))


def compliance(f, u):
    """f^T u, the objective of eq. (NumberTen)."""
    return float(np.dot(f, u))


def rigid_body_modes(coords, dim):
    """Columns spanning infinitesimal rigid motions at the given points."""
    n = coords.shape[0]
    x = coords.astype(np.float64)
    if dim == 2:
        R = np.zeros((2 * n, 3))
        R[0::2, 0] = 1.0
        R[1::2, 1] = 1.0
        R[0::2, 2] = -x[:, 1]
        R[1::2, 2] = x[:, 0]
        return R
    R = np.zeros((3 * n, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    # rotations about z, x, y
    R[0::3, 3] = -x[:, 1]
    R[1::3, 3] = x[:, 0]
    R[1::3, 4] = -x[:, 2]
    R[2::3, 4] = x[:, 1]
    R[2::3, 5] = -x[:, 0]
    R[0::3, 5] = x[:, 2]
    return R
