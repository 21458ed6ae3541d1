"""The benchmark workloads at full size, in the benchmark's launch
configuration (automatic dissection, autotuned substitution variants).

2D 512x256 SIMP cantilever (263k dofs, 512 subdomains): against the
oracle's direct solve.  3D 128x64x64 SIMP cantilever (1.6M dofs, 160 uneven
subdomains): displacements and compliance against the stored oracle
reference (tests/golden, written by make_reference.py: the oracle's Schur
route refined in long double to rel.res 3.6e-15), the oracle's
element-by-element K apply and its residual of the GPU solution, and
interior solves of sampled subdomains against the oracle's sparse
factorisation of that block, the S apply for vectors supported on one
interface face, and the interface preconditioner on the whole 83,178-node
skeleton against the oracle's inverse Lanczos."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as w
from oracle import fe, iface

from gpu_util import require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _reference(name):
    base = os.path.join(GOLDEN, f"{name}_u_ref")
    with open(base + ".json") as fh:
        meta = json.load(fh)
    return np.load(base + ".npy"), meta


def _problem(wk):
    from paper_1501_06211_amd import edd
    prob = edd.Problem.from_workload(wk)
    prob.set_element_moduli(to_cuda(wk.E))
    prob.autotune()
    return prob


def test_2d_512x256_against_direct_solve():
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = w.cantilever2d_simp_512x256()
    prob = _problem(wk)
    f = to_cuda(wk.f)
    uref = fe.solve_direct(wk)
    cref = fe.compliance(wk.f, uref)
    # kappa(K) ~ 1e7 here: the FP64 interface iteration stalls near 1e-10, so
    # the solve runs to that reachable residual and the parity bars apply to
    # displacements and compliance
    for mode in (edd.MODE_F64, edd.MODE_RELAXED):
        u, st = prob.solve(f, tol=1e-10, maxit=8000, precision=mode, mixed_inner_tol=0.1)
        un = to_np(u)
        err = float(np.linalg.norm(un - uref) / np.linalg.norm(uref))
        cerr = abs(st["compliance"] - cref) / abs(cref)
        print(f"2D 512x256 mode {mode}: its={st['iterations']} res={st['rel_residual']:.2e} "
              f"u_err={err:.2e} c_err={cerr:.2e} flags={st['flags']}")
        assert st["rel_residual"] <= 1e-10
        assert err <= 1e-8 and cerr <= 1e-10
    prob.close()


def _sub_block(wk, sid):
    """Subdomain sid as its own problem with its cut faces clamped: the free
    system is exactly the interior block K_{I_i I_i}."""
    nb = [len(c) - 1 for c in wk.cuts]
    b = [sid % nb[0], (sid // nb[0]) % nb[1], sid // (nb[0] * nb[1])]
    lo = [int(wk.cuts[a][b[a]]) for a in range(3)]
    hi = [int(wk.cuts[a][b[a] + 1]) for a in range(3)]
    E3 = wk.E.reshape(wk.nel[2], wk.nel[1], wk.nel[0])
    Es = E3[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].reshape(-1)
    dims = [hi[a] - lo[a] for a in range(3)]
    sub = w.cantilever3d(*dims, cuts=([0, dims[0]], [0, dims[1]], [0, dims[2]]), E=Es)
    clamp = 0
    for a in range(3):
        if lo[a] > 0 or (wk.clamp >> (2 * a)) & 1:
            clamp |= 1 << (2 * a)
        if hi[a] < wk.nel[a] or (wk.clamp >> (2 * a + 1)) & 1:
            clamp |= 1 << (2 * a + 1)
    sub.clamp = clamp
    return sub, lo


def test_3d_128x64x64_properties_and_sampled_interior_blocks():
    require_gpu()
    wk = w.cantilever3d_simp_128x64x64()
    prob = _problem(wk)
    assert prob.info["band_blocks"] > prob.info["n_sub"]  # the 16^3 blocks are dissected
    # full-size K apply
    rng = np.random.default_rng(5)
    v = rng.standard_normal(wk.ndof)
    y = to_np(prob.apply_K(to_cuda(v)))
    ref = fe.apply_K_elementwise(wk, v)
    kerr = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert kerr <= 1e-14
    # displacements and compliance against the stored oracle reference: the
    # benchmark's own solve (FP64, tol 1e-8), the tightest FP64 solve the
    # interface iteration reaches, and the mixed path at the benchmark's
    # switch point; the oracle also recomputes the residual of the GPU u
    from paper_1501_06211_amd import edd
    u_ref, meta = _reference(wk.name)
    assert meta["rel_residual_long_double"] <= 1e-13
    c_ref = meta["compliance"]
    f = to_cuda(wk.f)
    free = ~fe.dirichlet_dof_mask(wk)
    for label, opts in (("bench FP64 tol 1e-8", dict(tol=1e-8)),
                        ("FP64 tol 1e-11", dict(tol=1e-11)),
                        ("mixed, FP32 factors below 1e-3", dict(
                            tol=1e-8, precision=edd.MODE_RELAXED, mixed_inner_tol=1e-3))):
        u, st = prob.solve(f, maxit=5000, **opts)
        un = to_np(u)
        err = float(np.linalg.norm(un - u_ref) / np.linalg.norm(u_ref))
        cerr = abs(st["compliance"] - c_ref) / abs(c_ref)
        r = (wk.f - fe.apply_K_elementwise(wk, un))[free]
        rel = np.linalg.norm(r) / np.linalg.norm(wk.f[free])
        print(f"3D 128x64x64 {label}: its={st['iterations']} GPU res={st['rel_residual']:.2e} "
              f"oracle res={rel:.2e} u_err={err:.2e} c_err={cerr:.2e} flags={st['flags']}")
        assert abs(rel - st["rel_residual"]) <= 1e-2 * rel
        assert rel <= 1.01 * opts["tol"] or st["status"] == edd.NOT_CONVERGED
        assert err <= 1e-8 and cerr <= 1e-10
    # interior solves of sampled subdomains: 16^3 (dissected), 16x16x12,
    # and one touching the clamp
    b = rng.standard_normal(prob.n_interior_dofs)
    x = to_np(prob.solve_interior(to_cuda(b)))
    slots = prob.interior_nodes()
    nn = [n + 1 for n in wk.nel]
    nodes = slots
    node_xyz = np.stack([nodes % nn[0], (nodes // nn[0]) % nn[1], nodes // (nn[0] * nn[1])], 1)
    for sid in (5, 101, 64):
        sub, lo = _sub_block(wk, sid)
        Kff, _ = fe.free_system(sub)
        snn = [n + 1 for n in sub.nel]
        inside = np.all((node_xyz >= lo) & (node_xyz < np.array(lo) + np.array(snn)), axis=1)
        rel_xyz = node_xyz[inside] - np.array(lo)
        snode = rel_xyz[:, 0] + snn[0] * (rel_xyz[:, 1] + snn[1] * rel_xyz[:, 2])
        sfree = np.flatnonzero(~fe.dirichlet_dof_mask(sub))
        pos = np.full(sub.ndof, -1)
        pos[sfree] = np.arange(len(sfree))
        gslots = (np.flatnonzero(inside)[:, None] * 3 + np.arange(3)).reshape(-1)
        sdofs = (snode[:, None] * 3 + np.arange(3)).reshape(-1)
        assert (pos[sdofs] >= 0).all() and len(sdofs) == Kff.shape[0]
        bs = np.zeros(Kff.shape[0])
        bs[pos[sdofs]] = b[gslots]
        xs = spla.spsolve(Kff.tocsc(), bs)
        err = np.linalg.norm(x[gslots] - xs[pos[sdofs]]) / np.linalg.norm(xs)
        print(f"  subdomain {sid} ({Kff.shape[0]} dofs): interior solve rel err {err:.2e}")
        assert err <= 1e-12
    prob.close()


@pytest.mark.parametrize("mass", [0, 1])
def test_3d_128x64x64_preconditioner_against_oracle_lanczos(mass):
    """The interface preconditioner on the benchmark's whole skeleton (83,178
    interface nodes, modulus-weighted operators as in the benchmark): three
    inverse-Lanczos steps with Laplacian solves to 1e-14 against the
    oracle's three steps with exact (sparse LU) Laplacian solves, for the
    lumped (mass 0) and the consistent (mass 1) skeleton mass.  The
    benchmark's own fixed-step apply (four inner iterations per step)
    approximates the same operator; its distance is printed."""
    require_gpu()
    from paper_1501_06211_amd import edd
    wk = w.cantilever3d_simp_128x64x64()
    prob = _problem(wk)
    M, L, g = iface.skeleton_matrices(wk, lumped=(mass == 0), weighted=True)
    assert len(g) == prob.n_gamma
    lu = spla.splu(L.tocsc())
    r = np.random.default_rng(9).standard_normal((len(g), 3))
    zref = np.column_stack([iface.inverse_lanczos(M, L, 0.5, r[:, c], solve_L=lu.solve,
                                                  kmax=3, tol=0.0)[0]
                            for c in range(3)]).reshape(-1)
    rc = to_cuda(r.reshape(-1))
    z = to_np(prob.apply_precond(rc, precond=edd.PC_HTHETA, theta=0.5, lanczos_kmax=3,
                                 lanczos_tol=0.0, inner_tol=1e-14, inner_maxit=5000,
                                 interface_weighting=1, mass_matrix=mass))
    err = float(np.linalg.norm(z - zref) / np.linalg.norm(zref))
    zb = to_np(prob.apply_precond(rc, precond=edd.PC_HTHETA, mass_matrix=mass))
    errb = float(np.linalg.norm(zb - zref) / np.linalg.norm(zref))
    print(f"3D 128x64x64 preconditioner, mass {mass}: 3 exact-solve steps vs oracle {err:.2e}; "
          f"benchmark's 3 x 4 form vs oracle {errb:.2e}")
    assert err <= 1e-8
    prob.close()


def _interior_solve(wk, sid, b):
    """K_{I_i I_i}^{-1} b on subdomain sid's interior dofs (b full-length;
    only those entries read), by the oracle's sparse factorisation of the
    subdomain's own free system; full-length result, zero elsewhere."""
    sub, lo = _sub_block(wk, sid)
    Kff, _ = fe.free_system(sub)
    nn = [n + 1 for n in wk.nel]
    snn = [n + 1 for n in sub.nel]
    dofs = np.flatnonzero(~fe.dirichlet_dof_mask(sub))
    ln, comp = dofs // 3, dofs % 3
    lx, ly, lz = ln % snn[0], (ln // snn[0]) % snn[1], ln // (snn[0] * snn[1])
    gdof = 3 * ((lo[0] + lx) + nn[0] * ((lo[1] + ly) + nn[1] * (lo[2] + lz))) + comp
    out = np.zeros(wk.ndof)
    out[gdof] = spla.spsolve(Kff.tocsc(), b[gdof])
    return out


@pytest.mark.parametrize("layer", [0, 2])
def test_3d_128x64x64_S_apply_on_sampled_faces(layer):
    """S v at full size, in the benchmark's launch configuration, for v
    supported inside one interface face (x = 48 between the subdomains at
    x-blocks 2 and 3, y-block 1, z-block `layer`; layer 0 holds the 16^3
    subdomains whose interiors are dissected).  Then K [0; v] touches only
    those two interiors, and the oracle forms S v = (K [-K_II^{-1}
    (K [0; v])_I ; v])_Gamma with two sparse interior solves and two
    element-by-element K applies, compared on every interface dof."""
    require_gpu()
    from oracle import dd
    wk = w.cantilever3d_simp_128x64x64()
    prob = _problem(wk)
    nn = [n + 1 for n in wk.nel]
    zc = wk.cuts[2]
    ys, zs = np.arange(17, 32), np.arange(zc[layer] + 1, zc[layer + 1])
    face = (48 + nn[0] * (ys[:, None] + nn[1] * zs[None, :])).reshape(-1)
    rng = np.random.default_rng(11 + layer)
    v = np.zeros(wk.ndof)
    v[(3 * face[:, None] + np.arange(3)).reshape(-1)] = rng.standard_normal(3 * len(face))
    y = fe.apply_K_elementwise(wk, v)
    nb = [len(c) - 1 for c in wk.cuts]
    x = sum(_interior_solve(wk, sx + nb[0] * (1 + nb[1] * layer), y) for sx in (2, 3))
    Sv = fe.apply_K_elementwise(wk, v - x)
    g = np.flatnonzero(dd.classify(wk) == dd.GAMMA)
    gd = (3 * g[:, None] + np.arange(3)).reshape(-1)
    ref = Sv[gd]
    out = to_np(prob.apply_S(to_cuda(v[gd])))
    err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    print(f"3D 128x64x64 S v on a face of z-layer {layer} ({len(face)} nodes): rel err {err:.2e}")
    assert err <= 1e-12
    prob.close()


def test_3d_128x64x64_fgmres_on_K_against_reference():
    """The paper's own Krylov method at full size: flexible GMRES on the whole
    K, right-preconditioned by the block-triangular P~ with S~ = Hhat_theta,
    solved to the tightest residual the benchmark's FP64 solve reaches, then
    displacements and compliance against the stored oracle reference."""
    require_gpu()
    wk = w.cantilever3d_simp_128x64x64()
    prob = _problem(wk)
    u_ref, meta = _reference(wk.name)
    u, st = prob.solve_gmres(to_cuda(wk.f), tol=1e-11, maxit=3000)
    err = float(np.linalg.norm(to_np(u) - u_ref) / np.linalg.norm(u_ref))
    cerr = abs(st["compliance"] - meta["compliance"]) / abs(meta["compliance"])
    print(f"3D 128x64x64 FGMRES on K with P~: its={st['iterations']} "
          f"res={st['rel_residual']:.2e} u_err={err:.2e} c_err={cerr:.2e}")
    assert st["rel_residual"] <= 1e-11
    assert err <= 1e-8 and cerr <= 1e-10
    prob.close()


def _sub_block_2d(wk, sid):
    """2D subdomain sid as its own problem with its cut faces clamped."""
    nb = [len(c) - 1 for c in wk.cuts]
    b = [sid % nb[0], sid // nb[0]]
    lo = [int(wk.cuts[a][b[a]]) for a in range(2)]
    hi = [int(wk.cuts[a][b[a] + 1]) for a in range(2)]
    E2 = wk.E.reshape(wk.nel[1], wk.nel[0])
    Es = E2[lo[1]:hi[1], lo[0]:hi[0]].reshape(-1)
    dims = [hi[a] - lo[a] for a in range(2)]
    sub = w.cantilever2d(*dims, cuts=([0, dims[0]], [0, dims[1]]), E=Es)
    clamp = 0
    for a in range(2):
        if lo[a] > 0 or (wk.clamp >> (2 * a)) & 1:
            clamp |= 1 << (2 * a)
        if hi[a] < wk.nel[a] or (wk.clamp >> (2 * a + 1)) & 1:
            clamp |= 1 << (2 * a + 1)
    sub.clamp = clamp
    return sub, lo


def test_2d_512x256_S_apply_both_routes_on_a_sampled_edge():
    """S v at the 2D benchmark size (512 subdomains) through the interior
    factors and through the explicit local Schur complements S_i, for v
    inside one interface edge (x = 48 between x-blocks 2 and 3, y-block 3):
    against the oracle's S v from two sparse interior solves and two
    element-by-element K applies."""
    require_gpu()
    from oracle import dd
    wk = w.cantilever2d_simp_512x256()
    prob = _problem(wk)
    nn = [n + 1 for n in wk.nel]
    edge = 48 + nn[0] * np.arange(49, 64)
    v = np.zeros(wk.ndof)
    v[(2 * edge[:, None] + np.arange(2)).reshape(-1)] = \
        np.random.default_rng(13).standard_normal(2 * len(edge))
    y = fe.apply_K_elementwise(wk, v)
    x = np.zeros(wk.ndof)
    nb = [len(c) - 1 for c in wk.cuts]
    for sx in (2, 3):
        sub, lo = _sub_block_2d(wk, sx + nb[0] * 3)
        Kff, _ = fe.free_system(sub)
        snn = [n + 1 for n in sub.nel]
        dofs = np.flatnonzero(~fe.dirichlet_dof_mask(sub))
        ln, comp = dofs // 2, dofs % 2
        gdof = 2 * ((lo[0] + ln % snn[0]) + nn[0] * (lo[1] + ln // snn[0])) + comp
        x[gdof] = spla.spsolve(Kff.tocsc(), y[gdof])
    Sv = fe.apply_K_elementwise(wk, v - x)
    g = np.flatnonzero(dd.classify(wk) == dd.GAMMA)
    gd = (2 * g[:, None] + np.arange(2)).reshape(-1)
    ref = Sv[gd]
    for mode in (0, 1):
        prob.set_s_apply(mode)
        out = to_np(prob.apply_S(to_cuda(v[gd])))
        err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
        print(f"2D 512x256 S v on an edge, {'explicit S_i' if mode else 'interior factors'}: "
              f"rel err {err:.2e}")
        assert err <= 1e-12
    prob.close()
