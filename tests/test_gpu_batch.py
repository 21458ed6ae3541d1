"""Substitution variants chosen by the autotuner, and many independent
problems solved concurrently through edd_solve_batch, against the oracle and
against one-at-a-time solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as w
from oracle import dd, fe

from gpu_util import interior_perm, make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _wide():
    rng = np.random.default_rng(11)
    p = w.cantilever3d(16, 12, 12, cuts=(np.array([0, 7, 16]), np.array([0, 12]),
                                         np.array([0, 5, 12])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    return p


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
def test_every_substitution_variant_matches_the_oracle(variant):
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _wide()
    prob = make_problem(p, dissect=0)
    prob.set_solve_variants(variant, variant)
    perm = interior_perm(p, prob)
    KII, *_ = dd.blocks(p)
    b = np.random.default_rng(2).standard_normal(prob.n_interior_dofs)
    xr = spla.spsolve(KII.tocsc(), b[perm])
    x = to_np(prob.solve_interior(to_cuda(b)))
    x32 = to_np(prob.solve_interior(to_cuda(b), precision=edd.F32))
    e64 = np.linalg.norm(x[perm] - xr) / np.linalg.norm(xr)
    e32 = np.linalg.norm(x32[perm] - xr) / np.linalg.norm(xr)
    print(f"variant {variant}: FP64 {e64:.2e}, FP32 factors {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5
    prob.close()


@pytest.mark.parametrize("variant", [4, 5, 6, 7])
def test_dissected_interiors_match_the_oracle(variant):
    """Every interior split into two band halves and a separator plane (one
    level of nested dissection): the same K_II^{-1} as the oracle."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _wide()
    prob = make_problem(p, dissect=1)
    prob.set_solve_variants(variant, variant)
    perm = interior_perm(p, prob)
    KII, *_ = dd.blocks(p)
    b = np.random.default_rng(3).standard_normal(prob.n_interior_dofs)
    xr = spla.spsolve(KII.tocsc(), b[perm])
    x = to_np(prob.solve_interior(to_cuda(b)))
    x32 = to_np(prob.solve_interior(to_cuda(b), precision=edd.F32))
    xi = to_cuda(b)
    prob.solve_interior(xi, out=xi)  # in place
    e64 = np.linalg.norm(x[perm] - xr) / np.linalg.norm(xr)
    e32 = np.linalg.norm(x32[perm] - xr) / np.linalg.norm(xr)
    print(f"dissected, variant {variant}: FP64 {e64:.2e}, FP32 factors {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5
    assert np.array_equal(to_np(xi), x)
    with pytest.raises(edd.EddError):
        prob.set_solve_variants(1, 1)  # one-kernel variants have no sweep phases
    prob.close()


def _wider():
    """Half bandwidths above 448 (most of the 960 off-diagonal threads busy)."""
    rng = np.random.default_rng(12)
    p = w.cantilever3d(28, 14, 14, cuts=(np.array([0, 14, 28]), np.array([0, 14]),
                                         np.array([0, 14])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    return p


@pytest.mark.parametrize("variant,dissect", [(5, 0), (6, 0), (7, 0), (5, 1), (6, 1), (7, 1)])
def test_wide_variants_at_half_bandwidths_past_448(variant, dissect):
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _wider()
    prob = make_problem(p, dissect=dissect)
    assert prob.info["max_band"] > 448
    prob.set_solve_variants(variant, variant)
    perm = interior_perm(p, prob)
    KII, *_ = dd.blocks(p)
    b = np.random.default_rng(4).standard_normal(prob.n_interior_dofs)
    xr = spla.spsolve(KII.tocsc(), b[perm])
    x = to_np(prob.solve_interior(to_cuda(b)))
    x32 = to_np(prob.solve_interior(to_cuda(b), precision=edd.F32))
    e64 = np.linalg.norm(x[perm] - xr) / np.linalg.norm(xr)
    e32 = np.linalg.norm(x32[perm] - xr) / np.linalg.norm(xr)
    print(f"kd {prob.info['max_band']}, dissect {dissect}, variant {variant}: "
          f"FP64 {e64:.2e}, FP32 factors {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5
    prob.close()


@pytest.mark.parametrize("ny,kd,dissect", [(12, 509, 0), (12, 509, 1), (11, 473, 0), (11, 473, 1)])
def test_factor_windows_either_side_of_the_matrix_core_switch(ny, kd, dissect):
    """Factor windows of 541 rows (32 + kd 509: the matrix-core Cholesky,
    with fewer row tiles than four per wavefront) and of 505 rows (kd 473:
    the last vector configuration); dissected separators are dense blocks
    factored by the same kernel.  The interior solves from those factors
    against a sparse direct solve."""
    require_gpu()
    from paper_1501_06211_amd import edd
    rng = np.random.default_rng(ny)
    p = w.cantilever3d(24, ny, ny, cuts=(np.array([0, 12, 24]), np.array([0, ny]),
                                         np.array([0, ny])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    prob = make_problem(p, dissect=dissect)
    assert prob.info["max_band"] == kd
    perm = interior_perm(p, prob)
    KII, *_ = dd.blocks(p)
    b = rng.standard_normal(prob.n_interior_dofs)
    xr = spla.spsolve(KII.tocsc(), b[perm])
    x = to_np(prob.solve_interior(to_cuda(b)))
    x32 = to_np(prob.solve_interior(to_cuda(b), precision=edd.F32))
    e64 = np.linalg.norm(x[perm] - xr) / np.linalg.norm(xr)
    e32 = np.linalg.norm(x32[perm] - xr) / np.linalg.norm(xr)
    print(f"kd {kd}, dissect {dissect}: FP64 {e64:.2e}, FP32 factors {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5
    prob.close()


def test_autotune_picks_valid_variants_and_caches():
    require_gpu()
    from paper_1501_06211_amd import edd
    p = _wide()
    p64 = make_problem(p, factor_precision=edd.F64)
    v64 = p64.autotune(force=True)
    assert 1 <= v64[0] <= 7 and v64[1] == 0  # no FP32 factors: nothing to tune
    assert all(0 <= x <= 2 for x in v64[2:])
    p64.close()
    prob = make_problem(p)
    v = prob.autotune()  # factor precisions are part of the cache key
    assert all(1 <= x <= 7 for x in v[:2]) and all(0 <= x <= 2 for x in v[2:])
    prob2 = make_problem(p)
    assert prob2.autotune() == v  # same shape class: cached
    u, st = prob2.solve(to_cuda(p.f), tol=1e-12, maxit=3000)
    uref = fe.solve_direct(p)
    assert np.linalg.norm(to_np(u) - uref) <= 1e-8 * np.linalg.norm(uref)
    prob.close()
    prob2.close()


def _batch_problems():
    # small members of the uneven batch: 2D and 3D, each with its own field
    probs = []
    for k, (nx, ny) in enumerate([(64, 32), (80, 40), (96, 48)]):
        p = w.cantilever2d(nx, ny, E=w.simp_moduli(np.random.default_rng(k).uniform(0, 1, nx * ny)))
        probs.append(p)
    for k, (nx, ny, nz) in enumerate([(16, 16, 16), (24, 16, 16), (32, 20, 20)]):
        E = w.simp_moduli(np.random.default_rng(10 + k).uniform(0, 1, nx * ny * nz))
        probs.append(w.cantilever3d(nx, ny, nz, cuts=(w.even_cuts(nx, 16), w.even_cuts(ny, 16),
                                                      w.even_cuts(nz, 16)), E=E))
    return probs


def test_batch_matches_single_solves_and_the_oracle():
    require_gpu()
    from paper_1501_06211_amd import edd
    ws = _batch_problems()
    streams = [torch.cuda.Stream() for _ in ws]
    probs = []
    for wk, s in zip(ws, streams):
        prob = edd.Problem.from_workload(wk, stream=s)
        prob.set_element_moduli(torch.tensor(wk.E, device="cuda"))
        prob.autotune()
        probs.append(prob)
    fs = [to_cuda(wk.f) for wk in ws]
    us = [torch.zeros_like(f) for f in fs]
    torch.cuda.synchronize()
    # the parity bars (1e-8 on u, 1e-10 on compliance) need the solve at the
    # tightest residual these high-contrast members reach
    rc, stats = edd.solve_batch(probs, fs, us, tol=1e-11, maxit=6000)
    torch.cuda.synchronize()
    assert rc in (edd.OK, edd.NOT_CONVERGED)
    for wk, prob, f, u, st in zip(ws, probs, fs, us, stats):
        u1, st1 = prob.solve(f, tol=1e-11, maxit=6000)
        torch.cuda.synchronize()
        assert torch.equal(u, u1), wk.name  # deterministic kernels, same launches
        assert st["iterations"] == st1["iterations"]
        assert st["rel_residual"] <= 1e-10
    # every member against the oracle's direct solve
    for wk, u, st in zip(ws, us, stats):
        uref = fe.solve_direct(wk)
        cref = fe.compliance(wk.f, uref)
        err = np.linalg.norm(to_np(u) - uref) / np.linalg.norm(uref)
        cerr = abs(st["compliance"] - cref) / abs(cref)
        print(f"  {wk.name}: its={st['iterations']} res={st['rel_residual']:.1e} "
              f"u_err={err:.1e} c_err={cerr:.1e}")
        assert err <= 1e-8 and cerr <= 1e-10, wk.name
    lat = [s["t_total_ms"] for s in stats]
    print(f"batch of {len(ws)}: iterations {[s['iterations'] for s in stats]}, "
          f"latency ms {np.round(lat, 1).tolist()}")
    for prob in probs:
        prob.close()


def test_autotune_cache_file(tmp_path):
    """Choices persist in the cache file, one line per (kernel family, shape
    class), and are read back from it without re-timing."""
    require_gpu()
    from paper_1501_06211_amd import edd
    path = str(tmp_path / "tune.txt")
    edd.set_autotune_cache(path)
    try:
        p = _wide()
        prob = make_problem(p)
        v = prob.autotune(force=True)
        lines = open(path).read().splitlines()
        fams = sorted(l.split()[0] for l in lines)
        assert fams == ["apply_K", "band_solve", "s_apply"]
        # edit the stored tile shapes; a reload must return the file's values
        other = [(x + 1) % 3 for x in v[2:]]
        edited = [(" ".join(l.split()[:2] + [str(x) for x in other])
                   if l.startswith("apply_K") else l) for l in lines]
        open(path, "w").write("\n".join(edited) + "\n")
        edd.set_autotune_cache(path)
        prob2 = make_problem(p)
        v2 = prob2.autotune()
        assert v2 == (v[0], v[1], *other)
        prob.close()
        prob2.close()
    finally:
        edd.set_autotune_cache(None)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_tile_shapes_are_bitwise_equal(dim):
    require_gpu()
    from paper_1501_06211_amd import edd
    rng = np.random.default_rng(8)
    if dim == 2:
        p = w.cantilever2d(45, 23, cuts=(np.array([0, 20, 45]), np.array([0, 11, 23])))
    else:
        p = w.cantilever3d(19, 11, 9, cuts=(np.array([0, 9, 19]), np.array([0, 11]),
                                            np.array([0, 4, 9])))
    p.E = 1e-3 + rng.uniform(0, 1, p.n_el) ** 3
    prob = make_problem(p)
    u = rng.standard_normal(p.ndof)
    ref = fe.apply_K_elementwise(p, u)
    ys = []
    for v in range(3):
        prob.set_apply_variant(v)
        ys.append(to_np(prob.apply_K(to_cuda(u))))
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    assert np.linalg.norm(ys[0] - ref) <= 1e-14 * np.linalg.norm(ref)
    prob.close()
