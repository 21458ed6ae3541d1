"""Pins for oracle/reference.py (the Schur route with long-double
refinement) and for the stored full-size reference it wrote.

* On small meshes the refined Schur solution equals the sparse direct solve
  of the whole free system (eq. (NumberFour)) to the rounding level, and the
  block-by-block Schur operator equals the dense S of ``dd.schur_dense``.
* The stored 1.6M-dof reference was written by the committed scripts (their
  hashes are recorded), and the oracle's own element-by-element K apply
  confirms its residual and compliance."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as w
from oracle import dd, fe, reference

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _small3d():
    return w.cantilever3d_simp(16, 8, 8, ([0, 6, 16], [0, 4, 8], [0, 3, 8]), seed=9, ell=3.0)


def test_block_schur_operator_equals_dense_schur():
    p = _small3d()
    op = reference.BlockSchurOperator(p, workers=2)
    try:
        S = dd.schur_dense(p)
        V = np.random.default_rng(1).standard_normal((op.n, 3))
        SV = np.column_stack([op.apply(V[:, j]) for j in range(3)])
        assert np.linalg.norm(SV - S @ V) <= 1e-12 * np.linalg.norm(S @ V)
    finally:
        op.close()


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_refined_solve_equals_direct_solve(case):
    if case == "2d":
        p = w.cantilever2d(48, 24, E=w.simp_moduli(np.random.default_rng(3).uniform(0, 1, 48 * 24)))
    else:
        p = _small3d()
    u, rec = reference.refined_solve(p, tol=1e-14, workers=2)
    ud = fe.solve_direct(p)
    err = np.linalg.norm(np.asarray(u, dtype=np.float64) - ud) / np.linalg.norm(ud)
    assert rec["rel_residual"] <= 1e-14
    assert err <= 1e-12
    # each refinement round's correction shrinks
    corr = [r["correction_rel"] for r in rec["rounds"] if "correction_rel" in r]
    assert all(b < 1e-6 * a for a, b in zip(corr, corr[1:]))


def _sha(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def test_stored_reference_provenance_and_residual():
    base = os.path.join(GOLDEN, "cantilever3d_simp_128x64x64_u_ref")
    with open(base + ".json") as fh:
        meta = json.load(fh)
    assert meta["script_sha256"] == _sha(os.path.join(GOLDEN, "make_reference.py"))
    assert meta["oracle_reference_sha256"] == _sha(os.path.join(ROOT, "oracle", "reference.py"))
    wk = w.cantilever3d_simp_128x64x64()
    u = np.load(base + ".npy")
    assert u.shape == (wk.ndof,)
    assert np.all(u[fe.dirichlet_dof_mask(wk)] == 0.0)
    assert meta["rel_residual_long_double"] <= 1e-13
    # the oracle's matrix-free apply confirms the residual of the stored FP64 u
    res = fe.residual_norm(wk, u)
    assert res <= 1e-11
    assert abs(res - meta["rel_residual_fp64_of_stored_u"]) <= 1e-2 * res
    c = fe.compliance(wk.f, u)
    assert abs(c - meta["compliance"]) <= 1e-13 * abs(c)
