"""The correction network's HIP kernels against the FP64 oracle (same
FP16-rounded weights), called through the C ABI; and its use as a
line-searched initial guess inside the solve.  GPU arithmetic is FP32 with
FP16 weights; the errors against FP64 are printed and bounded."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle import cnn, fe

from gpu_util import make_problem, require_gpu, to_cuda, to_np

pytestmark = pytest.mark.gpu


def _case(dim):
    rng = np.random.default_rng(40 + dim)
    if dim == 2:
        p = w.cantilever2d(37, 21, cuts=(np.array([0, 9, 25, 37]), np.array([0, 10, 21])))
    else:
        p = w.cantilever3d(13, 9, 7, cuts=(np.array([0, 6, 13]), np.array([0, 4, 9]),
                                           np.array([0, 3, 7])))
    p.E = 10.0 ** rng.uniform(-3, 0, p.n_el)
    free = ~fe.dirichlet_dof_mask(p)
    r = rng.standard_normal(p.ndof) * free
    e = rng.standard_normal(p.ndof) * free
    params = w.cnn_initial_weights(dim, 1 + dim, 32, dim, seed=7 + dim)
    params = [(W, rng.standard_normal(b.shape) * 0.05) for W, b in params]
    return p, r, e, params


def _gpu(p, params):
    from paper_1501_06211_amd import learned
    prob = make_problem(p)
    n = prob.cnn_setup(32)
    flat = learned.flatten_params(params)
    assert flat.numel() == n
    prob.cnn_set_params(flat)
    return prob


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dim", [2, 3])
def test_cnn_predict_parity(dim):
    require_gpu()
    p, r, e, params = _case(dim)
    prob = _gpu(p, params)
    d = to_np(prob.cnn_predict(to_cuda(r)))
    ref = cnn.predict(cnn.round_fp16(params), p, r)
    err = _rel(d, ref)
    print(f"{dim}D forward: relative error vs FP64 oracle {err:.2e}")
    assert err < 1e-4
    # explicit moduli give the same result as the factored ones
    d2 = to_np(prob.cnn_predict(to_cuda(r), E=to_cuda(p.E)))
    assert np.array_equal(d, d2)
    prob.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_cnn_loss_and_gradient_parity(dim):
    require_gpu()
    from paper_1501_06211_amd import learned
    p, r, e, params = _case(dim)
    prob = _gpu(p, params)
    loss, g = prob.cnn_loss_grad(to_cuda(r), to_cuda(e))
    X = cnn.features(p, r)
    T = cnn.target(p, e)
    lref, gref = cnn.loss_and_grads(cnn.round_fp16(params), X, T, cnn.node_mask(p))
    gg = learned.unflatten_params(g, dim)
    lerr = abs(loss - lref) / lref
    errs = []
    for (gW, gb), (rW, rb) in zip(gg, gref):
        errs.append(_rel(gW, rW))
        errs.append(_rel(gb, rb))
    print(f"{dim}D loss {loss:.6f} (oracle {lref:.6f}, rel err {lerr:.1e}); "
          f"gradient rel errors per tensor max {max(errs):.2e}")
    assert lerr < 1e-5
    assert max(errs) < 1e-3
    # deterministic
    loss2, g2 = prob.cnn_loss_grad(to_cuda(r), to_cuda(e))
    assert loss2 == loss and torch.equal(g, g2)
    prob.close()


def test_cnn_adam_step():
    require_gpu()
    from paper_1501_06211_amd import learned
    p, r, e, params = _case(2)
    prob = _gpu(p, params)
    master = learned.unflatten_params(learned.flatten_params(params), 2)
    _, g = prob.cnn_loss_grad(to_cuda(r), to_cuda(e))
    gg = learned.unflatten_params(g, 2)
    prob.cnn_train_step(to_cuda(r), to_cuda(e), lr=1e-3)
    new = learned.unflatten_params(prob.cnn_get_params(), 2)
    ref = cnn.adam_step(master, gg, [{} for _ in master], t=1, lr=1e-3)
    worst = max(float(np.abs(a - b).max()) for (a, _), (b, _) in zip(new, ref))
    print(f"Adam step: max abs difference {worst:.2e} (lr 1e-3)")
    assert worst < 2e-7
    prob.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_learned_guess_keeps_the_solution(dim):
    """The proposal only moves the initial guess: the solution still matches
    the oracle's direct solve."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p, r, e, params = _case(dim)
    prob = _gpu(p, params)
    uref = fe.solve_direct(p)
    u, st = prob.solve(to_cuda(p.f), tol=1e-12, maxit=4000, learned_guess=1)
    un = to_np(u)
    err = _rel(un, uref)
    cerr = abs(st["compliance"] - fe.compliance(p.f, uref)) / abs(fe.compliance(p.f, uref))
    print(f"{dim}D learned guess: alpha={st['learned_alpha']:.3e} its={st['iterations']} "
          f"u_err={err:.2e} c_err={cerr:.2e}")
    assert st["flags"] & edd.FLAG_LEARNED_REJECTED == 0
    assert np.isfinite(st["learned_alpha"])
    assert err <= 1e-8 and cerr <= 1e-10
    prob.close()


def test_trained_network_gain_on_a_sequence():
    """Train on the warm-start corrections of a short density sequence
    (2D 128x64, 32 subdomains), then measure on held-out steps how much the
    line-searched proposal lowers the interface energy error of the warm
    start, trained against untrained (initial) weights."""
    require_gpu()
    from paper_1501_06211_amd import edd, learned
    ntrain, ntest, dim = 16, 8, 2
    seq = [torch.tensor(E, device="cuda")
           for E in w.to_sequence_2d(ntrain + ntest, 128, 64, ell=6.0)]
    p = w.cantilever2d(128, 64)
    prob = edd.Problem.from_workload(p)
    f = torch.tensor(p.f, device="cuda")
    prob.cnn_setup(32)
    init = learned.flatten_params(w.cnn_initial_weights(dim, 1 + dim, 32, dim, seed=1))
    tr, u_start = learned.warm_start_solves(prob, f, seq[:ntrain])
    gam = torch.tensor(prob.gamma_nodes(), device="cuda", dtype=torch.long)
    gidx = (gam[:, None] * dim + torch.arange(dim, device="cuda")).reshape(-1)

    def held_out(params):
        prob.cnn_set_params(params)
        u_prev, ratios, its = u_start.clone(), [], []
        for E in seq[ntrain:]:
            prob.set_element_moduli(E)
            r = f - prob.apply_K(u_prev)
            uw, sw = prob.solve(f, u_prev.clone(), use_initial_guess=1)
            ul, sl = prob.solve(f, u_prev.clone(), use_initial_guess=1, learned_guess=1)
            d = prob.cnn_predict(r)
            e0 = (uw - u_prev)[gidx].contiguous()
            e1 = e0 - sl["learned_alpha"] * d[gidx].contiguous()
            ratios.append(float(e1 @ prob.apply_S(e1)) / float(e0 @ prob.apply_S(e0)))
            its.append((sw["iterations"], sl["iterations"]))
            assert abs(sl["compliance"] - sw["compliance"]) <= 1e-8 * abs(sw["compliance"])
            u_prev = uw
        return np.array(ratios), its

    r0, its0 = held_out(init)
    hist = learned.train(prob, tr, epochs=40, lr=1e-3)
    r1, its1 = held_out(prob.cnn_get_params())
    print(f"training loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    print(f"energy-error ratio after the proposal: untrained {np.round(r0, 3).tolist()} "
          f"mean {r0.mean():.3f}; trained {np.round(r1, 3).tolist()} mean {r1.mean():.3f}")
    print(f"iterations (warm start, warm start + proposal): trained {its1}")
    assert (r1 <= 1.0 + 1e-9).all() and (r0 <= 1.0 + 1e-9).all()
    assert hist[-1] < hist[0]
    assert r1.mean() < r0.mean()
    prob.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_network_steps_inside_the_flexible_iteration(dim):
    """learned_correction = K: every K-th interface step takes the network's
    proposal for the interface residual (extended by zero) as its direction.
    The flexible iteration's exact line search keeps such steps safe: with
    random weights the solution still matches the direct solve; with all-zero
    weights every network step is dropped (flagged) and the other steps are
    those of the plain iteration."""
    require_gpu()
    from paper_1501_06211_amd import edd
    p, r, e, params = _case(dim)
    prob = _gpu(p, params)
    uref = fe.solve_direct(p)
    f = to_cuda(p.f)
    u0, s0 = prob.solve(f, tol=1e-11, maxit=4000)
    u1, s1 = prob.solve(f, tol=1e-11, maxit=4000, learned_correction=5)
    err = _rel(to_np(u1), uref)
    print(f"{dim}D network steps every 5: its {s1['iterations']} (plain {s0['iterations']}), "
          f"u_err {err:.1e}, flags {s1['flags']}")
    assert err <= 1e-8
    prob.cnn_set_params(torch.zeros(prob.cnn_setup(32), dtype=torch.float32, device="cuda"))
    u2, s2 = prob.solve(f, tol=1e-11, maxit=4000, learned_correction=5)
    assert s2["flags"] & edd.FLAG_LEARNED_REJECTED
    assert _rel(to_np(u2), uref) <= 1e-8
    prob.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_matrix_core_forward(dim):
    """edd_cnn_matrix_cores: the hidden 32 -> 32 layers as implicit GEMMs on
    the FP16 matrix cores (FP16 weights and activations, FP32 accumulation).
    Against the FP64 oracle with the same FP16 weights the relative error is
    that of FP16 activations (bound 1e-2, printed); training through it still
    lowers the loss."""
    require_gpu()
    p, r, e, params = _case(dim)
    prob = _gpu(p, params)
    d32 = to_np(prob.cnn_predict(to_cuda(r)))
    prob.cnn_matrix_cores(True)
    d16 = to_np(prob.cnn_predict(to_cuda(r)))
    ref = cnn.predict(cnn.round_fp16(params), p, r)
    err, err32 = _rel(d16, ref), _rel(d16, d32)
    print(f"{dim}D matrix-core forward: relative error vs FP64 oracle {err:.2e}, "
          f"vs the FP32 path {err32:.2e}")
    assert err < 1e-2
    assert np.array_equal(d16, to_np(prob.cnn_predict(to_cuda(r))))  # deterministic
    losses = [prob.cnn_train_step(to_cuda(r), to_cuda(e), lr=1e-3) for _ in range(20)]
    assert losses[-1] < losses[0]
    prob.close()
