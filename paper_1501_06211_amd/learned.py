"""The correction network along a sequence of element moduli.

A topology-optimisation run solves K(E_k) u_k = f for a slowly changing
sequence E_1, E_2, ...  Warm-starting step k from u_{k-1} leaves the
residual r_k = f - K(E_k) u_{k-1}, and the exact correction it calls for is
e_k = u_k - u_{k-1}.  The pairs (E_k, r_k, e_k) from the first solves train
the network (the library's own forward, backward and Adam kernels); later
solves add its proposal to the warm start through ``learned_guess``.  Every
step runs in the library; this module only sequences the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import edd


def flatten_params(params, device="cuda"):
    """[(W (taps, c_in, c_out), b (c_out,)), ...] -> flat FP32 device tensor in
    the library's parameter layout."""
    parts = []
    for W, b in params:
        parts.append(np.asarray(W, dtype=np.float64).reshape(-1))
        parts.append(np.asarray(b, dtype=np.float64).reshape(-1))
    return torch.tensor(np.concatenate(parts), dtype=torch.float32, device=device)


def unflatten_params(flat, dim, width=32):
    """Inverse of flatten_params (host float64 arrays)."""
    v = flat.detach().double().cpu().numpy() if torch.is_tensor(flat) else np.asarray(flat)
    ntap = 3 ** dim
    chans = [1 + dim, width, width, width, dim]
    out, o = [], 0
    for ci, co in zip(chans[:-1], chans[1:]):
        W = v[o:o + ntap * ci * co].reshape(ntap, ci, co)
        o += ntap * ci * co
        b = v[o:o + co]
        o += co
        out.append((W, b))
    assert o == v.size
    return out


def warm_start_solves(prob, f, moduli, learned=False, keep_pairs=True, log=None, **opts):
    """Solve the sequence, each step from the previous solution.

    Returns (records, u_last): a list of dicts with the solve statistics and,
    when keep_pairs, the training pair (E, r, e) on the device (formed by
    edd_cnn_training_pair), and the solution of the last step."""
    u_prev = torch.zeros_like(f)
    out = []
    for k, E in enumerate(moduli):
        prob.set_element_moduli(E)
        u, st = prob.solve(f, u_prev.clone(), use_initial_guess=1,
                           learned_guess=1 if learned else 0, **opts)
        rec = {"stats": st}
        if log is not None:
            log(f"solve {k}: {st['iterations']} iterations, {st['t_total_ms']:.0f} ms")
        if keep_pairs:
            r, e = prob.cnn_training_pair(f, u_prev, u)
            rec.update(E=E.clone(), r=r, e=e)
        out.append(rec)
        u_prev = u
    return out, u_prev


def train(prob, pairs, epochs=20, lr=1e-3, seed=0, log=None):
    """Adam over the pairs, shuffled each epoch.  Returns the mean loss of
    every epoch (before each step's update)."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        losses = []
        for i in rng.permutation(len(pairs)):
            pr = pairs[i]
            losses.append(prob.cnn_train_step(pr["r"], pr["e"], lr=lr, E=pr["E"]))
        hist.append(float(np.mean(losses)))
        if log is not None:
            log(f"epoch {ep}: mean loss {hist[-1]:.4f}")
    return hist
