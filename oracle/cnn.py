"""Reference forward/backward of the small correction network.

TEST INFRASTRUCTURE ONLY (see the package header).

The network is an addition to the paper's method: it proposes a
correction of the displacement from the element moduli and a residual, and
the solver uses it only as a safeguarded initial guess (a line search in the
interface energy norm), so the method and its result are unchanged.

Definition (plain FP64, slow, written for checking by eye):

* Arrays live on the node grid, channel last: shape (ny+1, nx+1, C) in 2D
  and (nz+1, ny+1, nx+1, C) in 3D, so flattening the grid axes gives node
  ids with x fastest, the layout of the nodal vectors u[dim*node + c].
* A layer is a same-size cross-correlation with 3^D taps and dilation s:
      out[n, o] = b[o] + sum_{t, i} W[t, i, o] * in[n + s*(t - 1), i]
  with zero padding outside the grid; tap t runs over {0,1,2}^D in C order
  (the last grid axis, x, fastest).
* Four layers, dilations (1, 2, 4, 1), ReLU after the first three.
* Inputs (feature channels): a nodal stiffness indicator (the mean over the
  elements touching the node of clip(1 + log10(E_e)/3, 0, 1)) and the
  residual divided by its root mean square over the free dofs.
* Output: dim channels, zero at Dirichlet nodes.
* Loss: relative squared L2 error sum (y - t)^2 / sum t^2 against the target
  correction divided by its own root mean square.
* Adam with bias correction updates FP32 master weights; the forward pass
  uses the weights rounded to FP16 (an input here).

Pinned by tests/test_oracle_cnn.py: central finite differences of every
gradient, a delta-input test of the tap orientation, an identity network, a
library cross-check against torch's CPU FP64 convolution, and the closed
form of Adam's first step.
"""
from __future__ import annotations

import itertools

import numpy as np

DILATIONS = (1, 2, 4, 1)


def grid_shape(prob):
    """Node-grid shape in array order ([z,] y, x)."""
    return tuple(reversed(prob.nnodes_axis))


def taps(dim):
    return list(itertools.product(range(3), repeat=dim))


def shift(x, off):
    """shifted[n] = x[n + off] inside the grid, 0 outside (grid axes first)."""
    out = np.zeros_like(x)
    src, dst = [], []
    for a, o in enumerate(off):
        n = x.shape[a]
        if o >= 0:
            src.append(slice(o, n))
            dst.append(slice(0, n - o))
        else:
            src.append(slice(0, n + o))
            dst.append(slice(-o, n))
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv(x, W, b, dil):
    """One layer's cross-correlation.  W has shape (3^D, Cin, Cout)."""
    dim = x.ndim - 1
    out = np.zeros(x.shape[:-1] + (W.shape[2],))
    for k, t in enumerate(taps(dim)):
        off = [(ti - 1) * dil for ti in t]
        out += shift(x, off) @ W[k]
    return out + b


def conv_backward(x, W, gout, dil):
    """Gradients of sum(gout * conv(x, W, b, dil)) w.r.t. x, W and b."""
    dim = x.ndim - 1
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for k, t in enumerate(taps(dim)):
        off = [(ti - 1) * dil for ti in t]
        xs = shift(x, off)
        gW[k] = xs.reshape(-1, x.shape[-1]).T @ gout.reshape(-1, gout.shape[-1])
        # out[n] picks x[n + off]: x[m] feeds out[m - off]
        gx += shift(gout, [-o for o in off]) @ W[k].T
    gb = gout.reshape(-1, gout.shape[-1]).sum(axis=0)
    return gx, gW, gb


def forward(params, X):
    """params: list of (W, b) for the four layers.  Returns the output and
    the list of layer inputs (the activations the backward pass needs)."""
    acts = [X]
    h = X
    for layer, ((W, b), dil) in enumerate(zip(params, DILATIONS)):
        h = conv(h, W, b, dil)
        if layer < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def backward(params, acts, gy):
    """Gradients of sum(gy * forward(params, X)) for every (W, b)."""
    grads = [None] * len(params)
    g = gy
    for layer in reversed(range(len(params))):
        W, b = params[layer]
        if layer < len(params) - 1:
            g = g * (acts[layer + 1] > 0.0)
        gx, gW, gb = conv_backward(acts[layer], W, g, DILATIONS[layer])
        grads[layer] = (gW, gb)
        g = gx
    return grads, g


def node_mask(prob):
    """1 at free nodes, 0 at Dirichlet nodes, on the node grid."""
    from . import fe
    m = (~fe.dirichlet_node_mask(prob)).astype(np.float64)
    return m.reshape(grid_shape(prob))


def stiffness_indicator(prob, E=None):
    """Nodal mean over adjacent elements of clip(1 + log10(E)/3, 0, 1)."""
    from . import fe
    E = prob.E if E is None else E
    s = np.clip(1.0 + np.log10(E) / 3.0, 0.0, 1.0)
    en = fe.element_nodes(prob)
    acc = np.zeros(prob.n_nodes)
    cnt = np.zeros(prob.n_nodes)
    for j in range(en.shape[1]):
        np.add.at(acc, en[:, j], s)
        np.add.at(cnt, en[:, j], 1.0)
    return (acc / cnt).reshape(grid_shape(prob))


def rms_free(prob, v):
    from . import fe
    free = ~fe.dirichlet_dof_mask(prob)
    return float(np.sqrt(np.mean(v[free] ** 2)))


def features(prob, r, E=None):
    """Input channels: stiffness indicator, residual / rms(residual)."""
    d = prob.dim
    gs = grid_shape(prob)
    s = rms_free(prob, r)
    rr = (r / s if s > 0 else r).reshape(gs + (d,))
    return np.concatenate([stiffness_indicator(prob, E)[..., None], rr], axis=-1)


def target(prob, e):
    d = prob.dim
    s = rms_free(prob, e)
    return (e / s if s > 0 else e).reshape(grid_shape(prob) + (d,))


def predict(params, prob, r, E=None):
    """Network output as a full-length nodal vector (Dirichlet dofs zero)."""
    y, _ = forward(params, features(prob, r, E))
    y = y * node_mask(prob)[..., None]
    return y.reshape(-1)


def loss_and_grads(params, X, T, mask):
    """Relative squared L2 loss of the masked output against T and its
    gradients."""
    y, acts = forward(params, X)
    m = mask[..., None]
    diff = (y - T) * m
    den = float(np.sum((T * m) ** 2))
    loss = float(np.sum(diff ** 2)) / den
    gy = 2.0 * diff * m / den
    grads, _ = backward(params, acts, gy)
    return loss, grads


def round_fp16(params):
    return [(W.astype(np.float16).astype(np.float64), b.astype(np.float16).astype(np.float64))
            for W, b in params]


def adam_step(master, grads, state, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1) on the list of (W, b) master arrays.
    state is a list of dicts with first and second moments, updated in place."""
    out = []
    for (W, b), (gW, gb), st in zip(master, grads, state):
        new = []
        for name, p, g in (("W", W, gW), ("b", b, gb)):
            m = st.setdefault("m" + name, np.zeros_like(p))
            v = st.setdefault("v" + name, np.zeros_like(p))
            m[...] = beta1 * m + (1.0 - beta1) * g
            v[...] = beta2 * v + (1.0 - beta2) * g * g
            mh = m / (1.0 - beta1 ** t)
            vh = v / (1.0 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append((new[0], new[1]))
    return out
