"""Pins for oracle/cnn.py: finite differences, tap orientation, identity
network, torch's CPU FP64 convolution, Adam's first step, features."""
import numpy as np
import pytest

import workloads as w
from oracle import cnn, fe


def _tiny(dim, width=3, seed=0):
    if dim == 2:
        p = w.cantilever2d(6, 5, block=3)
    else:
        p = w.cantilever3d(4, 3, 3, cuts=(np.array([0, 2, 4]), np.array([0, 3]),
                                          np.array([0, 3])))
    rng = np.random.default_rng(seed)
    p.E = 10.0 ** rng.uniform(-3, 0, p.n_el)
    params = w.cnn_initial_weights(dim, 1 + dim, width, dim, seed=seed + 1)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    r = rng.standard_normal(p.ndof) * (~fe.dirichlet_dof_mask(p))
    e = rng.standard_normal(p.ndof) * (~fe.dirichlet_dof_mask(p))
    X = cnn.features(p, r)
    T = cnn.target(p, e)
    return p, params, X, T


@pytest.mark.parametrize("dim", [2, 3])
def test_gradients_match_central_differences(dim):
    p, params, X, T = _tiny(dim)
    mask = cnn.node_mask(p)
    loss, grads = cnn.loss_and_grads(params, X, T, mask)
    rng = np.random.default_rng(5)
    h = 1e-4
    worst = 0.0

    def at(arr, idx, v):
        arr[idx] = v
        return cnn.loss_and_grads(params, X, T, mask)[0]

    for layer in range(4):
        for which in (0, 1):
            arr = params[layer][which]
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                # fourth-order central difference
                fd = (-at(arr, idx, old + 2 * h) + 8 * at(arr, idx, old + h)
                      - 8 * at(arr, idx, old - h) + at(arr, idx, old - 2 * h)) / (12 * h)
                arr[idx] = old
                an = grads[layer][which][idx]
                worst = max(worst, abs(fd - an) / max(abs(fd), abs(an), 1e-3))
    print(f"dim {dim}: worst relative gradient error {worst:.2e}")
    assert worst < 1e-7, worst


def test_tap_orientation_with_a_delta():
    # out[n] = sum_t W[t] x[n + s (t - 1)]: a delta at m shows W[t] at m - s(t-1)
    rng = np.random.default_rng(1)
    x = np.zeros((11, 13, 1))
    m = (5, 6)
    x[m + (0,)] = 1.0
    W = rng.standard_normal((9, 1, 1))
    for dil in (1, 2, 4):
        out = cnn.conv(x, W, np.zeros(1), dil)
        for k, t in enumerate(cnn.taps(2)):
            n = (m[0] - dil * (t[0] - 1), m[1] - dil * (t[1] - 1))
            assert out[n + (0,)] == W[k, 0, 0]
        assert np.count_nonzero(out) == 9


@pytest.mark.parametrize("dim", [2, 3])
def test_identity_network(dim):
    shape = (6, 7) if dim == 2 else (4, 5, 6)
    cin, width = 1 + dim, 5
    rng = np.random.default_rng(2)
    X = rng.uniform(0.1, 1.0, shape + (cin,))
    centre = (3 ** dim) // 2
    params = []
    for a, b in zip([cin, width, width, width], [width, width, width, dim]):
        W = np.zeros((3 ** dim, a, b))
        for c in range(min(a, b)):
            W[centre, c, c] = 1.0
        params.append((W, np.zeros(b)))
    y, _ = cnn.forward(params, X)
    assert np.array_equal(y, X[..., :dim])


@pytest.mark.parametrize("dim", [2, 3])
def test_matches_torch_cpu_convolution(dim):
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    p, params, X, T = _tiny(dim, width=4)
    mask = cnn.node_mask(p)
    y, _ = cnn.forward(params, X)
    loss, grads = cnn.loss_and_grads(params, X, T, mask)
    conv = F.conv2d if dim == 2 else F.conv3d
    tw = []
    for W, b in params:
        k = torch.tensor(W.reshape((3,) * dim + W.shape[1:]), dtype=torch.float64)
        # (taps..., ci, co) -> (co, ci, taps...)
        k = k.permute(*([dim + 1, dim] + list(range(dim)))).contiguous().requires_grad_()
        tw.append((k, torch.tensor(b, dtype=torch.float64, requires_grad=True)))
    h = torch.tensor(X, dtype=torch.float64).permute(*([dim] + list(range(dim))))[None]
    for layer, ((k, b), dil) in enumerate(zip(tw, cnn.DILATIONS)):
        h = conv(h, k, b, padding=dil, dilation=dil)
        if layer < 3:
            h = torch.relu(h)
    ty = h[0].permute(*(list(range(1, dim + 1)) + [0]))
    assert np.abs(ty.detach().numpy() - y).max() < 1e-12 * max(1.0, np.abs(y).max())
    m = torch.tensor(mask[..., None])
    tt = torch.tensor(T)
    tl = (((ty - tt) * m) ** 2).sum() / ((tt * m) ** 2).sum()
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12
    for (k, b), (gW, gb) in zip(tw, grads):
        gk = k.grad.permute(*(list(range(2, dim + 2)) + [1, 0])).reshape(gW.shape).numpy()
        assert np.abs(gk - gW).max() < 1e-12 * max(1.0, np.abs(gW).max())
        assert np.abs(b.grad.numpy() - gb).max() < 1e-12 * max(1.0, np.abs(gb).max())


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    master = [(rng.standard_normal((9, 2, 3)), rng.standard_normal(3))]
    grads = [(rng.standard_normal((9, 2, 3)), rng.standard_normal(3))]
    state = [{}]
    out = cnn.adam_step(master, grads, state, t=1, lr=1e-2, eps=1e-8)
    for p_new, p_old, g in zip(out[0], master[0], grads[0]):
        assert np.allclose(p_new, p_old - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_features():
    p = w.cantilever2d(8, 4, block=4)
    p.E = np.ones(p.n_el)
    r = np.random.default_rng(4).standard_normal(p.ndof) * (~fe.dirichlet_dof_mask(p))
    X = cnn.features(p, r)
    assert np.all(X[..., 0] == 1.0)
    free = ~fe.dirichlet_dof_mask(p)
    assert np.sqrt(np.mean(X[..., 1:].reshape(-1)[free] ** 2)) == pytest.approx(1.0, rel=1e-14)
    p.E = np.full(p.n_el, 1e-3)
    assert np.all(cnn.features(p, r)[..., 0] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_stiffness_indicator_brute_force(dim):
    """Per node, the mean over the elements that touch it of
    clip(1 + log10(E_e)/3, 0, 1), by explicit loops over the node grid and
    the (up to 2^dim) neighbouring element positions, with non-uniform E
    spanning the clip range."""
    if dim == 2:
        p = w.cantilever2d(5, 3, block=5)
    else:
        p = w.cantilever3d(4, 3, 2, cuts=([0, 4], [0, 3], [0, 2]))
    rng = np.random.default_rng(7)
    E = 10.0 ** rng.uniform(-4.0, 0.5, p.n_el)  # below, inside and above the clip range
    got = cnn.stiffness_indicator(p, E)
    nel = list(p.nel) + [1] * (3 - dim)
    nn = [n + 1 for n in p.nel] + [1] * (3 - dim)
    want = np.zeros(nn[::-1])
    for k in range(nn[2]):
        for j in range(nn[1]):
            for i in range(nn[0]):
                vals = []
                for ek in ((k - 1, k) if dim == 3 else (0,)):
                    for ej in (j - 1, j):
                        for ei in (i - 1, i):
                            if 0 <= ei < nel[0] and 0 <= ej < nel[1] and 0 <= ek < nel[2]:
                                e = ei + nel[0] * (ej + nel[1] * ek)
                                vals.append(min(1.0, max(0.0, 1.0 + np.log10(E[e]) / 3.0)))
                want[k, j, i] = sum(vals) / len(vals)
    want = want.reshape(got.shape)
    assert np.allclose(got, want, rtol=0, atol=1e-15)
    assert got.min() < 0.5 < got.max()
