"""Seeded generators for cantilever-like elasticity workloads.

Conventions shared by every consumer:

* Structured grid of unit-size elements, ``nel = (nx, ny[, nz])``.
* Node ``(i, j[, k])`` has id ``i + (nx+1) * (j + (ny+1) * k)`` (x fastest).
* Element ``(ex, ey[, ez])`` has id ``ex + nx * (ey + ny * ez)``.
* Degree of freedom ``c`` of node ``n`` is ``dim * n + c`` (node-major,
  components interleaved).
* ``cuts[a]`` lists the element-index positions of the subdomain cuts along
  axis ``a``, including ``0`` and ``nel[a]``; uneven blocks are allowed.
* ``clamp`` is a bitmask of clamped faces: bit 0 is ``x = 0``, bit 1
  ``x = nx``, bits 2/3 the y faces and bits 4/5 the z faces.  Every dof of a
  node on a clamped face is fixed to zero.

The element moduli follow a SIMP-style map ``E_e = Emin + rho_e^3 (1 - Emin)``
with ``rho`` a smooth random field squashed to ``[0, 1]``.  The random field
is white noise filtered by a Gaussian of standard deviation ``ell`` elements,
computed with FFTs on a zero-padded grid (so it is not periodic), then
standardised and mapped through the normal CDF.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
from scipy.special import ndtr

CLAMP_X0 = 1


@dataclass
class Problem:
    name: str
    dim: int
    nel: tuple
    cuts: tuple
    nu: float
    clamp: int
    E: np.ndarray
    f: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnodes_axis(self):
        return tuple(n + 1 for n in self.nel)

    @property
    def n_nodes(self):
        return int(np.prod(self.nnodes_axis))

    @property
    def n_el(self):
        return int(np.prod(self.nel))

    @property
    def ndof(self):
        return self.dim * self.n_nodes

    @property
    def n_sub(self):
        return int(np.prod([len(c) - 1 for c in self.cuts]))

    def node_id(self, *ijk):
        nn = self.nnodes_axis
        if self.dim == 2:
            i, j = ijk
            return i + nn[0] * j
        i, j, k = ijk
        return i + nn[0] * (j + nn[1] * k)


def even_cuts(n, block):
    """Cut positions every ``block`` elements; a shorter last block if needed."""
    c = list(range(0, n, block))
    c.append(n)
    return np.asarray(c, dtype=np.int64)


def gaussian_random_field(shape, ell, seed):
    """Standardised Gaussian-filtered white noise on an element grid."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    pad = int(np.ceil(3.0 * ell))
    padded = np.pad(noise, [(pad, pad)] * len(shape))
    spec = np.fft.rfftn(padded)
    # transfer function of a unit-mass Gaussian of std ``ell`` (in elements)
    filt = np.ones(spec.shape)
    for ax, n in enumerate(padded.shape):
        if ax == len(shape) - 1:
            k = np.fft.rfftfreq(n)
        else:
            k = np.fft.fftfreq(n)
        g = np.exp(-2.0 * (np.pi * ell * k) ** 2)
        sh = [1] * len(shape)
        sh[ax] = g.size
        filt = filt * g.reshape(sh)
    smooth = np.fft.irfftn(spec * filt, s=padded.shape, axes=tuple(range(len(shape))))
    sl = tuple(slice(pad, pad + n) for n in shape)
    g = smooth[sl]
    g = (g - g.mean()) / g.std()
    return g


def simp_moduli(rho, emin=1e-3):
    return emin + rho ** 3 * (1.0 - emin)


def _field_to_elements(g):
    """Array indexed [ex, ey(, ez)] -> flat element order (x fastest)."""
    return np.ascontiguousarray(g.transpose()).reshape(-1)


def _point_load(dim, nn, node_ijk, comp, value=-1.0):
    f = np.zeros(dim * int(np.prod(nn)))
    if dim == 2:
        n = node_ijk[0] + nn[0] * node_ijk[1]
    else:
        n = node_ijk[0] + nn[0] * (node_ijk[1] + nn[1] * node_ijk[2])
    f[dim * n + comp] = value
    return f


def cantilever2d(nx, ny, block=16, nu=0.3, E=None, load_node=None, name=None,
                 cuts=None):
    """Clamped at x=0, unit downward point load at (nx, load_node_y)."""
    nn = (nx + 1, ny + 1)
    if E is None:
        E = np.ones(nx * ny)
    if load_node is None:
        load_node = (nx, ny // 2)
    f = _point_load(2, nn, load_node, 1, -1.0)
    if cuts is None:
        cuts = (even_cuts(nx, block), even_cuts(ny, block))
    return Problem(name or f"cantilever2d_{nx}x{ny}", 2, (nx, ny), cuts, nu,
                   CLAMP_X0, np.asarray(E, dtype=np.float64), f)


def line_load_3d(nx, ny, nz):
    """Unit total force in -z along the line x=nx, z=0 (trapezoid weights)."""
    nn = (nx + 1, ny + 1, nz + 1)
    f = np.zeros(3 * nn[0] * nn[1] * nn[2])
    for j in range(ny + 1):
        w = 1.0 / ny if 0 < j < ny else 0.5 / ny
        n = nx + nn[0] * j
        f[3 * n + 2] = -w
    return f


def cantilever3d(nx, ny, nz, cuts, nu=0.3, E=None, name=None, f=None):
    if E is None:
        E = np.ones(nx * ny * nz)
    if f is None:
        f = line_load_3d(nx, ny, nz)
    return Problem(name or f"cantilever3d_{nx}x{ny}x{nz}", 3, (nx, ny, nz),
                   tuple(np.asarray(c, dtype=np.int64) for c in cuts), nu,
                   CLAMP_X0, np.asarray(E, dtype=np.float64), f)


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def cantilever2d_uniform_64x32():
    """64x32 Q1, E=1, nu=0.3, 4x2 subdomains of 16x16, load at (64, 16)."""
    return cantilever2d(64, 32, name="cantilever2d_uniform_64x32")


def cantilever2d_simp_512x256(seed=2, ell=20.0):
    """512x256 Q1, 32x16 subdomains, SIMP moduli from a seeded field."""
    rho = ndtr(gaussian_random_field((512, 256), ell, seed))
    E = simp_moduli(_field_to_elements(rho))
    p = cantilever2d(512, 256, E=E, name="cantilever2d_simp_512x256")
    p.meta.update(seed=seed, ell=ell)
    return p


def cantilever3d_simp(nx, ny, nz, cuts, seed, ell=20.0, name=None):
    rho = ndtr(gaussian_random_field((nx, ny, nz), ell, seed))
    E = simp_moduli(_field_to_elements(rho))
    p = cantilever3d(nx, ny, nz, cuts, E=E, name=name)
    p.meta.update(seed=seed, ell=ell)
    return p


def cantilever3d_simp_128x64x64(seed=3, ell=20.0):
    """128x64x64 hex8, 8x4x5 uneven subdomains (z blocks 16,12,12,12,12)."""
    cuts = (even_cuts(128, 16), even_cuts(64, 16),
            np.array([0, 16, 28, 40, 52, 64], dtype=np.int64))
    return cantilever3d_simp(128, 64, 64, cuts, seed, ell,
                             name="cantilever3d_simp_128x64x64")


def to_sequence_2d(nsteps=60, nx=1024, ny=512, ell=20.0, base_seed=4000,
                   blend=0.1):
    """Density sequence of a topology-optimisation-like run.

    phi_0 is a fresh field; phi_k = (1-blend) phi_{k-1} + blend g_k, then
    re-standardised; rho_k thresholds phi_k at its median (volume 1/2).
    Yields element moduli E = 1e-3 + rho^3 for each step.
    """
    phi = gaussian_random_field((nx, ny), ell, base_seed)
    for k in range(nsteps):
        if k > 0:
            g = gaussian_random_field((nx, ny), ell, base_seed + k)
            phi = (1.0 - blend) * phi + blend * g
            phi = (phi - phi.mean()) / phi.std()
        rho = (phi > np.median(phi)).astype(np.float64)
        yield 1e-3 + _field_to_elements(rho) ** 3


def to_sequence_3d(nsteps=60, nx=128, ny=64, nz=64, ell=20.0, base_seed=6000,
                   blend=0.1):
    """The density sequence of ``to_sequence_2d`` on a 3D element grid."""
    phi = gaussian_random_field((nx, ny, nz), ell, base_seed)
    for k in range(nsteps):
        if k > 0:
            g = gaussian_random_field((nx, ny, nz), ell, base_seed + k)
            phi = (1.0 - blend) * phi + blend * g
            phi = (phi - phi.mean()) / phi.std()
        rho = (phi > np.median(phi)).astype(np.float64)
        yield 1e-3 + _field_to_elements(rho) ** 3


def simp_sequence_3d(nsteps, nx=128, ny=64, nz=64, ell=20.0, base_seed=7000,
                     blend=0.1):
    """Moduli fields shaped like the 3D SIMP cantilever's (smooth field,
    rho = Phi(phi), E = 1e-3 + rho^3 (1 - 1e-3)), blended 10% per step toward
    a fresh field as in ``to_sequence_3d`` but not thresholded."""
    phi = gaussian_random_field((nx, ny, nz), ell, base_seed)
    for k in range(nsteps):
        if k > 0:
            g = gaussian_random_field((nx, ny, nz), ell, base_seed + k)
            phi = (1.0 - blend) * phi + blend * g
            phi = (phi - phi.mean()) / phi.std()
        yield simp_moduli(_field_to_elements(ndtr(phi)))


def cnn_initial_weights(dim, cin, width, cout, seed, nlayers=4):
    """Seeded initial weights of the correction network: per layer a tap
    array of shape (3^dim, c_in, c_out) drawn from N(0, 2 / (3^dim c_in))
    and zero biases.  Random numbers only; the network itself is not here."""
    rng = np.random.default_rng(seed)
    chans = [cin] + [width] * (nlayers - 1) + [cout]
    out = []
    for a, b in zip(chans[:-1], chans[1:]):
        fan_in = 3 ** dim * a
        W = rng.standard_normal((3 ** dim, a, b)) * np.sqrt(2.0 / fan_in)
        out.append((W, np.zeros(b)))
    return out


def batch_uneven_problem(p, ell=8.0):
    """Problem ``p`` of the uneven batch: 2D for p < 32, 3D otherwise."""
    seed = 5000 + p
    rng = np.random.default_rng(seed)
    if p < 32:
        nx = int(rng.choice(np.arange(64, 257, 16)))
        ny = nx // 2
        rho = ndtr(gaussian_random_field((nx, ny), ell, seed))
        E = simp_moduli(_field_to_elements(rho))
        jl = int(rng.integers(0, ny + 1))
        return cantilever2d(nx, ny, E=E, load_node=(nx, jl),
                            name=f"batch{p}_2d_{nx}x{ny}")
    t = rng.uniform()
    nx = 16 + 8 * int(round(4 * t))
    ny = nz = 16 + 4 * int(round(2 * t))
    rho = ndtr(gaussian_random_field((nx, ny, nz), ell, seed))
    E = simp_moduli(_field_to_elements(rho))
    jl = int(rng.integers(0, ny + 1))
    kl = int(rng.integers(0, nz + 1))
    f = _point_load(3, (nx + 1, ny + 1, nz + 1), (nx, jl, kl), 2, -1.0)
    cuts = (even_cuts(nx, 16), even_cuts(ny, 16), even_cuts(nz, 16))
    return cantilever3d(nx, ny, nz, cuts, E=E, f=f,
                        name=f"batch{p}_3d_{nx}x{ny}x{nz}")

