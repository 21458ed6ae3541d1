"""MI355X (gfx950) Schur-interface solver for linear elasticity.

Implements the hot path of Turner, Kocvara and Loghin, "Parallel Solution of
the Linear Elasticity problem with applications in Topology Optimisation"
(arXiv 1501.06211): matrix-free element stiffness products, batched banded
interior solves for all subdomains, and the preconditioned interface
(Schur-complement) iteration, in hand-written HIP kernels behind the C ABI
of include/edd.h.  ``edd`` is the Python binding.
"""
from . import edd  # noqa: F401
from .edd import Problem, EddError, default_opts  # noqa: F401
