"""CPU oracle for the Schur-interface elasticity solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 statement of
what the GPU path computes, written from the paper (Turner, Kocvara, Loghin,
"Parallel Solution of the Linear Elasticity problem with applications in
Topology Optimisation", arXiv 1501.06211).  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code
with the HIP library and imports nothing from the product package; the
seeded input generators live in ``workloads`` and hold none of the method.

Modules
  fe      element matrices, assembly, Dirichlet elimination, direct solve
  dd      node classification, K_II/K_IG/K_GG blocks, Schur complement
  iface   interface mass/Laplacian, H_theta closed forms, inverse Lanczos
  krylov  reference PCG / flexible CG / right-preconditioned GMRES
  cnn     reference forward/backward of the small correction network

Parity status of each function is stated in its docstring; every function
here is pinned by a ``-m "not gpu"`` test unless it says "parity unpinned".
"""
