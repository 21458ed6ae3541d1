"""ctypes binding of the edd C ABI (include/edd.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory (through the library's allocator callbacks,
so the caching allocator owns every buffer) and the HIP stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libedd.so")

# status codes
OK, NOT_CONVERGED = 0, 1
EINVAL, ENOMEM, EHIP, ESTATE, ENOTSPD, EBREAKDOWN = -1, -2, -3, -4, -5, -6
F64, F32 = 1, 2
CLAMP_X0, CLAMP_X1, CLAMP_Y0, CLAMP_Y1, CLAMP_Z0, CLAMP_Z1 = 1, 2, 4, 8, 16, 32
MODE_F64, MODE_MIXED, MODE_RELAXED = 0, 1, 2
PC_IDENTITY, PC_HTHETA, PC_SCHUR = 0, 1, 2
PCF_HTILDE_INV, PCF_H_INV, PCF_HTILDE_FWD, PCF_H_FWD = 0, 1, 2, 3
FLAG_TRUE_RES_RESTART, FLAG_MIXED_FALLBACK, FLAG_PC_DROPPED = 1, 2, 4
FLAG_LEARNED_REJECTED = 8

EXPORTS = [
    "edd_default_opts", "edd_setup_mesh", "edd_set_element_moduli",
    "edd_apply_K", "edd_solve_interface", "edd_solve_interior", "edd_apply_S",
    "edd_apply_precond", "edd_get_info", "edd_get_gamma_nodes",
    "edd_get_interior_nodes", "edd_destroy", "edd_strerror",
    "edd_last_hip_error", "edd_set_kernel_timing", "edd_get_kernel_times",
    "edd_apply_skeleton_op", "edd_cnn_setup", "edd_cnn_num_params",
    "edd_cnn_set_params", "edd_cnn_get_params", "edd_cnn_predict",
    "edd_cnn_loss_grad", "edd_cnn_train_step", "edd_solve_batch", "edd_autotune",
    "edd_set_solve_variants", "edd_apply_S_noalloc", "edd_cnn_training_pair",
    "edd_element_energies", "edd_oc_update", "edd_default_topopt_opts", "edd_topopt_run",
    "edd_solve_gmres", "edd_autotune_cache", "edd_set_apply_variant",
    "edd_cnn_matrix_cores", "edd_set_s_apply", "edd_get_s_apply",
]
NOALLOC_MAX_INTERIOR_DOFS = 1 << 21
KT_NAMES = ["band_solve", "band_cholesky", "apply_K", "apply_mapped", "assemble",
            "precond", "layouts", "band_solve32"]


class EddError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().edd_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} (status {code})")


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nel", ctypes.c_int * 3),
        ("ncuts", ctypes.c_int * 3),
        ("cuts", ctypes.POINTER(ctypes.c_int) * 3),
        ("nu", ctypes.c_double),
        ("clamp_faces", ctypes.c_int),
        ("factor_precision", ctypes.c_int),
        ("dissect", ctypes.c_int),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("theta", ctypes.c_double),
        ("lanczos_kmax", ctypes.c_int),
        ("lanczos_tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("inner_maxit", ctypes.c_int),
        ("use_initial_guess", ctypes.c_int),
        ("outer_maxit", ctypes.c_int),
        ("mixed_inner_tol", ctypes.c_double),
        ("flexible_window", ctypes.c_int),
        ("interface_weighting", ctypes.c_int),
        ("learned_guess", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("pc_form", ctypes.c_int),
        ("learned_correction", ctypes.c_int),
        ("mass_matrix", ctypes.c_int),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("iterations", ctypes.c_int),
        ("outer_iterations", ctypes.c_int),
        ("precond_applications", ctypes.c_int),
        ("lanczos_steps", ctypes.c_int),
        ("inner_iterations", ctypes.c_int),
        ("flags", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("compliance", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("t_krylov_ms", ctypes.c_double),
        ("learned_alpha", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_sub", ctypes.c_int),
        ("n_nodes", ctypes.c_int64), ("ndof", ctypes.c_int64),
        ("n_el", ctypes.c_int64), ("n_gamma", ctypes.c_int64),
        ("n_interior_dofs", ctypes.c_int64), ("factor_entries", ctypes.c_int64),
        ("max_band", ctypes.c_int), ("max_sub_dofs", ctypes.c_int),
        ("skeleton_faces", ctypes.c_int64), ("face_classes", ctypes.c_int),
        ("theta_default", ctypes.c_double),
        ("band_blocks", ctypes.c_int), ("coupling_entries", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OcParams(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("move", ctypes.c_double),
                ("eta", ctypes.c_double), ("penal", ctypes.c_double),
                ("emin", ctypes.c_double)]


class OcResult(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("volume", ctypes.c_double),
                ("max_change", ctypes.c_double)]

    def as_dict(self):
        return {"lambda": self.lambda_, "volume": self.volume, "max_change": self.max_change}


class TopoptOpts(ctypes.Structure):
    _fields_ = [("volfrac", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("move", ctypes.c_double),
                ("eta", ctypes.c_double), ("penal", ctypes.c_double),
                ("emin", ctypes.c_double), ("change_tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("adaptive_tol", ctypes.c_int),
                ("tol_min", ctypes.c_double), ("tol_max", ctypes.c_double),
                ("warm_start", ctypes.c_int)]


class TopoptStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int),
                ("converged", ctypes.c_int), ("krylov_iterations", ctypes.c_int),
                ("avg_krylov", ctypes.c_double), ("compliance", ctypes.c_double),
                ("max_change", ctypes.c_double), ("volume", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("t_moduli_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_update_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTimes(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64 * 8), ("total_ms", ctypes.c_double * 8)]


ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_T), ("free", FREE_T), ("ctx", ctypes.c_void_p)]


_LIB = None


def lib():
    """Load libedd.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.edd_default_opts.argtypes = [ctypes.POINTER(SolveOpts)]
    L.edd_default_opts.restype = None
    L.edd_setup_mesh.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(Allocator),
                                 vp, ctypes.POINTER(vp)]
    L.edd_set_element_moduli.argtypes = [vp, vp, i32]
    L.edd_apply_K.argtypes = [vp, vp, vp]
    L.edd_solve_interface.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts),
                                      ctypes.POINTER(SolveStats)]
    L.edd_solve_gmres.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts),
                                  ctypes.POINTER(SolveStats)]
    L.edd_solve_interior.argtypes = [vp, vp, vp, i32]
    L.edd_apply_S.argtypes = [vp, vp, vp, i32]
    L.edd_apply_S_noalloc.argtypes = [vp, vp, vp, i32]
    L.edd_apply_precond.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts)]
    L.edd_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.edd_get_gamma_nodes.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.edd_get_interior_nodes.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.edd_destroy.argtypes = [vp]
    L.edd_strerror.argtypes = [i32]
    L.edd_strerror.restype = ctypes.c_char_p
    L.edd_last_hip_error.argtypes = [vp]
    L.edd_set_kernel_timing.argtypes = [vp, i32]
    L.edd_apply_skeleton_op.argtypes = [vp, i32, i32, vp, vp, dbl, i32]
    L.edd_get_kernel_times.argtypes = [vp, ctypes.POINTER(KernelTimes)]
    L.edd_solve_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                  ctypes.POINTER(vp), ctypes.POINTER(SolveOpts),
                                  ctypes.POINTER(SolveStats), i32]
    L.edd_autotune.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.edd_autotune_cache.argtypes = [ctypes.c_char_p]
    L.edd_set_apply_variant.argtypes = [vp, i32]
    L.edd_set_solve_variants.argtypes = [vp, ctypes.POINTER(i32)]
    L.edd_set_s_apply.argtypes = [vp, i32]
    L.edd_get_s_apply.argtypes = [vp, ctypes.POINTER(i32)]
    L.edd_cnn_setup.argtypes = [vp, i32]
    L.edd_cnn_matrix_cores.argtypes = [vp, i32]
    L.edd_cnn_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.edd_cnn_set_params.argtypes = [vp, vp]
    L.edd_cnn_get_params.argtypes = [vp, vp]
    L.edd_cnn_predict.argtypes = [vp, vp, vp, vp]
    L.edd_cnn_loss_grad.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(dbl)]
    L.edd_cnn_train_step.argtypes = [vp, vp, vp, vp, dbl, ctypes.POINTER(dbl)]
    L.edd_cnn_training_pair.argtypes = [vp, vp, vp, vp, vp, vp]
    L.edd_element_energies.argtypes = [vp, vp, vp]
    L.edd_oc_update.argtypes = [vp, vp, vp, ctypes.POINTER(OcParams), vp, vp,
                                ctypes.POINTER(OcResult)]
    L.edd_default_topopt_opts.argtypes = [ctypes.POINTER(TopoptOpts)]
    L.edd_default_topopt_opts.restype = None
    L.edd_topopt_run.argtypes = [vp, vp, vp, vp, ctypes.POINTER(TopoptOpts),
                                 ctypes.POINTER(SolveOpts), ctypes.POINTER(TopoptStats),
                                 ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("edd_default_opts", "edd_strerror", "edd_default_topopt_opts"):
            f.restype = i32
    _LIB = L
    return L


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().edd_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown solve option {k!r}")
        setattr(o, k, v)
    return o


def _ptr(t, dtype=torch.float64, n=None, device=None, what="tensor"):
    """Device address of a contiguous CUDA tensor after checking its dtype,
    its length (``n`` entries) and its device, so that no library call ever
    sees a buffer shorter than the kernels index."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype \
            or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous CUDA {dtype} tensor")
    if n is not None and t.numel() != int(n):
        raise ValueError(f"{what}: expected {int(n)} entries, got {t.numel()}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what}: tensor on cuda:{t.device.index}, problem on cuda:{device}")
    return ctypes.c_void_p(t.data_ptr())


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching
    allocator on the handle's stream."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream

        def _alloc(ctx, nbytes):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                          self.stream)
            except Exception:  # pragma: no cover - reported as ENOMEM
                return None

        def _free(ctx, ptr):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = ALLOC_T(_alloc)
        self._free = FREE_T(_free)
        self.struct = Allocator(self._alloc, self._free, None)


class Problem:
    """One decomposed elasticity problem on the current GPU.

    dim, nel, cuts, nu, clamp describe the grid as in include/edd.h;
    factor_precision selects which interior factors are built (F64, F32 or
    both).  All vectors are FP64 CUDA tensors in node-major layout.
    """

    def __init__(self, dim, nel, cuts, nu=0.3, clamp=CLAMP_X0,
                 factor_precision=F64 | F32, stream=None, torch_allocator=True,
                 dissect=-1):
        L = lib()
        self.dim = int(dim)
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        d = MeshDesc()
        d.dim = self.dim
        self._cut_arrays = []
        for a in range(3):
            d.nel[a] = int(nel[a]) if a < dim else 1
            if a < dim:
                arr = (ctypes.c_int * len(cuts[a]))(*[int(c) for c in cuts[a]])
                self._cut_arrays.append(arr)
                d.cuts[a] = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int))
                d.ncuts[a] = len(cuts[a])
        d.nu = float(nu)
        d.clamp_faces = int(clamp)
        d.factor_precision = int(factor_precision)
        d.dissect = int(dissect)
        self.factor_precision = int(factor_precision)
        self._alloc = _TorchAllocator(self.device, self.stream) if torch_allocator else None
        h = ctypes.c_void_p()
        rc = L.edd_setup_mesh(ctypes.byref(d),
                              ctypes.byref(self._alloc.struct) if self._alloc else None,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise EddError(rc, "edd_setup_mesh")
        self.h = h
        info = Info()
        L.edd_get_info(self.h, ctypes.byref(info))
        self.info = info.as_dict()
        self.n_nodes = self.info["n_nodes"]
        self.ndof = self.info["ndof"]
        self.n_gamma = self.info["n_gamma"]
        self.n_interior_dofs = self.info["n_interior_dofs"]

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w.dim, w.nel, w.cuts, nu=w.nu, clamp=w.clamp, **kw)

    def _check(self, rc, what):
        if rc not in (OK, NOT_CONVERGED):
            if rc == EHIP:
                what = f"{what} (hipError_t {lib().edd_last_hip_error(self.h)})"
            raise EddError(rc, what)
        return rc

    # ---- argument checks and stream ordering ----------------------------------
    def _v(self, t, n, what, dtype=torch.float64):
        return _ptr(t, dtype, n=n, device=self.device, what=what)

    @contextlib.contextmanager
    def _ordered(self, *tensors):
        """The library runs on the handle's stream.  When that is not torch's
        current stream, the handle's stream first waits for the work already
        queued on the current one (inputs), and the current stream then waits
        for the library's work (outputs); the tensors are marked as used on
        the handle's stream so the caching allocator does not recycle them
        early."""
        cur = torch.cuda.current_stream(self.device)
        other = cur != self.stream
        if other:
            self.stream.wait_stream(cur)
        try:
            yield
        finally:
            if other:
                cur.wait_stream(self.stream)
                for t in tensors:
                    if t is not None:
                        t.record_stream(self.stream)

    @property
    def n_gamma_dofs(self):
        return self.n_gamma * self.dim

    def set_element_moduli(self, E: torch.Tensor):
        dt = {torch.float64: F64, torch.float32: F32}.get(E.dtype)
        if dt is None:
            raise ValueError("moduli must be float64 or float32")
        pe = self._v(E, self.info["n_el"], "E", E.dtype)
        self._E = E
        with self._ordered(E):
            self._check(lib().edd_set_element_moduli(self.h, pe, dt),
                        "edd_set_element_moduli")

    def apply_K(self, u: torch.Tensor, out: torch.Tensor | None = None):
        if out is None:
            out = torch.empty_like(u)
        pu, po = self._v(u, self.ndof, "u"), self._v(out, self.ndof, "out")
        with self._ordered(u, out):
            self._check(lib().edd_apply_K(self.h, pu, po), "edd_apply_K")
        return out

    def solve(self, f: torch.Tensor, u: torch.Tensor | None = None, **opts):
        if u is None:
            u = torch.zeros_like(f)
            opts.setdefault("use_initial_guess", 0)
        o = default_opts(**opts)
        st = SolveStats()
        pf, pu = self._v(f, self.ndof, "f"), self._v(u, self.ndof, "u")
        with self._ordered(f, u):
            rc = lib().edd_solve_interface(self.h, pf, pu, ctypes.byref(o), ctypes.byref(st))
        self._check(rc, "edd_solve_interface")
        return u, st.as_dict()

    def solve_gmres(self, f: torch.Tensor, u: torch.Tensor | None = None, **opts):
        """The paper's Krylov method: flexible GMRES on K with the block-
        triangular preconditioner P~ (edd_solve_gmres).  precond selects S~
        (PC_IDENTITY, PC_HTHETA, PC_SCHUR)."""
        if u is None:
            u = torch.zeros_like(f)
            opts.setdefault("use_initial_guess", 0)
        o = default_opts(**opts)
        st = SolveStats()
        pf, pu = self._v(f, self.ndof, "f"), self._v(u, self.ndof, "u")
        with self._ordered(f, u):
            rc = lib().edd_solve_gmres(self.h, pf, pu, ctypes.byref(o), ctypes.byref(st))
        self._check(rc, "edd_solve_gmres")
        return u, st.as_dict()

    # ---- tile shapes -----------------------------------------------------------
    def autotune(self, force=False):
        """(FP64 substitution variant, FP32 substitution variant, element tile
        shapes for all / interior / interface nodes) chosen by edd_autotune."""
        v = (ctypes.c_int * 5)()
        with self._ordered():
            self._check(lib().edd_autotune(self.h, int(force), v), "edd_autotune")
        return tuple(int(x) for x in v)

    def set_apply_variant(self, v):
        self._check(lib().edd_set_apply_variant(self.h, int(v)), "edd_set_apply_variant")

    def set_solve_variants(self, f64, f32):
        v = (ctypes.c_int * 2)(int(f64), int(f32))
        self._check(lib().edd_set_solve_variants(self.h, v), "edd_set_solve_variants")

    def set_s_apply(self, mode):
        """0: S v through the interior factors; 1: explicit local Schur
        complements (see edd_set_s_apply)."""
        self._check(lib().edd_set_s_apply(self.h, int(mode)), "edd_set_s_apply")

    @property
    def s_apply(self):
        m = ctypes.c_int()
        self._check(lib().edd_get_s_apply(self.h, ctypes.byref(m)), "edd_get_s_apply")
        return int(m.value)

    # ---- correction network -------------------------------------------------
    def _nparams(self):
        n = ctypes.c_int64()
        self._check(lib().edd_cnn_num_params(self.h, ctypes.byref(n)), "edd_cnn_num_params")
        return int(n.value)

    def cnn_setup(self, width=32):
        with self._ordered():
            self._check(lib().edd_cnn_setup(self.h, width), "edd_cnn_setup")
        return self._nparams()

    def cnn_matrix_cores(self, enable=True):
        """Hidden layers' forward pass on the FP16 matrix cores (edd_cnn_matrix_cores)."""
        self._check(lib().edd_cnn_matrix_cores(self.h, int(enable)), "edd_cnn_matrix_cores")

    def cnn_set_params(self, params: torch.Tensor):
        pp = self._v(params, self._nparams(), "params", torch.float32)
        with self._ordered(params):
            self._check(lib().edd_cnn_set_params(self.h, pp), "edd_cnn_set_params")

    def cnn_get_params(self):
        out = torch.empty(self._nparams(), dtype=torch.float32, device=self.device)
        with self._ordered(out):
            self._check(lib().edd_cnn_get_params(self.h, _ptr(out, torch.float32)),
                        "edd_cnn_get_params")
        return out

    def _optr(self, E):
        return None if E is None else self._v(E, self.info["n_el"], "E")

    def cnn_predict(self, r, out=None, E=None):
        if out is None:
            out = torch.empty_like(r)
        pe, pr, po = self._optr(E), self._v(r, self.ndof, "r"), self._v(out, self.ndof, "out")
        with self._ordered(E, r, out):
            self._check(lib().edd_cnn_predict(self.h, pe, pr, po), "edd_cnn_predict")
        return out

    def cnn_loss_grad(self, r, e, E=None):
        g = torch.empty(self._nparams(), dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        pe, pr, pq = self._optr(E), self._v(r, self.ndof, "r"), self._v(e, self.ndof, "e")
        with self._ordered(E, r, e, g):
            self._check(lib().edd_cnn_loss_grad(self.h, pe, pr, pq, _ptr(g, torch.float32),
                                                ctypes.byref(loss)), "edd_cnn_loss_grad")
        return float(loss.value), g

    def cnn_train_step(self, r, e, lr=1e-3, E=None):
        loss = ctypes.c_double()
        pe, pr, pq = self._optr(E), self._v(r, self.ndof, "r"), self._v(e, self.ndof, "e")
        with self._ordered(E, r, e):
            self._check(lib().edd_cnn_train_step(self.h, pe, pr, pq, lr, ctypes.byref(loss)),
                        "edd_cnn_train_step")
        return float(loss.value)

    def cnn_training_pair(self, f, u_prev, u):
        """(r, e) = (f - K u_prev, u - u_prev) for the moduli set last
        (edd_cnn_training_pair)."""
        r, e = torch.empty_like(f), torch.empty_like(f)
        n = self.ndof
        args = [self._v(t, n, nm) for t, nm in ((f, "f"), (u_prev, "u_prev"), (u, "u"),
                                                  (r, "r"), (e, "e"))]
        with self._ordered(f, u_prev, u, r, e):
            self._check(lib().edd_cnn_training_pair(self.h, *args), "edd_cnn_training_pair")
        return r, e

    # ---- topology optimisation (Section 5) -------------------------------------
    def element_energies(self, u, out=None):
        """s_e = u_e^T K0 u_e (edd_element_energies)."""
        n_el = self.info["n_el"]
        if out is None:
            out = torch.empty(n_el, dtype=torch.float64, device=self.device)
        pu, po = self._v(u, self.ndof, "u"), self._v(out, n_el, "out")
        with self._ordered(u, out):
            self._check(lib().edd_element_energies(self.h, pu, po), "edd_element_energies")
        return out

    def oc_update(self, rho, s, volume, rho_min=1e-3, rho_max=1.0, move=0.2, eta=0.5,
                  penal=1.0, emin=0.0):
        """One OC density update (edd_oc_update).  Returns (rho_new, E_new,
        result dict)."""
        n_el = self.info["n_el"]
        rho_new = torch.empty(n_el, dtype=torch.float64, device=self.device)
        E_new = torch.empty_like(rho_new)
        prm = OcParams(volume, rho_min, rho_max, move, eta, penal, emin)
        res = OcResult()
        pr, ps = self._v(rho, n_el, "rho"), self._v(s, n_el, "s")
        with self._ordered(rho, s, rho_new, E_new):
            self._check(lib().edd_oc_update(self.h, pr, ps, ctypes.byref(prm), _ptr(rho_new),
                                            _ptr(E_new), ctypes.byref(res)), "edd_oc_update")
        return rho_new, E_new, res.as_dict()

    def topopt(self, f, rho, u=None, solve_opts=None, **opts):
        """The fixed-point loop of Section 5 (edd_topopt_run).  rho (n_el,
        FP64) is overwritten by the final design.  Returns (rho, u, stats,
        history) with history an array of rows (compliance, tolerance,
        iterations, max change, residual) per step."""
        import numpy as np
        to = TopoptOpts()
        lib().edd_default_topopt_opts(ctypes.byref(to))
        for k, v in opts.items():
            if not hasattr(to, k):
                raise KeyError(f"unknown topology-optimisation option {k!r}")
            setattr(to, k, v)
        so = default_opts(**(solve_opts or {}))
        if u is None:
            u = torch.zeros_like(f)
        st = TopoptStats()
        hist = np.zeros(5 * to.maxit)
        pf, pr, pu = (self._v(f, self.ndof, "f"), self._v(rho, self.info["n_el"], "rho"),
                      self._v(u, self.ndof, "u"))
        with self._ordered(f, rho, u):
            rc = lib().edd_topopt_run(self.h, pf, pr, pu, ctypes.byref(to), ctypes.byref(so),
                                      ctypes.byref(st),
                                      hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._check(rc, "edd_topopt_run")
        d = st.as_dict()
        return rho, u, d, hist.reshape(-1, 5)[:d["steps"]]

    def solve_interior(self, b, out=None, precision=F64):
        if out is None:
            out = torch.empty_like(b)
        n = self.n_interior_dofs
        pb, po = self._v(b, n, "b"), self._v(out, n, "out")
        with self._ordered(b, out):
            self._check(lib().edd_solve_interior(self.h, pb, po, precision),
                        "edd_solve_interior")
        return out

    def apply_S(self, v, out=None, precision=F64):
        if out is None:
            out = torch.empty_like(v)
        n = self.n_gamma_dofs
        pv, po = self._v(v, n, "v"), self._v(out, n, "out")
        with self._ordered(v, out):
            self._check(lib().edd_apply_S(self.h, pv, po, precision), "edd_apply_S")
        return out

    def apply_S_noalloc(self, v, out, precision=F64):
        """edd_apply_S_noalloc: S v with the library's static work array (the
        output buffer is supplied by the caller)."""
        n = self.n_gamma_dofs
        pv, po = self._v(v, n, "v"), self._v(out, n, "out")
        with self._ordered(v, out):
            self._check(lib().edd_apply_S_noalloc(self.h, pv, po, precision),
                        "edd_apply_S_noalloc")
        return out

    def apply_precond(self, r, out=None, **opts):
        if out is None:
            out = torch.empty_like(r)
        o = default_opts(**opts)
        n = self.n_gamma_dofs
        pr, po = self._v(r, n, "r"), self._v(out, n, "out")
        with self._ordered(r, out):
            self._check(lib().edd_apply_precond(self.h, pr, po, ctypes.byref(o)),
                        "edd_apply_precond")
        return out

    def skeleton_op(self, which, x, weighting=1, tol=1e-12, maxit=1000, out=None):
        """which: 0 L, 1 M (lumped), 2 face-block preconditioner, 3 PCG solve,
        4 M (consistent), 5 M^{-1} (consistent, Chebyshev)."""
        if out is None:
            out = torch.empty_like(x)
        n = self.n_gamma_dofs
        px, po = self._v(x, n, "x"), self._v(out, n, "out")
        with self._ordered(x, out):
            self._check(lib().edd_apply_skeleton_op(self.h, int(which), int(weighting), px, po,
                                                    float(tol), int(maxit)),
                        "edd_apply_skeleton_op")
        return out

    def gamma_nodes(self):
        import numpy as np
        out = np.zeros(self.n_gamma, dtype=np.int32)
        lib().edd_get_gamma_nodes(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return out

    def interior_nodes(self):
        import numpy as np
        out = np.zeros(self.n_interior_dofs // self.dim, dtype=np.int32)
        lib().edd_get_interior_nodes(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return out

    def set_kernel_timing(self, enable=True):
        self._check(lib().edd_set_kernel_timing(self.h, int(enable)),
                    "edd_set_kernel_timing")

    def kernel_times(self):
        t = KernelTimes()
        self._check(lib().edd_get_kernel_times(self.h, ctypes.byref(t)),
                    "edd_get_kernel_times")
        return {n: (int(t.count[i]), float(t.total_ms[i]))
                for i, n in enumerate(KT_NAMES)}

    def close(self):
        if getattr(self, "h", None):
            lib().edd_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def set_autotune_cache(path):
    """edd_autotune_cache: persist autotuner choices in a file (None: memory only)."""
    lib().edd_autotune_cache(None if path is None else os.fsencode(path))


def solve_batch(problems, fs, us, nthreads=0, **opts):
    """Solve independent problems concurrently (edd_solve_batch).  Returns
    (status, [stats dict per problem]).  Each handle's stream first waits for
    the work queued on torch's current stream; the library synchronises every
    handle before returning."""
    n = len(problems)
    if len(fs) != n or len(us) != n:
        raise ValueError("solve_batch: one f and one u per problem")
    hs = (ctypes.c_void_p * n)(*[p.h.value for p in problems])
    fp = (ctypes.c_void_p * n)(*[p._v(f, p.ndof, "f").value for p, f in zip(problems, fs)])
    up = (ctypes.c_void_p * n)(*[p._v(u, p.ndof, "u").value for p, u in zip(problems, us)])
    for p in problems:
        cur = torch.cuda.current_stream(p.device)
        if cur != p.stream:
            p.stream.wait_stream(cur)
    o = default_opts(**opts)
    st = (SolveStats * n)()
    rc = lib().edd_solve_batch(hs, n, fp, up, ctypes.byref(o), st, int(nthreads))
    if rc not in (OK, NOT_CONVERGED):
        raise EddError(rc, "edd_solve_batch")
    return rc, [s.as_dict() for s in st]
