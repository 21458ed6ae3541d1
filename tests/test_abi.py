"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "edd.h")
LIB = os.path.join(ROOT, "paper_1501_06211_amd", "libedd.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(edd_[A-Za-z_]+)\s*\(", src)))


def test_header_declares_core_calls():
    names = _declared()
    for n in ("edd_setup_mesh", "edd_set_element_moduli", "edd_apply_K",
              "edd_solve_interface"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_struct_layout_and_defaults():
    from paper_1501_06211_amd import edd
    assert sorted(edd.EXPORTS) == _declared()
    o = edd.default_opts()
    assert o.tol == 1e-8 and o.maxit == 2000 and o.precond == edd.PC_HTHETA
    assert o.theta == 0.5 and o.lanczos_kmax == 3 and o.inner_maxit == 4 and o.inner_tol == 0.0
    assert o.interface_weighting == 1
    L = edd.lib()
    assert L.edd_strerror(-5).decode().startswith("interior block")
    # no-GPU-call error paths
    assert L.edd_setup_mesh(None, None, None, None) == edd.EINVAL
    d = edd.MeshDesc()
    d.dim = 4
    h = ctypes.c_void_p()
    assert L.edd_setup_mesh(ctypes.byref(d), None, None, ctypes.byref(h)) == edd.EINVAL
    assert L.edd_destroy(None) == edd.OK
