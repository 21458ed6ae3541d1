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


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror of a header struct has the header's field offsets
    and size, as a C compiler lays them out."""
    import shutil
    import subprocess
    from paper_1501_06211_amd import edd
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [(edd.Allocator, "edd_allocator"), (edd.MeshDesc, "edd_mesh_desc"),
             (edd.SolveOpts, "edd_solve_opts"), (edd.SolveStats, "edd_solve_stats"),
             (edd.Info, "edd_info"), (edd.OcParams, "edd_oc_params"),
             (edd.OcResult, "edd_oc_result"), (edd.TopoptOpts, "edd_topopt_opts"),
             (edd.TopoptStats, "edd_topopt_stats"), (edd.KernelTimes, "edd_kernel_times")]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "edd.h"', "int main(void) {"]
    for cls, cname in pairs:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in cls._fields_:  # a trailing _ avoids a Python keyword (lambda_)
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0].rstrip("_")}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cls, cname in pairs:
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
