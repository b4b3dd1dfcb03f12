"""The C-ABI library loads on the CPU and exports every entry point the header declares."""
import ctypes
import re
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "mgdwf.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgdwf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mgdwf_create", "mgdwf_apply_dwf", "mgdwf_set_nullvecs", "mgdwf_restrict", "mgdwf_prolong",
                     "mgdwf_build_coarse", "mgdwf_apply_coarse", "mgdwf_setup", "mgdwf_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(str(ROOT / "paper_1205_2933_amd" / "libmgdwf.so"))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    import paper_1205_2933_amd as mg
    assert set(declared_functions()) <= set(mg.exported_symbols())


def test_invalid_arguments_are_rejected_without_a_device():
    """Argument validation runs before any device work (no GPU needed)."""
    import paper_1205_2933_amd._lib as L
    a = L.mgdwf_action()
    a.L[:] = [4, 4, 1, 4]   # extent 1 is invalid
    a.Ls, a.M5, a.mf = 4, 1.8, 0.01
    a.bc[:] = [1, 1, 1, 1]
    h = ctypes.c_void_p()
    st = L._lib.mgdwf_create(ctypes.byref(a), None, ctypes.byref(h))
    assert st == L.MGDWF_ERR_INVALID_ARG
    assert b"extent" in L._lib.mgdwf_last_error(None)
    a.L[:] = [4, 4, 4, 4]
    a.bc[:] = [1, 2, 1, 1]
    assert L._lib.mgdwf_create(ctypes.byref(a), None, ctypes.byref(h)) == L.MGDWF_ERR_INVALID_ARG


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets
    (a C probe built with gcc against include/mgdwf.h prints them)."""
    import subprocess
    import paper_1205_2933_amd._lib as L
    structs = [L.mgdwf_action, L.mgdwf_mg_params, L.mgdwf_solve_params, L.mgdwf_solve_report,
               L.mgdwf_setup_report, L.mgdwf_tune_report, L.mgdwf_net_config]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mgdwf.h"', "int main(void) {"]
    for s in structs:
        n = s.__name__
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in s._fields_:
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", str(ROOT / "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_side = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for s in structs:
        n = s.__name__
        assert c_side[(n, "size")] == ctypes.sizeof(s), n
        for f, _ in s._fields_:
            assert c_side[(n, f)] == getattr(s, f).offset, (n, f)
