"""The C ABI library loads and exports every symbol its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "porestokes.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    import paper_2407_19868_amd as ps
    assert declared_symbols() == sorted(ps.EXPORTS)


def test_library_exports_every_declared_symbol():
    import paper_2407_19868_amd as ps
    lib = ps.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_host_only_calls():
    """Calls that touch no device: defaults and status strings."""
    import paper_2407_19868_amd as ps
    p = ps.params()
    assert p.re == 0.01 and p.c2 == 1.5e6 and p.dt == 2.0 ** -12 and p.tol == 1e-8
    assert p.check_every == 100 and p.precision == ps.FP64
    lib = ps.load_library()
    assert lib.pm_status_string(ps.PM_DIVERGED) == b"PM_DIVERGED"
    assert lib.pm_status_string(ps.PM_ERR_NO_FLOW) == b"PM_ERR_NO_FLOW"


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the sizes the C compiler gives them."""
    import subprocess
    import tempfile

    import paper_2407_19868_amd as ps
    src = ('#include "porestokes.h"\n#include <stdio.h>\n#include <stddef.h>\n'
           'int main(){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(pm_params), sizeof(pm_history),'
           ' sizeof(pm_instance), sizeof(pm_stats), sizeof(pm_pore_info), sizeof(pm_principal),'
           ' offsetof(pm_params, pore_cleanup));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    assert sizes == [ctypes.sizeof(ps.PmParams), ctypes.sizeof(ps.PmHistory),
                     ctypes.sizeof(ps.PmInstance), ctypes.sizeof(ps.PmStats), ctypes.sizeof(ps.PmPoreInfo),
                     ctypes.sizeof(ps.PmPrincipal), ps.PmParams.pore_cleanup.offset]


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2407_19868_amd as ps
    old = ps._lib
    try:
        ps._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            ps.load_library(str(tmp_path / "nope.so"))
    finally:
        ps._lib = old
