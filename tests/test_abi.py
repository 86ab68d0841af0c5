"""CPU checks of the C ABI boundary: the built library loads, exports every
function include/mdpd.h declares, and the binding's struct layouts match the
header (compiled with gcc).  No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdpd.h")
LIB = os.path.join(ROOT, "paper_1903_10134_amd", "libmdpd.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mdpd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def native():
    if not os.path.exists(LIB):
        from paper_1903_10134_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mdpd_create", "mdpd_step", "mdpd_read_observables", "mdpd_get_state",
                     "mdpd_destroy", "mdpd_last_error", "mdpd_debug_neighbors", "mdpd_debug_forces"):
        assert required in names


def test_library_exports_every_declared_symbol(native):
    missing = [n for n in declared_functions() if not hasattr(native, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_1903_10134_amd as m
    for n in declared_functions():
        assert hasattr(m, n), n


def test_struct_layouts_match_header(tmp_path):
    import paper_1903_10134_amd._native as nat
    c = tmp_path / "sizes.c"
    c.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mdpd.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(mdpd_params),"
        " offsetof(mdpd_params, seed), offsetof(mdpd_params, wall_model), offsetof(mdpd_params, wall_slip),"
        " sizeof(mdpd_observables),"
        " offsetof(mdpd_observables, ke), offsetof(mdpd_observables, momentum)); return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    P, O = nat.Params, nat.Observables
    assert vals == [ctypes.sizeof(P), P.seed.offset, P.wall_model.offset, P.wall_slip.offset, ctypes.sizeof(O),
                    O.ke.offset, O.momentum.offset]


def test_last_error_is_callable_without_a_device(native):
    native.mdpd_last_error.restype = ctypes.c_char_p
    assert isinstance(native.mdpd_last_error(), bytes)


def test_product_path_has_no_oracle_dependency():
    """The package must not import, link or read anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_1903_10134_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "mdpd_oracle" not in text and "liboracle" not in text, f
