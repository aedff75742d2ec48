"""The C-ABI library builds for gfx950, loads, and exports every call md.h declares.

No compute call is made here (this runs without a GPU).
"""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["md_init", "md_build_cells", "md_forces", "md_step", "md_observables",
                 "md_set_state", "md_get_state", "md_get_forces", "md_get_cells",
                 "md_get_neighbors", "md_destroy", "md_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1105_5613_amd import build, md
    if not os.path.exists(md.LIB_PATH):
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", md.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(md_[a-z_]+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    lib = md.lib()  # loads without a GPU
    for n in declared():
        assert hasattr(lib, n)
    assert set(md.EXPORTS) == set(declared())


def test_struct_layouts_match_header():
    """ctypes mirrors of md_params / md_obs have the C sizes (checked with the C compiler)."""
    import ctypes as C
    from paper_1105_5613_amd import md
    src = ('#include "md.h"\n#include <stdio.h>\n'
           'int main(void){printf("%zu %zu\\n", sizeof(md_params), sizeof(md_obs));return 0;}\n')
    exe = os.path.join(ROOT, "_build_abi_probe")
    r = subprocess.run(["gcc", "-x", "c", "-I", os.path.join(ROOT, "include"), "-", "-o", exe],
                       input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr
    try:
        sizes = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    finally:
        os.remove(exe)
    assert int(sizes[0]) == C.sizeof(md.Params)
    assert int(sizes[1]) == C.sizeof(md.Obs)
