"""CPU checks of the HIP library boundary: it loads and exports every entry
point include/gkb.h declares (no compute calls: this host has no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2606_31153_amd as gk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(gkb_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_loads_and_exports_every_declared_symbol():
    L = gk.lib()
    declared = declared_symbols()
    assert {"gkb_forward", "gkb_back", "gkb_ab_solve", "gkb_ba_solve"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(gk.EXPORTED) <= declared


def test_binding_names_match_c_abi():
    for name in ("gkb_forward", "gkb_back", "gkb_forward_adjoint", "gkb_back_adjoint", "gkb_ab_solve",
                 "gkb_ba_solve", "gkb_gkb_solve", "gkb_batch_solve"):
        assert callable(getattr(gk, name))


def test_struct_layouts_match_header(tmp_path):
    # compile the header with the host C compiler and compare the struct sizes
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "gkb.h"\n'
                   '#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu", sizeof(gkb_geometry), sizeof(gkb_solve_opts),'
                   ' sizeof(gkb_solve_info), sizeof(gkb_hybrid_opts), offsetof(gkb_hybrid_opts, tsvd_rank),'
                   ' offsetof(gkb_hybrid_opts, lambda_history), sizeof(gkb_tuning)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    sizes = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert sizes == [ctypes.sizeof(gk.Geometry), ctypes.sizeof(gk.SolveOpts), ctypes.sizeof(gk.SolveInfo),
                     ctypes.sizeof(gk.HybridOpts), gk.HybridOpts.tsvd_rank.offset,
                     gk.HybridOpts.lambda_history.offset, ctypes.sizeof(gk.Tuning)]


def test_last_error_is_a_string():
    assert isinstance(gk.lib().gkb_last_error(), bytes)


def test_create_rejects_null_out_pointer():
    # argument validation happens before any device call
    assert gk.lib().gkb_create(None, 0, None) == gk.GKB_EINVAL
