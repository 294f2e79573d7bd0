"""The C-ABI library loads and exports every entry point that include/gofd.h declares."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gofd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gofd_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("gofd_build_transfer", "gofd_fd_weights", "gofd_apply_Ah", "gofd_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2307_14437_amd as gofd
    out = subprocess.run(["nm", "-D", "--defined-only", gofd.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(gofd.lib, n)     # resolvable through the binding's CDLL


def test_status_names():
    import paper_2307_14437_amd as gofd
    assert gofd.lib.gofd_strerror(-4) == b"GOFD_E_ZERO_COLSUM"
    assert gofd.lib.gofd_strerror(0) == b"GOFD_OK"


def test_tuning_cache_roundtrip(tmp_path):
    import paper_2307_14437_amd as gofd
    path = str(tmp_path / "c.json")
    assert gofd.cache_lookup(path, "gfx950/d2/L2048/fp32") is None
    gofd.cache_store(path, "gfx950/d2/L2048/fp32", 1, [1.0, 0.5, 2.0, 3.0])
    gofd.cache_store(path, "gfx950/d2/L1024/fp64", 2, [1.0, 1.0, 0.5, 1.0])
    assert gofd.cache_lookup(path, "gfx950/d2/L2048/fp32") == 1
    assert gofd.cache_lookup(path, "gfx950/d2/L1024/fp64") == 2
    gofd.cache_store(path, "gfx950/d2/L2048/fp32", 0, [1.0, 2.0, 2.0, 3.0, 1.0, 0.8], row=16)
    assert gofd.cache_lookup(path, "gfx950/d2/L2048/fp32", full=True)["row"] == 16
    assert [gofd.fft_period(n) for n in (1, 2, 3, 32, 33, 512)] == [8, 8, 16, 128, 256, 2048]


def test_struct_layouts_match_binding(tmp_path):
    # every structure the binding mirrors has the C layout of include/gofd.h:
    # size and the offset of each field, from a C program built with gcc
    import ctypes
    import shutil
    import subprocess
    import paper_2307_14437_amd as gofd
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [("gofd_grid", gofd._Grid), ("gofd_transfer_info", gofd.TransferInfo),
             ("gofd_fdw_opts", gofd.FdwOpts), ("gofd_precond_info", gofd.PrecondInfo),
             ("gofd_solve_opts", gofd.SolveOpts), ("gofd_solve_info", gofd.SolveInfo),
             ("gofd_cg_tape_info", gofd.CgTapeInfo), ("gofd_mmpde_opts", gofd.MmpdeOpts),
             ("gofd_mmpde_kernel_stats", gofd.MmpdeKernelStats), ("gofd1d_info", gofd.Info1D),
             ("gofd1d_solve_info", gofd.SolveInfo1D),
             ("gofd_mmpde_info", gofd.MmpdeInfo)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gofd.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
