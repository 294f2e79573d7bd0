"""The C-ABI library loads and exports every entry point that include/gofd.h declares."""

import os
import re
import subprocess

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
    assert [gofd.fft_period(n) for n in (1, 2, 3, 32, 33, 512)] == [8, 8, 16, 128, 256, 2048]
