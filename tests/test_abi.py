"""The C-ABI library loads and exports every function include/kcore.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(kcore_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["kcore_decompose", "kcore_decompose32", "kcore_decompose_batch", "kcore_last_error",
                     "kcore_serve_create", "kcore_serve_submit", "kcore_serve_poll", "kcore_serve_wait",
                     "kcore_serve_stats", "kcore_serve_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2512_00233_amd as kc
    if not os.path.exists(kc.library_path()):
        pytest.skip("libkcore.so not built")
    lib = ctypes.CDLL(kc.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_without_gpu():
    import paper_2512_00233_amd as kc
    if not os.path.exists(kc.library_path()):
        pytest.skip("libkcore.so not built")
    assert "gfx950" in kc.version()
    lib = kc.load()
    # argument checks run before any device call
    assert lib.kcore_decompose(-5, None, None, None, None) == -1
    assert b"n must be" in lib.kcore_last_error()
    assert lib.kcore_probe_gather(None, -1, None, 0, None, None) == -1
    assert b"probe" in lib.kcore_last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2512_00233_amd as kc
    monkeypatch.setattr(kc, "_lib", None)
    monkeypatch.setattr(kc, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        kc.load()


def test_ctypes_mirrors_match_the_header(tmp_path):
    """Every structure the binding mirrors has the header's size and field offsets (compiled with gcc)."""
    import shutil
    import subprocess
    import paper_2512_00233_amd as kc
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    mirrors = {"kcore_tuning": kc.Tuning, "kcore_stats": kc.Stats, "kcore_kernel_stats": kc.KernelStats,
               "kcore_serve_config": kc.ServeConfig, "kcore_completion": kc.Completion,
               "kcore_serve_report": kc.ServeReport}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "kcore.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
