"""CPU checks of the C-ABI library: it loads and exports every entry point include/pmg.h declares.
(No compute call: there is no GPU here.)"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmg.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("pmg_residual", "pmg_vcycle", "pmg_tau_estimate", "pmg_solve", "pmg_restrict", "pmg_prolong",
              "pmg_smooth", "pmg_timestep", "pmg_solver_create", "pmg_mesh_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1806_11456_amd import pmg
    if not os.path.exists(pmg.LIB_PATH):
        from paper_1806_11456_amd import build
        build.build()
    lib = ctypes.CDLL(pmg.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pmg.EXPORTS) == declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1806_11456_amd import pmg
    monkeypatch.setattr(pmg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pmg, "_lib", None)
    with pytest.raises(RuntimeError):
        pmg.lib()


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: asked for more it exits with status 2 and says so, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_struct_layouts_match_the_header(tmp_path):
    """Every parameter struct the binding passes by pointer has the header's size and field offsets: a C program
    compiled against include/pmg.h prints them, the ctypes mirrors must agree field by field."""
    import ctypes
    import os
    import shutil
    import subprocess

    from paper_1806_11456_amd import pmg

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    mirrors = {"pmg_physics": pmg.Physics, "pmg_mg_params": pmg.MGParams, "pmg_adapt_params": pmg.AdaptParams,
               "pmg_multistage_params": pmg.MultistageParams, "pmg_stage_report": pmg.StageReport}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pmg.h"', "int main(void) {"]
    for cname, mirror in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in mirror._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            name, key, val = ln.split()
            got[(name, key)] = int(val)
    for cname, mirror in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(mirror), cname
        for field, _ in mirror._fields_:
            assert got[(cname, field)] == getattr(mirror, field).offset, (cname, field)
