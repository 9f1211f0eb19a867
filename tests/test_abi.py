"""The C-ABI library: it loads without a GPU, exports every function that
include/wmc.h declares, and shares torch's HIP runtime."""
import os
import re
import subprocess
import sys

import pytest

import paper_2006_15512_amd as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wmc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = "\n".join(ln for ln in src.splitlines() if not ln.lstrip().startswith("#"))
    src = src.replace('extern "C" {', " ").replace("}", "};")
    # return type, name, '(' -- at statement start, excluding typedefs
    names = set()
    for stmt in src.split(";"):
        stmt = " ".join(stmt.split())
        if stmt.startswith("typedef") or "(" not in stmt:
            continue
        m = re.match(r"^(?:const )?[A-Za-z_][A-Za-z0-9_]* ?\*? ?(wmc_[a-z0-9_]+)\(", stmt)
        if m:
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("wmc_build_network", "wmc_plan", "wmc_contract", "wmc_serve", "wmc_batch_contract",
                 "wmc_last_error"):
        assert must in names
    assert len(names) >= 28


def test_library_exports_every_declared_function():
    L = W.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert missing == []
    out = subprocess.run(["nm", "-D", "--defined-only", W.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {ln.split()[-1] for ln in out.stdout.splitlines() if " T " in ln}
    assert set(declared_functions()) <= exported


def test_binding_names_match_header():
    """Every symbol the Python binding types is declared in the header."""
    W.lib()
    declared = set(declared_functions())
    src = open(os.path.join(ROOT, "paper_2006_15512_amd", "__init__.py")).read()
    typed = set(re.findall(r'"(wmc_[a-z0-9_]+)":', src))
    assert typed and typed <= declared


def test_one_hip_runtime_in_process():
    """Loading the library binds it to the HIP runtime torch already carries
    (same soname), never a second copy."""
    code = ("import sys, re; sys.path.insert(0, %r); import paper_2006_15512_amd as W; W.lib(); "
            "m = open('/proc/self/maps').read(); "
            "print(len(set(re.findall(r'\\S*libamdhip64\\S*', m))))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_version_and_error_string():
    assert W.version()
    with pytest.raises(W.WmcError) as e:
        W.Network(2, [[1, 3]], [[0.5, 0.5], [0.5, 0.5]])  # literal beyond n_vars
    assert e.value.status == 1
    assert "wmc_build_network" in str(e.value) or str(e.value)
