"""C-ABI library checks that need no GPU: it loads, exports every function
that include/scan.h declares, and its host-side integer eps threshold agrees
with the oracle's exact 128-bit test.  Checks that load the library run in a
child interpreter (abi_probe.py)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
HEADER = os.path.join(ROOT, "include", "scan.h")
LIB = os.path.join(ROOT, "paper_2311_12281_amd", "libscan_mi355x.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(scan_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def probe(*args):
    return subprocess.run([sys.executable, os.path.join(HERE, "abi_probe.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (scan_[a-z_0-9]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    r = probe("symbols", *names)
    assert r.returncode == 0, r.stdout + r.stderr


def test_library_holds_gfx950_code_only(tmp_path):
    fb = tmp_path / "fatbin.bin"
    r = subprocess.run(["objcopy", f"--dump-section=.hip_fatbin={fb}", LIB], capture_output=True)
    if r.returncode != 0:
        pytest.skip("objcopy cannot read the fat binary section")
    out = subprocess.run(["/opt/rocm/llvm/bin/clang-offload-bundler", "--list", "--type=o",
                          f"--input={fb}"], capture_output=True, text=True, check=True)
    targets = [t for t in out.stdout.split() if "amdgcn" in t]
    assert targets and all(t.endswith("gfx950") for t in targets), out.stdout


def test_eps_threshold_matches_exact_test():
    r = probe("threshold")
    assert r.returncode == 0, r.stdout + r.stderr


def test_fails_loudly_without_device():
    r = probe("nodevice")
    if r.returncode == 4:
        pytest.skip("a GPU is present")
    assert r.returncode == 0, r.stdout + r.stderr


def test_binding_never_imports_the_oracle_or_torch():
    src = open(os.path.join(ROOT, "paper_2311_12281_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    assert "import torch" not in src


def test_binding_structs_match_header(tmp_path):
    """The ctypes mirrors of the public structs have the header's size and
    field offsets (gcc compiles a probe of the header; no library is loaded)."""
    import ctypes
    sys.path.insert(0, ROOT)
    import paper_2311_12281_amd as S
    structs = {"scan_opts": S.scan_opts, "scan_stats": S.scan_stats, "scan_batch": S.scan_batch}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "scan.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
    # and the same fields, in the same order, as the header declares
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for name, cls in structs.items():
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S).group(1)
        fields = re.findall(r"([A-Za-z_][A-Za-z_0-9]*)\s*(?:\[[^\]]*\])?\s*;", body)
        assert fields == [f for f, _ in cls._fields_], (name, fields)
