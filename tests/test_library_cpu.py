"""CPU-side checks of the C ABI: the built library loads, exports every entry
point include/bal.h declares, and the ctypes structures match the C layout.
No GPU call is made."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bal.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bal_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    from paper_2407_00046_amd import bal
    out = subprocess.run(["nm", "-D", "--defined-only", bal.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (bal_[a-z_]+)", out))
    names = declared()
    assert len(names) >= 19
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(bal.EXPORTED) == names


def test_status_strings():
    from paper_2407_00046_amd import bal
    assert bal.bal_status_string(0) == b"ok"
    assert b"zero distance" in bal.bal_status_string(-4)
    assert bal.bal_status_string(-99) == b"unknown status"


def test_ctypes_layout_matches_c():
    """Every field of the three ABI structures sits at the C offset, and the
    sizes agree."""
    import ctypes
    from paper_2407_00046_amd import bal
    fields = "\n".join(f"  P({T}, {f[0]});" for T in ("bal_scene_desc", "bal_step_stats", "bal_al_state")
                       for f in getattr(bal, T)._fields_)
    probe = r"""
#include <stdio.h>
#include <stddef.h>
#include "bal.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("bal_scene_desc %zu\n", sizeof(bal_scene_desc));
  printf("bal_step_stats %zu\n", sizeof(bal_step_stats));
  printf("bal_al_state %zu\n", sizeof(bal_al_state));
""" + fields + r"""
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(probe)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.split() for l in lines if l.strip())
    assert int(got["bal_scene_desc"]) == ctypes.sizeof(bal.bal_scene_desc)
    assert int(got["bal_step_stats"]) == ctypes.sizeof(bal.bal_step_stats)
    assert int(got["bal_al_state"]) == ctypes.sizeof(bal.bal_al_state)
    for key, v in got.items():
        if "." in key:
            T, f = key.split(".")
            assert getattr(getattr(bal, T), f).offset == int(v), key


def test_no_cpu_fallback_in_product_path():
    """The package imports only the HIP library; nothing under it touches the oracle."""
    pkg = os.path.join(ROOT, "paper_2407_00046_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits
    before touching a device."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout + r.stderr
