"""The C ABI: the library loads and exports every symbol the header declares;
the Python structs match the header's layout.  CPU only (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcloak.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1012_5107_amd import binding as B
    L = B.load()
    names = _declared_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    from paper_1012_5107_amd import binding as B
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gcloak.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gc_scene),'
                   ' sizeof(gc_camera), sizeof(gc_opts), sizeof(gc_stats), offsetof(gc_camera, seed),'
                   ' offsetof(gc_opts, max_steps), sizeof(gc_tune), sizeof(gc_autotune_opts),'
                   ' sizeof(gc_autotune_cand), sizeof(gc_autotune_report), offsetof(gc_autotune_report, tune));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(B.Scene), ctypes.sizeof(B.Camera), ctypes.sizeof(B.Opts), ctypes.sizeof(B.Stats),
            B.Camera.seed.offset, B.Opts.max_steps.offset, ctypes.sizeof(B.Tune), ctypes.sizeof(B.AutotuneOpts),
            ctypes.sizeof(B.AutotuneCand), ctypes.sizeof(B.AutotuneReport), B.AutotuneReport.tune.offset]
    assert got == want


def test_default_opts():
    from paper_1012_5107_amd import binding as B
    o = B.Opts()
    B.load().gc_default_opts(ctypes.byref(o))
    assert (o.prec, o.integ, o.h, o.rtol, o.max_events, o.max_steps) == (0, 0, 1e-3, 1e-8, 32, 100_000)
