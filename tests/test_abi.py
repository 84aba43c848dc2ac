"""Host-side checks of the C ABI (no GPU): the library loads and exports every function the
public header declares, the header's structs have the layout the binding marshals, and the
pure-host helper behaves."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "voldor.h")
LIB = os.path.join(ROOT, "paper_2104_06800_amd", "_lib", "libvoldor.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(voldor_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2104_06800_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    from paper_2104_06800_amd import binding
    assert binding.EXPORTS == names


def test_struct_layout_matches_header(tmp_path):
    from paper_2104_06800_amd import binding
    prog = tmp_path / "sz.c"
    prog.write_text('#include "voldor.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(voldor_window), sizeof(voldor_buffers),'
                    ' sizeof(voldor_align_params), offsetof(voldor_window, seed), offsetof(voldor_window, window_id));'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sw, sb, sa, oseed, owid = map(int, out)
    assert sw == ctypes.sizeof(binding.Window)
    assert sb == ctypes.sizeof(binding.Buffers)
    assert sa == ctypes.sizeof(binding.AlignParams)
    assert oseed == binding.Window.seed.offset and owid == binding.Window.window_id.offset


def test_lattice_shape_host_helper(lib):
    hc, wc = ctypes.c_int32(), ctypes.c_int32()
    f = lib.voldor_lattice_shape
    assert f(352, 1216, 4, ctypes.byref(hc), ctypes.byref(wc)) == 0 and (hc.value, wc.value) == (88, 304)
    assert f(48, 64, 4, ctypes.byref(hc), ctypes.byref(wc)) == 0 and (hc.value, wc.value) == (12, 16)
    assert f(7, 9, 3, ctypes.byref(hc), ctypes.byref(wc)) == 0 and (hc.value, wc.value) == (2, 3)
    assert f(10, 10, 1, ctypes.byref(hc), ctypes.byref(wc)) == 0 and (hc.value, wc.value) == (10, 10)
    assert f(10, 10, 0, ctypes.byref(hc), ctypes.byref(wc)) == 1
    from oracle import gem
    for H, W, s in [(352, 1216, 4), (48, 64, 4), (7, 9, 3), (37, 70, 4), (10, 10, 1), (13, 5, 8)]:
        assert f(H, W, s, ctypes.byref(hc), ctypes.byref(wc)) == 0
        assert (hc.value, wc.value) == gem.lattice_shape(H, W, s)


def test_null_context_is_rejected(lib):
    lib.voldor_gem_step.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_void_p]
    assert lib.voldor_gem_step(None, None, None, 0, None) == 1
    lib.voldor_align_p2p.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 8
    assert lib.voldor_align_p2p(None, None, 1, *([None] * 8)) == 1
