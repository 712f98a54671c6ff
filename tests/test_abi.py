"""C-ABI boundary checks that need no GPU: the library loads, exports every
entry point include/mirres.h declares, and rejects bad arguments with status
codes before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mirres.h")
LIB = os.path.join(ROOT, "paper_2406_16360_amd", "libmirres.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mrs_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2406_16360_amd.csrc import build
        build.build()
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_symbol():
    from paper_2406_16360_amd import mirres
    assert sorted(mirres.EXPORTS) == _declared()


def test_invalid_arguments_return_status(lib):
    lib.mrs_last_error.restype = C.c_char_p
    lib.mrs_build_bvh.restype = C.c_int32
    lib.mrs_build_bvh.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    out = C.c_void_p()
    assert lib.mrs_build_bvh(None, 3, None, 1, None, C.byref(out)) == -1
    assert b"null" in lib.mrs_last_error()
    assert out.value is None
    assert lib.mrs_build_bvh(None, 3, None, 1, None, None) == -1
    lib.mrs_render.restype = C.c_int32
    assert lib.mrs_render(None, None, 0, None, None, None, None) == -1
    assert lib.mrs_render_backward(None, None, 0, None, None, None, None, None) == -1
    lib.mrs_trace.restype = C.c_int32
    assert lib.mrs_trace(None, None, None, C.c_int64(0), 0, None, None) == -1
    lib.mrs_bvh_info.restype = C.c_int32
    assert lib.mrs_bvh_info(None, None, None, None) == -1


def test_tape_bytes_arithmetic():
    from paper_2406_16360_amd import mirres, synth
    w = synth.config1()
    o = mirres.RenderOptions.from_any(w.opts)
    # 64 * 64 pixels * 4 spp * 2 bounces * 36 bytes per vertex record
    assert mirres.tape_bytes(w.views, o) == 64 * 64 * 4 * 2 * 36


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the C structs have the C sizes and field offsets
    (the header compiled by gcc is the reference)."""
    import shutil
    import subprocess
    from paper_2406_16360_amd import mirres
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"mrs_scene": mirres._Scene, "mrs_view": mirres._View, "mrs_options": mirres._Options,
               "mrs_grads": mirres._Grads, "mrs_denoise_params": mirres._DenoiseParams}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
