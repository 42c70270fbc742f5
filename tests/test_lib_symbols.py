"""The C-ABI library loads and exports every function include/midbf.h declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "midbf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(midbf_\w+|phase_recover)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("midbf_build", "midbf_apply", "midbf_apply_adjoint"):
        assert must in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_1908_09376_amd", "libmidbf.so")
    assert os.path.exists(path), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1908_09376_amd import _lib
    assert set(declared_functions()) <= set(_lib.EXPORTED)


def test_error_path_without_gpu_work():
    # a null handle is rejected on the host, before any device call
    from paper_1908_09376_amd import _lib
    st = _lib.lib.midbf_apply(None, None, None, 1, 16, 0, None)
    assert st == -1 and b"null" in _lib.lib.midbf_last_error()


def test_output_block_checked_before_launch():
    # the binding rejects an output of the wrong dtype or on the host before calling the library
    import pytest
    import torch
    from paper_1908_09376_amd.midbf import MIDBF
    F = object.__new__(MIDBF)
    F.N = 16
    x = torch.zeros(16, dtype=torch.complex64)
    with pytest.raises(TypeError):
        F._out(x, torch.zeros(16, dtype=torch.complex128))
    with pytest.raises(TypeError):
        F._out(x, torch.zeros(16, dtype=torch.complex64))      # not a CUDA tensor


def test_factor_file_errors_without_gpu_work(tmp_path):
    # a missing file, a file that is not a factor file and a truncated header are refused on the
    # host, before any device call
    import ctypes as C
    from paper_1908_09376_amd import _lib
    h = C.c_void_p()
    st = _lib.lib.midbf_load(str(tmp_path / "absent.midbf").encode(), 0, None, None, C.byref(h))
    assert st == -8 and not h.value
    bad = tmp_path / "bad.midbf"
    bad.write_bytes(b"NOTMIDBF" + bytes(64))
    assert _lib.lib.midbf_load(str(bad).encode(), 0, None, None, C.byref(h)) == -8
    assert b"not a MIDBF factor file" in _lib.lib.midbf_last_error()
    short = tmp_path / "short.midbf"
    short.write_bytes(b"MIDBFf1\n" + bytes(8))
    assert _lib.lib.midbf_load(str(short).encode(), 0, None, None, C.byref(h)) == -8
    assert b"truncated" in _lib.lib.midbf_last_error()
    assert _lib.lib.midbf_save(None, b"x", None) == -1


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets that a C compiler gives the
    header's struct of the same role (a field added on one side only would shift the others)."""
    import shutil
    import subprocess
    from paper_1908_09376_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        import pytest
        pytest.skip("no C compiler")
    pairs = [(_lib.Params, "midbf_params"), (_lib.Stats, "midbf_stats"), (_lib.KernelTime, "midbf_kernel_time"),
             (_lib.BatchStats, "midbf_batch_stats"), (_lib.RecoverInfo, "phase_recover_info")]
    lines = ['#include "midbf.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    want = []
    for cls, cname in pairs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f[0]}));')
            want.append(getattr(cls, f[0]).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want
