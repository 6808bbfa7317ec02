"""Host-side checks that need no GPU: the library loads and exports what the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lens_api.h")
LIB = os.path.join(ROOT, "paper_2503_08586_amd", "liblens_mi355x.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:lens_status|void|const char \*)\s*\**\s*(lens_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lens_init", "lens_shutdown", "lens_load_data", "lens_unload", "lens_loglike_batch",
                 "lens_loglike_batch_device", "lens_loglike_multi", "lens_submit", "lens_poll",
                 "lens_wait", "lens_cancel", "lens_model_image", "lens_strerror", "lens_last_error"):
        assert must in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2503_08586_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2503_08586_amd import binding
    assert sorted(binding.EXPORTED) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(binding, name))


def test_peak_kinds_match_header():
    # binding.PEAK_OPS[i] names LENS_PEAK_<NAME> = i, and LENS_PEAK_COUNT ends the list
    from paper_2503_08586_amd import binding
    text = open(HEADER).read()
    vals = {m.group(1).lower(): int(m.group(2))
            for m in re.finditer(r"^#define LENS_PEAK_(\w+)\s+(\d+)", text, flags=re.M)}
    assert vals.pop("count") == len(binding.PEAK_OPS)
    assert vals == {name: i for i, name in enumerate(binding.PEAK_OPS)}


def test_strerror_without_device(lib):
    lib.lens_strerror.restype = ctypes.c_char_p
    lib.lens_strerror.argtypes = [ctypes.c_int32]
    assert lib.lens_strerror(0) == b"ok"
    assert lib.lens_strerror(-1) == b"invalid argument"
    assert lib.lens_strerror(12345) == b"unknown status"


def test_struct_layouts_match_header():
    # the ctypes mirrors of the ABI structs must have the C sizes (x86-64 SysV)
    from paper_2503_08586_amd import binding
    assert ctypes.sizeof(binding.lens_init_opts) == 4 + 4 + 8 + 4 + 4 + 8 * 4 + 8
    assert ctypes.sizeof(binding.lens_data_desc) == 4 + 4 + 8 + 4 + 4 + 8 * 4 + 4 + 4 + 8 + 4 + 4 + 8 * 4 + 4 + 4
    assert ctypes.sizeof(binding.lens_info) == 5 * 4 + 4 + 8 * 4 + 2 * 4 + 8 + 6 * 4
    assert ctypes.sizeof(binding.lens_stats) == 15 * 8


def test_struct_offsets_match_compiled_header(tmp_path):
    # every field of the ctypes mirrors sits at the offset a C compiler gives it
    import shutil
    import subprocess
    from paper_2503_08586_amd import binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [binding.lens_init_opts, binding.lens_data_desc, binding.lens_info, binding.lens_stats,
               binding.lens_ensemble_desc]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lens_api.h"', "int main(void) {"]
    expect = []
    for st in structs:
        name = st.__name__
        lines.append('printf("%%zu\\n", sizeof(%s));' % name)
        expect.append(ctypes.sizeof(st))
        for f, _ in st._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (name, f))
            expect.append(getattr(st, f).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_no_cpu_fallback_in_product_path():
    # the package must never import the oracle
    pkg = os.path.join(ROOT, "paper_2503_08586_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "lens_oracle" not in src, f
