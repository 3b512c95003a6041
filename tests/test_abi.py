"""Host-only checks of the C-ABI library: it loads and exports every symbol
the public header declares (no compute calls without a GPU)."""
import os
import re
import subprocess

from paper_2501_05244_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "nursd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nursd_[a-z_0-9]+)\s*\(", src)))


def test_library_loads_and_exports_header_symbols():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)
    assert set(names) == set(_lib.SIGNATURES)


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against the header with the system C compiler and
    compare every field offset and struct size with the ctypes mirror."""
    import ctypes
    structs = {"nursd_wavelet": _lib.Wavelet, "nursd_geometry": _lib.Geometry,
               "nursd_options": _lib.Options, "nursd_plan_info_t": _lib.PlanInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nursd.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_last_error_is_a_string():
    assert isinstance(_lib.load().nursd_last_error(), bytes)


def test_missing_library_fails_loudly():
    """Without the built library the package raises instead of falling back
    to any CPU path (checked in a fresh interpreter)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2501_05244_amd import _lib\n"
            "_lib.LIB_PATH = '/nonexistent/libnursd.so'\n"
            "try:\n"
            "    _lib.load()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(1)\n") % ROOT
    r = subprocess.run(["python3", "-c", code], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "is missing" in r.stdout
