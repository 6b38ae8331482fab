"""CPU-side checks of the C ABI: the library loads and exports every symbol
the header declares (no compute calls: there is no GPU here)."""
import os
import re

import pytest

from paper_1705_10845_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xlbomd.h")).read()
    return sorted(set(re.findall(r"\b(xlbomd_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("xlbomd_init_system", "xlbomd_step", "xlbomd_kernel_update",
              "xlbomd_forces"):
        assert n in names
    assert set(names) == set(binding.EXPORTED)


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH),
                    reason="library not built")
def test_library_exports_every_declared_symbol():
    L = binding.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert L.xlbomd_version().startswith(b"xlbomd")


def test_struct_layout_matches_header(tmp_path):
    """Every field offset and the size of the descriptor, the report and the
    allocator struct, from a C program compiled against the header, equal
    the ctypes layouts the binding passes."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = (("xlbomd_desc", binding.Desc), ("xlbomd_report", binding.Report),
               ("xlbomd_allocator", binding.Allocator))
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "xlbomd.h"',
             "int main(void) {"]
    for cname, py in structs:
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for cname, py in structs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
