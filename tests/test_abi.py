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


def test_struct_layout_matches_header():
    import ctypes
    # 2 int32 + 6 pointers + 3 doubles + pointer + 6 doubles + 4 int32 +
    # double + int32 (+pad) + double + 2 int32 + pointer
    assert ctypes.sizeof(binding.Desc) == 8 + 48 + 24 + 8 + 48 + 16 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(binding.Report) == 10 * 8 + 7 * 4 + 4 + 8
