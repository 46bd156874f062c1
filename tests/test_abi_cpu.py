"""CPU-only checks of the C-ABI library: it loads, exports every function that
include/wbpr.h declares, and the binding's structs match the header sizes.
No compute call is made (there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2404_00270_amd import wbpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wbpr.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wbpr_[a-z_]+)\s*\(", src)))


def test_library_present_and_exports_every_declared_symbol():
    lib = wbpr.load_library()
    names = header_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(lib, n), f"missing export {n}"
    assert set(names) == set(wbpr.EXPORTS)


def test_version_string():
    assert "gfx950" in wbpr.wbpr_version()


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against include/wbpr.h with gcc and compare sizes/offsets."""
    import subprocess

    probe = tmp_path / "probe.c"
    probe.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "wbpr.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(wbpr_csr), sizeof(wbpr_options), sizeof(wbpr_stats));
  printf("%zu %zu %zu\n", offsetof(wbpr_options, max_sweeps), offsetof(wbpr_options, time_kernels),
         offsetof(wbpr_stats, ms_build));
  printf("%zu %zu\n", offsetof(wbpr_stats, lanes_per_vertex), offsetof(wbpr_stats, kernel_queued));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    sizes = list(map(int, out))
    assert sizes[0:3] == [ctypes.sizeof(wbpr.wbpr_csr), ctypes.sizeof(wbpr.wbpr_options),
                          ctypes.sizeof(wbpr.wbpr_stats)]
    assert sizes[3] == wbpr.wbpr_options.max_sweeps.offset
    assert sizes[4] == wbpr.wbpr_options.time_kernels.offset
    assert sizes[5] == wbpr.wbpr_stats.ms_build.offset
    assert sizes[6] == wbpr.wbpr_stats.lanes_per_vertex.offset
    assert sizes[7] == wbpr.wbpr_stats.kernel_queued.offset


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        wbpr._lib_backup = wbpr._lib
        try:
            wbpr._lib = None
            wbpr.load_library(str(tmp_path / "nope.so"))
        finally:
            wbpr._lib = wbpr._lib_backup


def test_server_struct_layouts_match_header(tmp_path):
    import subprocess

    probe = tmp_path / "probe_srv.c"
    probe.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "wbpr.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(wbpr_server_options), sizeof(wbpr_result), sizeof(wbpr_server_stats));
  printf("%zu %zu %zu %zu\n", offsetof(wbpr_result, value), offsetof(wbpr_result, cut_side),
         offsetof(wbpr_server_stats, p99_ms), offsetof(wbpr_server_stats, peak_resident));
  return 0;
}
""")
    exe = tmp_path / "probe_srv"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    got = list(map(int, subprocess.check_output([str(exe)]).decode().split()))
    assert got == [ctypes.sizeof(wbpr.wbpr_server_options), ctypes.sizeof(wbpr.wbpr_result),
                   ctypes.sizeof(wbpr.wbpr_server_stats), wbpr.wbpr_result.value.offset,
                   wbpr.wbpr_result.cut_side.offset, wbpr.wbpr_server_stats.p99_ms.offset,
                   wbpr.wbpr_server_stats.peak_resident.offset]


def test_admission_footprint_formula():
    """Arena bytes per resident instance: 69 V + 44 E + ceil(E/32) (pure host call)."""
    for V, E in [(2, 0), (1000, 8000), (65536, 524288), (4194304, 65242560)]:
        assert wbpr.wbpr_server_footprint(V, E) == 69 * V + 44 * E + (E + 31) // 32
    # O(V + E): doubling both doubles the footprint up to the rounding term
    a, b = wbpr.wbpr_server_footprint(10_000, 80_000), wbpr.wbpr_server_footprint(20_000, 160_000)
    assert abs(b - 2 * a) <= 1
    with pytest.raises(wbpr.WbprError):
        wbpr.wbpr_server_footprint(-1, 5)
