"""C ABI contract checks that need no GPU: the library loads, exports every
function ``include/hough_hier.h`` declares, and rejects bad arguments before
touching a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hough_hier.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"HH_API\s+[\w\s\*]+?\b(hough_hier_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("hough_hier_create", "hough_hier_destroy", "hough_hier_detect", "hough_hier_detect_batch",
              "hough_hier_result_cells", "hough_hier_result_members", "hough_hier_result_stats",
              "hough_hier_result_info", "hough_hier_result_free", "hough_hier_last_error",
              "hough_hier_serve_start", "hough_hier_submit", "hough_hier_poll", "hough_hier_solution",
              "hough_hier_result_solution"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1007_0547_amd as hh
    lib = hh.library()
    for n in declared_functions():
        assert hasattr(lib, n), n
    # nothing else with the prefix is exported by accident
    out = subprocess.run(["nm", "-D", "--defined-only", hh.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted(set(re.findall(r"\b(hough_hier_\w+)\b", out)))
    assert exported == declared_functions()


def header_sizes(tmp_path):
    """sizeof of the ABI structs as the C compiler lays them out from the header."""
    src = tmp_path / "sizes.c"
    names = ["hh_config", "hh_input", "hh_solution", "hh_cell", "hh_level_stats", "hh_launch",
             "hh_result_info", "hh_timing", "hh_serve_config", "hh_serve_stats"]
    src.write_text('#include <stdio.h>\n#include "hough_hier.h"\nint main(void) {\n' +
                   "".join(f'printf("{n} %zu\\n", sizeof({n}));\n' for n in names) + "return 0; }\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.splitlines())}


def test_struct_layouts_match_header(tmp_path):
    import paper_1007_0547_amd as hh
    sz = header_sizes(tmp_path)
    assert C.sizeof(hh._Config) == sz["hh_config"]
    assert C.sizeof(hh._Input) == sz["hh_input"]
    assert C.sizeof(hh._Solution) == sz["hh_solution"]
    assert C.sizeof(hh._Launch) == sz["hh_launch"]
    assert C.sizeof(hh._Info) == sz["hh_result_info"]
    assert C.sizeof(hh._Timing) == sz["hh_timing"]
    assert C.sizeof(hh._ServeConfig) == sz["hh_serve_config"]
    assert C.sizeof(hh._ServeStats) == sz["hh_serve_stats"]
    assert hh.CELL_DTYPE.itemsize == sz["hh_cell"]
    assert hh.STATS_DTYPE.itemsize == sz["hh_level_stats"]


def test_null_arguments_and_bad_config():
    import paper_1007_0547_amd as hh
    lib = hh.library()
    h = C.c_void_p()
    assert lib.hough_hier_create(None, C.byref(h)) == -1
    cfg = hh._Config()
    assert lib.hough_hier_create(C.byref(cfg), None) == -1
    for field, bad in (("threshold", -1), ("max_depth", 16), ("max_depth", -2), ("variant", 2),
                       ("passes", 4), ("membership", 2), ("arena_limit_mib", -1)):
        cfg = hh._Config()
        setattr(cfg, field, bad)
        assert lib.hough_hier_create(C.byref(cfg), C.byref(h)) == -1, field
    lib.hough_hier_destroy(None)
    assert lib.hough_hier_last_error(None) == b""
    assert lib.hough_hier_detect(None, None, None) == -1
    assert lib.hough_hier_detect_batch(None, None, 0, None) == -1
    assert lib.hough_hier_serve_start(None, None) == -1
    t, out = C.c_uint64(), C.c_void_p()
    assert lib.hough_hier_submit(None, None, C.byref(t)) == -1
    assert lib.hough_hier_poll(None, 1, 0, C.byref(out)) == -1
    p, n = C.c_void_p(), C.c_int64()
    assert lib.hough_hier_result_cells(None, 0, 0, C.byref(p), C.byref(n)) == -1
    assert lib.hough_hier_result_members(None, 0, C.byref(p), C.byref(n)) == -1
    n32 = C.c_int32()
    assert lib.hough_hier_result_stats(None, 0, C.byref(p), C.byref(n32)) == -1
    assert lib.hough_hier_result_info(None, None) == -1
    lib.hough_hier_result_free(None)


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1007_0547_amd as hh
    with pytest.raises(hh.HHError) as e:
        hh.HoughHier(threshold=1)
    assert e.value.status == -4


def test_solution_null_arguments():
    """hough_hier_solution and its accessor reject null arguments and bad
    passes without a device; an empty list is a no-op."""
    import paper_1007_0547_amd as hh
    lib = hh.library()
    ms = C.c_double(-1.0)
    assert lib.hough_hier_solution(None, 1, C.byref(ms)) == -1
    assert lib.hough_hier_solution(None, -1, None) == -1
    assert lib.hough_hier_solution(None, 0, C.byref(ms)) == 0 and ms.value == 0.0
    arr = (C.c_void_p * 2)(None, None)
    assert lib.hough_hier_solution(arr, 2, None) == -1
    out = hh._Solution()
    assert lib.hough_hier_result_solution(None, 0, 0, C.byref(out)) == -1
    assert lib.hough_hier_result_solution(None, 0, 0, None) == -1
    assert lib.hough_hier_result_solution_image(None, None, 0, 0) == -1
