"""The C-ABI library loads and exports every entry point the public header
declares; host-only queries work without a GPU."""
import os
import re

import pytest

import paper_1506_03265_amd as cd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cldiam.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cldiam_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cd.LIB_PATH):
        from paper_1506_03265_amd import build
        build.build()
    return cd.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    assert names == sorted(cd.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.cldiam_strerror(cd.CLDIAM_OK) == b"ok"
    assert b"overflow" in lib.cldiam_strerror(cd.CLDIAM_EOVERFLOW)
    assert b"gfx950" in lib.cldiam_version()


def test_workspace_queries_are_monotone(lib):
    small = lib.cldiam_decompose_workspace_size(1000, 1)
    big = lib.cldiam_decompose_workspace_size(10**7, 1)
    assert 0 < small < big
    assert lib.cldiam_decompose_workspace_size(0, 1) == 0
    assert lib.cldiam_decompose_workspace_size(1000, 256) > small
    assert lib.cldiam_load_csr_workspace_size(100, 400) > 0
    assert lib.cldiam_quotient_workspace_size(100, 400) > 0
    assert lib.cldiam_estimate_workspace_size(10, 20) > 0
    assert lib.cldiam_sssp_workspace_size(100, 400) > 0


def test_invalid_arguments_fail_before_touching_a_device(lib):
    # no graphs at all: rejected by host validation
    assert lib.cldiam_decompose_batch(0, None, None, 0, None, None, 0, None) == cd.CLDIAM_EINVAL
    assert b"num_graphs" in lib.cldiam_last_error()
    # null quotient outputs
    assert lib.cldiam_build_quotient(0, 0, None, None, None, None, None, None, None, None, None, None, None, 0,
                                     None) == cd.CLDIAM_EINVAL
    assert lib.cldiam_sssp_delta_stepping(10, 0, None, None, 0, 1, None, None, None, 0, None) == cd.CLDIAM_EINVAL


def test_sssp_accepts_the_default_width_marker(lib):
    """bucket_delta = 0 selects the library's default width; it is not an
    argument error (an invalid source still is)."""
    assert lib.cldiam_sssp_delta_stepping(10, 0, None, None, 0, 0, None, None, None, 0, None) == cd.CLDIAM_EINVAL
    assert b"bucket" not in lib.cldiam_last_error()


def test_noalloc_estimate_rejects_k_above_its_maximum_before_device_work(lib):
    import ctypes
    phi, approx = ctypes.c_uint64(), ctypes.c_uint64()
    fake = ctypes.c_void_p(256)   # never dereferenced: the size check comes first
    rc = lib.cldiam_estimate_diameter_noalloc(cd.CLDIAM_NOALLOC_MAX_K + 1, 0, fake, None, None, 0,
                                              ctypes.byref(phi), ctypes.byref(approx), None)
    assert rc == cd.CLDIAM_EINVAL
    assert b"maximum" in lib.cldiam_last_error()


def test_pinned_host_bytes_is_a_pool_of_whole_buffers(lib):
    b = lib.cldiam_pinned_host_bytes()
    assert b >= 0 and b % 4096 == 0


def test_python_structures_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structures have the C compiler's
    sizes and field offsets (a plain C program including cldiam.h prints them)."""
    import ctypes
    import subprocess
    fields = {
        "cldiam_csr": (cd._Csr, ["n", "m", "d_row_ptr", "d_col", "d_w"]),
        "cldiam_params": (cd._Params, ["tau", "delta0", "seed", "variant", "step_cap"]),
        "cldiam_tuning": (cd._Tuning, ["local_rounds", "grid_blocks", "bucket_width", "row_bucket_shift",
                                        "chunk_factor", "wave_row_min", "group_row_min", "local_queue",
                                        "local_cutoff", "pull_mode"]),
        "cldiam_graph": (cd._Graph, ["m", "d_arcs", "weight_sum", "params", "d_cluster", "d_D"]),
        "cldiam_stats": (cd._Stats, ["stages", "radius", "arcs_scanned", "status", "kernel_ms", "iterations",
                                     "rounds", "messages", "updates", "radius1", "stage_uncovered",
                                     "stage_delta"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cldiam.h"', "int main(void) {"]
    for cname, (_, names) in fields.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in names or []:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        parts = line.split()
        got[(parts[0], parts[1])] = int(parts[2])
    for cname, (py, names) in fields.items():
        assert ctypes.sizeof(py) == got[(cname, "size")], cname
        for f in names or []:
            assert getattr(py, f).offset == got[(cname, f)], (cname, f)


def test_c_example_builds_against_the_header(tmp_path):
    """The plain-C example that drives the whole path through the ABI
    (ingest, decomposition, quotient, estimate) compiles and links with gcc."""
    import shutil
    import subprocess
    rocm = "/opt/rocm"
    lib_dir = os.path.join(ROOT, "paper_1506_03265_amd")
    if not os.path.exists(os.path.join(lib_dir, "libcldiam.so")) or not os.path.exists(rocm) or not shutil.which("gcc"):
        pytest.skip("needs libcldiam.so, ROCm headers and gcc")
    exe = tmp_path / "diameter"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
                           os.path.join(lib_dir, "examples", "diameter.c"), "-o", str(exe),
                           "-L", lib_dir, "-lcldiam", "-L", os.path.join(rocm, "lib"), "-lamdhip64"])
    assert exe.exists()
