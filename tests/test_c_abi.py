"""The boundary used from C: a C program built against include/cbspmv.h and linked to the library
prints its struct layouts (compared with the Python binding's ctypes mirrors) and converts a small
matrix on the host and exports it back (no GPU)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2605_18515_amd import cbspmv as cb

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MIRRORS = {"cb_options_t": cb.CbOptions, "cb_info_t": cb.CbInfo, "cb_structure_t": cb.CbStructure,
           "cb_cg_options_t": cb.CbCgOptions, "cb_cg_result_t": cb.CbCgResult,
           "cb_server_options_t": cb.CbServerOptions, "cb_request_t": cb.CbRequest, "cb_response_t": cb.CbResponse,
           "cb_server_stats_t": cb.CbServerStats, "cb_tune_options_t": cb.CbTuneOptions,
           "cb_tune_candidate_t": cb.CbTuneCandidate, "cb_tune_report_t": cb.CbTuneReport}
RENAMED = {("cb_request_t", "in"): "in_"}


@pytest.fixture(scope="module")
def c_output(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("gcc is not available")
    exe = str(tmp_path_factory.mktemp("abi") / "abi_check")
    libdir = os.path.dirname(cb.LIB_PATH)
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "c_abi", "abi_check.c"), "-L", libdir, "-lcbspmv",
                    f"-Wl,-rpath,{libdir}", "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.splitlines()


def test_struct_layouts_match_the_binding(c_output):
    checked = 0
    for line in c_output:
        name, _, val = line.partition(" ")
        if name not in MIRRORS and "." not in name:
            continue
        if "." in name:
            t, f = name.split(".")
            assert getattr(MIRRORS[t], RENAMED.get((t, f), f)).offset == int(val), name
        else:
            assert ctypes.sizeof(MIRRORS[name]) == int(val), name
        checked += 1
    assert checked >= 40


def test_host_conversion_from_c(c_output):
    line = next(l for l in c_output if l.startswith("tiles"))
    assert "roundtrip ok" in line and "on_device 0" in line and "nnz 6" in line
    bad = next(l for l in c_output if l.startswith("bad row_ptr"))
    assert f"status {cb.CB_ERROR_INVALID_VALUE}" in bad and bad.endswith("set")


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the binding next to no built library refuses to import (there is no fallback path)."""
    import importlib.util
    import shutil as sh

    src = os.path.join(ROOT, "paper_2605_18515_amd", "cbspmv.py")
    pkg = tmp_path / "pkg"
    pkg.mkdir()
    sh.copy(src, pkg / "cbspmv.py")
    spec = importlib.util.spec_from_file_location("cbspmv_copy", str(pkg / "cbspmv.py"))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="libcbspmv.so is missing"):
        spec.loader.exec_module(mod)
