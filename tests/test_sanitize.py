"""The host converter under AddressSanitizer and UndefinedBehaviorSanitizer: a fuzz driver built with
g++ from the converter's source (host code only, no GPU) converts a few hundred random matrices and
checks their round trip."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_converter_fuzz_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "convert_fuzz")
    src = os.path.join(ROOT, "paper_2605_18515_amd", "csrc")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", src,
             os.path.join(HERE, "sanitize", "convert_fuzz.cpp"), os.path.join(src, "convert.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "400"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "failures 0" in r.stdout


def test_range_span_limit_is_enforced(tmp_path):
    """A work range whose payload would not fit the streaming kernel's 32-bit offsets is refused with
    CB_ERROR_INVALID_VALUE (checked against a small limit; the real one is 2 GiB)."""
    if not shutil.which("g++"):
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "range_span")
    src = os.path.join(ROOT, "paper_2605_18515_amd", "csrc")
    build = ["g++", "-std=c++17", "-O1", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", src,
             os.path.join(HERE, "sanitize", "range_span.cpp"), os.path.join(src, "convert.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
