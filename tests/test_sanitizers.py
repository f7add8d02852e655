"""Host code under the address and undefined-behaviour sanitizers (gcc/g++,
CPU only): the oracle (every entry point on small systems), the bin packing
of the register-resident kernel and the C-ABI's argument validation and
workspace layout. Any invalid access or undefined operation aborts the
driver, which fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_15269_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not found")


def _run(exe, inp=None):
    r = subprocess.run([exe], input=inp, capture_output=True, text=True,
                       env=ENV, timeout=120)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", *SAN, "-std=c99",
                    os.path.join(ROOT, "oracle", "oracle.c"),
                    os.path.join(ROOT, "tests", "oracle_driver.c"), "-lm",
                    "-o", exe], check=True)
    assert "oracle driver ok" in _run(exe)


def test_validation_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "validate_driver")
    subprocess.run(["g++", *SAN, "-std=c++17", "-I", CSRC, "-I",
                    os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "validate_driver.cpp"),
                    "-o", exe], check=True)
    assert "validate driver ok" in _run(exe)


def test_bin_packing_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "pack_driver")
    subprocess.run(["g++", *SAN, "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "pack_driver.cpp"), "-o", exe],
                   check=True)
    import numpy as np
    rng = np.random.default_rng(7)
    for lens, rpw, cap, maxper, slots in (
            (rng.integers(16, 257, 2048), 16, 256, 64, 256),
            (rng.integers(1, 9, 500), 16, 256, 64, 512),
            (np.full(100, 256), 16, 256, 64, 256),
            (np.array([1]), 64, 64, 1, 1)):
        inp = f"{len(lens)} {rpw} {cap} {maxper} {slots}\n" + \
            " ".join(str(int(x)) for x in lens) + "\n"
        _run(exe, inp)
