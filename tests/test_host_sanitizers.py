"""The library's host code (engine schedule, C ABI, serving threads, sessions, allocators) built for
the CPU under AddressSanitizer and UBSan, with the device backend replaced by a host stand-in
(tests/host/stub_backend.cpp), and driven through the C ABI by tests/host/abi_driver.cpp.  Any
out-of-bounds access, use after free, leak or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "paper_2306_14887_amd", "csrc", "engine.cpp"),
           os.path.join(ROOT, "paper_2306_14887_amd", "csrc", "api.cpp"),
           os.path.join(ROOT, "tests", "host", "stub_backend.cpp"),
           os.path.join(ROOT, "tests", "host", "abi_driver.cpp")]
FLAGS = ["-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-Wall"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(d, os.path.basename(src) + ".o")
            objs.append(obj)
            procs.append(subprocess.Popen(["g++", *FLAGS, "-c", src, "-o", obj],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                          text=True))
        for p, src in zip(procs, SOURCES):
            out = p.communicate(timeout=600)[0]
            assert p.returncode == 0, f"compile {src}:\n{out}"
        exe = os.path.join(d, "abi_driver")
        r = subprocess.run(["g++", "-fsanitize=address,undefined", *objs, "-o", exe, "-lpthread"],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "host ABI checks passed" in r.stdout
