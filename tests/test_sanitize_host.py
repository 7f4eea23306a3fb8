"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The CPU oracle (oracle/oracle.c), the seeded input generators
(gen/spmvgen.c) and the host-only part of the library
(paper_2407_00019_amd/csrc/host_core.cpp: the server's offset allocator,
D_mat from the row moments, the auto-tuner's decision) are compiled with
both sanitizers by the plain host compiler and driven by
tests/sanitize/host_check.cpp; a sanitizer report or a failed check fails
the test.  No GPU code is involved.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _have(tool):
    return shutil.which(tool) is not None


@pytest.mark.skipif(not (_have("gcc") and _have("g++")), reason="no host C/C++ compiler")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    objs = []

    def cc(compiler, src, extra):
        out = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([compiler, *SAN, *extra, "-c", os.path.join(ROOT, src), "-o", out], check=True)
        objs.append(out)

    # the oracle keeps its own floating-point flags; the generators build
    # without OpenMP here (their draws do not depend on the thread count)
    cc("gcc", "oracle/oracle.c", ["-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-Wall"])
    cc("gcc", "gen/spmvgen.c", ["-std=gnu11", "-Wall", "-Wno-unknown-pragmas"])
    cc("g++", "paper_2407_00019_amd/csrc/host_core.cpp", ["-std=c++17", "-Wall", "-Wextra"])
    cc("g++", "tests/sanitize/host_check.cpp", ["-std=c++17", "-Wall"])
    exe = str(tmp_path / "host_check")
    subprocess.run(["g++", *SAN, *objs, "-o", exe, "-lm"], check=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-4000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ok:" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
