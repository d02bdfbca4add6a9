"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the library's sources are compiled with the sanitizers on their host
side only (device code as usual) and linked with tests/host/
library_host_checks.cpp, which drives every host path that needs no GPU;
the oracle is compiled with tests/host/oracle_checks.c and run on small
inputs.  A sanitizer report or a failed check fails the test."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1602_02620_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# each sanitizer flag is put right after -Xarch_host: host code only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-4000:]}\n{p.stderr[-4000:]}"
    return p


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_1602_02620_amd import build as B

    def comp(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN,
              "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])
        return obj

    srcs = [os.path.join(CSRC, s) for s in B.SOURCES] + [os.path.join(HOST, "library_host_checks.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    exe = str(tmp_path / "library_host_checks")
    _run([HIPCC, "--offload-arch=gfx950", *SAN, *objs, "-o", exe])
    p = _run([exe], env=ENV, timeout=600)
    assert "library host checks passed" in p.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-Wall", "-Wextra", "-Werror",
          os.path.join(HOST, "oracle_checks.c"), os.path.join(ROOT, "oracle", "fclsh_oracle.c"), "-o", exe])
    p = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"), timeout=600)
    assert "oracle checks passed" in p.stdout
