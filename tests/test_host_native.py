"""Host builds of native code, no GPU: (1) the univariate setup (setup1d.cpp)
under the address and undefined-behaviour sanitizers, driven through every
degree, jittered and repeated knots, the threaded eigenvector update and the
error paths; (2) the audit of the reduction grids: at the workload sizes
(the 128^3 ring, the p = 5 and p = 4 warped cubes, the 64-problem batch, the
2D square, the L-shaped grid, the 513^3 cube) no kernel shape the library can
select writes more block partials than its partial-sum buffer holds -- the
regression test of an overrun of that buffer by an A-product shape with a
larger grid than the vector kernels'."""
import os
import shutil
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1602_01636_amd", "csrc")
INC = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-3000:]
    return res


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_setup1d_under_sanitizers(tmp_path):
    exe = str(tmp_path / "setup1d_asan")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *INC,
          os.path.join(ROOT, "tests", "host", "setup1d_asan.cpp"), os.path.join(CSRC, "setup1d.cpp"),
          "-o", exe, "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = _run([exe], env=env)
    assert res.stdout.strip().endswith("OK")


def _sizes():
    lines = []
    for E, p in ((128, 3), (96, 5), (112, 4)):
        n = E + p - 2
        lines.append(f"3 {p} {n} {n} {n}")
    for pr in synth.batch_problems(seed=4):
        p = pr["degree"]
        n = [len(k) - p - 3 for k in pr["knots"]]
        lines.append(f"3 {p} {n[0]} {n[1]} {n[2]}")
    lines += ["2 3 65 65 1", "2 3 2051 2051 1", "3 3 513 513 513", "3 1 2 2 2", "3 6 7 160 9"]
    return "\n".join(lines) + "\n"


def test_reduction_grids_fit_the_partial_buffer(tmp_path):
    lib = os.path.join(ROOT, "paper_1602_01636_amd", "libigafd.so")
    if not os.path.exists(lib):
        pytest.skip("libigafd.so not built")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("needs hipcc")
    exe = str(tmp_path / "partials_audit")
    _run([hipcc, "-std=c++17", "-O1", *INC, os.path.join(ROOT, "tests", "host", "partials_audit.cpp"), "-o", exe,
          "-L" + os.path.dirname(lib), "-ligafd", "-Wl,-rpath," + os.path.dirname(lib)])
    res = _run([exe], input=_sizes())
    last = res.stdout.strip().splitlines()[-1]
    assert last.startswith("OK") and int(last.split()[1]) > 4000, res.stdout[-2000:]
