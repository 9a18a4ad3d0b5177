"""CPU: the oracle and the library's host-side validation under AddressSanitizer
and UndefinedBehaviorSanitizer.

Two C drivers walk the code paths: ``oracle_sanitize.c`` runs every oracle
entry point (both algorithms, both deflation forms, every start mode, both
stop rules, the three Gram-Schmidt forms, replay, degenerate and non-finite
inputs, codecs, the network and Adam); ``abi_sanitize.c`` runs the C ABI's
validation of sizes, pointers, options and workspaces, which answers without
a GPU.  Each is built with the sanitizers and must exit 0 with no report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
ORACLE = [os.path.join(ROOT, "oracle", f) for f in ("pca_oracle.c", "codec_oracle.c",
                                                       "mlp_oracle.c")]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe, env):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "runtime error" not in report and "AddressSanitizer" not in report, report


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-O1", "-g", *SAN, "-fno-fast-math", "-ffp-contract=off", "-std=c99", "-Wall",
           "-o", exe, os.path.join(HERE, "oracle_sanitize.c"), *ORACLE, "-lm"]
    subprocess.run(cmd, check=True, timeout=300)
    _run(exe, ENV)


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def test_host_validation_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    clang = "/opt/rocm/llvm/bin/clang"
    if hipcc is None or not os.path.exists(clang):
        pytest.skip("ROCm toolchain not available")
    csrc = os.path.join(ROOT, "paper_0811_1081_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    lib = str(tmp_path / "libgspca_hostsan.so")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    # sanitizers on the host pass only: every -fsanitize= follows -Xarch_host
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared", *host_san,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + inc, "-I" + csrc, "-o", lib, *srcs]
    subprocess.run(cmd, check=True, timeout=900, capture_output=True)
    exe = str(tmp_path / "abi_san")
    subprocess.run([clang, "-O1", "-g", *SAN, "-I" + inc, "-o", exe,
                    os.path.join(HERE, "abi_sanitize.c"), lib, "-Wl,-rpath," + str(tmp_path)],
                   check=True, timeout=300)
    # the HIP runtime keeps allocations for the process lifetime: no leak check
    _run(exe, dict(ENV, ASAN_OPTIONS="detect_leaks=0"))
