"""Sanitizer builds of the host code (CPU only): the C oracle linked with a
driver under AddressSanitizer + UndefinedBehaviorSanitizer, and the routing
helpers of the HIP runtime's header compiled for the host with the same
sanitizers, each run on its own inputs with every sanitizer report fatal."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-Wall", "-pthread",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_sanitize.c"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


def test_host_routing_helpers_under_asan_ubsan(tmp_path):
    """The same commands as the plain host-logic build, every output equal."""
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2205_07610_amd", "csrc")]
    src = os.path.join(HERE, "host_logic.hip")
    plain, san = str(tmp_path / "plain"), str(tmp_path / "san")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", *inc, src, "-o", plain])
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all", *inc, src, "-o", san])
    cmds = ["c"]
    for m in (1, 7, 150, 1000, 5000, 20000):
        for n in (m, m + 3, m + 900):
            for a, b in ((5, 2), (11, 1), (3, 3)):
                cmds.append(f"w {m} {n} {-m} 2 {a} {b}")
                cmds.append(f"r {m} {n} 320 2 {b} {a} {b}")
                cmds.append(f"p {m} {n} {m // 7} 2 {b} {a} {b}")
    cmds += [f"f {v}" for v in range(17)]
    text = "\n".join(cmds) + "\n"
    want = subprocess.run([plain], input=text, capture_output=True, text=True, check=True).stdout
    r = subprocess.run([san], input=text, capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stderr[-4000:])
    assert r.stdout == want
