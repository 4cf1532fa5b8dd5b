"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (CPU only).

* The oracle built with -fsanitize=address,undefined runs its pin suites.
* The library's host code (descriptor validation, layout, tile lists, the
  server's scheduler in dry-run mode, argument checks) built with host-only
  sanitizers (hipcc: -Xarch_host before each -fsanitize=; device code is
  untouched) runs the ABI and dry-run server tests.

Each run is a child Python process with the sanitizer runtime preloaded, leak
checks off (the interpreter's own allocations are not ours) and every report
fatal, so a finding fails the test with its report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _run(args, env, tmp_path):
    log = tmp_path / "san"
    env = dict(env)
    env["ASAN_OPTIONS"] = env.get("ASAN_OPTIONS", "") + f":log_path={log}"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *args], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    reports = ""
    for f in tmp_path.glob("san*"):
        reports += f.read_text()[:4000]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:], reports)
    assert not reports, reports


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import oracle as O
    O.build(force=True, sanitize=True)
    _run(["tests/test_oracle_pins.py", "tests/test_oracle_ns.py", "tests/test_oracle_solutions.py"],
         O.sanitize_env(), tmp_path)


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2305_18057_amd import build as B
    lib = str(tmp_path / "libfv_san.so")
    B.build(extra=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"],
            out=lib, build_dir=str(tmp_path / "build"))
    # the ASan runtime of the clang that hipcc drives
    clang = os.path.join(os.path.dirname(os.path.realpath(B.hipcc())), "..", "llvm", "bin", "clang")
    rt = subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                 text=True).strip()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["FV_LIBRARY"] = lib
    _run(["tests/test_server_logic.py", "tests/test_abi.py"], env, tmp_path)
