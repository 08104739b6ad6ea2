"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code) and run on small seeded inputs through every entry point,
including the degenerate sizes (k = 1, k = n - 1, self-inclusive k = n) and
exact distance ties: no out-of-bounds access, leak or undefined behaviour.
And the request server's host logic (admission, swapping, coalescing, graph
bookkeeping, request parts, latency statistics) built with ThreadSanitizer,
and with AddressSanitizer and UndefinedBehaviorSanitizer (leaks included),
against a host-only stand-in for the HIP runtime and a fake prediction, driven
by several client threads: no data race, every served row correct."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "fmg_oracle.c"),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr
    assert "all calls clean" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_server_host_logic_under_sanitizers(tmp_path, sanitizer):
    # The server source is host code; it is copied to a .cpp file and built
    # for the host only, against tests/sanitize/fake_hip.
    src = tmp_path / "fmg_server_host.cpp"
    shutil.copyfile(os.path.join(ROOT, "paper_2205_10879_amd", "csrc", "fmg_server.hip"), src)
    san = os.path.join(ROOT, "tests", "sanitize")
    exe = str(tmp_path / "server_sanitized")
    flags = ["-fsanitize=" + sanitizer]
    if sanitizer == "thread":
        flags += ["-include", os.path.join(san, "tsan_compat.h")]
    else:
        flags += ["-fno-sanitize-recover=all"]
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + flags +
           ["-I", os.path.join(san, "fake_hip"), "-I", os.path.join(ROOT, "include"),
            "-I", os.path.join(ROOT, "paper_2205_10879_amd", "csrc"),
            str(src), os.path.join(san, "server_fake_runtime.cpp"),
            os.path.join(san, "server_driver.cpp"), "-lpthread", "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "server runs clean" in r.stdout
