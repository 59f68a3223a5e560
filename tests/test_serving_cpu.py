"""The serving scheduler's admission policy on the host, with no device.

``paper_2404_06359_amd/csrc/admission.h`` holds the server's arena, first-come
first-served queue, batch formation, completion and cancellation logic, free
of HIP calls; the server's scheduler thread drives it and adds the streams
and launches.  ``tests/native/admission_test.cpp`` drives it with a fake
executor (batches finish when and how the test says: in any slot order, or
failed) and checks admission order, head-of-line blocking, slot reuse, batch
limits, error propagation, release and cancel rules, the arena allocator, and
a randomized run against a plain model.  It is built with g++ twice: plain,
and with AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "admission_test.cpp")
INC = [f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(ROOT, 'paper_2404_06359_amd', 'csrc')}"]


def _asan_available():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    return r.returncode == 0 and os.path.isabs(r.stdout.strip()) and os.path.exists(r.stdout.strip())


@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan-ubsan"])
def test_admission_policy(tmp_path, sanitize):
    if sanitize and not _asan_available():
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    exe = tmp_path / "admission_test"
    flags = ["-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror"]
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    subprocess.run(["g++", *flags, *INC, SRC, "-o", str(exe)], check=True)
    # (other preloaded libraries stay; the runtime need not come first)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checks passed" in r.stdout
