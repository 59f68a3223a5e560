"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds sanitized copies of the library's host C++ (encoder, validator,
planner, quantizer, cones, tuner, server; the HIP translation units keep
their normal build), of the oracle's C and of the mesh generator's C, then
runs every other CPU test against them in a child process with the
sanitizer runtime preloaded.  Any invalid access or undefined behaviour
aborts the child.  A planted heap overflow first shows that the toolchain
catches one."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    return path


def _env(asan):
    env = dict(os.environ)
    # the sanitizer runtime goes first; libraries already preloaded stay after it
    preload = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env.update({
        "LD_PRELOAD": preload,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "GTSR_LIBRARY": os.path.join(ROOT, "_build", "sanitize", "libgtsr.so"),
        "ORACLE_LIBRARY": os.path.join(ROOT, "_build", "sanitize", "liboracle.so"),
        "MESHGEN_LIBRARY": os.path.join(ROOT, "_build", "sanitize", "libmeshgen.so"),
    })
    return env


def test_toolchain_catches_a_planted_overflow(tmp_path):
    asan = _asan_runtime()
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\nint main(void){ volatile char* p = malloc(8); p[8] = 1; "
                   "free((void*)p); return 0; }\n")
    exe = tmp_path / "overflow"
    subprocess.run(["gcc", "-fsanitize=address", "-g", str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env={"ASAN_OPTIONS": "detect_leaks=0"})
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
    del asan


@pytest.mark.timeout(600)
def test_cpu_suite_under_sanitizers():
    asan = _asan_runtime()
    import meshgen
    import oracle
    from paper_2404_06359_amd import build as b

    b.build_sanitized()
    oracle.build_sanitized()
    meshgen.build_sanitized()
    env = _env(asan)
    probe = textwrap.dedent("""
        import meshgen, oracle, paper_2404_06359_amd as P
        P.lib(); oracle.lib(); meshgen._clib()
        maps = open("/proc/self/maps").read()
        for name in ("sanitize/libgtsr.so", "sanitize/liboracle.so", "sanitize/libmeshgen.so", "libasan"):
            assert name in maps, name
        print("sanitized libraries loaded")
    """)
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    cmd = [sys.executable, "-m", "pytest", "tests", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           "--ignore", os.path.join("tests", os.path.basename(__file__))]
    try:
        import xdist  # noqa: F401
        cmd += ["-n", "4"]
    except ImportError:
        pass
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
