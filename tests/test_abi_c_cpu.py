"""The C ABI from plain C99 (``tests/native/abi_host_test.c``): host calls
only -- encode, validate, plan a batch, convert to plain GTS, write and read
a .gtsr file, and the error paths' status codes and messages -- built with
gcc against the library, as a C caller would."""
import os
import subprocess

import pytest

import paper_2404_06359_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_from_c(tmp_path):
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libgtsr.so is not built")
    exe = tmp_path / "abi_host_test"
    libdir = os.path.dirname(P.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
                    os.path.join(ROOT, "tests", "native", "abi_host_test.c"), "-o", str(exe),
                    f"-L{libdir}", f"-l:{os.path.basename(P.LIB_PATH)}", f"-Wl,-rpath,{libdir}",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    r = subprocess.run([str(exe), str(tmp_path / "two.gtsr")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checks passed" in r.stdout
    assert P.load(str(tmp_path / "two.gtsr"))[1].format == P.FORMAT_GTS
