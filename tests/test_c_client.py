"""The C-ABI from C: a C99 program compiled against include/sfhad.h alone
(-std=c99 -Wall -Wextra -Werror -pedantic) and linked to libsfhad.so runs the
host-only entry points and argument checks (no device call)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client(tmp_path):
    from paper_2306_11665_amd import sfhad
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lib = sfhad.LIB_PATH
    assert os.path.exists(lib), "libsfhad.so is not built"
    exe = tmp_path / "client"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_client", "sfhad_c_client.c"), lib,
           "-Wl,-rpath," + os.path.dirname(lib), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"


@pytest.mark.gpu
def test_c_client_on_the_gpu(tmp_path, orc):
    """The same from C on the device: hipMalloc'd buffers and a stream from
    the HIP runtime API, the volume term in FP64 and FP32-split through the
    C-ABI, checked against the oracle's dense definition (liboracle linked by
    this test only)."""
    from paper_2306_11665_amd import sfhad
    import oracle
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lib = sfhad.LIB_PATH
    olib = oracle._LIB
    assert os.path.exists(lib) and os.path.exists(olib)
    exe = tmp_path / "gpu_client"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-D__HIP_PLATFORM_AMD__",
           "-isystem", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_client", "sfhad_c_gpu_client.c"), lib, olib,
           "-L/opt/rocm/lib", "-lamdhip64", "-lm",
           "-Wl,-rpath," + os.path.dirname(lib) + ":" + os.path.dirname(olib) + ":/opt/rocm/lib",
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
