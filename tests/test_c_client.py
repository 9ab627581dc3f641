"""The library from a C program: tests/c_client.c includes only include/tprec.h and the
HIP runtime header, is compiled with gcc and linked against libtprec.so."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    from paper_0910_0992_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtprec.so missing: build with __graft_entry__.build()")
    exe = str(tmp_path_factory.mktemp("c") / "c_client")
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_client.c"), "-o", exe,
           "-L", libdir, "-ltprec", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath," + libdir, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_client_host_checks(client):
    r = subprocess.run([client, "--host-checks"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks ok" in r.stdout


@pytest.mark.gpu
def test_c_client_solve(client):
    r = subprocess.run([client], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "solve ok" in r.stdout


@pytest.mark.gpu
def test_c_client_allocator(client):
    r = subprocess.run([client, "--allocator"], capture_output=True, text=True, timeout=180)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "allocator ok" in r.stdout
