"""The C ABI from plain C: tests/c/abi_host.c compiles as strict C99 against include/tamm_mi.h
(-std=c99 -pedantic -Wall -Wextra -Werror), links the built library and runs its host-only checks
(spaces, tensors, a plan and its statistics, error codes, the one-shot cache's host half)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2201_01257_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_abi_from_c99(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libtamm_mi.so")):
        pytest.fail("libtamm_mi.so is not built (run __graft_entry__.build())")
    exe = str(tmp_path / "abi_host")
    subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                    "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_host.c"),
                    "-L" + LIBDIR, "-ltamm_mi", "-Wl,-rpath," + LIBDIR, "-o", exe], check=True)
    env = dict(os.environ)
    rocm_lib = "/opt/rocm/lib"
    env["LD_LIBRARY_PATH"] = rocm_lib + (":" + env["LD_LIBRARY_PATH"] if env.get("LD_LIBRARY_PATH") else "")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout
