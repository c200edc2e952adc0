"""The C ABI without a GPU: the built library loads, exports every function
that include/tpkmc.h declares (and no other tpkmc_ symbol), and its
argument-free calls answer.  Nothing here launches a kernel."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpkmc.h")
LIB = os.path.join(ROOT, "paper_1210_8084_amd", "libtpkmc.so")


def declared():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tpkmc_\w+)\s*\(", text, flags=re.M))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libtpkmc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for f in ("tpkmc_version", "tpkmc_strerror", "tpkmc_create", "tpkmc_destroy", "tpkmc_step",
              "tpkmc_step_batched", "tpkmc_run", "tpkmc_autotune", "tpkmc_status", "tpkmc_step_noalloc",
              "tpkmc_tuned_cells", "tpkmc_search_order", "tpkmc_set_search_order"):
        assert f in names


def test_every_declared_function_is_exported(lib):
    names = declared()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line and "tpkmc_" in line}
    assert names == exported, f"declared only: {names - exported}; exported only: {exported - names}"
    for f in names:
        assert getattr(lib, f) is not None


def test_argument_free_calls(lib):
    from paper_1210_8084_amd import tpkmc
    lib.tpkmc_strerror.restype = ctypes.c_char_p
    assert lib.tpkmc_version() == 2
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.tpkmc_strerror(code)
    assert lib.tpkmc_strerror(-99) == b"unknown error code"
    # Null handles are refused before anything touches a device.
    assert lib.tpkmc_destroy(None) == tpkmc.OK
    assert lib.tpkmc_step(None, None, None, None, None, None) == tpkmc.EINVAL
    assert lib.tpkmc_status(None, None) == tpkmc.EINVAL
    assert lib.tpkmc_tuned_cells(None, 0, None) == tpkmc.EINVAL
    assert lib.tpkmc_search_order(None, None) == tpkmc.EINVAL
    assert lib.tpkmc_set_search_order(None, 1) == tpkmc.EINVAL
    assert lib.tpkmc_step_noalloc(0, 0, None, None, None, None, None) == tpkmc.EINVAL
    assert lib.tpkmc_step_noalloc(7, 0, None, None, None, None, None) == tpkmc.EINVAL
