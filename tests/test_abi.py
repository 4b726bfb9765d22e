"""The C-ABI library loads and exports every function include/pic.h
declares (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")
LIB = os.path.join(ROOT, "paper_2606_05893_amd", "libpic.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(pic_\w+|poisson_solve)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared()
    for req in ("pic_init", "pic_inject", "pic_step", "poisson_solve",
                "pic_workspace_bytes", "pic_destroy"):
        assert req in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libpic.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.pic_abi_version.restype = ctypes.c_int32
    hdr = open(os.path.join(ROOT, "include", "pic.h")).read()
    ver = int(re.search(r"#define PIC_ABI_VERSION (\d+)", hdr).group(1))
    assert lib.pic_abi_version() == ver


def test_workspace_size_and_validation_on_host():
    """pic_workspace_bytes runs on the host only: sizes grow with capacity,
    invalid configurations are rejected."""
    if not os.path.exists(LIB):
        pytest.skip("libpic.so not built")
    import sys
    sys.path.insert(0, ROOT)
    from paper_2606_05893_amd import pic as G
    import workloads as W
    lib = G.load_library()
    p = W.config("c1")
    sizes = []
    for cap in (1000, 100000):
        c = G.make_config(p, capacity=(cap,) * 3)
        n = ctypes.c_size_t()
        assert lib.pic_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == 0
        sizes.append(n.value)
    assert sizes[1] > sizes[0] + 3 * 99000 * 2 * 56
    bad = G.make_config(dict(p, bc_lo=1, bc_hi=1))
    n = ctypes.c_size_t()
    assert lib.pic_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    odd = G.make_config(dict(p, nx=33))
    assert lib.pic_workspace_bytes(ctypes.byref(odd), ctypes.byref(n)) == -1
    tol = G.make_config(p, rel_tol=0.0)
    assert lib.pic_workspace_bytes(ctypes.byref(tol), ctypes.byref(n)) == -1
    # Cell groups: the three capacities together within 32-bit index words.
    ok = G.make_config(p, capacity=(0xFFFFFFF0 - 2, 1, 1), flags=G.FLAG_CELL_GROUPS)
    assert lib.pic_workspace_bytes(ctypes.byref(ok), ctypes.byref(n)) == 0
    big = G.make_config(p, capacity=(0xFFFFFFF0 - 1, 1, 1), flags=G.FLAG_CELL_GROUPS)
    assert lib.pic_workspace_bytes(ctypes.byref(big), ctypes.byref(n)) == -1
    free = G.make_config(p, capacity=(0xFFFFFFF0 - 1, 1, 1))
    assert lib.pic_workspace_bytes(ctypes.byref(free), ctypes.byref(n)) == 0
