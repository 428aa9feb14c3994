"""Host-side checks of the C-ABI library that need no GPU."""

import ctypes
import os
import re

import pytest

import paper_2408_04066_amd as mfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfs_[a-z_]+)\s*\(", text)))


def test_library_built_and_exports_every_declared_symbol():
    if not os.path.exists(mfs.LIB_PATH):
        pytest.fail("libmfs.so is not built (run __graft_entry__.build())")
    names = declared_functions()
    assert len(names) >= 13
    L = ctypes.CDLL(mfs.LIB_PATH)
    for name in names:
        assert hasattr(L, name), f"{name} declared in mfs.h but not exported"
    assert set(names) == set(mfs.EXPORTED)


def test_host_only_calls():
    o = mfs.default_opts()
    assert o.precision == mfs.FP64 and o.max_newton == 50 and o.cg_tol == 1e-10
    assert o.step_tol == 1e-10 and o.cg_max == 20000 and o.warm_start == mfs.WARM_REST
    assert mfs.lib().mfs_status_string(-2).decode() == "degenerate rest element"
    assert mfs.lib().mfs_status_string(1).decode().startswith("not converged")
    with pytest.raises(TypeError):
        mfs.default_opts(no_such_option=1)


def test_struct_layouts_match_header():
    # offsets implied by the C declarations (natural alignment, LP64)
    assert ctypes.sizeof(mfs.MeshDesc) == 112
    assert mfs.MeshDesc.pin_stiffness.offset == 96
    assert ctypes.sizeof(mfs.SolveOpts) == 56
    assert mfs.SolveOpts.step_tol.offset == 16 and mfs.SolveOpts.cg_max.offset == 32
    assert ctypes.sizeof(mfs.SolveStats) == 64
    assert mfs.SolveStats.energy.offset == 32
