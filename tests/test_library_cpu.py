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


STRUCTS = {"mfs_mesh_desc": "MeshDesc", "mfs_solve_opts": "SolveOpts", "mfs_solve_stats": "SolveStats",
           "mfs_character_info": "CharacterInfo", "mfs_tuning": "Tuning", "mfs_profile": "Profile",
           "mfs_server_opts": "ServerOpts", "mfs_request_times": "RequestTimes",
           "mfs_server_info": "ServerInfo"}


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror has the size and field offsets that gcc gives the
    header's declarations."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mfs.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append(f'  printf("{pyname} size %zu\\n", sizeof({cname}));')
        for field, _ in getattr(mfs, pyname)._fields_:
            lines.append(f'  printf("{pyname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        pyname, field, value = line.split()
        cls = getattr(mfs, pyname)
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), f"{pyname}.{field}: ctypes {got}, C {value}"
        seen += 1
    assert seen == sum(len(getattr(mfs, p)._fields_) + 1 for p in STRUCTS.values())


def test_missing_library_and_missing_gpu_fail_loudly():
    """No CPU fallback: without the built library a call into it raises
    MfsUnavailable, and with it but without a GPU a context cannot be
    created (an exception, never a context).  Each case runs in a fresh
    interpreter."""
    import subprocess
    import sys
    code_missing = (
        "import paper_2408_04066_amd as m\n"
        "m.LIB_PATH = '/nonexistent/libmfs.so'\n"
        "try:\n"
        "    m.default_opts()\n"
        "except m.MfsUnavailable:\n"
        "    print('unavailable')\n")
    r = subprocess.run([sys.executable, "-c", code_missing], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.stdout.strip() == "unavailable", r.stderr
    code_nogpu = (
        "import os\n"
        "os.environ['HIP_VISIBLE_DEVICES'] = ''\n"
        "import paper_2408_04066_amd as m\n"
        "try:\n"
        "    m.Context(0)\n"
        "    print('created')\n"
        "except Exception as e:\n"
        "    print('error', type(e).__name__)\n")
    r = subprocess.run([sys.executable, "-c", code_nogpu], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.stdout.startswith("error"), (r.stdout, r.stderr)


def _fp(T, n, n_pins=3):
    import numpy as np
    T = np.asarray(T, dtype=np.int32)
    prob = {"X": np.zeros((n, 3)), "T": T, "pin_vertex": np.arange(n_pins)}
    return mfs.mesh_footprint(prob)


def test_footprint_from_descriptor_on_the_host():
    """mfs_character_footprint reads only the tets and sizes (host arrays, no
    GPU work): the matrix has one block per vertex and two per distinct
    edge, 8 resident bytes per block (column index and slot pointer), and a
    pin costs 4 resident bytes."""
    # three tets on six vertices: around one face (12 distinct edges) or in a
    # ring (15 distinct edges); the same n, m and pins
    fan = [(0, 1, 2, 3), (0, 1, 2, 4), (0, 1, 2, 5)]
    ring = [(0, 1, 2, 3), (2, 3, 4, 5), (0, 1, 4, 5)]
    r_fan, w_fan = _fp(fan, 6)
    r_ring, w_ring = _fp(ring, 6)
    assert r_ring - r_fan == 8 * 2 * (15 - 12)
    assert w_ring >= w_fan
    assert _fp(ring, 6, n_pins=4)[0] - r_ring == 4
    for T, n in (([(0, 1, 2, 6)], 6), ([(0, 1, 1, 2)], 4), ([(0, 1, 2, 3)], 5)):
        with pytest.raises(mfs.MfsError) as e:
            _fp(T, n)
        assert e.value.code == -1
