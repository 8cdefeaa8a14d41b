"""The C-ABI library loads, exports every function declared in include/heatbem.h, and its
host-only mesh check agrees with the oracle's pair classification (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from synthetic import cube, icosphere, octahedron, tetrahedron

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heatbem.h")
LIB = os.path.join(ROOT, "paper_2102_09811_amd", "libheatbem.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def hb():
    if not os.path.exists(LIB):
        pytest.fail("libheatbem.so is not built (run __graft_entry__.build())")
    from paper_2102_09811_amd import binding
    return binding


def test_exports_every_declared_symbol(hb):
    L = ctypes.CDLL(LIB)
    names = declared_functions()
    assert "hb_create" in names and "hb_assemble" in names and len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert sorted(hb.EXPORTED) == names, (set(hb.EXPORTED) ^ set(names))


@pytest.mark.parametrize("mesh", ["cube", "icosphere", "octahedron", "tetrahedron"])
def test_check_mesh_class_counts_match_oracle(hb, mesh):
    v, t = {"cube": cube(3), "icosphere": icosphere(1), "octahedron": octahedron(),
            "tetrahedron": tetrahedron()}[mesh]
    rc, counts, msg = hb.check_mesh(v, t)
    assert rc == 0, msg
    ref = np.zeros(4, dtype=np.int64)
    for a in range(len(t)):
        for b in range(len(t)):
            ref[oracle.pair_points(v, t, a, b, 1)["cls"]] += 1
    assert np.array_equal(counts, ref)


def test_check_mesh_rejects_bad_meshes(hb):
    v, t = cube(2)
    assert hb.check_mesh(v, t[::-1, ::-1].copy())[0] == hb.HB_EORIENT       # all flipped
    tt = t.copy()
    tt[0] = tt[0, ::-1]
    assert hb.check_mesh(v, tt)[0] == hb.HB_EORIENT                         # one flipped
    assert hb.check_mesh(v, t[:-1])[0] == hb.HB_EMESH                       # open surface
    tt = t.copy()
    tt[3, 1] = tt[3, 0]
    assert hb.check_mesh(v, tt)[0] == hb.HB_EMESH                           # repeated vertex
    vv = np.vstack([v, v[:1]])
    tt = t.copy()
    tt[tt == 0] = len(v)                                                     # coincident vertices
    assert hb.check_mesh(vv, np.vstack([tt]))[0] == hb.HB_EMESH
    tt = t.copy()
    tt[0, 0] = len(v) + 5
    assert hb.check_mesh(v, tt)[0] == hb.HB_EMESH                           # index out of range
    assert hb.check_mesh(v[:3], t[:2])[0] == hb.HB_EMESH                    # too small
