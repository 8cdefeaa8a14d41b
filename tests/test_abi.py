"""The C-ABI library loads, exports every function declared in include/heatbem.h, and its
host-only mesh check agrees with the oracle's pair classification; network files that are missing,
short or inconsistent are rejected before any device call (no GPU needed)."""
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


def test_network_file_errors(hb, tmp_path):
    """hb_pcnet_load checks the file before it touches the device: missing, wrong magic, wrong
    dims, truncated and overlong files are HB_EINVAL with a message."""
    import struct
    L = hb.lib()
    h = ctypes.c_void_p()
    assert L.hb_pcnet_load(os.fsencode(str(tmp_path / "absent.bin")), ctypes.byref(h)) == hb.HB_EINVAL
    assert b"cannot open" in L.hb_last_error(None)
    F, H, O = hb.HB_PC_FEATURES, 8, hb.HB_PC_SLOTS
    n = H * F + H + H * H + H + O * H + O
    good = b"HBPCNET1" + struct.pack("<3iq", F, H, O, n) + b"\0" * (4 * n)
    cases = {"magic": b"HBPCNET2" + good[8:], "dims": b"HBPCNET1" + struct.pack("<3iq", F + 1, H, O, n),
             "count": b"HBPCNET1" + struct.pack("<3iq", F, H, O, n + 1) + b"\0" * (4 * n + 4),
             "short": good[:-4], "long": good + b"\0"}
    for name, data in cases.items():
        f = tmp_path / (name + ".bin")
        f.write_bytes(data)
        assert L.hb_pcnet_load(os.fsencode(str(f)), ctypes.byref(h)) == hb.HB_EINVAL, name
        assert b"not a complete network file" in L.hb_last_error(None), name
    o = hb.TrainOpts()
    L.hb_default_train_opts(ctypes.byref(o))
    assert (o.epochs, o.batch, o.n_hidden, o.seed) == (30, 2048, 256, 0) and abs(o.lr - 1e-3) < 1e-9
    assert L.hb_precond_train(None, 0, None, ctypes.byref(h), None, None) == hb.HB_EINVAL
