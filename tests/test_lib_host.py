"""Host-side checks of the HIP library that need no GPU: it loads, exports
every entry point include/wcsim.h declares, and validates arguments before
launching anything."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2304_01841_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcsim.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wcsim_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def ws():
    from paper_2304_01841_amd import wcsim
    return wcsim


def test_library_exports_every_declared_symbol(ws):
    names = _declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(ws.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(ws.EXPORTED) == names


def test_version_and_error_string(ws):
    assert ws.version() == 10400
    assert isinstance(ws._lib.wcsim_last_error(), bytes)


def _desc(ws, **over):
    pl = W.plane(10, 100)
    pl.update(over)
    R = W.response("bipolar", Rp=21, Rt=20, r0=10)
    d = ws.PlaneDesc(pl["plane_id"], pl["nwires"], pl["nimpact"], pl["nticks"], pl["pitch"],
                     pl["tick"], pl["t0"], pl["plane_x"], pl["dir_y"], pl["dir_z"],
                     pl["pitch_origin"], 21, 20, over.get("r0", 10), 0,
                     R.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return d, R


@pytest.mark.parametrize("field,value", [("nwires", 0), ("nimpact", 0), ("nticks", -5),
                                         ("pitch", 0.0), ("tick", -1.0), ("dir_z", 0.5),
                                         ("t0", float("nan")), ("r0", 21), ("r0", -1)])
def test_plane_create_rejects_bad_descriptor(ws, field, value):
    d, R = _desc(ws, **{field: value})
    ph = ws.physics_struct(W.physics(False))
    h = ctypes.c_void_p()
    st = ws._lib.wcsim_plane_create(ctypes.byref(d), ctypes.byref(ph), None, ctypes.byref(h))
    assert st == ws.E_INVALID
    assert not h.value
    assert len(ws._lib.wcsim_last_error()) > 0


@pytest.mark.parametrize("field,value", [("drift_speed", 0.0), ("DL", -1.0), ("nsigma", -3.0),
                                         ("fluctuate", 2), ("DT", float("inf")),
                                         ("drift_accel", float("nan"))])
def test_plane_create_rejects_bad_physics(ws, field, value):
    d, R = _desc(ws)
    p = W.physics(False)
    p[field] = value
    ph = ws.physics_struct(p)
    h = ctypes.c_void_p()
    st = ws._lib.wcsim_plane_create(ctypes.byref(d), ctypes.byref(ph), None, ctypes.byref(h))
    assert st == ws.E_INVALID


def test_null_arguments_are_rejected(ws):
    L = ws._lib
    h = ctypes.c_void_p()
    assert L.wcsim_plane_create(None, None, None, ctypes.byref(h)) == ws.E_INVALID
    assert L.wcsim_rasterize(None, None, 0, 0, 0, None, ctypes.byref(h)) == ws.E_STATE
    assert L.wcsim_convolve(None, None, None, 0, None, None) == ws.E_STATE
    assert L.wcsim_simulate_event(None, None, 0, 0, 0, None, 0, 0, None, None) == ws.E_STATE
    assert L.wcsim_scatter_add(None, None, None, 0, None) == ws.E_STATE
    assert L.wcsim_philox4x32_10(None, None, -1, None, None) == ws.E_INVALID
    assert L.wcsim_convolve_workspace_bytes(None, 0) == 0
    L.wcsim_plane_destroy(None)
    L.wcsim_patches_destroy(None)


def test_binding_structs_match_the_header(ws, tmp_path):
    """The ctypes structures of the binding have the C header's sizes and
    field offsets (compiled and printed by the host compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"wcsim_depo": ws.Depo, "wcsim_physics": ws.Physics,
               "wcsim_plane_desc": ws.PlaneDesc, "wcsim_schedule": ws.Schedule,
               "wcsim_plane_info": ws.PlaneInfo}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "wcsim.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[cname + "." + f]) == getattr(py, f).offset, (cname, f)
