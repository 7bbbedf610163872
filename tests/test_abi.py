"""CPU checks of the C-ABI library: it loads, exports every function the
public header declares, and rejects bad meshes synchronously (validation runs
before any device call, so no GPU is needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ipibm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_symbols_exported():
    names = declared_functions()
    assert {"ip_forces", "ibm_interp", "ibm_spread", "ip_step"} <= set(names)
    lib = C.CDLL(N.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def _mesh_struct(wl, **over):
    arrs = dict(node_off=np.ascontiguousarray(wl.node_off, np.int64),
                edge_off=np.ascontiguousarray(wl.edge_off, np.int64),
                face_off=np.ascontiguousarray(wl.face_off, np.int64),
                faces=np.ascontiguousarray(wl.faces, np.int32),
                edges4=np.ascontiguousarray(wl.edges4, np.int32),
                closed=np.ascontiguousarray(wl.closed, np.uint8))
    arrs.update(over)
    m = N.ip_mesh(len(arrs["node_off"]) - 1, *(arrs[k].ctypes.data for k in
                  ("node_off", "edge_off", "face_off", "faces", "edges4", "closed")), None)
    return m, arrs


@pytest.mark.parametrize("mutate,needle", [
    ("bad_offset", "node_off"),
    ("edge_out_of_body", "edges4"),
    ("bad_wing", "wing"),
    ("face_repeat", "faces"),
    ("bad_grid", "grid"),
    ("open_edge_in_closed_body", "closed"),
])
def test_invalid_mesh_rejected(mutate, needle):
    wl = W.small_suspension(2, 1, 16)
    over = {}
    grid = N.ip_grid(16, 16, 16, 1.0 / 16)
    if mutate == "bad_offset":
        no = wl.node_off.copy()
        no[1] = no[2] + 1
        over["node_off"] = no
    elif mutate == "edge_out_of_body":
        e4 = wl.edges4.copy()
        e4[0, 1] = wl.node_off[1]          # node of body 1 in an edge of body 0
        over["edges4"] = e4
    elif mutate == "bad_wing":
        e4 = wl.edges4.copy()
        e4[3, 2] = -5
        over["edges4"] = e4
    elif mutate == "face_repeat":
        fa = wl.faces.copy()
        fa[2, 1] = fa[2, 0]
        over["faces"] = fa
    elif mutate == "open_edge_in_closed_body":
        e4 = wl.edges4.copy()
        e4[5, 3] = -1
        over["edges4"] = e4
    elif mutate == "bad_grid":
        grid = N.ip_grid(16, 2, 16, 1.0 / 16)
    m, keep = _mesh_struct(wl, **over)
    h = C.c_void_p()
    code = N.LIB.ip_plan_create(C.byref(h), C.byref(m), C.byref(grid), N.IP_F64)
    assert code == N.IP_ERR_ARG
    assert not h.value
    assert needle in N.LIB.ip_last_error().decode()


def test_null_arguments_rejected():
    assert N.LIB.ip_plan_create(None, None, None, 0) == N.IP_ERR_ARG
    h = C.c_void_p()
    assert N.LIB.ip_plan_create(C.byref(h), None, None, 0) == N.IP_ERR_ARG
    assert N.LIB.ip_forces(None, None, None, None, None, None, None, None, None) == N.IP_ERR_ARG
    assert N.LIB.ip_step(None, None, None, None, None, None, 0.0, None, None, None) == N.IP_ERR_ARG
    assert N.LIB.ip_plan_destroy(None) == N.IP_OK


@pytest.mark.parametrize("opts", [(-1, 0, 0, 0, 0), (0, 8, 0, 0, 0), (0, 0, 1024, 0, 0),
                                  (0, 0, 0, 512, 0), (0, 0, 0, 64, 0), (0, 0, 0, 0, 9),
                                  (0, 0, 0, 0, -1)])
def test_invalid_plan_options_rejected(opts):
    wl = W.small_suspension(2, 1, 16)
    m, keep = _mesh_struct(wl)
    grid = N.ip_grid(16, 16, 16, 1.0 / 16)
    h = C.c_void_p()
    o = N.ip_plan_options(*opts)
    code = N.LIB.ip_plan_create_ex(C.byref(h), C.byref(m), C.byref(grid), N.IP_F64, C.byref(o))
    assert code == N.IP_ERR_ARG and not h.value
    assert "options" in N.LIB.ip_last_error().decode()
