"""Host-side checks of the C ABI (CPU): the library loads, exports every
symbol that include/mpdc.h declares, rejects invalid meshes and derives the
tables of valid ones with the host-only mpdc_mesh_check (no device access)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mpdc():
    import paper_2404_08849_amd.mpdc as m
    return m


def test_every_declared_symbol_is_exported(mpdc):
    hdr = open(os.path.join(ROOT, "include", "mpdc.h")).read()
    names = set(re.findall(r"\b(mpdc_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(mpdc.lib, n), n


def test_strerror_and_version(mpdc):
    assert mpdc.lib.mpdc_strerror(-2) == b"invalid mesh"
    assert mpdc.lib.mpdc_version().startswith(b"mpdc")


def _create(mpdc, mesh):
    g = mpdc.Mesh.__new__(mpdc.Mesh)
    desc_mesh = dict(mesh)
    keep = {}
    for k in ["cells_on_edge", "vertices_on_edge", "eoc_offset", "edges_on_cell", "vertices_on_cell",
              "cells_on_vertex", "edges_on_vertex"]:
        keep[k] = np.ascontiguousarray(desc_mesh[k], dtype=np.int32)
    for k in ["xCell", "xVertex", "xEdge", "dEdge", "lEdge", "areaCell", "areaVertex", "kiteArea", "fVertex"]:
        keep[k] = np.ascontiguousarray(desc_mesh[k], dtype=np.float64)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d = mpdc.MeshDesc(mesh["nCells"], mesh["nEdges"], mesh["nVertices"],
                      *[ip(keep[k]) for k in ["cells_on_edge", "vertices_on_edge", "eoc_offset", "edges_on_cell",
                                              "vertices_on_cell", "cells_on_vertex", "edges_on_vertex"]],
                      *[dp(keep[k]) for k in ["xCell", "xVertex", "xEdge", "dEdge", "lEdge", "areaCell",
                                              "areaVertex", "kiteArea", "fVertex"]], float(mesh["radius"]))
    # the host-only check runs the same validation and table derivation as
    # mpdc_mesh_create, without touching any device
    rc = mpdc.lib.mpdc_mesh_check(ctypes.byref(d))
    return rc, mpdc.lib.mpdc_last_error().decode(), None


def _broken(mesh_cache, what):
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in mesh_cache(2).items()}
    if what == "index":
        m["cells_on_edge"][5, 1] = m["nCells"] + 3
    elif what == "orientation":
        off = m["eoc_offset"]
        i = 17
        m["edges_on_cell"][off[i]:off[i + 1]] = m["edges_on_cell"][off[i]:off[i + 1]][::-1].copy()
        m["vertices_on_cell"][off[i]:off[i + 1]] = m["vertices_on_cell"][off[i]:off[i + 1]][::-1].copy()
    elif what == "duplicate":
        off = m["eoc_offset"]
        m["edges_on_cell"][off[3] + 1] = m["edges_on_cell"][off[3]]
    elif what == "area":
        m["areaCell"][9] = -1.0
    elif what == "euler":
        m["nVertices"] = m["nVertices"] - 1
    elif what == "tangent":
        m["vertices_on_edge"][11] = m["vertices_on_edge"][11][::-1].copy()
    return m


@pytest.mark.parametrize("what", ["index", "orientation", "duplicate", "area", "euler", "tangent"])
def test_invalid_mesh_rejected_on_host(mpdc, mesh_cache, what):
    rc, msg, _ = _create(mpdc, _broken(mesh_cache, what))
    assert rc == -2, (what, rc, msg)
    assert msg


def test_null_arguments(mpdc):
    out = ctypes.c_void_p()
    assert mpdc.lib.mpdc_mesh_create(None, None, 0, None, ctypes.byref(out)) == -1
    assert mpdc.lib.mpdc_mesh_workspace_bytes(None) == 0
    assert mpdc.lib.mpdc_mesh_check(None) == -1
    assert mpdc.lib.mpdc_dycore_step(None, 1, None) == -1
    assert mpdc.lib.mpdc_state_read(None, 0, None, 0, 0, None) == -1


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5, 6])
def test_valid_meshes_derive_on_host(mpdc, mesh_cache, level):
    """Every icosahedral mesh validates and derives its tables on the host."""
    rc, msg, _ = _create(mpdc, mesh_cache(level))
    assert rc == 0, (level, msg)


def test_relabelled_mesh_is_valid(mpdc, mesh_cache):
    # a randomly renumbered mesh (the GPU invariance test's input) passes the
    # library's validation and table derivation
    from mesh_relabel import relabel
    mp, _, _, _ = relabel(mesh_cache(3))
    rc, msg, _ = _create(mpdc, mp)
    assert rc == 0, msg


def test_trisected_mesh_is_valid(mpdc, mesh_cache):
    # the B3-style grid (one trisection, then bisections) passes the library's
    # validation and table derivation
    rc, msg, _ = _create(mpdc, mesh_cache(1, 1))
    assert rc == 0, msg
