"""The library's host mesh code (validation and TRiSK/least-squares table
derivation, the part of mpdc_mesh_create that runs on the CPU) under
AddressSanitizer and UndefinedBehaviorSanitizer: a g++ build of mesh.cpp and
a small driver.  Valid meshes (G0-G3, a trisected G2B3, a relabelled G2)
pass; corrupted ones (an index out of range, a reversed cell, a zero area,
a broken edge-vertex link, a truncated offset list) are rejected with a
reason and no invalid access."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from mesh_relabel import relabel

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_08849_amd", "csrc")
INTS = ("cells_on_edge", "vertices_on_edge", "eoc_offset", "edges_on_cell", "vertices_on_cell",
        "cells_on_vertex", "edges_on_vertex")
DBLS = ("xCell", "xVertex", "xEdge", "dEdge", "lEdge", "areaCell", "areaVertex", "kiteArea", "fVertex")


def _write(path, m):
    with open(path, "wb") as f:
        np.array([m["nCells"], m["nEdges"], m["nVertices"]], np.int32).tofile(f)
        np.array([m["radius"]], np.float64).tofile(f)
        for k in INTS:
            np.ascontiguousarray(m[k], np.int32).tofile(f)
        for k in DBLS:
            np.ascontiguousarray(m[k], np.float64).tofile(f)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("meshsan") / "mesh_sanitized")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + "address,undefined",
             "-fno-sanitize-recover=all", "-ffp-contract=off", "-I", CSRC, "-I", "/opt/rocm/include",
             "-D__HIP_PLATFORM_AMD__"]
    r = subprocess.run([gxx] + flags + [os.path.join(CSRC, "mesh.cpp"), os.path.join(HERE, "mesh_sanitize_driver.cpp"),
                                        "-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "hip" in (r.stderr or "").lower() and "no such file" in (r.stderr or "").lower():
        pytest.skip("HIP headers not available")
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, m, tmp_path, name):
    path = str(tmp_path / (name + ".bin"))
    _write(path, m)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=300)


def _copy(m):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}


def test_valid_meshes_pass(driver, mesh_cache, tmp_path):
    cases = [("g%d" % lev, mesh_cache(lev)) for lev in range(4)]
    cases.append(("g2b3", mesh_cache(2, 1)))
    cases.append(("g2_relabelled", relabel(mesh_cache(2), seed=11)[0]))
    for name, m in cases:
        r = _run(driver, m, tmp_path, name)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (name, r.stdout[-300:], r.stderr[-3000:])


def _corruptions(m):
    N, E = m["nCells"], m["nEdges"]
    a = _copy(m)
    a["cells_on_edge"].reshape(-1)[7] = N + 5                     # index out of range
    yield "cell index out of range", a
    a = _copy(m)
    a["edges_on_cell"].reshape(-1)[-3] = -E                       # negative index
    yield "negative edge index", a
    a = _copy(m)
    o = a["eoc_offset"]
    a["edges_on_cell"][o[4]:o[5]] = a["edges_on_cell"][o[4]:o[5]][::-1].copy()   # clockwise cell
    a["vertices_on_cell"][o[4]:o[5]] = a["vertices_on_cell"][o[4]:o[5]][::-1].copy()
    yield "reversed cell", a
    a = _copy(m)
    a["areaCell"][3] = 0.0
    yield "zero area", a
    a = _copy(m)
    voe = a["vertices_on_edge"].reshape(-1, 2)
    voe[5] = voe[5][::-1].copy()                                  # edge tangent flipped against its vertices
    yield "flipped edge vertices", a
    a = _copy(m)
    a["eoc_offset"][N] = a["eoc_offset"][N] + 4                   # offsets run past the lists
    yield "offsets past the end", a


def test_corrupted_meshes_are_rejected_cleanly(driver, mesh_cache, tmp_path):
    m = mesh_cache(2)
    for i, (what, bad) in enumerate(_corruptions(m)):
        r = _run(driver, bad, tmp_path, "bad%d" % i)
        assert r.returncode == 3 and r.stdout.startswith("rejected: "), (what, r.returncode, r.stdout[-300:],
                                                                         r.stderr[-3000:])
