"""Mesh input generator: counts, topology, orientation and areas (CPU).

Pins: the cell counts of the paper's Table 1 (stored in
``golden/table1_cell_counts.txt``; G9B3 through the trisection count), the
closed forms N = 10 n^2 + 2, E = 30 n^2, V = 20 n^2 for n = 3^t 2^l segments
per icosahedron edge (bisection and trisection grids), Euler characteristic
2, exactly 12 pentagons, areas tiling the sphere, and the orientation
conventions the operators rely on.
"""
import os

import numpy as np
import pytest

from paper_2404_08849_amd.inputs.meshgen import mesh_counts

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_cell_counts.txt")


def _table1():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, _, cells = line.split()
        rows[name] = int(cells)
    return rows


def test_table1_counts_match_bisection_formula():
    t = _table1()
    for n in (6, 7, 8):
        assert mesh_counts(n)[0] == t["G%d" % n]
    # G9B3: one trisection and nine bisections split each icosahedron edge into
    # 3 * 2^9 segments, so N = 10 * (3 * 2^9)^2 + 2
    assert 10 * (3 * 2 ** 9) ** 2 + 2 == t["G9B3"]
    assert mesh_counts(9, trisections=1)[0] == t["G9B3"]


@pytest.mark.parametrize("level,tri", [(0, 0), (1, 0), (2, 0), (3, 0), (5, 0), (0, 1), (1, 1), (3, 1), (0, 2)])
def test_counts_and_topology(mesh_cache, level, tri):
    m = mesh_cache(level, tri)
    N, E, V = mesh_counts(level, tri)
    n = 3 ** tri * 2 ** level                      # segments per icosahedron edge
    assert N == 10 * n * n + 2
    assert (m["nCells"], m["nEdges"], m["nVertices"]) == (N, E, V)
    assert N - E + V == 2
    deg = np.diff(m["eoc_offset"])
    assert (deg == 5).sum() == 12 and ((deg == 5) | (deg == 6)).all()
    assert m["edges_on_cell"].shape == (2 * E,)
    # every edge appears exactly twice in the CSR lists, once per cell
    assert np.all(np.bincount(m["edges_on_cell"], minlength=E) == 2)
    assert np.all(np.bincount(m["edges_on_vertex"].ravel(), minlength=E) == 2)
    assert np.all(np.bincount(m["cells_on_vertex"].ravel(), minlength=N) == deg)


def test_generated_g6_matches_table1(mesh_cache):
    assert mesh_cache(6)["nCells"] == _table1()["G6"]


@pytest.mark.parametrize("level,tri", [(2, 0), (5, 0), (2, 1)])
def test_areas_tile_sphere(mesh_cache, level, tri):
    m = mesh_cache(level, tri)
    a = m["radius"]
    sphere = 4.0 * np.pi * a * a
    assert abs(m["areaCell"].sum() / sphere - 1.0) < 1e-13
    assert abs(m["areaVertex"].sum() / sphere - 1.0) < 1e-13
    assert (m["kiteArea"] > 0).all()
    # each cell area is the sum of its kites
    ac = np.zeros(m["nCells"])
    np.add.at(ac, m["cells_on_vertex"].ravel(), m["kiteArea"].ravel())
    assert np.allclose(ac, m["areaCell"], rtol=1e-14, atol=0)


@pytest.mark.parametrize("level,tri", [(1, 0), (4, 0), (1, 1)])
def test_orientation_conventions(mesh_cache, level, tri):
    m = mesh_cache(level, tri)
    xc, xv = m["xCell"], m["xVertex"]
    c1, c2 = m["cells_on_edge"].T
    v1, v2 = m["vertices_on_edge"].T
    n = xc[c2] - xc[c1]
    t = np.cross(m["xEdge"], n)                     # k x n_e
    assert (np.einsum("ij,ij->i", t, xv[v2] - xv[v1]) > 0).all()
    # CSR: vertex j lies between edges j-1 and j, all counter-clockwise
    off = m["eoc_offset"]
    for i in range(0, m["nCells"], max(1, m["nCells"] // 97)):
        es = m["edges_on_cell"][off[i]:off[i + 1]]
        vs = m["vertices_on_cell"][off[i]:off[i + 1]]
        d = len(es)
        for j in range(d):
            assert vs[j] in m["vertices_on_edge"][es[j - 1]] and vs[j] in m["vertices_on_edge"][es[j]]
        # counter-clockwise seen from outside: successive vertex directions turn left
        k = xc[i]
        for j in range(d):
            a_, b_ = xv[vs[j]] - k, xv[vs[(j + 1) % d]] - k
            assert np.dot(np.cross(a_, b_), k) > 0
    # cells_on_vertex counter-clockwise, edge j joins cells j and j+1
    cov, eov = m["cells_on_vertex"], m["edges_on_vertex"]
    a_, b_, c_ = xc[cov[:, 0]], xc[cov[:, 1]], xc[cov[:, 2]]
    assert (np.einsum("ij,ij->i", np.cross(b_ - a_, c_ - a_), xv) > 0).all()
    for j in range(3):
        ce = np.sort(m["cells_on_edge"][eov[:, j]], axis=1)
        want = np.sort(np.stack([cov[:, j], cov[:, (j + 1) % 3]], 1), axis=1)
        assert np.array_equal(ce, want)


def test_geometry_lengths(mesh_cache):
    m = mesh_cache(3)
    a = m["radius"]
    xc, xv = m["xCell"], m["xVertex"]
    c1, c2 = m["cells_on_edge"].T
    v1, v2 = m["vertices_on_edge"].T
    arc = lambda p, q: np.arccos(np.clip(np.einsum("ij,ij->i", p, q), -1, 1))
    assert np.allclose(m["dEdge"], a * arc(xc[c1], xc[c2]), rtol=1e-12)
    assert np.allclose(m["lEdge"], a * arc(xv[v1], xv[v2]), rtol=1e-12)
    # Voronoi property: each vertex is equidistant from its three cells
    cov = m["cells_on_vertex"]
    d = np.stack([arc(xv, xc[cov[:, j]]) for j in range(3)], 1)
    assert np.allclose(d, d[:, :1], rtol=1e-12)
