"""Random relabelling of a mesh (test helper): cells, edges and vertices are
renumbered by seeded permutations; each cell keeps its counter-clockwise
edge order and each edge its orientation."""
import numpy as np


def relabel(m, seed=11):
    """The mesh with permuted cell, edge and vertex numbers, and the maps:
    new index of old cell c is pc[c] (likewise pe, pv)."""
    r = np.random.default_rng(seed)
    N, E, V = m["nCells"], m["nEdges"], m["nVertices"]
    pc, pe, pv = r.permutation(N), r.permutation(E), r.permutation(V)
    ic_, ie, iv = np.argsort(pc), np.argsort(pe), np.argsort(pv)      # old index of new entity
    out = dict(m)
    out["cells_on_edge"] = np.ascontiguousarray(pc[m["cells_on_edge"][ie]].astype(np.int32))
    out["vertices_on_edge"] = np.ascontiguousarray(pv[m["vertices_on_edge"][ie]].astype(np.int32))
    off, eoc, voc = m["eoc_offset"], m["edges_on_cell"], m["vertices_on_cell"]
    deg = np.diff(off)[ic_]
    noff = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    neoc = np.concatenate([pe[eoc[off[c]:off[c + 1]]] for c in ic_]).astype(np.int32)
    nvoc = np.concatenate([pv[voc[off[c]:off[c + 1]]] for c in ic_]).astype(np.int32)
    out["eoc_offset"], out["edges_on_cell"], out["vertices_on_cell"] = noff, neoc, nvoc
    out["cells_on_vertex"] = np.ascontiguousarray(pc[m["cells_on_vertex"][iv]].astype(np.int32))
    out["edges_on_vertex"] = np.ascontiguousarray(pe[m["edges_on_vertex"][iv]].astype(np.int32))
    for k in ("xCell", "areaCell"):
        out[k] = np.ascontiguousarray(m[k][ic_])
    for k in ("xEdge", "dEdge", "lEdge"):
        out[k] = np.ascontiguousarray(m[k][ie])
    for k in ("xVertex", "areaVertex", "kiteArea", "fVertex"):
        out[k] = np.ascontiguousarray(m[k][iv])
    return out, ic_, ie, iv
