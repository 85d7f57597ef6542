"""Synthetic icosahedral Voronoi C-grid meshes (an input generator).

The paper runs GRIST on its own icosahedral grids G6..G9B3 (Section 2.1,
Table 1); those grid files are not available, so this module builds the
plain recursive-bisection analogue with the same cell counts
N = 10*4^n + 2.  The mesh is an *input* of the method: connectivity and
FP64 geometry produced here are handed unchanged to both the CPU oracle and
the library's ``mpdc_mesh_create``; each derives its own operator tables.

Construction (all geometry on the unit sphere, lengths scaled by ``radius``):

* icosahedron with a vertex at each pole and two rings of five at latitude
  +-atan(1/2) (longitudes 2*pi*j/5 and 2*pi*j/5 + pi/5);
* optionally one or more trisections first (each face into nine: two
  points on every edge at a third and two thirds of the chord, one at the
  face centre; the "B3" grids of Table 1, G9B3 = one trisection and nine
  bisections), then ``level`` recursive bisections, each new point
  normalised onto the sphere; an icosahedron edge ends up in
  n = 3^t 2^level segments and N = 10 n^2 + 2;
* Voronoi vertices are the spherical circumcentres of the Delaunay
  triangles; the edge point x_e is normalize(x_c1 + x_c2);
* cells, edges and vertices are renumbered along a 3-D Hilbert curve so that
  mesh neighbours are close in memory;
* n_e points from c1 to c2 (c1 < c2 after renumbering); t_e = k x n_e points
  from v1 to v2;
* ``edges_on_cell`` / ``vertices_on_cell`` are CSR lists in counter-clockwise
  order with vertex j between edges j-1 and j;
* ``cells_on_vertex`` / ``edges_on_vertex`` are counter-clockwise with edge j
  joining cells j and j+1;
* kite area R[v][j] of cell cells_on_vertex[v][j] is the sum of the two
  spherical triangles (x_i, x_e, x_v) over the two edges that cell i and
  vertex v share (triangle area by the Van Oosterom-Strackee formula);
  A_i and A_v are sums of kites, so the areas tile the sphere.
"""
import numpy as np

EARTH_RADIUS = 6.371e6
OMEGA = 7.292e-5


def mesh_counts(level, trisections=0):
    """(cells, edges, vertices) after ``trisections`` trisections and ``level`` bisections."""
    n2 = 9 ** trisections * 4 ** level
    return 10 * n2 + 2, 30 * n2, 20 * n2


def _normalize(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _icosahedron():
    lat = np.arctan(0.5)
    pts = [[0.0, 0.0, 1.0]]
    for j in range(5):
        lon = 2.0 * np.pi * j / 5.0
        pts.append([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])
    for j in range(5):
        lon = 2.0 * np.pi * j / 5.0 + np.pi / 5.0
        pts.append([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), -np.sin(lat)])
    pts.append([0.0, 0.0, -1.0])
    faces = []
    for j in range(5):
        jn = (j + 1) % 5
        faces.append([0, 1 + j, 1 + jn])
        faces.append([1 + j, 6 + j, 1 + jn])
        faces.append([1 + jn, 6 + j, 6 + jn])
        faces.append([11, 6 + jn, 6 + j])
    pts = np.array(pts)
    faces = np.array(faces, dtype=np.int64)
    # orient every face counter-clockwise seen from outside
    a, b, c = pts[faces[:, 0]], pts[faces[:, 1]], pts[faces[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    faces[flip] = faces[flip][:, [0, 2, 1]]
    return pts, faces


def _bisect(pts, faces):
    n = pts.shape[0]
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
    key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    ukey, inv = np.unique(key, return_inverse=True)
    ea, eb = ukey // n, ukey % n
    mid = _normalize(pts[ea] + pts[eb])
    m = n + inv.reshape(3, -1)          # midpoint ids of edges 01, 12, 20
    m01, m12, m20 = m[0], m[1], m[2]
    f0, f1, f2 = faces[:, 0], faces[:, 1], faces[:, 2]
    newf = np.concatenate([
        np.stack([f0, m01, m20], 1),
        np.stack([f1, m12, m01], 1),
        np.stack([f2, m20, m12], 1),
        np.stack([m01, m12, m20], 1),
    ])
    return np.concatenate([pts, mid]), newf


def _trisect(pts, faces):
    """Split every face into nine: points at 1/3 and 2/3 of each edge's chord
    (shared by the two faces of the edge) and at the face centre."""
    n = pts.shape[0]
    F = faces.shape[0]
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
    key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    ukey, inv = np.unique(key, return_inverse=True)
    ea, eb = ukey // n, ukey % n                      # ea < eb
    nE = ukey.shape[0]
    near_a = _normalize(2.0 * pts[ea] + pts[eb])      # a third of the way from ea
    near_b = _normalize(pts[ea] + 2.0 * pts[eb])      # a third of the way from eb
    f0, f1, f2 = faces[:, 0], faces[:, 1], faces[:, 2]
    cen = _normalize(pts[f0] + pts[f1] + pts[f2])
    inv = inv.reshape(3, F)

    def third(k, src):
        """id of the point a third of the way from src along face edge k"""
        ed = inv[k]
        return np.where(src == ea[ed], n + ed, n + nE + ed)

    a, b, c = f0, f1, f2
    ab1, ab2 = third(0, a), third(0, b)               # edge a-b: near a, near b
    bc1, bc2 = third(1, b), third(1, c)
    ca1, ca2 = third(2, c), third(2, a)
    g = n + 2 * nE + np.arange(F)
    # lattice P(i, j) = a + i/3 (b - a) + j/3 (c - a): six upward, three downward triangles
    newf = np.concatenate([
        np.stack([a, ab1, ca2], 1), np.stack([ab1, ab2, g], 1), np.stack([ab2, b, bc1], 1),
        np.stack([ca2, g, ca1], 1), np.stack([g, bc1, bc2], 1), np.stack([ca1, bc2, c], 1),
        np.stack([ab1, g, ca2], 1), np.stack([ab2, bc1, g], 1), np.stack([g, bc2, ca1], 1),
    ])
    return np.concatenate([pts, near_a, near_b, cen]), newf


def _hilbert_key(x, bits=20):
    """3-D Hilbert index (Skilling 2004, transpose form) of points in [-1,1]^3."""
    scale = (1 << bits) - 1
    X = np.clip(((x + 1.0) * 0.5 * scale).round(), 0, scale).astype(np.int64)
    X = [X[:, 0].copy(), X[:, 1].copy(), X[:, 2].copy()]
    Q = 1 << (bits - 1)
    while Q > 1:
        P = Q - 1
        for i in range(3):
            hit = (X[i] & Q) != 0
            X[0] = np.where(hit, X[0] ^ P, X[0])
            t = np.where(hit, 0, (X[0] ^ X[i]) & P)
            X[0] ^= t
            if i:
                X[i] ^= t
        Q >>= 1
    X[1] ^= X[0]
    X[2] ^= X[1]
    t = np.zeros_like(X[0])
    Q = 1 << (bits - 1)
    while Q > 1:
        t = np.where((X[2] & Q) != 0, t ^ (Q - 1), t)
        Q >>= 1
    for i in range(3):
        X[i] ^= t
    key = np.zeros_like(X[0])
    for b in range(bits - 1, -1, -1):
        for i in range(3):
            key = (key << 1) | ((X[i] >> b) & 1)
    return key


def _arc(a, b):
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.einsum("ij,ij->i", a, b))


def _tri_area(a, b, c):
    num = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c)))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def icosahedral_mesh(level, radius=EARTH_RADIUS, omega=OMEGA, reorder=True, trisections=0):
    """Build the Voronoi mesh of ``trisections`` trisections and ``level``
    bisections of the icosahedron; return a dict of arrays.

    Index arrays are int32, geometry float64.  Positions are unit vectors;
    lengths (de, le) are in metres and areas in m^2 on a sphere of
    ``radius``.
    """
    pts, faces = _icosahedron()
    for _ in range(trisections):
        pts, faces = _trisect(pts, faces)
    for _ in range(level):
        pts, faces = _bisect(pts, faces)
    N = pts.shape[0]
    nF = faces.shape[0]

    if reorder:
        perm = np.argsort(_hilbert_key(pts), kind="stable")
        rank = np.empty(N, np.int64)
        rank[perm] = np.arange(N)
        pts = pts[perm]
        faces = rank[faces]
        fc = _normalize(pts[faces[:, 0]] + pts[faces[:, 1]] + pts[faces[:, 2]])
        faces = faces[np.argsort(_hilbert_key(fc), kind="stable")]

    a, b, c = pts[faces[:, 0]], pts[faces[:, 1]], pts[faces[:, 2]]
    xv = _normalize(np.cross(b - a, c - a))

    # undirected Delaunay edges, one per Voronoi edge; left face of each directed half edge
    he_from = faces.reshape(-1)
    he_to = faces[:, [1, 2, 0]].reshape(-1)
    he_face = np.repeat(np.arange(nF), 3)
    lo, hi = np.minimum(he_from, he_to), np.maximum(he_from, he_to)
    key = lo * N + hi
    ukey, first = np.unique(key, return_index=True)
    E = ukey.shape[0]
    c1, c2 = ukey // N, ukey % N
    if reorder:
        xe0 = _normalize(pts[c1] + pts[c2])
        eperm = np.argsort(_hilbert_key(xe0), kind="stable")
        ukey, c1, c2 = ukey[eperm], c1[eperm], c2[eperm]
    # face left of c1->c2 is v2; face left of c2->c1 is v1
    order = np.argsort(he_from * N + he_to)
    sorted_dir = (he_from * N + he_to)[order]

    def left_face(src, dst):
        idx = np.searchsorted(sorted_dir, src * N + dst)
        assert np.all(sorted_dir[idx] == src * N + dst)
        return he_face[order[idx]]

    v2 = left_face(c1, c2)
    v1 = left_face(c2, c1)

    xc = pts
    xe = _normalize(xc[c1] + xc[c2])
    de = radius * _arc(xc[c1], xc[c2])
    le = radius * _arc(xv[v1], xv[v2])

    def edge_of(i, j):
        k = np.minimum(i, j) * N + np.maximum(i, j)
        idx = np.searchsorted(ukey_sorted, k)
        assert np.all(ukey_sorted[idx] == k)
        return eidx_sorted[idx]

    so = np.argsort(ukey)
    ukey_sorted, eidx_sorted = ukey[so], so

    # vertices around each cell, counter-clockwise
    inc_cell = faces.reshape(-1)
    inc_face = np.repeat(np.arange(nF), 3)
    inc_corner = np.tile(np.arange(3), nF)
    k_hat = xc[inc_cell]
    ref = np.where(np.abs(k_hat[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = _normalize(np.cross(ref, k_hat))
    e2 = np.cross(k_hat, e1)
    dv = xv[inc_face]
    ang = np.arctan2(np.einsum("ij,ij->i", dv, e2), np.einsum("ij,ij->i", dv, e1))
    o = np.lexsort((ang, inc_cell))
    inc_cell, inc_face, inc_corner = inc_cell[o], inc_face[o], inc_corner[o]
    deg = np.bincount(inc_cell, minlength=N)
    off = np.zeros(N + 1, np.int64)
    off[1:] = np.cumsum(deg)
    voc = inc_face                               # vertex j of cell i (CSR)
    # edge j joins vertex j and vertex j+1: it is the Delaunay edge (i, x) where x is the
    # vertex preceding i in face j (face (i, a, x) ccw; next face ccw around i is left of i->x)
    prev_corner = faces[inc_face, (inc_corner + 2) % 3]
    eoc = edge_of(inc_cell, prev_corner)
    # the next face around i must be the left face of i -> prev
    nxt = np.roll(np.arange(off[-1]), -1)
    last = off[1:] - 1
    nxt[last] = off[:-1]
    assert np.all(left_face(inc_cell, prev_corner) == voc[nxt]), "ccw cell ordering broken"
    # rotate so that vertex j sits between edges j-1 and j (voc as built has vertex j
    # between edge j-1 and j already: edge j joins voc[j] and voc[j+1])

    cov = faces.astype(np.int64)                                   # ccw cells of each vertex
    eov = np.stack([edge_of(cov[:, 0], cov[:, 1]), edge_of(cov[:, 1], cov[:, 2]),
                    edge_of(cov[:, 2], cov[:, 0])], 1)

    # kites: cell cov[v][j] shares edges eov[v][j] (cells j, j+1) and eov[v][j-1] (cells j-1, j)
    kite = np.zeros((nF, 3))
    for j in range(3):
        xi = xc[cov[:, j]]
        ea = xe[eov[:, j]]
        eb = xe[eov[:, (j + 2) % 3]]
        kite[:, j] = _tri_area(xi, ea, xv) + _tri_area(xi, eb, xv)
    kite *= radius ** 2
    areaC = np.zeros(N)
    np.add.at(areaC, cov.reshape(-1), kite.reshape(-1))
    areaV = kite.sum(1)
    fv = 2.0 * omega * xv[:, 2]

    return dict(
        level=level, trisections=trisections, radius=radius, omega=omega,
        nCells=N, nEdges=E, nVertices=nF,
        cells_on_edge=np.stack([c1, c2], 1).astype(np.int32),
        vertices_on_edge=np.stack([v1, v2], 1).astype(np.int32),
        eoc_offset=off.astype(np.int32),
        edges_on_cell=eoc.astype(np.int32),
        vertices_on_cell=voc.astype(np.int32),
        cells_on_vertex=cov.astype(np.int32),
        edges_on_vertex=eov.astype(np.int32),
        xCell=np.ascontiguousarray(xc), xVertex=np.ascontiguousarray(xv), xEdge=np.ascontiguousarray(xe),
        dEdge=de, lEdge=le, areaCell=areaC, areaVertex=areaV, kiteArea=np.ascontiguousarray(kite),
        fVertex=fv,
    )


def lonlat(x):
    """(lon, lat) in radians of unit vectors ``x``."""
    return np.arctan2(x[:, 1], x[:, 0]), np.arcsin(np.clip(x[:, 2], -1.0, 1.0))
