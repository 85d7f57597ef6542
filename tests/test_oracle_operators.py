"""Pins of the FP64 oracle's discrete operators against mathematics (CPU).

Each test checks the oracle against something other than itself: mimetic
identities of the C-grid (gradient of a constant, curl of a gradient,
divergence of a rotational field, telescoping, adjointness), the exact
streamfunction identity that defines the TRiSK weights, antisymmetry and
energy neutrality of the Coriolis term, rank/null-space facts of the dense
operator matrices on tiny meshes, exactness of the quadratic fit, the 1-D
third-order upwind stencil, and the Thomas solve against dense LU.
"""
import numpy as np
import pytest

from oracle import OracleMesh, thomas, oracle_lib
from paper_2404_08849_amd.inputs.initial import velocity_from_streamfunction


@pytest.fixture(scope="module", params=[(3, 0), (2, 1)], ids=["G3", "G2B3"])
def g3(mesh_cache, request):
    # a bisection grid and a trisection ("B3") grid of similar size
    m = mesh_cache(*request.param)
    return m, OracleMesh(m)


def test_gradient_of_constant_is_exactly_zero(g3):
    m, om = g3
    assert np.all(om.gradient(np.full(om.N, 3.25e4)) == 0.0)


def test_curl_of_gradient_vanishes(g3):
    m, om = g3
    psi = np.random.default_rng(1).standard_normal(om.N)
    g = om.gradient(psi)
    assert np.abs(om.curl(g)).max() * m["dEdge"].mean() <= 1e-14 * np.abs(g).max()


def test_divergence_of_rotational_flow_vanishes(g3):
    m, om = g3
    psiv = np.random.default_rng(2).standard_normal(om.V)
    u = velocity_from_streamfunction(m, psiv)
    assert np.abs(om.divergence(u)).max() * m["dEdge"].mean() <= 1e-14 * np.abs(u).max()


def test_divergence_telescopes_and_is_adjoint_of_gradient(g3):
    m, om = g3
    r = np.random.default_rng(3)
    F, psi = r.standard_normal(om.E), r.standard_normal(om.N)
    D = om.divergence(F)
    A = m["areaCell"]
    assert abs((A * D).sum()) <= 1e-14 * (A * np.abs(D)).sum()
    lhs = (m["lEdge"] * m["dEdge"] * F * om.gradient(psi)).sum()
    rhs = -(A * psi * D).sum()
    assert abs(lhs - rhs) <= 1e-14 * np.abs(m["lEdge"] * m["dEdge"] * F * om.gradient(psi)).sum()


def test_trisk_weights_antisymmetric(g3):
    m, om = g3
    t = om.tables()
    W = {}
    for e in range(om.E):
        for j in range(t["trisk_offset"][e], t["trisk_offset"][e + 1]):
            W[(e, int(t["trisk_edge"][j]))] = t["trisk_weight"][j]
    assert len(W) == t["trisk_offset"][-1]
    assert max(abs(W[(a, b)] + W[(b, a)]) for (a, b) in W) <= 1e-15


def test_trisk_streamfunction_identity(g3):
    """For u = -(psi_v2 - psi_v1)/l, the reconstructed tangential flux equals the
    gradient of the kite-weighted cell mean psi_bar_i = sum_v R_iv psi_v / A_i."""
    m, om = g3
    psiv = np.random.default_rng(4).standard_normal(om.V)
    u = velocity_from_streamfunction(m, psiv)
    psib = np.zeros(om.N)
    np.add.at(psib, m["cells_on_vertex"].ravel(), (m["kiteArea"] * psiv[:, None]).ravel())
    psib /= m["areaCell"]
    ref = (psib[m["cells_on_edge"][:, 1]] - psib[m["cells_on_edge"][:, 0]]) / m["dEdge"]
    assert np.abs(om.perp_flux(u) - ref).max() <= 1e-14 * np.abs(ref).max()


def test_coriolis_does_no_work(g3):
    m, om = g3
    r = np.random.default_rng(5)
    F, qv = r.standard_normal(om.E), r.standard_normal(om.V)
    Q = om.coriolis(F, qv)
    w = m["lEdge"] * m["dEdge"]
    assert abs((w * F * Q).sum()) <= 1e-14 * (w * np.abs(F * Q)).sum()


def test_kinetic_energy_of_solid_body_rotation(mesh_cache):
    """K = u^2/2 is recovered to first order for u = u0 cos(lat)."""
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        u0 = 20.0
        latv = np.arcsin(m["xVertex"][:, 2])
        u = velocity_from_streamfunction(m, -m["radius"] * u0 * np.sin(latv))
        ke = om.kinetic_energy(u)
        exact = 0.5 * (u0 * np.cos(np.arcsin(m["xCell"][:, 2]))) ** 2
        errs.append(np.sqrt((m["areaCell"] * (ke - exact) ** 2).sum() / (m["areaCell"] * exact ** 2).sum()))
    assert errs[0] > errs[1] > errs[2]


def test_vertex_mass_of_constant(g3):
    m, om = g3
    hv = om.vertex_mass(np.full(om.N, 7.5))
    assert np.allclose(hv, 7.5, rtol=1e-14)


def test_dense_operator_matrices_on_tiny_meshes(mesh_cache):
    for lev in (0, 1, 2):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        N, E, V = om.N, om.E, om.V
        D = om.divergence(np.eye(E)).reshape(N, E)          # column j = D(unit flux j)
        G = om.gradient(np.eye(N)).reshape(E, N)
        C = om.curl(np.eye(E)).reshape(V, E)
        S = np.zeros((E, V))                                 # rotational velocity from vertex psi
        v1, v2 = m["vertices_on_edge"].T
        S[np.arange(E), v2] = -1.0 / m["lEdge"]
        S[np.arange(E), v1] += 1.0 / m["lEdge"]
        assert np.linalg.matrix_rank(D) == N - 1
        assert np.linalg.matrix_rank(G) == N - 1
        assert np.allclose(G @ np.ones(N), 0.0, atol=0)
        assert np.abs(C @ G).max() <= 1e-13 * np.abs(C).max() * np.abs(G).max()
        assert np.abs(D @ S).max() <= 1e-13 * np.abs(D).max() * np.abs(S).max()
        assert np.linalg.matrix_rank(C) == V - 1


def _bearing_coords(x_i, x_k, radius, east, north):
    """Azimuthal-equidistant coordinates of x_k around x_i in an east/north basis."""
    r = np.arctan2(np.linalg.norm(np.cross(x_i, x_k)), np.dot(x_i, x_k))
    t = x_k - np.dot(x_k, x_i) * x_i
    t /= np.linalg.norm(t)
    return radius * r * np.dot(t, east), radius * r * np.dot(t, north), np.dot(t, east), np.dot(t, north)


def test_hessian_fit_reproduces_quadratics(mesh_cache):
    """A quadratic in local (arc length x bearing) coordinates, written in an
    east/north basis different from the oracle's, is differentiated exactly
    along every neighbour direction (pentagons and hexagons)."""
    m = mesh_cache(3)
    om = OracleMesh(m)
    off, coc = m["eoc_offset"], om.tables()["cells_on_cell"]
    r = np.random.default_rng(6)
    deg = np.diff(off)
    cells = list(np.where(deg == 5)[0][:4]) + list(r.choice(np.where(deg == 6)[0], 20, replace=False))
    L = m["dEdge"].mean()
    for i in cells:
        xi = m["xCell"][i]
        ref = [0.0, 0.0, 1.0] if abs(xi[2]) < 0.9 else [1.0, 0.0, 0.0]
        east = np.cross(ref, xi)
        east /= np.linalg.norm(east)
        north = np.cross(xi, east)
        a, b, c, d, e, f = r.standard_normal(6)
        Qf = lambda x, y: a + b * x / L + c * y / L + d * (x / L) ** 2 + e * (x * y) / L ** 2 + f * (y / L) ** 2
        q = np.zeros(om.N)
        q[i] = Qf(0.0, 0.0)
        nbrs = coc[off[i]:off[i + 1]]
        dirs = []
        for k in nbrs:
            x, y, ce, sn = _bearing_coords(xi, m["xCell"][k], m["radius"], east, north)
            q[k] = Qf(x, y)
            dirs.append((ce, sn))
        got = om.hessian_dir(q)[off[i]:off[i + 1]]
        want = np.array([(2 * d * ce * ce + 2 * e * ce * sn + 2 * f * sn * sn) / L ** 2 for ce, sn in dirs])
        assert np.allclose(got, want, rtol=1e-9, atol=1e-12 / L ** 2), (i, got, want)


def test_hessian_zero_for_constant_and_linear(g3):
    m, om = g3
    assert np.abs(om.hessian_dir(np.full(om.N, 4.0))).max() == 0.0


def test_hessian_converges_on_sphere(mesh_cache):
    """For q = z on the sphere every second derivative along a great circle is -z/a^2."""
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        z = m["xCell"][:, 2]
        hd = om.hessian_dir(z)
        cell_of_slot = np.repeat(np.arange(om.N), np.diff(m["eoc_offset"]))
        exact = -z[cell_of_slot] / m["radius"] ** 2
        errs.append(np.abs(hd - exact).max() / np.abs(exact).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


def test_edge_value_matches_1d_third_order_stencil():
    """On a uniform line with q'' = (q_{i+1} - 2 q_i + q_{i-1})/dx^2 the edge value is
    the kappa = 1/3 upwind stencil: q_{i+1/2} = q_{i+1}/3 + 5 q_i/6 - q_{i-1}/6 for F > 0,
    and the mirror image for F < 0."""
    lib = oracle_lib()
    r = np.random.default_rng(7)
    n, dx = 50, 3.0e4
    q = r.standard_normal(n + 3)
    lap = (q[2:] - 2 * q[1:-1] + q[:-2]) / dx ** 2        # at cells 1 .. n+1
    import ctypes
    dp = ctypes.POINTER(ctypes.c_double)
    for sign in (1.0, -1.0):
        q1 = np.ascontiguousarray(q[1:n + 1])
        q2 = np.ascontiguousarray(q[2:n + 2])
        h1 = np.ascontiguousarray(lap[0:n])
        h2 = np.ascontiguousarray(lap[1:n + 1])
        d = np.full(n, dx)
        F = np.full(n, sign)
        out = np.empty(n)
        lib.or_edge_value3_formula(n, *[a.ctypes.data_as(dp) for a in (q1, q2, h1, h2, d, F, out)])
        if sign > 0:
            want = q[2:n + 2] / 3 + 5 * q[1:n + 1] / 6 - q[0:n] / 6
        else:
            want = q[1:n + 1] / 3 + 5 * q[2:n + 2] / 6 - q[3:n + 3] / 6
        assert np.allclose(out, want, rtol=0, atol=1e-14 * np.abs(q).max())


def test_thomas_matches_dense_solve():
    r = np.random.default_rng(8)
    for n in (1, 2, 7, 59):
        sub, sup = r.standard_normal(n), r.standard_normal(n)
        diag = np.abs(sub) + np.abs(sup) + 1.0 + r.random(n)
        rhs = r.standard_normal(n)
        A = np.diag(diag) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
        x = thomas(sub, diag, sup, rhs)
        assert np.allclose(x, np.linalg.solve(A, rhs), rtol=1e-13, atol=1e-13)
