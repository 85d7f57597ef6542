"""Pins of three oracle parts against mathematics (CPU): the advection of an
interface field in the non-hydrostatic w and phi equations (Eqs. 6-7), the
kite-weighted vertex mass of the potential vorticity (Eq. 5, zeta_p, the FP64
term of Section 2.3) and the error norms of the precision criterion
(Section 2.2, Eqs. 1-2).

Each pin is a closed form or an exact identity derived by hand below, so a
dropped term, a flipped sign, a mis-paired weight or a missing normalisation
in the oracle fails it.
"""
import numpy as np
import pytest

from oracle import OracleMesh, norms
from paper_2404_08849_amd.inputs.initial import velocity_from_streamfunction

# Solid-body rotation about a tilted axis: V = w_rot (Omega_hat x r),
# streamfunction psi = -w_rot a^2 (Omega_hat . r_hat) with V = k x grad psi.
ALPHA = np.deg2rad(45.0)
AXIS = np.array([np.sin(ALPHA), 0.0, np.cos(ALPHA)])
U0 = 40.0                                    # equatorial speed about the axis (m/s)

# A smooth interface field X(r_hat) = c . r_hat + r_hat^T B r_hat (B symmetric)
C_LIN = np.array([0.3, -1.1, 0.7])
B_QUAD = np.array([[0.5, 0.2, -0.4], [0.2, -0.8, 0.3], [-0.4, 0.3, 0.6]])


def _x_field(xyz):
    return xyz @ C_LIN + np.einsum("ni,ij,nj->n", xyz, B_QUAD, xyz)


def _x_advected(xyz, a):
    """Exact V.grad X on the sphere: X depends on r_hat only, and r_hat moves
    with d r_hat/dt = V / a = (U0 / a) Omega_hat x r_hat, so
    V.grad X = (U0 / a) (c + 2 B r_hat) . (Omega_hat x r_hat)."""
    grad = C_LIN[None, :] + 2.0 * xyz @ B_QUAD
    return (U0 / a) * (grad * np.cross(AXIS[None, :], xyz)).sum(axis=1)


def _layer_masses(N, K, seed):
    """Unequal layer masses (Pa), the same shape in every column up to a factor."""
    r = np.random.default_rng(seed)
    prof = 500.0 + 3000.0 * r.random(K)
    return prof[None, :] * (1.0 + 0.2 * r.random(N))[:, None]


@pytest.mark.parametrize("K", [1, 4])
def test_iface_horizontal_advection_converges_to_closed_form(mesh_cache, K):
    """With F_k = dpi_k u (every layer moving with the same solid-body velocity
    u) the interface mass flux divided by the interface mass is u at every
    interface, including the lid and surface half layers, so the horizontal
    term must approach the exact V.grad X at every level; with no vertical
    flux there is nothing else.  The error falls with resolution and is small
    at G5: a flipped or dropped horizontal term gives a relative error of 2
    or 1."""
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        a = m["radius"]
        psiv = -(U0 * a) * (m["xVertex"] @ AXIS)
        u = velocity_from_streamfunction(m, psiv)
        # unequal layers, the same in every column, so F^/dpi^ = u at every interface
        dpi = np.repeat(_layer_masses(1, K, seed=11), om.N, axis=0)
        F = dpi[0][None, :] * u[:, None]
        X1 = _x_field(m["xCell"])
        X = np.stack([(1.0 + 0.25 * k) * X1 + 100.0 * k for k in range(K + 1)], axis=1)
        out = om.iface_advection(F, dpi, np.zeros((om.N, K + 1)), X)
        ex1 = _x_advected(m["xCell"], a)
        exact = np.stack([(1.0 + 0.25 * k) * ex1 for k in range(K + 1)], axis=1)
        A = m["areaCell"][:, None]
        errs.append(float(np.sqrt((A * (out - exact) ** 2).sum() / (A * exact ** 2).sum())))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] <= 1e-2, errs


def test_iface_vertical_advection_uniform_mdot_is_exact():
    """X linear in the interface pressure, X_k = b pi_k, and a uniform vertical
    mass flux m0: the centred vertical term is exactly m0 b at every interface
    for any layer masses -- interior: m0 (X_{k+1} - X_{k-1}) / (dpi_{k-1} +
    dpi_k) = m0 b; lid and surface: m0 b dpi / (2 dpi / 2).  This pins the sign
    of the term, the half-layer interface masses at the ends and the
    averaging weights."""
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    m = icosahedral_mesh(1)
    om = OracleMesh(m)
    K = 7
    dpi = _layer_masses(om.N, K, seed=12)
    pi = np.concatenate([np.zeros((om.N, 1)), np.cumsum(dpi, axis=1)], axis=1) + 1000.0
    b, m0 = 3.7e-2, -0.45
    out = om.iface_advection(np.zeros((om.E, K)), dpi, np.full((om.N, K + 1), m0), b * pi)
    assert np.abs(out - m0 * b).max() <= 1e-13 * abs(m0 * b)


def test_iface_vertical_advection_quadratic_mdot_closed_form():
    """Uniform layers (dpi = Delta), X_k = b pi_k and mdot_k = pi_k^2: the layer
    means of mdot are averaged over the two layers of an interface, so the
    interior value is b (m_{k-1} + 2 m_k + m_{k+1}) / 4 = b (pi_k^2 + Delta^2/2),
    and at the lid and surface b (m_0 + m_1)/2 and b (m_{K-1} + m_K)/2.  A
    stencil that uses the wrong interfaces (m_{k+-1} without m_k, or the
    neighbouring layer's mean) misses the Delta^2/2."""
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    m = icosahedral_mesh(1)
    om = OracleMesh(m)
    K, delta, b = 6, 2.0, 0.5
    pi = 1.0 + delta * np.arange(K + 1, dtype=np.float64)
    dpi = np.full((om.N, K), delta)
    md = np.repeat((pi ** 2)[None, :], om.N, axis=0)
    out = om.iface_advection(np.zeros((om.E, K)), dpi, md, np.repeat((b * pi)[None, :], om.N, axis=0))
    exact = b * (pi ** 2 + 0.5 * delta ** 2)
    exact[0] = b * 0.5 * (pi[0] ** 2 + pi[1] ** 2)
    exact[K] = b * 0.5 * (pi[K - 1] ** 2 + pi[K] ** 2)
    assert np.abs(out - exact[None, :]).max() <= 1e-14 * np.abs(exact).max()


def test_iface_advection_of_constant_is_zero(mesh_cache):
    """A field constant in the horizontal and in the vertical is not advected by
    any flux (both terms are differences of X)."""
    m = mesh_cache(3)
    om = OracleMesh(m)
    K = 5
    r = np.random.default_rng(13)
    out = om.iface_advection(r.standard_normal((om.E, K)), _layer_masses(om.N, K, 14),
                             r.standard_normal((om.N, K + 1)), np.full((om.N, K + 1), 42.0))
    assert np.all(out == 0.0)


@pytest.mark.parametrize("lev,tri", [(3, 0), (2, 1)])
def test_vertex_mass_kite_partition(mesh_cache, lev, tri):
    """sum_v A_v h_v = sum_v sum_{i of v} R_{i,v} h_i = sum_i h_i sum_{v of i} R_{i,v}
    = sum_i A_i h_i for any h, because the kites of a cell tile it.  Pairing a
    kite with the wrong cell of its vertex breaks the identity for a random
    field."""
    m = mesh_cache(lev, tri)
    om = OracleMesh(m)
    h = np.random.default_rng(15).standard_normal((om.N, 3)) + 2.0
    hv = om.vertex_mass(h)
    lhs = (m["areaVertex"][:, None] * hv).sum(axis=0)
    rhs = (m["areaCell"][:, None] * h).sum(axis=0)
    scale = (m["areaCell"][:, None] * np.abs(h)).sum(axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-14 * scale)


def test_vertex_mass_is_a_convex_combination(mesh_cache):
    """The kite weights R_{i,v}/A_v are positive and sum to one, so each vertex
    value lies between the smallest and largest of its three cells."""
    m = mesh_cache(3)
    om = OracleMesh(m)
    h = np.random.default_rng(16).standard_normal(om.N)
    hv = om.vertex_mass(h)
    hc = h[m["cells_on_vertex"]]
    tol = 1e-14 * np.abs(h).max()
    assert np.all(hv >= hc.min(axis=1) - tol) and np.all(hv <= hc.max(axis=1) + tol)


def test_norms_hand_computed():
    """Area-weighted normalised norms of Eq. 2 (Williamson et al. 1992) on a
    3-entity, 2-level example worked by hand:
      areas (1, 2, 3); x = [[1, 2], [3, 4], [5, 6]]; r = [[1, 1], [2, 2], [4, 8]];
      d = x - r = [[0, 1], [1, 2], [1, -2]];
      l1 = (1*1 + 2*3 + 3*3) / (1*2 + 2*4 + 3*12) = 16/46 = 8/23;
      l2 = sqrt((1*1 + 2*5 + 3*5) / (1*2 + 2*8 + 3*80)) = sqrt(26/258);
      linf = max|d| / max|r| = 2/8."""
    area = np.array([1.0, 2.0, 3.0])
    x = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    r = np.array([[1.0, 1.0], [2.0, 2.0], [4.0, 8.0]])
    l1, l2, li = norms(area, x, r)
    assert abs(l1 - 8.0 / 23.0) <= 1e-15
    assert abs(l2 - np.sqrt(26.0 / 258.0)) <= 1e-15
    assert li == 0.25


def test_norms_single_level_and_scaling():
    """K = 1 by hand (areas (1, 3), x = (2, 0), r = (1, 2): l1 = (1 + 6)/(1 + 6) = 1,
    l2 = sqrt((1 + 12)/(1 + 12)) = 1, linf = 2/2 = 1), and the norms of
    (x - r) = c r are |c| whatever the areas (normalisation)."""
    l1, l2, li = norms(np.array([1.0, 3.0]), np.array([2.0, 0.0]), np.array([1.0, 2.0]))
    assert (l1, l2, li) == (1.0, 1.0, 1.0)
    rng = np.random.default_rng(17)
    area = rng.random(50) + 0.1
    r = rng.standard_normal((50, 4))
    out = norms(area, 1.25 * r, r)
    assert np.allclose(out, 0.25, rtol=1e-14, atol=0)
