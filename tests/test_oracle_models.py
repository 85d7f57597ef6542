"""Pins of the FP64 oracle's time steppers against closed forms and invariants (CPU).

* shallow water: the steady zonal geostrophic flow is an exact solution of the
  continuous equations; the oracle's error after a fixed time falls as the
  mesh is refined, and mass is conserved to rounding;
* hydrostatic dycore: the isothermal jet u = u0 cos^2(lat) with its
  gradient-wind-balanced surface pressure is a steady state; errors below the
  top layer fall with resolution (the top layer carries a vertical truncation
  error that horizontal refinement cannot remove); mass to rounding (the flux
  form of Eq. 3 conserves global mass at double-precision level);
* non-hydrostatic dycore: the isothermal rest state in discrete hydrostatic
  balance stays at rest (w = 0, phi unchanged);
* tracer transport: a constant stays constant, no new extrema, tracer mass is
  conserved, the limiter switched off reproduces the unlimited third-order
  RK3 built from the oracle's edge-value and divergence operators, and the
  cosine bell after one revolution converges.
"""
import numpy as np
import pytest

from oracle import OracleMesh, area_sum, norms
from paper_2404_08849_amd.inputs import initial as ic


def test_sw_geostrophic_converges(mesh_cache):
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        s = ic.sw_geostrophic(m, bump=0)
        n = 10 * 2 ** (lev - 3)
        h, u = om.sw_run(s["h"], s["u"], s["b"], 2400.0 / 2 ** (lev - 3), n)
        eh = norms(m["areaCell"], h, s["h"])
        eu = norms(m["lEdge"] * m["dEdge"], u, s["u"])
        errs.append((eh[0], eh[1], eu[1]))
    errs = np.array(errs)
    assert np.all(errs[0] > errs[1]) and np.all(errs[1] > errs[2])
    # at least first order in l1 and l2 of h
    assert np.all(np.log2(errs[1, :2] / errs[2, :2]) > 1.0)


def test_sw_mass_conserved(mesh_cache):
    m = mesh_cache(4)
    om = OracleMesh(m)
    s = ic.sw_geostrophic(m)
    h, u = om.sw_run(s["h"], s["u"], s["b"], 1200.0, 20)
    m0 = area_sum(m["areaCell"], s["h"])
    assert abs(area_sum(m["areaCell"], h) - m0) <= 1e-14 * m0
    assert np.abs(h - s["h"]).max() > 1e-3       # the bump does move


def test_hdc_jet_steady_state_converges(mesh_cache):
    K = 30
    eps, eus = [], []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        s = ic.hdc_jet(m, K, pert=0)
        ps, Th, u = om.hdc_run(s["ps"], s["Theta"], s["u"], 2400.0 / 2 ** (lev - 3), 4 * 2 ** (lev - 3))
        eps.append(norms(m["areaCell"], ps, s["ps"]))
        eus.append(norms(m["lEdge"] * m["dEdge"], u[:, 1:], s["u"][:, 1:]))
    eps, eus = np.array(eps), np.array(eus)
    assert np.all(eps[0] > eps[1]) and np.all(eps[1] > eps[2])
    assert np.all(eus[0, :2] > eus[1, :2]) and np.all(eus[1, :2] > eus[2, :2])


def test_hdc_mass_conserved(mesh_cache):
    m = mesh_cache(4)
    om = OracleMesh(m)
    s = ic.hdc_jet(m, 10)
    ps, Th, u = om.hdc_run(s["ps"], s["Theta"], s["u"], 1200.0, 5)
    dm = area_sum(m["areaCell"], ps - 1000.0) - area_sum(m["areaCell"], s["ps"] - 1000.0)
    assert abs(dm) <= 1e-14 * area_sum(m["areaCell"], s["ps"] - 1000.0)
    assert np.abs(u - s["u"]).max() > 1e-3


def test_ndc_rest_state_is_steady(mesh_cache):
    m = mesh_cache(4)
    om = OracleMesh(m)
    s = ic.nh_warm_bubble(m, 20, dtheta=0)
    ps, Th, u, w, phi = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], 60.0, 5)
    assert np.abs(w).max() <= 1e-10
    assert np.abs(u).max() <= 1e-10
    assert np.abs(phi - s["phi"]).max() <= 1e-10 * np.abs(s["phi"]).max()


def test_ndc_bubble_rises(mesh_cache):
    """A warm anomaly produces upward motion over it and no NaNs."""
    m = mesh_cache(5)
    om = OracleMesh(m)
    s = ic.nh_warm_bubble(m, 20, rh=4.0e5)
    base = ic.nh_warm_bubble(m, 20, dtheta=0)
    ps, Th, u, w, phi = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], 60.0, 10)
    assert np.isfinite(w).all() and np.isfinite(u).all()
    hot = (s["Theta"] - base["Theta"]).max(1) > 0
    assert hot.any()
    assert w[hot].max() > 1e-4 and w[hot].max() > np.abs(w[~hot]).max()


@pytest.fixture(scope="module")
def tracer_g4(mesh_cache):
    m = mesh_cache(4)
    om = OracleMesh(m)
    s = ic.tracer_solid_body(m, 2, 3)
    q = s["q"].copy()
    q[:, :, 2] = 0.37
    return m, om, s, q


def test_tracer_constant_stays_constant(tracer_g4):
    m, om, s, q = tracer_g4
    dpi, qn = om.tracer_run(s["F"], s["dpi"], q, 3000.0, 10)
    assert np.abs(qn[:, :, 2] - 0.37).max() <= 1e-14


def test_tracer_bounds_and_mass(tracer_g4):
    m, om, s, q = tracer_g4
    dpi, qn = om.tracer_run(s["F"], s["dpi"], q, 3000.0, 20)
    for t in range(2):
        assert qn[:, :, t].min() >= q[:, :, t].min() - 1e-14
        assert qn[:, :, t].max() <= q[:, :, t].max() + 1e-14
        m0 = area_sum(m["areaCell"], s["dpi"] * q[:, :, t])
        assert abs(area_sum(m["areaCell"], dpi * qn[:, :, t]) - m0) <= 1e-13 * m0


def test_tracer_unlimited_matches_plain_rk3(tracer_g4):
    """With the limiter's bounds at +-infinity the step is the unlimited
    third-order RK3: q^(s) = [dpi q^n - dt_s D(F q~(q^(s-1)))] / (dpi - dt_s D(F))."""
    m, om, s, q = tracer_g4
    dt = 3000.0
    dpi, qn = om.tracer_run(s["F"], s["dpi"], q, dt, 2, fct=False)
    F = s["F"]
    divF = om.divergence(F)
    d = s["dpi"].copy()
    qq = q.copy()
    for _ in range(2):
        for t in range(q.shape[2]):
            q0 = qq[:, :, t].copy()
            qs = q0.copy()
            for frac in (1.0 / 3.0, 0.5, 1.0):
                dn = d - frac * dt * divF
                qs = (d * q0 - frac * dt * om.divergence(F * om.edge_value3(qs, F))) / dn
            qq[:, :, t] = qs
        d = d - dt * divF
    assert np.allclose(qn, qq, rtol=0, atol=1e-13)
    assert np.allclose(dpi, d, rtol=1e-15, atol=0)


def test_cosine_bell_revolution_converges(mesh_cache):
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        s = ic.tracer_solid_body(m, 1, 1)
        n = 108 * 2 ** (lev - 3)                     # Courant number ~0.4 at every level
        dpi, qn = om.tracer_run(s["F"], s["dpi"], s["q"], s["period"] / n, n)
        assert qn.min() >= -1e-14 and qn.max() <= 1.0 + 1e-14
        errs.append(norms(m["areaCell"], qn[:, 0, 0], s["q"][:, 0, 0]))
    errs = np.array(errs)
    assert np.all(errs[0] > errs[1]) and np.all(errs[1] > errs[2])


def test_hdc_uniform_theta_is_compatible_with_continuity(mesh_cache):
    """With theta uniform (Theta = c dpi) the theta_m equation (Eq. 4) reduces to
    c times the layer continuity equation, so theta stays c in every layer even
    under a strongly divergent wind that drives vertical mass fluxes."""
    m = mesh_cache(4)
    om = OracleMesh(m)
    K = 12
    s = ic.hdc_jet(m, K, pert=0)
    r = np.random.default_rng(11)
    u = 10.0 * r.standard_normal((om.E, K))
    ps = s["ps"]
    dpi = np.outer(ps - 1000.0, np.diff(ic.sigma_interfaces(K)))
    Th = 300.0 * dpi
    ps1, Th1, u1 = om.hdc_run(ps, Th, u, 120.0, 2)
    dpi1 = np.outer(ps1 - 1000.0, np.diff(ic.sigma_interfaces(K)))
    assert np.abs(ps1 - ps).max() > 1.0                      # the column mass does change
    assert np.abs(Th1 / dpi1 - 300.0).max() <= 1e-9


def test_nh_column_solve_satisfies_its_equations():
    """The implicit solution satisfies the linearised acoustic equations:
    phi = phi* + g dt w and w_k = w*_k + g dt ((p_k - p_{k-1})/dpi^_k - 1), with
    p_k = p*_k + (dp/d dphi)_k (dphi_k - dphi*_k) and dp/d dphi from a centred
    finite difference of the equation of state (Eq. 9); w = 0 at the lid and surface."""
    from oracle import OracleMesh as _OM  # noqa: F401
    import oracle.pyoracle as po
    K = 20
    r = np.random.default_rng(12)
    dsig = np.diff(ic.sigma_interfaces(K))
    dpi = (1.0e5 - 1000.0) * dsig
    pmid = 1000.0 + (1.0e5 - 1000.0) * (np.cumsum(dsig) - 0.5 * dsig)
    T = 300.0 + 5.0 * r.standard_normal(K)
    dphi = po.RD * T / pmid * dpi
    phis = np.concatenate([np.cumsum(dphi[::-1])[::-1], [0.0]]) + 50.0 * np.concatenate([r.standard_normal(K), [0.0]])
    theta = 300.0 * (1.0e5 / pmid) ** (po.RD / po.CP) * (1 + 0.01 * r.standard_normal(K))
    Th = theta * dpi
    ws = np.concatenate([[0.0], 0.5 * r.standard_normal(K - 1), [0.0]])
    dts = 40.0

    class _M:  # the column solve needs no mesh
        pass
    om = OracleMesh.__new__(OracleMesh)
    om.lib = po.oracle_lib()
    w, phi = om.nh_column_solve(Th, dpi, ws, phis, dts)
    g = po.GRAV
    gam = po.CP / (po.CP - po.RD)
    eos = lambda Thk, d: po.P0 * (po.RD * Thk / (po.P0 * d)) ** gam
    assert w[0] == 0.0 and w[K] == 0.0
    assert np.allclose(phi, phis + g * dts * w, rtol=1e-15, atol=1e-9)
    dphis = phis[:-1] - phis[1:]
    dphin = phi[:-1] - phi[1:]
    pst = eos(Th, dphis)
    h = 1e-6 * dphis
    dpdd = (eos(Th, dphis + h) - eos(Th, dphis - h)) / (2 * h)
    plin = pst + dpdd * (dphin - dphis)
    dh = 0.5 * (dpi[:-1] + dpi[1:])
    want = ws[1:K] + g * dts * ((plin[1:] - plin[:-1]) / dh - 1.0)
    assert np.allclose(w[1:K], want, rtol=0, atol=1e-6 * np.abs(want).max())


def test_ndc_hydrostatic_limit_matches_hdc(mesh_cache):
    """A hydrostatically balanced NH state (delta phi from alpha dpi, w = 0) has
    mu = dp/dpi = 1 and the same PGF as the hydrostatic model, so one short step of
    both dycores agrees closely on the large-scale jet."""
    m = mesh_cache(4)
    om = OracleMesh(m)
    K = 10
    s = ic.hdc_jet(m, K, pert=0.0)
    sig = ic.sigma_interfaces(K)
    dpi = np.outer(s["ps"] - 1000.0, np.diff(sig))
    p = 1000.0 + np.outer(s["ps"] - 1000.0, 0.5 * (sig[:-1] + sig[1:]))
    theta = s["Theta"] / dpi
    alpha = 287.0 * theta * (p / 1.0e5) ** (287.0 / 1004.5) / p
    phi = np.zeros((om.N, K + 1))
    for k in range(K - 1, -1, -1):
        phi[:, k] = phi[:, k + 1] + alpha[:, k] * dpi[:, k]
    w = np.zeros((om.N, K + 1))
    dt = 60.0
    psh, Thh, uh = om.hdc_run(s["ps"], s["Theta"], s["u"], dt, 1)
    psn, Thn, un, wn, phin = om.ndc_run(s["ps"], s["Theta"], s["u"], w, phi, dt, 1)
    du = np.abs(uh - s["u"]).max()
    assert du > 1e-6
    assert np.abs(un - uh).max() <= 1e-3 * du
    assert np.abs(psn - psh).max() <= 1e-9 * s["ps"].max()


def test_momentum_vertical_advection_conserves_kinetic_energy(mesh_cache):
    """The vertical part of the momentum tendency, recovered by removing the
    Coriolis and kinetic-energy-gradient terms (built from the pinned single
    operators), conserves the column kinetic energy together with the vertical
    mass-flux divergence:  sum_k dpi_k u_k V_k + 1/2 sum_k u_k^2 (m_{k+1} - m_k) = 0
    for every edge column (V the vertical advection, m the interface mass flux
    averaged to the edge).  For u increasing downwards and m > 0 the term
    lowers u (it carries slower air down)."""
    m = mesh_cache(3)
    om = OracleMesh(m)
    K = 8
    r = np.random.default_rng(13)
    s = ic.hdc_jet(m, K, pert=0)
    u = 5.0 * r.standard_normal((om.E, 1)) + 2.0 * np.arange(K)[None, :] + 3.0 * r.standard_normal((om.E, K))
    sig = ic.sigma_interfaces(K)
    ps = s["ps"] + 500.0 * r.standard_normal(om.N)
    dps, dTh, du, md = om.hdc_tendency(ps, s["Theta"], u)
    dpi = np.outer(ps - 1000.0, np.diff(sig))
    c1, c2 = m["cells_on_edge"].T
    dpie = 0.5 * (dpi[c1] + dpi[c2])
    F = dpie * u
    zeta = om.curl(u)
    qv = (zeta + m["fVertex"][:, None]) / om.vertex_mass(dpi)
    Q = om.coriolis(F, qv)
    ke = om.kinetic_energy(u)
    gk = (ke[c2] - ke[c1]) / m["dEdge"][:, None]
    V = Q - gk - du                                 # vertical advection of u
    me = 0.5 * (md[c1] + md[c2])                    # [E][K+1]
    lhs = (dpie * u * V).sum(1) + 0.5 * (u * u * (me[:, 1:] - me[:, :-1])).sum(1)
    scale = (np.abs(dpie * u * V).sum(1) + 0.5 * np.abs(u * u * (me[:, 1:] - me[:, :-1])).sum(1))
    assert np.abs(lhs).max() <= 1e-9 * scale.max()
    assert np.abs(V).max() > 1e-6
    # direction: interior level with m > 0 above and below and u increasing with k
    du_dk_pos = (u[:, 2:] > u[:, 1:-1]) & (u[:, 1:-1] > u[:, :-2])
    down = (me[:, 1:-2] > 0) & (me[:, 2:-1] > 0)
    sel = du_dk_pos & down
    assert sel.sum() > 10 and np.all(V[:, 1:-1][sel] > 0)
