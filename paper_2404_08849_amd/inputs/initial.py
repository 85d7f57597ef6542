"""Seeded analytic initial states on an icosahedral mesh (input generators).

Every state is built on the host in FP64 and handed identically to the CPU
oracle and to the GPU library (the paper keeps model initialisation in
double precision and converts to single only inside the solver, Section
2.2).  The paper's own test cases (DCMIP2016, Reed-Jablonowski, AMIP and the
real-data run of Section 4) need physics and data that are out of scope;
the analytic states below stand in for them at the paper's grid sizes
(Table 1).  Seeds: workload c uses base seed 1000*c; ensemble member m adds
m, tracer t adds 100*t (SplitMix64, see ``rng``).

Layouts are level-innermost: cell fields [N][K], edge fields [E][K],
interface fields [N][K+1], tracers [N][K][T], ensembles [..][K][M].
"""
import numpy as np

from . import rng
from .meshgen import lonlat

GRAV = 9.80616
RD = 287.0
CP = 1004.5
P0 = 1.0e5
PTOP = 1000.0
KAPPA = RD / CP


def sigma_interfaces(K):
    """Uniform pure-sigma interfaces 0 = sigma_0 < ... < sigma_K = 1 (top to bottom)."""
    return np.arange(K + 1, dtype=np.float64) / K


def _great_circle(x, lon0, lat0):
    c = np.array([np.cos(lat0) * np.cos(lon0), np.cos(lat0) * np.sin(lon0), np.sin(lat0)])
    return np.arctan2(np.linalg.norm(np.cross(x, c), axis=1), x @ c)


def _edge_normal(mesh):
    xc = mesh["xCell"]
    c1, c2 = mesh["cells_on_edge"][:, 0], mesh["cells_on_edge"][:, 1]
    n = xc[c2] - xc[c1]
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _east(x):
    e = np.stack([-x[:, 1], x[:, 0], np.zeros(len(x))], 1)
    return e / np.maximum(np.linalg.norm(e, axis=1, keepdims=True), 1e-300)


def velocity_from_streamfunction(mesh, psi_v):
    """Normal velocity u_e = -(psi_v2 - psi_v1) / l_e (V = k x grad psi)."""
    v = mesh["vertices_on_edge"]
    return -(psi_v[v[:, 1]] - psi_v[v[:, 0]]) / mesh["lEdge"]


def _seeded_centre(seed, lat_max_deg):
    u = rng.uniform(seed, 2)
    lon = 2.0 * np.pi * u[0]
    lat = np.deg2rad(-lat_max_deg + 2.0 * lat_max_deg * u[1])
    return lon, lat


def sw_geostrophic(mesh, u0=38.6, gh0=2.94e4, bump=1.0, bump_radius=1.0e6, seed=1000):
    """Shallow-water steady zonal geostrophic flow plus a seeded Gaussian height bump.

    u = u0 cos(lat) from psi = -a u0 sin(lat); g h = g h0 - (a Omega u0 + u0^2/2) sin^2(lat).
    Returns dict(h[N], u[E], b[N]).
    """
    a, om = mesh["radius"], mesh["omega"]
    _, latc = lonlat(mesh["xCell"])
    _, latv = lonlat(mesh["xVertex"])
    psi = -a * u0 * np.sin(latv)
    u = velocity_from_streamfunction(mesh, psi)
    h = (gh0 - (a * om * u0 + 0.5 * u0 * u0) * np.sin(latc) ** 2) / GRAV
    if bump:
        lon0, lat0 = _seeded_centre(seed, 60.0)
        r = a * _great_circle(mesh["xCell"], lon0, lat0)
        h = h + bump * np.exp(-(r / bump_radius) ** 2)
    return dict(h=h, u=u, b=np.zeros_like(h))


def hdc_jet_surface_pressure(lat, a, om, u0=35.0, T0=300.0, p_eq=1.0e5):
    """Surface pressure of the isothermal barotropic jet u = u0 cos^2(lat) in gradient-wind balance."""
    gam = lambda p: (2.0 * om * a * u0 / 3.0) * np.cos(p) ** 3 + 0.25 * u0 * u0 * np.cos(p) ** 4
    return p_eq * np.exp((gam(lat) - gam(0.0)) / (RD * T0))


def hdc_jet(mesh, K, u0=35.0, T0=300.0, pert=1.0, seed=2000):
    """Hydrostatic isothermal jet u = u0 cos^2(lat), balanced surface pressure,
    plus a seeded zonal wind bump pert*exp(-(r/(a/10))^2) at every level.

    Returns dict(ps[N], Theta[N][K], u[E][K]).
    """
    a, om = mesh["radius"], mesh["omega"]
    _, latc = lonlat(mesh["xCell"])
    _, latv = lonlat(mesh["xVertex"])
    ps = hdc_jet_surface_pressure(latc, a, om, u0, T0)
    psi = -a * u0 * (0.5 * latv + 0.25 * np.sin(2.0 * latv))
    u1 = velocity_from_streamfunction(mesh, psi)
    if pert:
        lon0, lat0 = _seeded_centre(seed, 60.0)
        xe = mesh["xEdge"]
        r = a * _great_circle(xe, lon0, lat0)
        u1 = u1 + pert * np.exp(-(r / (a / 10.0)) ** 2) * np.einsum("ij,ij->i", _east(xe), _edge_normal(mesh))
    sig = sigma_interfaces(K)
    smid = 0.5 * (sig[:-1] + sig[1:])
    dsig = np.diff(sig)
    dpi = np.outer(ps - PTOP, dsig)
    p = PTOP + np.outer(ps - PTOP, smid)
    theta = T0 * (P0 / p) ** KAPPA
    u = np.repeat(u1[:, None], K, axis=1)
    return dict(ps=ps, Theta=dpi * theta, u=np.ascontiguousarray(u))


def baroclinic_jet_profile(x, x_jet=np.log(4.0)):
    """Vertical shape s(x) of the baroclinic jet, x = ln(p0/p): zero at the
    surface, 1 at the jet level x_jet, decaying above; returns (s, ds/dln p)."""
    c = np.exp(0.5) / x_jet
    g = np.exp(-0.5 * (x / x_jet) ** 2)
    s = c * x * g
    ds_dx = c * g * (1.0 - (x / x_jet) ** 2)
    return s, -ds_dx


def baroclinic_jet_terms(lat, a, om, u0):
    """Gamma(lat) = int_0^lat 2 Omega a sin U and Delta(lat) = int_0^lat U^2 tan
    for U = u0 sin^2(2 lat), in closed form (c = cos lat)."""
    c = np.cos(lat)
    gam = 2.0 * om * a * 4.0 * u0 * (-c ** 3 / 3.0 + c ** 5 / 5.0 + 2.0 / 15.0)
    dlt = 16.0 * u0 * u0 * (-(c ** 4 / 4.0 - c ** 6 / 3.0 + c ** 8 / 8.0) + 1.0 / 24.0)
    return gam, dlt


def baroclinic_reference_temperature(p, T_s=288.0, lapse=0.005, T_trop=220.0, p_s=1.0e5):
    """Latitude-independent reference profile T_0(p): a constant lapse rate
    (K/m) from T_s at p_s, isothermal at T_trop above the tropopause."""
    return np.maximum(T_s * (p / p_s) ** (RD * lapse / GRAV), T_trop)


def baroclinic_jet_temperature(lat, p, a, om, u0=30.0, p_s=1.0e5):
    """Temperature of the baroclinic jet u = u0 sin^2(2 lat) s(ln(p_s/p)) in
    gradient-wind and hydrostatic balance over a flat surface at p_s.

    On pressure surfaces the geopotential is Phi = Phi_0(p) - Gamma s
    - Delta s^2 (Phi_0: the reference profile's geopotential, independent of
    latitude), whose latitude derivative is minus the gradient-wind term
    (2 Omega a sin lat u + u^2 tan lat); the hydrostatic relation
    dPhi/dln p = -R_d T then gives T = T_0(p) + (ds/dln p)(Gamma + 2 s Delta)/R_d."""
    s, sl = baroclinic_jet_profile(np.log(p_s / p))
    gam, dlt = baroclinic_jet_terms(lat, a, om, u0)
    return baroclinic_reference_temperature(p, p_s=p_s) + sl * (gam + 2.0 * s * dlt) / RD


def hdc_baroclinic_jet(mesh, K, u0=30.0, pert=1.0, seed=2000):
    """Hydrostatic baroclinic jet: zonal wind u0 sin^2(2 lat) s(p), zero at the
    surface and strongest near 250 hPa, in gradient-wind and thermal-wind
    balance with the temperature of baroclinic_jet_temperature over a flat
    surface at 1000 hPa (so pi_s is uniform; the reference profile has a
    5 K/km lapse rate from 288 K up to a 220 K tropopause), plus a seeded zonal wind bump
    pert*exp(-(r/(a/10))^2) scaled by s(p), which starts the baroclinic wave.
    Mid-latitude jets of both hemispheres; the poles are cold at the surface.

    Returns dict(ps[N], Theta[N][K], u[E][K])."""
    a, om = mesh["radius"], mesh["omega"]
    N = mesh["nCells"]
    _, latc = lonlat(mesh["xCell"])
    _, latv = lonlat(mesh["xVertex"])
    ps = np.full(N, P0)
    sig = sigma_interfaces(K)
    smid = 0.5 * (sig[:-1] + sig[1:])
    dpi = np.outer(ps - PTOP, np.diff(sig))
    p = PTOP + np.outer(ps - PTOP, smid)
    T = baroclinic_jet_temperature(latc[:, None], p, a, om, u0, P0)
    theta = T * (P0 / p) ** KAPPA
    # U = u0 sin^2(2 lat) = u0 (1 - cos 4 lat)/2 from psi = -a int U
    psi = -a * u0 * (0.5 * latv - np.sin(4.0 * latv) / 8.0)
    u1 = velocity_from_streamfunction(mesh, psi)
    if pert:
        lon0, lat0 = _seeded_centre(seed, 60.0)
        xe = mesh["xEdge"]
        r = a * _great_circle(xe, lon0, lat0)
        u1 = u1 + pert * np.exp(-(r / (a / 10.0)) ** 2) * np.einsum("ij,ij->i", _east(xe), _edge_normal(mesh))
    s_k, _ = baroclinic_jet_profile(np.log(P0 / (PTOP + (P0 - PTOP) * smid)))
    u = np.outer(u1, s_k)
    return dict(ps=ps, Theta=dpi * theta, u=np.ascontiguousarray(u))


def ensemble(state, M, sigma=0.1, seed=5000, relative=None):
    """Stack M copies of a hydrostatic state member-innermost, with independent
    N(0, sigma) perturbations on every u_{e,k} of member m (seed + m), or, if
    relative is given, u scaled by 1 + U(-relative, relative) (the paper's
    perturbation "within 2%" of the wind is relative = 0.02)."""
    ps, Th, u = state["ps"], state["Theta"], state["u"]
    E, K = u.shape
    um = np.empty((E, K, M))
    for m in range(M):
        if relative is None:
            um[:, :, m] = u + sigma * rng.normal(seed + m, E * K).reshape(E, K)
        else:
            um[:, :, m] = u * (1.0 + relative * (2.0 * rng.uniform(seed + m, E * K).reshape(E, K) - 1.0))
    return dict(ps=np.repeat(ps[:, None], M, 1), Theta=np.repeat(Th[:, :, None], M, 2), u=um)


def nh_warm_bubble(mesh, K, T0=300.0, dtheta=1.0, rh=2.0e5, zc=2.0e3, rz=2.0e3, seed=4000):
    """Isothermal atmosphere at rest in discrete hydrostatic balance plus a seeded
    warm bubble added to Theta.

    Balance: p_k equals the hydrostatic mid-layer pressure and the layer
    thickness is delta phi_k = (R_d T0 / p_k) delta pi_k, so the equation of
    state returns p_k exactly.  Returns dict(ps, Theta, u, w[N][K+1], phi[N][K+1]).
    """
    N, E = mesh["nCells"], mesh["nEdges"]
    a = mesh["radius"]
    ps = np.full(N, 1.0e5)
    sig = sigma_interfaces(K)
    smid = 0.5 * (sig[:-1] + sig[1:])
    dpi = np.outer(ps - PTOP, np.diff(sig))
    p = PTOP + np.outer(ps - PTOP, smid)
    theta = T0 * (P0 / p) ** KAPPA
    dphi = RD * T0 / p * dpi
    phi = np.zeros((N, K + 1))
    for k in range(K - 1, -1, -1):
        phi[:, k] = phi[:, k + 1] + dphi[:, k]
    Theta = dpi * theta
    if dtheta:
        lon0, lat0 = _seeded_centre(seed, 60.0)
        r = a * _great_circle(mesh["xCell"], lon0, lat0)
        z = 0.5 * (phi[:, :-1] + phi[:, 1:]) / GRAV
        rho = np.sqrt((r[:, None] / rh) ** 2 + ((z - zc) / rz) ** 2)
        bub = np.where(rho <= 1.0, dtheta * np.cos(0.5 * np.pi * rho) ** 2, 0.0)
        Theta = Theta + dpi * bub
    return dict(ps=ps, Theta=Theta, u=np.zeros((E, K)), w=np.zeros((N, K + 1)), phi=phi)


def ndc_rest_over_terrain(mesh, K, phis, T0=300.0, p_ref=1.0e5):
    """Non-hydrostatic isothermal atmosphere at rest over terrain, in discrete
    hydrostatic balance: pi_s and Theta as hdc_rest_over_terrain, the
    geopotential integrated upwards from the surface value phis with
    delta phi_k = (R_d T0 / p_k) delta pi_k (so the equation of state returns
    the hydrostatic mid-layer pressure p_k), w = 0.  The bottom interface of
    phi is the surface geopotential.
    Returns dict(ps, Theta, u, w[N][K+1], phi[N][K+1])."""
    s = hdc_rest_over_terrain(mesh, K, phis, T0, p_ref)
    ps = s["ps"]
    sig = sigma_interfaces(K)
    dpi = np.outer(ps - PTOP, np.diff(sig))
    p = PTOP + np.outer(ps - PTOP, 0.5 * (sig[:-1] + sig[1:]))
    dphi = RD * T0 / p * dpi
    N = mesh["nCells"]
    phi = np.zeros((N, K + 1))
    phi[:, K] = phis
    for k in range(K - 1, -1, -1):
        phi[:, k] = phi[:, k + 1] + dphi[:, k]
    return dict(ps=ps, Theta=s["Theta"], u=s["u"], w=np.zeros((N, K + 1)), phi=phi)


def solid_body_wind(mesh, K, u0=20.0, axis=(0.0, 0.0, 1.0)):
    """Solid-body rotation of speed u0 at the equator of the rotation axis,
    the same at every level, as normal velocities [E][K] from its
    streamfunction psi = -a u0 (axis . x) at the vertices (nondivergent)."""
    ax = np.asarray(axis, dtype=np.float64)
    ax = ax / np.linalg.norm(ax)
    psi = -mesh["radius"] * u0 * (mesh["xVertex"] @ ax)
    u1 = velocity_from_streamfunction(mesh, psi)
    return np.ascontiguousarray(np.repeat(u1[:, None], K, axis=1))


def _harmonics_deg3(x):
    """The 16 real spherical harmonics of degree <= 3 as Cartesian polynomials (unnormalised)."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return np.stack([
        np.ones_like(X),
        X, Y, Z,
        X * Y, Y * Z, Z * X, X * X - Y * Y, 3 * Z * Z - 1,
        X * (X * X - 3 * Y * Y), Y * (3 * X * X - Y * Y), Z * (X * X - Y * Y), X * Y * Z,
        X * (5 * Z * Z - 1), Y * (5 * Z * Z - 1), Z * (5 * Z * Z - 3),
    ], 1)


def cosine_bell(mesh, lon0=1.5 * np.pi, lat0=0.0, rb_frac=1.0 / 3.0):
    """0.5 (1 + cos(pi r / R_b)) inside r < R_b = a/3, else 0."""
    a = mesh["radius"]
    r = a * _great_circle(mesh["xCell"], lon0, lat0)
    rb = rb_frac * a
    return np.where(r < rb, 0.5 * (1.0 + np.cos(np.pi * r / rb)), 0.0)


def tracer_solid_body(mesh, K, T, days=12.0, tilt_deg=45.0, ps=1.0e5, seed=3000):
    """Prescribed nondivergent FP64 mass flux of tilted solid-body rotation plus tracers.

    F_{e,k} = dpi_k u_e with u_e from psi = -a u0 (sin(lat) cos(al) - cos(lon) cos(lat) sin(al)),
    u0 = 2 pi a / (12 days).  Tracer 0 is the cosine bell; tracers 1..T-1 at each level are
    sum_j c_j Y_j (c_j ~ N(0,1), seed + 100 t) rescaled to [0, 1] over the cells.
    Returns dict(F[E][K], dpi[N][K], q[N][K][T], u0, period).
    """
    a = mesh["radius"]
    period = days * 86400.0
    u0 = 2.0 * np.pi * a / period
    al = np.deg2rad(tilt_deg)
    lonv, latv = lonlat(mesh["xVertex"])
    psi = -a * u0 * (np.sin(latv) * np.cos(al) - np.cos(lonv) * np.cos(latv) * np.sin(al))
    ue = velocity_from_streamfunction(mesh, psi)
    N = mesh["nCells"]
    sig = sigma_interfaces(K)
    dpi1 = (ps - PTOP) * np.diff(sig)
    F = np.ascontiguousarray(ue[:, None] * dpi1[None, :])
    dpi = np.ascontiguousarray(np.repeat(dpi1[None, :], N, 0))
    q = np.empty((N, K, T))
    if T > 0:
        q[:, :, 0] = cosine_bell(mesh)[:, None]
    Y = _harmonics_deg3(mesh["xCell"])
    for t in range(1, T):
        c = rng.normal(seed + 100 * t, 16 * K).reshape(K, 16)
        f = Y @ c.T                                    # [N][K]
        lo, hi = f.min(0, keepdims=True), f.max(0, keepdims=True)
        q[:, :, t] = (f - lo) / (hi - lo)
    return dict(F=F, dpi=dpi, q=q, u0=u0, period=period)


def tracer_vertical_flux(dpi, dt, amp=0.3, seed=3100):
    """Synthetic interface mass flux [N][K+1] (positive towards the surface,
    zero at the lid and the surface) that changes each layer mass over dt by
    a random fraction of at most about amp: dt (m_{k+1} - m_k) = amp xi_k dpi_k
    with xi uniform in [-1, 1] and sum_k xi_k dpi_k = 0 per column.  The
    Courant numbers of the interior interfaces reach about amp K / 2."""
    r = np.random.default_rng(seed)
    dpi = np.asarray(dpi, dtype=np.float64)
    N, K = dpi.shape
    xi = r.uniform(-1.0, 1.0, (N, K))
    xi -= ((xi * dpi).sum(1) / dpi.sum(1))[:, None]          # zero column sum of xi dpi
    xi /= np.maximum(np.abs(xi).max(1), 1e-300)[:, None]      # |xi| <= 1 again
    m = np.zeros((N, K + 1))
    m[:, 1:] = np.cumsum(amp * xi * dpi, axis=1) / dt
    m[:, K] = 0.0
    return m


def mountain(mesh, h0=3000.0, radius=1.5e6, lon0=0.5 * np.pi, lat0=np.pi / 6.0):
    """Surface geopotential [N] of an isolated mountain of height h0 (m):
    g h0 cos^2(pi r / (2 radius)) within radius of (lon0, lat0), 0 outside."""
    r = mesh["radius"] * _great_circle(mesh["xCell"], lon0, lat0)
    h = np.where(r < radius, h0 * np.cos(0.5 * np.pi * r / radius) ** 2, 0.0)
    return GRAV * h


def hdc_rest_over_terrain(mesh, K, phis, T0=300.0, p_ref=1.0e5):
    """Isothermal atmosphere at rest over terrain: pi_s = p_ref exp(-phis / (R_d T0))
    (hydrostatic balance of the continuous equations), theta at the layer
    midpoints such that T = T0 there, u = 0.  Returns dict(ps[N], Theta[N][K], u[E][K])."""
    ps = p_ref * np.exp(-np.asarray(phis) / (RD * T0))
    sig = sigma_interfaces(K)
    smid = 0.5 * (sig[:-1] + sig[1:])
    dpi = np.outer(ps - PTOP, np.diff(sig))
    p = PTOP + np.outer(ps - PTOP, smid)
    theta = T0 * (P0 / p) ** KAPPA
    return dict(ps=ps, Theta=dpi * theta, u=np.zeros((mesh["nEdges"], K)))
