"""Pins of the oracle's total-energy diagnostic (Section 2.2 diagnostics of a
run; kinetic + internal + potential energy of every layer's mass) against
closed forms and exact identities (CPU)."""
import numpy as np
import pytest

from oracle import OracleMesh
from paper_2404_08849_amd.inputs import initial as ic
from paper_2404_08849_amd.inputs.initial import velocity_from_streamfunction

G, RD, CP, P0, PT = 9.80616, 287.0, 1004.5, 1.0e5, 1000.0
CV = CP - RD


def _sphere(m):
    return 4.0 * np.pi * m["radius"] ** 2


def test_shallow_water_rest_state_is_exact(mesh_cache):
    """h = h0, u = 0, b = 0: E = sum A h0 g h0/2 = g h0^2/2 times the sphere's area."""
    m = mesh_cache(3)
    om = OracleMesh(m)
    h0 = 2.94e4 / G
    e = om.energy("SW", np.full(om.N, h0), np.zeros(om.E), b=np.zeros(om.N))
    assert abs(e - 0.5 * G * h0 ** 2 * _sphere(m)) <= 1e-13 * e


def test_shallow_water_kinetic_energy_converges(mesh_cache):
    """u = u0 cos(lat) over a flat h0: E - E_rest = h0 sum A K -> h0 u0^2/2 *
    integral of cos^2(lat) over the sphere = h0 u0^2/2 (2/3) 4 pi a^2."""
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        h0, u0 = 1000.0, 30.0
        latv = np.arcsin(m["xVertex"][:, 2])
        u = velocity_from_streamfunction(m, -m["radius"] * u0 * np.sin(latv))
        h, b = np.full(om.N, h0), np.zeros(om.N)
        ek = om.energy("SW", h, u, b=b) - om.energy("SW", h, np.zeros(om.E), b=b)
        exact = h0 * 0.5 * u0 ** 2 * (2.0 / 3.0) * _sphere(m)
        errs.append(abs(ek - exact) / exact)
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 1e-2, errs


def _isothermal(m, K, T0=300.0, ps=1.0e5):
    sig = ic.sigma_interfaces(K)
    smid = 0.5 * (sig[:-1] + sig[1:])
    dpi = np.outer(np.full(m["nCells"], ps - PT), np.diff(sig))
    p = PT + np.outer(np.full(m["nCells"], ps - PT), smid)
    Theta = dpi * T0 * (P0 / p) ** (RD / CP)
    return np.full(m["nCells"], ps), Theta


def test_hydrostatic_isothermal_column_converges_to_closed_form(mesh_cache):
    """Isothermal T0 at rest between pi_t and pi_s: internal energy c_v T0 (pi_s -
    pi_t)/g per unit area, and with phi(p) = R T0 ln(pi_s/p),
    int phi dp = R T0 (pi_s - pi_t - pi_t ln(pi_s/pi_t)); so
    E = 4 pi a^2 [c_p T0 (pi_s - pi_t) - R T0 pi_t ln(pi_s/pi_t)] / g.
    The discrete sum approaches it as the layers are refined."""
    m = mesh_cache(2)
    om = OracleMesh(m)
    T0, ps = 300.0, 1.0e5
    exact = _sphere(m) * (CP * T0 * (ps - PT) - RD * T0 * PT * np.log(ps / PT)) / G
    errs = []
    for K in (10, 20, 40, 80):
        p_s, Th = _isothermal(m, K, T0, ps)
        errs.append(abs(om.energy("HDC", p_s, np.zeros((om.E, K)), Theta=Th) - exact) / exact)
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] <= 1e-3 and errs[-2] / errs[-1] > 1.5, errs


def test_hydrostatic_terrain_shifts_potential_energy(mesh_cache):
    """A uniform surface geopotential Phi raises every layer's geopotential by
    Phi: E grows by Phi (pi_s - pi_t) 4 pi a^2 / g."""
    m = mesh_cache(2)
    om = OracleMesh(m)
    K, Phi = 12, 4000.0
    ps, Th = _isothermal(m, K)
    u = np.zeros((om.E, K))
    e0 = om.energy("HDC", ps, u, Theta=Th)
    e1 = om.energy("HDC", ps, u, Theta=Th, phis=np.full(om.N, Phi))
    exact = Phi * (1.0e5 - PT) * m["areaCell"].sum() / G
    assert abs((e1 - e0) - exact) <= 1e-12 * e0


def test_nonhydrostatic_rest_state_matches_hydrostatic(mesh_cache):
    """The NH rest state in discrete hydrostatic balance (the equation of state
    returns the mid-layer pressure, dphi = R T0 dpi / p) has the hydrostatic
    energy of the same (pi_s, Theta); a uniform w = c adds c^2/2 (pi_s - pi_t)
    4 pi a^2 / g of vertical kinetic energy."""
    m = mesh_cache(2)
    om = OracleMesh(m)
    K = 16
    s = ic.nh_warm_bubble(m, K, dtheta=0.0)
    eh = om.energy("HDC", s["ps"], s["u"], Theta=s["Theta"])
    en = om.energy("NDC", s["ps"], s["u"], Theta=s["Theta"], w=s["w"], phi=s["phi"])
    assert abs(en - eh) <= 1e-13 * eh
    c = 3.0
    ew = om.energy("NDC", s["ps"], s["u"], Theta=s["Theta"], w=np.full_like(s["w"], c), phi=s["phi"])
    exact = 0.5 * c * c * (1.0e5 - PT) * m["areaCell"].sum() / G
    assert abs((ew - en) - exact) <= 1e-12 * en
