"""GPU parity of the non-hydrostatic dycore over terrain, and the precision
sensitivity of its pressure-gradient term there (Section 2.3, Section 4).

The bottom interface of phi is the surface geopotential phi_s: it stays
fixed, and w there is the kinematic value g w_s = V.grad phi_s of the stage's
flow (Eq. 7 at the surface).  A solid-body wind over a 3 km mountain, on an
isothermal atmosphere in discrete hydrostatic balance over the terrain,
runs 10 steps against the oracle with the usual bars: all-FP64 1e-12
(pi_s, Theta, phi) and the element-wise bounds of the cancelling terms (w,
u); mixed 1e-5, 16 FP32 unit roundoffs per 10 steps for u, and for w, a
hundred times weaker than the wind here, the same bar of the flow speed
(gpu_helpers.mix_w_bar).  The surface keeps
phi_s bitwise and its w follows the flow.  MIX_PGF32 (the FP32 equation of
state, column solve and pressure-gradient term) is then held to being far
less accurate than MIX over the mountain.
"""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import (MIX_TOL, MIX_U_TOL, compare, compare_abs, compare_dbl, gpu_ndc, mix_w_bar,
                         nh_dbl_bounds, rel_l2)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpdc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_08849_amd.mpdc as m
    return m


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    return oracle


def _say(*a):
    print(*a, flush=True)


def _wind_over_mountain(m, K, u0=15.0, flat=False):
    phis = np.zeros(m["nCells"]) if flat else ic.mountain(m)
    s = ic.ndc_rest_over_terrain(m, K, phis)
    s["u"] = ic.solid_body_wind(m, K, u0, (0.0, 0.0, 1.0))
    return phis, s


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_nh_terrain_parity_g4(mpdc, oracle_mod, mesh_cache, policy):
    m = mesh_cache(4)
    K, dt, n = 8, 120.0, 10
    phis, s = _wind_over_mountain(m, K)
    om = oracle_mod.OracleMesh(m)
    ref = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], dt, n)
    g = mpdc.Mesh(m)
    _say("ndc G4x%d, solid-body wind over a 3 km mountain, %d steps" % (K, n), policy)
    st, (ps, Th, u, w, phi) = gpu_ndc(mpdc, g, s, K, dt, n, getattr(mpdc, "POLICY_" + policy))
    A = m["areaCell"]
    if policy == "DBL":
        bw, bu = nh_dbl_bounds(ref[4], 9.80616, dt, n, float(m["dEdge"].min()))
        compare_dbl("ps", ps, ref[0], A)
        compare_dbl("Theta", Th, ref[1], A)
        compare_dbl("phi", phi, ref[4], A)
        compare_abs("w", w, ref[3], bw)
        compare_abs("u", u, ref[2], bu)
    else:
        compare("ps", ps, ref[0], A, MIX_TOL, MIX_TOL)
        compare("Theta", Th, ref[1], A, MIX_TOL, MIX_TOL)
        compare("phi", phi, ref[4], A, MIX_TOL, MIX_TOL)
        compare("u", u, ref[2], None, MIX_U_TOL, MIX_U_TOL)
        compare_abs("w", w, ref[3], mix_w_bar(ref[2], ref[3], n))
    # the surface: phi_s kept bitwise; w follows the flow over the slopes only
    assert np.array_equal(phi[:, K], phis)
    ws, wr = w[:, K], ref[3][:, K]
    _say("    surface w: max %.3e, oracle %.3e" % (np.abs(ws).max(), np.abs(wr).max()))
    assert np.abs(wr).max() > 1e-3 and np.all(ws[wr == 0.0] == 0.0)
    # the terrain acted: the same wind over a flat surface gives another flow
    _, sf = _wind_over_mountain(m, K, flat=True)
    st2, flat = gpu_ndc(mpdc, g, sf, K, dt, n, getattr(mpdc, "POLICY_" + policy))
    assert rel_l2(flat[2], u) > 1e-3 and np.all(flat[3][:, K] == 0.0)


def test_nh_fp32_pressure_gradient_is_less_accurate(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(5)
    K, dt, n = 10, 60.0, 10
    g = mpdc.Mesh(m)
    phis, s = _wind_over_mountain(m, K)
    ref = oracle_mod.OracleMesh(m).ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], dt, n)
    A = m["areaCell"]
    err = {}
    for pol in ("MIX", "MIX_PGF32"):
        st, (ps, Th, u, w, phi) = gpu_ndc(mpdc, g, s, K, dt, n, getattr(mpdc, "POLICY_" + pol))
        assert np.array_equal(phi[:, K], phis)
        err[pol] = (rel_l2(ps, ref[0], A), rel_l2(u, ref[2]), rel_l2(w, ref[3], A), rel_l2(phi, ref[4], A))
        _say("ndc G5x%d wind over a mountain, %d steps, %s: ps %.3e  u %.3e  w %.3e  phi %.3e"
             % ((K, n, pol) + err[pol]))
        if pol == "MIX":
            compare("u MIX", u, ref[2], None, MIX_U_TOL, MIX_U_TOL)
            compare_abs("w MIX", w, ref[3], mix_w_bar(ref[2], ref[3], n))
    # the FP32 column solve and force: u and w over 8x less accurate
    assert err["MIX_PGF32"][1] > 8.0 * err["MIX"][1] and err["MIX_PGF32"][2] > 8.0 * err["MIX"][2]


def test_surface_w_follows_the_written_surface(mpdc, mesh_cache):
    """The kinematic surface w is formed once the written phi has terrain (from
    host or device memory) and is exactly zero after a flat surface is written."""
    import torch
    m = mesh_cache(3)
    K, dt = 6, 240.0
    phis, s = _wind_over_mountain(m, K)
    _, sf = _wind_over_mountain(m, K, flat=True)
    g = mpdc.Mesh(m)

    def run(phi_writes):
        st = mpdc.State(g, mpdc.MODEL_NDC, mpdc.POLICY_DBL, K=K, M=1, dt=dt, sigma=ic.sigma_interfaces(K))
        st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
        st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
        st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
        st.state_write(mpdc.FIELD_W, s["w"][:, :, None])
        for phi in phi_writes:
            st.state_write(mpdc.FIELD_PHI, phi)
        st.dycore_step(1)
        return st.state_read(mpdc.FIELD_W)[:, K, 0]

    host = run([s["phi"][:, :, None]])
    assert np.abs(host).max() > 1e-3
    flat_after = run([s["phi"][:, :, None], sf["phi"][:, :, None]])
    assert np.array_equal(flat_after, np.zeros(m["nCells"]))
    dev = run([sf["phi"][:, :, None], torch.from_numpy(s["phi"][:, :, None].copy()).cuda()])
    assert np.array_equal(dev, host)
