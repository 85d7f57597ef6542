"""GPU parity of the hydrostatic dycore over terrain, and the precision
sensitivity of its pressure-gradient term (Section 2.3).

With a surface geopotential the hydrostatic geopotential starts from phi_s
(Eq. 8).  DBL and MIX are held to the usual bars against the oracle.  The
variant MIX_PGF32 computes the column diagnostics and the pressure-gradient
and gravity term in FP32, as the single-precision model does; after 10 steps
its surface-pressure and wind errors are more than an order of magnitude
above the mixed policy's (measured: 13-15x at G5, over a mountain and over a
flat surface alike -- the rounding of the FP32 geopotential itself dominates
at this length), which is the paper's reason to keep these terms in FP64.
"""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import MIX_TOL, MIX_U_TOL, compare, compare_dbl, rel_l2

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


def _run(mpdc, g, s, K, dt, n, policy, phis, M=1):
    st = mpdc.State(g, mpdc.MODEL_HDC, policy, K=K, M=M, dt=dt, sigma=ic.sigma_interfaces(K))
    st.state_write(mpdc.FIELD_PHIS, phis)
    ex = (lambda x: x[..., None]) if M == 1 else (lambda x: x)
    st.state_write(mpdc.FIELD_PS, ex(s["ps"]))
    st.state_write(mpdc.FIELD_THETA, ex(s["Theta"]))
    st.state_write(mpdc.FIELD_U, ex(s["u"]))
    st.dycore_step(n)
    out = [st.state_read(f) for f in (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U)]
    return [x[..., 0] for x in out] if M == 1 else out


def _jet_over_mountain(m, K):
    phis = ic.mountain(m)
    rest = ic.hdc_rest_over_terrain(m, K, phis)
    jet = ic.hdc_jet(m, K, seed=2000)
    return phis, dict(ps=rest["ps"], Theta=rest["Theta"], u=jet["u"])


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_terrain_parity_g4(mpdc, oracle_mod, mesh_cache, policy):
    m = mesh_cache(4)
    K, dt, n = 10, 600.0, 10
    phis, s = _jet_over_mountain(m, K)
    ref = oracle_mod.OracleMesh(m).hdc_run(s["ps"], s["Theta"], s["u"], dt, n, phis=phis)
    g = mpdc.Mesh(m)
    _say("hdc G4x%d over a 3 km mountain, %d steps" % (K, n), policy)
    ps, Th, u = _run(mpdc, g, s, K, dt, n, getattr(mpdc, "POLICY_" + policy), phis)
    A = m["areaCell"]
    if policy == "DBL":
        compare_dbl("ps", ps, ref[0], A)
        compare_dbl("Theta", Th, ref[1], A)
        compare_dbl("u", u, ref[2])
    else:
        compare("ps", ps, ref[0], A, MIX_TOL, MIX_TOL)
        compare("Theta", Th, ref[1], A, MIX_TOL, MIX_TOL)
        compare("u", u, ref[2], None, MIX_U_TOL, MIX_U_TOL)
    # the terrain acted: the same run on a flat surface differs
    flat = _run(mpdc, g, s, K, dt, n, getattr(mpdc, "POLICY_" + policy), np.zeros(m["nCells"]))
    assert rel_l2(flat[2], u) > 1e-3


def test_terrain_members_share_the_surface(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(3)
    K, M, dt, n = 8, 2, 900.0, 4
    phis, s = _jet_over_mountain(m, K)
    ens = ic.ensemble(s, M, sigma=0.1, seed=5000)
    g = mpdc.Mesh(m)
    om = oracle_mod.OracleMesh(m)
    _say("hdc ensemble G3x%dx%d over a mountain, DBL" % (K, M))
    ps, Th, u = _run(mpdc, g, ens, K, dt, n, mpdc.POLICY_DBL, phis, M=M)
    for j in range(M):
        r = om.hdc_run(ens["ps"][:, j], ens["Theta"][:, :, j], ens["u"][:, :, j], dt, n, phis=phis)
        compare_dbl("ps m%d" % j, ps[:, j], r[0], m["areaCell"])
        compare_dbl("Theta m%d" % j, Th[:, :, j], r[1], m["areaCell"])
        compare_dbl("u m%d" % j, u[:, :, j], r[2])


def test_fp32_pressure_gradient_is_less_accurate(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(5)
    K, dt, n = 10, 300.0, 10
    g = mpdc.Mesh(m)
    om = oracle_mod.OracleMesh(m)
    for case in ("mountain", "flat"):
        phis, s = _jet_over_mountain(m, K)
        if case == "flat":
            phis = np.zeros(m["nCells"])
            s = ic.hdc_jet(m, K, seed=2000)
        ref = om.hdc_run(s["ps"], s["Theta"], s["u"], dt, n, phis=phis)
        res = {}
        for pol in ("MIX", "MIX_PGF32"):
            ps, Th, u = _run(mpdc, g, s, K, dt, n, getattr(mpdc, "POLICY_" + pol), phis)
            if pol == "MIX":
                ps_mix, u_mix = ps, u
            res[pol] = (rel_l2(ps, ref[0], m["areaCell"]), rel_l2(u, ref[2]))
            _say("hdc G5x%d %s, %d steps, %s: ps %.3e  u %.3e" % ((K, case, n, pol) + res[pol]))
        # the mixed policy passes its bars; the FP32 force is over 8x less accurate
        compare("ps MIX", ps_mix, ref[0], m["areaCell"], MIX_TOL, MIX_TOL)
        compare("u MIX", u_mix, ref[2], None, MIX_U_TOL, MIX_U_TOL)
        assert res["MIX_PGF32"][0] > 8.0 * res["MIX"][0] and res["MIX_PGF32"][1] > 8.0 * res["MIX"][1]


def test_sgl_parity_and_ordering(mpdc, oracle_mod, mesh_cache):
    # the all-FP32 configuration runs (finite, close to the oracle after 10
    # steps) and is no more accurate than MIX_PGF32, which it contains
    m = mesh_cache(5)
    K, dt, n = 10, 300.0, 10
    g = mpdc.Mesh(m)
    s = ic.hdc_jet(m, K, seed=2000)
    zero = np.zeros(m["nCells"])
    ref = oracle_mod.OracleMesh(m).hdc_run(s["ps"], s["Theta"], s["u"], dt, n)
    err = {}
    for pol in ("MIX", "MIX_PGF32", "SGL"):
        ps, Th, u = _run(mpdc, g, s, K, dt, n, getattr(mpdc, "POLICY_" + pol), zero)
        assert np.isfinite(ps).all() and np.isfinite(u).all()
        err[pol] = (rel_l2(ps, ref[0], m["areaCell"]), rel_l2(u, ref[2]))
        _say("hdc G5x%d jet, %d steps, %s: ps %.3e  u %.3e" % ((K, n, pol) + err[pol]))
    # SGL computes the pressure-gradient term and everything else in FP32: it is
    # held to the surface-pressure bar only (both norms); its wind is checked to
    # be worse than MIX's, as the paper finds
    compare("ps SGL", ps, ref[0], m["areaCell"], MIX_TOL, MIX_TOL)
    assert err["SGL"][1] <= 1e-3
    assert err["SGL"][1] > 8.0 * err["MIX"][1]
