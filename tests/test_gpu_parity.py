"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (the workload definitions, plus element-wise forms of them):
 - all-FP64 path: every prognostic field within 1e-12 of the oracle in
   normalised L2 and in relative max error (max|x - r| / max|r|); the
   non-hydrostatic w and u, small residuals of large cancelling FP64 terms,
   element-wise within 16 unit roundoffs of those terms' size, integrated
   over the steps (gpu_helpers.nh_dbl_bounds);
 - mixed path: h / surface pressure (and Theta, phi) within 1e-5 after 10
   steps in both norms; the velocity within 16 FP32 unit roundoffs (its
   advective tendencies are FP32);
 - integer mesh tables bit-exact.
"""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import (DBL_TOL, MIX_TOL, MIX_U_TOL, compare, compare_abs, compare_dbl, gpu_hdc, gpu_ndc, gpu_sw,
                         gpu_tracer, nh_dbl_bounds, rel_l2)

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


def test_mesh_tables_match_oracle(mpdc, oracle_mod, mesh_cache):
    for lev in (2, 4):
        m = mesh_cache(lev)
        g = mpdc.Mesh(m)
        o = oracle_mod.OracleMesh(m).tables()
        assert np.array_equal(g.table(mpdc.TABLE_CELLS_ON_CELL), o["cells_on_cell"])
        assert np.array_equal(g.table(mpdc.TABLE_EDGE_SIGN), o["edge_sign"])
        assert np.array_equal(g.table(mpdc.TABLE_VERTEX_SIGN), o["vertex_sign"].ravel())
        assert np.array_equal(g.table(mpdc.TABLE_TRISK_OFFSET), o["trisk_offset"])
        assert np.array_equal(g.table(mpdc.TABLE_TRISK_EDGE), o["trisk_edge"])
        assert np.abs(g.table(mpdc.TABLE_TRISK_WEIGHT) - o["trisk_weight"]).max() <= 1e-14
        hg = g.table(mpdc.TABLE_HESSIAN).reshape(-1, 6)
        scale = np.abs(o["hessian"]).max()
        assert np.abs(hg - o["hessian"]).max() <= 1e-9 * scale


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_sw_parity_g5(mpdc, oracle_mod, mesh_cache, policy):
    m = mesh_cache(5)
    s = ic.sw_geostrophic(m, seed=1000)
    om = oracle_mod.OracleMesh(m)
    h_o, u_o = om.sw_run(s["h"], s["u"], s["b"], 600.0, 10)
    g = mpdc.Mesh(m)
    pol = getattr(mpdc, "POLICY_" + policy)
    _say("sw G5 10 steps", policy)
    st, h, u = gpu_sw(mpdc, g, s, 600.0, 10, pol)
    # the bump's signal (h - h0) must also agree, not only the mean depth
    eb = rel_l2(h - s["h"], h_o - s["h"], m["areaCell"])
    _say("  dh %.3e" % eb)
    if policy == "DBL":
        compare_dbl("h", h, h_o, m["areaCell"])
        compare_dbl("u", u, u_o)
        assert eb <= 1e-9
    else:
        compare("h", h, h_o, m["areaCell"], MIX_TOL, MIX_TOL)
        compare("u", u, u_o, None, MIX_U_TOL, MIX_U_TOL)
        assert eb <= 1e-2


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_hdc_parity_g4(mpdc, oracle_mod, mesh_cache, policy):
    m = mesh_cache(4)
    K = 30
    s = ic.hdc_jet(m, K, seed=2000)
    om = oracle_mod.OracleMesh(m)
    ps_o, Th_o, u_o = om.hdc_run(s["ps"], s["Theta"], s["u"], 600.0, 10)
    g = mpdc.Mesh(m)
    pol = getattr(mpdc, "POLICY_" + policy)
    _say("hdc G4x30 10 steps", policy)
    st, (ps, Th, u) = gpu_hdc(mpdc, g, s, K, 600.0, 10, pol)
    du = rel_l2(u - s["u"], u_o - s["u"])
    _say("  du %.3e" % du)
    if policy == "DBL":
        for n, x, r, w in (("ps", ps, ps_o, m["areaCell"]), ("Theta", Th, Th_o, m["areaCell"]), ("u", u, u_o, None)):
            compare_dbl(n, x, r, w)
        assert du <= 1e-9
    else:
        compare("ps", ps, ps_o, m["areaCell"], MIX_TOL, MIX_TOL)
        compare("Theta", Th, Th_o, m["areaCell"], MIX_TOL, MIX_TOL)
        compare("u", u, u_o, None, MIX_U_TOL, MIX_U_TOL)


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_ndc_parity_g4(mpdc, oracle_mod, mesh_cache, policy):
    m = mesh_cache(4)
    K = 20
    s = ic.nh_warm_bubble(m, K, rh=6.0e5, seed=4000)
    om = oracle_mod.OracleMesh(m)
    ref = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], 60.0, 10)
    g = mpdc.Mesh(m)
    pol = getattr(mpdc, "POLICY_" + policy)
    _say("ndc G4x20 10 steps", policy)
    st, out = gpu_ndc(mpdc, g, s, K, 60.0, 10, pol)
    ps, Th, u, w, phi = out
    _say("  dphi L2 %.3e" % rel_l2(phi - s["phi"], ref[4] - s["phi"]))
    assert np.abs(ref[3]).max() > 1e-4          # the bubble produces vertical motion
    if policy == "DBL":
        compare_dbl("ps", ps, ref[0], m["areaCell"])
        compare_dbl("Theta", Th, ref[1], m["areaCell"])
        compare_dbl("phi", phi, ref[4], m["areaCell"])
        bw, bu = nh_dbl_bounds(ref[4], 9.80616, 60.0, 10, float(m["dEdge"].min()))
        compare_abs("w", w, ref[3], bw)
        compare_abs("u", u, ref[2], bu)
    else:
        compare("ps", ps, ref[0], m["areaCell"], MIX_TOL, MIX_TOL)
        compare("Theta", Th, ref[1], m["areaCell"], MIX_TOL, MIX_TOL)
        compare("phi", phi, ref[4], m["areaCell"], MIX_TOL, MIX_TOL)
        compare("u", u, ref[2], None, MIX_U_TOL, MIX_U_TOL)
        compare("w", w, ref[3], m["areaCell"], MIX_U_TOL, MIX_U_TOL)


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_tracer_parity_g4(mpdc, oracle_mod, mesh_cache, policy):
    m = mesh_cache(4)
    tr = ic.tracer_solid_body(m, 5, 4, seed=3000)
    om = oracle_mod.OracleMesh(m)
    dt = 3000.0
    dpi_o, q_o = om.tracer_run(tr["F"], tr["dpi"], tr["q"], dt, 6)
    g = mpdc.Mesh(m)
    pol = getattr(mpdc, "POLICY_" + policy)
    _say("tracer G4x5x4 6 steps", policy)
    st, dpi, q = gpu_tracer(mpdc, g, tr, dt, 6, pol)
    _say("  min %.3e max %.3e" % (q.min(), q.max()))
    compare_dbl("dpi", dpi, dpi_o, m["areaCell"])
    for t in range(q.shape[2]):
        if policy == "DBL":
            compare_dbl("q%d" % t, q[:, :, t], q_o[:, :, t], m["areaCell"])
        else:
            compare("q%d" % t, q[:, :, t], q_o[:, :, t], m["areaCell"], MIX_TOL, MIX_TOL)
    if policy != "DBL":
        assert q.min() >= -1e-6 and q.max() <= 1.0 + 1e-6


def test_hdc_ensemble_members_match_single_runs(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(3)
    K, M = 8, 3
    base = ic.hdc_jet(m, K, seed=5000)
    ens = ic.ensemble(base, M, sigma=0.1, seed=5000)
    g = mpdc.Mesh(m)
    om = oracle_mod.OracleMesh(m)
    _say("hdc ensemble G3x8x3 5 steps DBL")
    st, (ps, Th, u) = gpu_hdc(mpdc, g, ens, K, 900.0, 5, mpdc.POLICY_DBL, M=M)
    for j in range(M):
        ps_o, Th_o, u_o = om.hdc_run(ens["ps"][:, j], ens["Theta"][:, :, j], ens["u"][:, :, j], 900.0, 5)
        compare_dbl("ps m%d" % j, ps[:, j], ps_o)
        compare_dbl("Theta m%d" % j, Th[:, :, j], Th_o)
        compare_dbl("u m%d" % j, u[:, :, j], u_o)


def test_graph_replay_and_launch_shapes_are_bitwise_identical(mpdc, mesh_cache):
    m = mesh_cache(4)
    K = 10
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    ref = None
    for graph, launch in [(False, None), (True, None), (False, (1, 64)), (True, (3, 512)), (False, (25, 128))]:
        _say("hdc G4x10 graph=%s launch=%s" % (graph, launch))
        st, out = gpu_hdc(mpdc, g, s, K, 600.0, 4, mpdc.POLICY_MIX, graph=graph, launch=launch)
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            assert np.array_equal(a, b)
    # per-kernel values per lane and work-group sizes, and the autotuner's choice
    for shapes in ([(1, 8), (1, 64), (1, 4), (1, 128)], [(2, 3), (4, 256), (2, 1), (4, 512)]):
        _say("hdc G4x10 per-kernel shapes %s" % (shapes,))
        st = mpdc.State(g, mpdc.MODEL_HDC, mpdc.POLICY_MIX, K=K, dt=600.0, sigma=ic.sigma_interfaces(K))
        for kid, (vpl, grp) in enumerate(shapes):
            if vpl == 4 and K % 4:
                vpl = 2
            st.set_kernel_launch(kid, vpl, grp)
        st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
        st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
        st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
        st.dycore_step(4)
        out = [st.state_read(f)[..., 0] for f in (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U)]
        for a, b in zip(out, ref):
            assert np.array_equal(a, b)
    st = mpdc.State(g, mpdc.MODEL_HDC, mpdc.POLICY_MIX, K=K, dt=600.0, sigma=ic.sigma_interfaces(K))
    st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
    st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
    st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
    st.autotune()
    _say("  autotuned " + str([st.get_kernel_launch(k) for k in range(4)]))
    st.dycore_step(4)
    out = [st.state_read(f)[..., 0] for f in (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U)]
    for a, b in zip(out, ref):
        assert np.array_equal(a, b)
    tr = ic.tracer_solid_body(m, 3, 2, seed=3000)
    tref = None
    for graph, launch in [(False, None), (True, None), (True, (0, 128))]:
        _say("tracer G4 graph=%s launch=%s" % (graph, launch))
        st, dpi, q = gpu_tracer(mpdc, g, tr, 3000.0, 3, mpdc.POLICY_MIX, graph=graph, launch=launch)
        if tref is None:
            tref = (dpi, q)
        assert np.array_equal(dpi, tref[0]) and np.array_equal(q, tref[1])
    tr4 = ic.tracer_solid_body(m, 3, 8, seed=3000)
    t4 = None
    for vpl in (1, 2, 4, 8):
        _say("tracer G4 T=8 values per lane %d" % vpl)
        st = mpdc.State(g, mpdc.MODEL_TRACER, mpdc.POLICY_MIX, K=3, T=8, dt=3000.0)
        for kid in range(3):
            st.set_kernel_launch(kid, vpl, 128)
        st.state_write(mpdc.FIELD_TR_FLUX, tr4["F"])
        st.state_write(mpdc.FIELD_TR_DPI, tr4["dpi"])
        st.state_write(mpdc.FIELD_TR_Q, tr4["q"])
        st.tracer_step(3)
        q = st.state_read(mpdc.FIELD_TR_Q)
        if t4 is None:
            t4 = q
        assert np.array_equal(q, t4)


def test_diagnostics_match_oracle(mpdc, oracle_mod, mesh_cache):
    import torch
    m = mesh_cache(4)
    K = 10
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    _say("diagnostics G4x10")
    st, (ps, Th, u) = gpu_hdc(mpdc, g, s, K, 600.0, 3, mpdc.POLICY_DBL)
    ref = torch.from_numpy(s["Theta"][:, :, None].copy()).cuda()
    d = st.diagnostics(mpdc.FIELD_THETA, ref)
    n = oracle_mod.norms(m["areaCell"], Th, s["Theta"])
    assert np.allclose([d["l1"], d["l2"], d["linf"]], n, rtol=1e-10)
    mass = oracle_mod.area_sum(m["areaCell"], ps - 1000.0)
    assert abs(d["mass"] - mass) <= 1e-12 * mass
    assert d["min"] == Th.min() and d["max"] == Th.max()
    assert d["nonfinite"] == 0
    # mass conservation of the GPU path at FP64 level in both policies
    for pol in (mpdc.POLICY_DBL, mpdc.POLICY_MIX):
        st, (ps, Th, u) = gpu_hdc(mpdc, g, s, K, 600.0, 10, pol)
        m0 = oracle_mod.area_sum(m["areaCell"], s["ps"] - 1000.0)
        m1 = oracle_mod.area_sum(m["areaCell"], ps - 1000.0)
        assert abs(m1 - m0) <= 1e-13 * m0


def test_diagnostics_flag_nonfinite(mpdc, mesh_cache):
    m = mesh_cache(3)
    s = ic.sw_geostrophic(m)
    g = mpdc.Mesh(m)
    st = mpdc.State(g, mpdc.MODEL_SW, mpdc.POLICY_DBL, dt=600.0)
    h = s["h"].copy()
    h[7] = np.nan
    st.state_write(mpdc.FIELD_H, h[:, None])
    st.state_write(mpdc.FIELD_U, s["u"][:, None, None])
    st.state_write(mpdc.FIELD_B, s["b"])
    d = st.diagnostics(mpdc.FIELD_H, check=False)
    assert d["rc"] == -5 and d["nonfinite"] == 1
    with pytest.raises(mpdc.MpdcError):
        st.diagnostics(mpdc.FIELD_H)
