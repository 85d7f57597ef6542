"""GPU state handling through the C ABI: checkpoint and resume through
state_read / state_write is bitwise exact (the prognostic state is all a step
carries over), and the error paths return their documented codes."""
import ctypes

import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpdc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_08849_amd.mpdc as m
    return m


def _say(*a):
    print(*a, flush=True)


def _dycore_state(mpdc, g, model, K, fields):
    st = mpdc.State(g, model, mpdc.POLICY_MIX, K=K, dt=300.0 if model == mpdc.MODEL_HDC else 60.0,
                    sigma=ic.sigma_interfaces(K))
    for f, x in fields.items():
        st.state_write(f, x)
    return st


@pytest.mark.parametrize("model", ["HDC", "NDC"])
def test_checkpoint_resume_is_bitwise(mpdc, mesh_cache, model):
    m = mesh_cache(4)
    K = 12
    g = mpdc.Mesh(m)
    if model == "HDC":
        s = ic.hdc_jet(m, K, seed=2000)
        fs = {mpdc.FIELD_PS: s["ps"][:, None], mpdc.FIELD_THETA: s["Theta"][:, :, None],
              mpdc.FIELD_U: s["u"][:, :, None]}
        mid = mpdc.MODEL_HDC
    else:
        s = ic.nh_warm_bubble(m, K, rh=6.0e5, seed=4000)
        fs = {mpdc.FIELD_PS: s["ps"][:, None], mpdc.FIELD_THETA: s["Theta"][:, :, None],
              mpdc.FIELD_U: s["u"][:, :, None], mpdc.FIELD_W: s["w"][:, :, None],
              mpdc.FIELD_PHI: s["phi"][:, :, None]}
        mid = mpdc.MODEL_NDC
    _say("%s G4x%d MIX: 10 steps straight vs 5 + checkpoint + 5" % (model, K))
    a = _dycore_state(mpdc, g, mid, K, fs)
    a.dycore_step(10)
    ref = {f: a.state_read(f) for f in fs}
    b = _dycore_state(mpdc, g, mid, K, fs)
    b.dycore_step(5)
    ck = {f: b.state_read(f) for f in fs}
    del b
    c = _dycore_state(mpdc, g, mid, K, ck)
    c.dycore_step(5)
    for f in fs:
        assert np.array_equal(c.state_read(f), ref[f]), f


def test_tracer_checkpoint_resume_is_bitwise(mpdc, mesh_cache):
    m = mesh_cache(4)
    tr = ic.tracer_solid_body(m, 3, 4, seed=3000)
    g = mpdc.Mesh(m)

    def make(dpi, q):
        st = mpdc.State(g, mpdc.MODEL_TRACER, mpdc.POLICY_MIX, K=3, T=4, dt=3000.0)
        st.state_write(mpdc.FIELD_TR_FLUX, tr["F"])
        st.state_write(mpdc.FIELD_TR_DPI, dpi)
        st.state_write(mpdc.FIELD_TR_Q, q)
        return st

    _say("tracer G4x3x4 MIX: 6 steps straight vs 3 + checkpoint + 3")
    a = make(tr["dpi"], tr["q"])
    a.tracer_step(6)
    b = make(tr["dpi"], tr["q"])
    b.tracer_step(3)
    c = make(b.state_read(mpdc.FIELD_TR_DPI), b.state_read(mpdc.FIELD_TR_Q))
    c.tracer_step(3)
    assert np.array_equal(c.state_read(mpdc.FIELD_TR_DPI), a.state_read(mpdc.FIELD_TR_DPI))
    assert np.array_equal(c.state_read(mpdc.FIELD_TR_Q), a.state_read(mpdc.FIELD_TR_Q))


def test_error_paths(mpdc, mesh_cache):
    import torch
    m = mesh_cache(2)
    g = mpdc.Mesh(m)
    K = 4
    hdc = mpdc.State(g, mpdc.MODEL_HDC, mpdc.POLICY_MIX, K=K, dt=600.0, sigma=ic.sigma_interfaces(K))
    trs = mpdc.State(g, mpdc.MODEL_TRACER, mpdc.POLICY_MIX, K=K, T=2, dt=600.0)
    lib = mpdc.lib

    # workspace too small: the state is not created
    cfg = hdc.cfg
    need = lib.mpdc_state_workspace_bytes(g.h, ctypes.byref(cfg))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = ctypes.c_void_p()
    assert lib.mpdc_state_create(g.h, ctypes.byref(cfg), ctypes.c_void_p(ws.data_ptr()), need - 1,
                                 ctypes.byref(out)) == -3
    assert out.value is None
    # a workspace that is not 256-byte aligned (checked before anything is written)
    assert lib.mpdc_state_create(g.h, ctypes.byref(cfg), ctypes.c_void_p(ws.data_ptr() + 64), need,
                                 ctypes.byref(out)) == -1
    assert out.value is None
    # steps of the wrong kind
    assert lib.mpdc_dycore_step(trs.h, 1, None) == -7
    assert lib.mpdc_tracer_step(hdc.h, 1, None) == -7
    # a field the model does not have, a wrong byte count, a negative step count
    x = np.zeros((g.N, K + 1), np.float64)
    assert lib.mpdc_state_write(hdc.h, mpdc.FIELD_W, x.ctypes.data_as(ctypes.c_void_p), 0, x.nbytes, None) == -1
    y = np.zeros(g.N + 1, np.float64)
    assert lib.mpdc_state_write(hdc.h, mpdc.FIELD_PS, y.ctypes.data_as(ctypes.c_void_p), 0, y.nbytes, None) == -1
    assert lib.mpdc_dycore_step(hdc.h, -1, None) == -1
    # launch shapes outside the legal set
    assert lib.mpdc_set_kernel_launch(hdc.h, 4, 0, 0) == -1          # kernel id
    assert lib.mpdc_set_kernel_launch(hdc.h, 0, 3, 0) == -1          # values per lane
    assert lib.mpdc_set_kernel_launch(hdc.h, 0, 4, 0) == -1          # four per lane in a column: ensembles only
    ens = {p: mpdc.State(g, mpdc.MODEL_HDC, p, K=K, M=4, dt=600.0, sigma=ic.sigma_interfaces(K))
           for p in (mpdc.POLICY_MIX, mpdc.POLICY_DBL)}
    assert lib.mpdc_set_kernel_launch(ens[mpdc.POLICY_MIX].h, 2, 4, 1) == 0    # FP32, one cell per work-group
    assert lib.mpdc_set_kernel_launch(ens[mpdc.POLICY_MIX].h, 2, 4, 2) == -1   # ... and only one
    assert lib.mpdc_set_kernel_launch(ens[mpdc.POLICY_DBL].h, 0, 4, 1) == -1   # not in the all-FP64 policy
    del ens
    assert lib.mpdc_set_kernel_launch(hdc.h, 0, 1, 1000) == -1       # column work-group over 512 lanes
    assert lib.mpdc_set_kernel_launch(hdc.h, 3, 2, 100) == -1        # not a multiple of 64
    assert lib.mpdc_set_kernel_launch(trs.h, 0, 4, 128) == -1        # 4 does not divide T = 2
    assert lib.mpdc_set_kernel_launch(trs.h, 3, 0, 0) == -1          # the tracer has three kernels
    # one cell per work-group (tracer): K T / values_per_lane <= 512 threads, also
    # when only the values per lane change afterwards
    big = mpdc.State(g, mpdc.MODEL_TRACER, mpdc.POLICY_MIX, K=60, T=16, dt=600.0)
    assert lib.mpdc_set_kernel_launch(big.h, 0, 1, 1) == -1          # 960 threads
    assert lib.mpdc_set_kernel_launch(big.h, 0, 2, 1) == 0           # 480 threads
    assert lib.mpdc_set_kernel_launch(big.h, 0, 1, 0) == -1          # keeps one cell: 960 again
    assert big.get_kernel_launch(0) == (2, 1)
    del big
    # the states still step after the rejected calls
    hdc.state_write(mpdc.FIELD_PS, np.full((g.N, 1), 1.0e5))
    hdc.state_write(mpdc.FIELD_THETA, np.full((g.N, K, 1), 300.0 * 9.9e4 / K))
    hdc.state_write(mpdc.FIELD_U, np.zeros((g.E, K, 1)))
    hdc.dycore_step(1)
    assert np.isfinite(hdc.state_read(mpdc.FIELD_PS)).all()


def test_instability_is_flagged(mpdc, mesh_cache):
    # a stable step reports finite fields and a Courant number below one; fifty
    # times that step makes the run blow up, which the diagnostics flag (a
    # Courant number above one, or MPDC_E_NUMERIC once values are no longer finite)
    m = mesh_cache(3)
    K = 6
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    for dt in (900.0, 50 * 900.0):
        st2 = mpdc.State(g, mpdc.MODEL_HDC, mpdc.POLICY_MIX, K=K, dt=dt, sigma=ic.sigma_interfaces(K))
        st2.state_write(mpdc.FIELD_PS, s["ps"][:, None])
        st2.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
        st2.state_write(mpdc.FIELD_U, s["u"][:, :, None])
        st2.dycore_step(40)
        d = st2.diagnostics(mpdc.FIELD_PS, check=False)
        _say("hdc G3x%d MIX dt %.0f s, 40 steps: rc %d nonfinite %d cfl_max %.3g" % (K, dt, d["rc"], d["nonfinite"],
                                                                                d["cfl_max"]))
        if dt == 900.0:
            assert d["rc"] == 0 and d["nonfinite"] == 0 and 0.0 < d["cfl_max"] < 1.0
        else:
            assert d["rc"] == -5 or d["cfl_max"] > 1.0
            if d["rc"] == -5:
                assert d["nonfinite"] > 0


def test_stage_byte_counts(mpdc, mesh_cache):
    # the byte model per RK stage: its mean is mpdc_kernel_bytes; the mixed
    # policy stores the FP64 u (edge kernel) and Theta (second cell kernel) in
    # the last stage only, the all-FP64 policy in every stage
    m = mesh_cache(3)
    K = 6
    g = mpdc.Mesh(m)
    E, N = g.E, g.N
    for name in ("DBL", "MIX", "MIX_BOX"):
        st = mpdc.State(g, mpdc.MODEL_HDC, getattr(mpdc, "POLICY_" + name), K=K, dt=600.0,
                        sigma=ic.sigma_interfaces(K))
        for kid in range(4):
            b = [st.stage_kernel_bytes(kid, s) for s in range(3)]
            assert all(x > 0 for x in b)
            assert abs(sum(b) / 3.0 - st.kernel_bytes(kid)) <= 1e-9 * st.kernel_bytes(kid)
        assert st.stage_kernel_bytes(0, 3) == 0.0 and st.stage_kernel_bytes(0, -1) == 0.0
        skip = {3: E * K * 8, 2: N * K * 8}
        for kid in (0, 1, 2, 3):
            d = st.stage_kernel_bytes(kid, 2) - st.stage_kernel_bytes(kid, 1)
            if name == "MIX" and kid in skip:
                assert d == skip[kid], (name, kid, d)
            else:
                assert d == 0.0, (name, kid, d)
        assert abs(st.step_bytes() - sum(st.stage_kernel_bytes(k, s) for k in range(4) for s in range(3))) \
            <= 1e-9 * st.step_bytes()
