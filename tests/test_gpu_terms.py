"""GPU parity of the per-term precision engine (POLICY_TERMS, the precision
table of Section 2.2's iterative reduction): with no term in FP32 it is an
all-FP64 stage and meets the all-FP64 bars against the oracle (jet and
terrain); with the mixed policy's FP32 terms it meets the mixed bars and
stays within FP32 rounding of the fused mixed kernels; every term's FP32
switch changes the result; graph replay is bitwise; the combinations it is
not built for are rejected."""
import ctypes

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


def _run(mpdc, g, s, K, dt, n, policy, mask=0, phis=None, graph=False):
    import torch
    st = mpdc.State(g, mpdc.MODEL_HDC, policy, K=K, dt=dt, sigma=ic.sigma_interfaces(K), term_fp32=mask)
    if phis is not None:
        st.state_write(mpdc.FIELD_PHIS, phis)
    st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
    st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
    st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
    st.set_graph(graph)
    with torch.cuda.stream(torch.cuda.Stream()):
        st.dycore_step(n)
        torch.cuda.current_stream().synchronize()
    return [st.state_read(f)[..., 0] for f in (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U)]


def test_terms_fp64_and_mixed_split_against_oracle(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(4)
    K = 30
    s = ic.hdc_jet(m, K, seed=2000)
    ref = oracle_mod.OracleMesh(m).hdc_run(s["ps"], s["Theta"], s["u"], 600.0, 10)
    g = mpdc.Mesh(m)
    A = m["areaCell"]
    _say("terms engine G4x30 10 steps, no FP32 term")
    ps, Th, u = _run(mpdc, g, s, K, 600.0, 10, mpdc.POLICY_TERMS, 0)
    compare_dbl("ps", ps, ref[0], A)
    compare_dbl("Theta", Th, ref[1], A)
    compare_dbl("u", u, ref[2])
    _say("terms engine G4x30 10 steps, the mixed split")
    ps, Th, u = _run(mpdc, g, s, K, 600.0, 10, mpdc.POLICY_TERMS, mpdc.TERMS_MIX)
    compare("ps", ps, ref[0], A, MIX_TOL, MIX_TOL)
    compare("Theta", Th, ref[1], A, MIX_TOL, MIX_TOL)
    compare("u", u, ref[2], None, MIX_U_TOL, MIX_U_TOL)
    # the fused mixed kernels round the same terms to FP32 (in other places and
    # orders): the two runs differ by FP32 roundings, not by more
    mix = _run(mpdc, g, s, K, 600.0, 10, mpdc.POLICY_MIX)
    for n_, a, b in zip(("ps", "Theta", "u"), (ps, Th, u), mix):
        d = rel_l2(a, b)
        _say("    vs fused MIX %-6s %.3e" % (n_, d))
        assert d <= MIX_U_TOL


def test_terms_fp64_over_terrain(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(4)
    K = 10
    phis = ic.mountain(m)
    rest = ic.hdc_rest_over_terrain(m, K, phis)
    s = dict(ps=rest["ps"], Theta=rest["Theta"], u=ic.hdc_jet(m, K, seed=2000)["u"])
    ref = oracle_mod.OracleMesh(m).hdc_run(s["ps"], s["Theta"], s["u"], 600.0, 10, phis=phis)
    _say("terms engine G4x10 over a 3 km mountain, no FP32 term")
    ps, Th, u = _run(mpdc, mpdc.Mesh(m), s, K, 600.0, 10, mpdc.POLICY_TERMS, 0, phis=phis)
    compare_dbl("ps", ps, ref[0], m["areaCell"])
    compare_dbl("Theta", Th, ref[1], m["areaCell"])
    compare_dbl("u", u, ref[2])


def test_every_term_switch_acts_and_graph_is_bitwise(mpdc, mesh_cache):
    m = mesh_cache(3)
    K = 8
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    base = _run(mpdc, g, s, K, 900.0, 3, mpdc.POLICY_TERMS, 0)
    for name, bit in mpdc.TERM_BIT.items():
        out = _run(mpdc, g, s, K, 900.0, 3, mpdc.POLICY_TERMS, 1 << bit)
        d = max(rel_l2(a, b) for a, b in zip(out, base))
        _say("  FP32 %-20s max field difference from all-FP64 %.3e" % (name, d))
        assert all(np.isfinite(x).all() for x in out)
        assert 0.0 < d < 1e-4, name
    allm = (1 << len(mpdc.TERMS)) - 1
    a = _run(mpdc, g, s, K, 900.0, 3, mpdc.POLICY_TERMS, allm)
    b = _run(mpdc, g, s, K, 900.0, 3, mpdc.POLICY_TERMS, allm, graph=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_terms_rejected_where_not_built(mpdc, mesh_cache):
    m = mesh_cache(2)
    g = mpdc.Mesh(m)
    sig = np.ascontiguousarray(ic.sigma_interfaces(4))
    sp = sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def bytes_for(model, policy, M=1, mask=0):
        cfg = mpdc.Config(model, policy, 4, M, 2 if model == mpdc.MODEL_TRACER else 0, 1, 600.0, 9.80616, 287.0,
                          1004.5, 1.0e5, 1000.0, sp, 0, 0, mask)
        return mpdc.lib.mpdc_state_workspace_bytes(g.h, ctypes.byref(cfg))

    assert bytes_for(mpdc.MODEL_HDC, mpdc.POLICY_TERMS, mask=mpdc.TERMS_MIX) > 0
    assert bytes_for(mpdc.MODEL_NDC, mpdc.POLICY_TERMS) == 0
    assert bytes_for(mpdc.MODEL_HDC, mpdc.POLICY_TERMS, M=2) == 0
    assert bytes_for(mpdc.MODEL_HDC, mpdc.POLICY_MIX, mask=1) == 0           # a mask needs POLICY_TERMS
    assert bytes_for(mpdc.MODEL_HDC, mpdc.POLICY_TERMS, mask=1 << 10) == 0   # no such term
    st = mpdc.State(g, mpdc.MODEL_HDC, mpdc.POLICY_TERMS, K=4, dt=600.0, sigma=sig, term_fp32=mpdc.TERMS_MIX)
    with pytest.raises(mpdc.MpdcError) as e:
        st.time_kernel(0)
    assert e.value.code == -6
