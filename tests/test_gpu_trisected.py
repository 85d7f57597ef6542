"""GPU parity on a trisection ("B3") grid -- the construction of Table 1's
G9B3, one trisection and then bisections -- at small size (G3B3: n = 24
segments per icosahedron edge, 5,762 cells): hydrostatic and
non-hydrostatic dycore and tracer transport against the oracle, to the
usual bars."""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import MIX_TOL, MIX_U_TOL, compare, compare_dbl, gpu_hdc, gpu_ndc, gpu_tracer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpdc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_08849_amd.mpdc as m
    return m


@pytest.fixture(scope="module")
def b3(mesh_cache):
    import oracle
    m = mesh_cache(3, 1)
    return m, oracle.OracleMesh(m)


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_hdc_on_trisected_grid(mpdc, b3, policy):
    m, om = b3
    K = 20
    s = ic.hdc_jet(m, K, seed=2000)
    ref = om.hdc_run(s["ps"], s["Theta"], s["u"], 450.0, 10)
    _say("hdc G3B3x%d 10 steps" % K, policy)
    _, (ps, Th, u) = gpu_hdc(mpdc, mpdc.Mesh(m), s, K, 450.0, 10, getattr(mpdc, "POLICY_" + policy))
    A = m["areaCell"]
    if policy == "DBL":
        compare_dbl("ps", ps, ref[0], A)
        compare_dbl("Theta", Th, ref[1], A)
        compare_dbl("u", u, ref[2])
    else:
        compare("ps", ps, ref[0], A, MIX_TOL, MIX_TOL)
        compare("Theta", Th, ref[1], A, MIX_TOL, MIX_TOL)
        compare("u", u, ref[2], None, MIX_U_TOL, MIX_U_TOL)


def test_ndc_on_trisected_grid(mpdc, b3):
    m, om = b3
    K = 12
    s = ic.nh_warm_bubble(m, K, rh=6.0e5, seed=4000)
    ref = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], 60.0, 5)
    _say("ndc G3B3x%d 5 steps MIX" % K)
    _, out = gpu_ndc(mpdc, mpdc.Mesh(m), s, K, 60.0, 5, mpdc.POLICY_MIX)
    A = m["areaCell"]
    for n, x, r, w, tol in zip(["ps", "Theta", "u", "w", "phi"], out, ref, [A, A, None, A, A],
                               [MIX_TOL, MIX_TOL, MIX_U_TOL, MIX_U_TOL, MIX_TOL]):
        compare(n, x, r, w, tol, tol)


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_tracer_on_trisected_grid(mpdc, b3, policy):
    m, om = b3
    tr = ic.tracer_solid_body(m, 4, 4, seed=3000)
    dpi_o, q_o = om.tracer_run(tr["F"], tr["dpi"], tr["q"], 1500.0, 4)
    _say("tracer G3B3x4x4 4 steps", policy)
    _, dpi, q = gpu_tracer(mpdc, mpdc.Mesh(m), tr, 1500.0, 4, getattr(mpdc, "POLICY_" + policy))
    compare_dbl("dpi", dpi, dpi_o, m["areaCell"])
    for t in range(q.shape[2]):
        tol = 1e-12 if policy == "DBL" else MIX_TOL
        compare("q%d" % t, q[:, :, t], q_o[:, :, t], m["areaCell"], tol, tol)
    assert q.min() >= -1e-6 and q.max() <= 1.0 + 1e-6
