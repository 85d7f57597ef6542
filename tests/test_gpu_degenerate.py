"""GPU parity on the degenerate and ragged cases of the method, against the
FP64 oracle on the same seeded inputs.

* the smallest icosahedral meshes: G0 (12 cells, every cell a pentagon, so
  every column kernel takes its pad slot) and G1 (42 cells); grids of fewer
  cells than one work-group;
* a single layer (K = 1: no interior interface, empty vertical scans) and an
  odd number of layers (one value per lane, no two-level packing);
* the shortest non-hydrostatic columns (K = 2 and 3) for the vertical
  acoustic solve;
* a single tracer and an odd number of tracers (one tracer per lane);
* zero steps: the state is left bitwise unchanged (the mixed policy's
  FP32 mixing ratios read back as written, rounded to FP32).

Bars as elsewhere, each on the normalised L2 and the relative max error:
all-FP64 within 1e-12 (non-hydrostatic w and u: the element-wise bounds from
the FP64 roundings of their cancelling terms, g dt per step for w and the
pressure-gradient force's two terms for u); mixed within 1e-5 on pi_s,
Theta, phi and the mixing ratios, and 16 FP32 unit roundoffs on u and w.
"""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import (DBL_TOL, MIX_TOL, MIX_U_TOL, compare, compare_abs, compare_dbl, gpu_hdc, gpu_ndc, gpu_tracer,
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


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
@pytest.mark.parametrize("level,K", [(0, 1), (0, 3), (1, 1), (1, 3)])
def test_hdc_smallest_meshes_and_columns(mpdc, oracle_mod, mesh_cache, level, K, policy):
    m = mesh_cache(level)
    s = ic.hdc_jet(m, K, seed=2000)
    ref = oracle_mod.OracleMesh(m).hdc_run(s["ps"], s["Theta"], s["u"], 600.0, 3)
    _say("hdc G%d x %d, 3 steps" % (level, K), policy)
    st, out = gpu_hdc(mpdc, mpdc.Mesh(m), s, K, 600.0, 3, getattr(mpdc, "POLICY_" + policy))
    du = rel_l2(out[2] - s["u"], ref[2] - s["u"])
    _say("  du %.3e" % du)
    assert rel_l2(ref[0], s["ps"]) > 1e-9        # the state moved
    A = m["areaCell"]
    if policy == "DBL":
        compare_dbl("ps", out[0], ref[0], A)
        compare_dbl("Theta", out[1], ref[1], A)
        compare_dbl("u", out[2], ref[2])
        assert du <= 1e-9
    else:
        compare("ps", out[0], ref[0], A, MIX_TOL, MIX_TOL)
        compare("Theta", out[1], ref[1], A, MIX_TOL, MIX_TOL)
        compare("u", out[2], ref[2], None, MIX_U_TOL, MIX_U_TOL)


@pytest.mark.parametrize("K", [2, 3])
def test_ndc_shortest_columns(mpdc, oracle_mod, mesh_cache, K):
    m = mesh_cache(1)
    # a bubble of 3000 km radius: resolved by the 42 cells of G1
    s = ic.nh_warm_bubble(m, K, rh=3.0e6, seed=4000)
    om = oracle_mod.OracleMesh(m)
    ref = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], 60.0, 3)
    assert np.abs(ref[2]).max() > 1e-3 and np.abs(ref[3]).max() > 1e-3   # the bubble drives u and w
    A = m["areaCell"]
    for policy in ("DBL", "MIX"):
        _say("ndc G1 x %d, 3 steps" % K, policy)
        st, out = gpu_ndc(mpdc, mpdc.Mesh(m), s, K, 60.0, 3, getattr(mpdc, "POLICY_" + policy))
        ps, Th, u, w, phi = out
        if policy == "DBL":
            compare_dbl("ps", ps, ref[0], A)
            compare_dbl("Theta", Th, ref[1], A)
            compare_dbl("phi", phi, ref[4], A)
            bw, bu = nh_dbl_bounds(ref[4], 9.80616, 60.0, 3, float(m["dEdge"].min()))
            compare_abs("w", w, ref[3], bw)
            compare_abs("u", u, ref[2], bu)
        else:
            for n, x, r, wt, tol in zip(["ps", "Theta", "u", "w", "phi"], out, ref, [A, A, None, A, A],
                                        [MIX_TOL, MIX_TOL, MIX_U_TOL, MIX_U_TOL, MIX_TOL]):
                compare(n, x, r, wt, tol, tol)
        del st


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
@pytest.mark.parametrize("level,T", [(0, 2), (1, 1), (1, 3)])
def test_tracer_single_and_odd_tracer_counts(mpdc, oracle_mod, mesh_cache, level, T, policy):
    m = mesh_cache(level)
    K = 3
    tr = ic.tracer_solid_body(m, K, T, seed=3000)
    dpi_o, q_o = oracle_mod.OracleMesh(m).tracer_run(tr["F"], tr["dpi"], tr["q"], 3000.0, 2)
    _say("tracer G%d x %d x %d, 2 steps" % (level, K, T), policy)
    st, dpi, q = gpu_tracer(mpdc, mpdc.Mesh(m), tr, 3000.0, 2, getattr(mpdc, "POLICY_" + policy))
    compare_dbl("dpi", dpi, dpi_o)
    for t in range(T):
        if np.abs(q_o[:, :, t]).max() > 0:
            tol = DBL_TOL if policy == "DBL" else MIX_TOL
            compare("q%d" % t, q[:, :, t], q_o[:, :, t], None, tol, tol)
    assert q.min() >= -1e-6 and q.max() <= 1.0 + 1e-6


def test_zero_steps_leave_the_state_unchanged(mpdc, mesh_cache):
    m = mesh_cache(2)
    K, T = 4, 2
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    tr = ic.tracer_solid_body(m, K, T, seed=3000)
    for name in ("DBL", "MIX"):
        policy = getattr(mpdc, "POLICY_" + name)
        _say("zero steps", name)
        st, out = gpu_hdc(mpdc, g, s, K, 600.0, 0, policy)
        # the dycore's prognostic state is FP64 in both policies
        for x, r in zip(out, (s["ps"], s["Theta"], s["u"])):
            assert np.array_equal(x, r), name
        st, dpi, q = gpu_tracer(mpdc, g, tr, 3000.0, 0, policy)
        assert np.array_equal(dpi, tr["dpi"]), name
        # the mixed policy holds the mixing ratios in FP32
        q_ref = tr["q"] if name == "DBL" else tr["q"].astype(np.float32).astype(np.float64)
        assert np.array_equal(q, q_ref), name
