"""GPU parity at the benchmark workloads' full sizes, in the benchmark's launch
configuration (autotuned shapes, HIP-graph replay on a non-default stream).

The G6 x 30 hydrostatic jet runs its 20 steps against the oracle run live.
The G8 and G7 workloads run 10 steps against the oracle's results stored by
`tests/golden/make_fullsize_refs.py` (a committed script that calls only the
oracle and the input generators): every level of the 12 pentagons, of their
edges, of 500 random cells and edges and of the 500 cells and edges where
the oracle's state changed most over the steps.  The test rebuilds the same seeded
input (signatures checked), runs the GPU path and compares those samples
element by element, with the bars of the small-mesh parity tests:
 - all-FP64: 1e-12 in normalised L2 over the samples and in relative max
   error; the non-hydrostatic w and u against the absolute bounds of
   gpu_helpers.nh_dbl_bounds;
 - mixed: surface pressure, Theta and phi 1e-5, velocities 16 FP32 unit
   roundoffs per 10 steps, both norms;
and, over the whole field, global mass (and tracer mass) against the
oracle's and tracer bounds.
"""
import os
import sys

import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import (DBL_TOL, MIX_TOL, MIX_U_TOL, compare, compare_abs, compare_dbl, gpu_hdc, gpu_ndc,
                         gpu_tracer, mix_u_tol, nh_dbl_bounds, rel_l2)

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize_refs as refs   # noqa: E402

pytestmark = pytest.mark.gpu
PTOP = 1000.0


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


def load_case(case):
    """Stored oracle samples and the rebuilt seeded input of a full-size case."""
    path = refs.ref_path(case)
    assert os.path.exists(path), "missing %s: run tests/golden/make_fullsize_refs.py %s" % (path, case)
    ref = dict(np.load(path))
    _say("%s: building the input" % case)
    mesh, st, sig = refs.build_case(case)
    assert np.allclose(refs.mesh_signature(mesh), ref["mesh_sig"], rtol=1e-14, atol=0), \
        "the mesh generator no longer builds the mesh the reference was taken on"
    assert np.allclose(sig, ref["state_sig"], rtol=1e-14, atol=0), \
        "the input generator no longer builds the state the reference was taken on"
    return mesh, st, ref


def test_hdc_g6x30_20_steps(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(6)
    K = 30
    s = ic.hdc_jet(m, K, seed=2000)
    _say("hdc G6x30 20 steps: oracle")
    om = oracle_mod.OracleMesh(m)
    ps_o, Th_o, u_o = om.hdc_run(s["ps"], s["Theta"], s["u"], 300.0, 20)
    g = mpdc.Mesh(m)
    A = m["areaCell"]
    for policy in ("DBL", "MIX"):
        _say("hdc G6x30 20 steps", policy, "autotuned, graph")
        st, (ps, Th, u) = gpu_hdc(mpdc, g, s, K, 300.0, 20, getattr(mpdc, "POLICY_" + policy), graph=True,
                                  autotune=True)
        du = rel_l2(u - s["u"], u_o - s["u"])
        _say("  du %.3e" % du)
        if policy == "DBL":
            compare_dbl("ps", ps, ps_o, A)
            compare_dbl("Theta", Th, Th_o, A)
            compare_dbl("u", u, u_o)
            assert du <= 1e-9
        else:
            compare("ps", ps, ps_o, A, MIX_TOL, MIX_TOL)
            compare("Theta", Th, Th_o, A, MIX_TOL, MIX_TOL)
            compare("u", u, u_o, None, mix_u_tol(20), mix_u_tol(20))


def _hdc_checks(policy, label, ps, Th, u, ref, suffix, cells, edges):
    r_ps, r_th, r_u = ref["ps" + suffix], ref["Theta" + suffix], ref["u" + suffix]
    if policy == "DBL":
        compare_dbl("ps " + label, ps[cells], r_ps)
        compare_dbl("Theta " + label, Th[cells], r_th)
        compare_dbl("u " + label, u[edges], r_u)
    else:
        compare("ps " + label, ps[cells], r_ps, None, MIX_TOL, MIX_TOL)
        compare("Theta " + label, Th[cells], r_th, None, MIX_TOL, MIX_TOL)
        compare("u " + label, u[edges], r_u, None, MIX_U_TOL, MIX_U_TOL)


def _mass_check(label, area, ps, ps0, mass_ref):
    m0 = float(np.sum(area * (ps0 - PTOP)))
    m1 = float(np.sum(area * (ps - PTOP)))
    _say("    %-10s mass drift %.3e  vs oracle %.3e" % (label, abs(m1 - m0) / m0, abs(m1 - mass_ref) / m0))
    assert abs(m1 - m0) <= 1e-13 * m0 and abs(m1 - mass_ref) <= 1e-13 * m0


@pytest.mark.timeout(600)
def test_hdc_ensemble_g7x30x16_10_steps(mpdc):
    case = "ens_g7x30x16"
    c = refs.CASES[case]
    m, ens, ref = load_case(case)
    cells, edges = ref["cells"], ref["edges"]
    g = mpdc.Mesh(m)
    for policy in ("DBL", "MIX"):
        _say("hdc G7x30x16 10 steps", policy, "autotuned, graph")
        st, (ps, Th, u) = gpu_hdc(mpdc, g, ens, c["K"], c["dt"], refs.NSTEPS, getattr(mpdc, "POLICY_" + policy),
                                  M=c["M"], graph=True, autotune=True)
        for j in ref["members"]:
            _hdc_checks(policy, "m%d" % j, ps[:, j], Th[:, :, j], u[:, :, j], ref, "_%d" % j, cells, edges)
        # the members differ (each carries its own perturbation) and every one stayed finite
        assert not np.array_equal(u[:, :, 0], u[:, :, c["M"] - 1])
        assert np.isfinite(ps).all() and np.isfinite(u).all()
        del st, ps, Th, u


@pytest.mark.timeout(600)
def test_ndc_g8x60_10_steps(mpdc):
    case = "ndc_g8x60"
    c = refs.CASES[case]
    m, s, ref = load_case(case)
    cells, edges = ref["cells"], ref["edges"]
    g = mpdc.Mesh(m)
    bw, bu = nh_dbl_bounds(ref["phi"], 9.80616, c["dt"], refs.NSTEPS, float(m["dEdge"].min()))
    for policy in ("DBL", "MIX"):
        _say("ndc G8x60 10 steps", policy, "autotuned, graph")
        st, (ps, Th, u, w, phi) = gpu_ndc(mpdc, g, s, c["K"], c["dt"], refs.NSTEPS,
                                          getattr(mpdc, "POLICY_" + policy), graph=True, autotune=True)
        assert all(np.isfinite(x).all() for x in (ps, Th, u, w, phi))
        if policy == "DBL":
            compare_dbl("ps", ps[cells], ref["ps"])
            compare_dbl("Theta", Th[cells], ref["Theta"])
            compare_dbl("phi", phi[cells], ref["phi"])
            compare_abs("w", w[cells], ref["w"], bw)
            compare_abs("u", u[edges], ref["u"], bu)
        else:
            compare("ps", ps[cells], ref["ps"], None, MIX_TOL, MIX_TOL)
            compare("Theta", Th[cells], ref["Theta"], None, MIX_TOL, MIX_TOL)
            compare("phi", phi[cells], ref["phi"], None, MIX_TOL, MIX_TOL)
            compare("u", u[edges], ref["u"], None, MIX_U_TOL, MIX_U_TOL)
            compare("w", w[cells], ref["w"], None, MIX_U_TOL, MIX_U_TOL)
        _mass_check(policy, m["areaCell"], ps, s["ps"], float(ref["mass"]))
        del st, ps, Th, u, w, phi


@pytest.mark.timeout(600)
def test_tracer_g8x30x8_10_steps(mpdc):
    case = "tracer_g8x30x8"
    c = refs.CASES[case]
    m, tr, ref = load_case(case)
    cells = ref["cells"]
    g = mpdc.Mesh(m)
    A = m["areaCell"]
    for policy in ("DBL", "MIX"):
        _say("tracer G8x30x8 10 steps", policy, "autotuned, graph")
        st, dpi, q = gpu_tracer(mpdc, g, tr, c["dt"], refs.NSTEPS, getattr(mpdc, "POLICY_" + policy), graph=True,
                                autotune=True)
        compare_dbl("dpi", dpi[cells], ref["dpi"])
        tol = DBL_TOL if policy == "DBL" else MIX_TOL
        for t in range(c["T"]):
            compare("q%d" % t, q[cells, :, t], ref["q"][:, :, t], None, tol, tol)
        mass = np.einsum("i,ik,ikt->t", A, dpi, q)
        em = np.abs(mass - ref["tracer_mass"]) / np.abs(ref["tracer_mass"])
        _say("    tracer mass vs oracle: max rel %.3e  min %.3e  max %.3e" % (em.max(), q.min(), q.max()))
        assert em.max() <= tol
        assert q.min() >= -1e-6 and q.max() <= 1.0 + 1e-6
        del st, dpi, q
