"""GPU parity at the benchmark workloads' full sizes, in the benchmark's launch
configuration (autotuned shapes, HIP-graph replay on a non-default stream).

The oracle runs the whole workload where it finishes in seconds (the G6 x 30
hydrostatic jet, 20 steps) and one or two steps of the G8 and G7 workloads
(each about 10-20 s of host time); the bars are those of the small-mesh
parity tests: all-FP64 within 1e-12 normalised L2 (NH w and u: ten times the
oracle's own sensitivity to a 1e-15 relative perturbation of Theta), mixed
within 1e-5 on the surface pressure / Theta / phi and 1e-3 on u.
"""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import gpu_hdc, gpu_ndc, gpu_tracer, rel_l2

pytestmark = pytest.mark.gpu

DBL_TOL = 1e-12
MIX_TOL = 1e-5


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


def test_hdc_g6x30_20_steps(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(6)
    K = 30
    s = ic.hdc_jet(m, K, seed=2000)
    _say("hdc G6x30 20 steps: oracle")
    om = oracle_mod.OracleMesh(m)
    ps_o, Th_o, u_o = om.hdc_run(s["ps"], s["Theta"], s["u"], 300.0, 20)
    g = mpdc.Mesh(m)
    for policy in ("DBL", "MIX"):
        _say("hdc G6x30 20 steps", policy, "autotuned, graph")
        st, (ps, Th, u) = gpu_hdc(mpdc, g, s, K, 300.0, 20, getattr(mpdc, "POLICY_" + policy), graph=True,
                                  autotune=True)
        e = (rel_l2(ps, ps_o, m["areaCell"]), rel_l2(Th, Th_o, m["areaCell"]), rel_l2(u, u_o))
        du = rel_l2(u - s["u"], u_o - s["u"])
        _say("  ps %.3e  Theta %.3e  u %.3e  du %.3e" % (e + (du,)))
        if policy == "DBL":
            assert max(e) <= DBL_TOL and du <= 1e-9
        else:
            assert e[0] <= MIX_TOL and e[1] <= MIX_TOL and e[2] <= 1e-3


def test_hdc_ensemble_g7x30x16_2_steps(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(7)
    K, M = 30, 16
    base = ic.hdc_jet(m, K, seed=2000)
    ens = ic.ensemble(base, M, sigma=0.1, seed=5000)
    om = oracle_mod.OracleMesh(m)
    g = mpdc.Mesh(m)
    ref = {}
    for j in (0, M - 1):
        _say("hdc G7x30 member %d 2 steps: oracle" % j)
        ref[j] = om.hdc_run(ens["ps"][:, j], ens["Theta"][:, :, j], ens["u"][:, :, j], 150.0, 2)
    for policy in ("DBL", "MIX"):
        _say("hdc G7x30x16 2 steps", policy, "autotuned, graph")
        st, (ps, Th, u) = gpu_hdc(mpdc, g, ens, K, 150.0, 2, getattr(mpdc, "POLICY_" + policy), M=M, graph=True,
                                  autotune=True)
        for j, (ps_o, Th_o, u_o) in ref.items():
            e = (rel_l2(ps[:, j], ps_o, m["areaCell"]), rel_l2(Th[:, :, j], Th_o, m["areaCell"]),
                 rel_l2(u[:, :, j], u_o))
            _say("  member %d: ps %.3e  Theta %.3e  u %.3e" % ((j,) + e))
            if policy == "DBL":
                assert max(e) <= DBL_TOL
            else:
                assert e[0] <= MIX_TOL and e[1] <= MIX_TOL and e[2] <= 1e-3


def test_ndc_g8x60_1_step(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(8)
    K = 60
    s = ic.nh_warm_bubble(m, K, seed=4000)
    om = oracle_mod.OracleMesh(m)
    names = ["ps", "Theta", "u", "w", "phi"]
    _say("ndc G8x60 1 step: oracle, and its sensitivity to a 1e-15 perturbation of Theta")
    ref = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], 60.0, 1)
    r = np.random.default_rng(9)
    Thp = s["Theta"] * (1.0 + 1e-15 * r.standard_normal(s["Theta"].shape))
    refp = om.ndc_run(s["ps"], Thp, s["u"], s["w"], s["phi"], 60.0, 1)
    sens = {n: rel_l2(a, b) for n, a, b in zip(names, refp, ref)}
    _say("  oracle sensitivity " + "  ".join("%s %.3e" % kv for kv in sens.items()))
    g = mpdc.Mesh(m)
    for policy in ("DBL", "MIX"):
        _say("ndc G8x60 1 step", policy, "autotuned, graph")
        st, out = gpu_ndc(mpdc, g, s, K, 60.0, 1, getattr(mpdc, "POLICY_" + policy), graph=True, autotune=True)
        errs = {n: rel_l2(x, rr) for n, x, rr in zip(names, out, ref)}
        _say("  " + "  ".join("%s %.3e" % kv for kv in errs.items()))
        assert all(np.isfinite(x).all() for x in out)
        if policy == "DBL":
            for n in names:
                assert errs[n] <= max(DBL_TOL, 10.0 * sens[n]), n
        else:
            assert errs["ps"] <= MIX_TOL and errs["Theta"] <= MIX_TOL and errs["phi"] <= MIX_TOL


def test_tracer_g8x30x8_1_step(mpdc, oracle_mod, mesh_cache):
    m = mesh_cache(8)
    tr = ic.tracer_solid_body(m, 30, 8, seed=3000)
    om = oracle_mod.OracleMesh(m)
    _say("tracer G8x30x8 1 step: oracle")
    dpi_o, q_o = om.tracer_run(tr["F"], tr["dpi"], tr["q"], 300.0, 1)
    g = mpdc.Mesh(m)
    for policy in ("DBL", "MIX"):
        _say("tracer G8x30x8 1 step", policy, "autotuned, graph")
        st, dpi, q = gpu_tracer(mpdc, g, tr, 300.0, 1, getattr(mpdc, "POLICY_" + policy), graph=True,
                                autotune=True)
        eq = max(rel_l2(q[:, :, t], q_o[:, :, t], m["areaCell"]) for t in range(q.shape[2]))
        ed = rel_l2(dpi, dpi_o, m["areaCell"])
        _say("  q %.3e  dpi %.3e  min %.3e max %.3e" % (eq, ed, q.min(), q.max()))
        assert ed <= DBL_TOL
        assert q.min() >= -1e-6 and q.max() <= 1.0 + 1e-6
        assert eq <= (DBL_TOL if policy == "DBL" else MIX_TOL)
