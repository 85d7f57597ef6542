"""GPU parity at the largest hydrostatic workload, G9 x 30 (2,621,442 cells;
the G9 column of Table 1), in the benchmark's launch configuration
(autotuned shapes, HIP-graph replay): 10 steps of dt = 37.5 s against the
FP64 oracle's 10 steps stored by `tests/golden/make_fullsize_refs.py`
(every level of the pentagons, their edges and 500 random cells and edges),
to the bars of the other full-size tests, plus the global mass over the
whole field.  Named to run last: generating the G9 mesh takes about a
minute on the host."""
import os
import sys

import numpy as np
import pytest

from gpu_helpers import MIX_TOL, MIX_U_TOL, compare, compare_dbl, gpu_hdc

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize_refs as refs   # noqa: E402

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


@pytest.mark.timeout(900)
def test_hdc_g9x30_10_steps(mpdc):
    case = "hdc_g9x30"
    c = refs.CASES[case]
    ref = dict(np.load(refs.ref_path(case)))
    _say("hdc G9x30: mesh and input")
    m, s, sig = refs.build_case(case)
    assert np.allclose(refs.mesh_signature(m), ref["mesh_sig"], rtol=1e-14, atol=0)
    assert np.allclose(sig, ref["state_sig"], rtol=1e-14, atol=0)
    cells, edges = ref["cells"], ref["edges"]
    g = mpdc.Mesh(m)
    A = m["areaCell"]
    m0 = float(np.sum(A * (s["ps"] - 1000.0)))
    for policy in ("DBL", "MIX"):
        _say("hdc G9x30 10 steps", policy, "autotuned, graph")
        st, (ps, Th, u) = gpu_hdc(mpdc, g, s, c["K"], c["dt"], refs.NSTEPS, getattr(mpdc, "POLICY_" + policy),
                                  graph=True, autotune=True)
        assert np.isfinite(ps).all() and np.isfinite(Th).all() and np.isfinite(u).all()
        if policy == "DBL":
            compare_dbl("ps", ps[cells], ref["ps"])
            compare_dbl("Theta", Th[cells], ref["Theta"])
            compare_dbl("u", u[edges], ref["u"])
        else:
            compare("ps", ps[cells], ref["ps"], None, MIX_TOL, MIX_TOL)
            compare("Theta", Th[cells], ref["Theta"], None, MIX_TOL, MIX_TOL)
            compare("u", u[edges], ref["u"], None, MIX_U_TOL, MIX_U_TOL)
        m1 = float(np.sum(A * (ps - 1000.0)))
        _say("    mass drift %.3e  vs oracle %.3e" % (abs(m1 - m0) / m0, abs(m1 - float(ref["mass"])) / m0))
        assert abs(m1 - m0) <= 1e-13 * m0 and abs(m1 - float(ref["mass"])) <= 1e-13 * m0
        del st, ps, Th, u
