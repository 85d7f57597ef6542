"""Tracer transport with one cell per work-group (the shape whose per-cell and
per-edge tables are read with scalar loads).

* bitwise the same mixing ratios and layer masses as the general shape (128
  threads per work-group), for every legal number of tracers per lane, in
  the three policies, on G3 x 30 levels x 8 tracers (one to four waves per
  work-group) and on G4 x 3 levels x 8 tracers (work-groups of 3 to 24
  lanes);
* against the FP64 oracle on the same seeded inputs, within the bars of the
  other tracer parity tests.
"""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import DBL_TOL, MIX_TOL, compare, compare_dbl

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


def _run(mpdc, g, tr, policy, vpl, group, dt, n):
    K, T = tr["q"].shape[1], tr["q"].shape[2]
    st = mpdc.State(g, mpdc.MODEL_TRACER, policy, K=K, T=T, dt=dt)
    for kid in range(3):
        st.set_kernel_launch(kid, vpl, group)
    assert [st.get_kernel_launch(k) for k in range(3)] == [(vpl, group)] * 3
    st.state_write(mpdc.FIELD_TR_FLUX, tr["F"])
    st.state_write(mpdc.FIELD_TR_DPI, tr["dpi"])
    st.state_write(mpdc.FIELD_TR_Q, tr["q"])
    st.tracer_step(n)
    return st.state_read(mpdc.FIELD_TR_DPI), st.state_read(mpdc.FIELD_TR_Q)


@pytest.mark.parametrize("policy", ["DBL", "MIX", "SGL"])
@pytest.mark.parametrize("level,K", [(3, 30), (4, 3)])
def test_one_cell_per_work_group_is_bitwise_identical(mpdc, mesh_cache, policy, level, K):
    m = mesh_cache(level)
    T = 8
    tr = ic.tracer_solid_body(m, K, T, seed=3000)
    g = mpdc.Mesh(m)
    pol = getattr(mpdc, "POLICY_" + policy)
    vpls = (1, 2, 4, 8) if policy == "MIX" else (1, 2, 4)   # eight FP32 tracers per lane: MIX
    for vpl in vpls:
        _say("tracer G%d x %d x %d %s, %d tracers per lane: 128 threads, then one cell per work-group"
             % (level, K, T, policy, vpl))
        ref = _run(mpdc, g, tr, pol, vpl, 128, 3000.0, 3)
        out = _run(mpdc, g, tr, pol, vpl, 1, 3000.0, 3)
        assert np.isfinite(out[1]).all()
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_one_cell_per_work_group_matches_oracle(mpdc, mesh_cache, policy):
    import oracle
    m = mesh_cache(3)
    K, T = 30, 8
    tr = ic.tracer_solid_body(m, K, T, seed=3000)
    dpi_o, q_o = oracle.OracleMesh(m).tracer_run(tr["F"], tr["dpi"], tr["q"], 3000.0, 3)
    g = mpdc.Mesh(m)
    vpl = 4
    _say("tracer G3 x %d x %d %s, one cell per work-group, 3 steps" % (K, T, policy))
    dpi, q = _run(mpdc, g, tr, getattr(mpdc, "POLICY_" + policy), vpl, 1, 3000.0, 3)
    compare_dbl("dpi", dpi, dpi_o)
    tol = DBL_TOL if policy == "DBL" else MIX_TOL
    for t in range(T):
        if np.abs(q_o[:, :, t]).max() > 0:
            compare("q%d" % t, q[:, :, t], q_o[:, :, t], m["areaCell"], tol, tol)
    assert q.min() >= -1e-6 and q.max() <= 1.0 + 1e-6
