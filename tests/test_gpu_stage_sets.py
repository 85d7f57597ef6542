"""GPU: the mixed policies whose RK stages store only the FP32 shadows of u and
Theta (MIX, MIX_F32_DIV, MIX_PGF32, SGL; the FP64 values of the first two
stages are written by no stage) never read those FP64 arrays.  A child
process with MPDC_POISON_STAGE_SETS=1 fills them with NaN at state creation;
its results must be finite and bitwise those of a run without the switch,
for one member and for an ensemble, in direct launches and graph replay."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2404_08849_amd.mpdc as mpdc
from paper_2404_08849_amd.inputs import initial as ic
from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
m = icosahedral_mesh(3)
g = mpdc.Mesh(m)
K = 8
out = {}
for name in ("MIX", "MIX_F32_DIV", "MIX_PGF32", "SGL", "MIX_BOX", "DBL"):
    for M, graph in ((1, False), (3, True)):
        base = ic.hdc_jet(m, K, seed=2000)
        s = ic.ensemble(base, M, sigma=0.1, seed=5000) if M > 1 else {k: v[..., None] for k, v in base.items()}
        st = mpdc.State(g, mpdc.MODEL_HDC, getattr(mpdc, "POLICY_" + name), K=K, M=M, dt=900.0,
                        sigma=ic.sigma_interfaces(K))
        st.state_write(mpdc.FIELD_PS, s["ps"])
        st.state_write(mpdc.FIELD_THETA, s["Theta"])
        st.state_write(mpdc.FIELD_U, s["u"])
        st.set_graph(graph)
        with torch.cuda.stream(torch.cuda.Stream()):
            st.dycore_step(4)
            torch.cuda.current_stream().synchronize()
        for f, fn in ((mpdc.FIELD_PS, "ps"), (mpdc.FIELD_THETA, "Theta"), (mpdc.FIELD_U, "u")):
            out["%s_%d_%s" % (name, M, fn)] = st.state_read(f)
np.savez(sys.argv[2], **out)
'''


def _run(tmp_path, poison):
    path = str(tmp_path / ("poison.npz" if poison else "plain.npz"))
    env = dict(os.environ)
    env.pop("MPDC_POISON_STAGE_SETS", None)
    if poison:
        env["MPDC_POISON_STAGE_SETS"] = "1"
    print("child run, poison=%s" % poison, flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, path], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return dict(np.load(path))


def test_mixed_stages_never_read_unwritten_fp64_state(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    plain = _run(tmp_path, False)
    poison = _run(tmp_path, True)
    for k, v in plain.items():
        assert np.isfinite(v).all(), k
        assert np.isfinite(poison[k]).all(), k
        assert np.array_equal(poison[k], v), k
