"""The stored FP64 oracle samples of the full-size workloads (CPU): present,
shaped for their workload, sampled at the 12 pentagons and where the state
moves, and taken on the mesh the generator builds today (checked for the G7
case, whose mesh takes seconds to build)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize_refs as refs   # noqa: E402


@pytest.mark.parametrize("case", sorted(refs.CASES))
def test_reference_file_is_complete(case):
    c = refs.CASES[case]
    r = dict(np.load(refs.ref_path(case)))
    assert int(r["nsteps"]) == 10
    n = 10 * 4 ** c["level"] + 2
    cells, edges = r["cells"], r["edges"]
    assert np.all(np.diff(cells) > 0) and cells[-1] < n and len(cells) >= refs.NSAMPLE + 12
    assert np.all(np.diff(edges) > 0) and edges[-1] < 30 * 4 ** c["level"]
    assert int(r["mesh_sig"][0]) == n
    K = c["K"]
    if c["model"] == "NDC":
        assert r["Theta"].shape == (len(cells), K) and r["w"].shape == (len(cells), K + 1)
        assert r["u"].shape == (len(edges), K) and r["phi"].shape == (len(cells), K + 1)
        assert np.abs(r["w"]).max() > 1e-3          # the sample holds the rising bubble
        assert (np.abs(r["w"]).max(axis=1) > 1e-6).sum() >= 400
    elif c["model"] == "TRACER":
        assert r["q"].shape == (len(cells), K, c["T"]) and r["tracer_mass"].shape == (c["T"],)
        assert r["q"].min() >= -1e-15 and r["q"].max() <= 1.0 + 1e-15    # bounds kept to rounding
    elif c["model"] == "HDC":
        assert r["ps"].shape == (len(cells),) and r["u"].shape == (len(edges), K)
    else:
        for j in r["members"]:
            assert r["ps_%d" % j].shape == (len(cells),) and r["u_%d" % j].shape == (len(edges), K)
        assert not np.array_equal(r["u_0"], r["u_15"])
    for v in r.values():
        assert np.isfinite(v).all()


def test_samples_include_the_pentagons_and_the_mesh_is_unchanged():
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    case = "ens_g7x30x16"
    r = dict(np.load(refs.ref_path(case)))
    m = icosahedral_mesh(refs.CASES[case]["level"])
    assert np.allclose(refs.mesh_signature(m), r["mesh_sig"], rtol=1e-14, atol=0)
    cells, edges = refs.sample_entities(m)
    assert np.isin(cells, r["cells"]).all() and np.isin(edges, r["edges"]).all()
    pent = np.nonzero(np.diff(m["eoc_offset"]) == 5)[0]
    assert len(pent) == 12 and np.isin(pent, cells).all()
