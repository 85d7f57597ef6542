"""Invariance of the GPU path under a random relabelling of the mesh: the
cells, edges and vertices of a G4 mesh are renumbered (seeded permutations;
each cell keeps its counter-clockwise edge order and each edge its
orientation), the same state is stepped on both meshes, and the results,
mapped back, are bitwise identical -- every value depends on the stencil,
not on where an entity sits in memory (which is what the work-group
numbering and the autotuned shapes change)."""
import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic
from gpu_helpers import gpu_hdc, gpu_ndc, gpu_tracer
from mesh_relabel import relabel

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


@pytest.mark.parametrize("policy", ["DBL", "MIX"])
def test_hydrostatic_relabelled_mesh_is_bitwise_identical(mpdc, mesh_cache, policy):
    m = mesh_cache(4)
    K = 10
    s = ic.hdc_jet(m, K, seed=2000)
    mp, ic_, ie, iv = relabel(m)
    sp = dict(ps=s["ps"][ic_], Theta=s["Theta"][ic_], u=s["u"][ie])
    pol = getattr(mpdc, "POLICY_" + policy)
    _say("hdc G4x%d, 5 steps, %s: original and relabelled mesh" % (K, policy))
    _, a = gpu_hdc(mpdc, mpdc.Mesh(m), s, K, 600.0, 5, pol)
    _, b = gpu_hdc(mpdc, mpdc.Mesh(mp), sp, K, 600.0, 5, pol)
    assert np.array_equal(b[0], a[0][ic_]) and np.array_equal(b[1], a[1][ic_]) and np.array_equal(b[2], a[2][ie])


def test_nonhydrostatic_relabelled_mesh_is_bitwise_identical(mpdc, mesh_cache):
    m = mesh_cache(4)
    K = 10
    s = ic.nh_warm_bubble(m, K, rh=6.0e5, seed=4000)
    mp, ic_, ie, iv = relabel(m, seed=12)
    sp = dict(ps=s["ps"][ic_], Theta=s["Theta"][ic_], u=s["u"][ie], w=s["w"][ic_], phi=s["phi"][ic_])
    _say("ndc G4x%d, 3 steps, MIX: original and relabelled mesh" % K)
    _, a = gpu_ndc(mpdc, mpdc.Mesh(m), s, K, 60.0, 3, mpdc.POLICY_MIX)
    _, b = gpu_ndc(mpdc, mpdc.Mesh(mp), sp, K, 60.0, 3, mpdc.POLICY_MIX)
    for x, y, p in zip(a, b, (ic_, ic_, ie, ic_, ic_)):
        assert np.array_equal(y, x[p])


def test_tracer_relabelled_mesh_is_bitwise_identical(mpdc, mesh_cache):
    m = mesh_cache(4)
    tr = ic.tracer_solid_body(m, 5, 4, seed=3000)
    mp, ic_, ie, iv = relabel(m, seed=13)
    # the flux is oriented c1 -> c2 and the relabelling keeps each edge's orientation
    trp = dict(F=tr["F"][ie], dpi=tr["dpi"][ic_], q=tr["q"][ic_])
    _say("tracer G4x5x4, 3 steps, MIX: original and relabelled mesh")
    _, d1, q1 = gpu_tracer(mpdc, mpdc.Mesh(m), tr, 3000.0, 3, mpdc.POLICY_MIX)
    _, d2, q2 = gpu_tracer(mpdc, mpdc.Mesh(mp), trp, 3000.0, 3, mpdc.POLICY_MIX)
    assert np.array_equal(d2, d1[ic_]) and np.array_equal(q2, q1[ic_])
