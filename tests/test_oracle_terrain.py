"""Pins of the oracle's hydrostatic pressure-gradient term over terrain (CPU).

With a surface geopotential phi_s the geopotential of the hydrostatic model
is integrated upwards from phi_s (Eq. 8), and over a mountain the two terms of
the pressure-gradient force (alpha grad p and grad phi on sigma surfaces)
nearly cancel -- the term whose precision sensitivity the paper reports.
For an isothermal atmosphere at rest over a mountain (an exact steady state
of the continuous equations):

* the discrete force in the lower half of the column (away from the
  vertical truncation at the model top, which no horizontal refinement
  removes) falls as the mesh is refined, G3 -> G4 -> G5, with order above
  1.5 from G4 to G5, and is over two orders of magnitude below either
  cancelling term;
* a flat surface gives exactly zero force;
* adding a constant to phi_s changes the force only by rounding;
* the run with phi_s = 0 equals the run without terrain bitwise.
"""
import numpy as np

from oracle import OracleMesh
from paper_2404_08849_amd.inputs import initial as ic


def test_rest_over_mountain_converges(mesh_cache):
    errs = []
    for lev in (3, 4, 5):
        m = mesh_cache(lev)
        om = OracleMesh(m)
        phis = ic.mountain(m)
        s = ic.hdc_rest_over_terrain(m, 10, phis)
        pgf = om.hdc_pgf(s["ps"], s["Theta"], phis=phis)
        errs.append(np.abs(pgf[:, 5:]).max())
    errs = np.array(errs)
    assert errs[0] > errs[1] > errs[2]
    assert np.log2(errs[1] / errs[2]) > 1.5
    # each cancelling term is over two orders of magnitude larger than what is left
    m = mesh_cache(5)
    phis = ic.mountain(m)
    c1, c2 = m["cells_on_edge"][:, 0], m["cells_on_edge"][:, 1]
    assert np.abs((phis[c2] - phis[c1]) / m["dEdge"]).max() > 300.0 * errs[2]


def test_flat_and_shifted_surface(mesh_cache):
    m = mesh_cache(4)
    om = OracleMesh(m)
    K = 8
    flat = ic.hdc_rest_over_terrain(m, K, np.zeros(m["nCells"]))
    assert np.array_equal(om.hdc_pgf(flat["ps"], flat["Theta"]), np.zeros((m["nEdges"], K)))
    phis = ic.mountain(m)
    s = ic.hdc_rest_over_terrain(m, K, phis)
    a = om.hdc_pgf(s["ps"], s["Theta"], phis=phis)
    b = om.hdc_pgf(s["ps"], s["Theta"], phis=phis + 5.0e3)
    scale = np.abs((phis[m["cells_on_edge"][:, 1]] - phis[m["cells_on_edge"][:, 0]]) / m["dEdge"]).max()
    assert np.abs(a - b).max() <= 1e-11 * scale
    j = ic.hdc_jet(m, K, seed=2000)
    r0 = om.hdc_run(j["ps"], j["Theta"], j["u"], 600.0, 3)
    r1 = om.hdc_run(j["ps"], j["Theta"], j["u"], 600.0, 3, phis=np.zeros(m["nCells"]))
    for x, y in zip(r0, r1):
        assert np.array_equal(x, y)
