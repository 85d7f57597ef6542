"""Write the FP64 oracle's results of the full-size workloads after 10 steps,
sampled at a fixed set of cells and edges, for the full-size GPU parity tests.

Each case runs the oracle (plain C, FP64) on the seeded synthetic input the
GPU test builds, for 10 steps, then keeps every level of the 12 pentagons, of
their edges, of 500 random cells and edges, and of the 500 cells and 500
edges where the oracle's state changed most over the steps (the moving part
of a local disturbance such as the warm bubble, which a random sample of a
G8 mesh would almost never hit).  The stored file also holds a
signature of the mesh and of the initial state, so a test can tell that it
rebuilt the same input.  Only `oracle/` and the input generators are called.

    python tests/golden/make_fullsize_refs.py [case ...]

Cases: ndc_g8x60, tracer_g8x30x8, hdc_g9x30, ens_g7x30x16 (about 15 minutes
of host time on 8 cores in all).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

NSTEPS = 10
CASES = {
    "ndc_g8x60": dict(model="NDC", level=8, K=60, dt=60.0, seed=4000),
    "tracer_g8x30x8": dict(model="TRACER", level=8, K=30, T=8, dt=300.0, seed=3000),
    "hdc_g9x30": dict(model="HDC", level=9, K=30, dt=37.5, seed=2000),
    "ens_g7x30x16": dict(model="ENS", level=7, K=30, M=16, dt=150.0, seed=2000, ens_seed=5000, members=(0, 15)),
}
NSAMPLE = 500


def ref_path(case):
    return os.path.join(HERE, "fullsize_%s.npz" % case)


def mesh_signature(mesh):
    """Sums that change if the generated mesh changes in any bit that matters."""
    return np.array([mesh["nCells"], mesh["nEdges"], mesh["nVertices"],
                     float(np.sum(mesh["xCell"] * np.arange(1, 4))), float(np.sum(mesh["areaCell"])),
                     float(np.sum(mesh["dEdge"] * mesh["lEdge"])), float(np.sum(mesh["kiteArea"][:, 0])),
                     float(np.sum(mesh["cells_on_edge"][:, 1].astype(np.float64)))])


def state_signature(arrays):
    return np.array([float(np.sum(a)) for a in arrays] + [float(np.sum(np.abs(a))) for a in arrays])


def active(change, n=NSAMPLE):
    """Indices of the n entities whose largest change over their levels is
    largest (change: [entities][...])."""
    c = np.abs(change).reshape(change.shape[0], -1).max(axis=1)
    return np.argsort(-c, kind="stable")[:n]


def sample_entities(mesh, seed=7):
    """The 12 pentagons and their edges, plus NSAMPLE random cells and edges."""
    off = mesh["eoc_offset"]
    deg = np.diff(off)
    pent = np.nonzero(deg == 5)[0]
    pedges = np.concatenate([mesh["edges_on_cell"][off[i]:off[i + 1]] for i in pent])
    r = np.random.default_rng(seed)
    cells = np.unique(np.concatenate([pent, r.choice(mesh["nCells"], NSAMPLE, replace=False)]))
    edges = np.unique(np.concatenate([pedges, r.choice(mesh["nEdges"], NSAMPLE, replace=False)]))
    return cells.astype(np.int64), edges.astype(np.int64)


def build_case(case):
    """Mesh and seeded initial state of a case, exactly as the GPU test builds them."""
    from paper_2404_08849_amd.inputs import initial as ic
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    c = CASES[case]
    mesh = icosahedral_mesh(c["level"])
    if c["model"] == "NDC":
        st = ic.nh_warm_bubble(mesh, c["K"], seed=c["seed"])
        sig = state_signature([st["Theta"], st["u"], st["phi"]])
    elif c["model"] == "TRACER":
        st = ic.tracer_solid_body(mesh, c["K"], c["T"], seed=c["seed"])
        sig = state_signature([st["F"], st["dpi"], st["q"]])
    elif c["model"] == "HDC":
        st = ic.hdc_jet(mesh, c["K"], seed=c["seed"])
        sig = state_signature([st["ps"], st["Theta"], st["u"]])
    else:
        base = ic.hdc_jet(mesh, c["K"], seed=c["seed"])
        st = ic.ensemble(base, c["M"], sigma=0.1, seed=c["ens_seed"])
        sig = state_signature([st["ps"], st["Theta"], st["u"]])
    return mesh, st, sig


def make(case):
    from oracle import OracleMesh
    c = CASES[case]
    t0 = time.perf_counter()
    mesh, st, sig = build_case(case)
    cells, edges = sample_entities(mesh)
    om = OracleMesh(mesh)
    out = dict(mesh_sig=mesh_signature(mesh), state_sig=sig, nsteps=NSTEPS)
    area = mesh["areaCell"]
    res = {}
    if c["model"] == "NDC":
        ps, Th, u, w, phi = om.ndc_run(st["ps"], st["Theta"], st["u"], st["w"], st["phi"], c["dt"], NSTEPS)
        res = dict(ps=ps, Theta=Th, u=u, w=w, phi=phi)
        acell, aedge = active(w - st["w"]), active(u - st["u"])
        out["mass"] = float(np.sum(area * (ps - 1000.0)))
    elif c["model"] == "TRACER":
        dpi, q = om.tracer_run(st["F"], st["dpi"], st["q"], c["dt"], NSTEPS)
        res = dict(dpi=dpi, q=q)
        acell, aedge = active(q - st["q"]), np.zeros(0, np.int64)
        out["tracer_mass"] = np.einsum("i,ik,ikt->t", area, dpi, q)
    elif c["model"] == "HDC":
        ps, Th, u = om.hdc_run(st["ps"], st["Theta"], st["u"], c["dt"], NSTEPS)
        res = dict(ps=ps, Theta=Th, u=u)
        acell, aedge = active(ps - st["ps"]), active(u - st["u"])
        out["mass"] = float(np.sum(area * (ps - 1000.0)))
    else:
        out["members"] = np.array(c["members"])
        acell, aedge = [], []
        for j in c["members"]:
            ps, Th, u = om.hdc_run(st["ps"][:, j], st["Theta"][:, :, j], st["u"][:, :, j], c["dt"], NSTEPS)
            res.update({"ps_%d" % j: ps, "Theta_%d" % j: Th, "u_%d" % j: u})
            acell.append(active(ps - st["ps"][:, j]))
            aedge.append(active(u - st["u"][:, :, j]))
        acell, aedge = np.concatenate(acell), np.concatenate(aedge)
    cells = np.unique(np.concatenate([cells, acell])).astype(np.int64)
    edges = np.unique(np.concatenate([edges, aedge])).astype(np.int64)
    out.update(cells=cells, edges=edges)
    for k, v in res.items():
        out[k] = v[edges] if k.split("_")[0] == "u" else v[cells]
    np.savez_compressed(ref_path(case), **out)
    print("%s: %d cells, %d edges sampled, %.0f s" % (case, len(cells), len(edges), time.perf_counter() - t0),
          flush=True)


if __name__ == "__main__":
    for case in (sys.argv[1:] or list(CASES)):
        make(case)
