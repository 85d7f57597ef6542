"""The iterative precision search of Section 2.2 over the library's policies.

The paper lowers the precision of selected terms one change at a time and
keeps a change only if the overall error of a run against the all-FP64 run,

    E = max(L(ps), L(vor)),   L(x) = max(L1, L2, Linf)         (Eqs. 1-2)

(normalised area-weighted norms of the surface pressure and of the relative
vorticity), stays within alpha = 0.05.  Here the changes are the library's
precision policies, ordered by how much they take out of FP64: MIX (the
paper's split) first, then each further reduction built on MIX (MIX_F32_DIV:
FP32 continuity divergence; MIX_PGF32: FP32 column diagnostics and
pressure-gradient term; SGL: every term in FP32).  A reduction is tried only on top of an accepted
MIX.  Every run, the norms and the vorticity are computed on the GPU through
the C ABI (``mpdc_diagnostics`` with ``MPDC_FIELD_VORT``).

Beside the candidates the search reports the run's intrinsic sensitivity: E
of an all-FP64 run whose initial Theta carries a 1e-14 relative perturbation,
and of one whose perturbation is the FP32 unit roundoff (2^-24).  This model
has no explicit dissipation, so on an unstable jet any rounding difference
grows; a candidate whose E is near the first differs from FP64 no more than
FP64 differs from itself, and one whose E is near the second differs no more
than an FP32-sized uncertainty in the initial state would make it (the
ensemble-spread argument of Section 4.4).  These references are reported,
not used for acceptance, which follows Eq. 1 with alpha.

Usage: python -m paper_2404_08849_amd.precision_search [--level 6] [--days 10] [--alpha 0.05]
"""
import argparse
import json

import numpy as np

from .inputs import initial as ic

# candidate reductions in the order they are tried, each with the
# configuration it builds on
CANDIDATES = [("MIX", "DBL"), ("MIX_F32_DIV", "MIX"), ("MIX_PGF32", "MIX"), ("SGL", "MIX")]


def _run(mpdc, g, s, K, dt, nsteps, policy, phis=None, perturb=0.0):
    import torch
    if perturb:
        r = np.random.default_rng(77)
        s = dict(s, Theta=s["Theta"] * (1.0 + perturb * r.standard_normal(s["Theta"].shape)))
    st = mpdc.State(g, mpdc.MODEL_HDC, getattr(mpdc, "POLICY_" + policy), K=K, dt=dt,
                    sigma=ic.sigma_interfaces(K))
    if phis is not None:
        st.state_write(mpdc.FIELD_PHIS, phis)
    st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
    st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
    st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
    stream = torch.cuda.Stream()
    st.set_graph(True)
    with torch.cuda.stream(stream):
        st.dycore_step(nsteps, stream=stream)
        torch.cuda.synchronize()
    return st


def error_measure(mpdc, st, ref):
    """E of Eq. 1 for state st against the reference state ref (both on the GPU)."""
    norms = {}
    for name, f in (("ps", mpdc.FIELD_PS), ("vor", mpdc.FIELD_VORT)):
        d = st.diagnostics(f, ref.state_read_device(f), check=False)
        norms[name] = max(d["l1"], d["l2"], d["linf"])
    return max(norms.values()), norms


def search(level=6, K=30, days=10.0, dt=None, alpha=0.05, terrain=False, candidates=CANDIDATES, log=print):
    """Run the search on the hydrostatic jet (optionally over a mountain);
    returns the list of trials and the final accepted configuration."""
    import paper_2404_08849_amd.mpdc as mpdc
    from .inputs.meshgen import icosahedral_mesh
    mesh = icosahedral_mesh(level)
    if dt is None:
        dt = 300.0 * 2 ** (6 - level)          # the G6 workload's step, scaled with the mesh spacing
    nsteps = int(round(days * 86400.0 / dt))
    s = ic.hdc_jet(mesh, K, seed=2000)
    phis = None
    if terrain:
        phis = ic.mountain(mesh)
        rest = ic.hdc_rest_over_terrain(mesh, K, phis)
        s = dict(ps=rest["ps"], Theta=rest["Theta"], u=s["u"])
    g = mpdc.Mesh(mesh)
    log("reference: DBL, G%d x %d, %d steps of %.1f s (%.1f days)" % (level, K, nsteps, dt, nsteps * dt / 86400.0))
    ref = _run(mpdc, g, s, K, dt, nsteps, "DBL", phis)
    accepted = {"DBL"}
    trials = []
    for name, eps in (("DBL+1e-14", 1e-14), ("DBL+6e-8", 2.0 ** -24)):
        E0, n0 = error_measure(mpdc, _run(mpdc, g, s, K, dt, nsteps, "DBL", phis, perturb=eps), ref)
        log("%-13s E = %.3e (L(ps) %.3e, L(vor) %.3e): FP64 run with Theta perturbed by %.2g (reference, not a candidate)"
            % (name, E0, n0["ps"], n0["vor"], eps))
        trials.append(dict(policy=name, base="DBL", E=E0, L_ps=n0["ps"], L_vor=n0["vor"], spread=True))
    for policy, base in candidates:
        if base not in accepted:
            trials.append(dict(policy=policy, base=base, skipped=True))
            log("%-13s skipped (builds on %s, not accepted)" % (policy, base))
            continue
        st = _run(mpdc, g, s, K, dt, nsteps, policy, phis)
        E, norms = error_measure(mpdc, st, ref)
        ok = bool(E <= alpha)
        if ok:
            accepted.add(policy)
        trials.append(dict(policy=policy, base=base, E=E, L_ps=norms["ps"], L_vor=norms["vor"], accepted=ok))
        log("%-13s E = %.3e (L(ps) %.3e, L(vor) %.3e): %s" % (policy, E, norms["ps"], norms["vor"],
                                                              "accepted" if ok else "rejected"))
        del st
    return trials, sorted(accepted)


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--level", type=int, default=6)
    p.add_argument("--levels", type=int, default=30, help="layers K")
    p.add_argument("--days", type=float, default=10.0)
    p.add_argument("--dt", type=float, default=None)
    p.add_argument("--alpha", type=float, default=0.05)
    p.add_argument("--terrain", action="store_true", help="the jet over a 3 km mountain")
    a = p.parse_args()
    trials, accepted = search(a.level, a.levels, a.days, a.dt, a.alpha, a.terrain)
    print(json.dumps({"trials": trials, "accepted": accepted}))


if __name__ == "__main__":
    main()
