"""The iterative precision search of Section 2.2 over a per-term precision table.

The paper lowers the precision of selected terms one change at a time and
keeps a change only if the overall error of a run against the all-FP64 run,

    E = max(L(ps), L(vor)),   L(x) = max(L1, L2, Linf)         (Eqs. 1-2)

(normalised area-weighted norms of the surface pressure and of the relative
vorticity), stays within alpha = 0.05; every accepted change is the base of
the next.  Here the changes are the terms of the hydrostatic dycore's stage
(``mpdc.TERMS``: mass flux, divergence, kinetic energy, vorticity, vertex
mass, Coriolis, theta flux, vertical advection, column diagnostics, pressure
gradient), switched one at a time from FP64 to FP32 in the library's
per-term engine (``POLICY_TERMS`` with the ``term_fp32`` bit mask), in the
order of ``ORDER``: the advective terms first (the paper's computational
burden), the precision-sensitive ones last.  Every run, the norms and the
vorticity are computed on the GPU through the C ABI (``mpdc_diagnostics``
with ``MPDC_FIELD_VORT``).

The test state.  The paper searches on a dry baroclinic wave.  The default
state here is a baroclinic jet of its own (``inputs.initial.hdc_baroclinic_jet``:
zonal wind u0 sin^2(2 lat), zero at the surface and strongest near 250 hPa,
in gradient-wind and thermal-wind balance over a flat surface, plus a local
wind bump that starts the wave); the isothermal barotropic jet u0 cos^2(lat)
is the alternative (``--state barotropic``).

The window.  The paper runs 10 days in a model with its own dissipation.
This dry core has none, and on either jet any rounding difference grows:
after 10 days even an FP64 run whose initial Theta is perturbed by the FP32
unit roundoff is far outside alpha, so a 10-day window would reject every
FP32 term, whatever its accuracy.  The window is therefore set from the
FP64 model alone, before any FP32 term is tried: the longest whole number
of days, up to 10, over which an FP64 run with Theta perturbed by 2^-24 (an
FP32-sized uncertainty of the initial state) stays within alpha/2 of the
unperturbed run -- the horizon over which the model can tell FP32-level
differences apart at all.  Beside the search the tool reports E of the
mixed policy's split and of all-FP32, and of FP64 runs perturbed by 1e-14
and 2^-24.

Usage: python -m paper_2404_08849_amd.precision_search [--level 6] [--days D] [--alpha 0.05]
       [--state baroclinic|barotropic] [--terrain]
"""
import argparse
import json

import numpy as np

from .inputs import initial as ic

# the order in which the terms are lowered: advective terms first
ORDER = ["Coriolis", "theta flux", "kinetic energy", "vertical advection", "mass flux", "vorticity", "divergence",
         "vertex mass", "column diagnostics", "pressure gradient"]


def _state(mpdc, g, s, K, dt, policy, mask=0, phis=None, perturb=0.0):
    if perturb:
        r = np.random.default_rng(77)
        s = dict(s, Theta=s["Theta"] * (1.0 + perturb * r.standard_normal(s["Theta"].shape)))
    pol = policy if isinstance(policy, int) else getattr(mpdc, "POLICY_" + policy)
    st = mpdc.State(g, mpdc.MODEL_HDC, pol, K=K, dt=dt, sigma=ic.sigma_interfaces(K),
                    term_fp32=mask if pol == mpdc.POLICY_TERMS else 0)
    if phis is not None:
        st.state_write(mpdc.FIELD_PHIS, phis)
    st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
    st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
    st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
    st.set_graph(True)
    return st


def _advance(st, nsteps):
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        st.dycore_step(nsteps, stream=stream)
        torch.cuda.synchronize()


def _run(mpdc, g, s, K, dt, nsteps, policy, phis=None, perturb=0.0, mask=0):
    st = _state(mpdc, g, s, K, dt, policy, mask, phis, perturb)
    _advance(st, nsteps)
    return st


def error_measure(mpdc, st, ref):
    """E of Eq. 1 for state st against the reference state ref (both on the GPU)."""
    norms = {}
    for name, f in (("ps", mpdc.FIELD_PS), ("vor", mpdc.FIELD_VORT)):
        d = st.diagnostics(f, ref.state_read_device(f), check=False)
        norms[name] = max(d["l1"], d["l2"], d["linf"])
    return max(norms.values()), norms


def predictability_window(mpdc, g, s, K, dt, alpha, phis=None, max_days=10, eps=2.0 ** -24, log=print):
    """The longest whole number of days (at least 1, at most max_days) over which
    an FP64 run with Theta perturbed by eps stays within alpha/2 of the
    unperturbed FP64 run; returns (days, [E after each day])."""
    per_day = int(round(86400.0 / dt))
    ref = _state(mpdc, g, s, K, dt, "DBL", phis=phis)
    pert = _state(mpdc, g, s, K, dt, "DBL", phis=phis, perturb=eps)
    Es, days = [], 0
    for d in range(1, max_days + 1):
        _advance(ref, per_day)
        _advance(pert, per_day)
        E, _ = error_measure(mpdc, pert, ref)
        Es.append(E)
        log("  day %2d: FP64 with Theta perturbed by %.2g: E = %.3e" % (d, eps, E))
        if E > 0.5 * alpha:
            break
        days = d
    return max(days, 1), Es


STATES = ("baroclinic", "barotropic")


def initial_state(mesh, K, state):
    """The search's test state: the baroclinic jet (zonal wind u0 sin^2(2 lat)
    growing from zero at the surface to a maximum near 250 hPa, in thermal-wind
    balance, with a local wind bump that starts a baroclinic wave) or the
    isothermal barotropic jet u0 cos^2(lat) with the same kind of bump."""
    if state == "baroclinic":
        return ic.hdc_baroclinic_jet(mesh, K, seed=2000)
    if state == "barotropic":
        return ic.hdc_jet(mesh, K, seed=2000)
    raise ValueError("state must be one of %s" % (STATES,))


def search(level=6, K=30, days=None, dt=None, alpha=0.05, terrain=False, order=ORDER, state="baroclinic",
           log=print):
    """The per-term search on a hydrostatic jet (optionally over a mountain);
    returns a dict: the window, every trial, the accepted FP32 terms and mask."""
    import paper_2404_08849_amd.mpdc as mpdc
    from .inputs.meshgen import icosahedral_mesh
    mesh = icosahedral_mesh(level)
    if dt is None:
        dt = 300.0 * 2 ** (6 - level)          # the G6 workload's step, scaled with the mesh spacing
    s = initial_state(mesh, K, state)
    phis = None
    if terrain:
        phis = ic.mountain(mesh)
        rest = ic.hdc_rest_over_terrain(mesh, K, phis)
        s = dict(ps=rest["ps"], Theta=rest["Theta"], u=s["u"])
    g = mpdc.Mesh(mesh)
    window_log = None
    if days is None:
        log("window: FP64 predictability at FP32 level, %s jet, G%d x %d, dt %.1f s" % (state, level, K, dt))
        days, window_log = predictability_window(mpdc, g, s, K, dt, alpha, phis, log=log)
    nsteps = int(round(days * 86400.0 / dt))
    log("reference: DBL, G%d x %d, %d steps of %.1f s (%.1f days)" % (level, K, nsteps, dt, nsteps * dt / 86400.0))
    ref = _run(mpdc, g, s, K, dt, nsteps, "DBL", phis)
    trials = []

    def trial(name, **kw):
        st = _run(mpdc, g, s, K, dt, nsteps, kw.pop("policy", "TERMS"), phis, **kw)
        E, norms = error_measure(mpdc, st, ref)
        del st
        return E, norms

    for name, eps in (("FP64, Theta perturbed by 1e-14", 1e-14), ("FP64, Theta perturbed by 2^-24", 2.0 ** -24)):
        E, n = trial(name, policy="DBL", perturb=eps)
        log("%-34s E = %.3e (L(ps) %.3e, L(vor) %.3e)  [reference]" % (name, E, n["ps"], n["vor"]))
        trials.append(dict(name=name, E=E, L_ps=n["ps"], L_vor=n["vor"], reference=True))
    accepted = 0
    for term in order:
        mask = accepted | (1 << mpdc.TERM_BIT[term])
        E, n = trial(term, mask=mask)
        ok = bool(E <= alpha)
        if ok:
            accepted = mask
        log("%-34s E = %.3e (L(ps) %.3e, L(vor) %.3e)  %s" % ("FP32 " + term, E, n["ps"], n["vor"],
                                                             "accepted" if ok else "rejected"))
        trials.append(dict(name=term, mask=mask, E=E, L_ps=n["ps"], L_vor=n["vor"], accepted=ok))
    for name, mask in (("the mixed policy's split", mpdc.TERMS_MIX), ("all terms FP32", (1 << len(mpdc.TERMS)) - 1)):
        E, n = trial(name, mask=mask)
        log("%-34s E = %.3e (L(ps) %.3e, L(vor) %.3e)  [reference]" % (name, E, n["ps"], n["vor"]))
        trials.append(dict(name=name, mask=mask, E=E, L_ps=n["ps"], L_vor=n["vor"], reference=True))
    fp32 = [t for t in mpdc.TERMS if accepted & (1 << mpdc.TERM_BIT[t])]
    return dict(state=state, days=days, dt=dt, steps=nsteps, window_log=window_log, alpha=alpha, trials=trials,
                accepted_mask=accepted, fp32_terms=fp32,
                fp64_terms=[t for t in mpdc.TERMS if t not in fp32])


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--level", type=int, default=6)
    p.add_argument("--levels", type=int, default=30, help="layers K")
    p.add_argument("--days", type=float, default=None, help="fixed window (default: the FP64 predictability window)")
    p.add_argument("--dt", type=float, default=None)
    p.add_argument("--alpha", type=float, default=0.05)
    p.add_argument("--terrain", action="store_true", help="the jet over a 3 km mountain")
    p.add_argument("--state", default="baroclinic", choices=STATES)
    a = p.parse_args()
    print(json.dumps(search(a.level, a.levels, a.days, a.dt, a.alpha, a.terrain, state=a.state)))


if __name__ == "__main__":
    main()
