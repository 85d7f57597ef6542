"""Benchmark of the mixed-precision icosahedral dycore on one MI355X.

Default workload: the batched ensemble of the hydrostatic dry dycore
(continuity, theta_m transport, momentum with TRiSK Coriolis and FP64
pressure gradient; RK3 forward-backward): 16 members on the G7 icosahedral
mesh (163,842 cells) x 30 sigma levels, isothermal jet plus a seeded wind
perturbation with N(0, 0.1 m/s) member perturbations, dt = 150 s -- run in
the mixed policy (the paper's term split) and in all-FP64.  One "step" is
one full RK3 dycore step of all members (three stages, four kernels each,
one launch per operator for all members) replayed from a HIP graph.

Prints ONE JSON line: value = mixed-policy cell-level-steps/s with inputs
resident in HBM (cells x levels x members per second); the all-FP64 rate,
the mixed/FP64 speedup, the accuracy gate (mixed vs all-FP64 after the
workload's steps, and both against the FP64 oracle's stored 10-step
results), the roofline of the dominant kernel (algorithmic bytes / HIP-event
duration, against the 8 TB/s peak and against the library's own streaming
kernels), the median of five further timed repetitions, a secondary line for
the cache-resident G6 workload, and the FP64 oracle timed on the host cores
(N threads and 1 thread).

Other workloads (--workload): sw-g5, hdc-g6, tracer-g8, tracer3d-g8 (with the
vertical step), coupled-g6 (dycore, flux hand-over and tracer step), ndc-g8,
ens-g7 (default), hdc-g9.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X last-level (MALL / Infinity Cache) capacity: a launch whose
# algorithmic bytes fit here is cache-resident, not HBM-bound
MALL_BYTES = 256 * 2 ** 20
# the workloads whose FP64 oracle results after 10 steps are stored (sampled)
STORED_REFS = {"ens-g7": "ens_g7x30x16", "ndc-g8": "ndc_g8x60", "tracer-g8": "tracer_g8x30x8",
               "hdc-g9": "hdc_g9x30"}
KERNEL_NAMES = {
    "dycore": ["k_cell_a", "k_vertex", "k_cell_b", "k_edge"],
    "tracer": ["k_tr_low", "k_tr_limit", "k_tr_update", "k_tr_vert"],
}

WORKLOADS = {
    "sw-g5": dict(model="SW", level=5, K=1, M=1, T=0, dt=600.0, steps=10,
                  desc="shallow water G5 (10242 cells), geostrophic flow + bump, dt=600 s"),
    "hdc-g6": dict(model="HDC", level=6, K=30, M=1, T=0, dt=300.0, steps=20,
                   desc="hydrostatic dycore G6 (40962 cells) x 30 levels, jet + wind bump, dt=300 s"),
    "tracer-g8": dict(model="TRACER", level=8, K=30, M=1, T=8, dt=300.0, steps=10,
                      desc="tracer FCT transport G8 (655362 cells) x 30 levels x 8 tracers, solid-body rotation, dt=300 s"),
    "tracer3d-g8": dict(model="TRACER", level=8, K=30, M=1, T=8, dt=300.0, steps=10, vflux=True,
                        desc="tracer FCT transport G8 (655362 cells) x 30 levels x 8 tracers, solid-body rotation "
                             "plus a vertical mass flux (layer masses change by up to 0.1% a step), dt=300 s"),
    "ndc-g8": dict(model="NDC", level=8, K=60, M=1, T=0, dt=60.0, steps=10,
                   desc="non-hydrostatic dycore G8 (655362 cells) x 60 levels, warm bubble, dt=60 s"),
    "ens-g7": dict(model="HDC", level=7, K=30, M=16, T=0, dt=150.0, steps=20,
                   desc="hydrostatic dycore ensemble G7 (163842 cells) x 30 levels x 16 members, dt=150 s"),
    "coupled-g6": dict(model="COUPLED", level=6, K=30, M=1, T=8, dt=300.0, nsub=2, steps=10,
                       desc="hydrostatic dycore G6 (40962 cells) x 30 levels coupled to 8 tracers: one tracer step "
                            "(dt=600 s, with its vertical step) per 2 dycore steps (dt=300 s) on their accumulated "
                            "mass fluxes"),
    "hdc-g9": dict(model="HDC", level=9, K=30, M=1, T=0, dt=37.5, steps=10,
                   desc="hydrostatic dycore G9 (2621442 cells) x 30 levels, jet, dt=37.5 s"),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="ens-g7", choices=sorted(WORKLOADS))
    p.add_argument("--no-secondary", action="store_true", help="skip the cache-resident G6 secondary line")
    p.add_argument("--repeats", type=int, default=5, help="further timed repetitions of --steps steps (median)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-dbl", action="store_true", help="skip the all-FP64 timing")
    p.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the policy variants (MIX_BOX, MIX_DBL_MASS, MIX_F32_DIV, MIX_PGF32 and SGL of the "
                        "layered dycores; SGL of the tracer transport)")
    p.add_argument("--profile-steps", type=int, default=20,
                   help="steps run with HIP events between launches for per-kernel durations")
    p.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of this many MiB (HBM counter calibration)")
    p.add_argument("--shapes", default=None, metavar="JSON",
                   help='fixed launch shapes instead of autotuning, e.g. {"mix": [[2,16],[2,256],[2,16],[2,512]], '
                        '"dbl": [...]}: (values per lane, cells or threads per work-group) per kernel; '
                        'for coupled-g6 each policy holds {"dycore": [...], "tracer": [...]}')
    return p.parse_args()


def build_inputs(w):
    from paper_2404_08849_amd.inputs import initial as ic
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    mesh = icosahedral_mesh(w["level"])
    K, M, T = w["K"], w["M"], w["T"]
    if w["model"] == "SW":
        st = ic.sw_geostrophic(mesh, seed=1000)
    elif w["model"] == "HDC":
        base = ic.hdc_jet(mesh, K, seed=2000)
        st = ic.ensemble(base, M, sigma=0.1, seed=5000) if M > 1 else base
    elif w["model"] == "NDC":
        st = ic.nh_warm_bubble(mesh, K, seed=4000)
    else:
        st = ic.tracer_solid_body(mesh, K, T, seed=3000)
        if w.get("vflux"):
            # small enough that the layer masses stay positive over hundreds of steps (the
            # vertical step solves its tridiagonal systems whatever the Courant numbers)
            st["vflux"] = ic.tracer_vertical_flux(st["dpi"], w["dt"], amp=0.001, seed=3100)
    return mesh, st


def make_state(mpdc, g, w, st, policy, shapes=None):
    from paper_2404_08849_amd.inputs import initial as ic
    K, M, T = w["K"], w["M"], w["T"]
    model = getattr(mpdc, "MODEL_" + w["model"])
    s = mpdc.State(g, model, policy, K=K, M=M, T=T, dt=w["dt"],
                   sigma=ic.sigma_interfaces(K) if w["model"] != "SW" else None)
    for k, (v, grp) in enumerate(shapes or []):
        s.set_kernel_launch(k, v, grp)
    if w["model"] == "SW":
        s.state_write(mpdc.FIELD_H, st["h"])
        s.state_write(mpdc.FIELD_U, st["u"])
        s.state_write(mpdc.FIELD_B, st["b"])
    elif w["model"] == "TRACER":
        s.state_write(mpdc.FIELD_TR_FLUX, st["F"])
        s.state_write(mpdc.FIELD_TR_DPI, st["dpi"])
        s.state_write(mpdc.FIELD_TR_Q, st["q"])
        if "vflux" in st:
            s.state_write(mpdc.FIELD_TR_VFLUX, st["vflux"])
    else:
        exp = (lambda a: a) if M > 1 else (lambda a: a[..., None])
        s.state_write(mpdc.FIELD_PS, exp(st["ps"]))
        s.state_write(mpdc.FIELD_THETA, exp(st["Theta"]))
        s.state_write(mpdc.FIELD_U, exp(st["u"]))
        if w["model"] == "NDC":
            s.state_write(mpdc.FIELD_W, st["w"][..., None])
            s.state_write(mpdc.FIELD_PHI, st["phi"][..., None])
    return s


def step(s, w, n, stream):
    if w["model"] == "TRACER":
        s.tracer_step(n, stream=stream)
    else:
        s.dycore_step(n, stream=stream)


def key_field(mpdc, w):
    return {"SW": mpdc.FIELD_H, "TRACER": mpdc.FIELD_TR_Q}.get(w["model"], mpdc.FIELD_PS)


def timed_run(torch, mpdc, g, w, st, policy, steps, warmup, stream, autotune=True, fixed=None):
    s = make_state(mpdc, g, w, st, policy, fixed)
    if autotune and not fixed:
        with torch.cuda.stream(stream):
            s.autotune(stream=stream)
    nk = 3 if w["model"] == "TRACER" else 4
    shapes = [list(s.get_kernel_launch(k)) for k in range(nk)]
    s.set_graph(True)
    with torch.cuda.stream(stream):
        step(s, w, warmup, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(s, w, steps, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    s.launch_shapes = shapes
    return s, (t1 - t0) / max(steps, 1)


def kernel_times(torch, s, w, nsteps, stream, nreps=20):
    """Per-kernel mean launch duration with HIP events on the launch stream:
    `ms_in_step` from events recorded between the launches of nsteps real
    steps (continuing the timed run's state; each interval also holds the
    event and launch overhead), `ms` from events around nreps back-to-back
    launches of that kernel on the same inputs (the first RK stage's).  With
    the algorithmic bytes of the launch timed back to back (`bytes`) and their
    mean over the stages (`bytes_mean`, what a profiler's per-dispatch
    average covers)."""
    kind = "tracer" if w["model"] == "TRACER" else "dycore"
    with torch.cuda.stream(stream):
        prof = s.profile_steps(nsteps, stream=stream)
        # (the tracer's vertical step works in place, so it is timed inside the steps only)
        b2b = {kid: s.time_kernel(kid, nreps, stream=stream) for kid in prof if not (kind == "tracer" and kid == 3)}
    out = {}
    for kid, (ms, n) in prof.items():
        out[KERNEL_NAMES[kind][kid]] = dict(ms=b2b.get(kid, ms / n), ms_in_step=ms / n, launches=n,
                                            bytes=s.stage_kernel_bytes(kid, 0) if kid in b2b else s.kernel_bytes(kid),
                                            bytes_mean=s.kernel_bytes(kid))
    return out


def accuracy_run(torch, mpdc, g, w, st, stream, shapes, names=("DBL", "MIX")):
    """The policies for the workload's own step count from the same input, in
    the launch shapes of the timed runs; with the relative drift of the global
    mass sum (dycores)."""
    res = {}
    for name in names:
        s = make_state(mpdc, g, w, st, getattr(mpdc, "POLICY_" + name), shapes.get(name.lower()))
        if w["model"] != "TRACER":
            m0 = s.diagnostics(key_field(mpdc, w), stream=stream, check=False)["mass"]
        with torch.cuda.stream(stream):
            step(s, w, w["steps"], stream)
            torch.cuda.synchronize()
        if w["model"] != "TRACER":
            m1 = s.diagnostics(key_field(mpdc, w), stream=stream, check=False)["mass"]
            res[name + "_mass_drift"] = abs(m1 - m0) / abs(m0)
        res[name] = s.state_read(key_field(mpdc, w), stream=stream)
        d = s.diagnostics(key_field(mpdc, w), stream=stream, check=False)
        res[name + "_nonfinite"] = d["nonfinite"]
    return res


def oracle_baseline(mesh, w, st, nsteps, min_seconds=10.0, max_seconds=30.0):
    """The oracle on the host: nsteps from the workload's input (their result
    is the accuracy reference), then further chunks of nsteps from where it
    left off until about min_seconds of work; returns (reference, seconds,
    steps, threads)."""
    from oracle import OracleMesh, oracle_lib
    om = OracleMesh(mesh)
    vf = st.get("vflux")
    if w["model"] == "SW":
        state = (st["h"], st["u"])
        run = lambda s, n: om.sw_run(s[0], s[1], st["b"], w["dt"], n)
        key_of = lambda s: s[0]
    elif w["model"] == "HDC":
        ps0, Th0, u0 = st["ps"], st["Theta"], st["u"]
        if w["M"] > 1:
            ps0, Th0, u0 = ps0[:, 0], Th0[:, :, 0], u0[:, :, 0]
        state = (ps0, Th0, u0)
        run = lambda s, n: om.hdc_run(s[0], s[1], s[2], w["dt"], n)
        key_of = lambda s: s[0]
    elif w["model"] == "NDC":
        state = (st["ps"], st["Theta"], st["u"], st["w"], st["phi"])
        run = lambda s, n: om.ndc_run(*s, w["dt"], n)
        key_of = lambda s: s[0]
    else:
        state = (st["dpi"], st["q"])
        run = lambda s, n: om.tracer_run(st["F"], s[0], s[1], w["dt"], n, vflux=vf)
        key_of = lambda s: s[1]
    t0 = time.perf_counter()
    state = run(state, nsteps)
    key = key_of(state)
    steps = nsteps
    while time.perf_counter() - t0 < min_seconds:
        t1 = time.perf_counter()
        state = run(state, nsteps)
        steps += nsteps
        if time.perf_counter() - t0 + (time.perf_counter() - t1) > max_seconds:
            break
    el = time.perf_counter() - t0
    return key, el, steps, oracle_lib().or_num_threads()


def rel_l2(x, r):
    x, r = np.asarray(x, np.float64).ravel(), np.asarray(r, np.float64).ravel()
    return float(np.sqrt(((x - r) ** 2).sum() / (r ** 2).sum()))


def recorded_traffic(workload, kernel, shape, digest):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary of
    this workload, if it was taken from these sources in this launch shape."""
    from paper_2404_08849_amd.profsum import read_record
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload.replace("-", "_")))
    rec = read_record(path)
    if not rec:
        return None, "no counter summary for this kernel and workload"
    if rec.get("source_sha256") != digest:
        return None, "counters were taken from other library sources"
    if rec.get("kernel") != kernel or int(rec["values_per_lane"]) != int(shape[0]):
        return None, "counters were taken from another instance (values per lane %s)" % rec.get("values_per_lane")
    # the work-group size changes only which neighbour rows are still cached
    note = "" if int(rec["group"]) == int(shape[1]) else " (counters taken at work-group %s)" % rec["group"]
    return float(rec["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT) + note


def stream_ceilings(torch, mpdc, stream, mib=2048, reps=10):
    """Bandwidth of the library's hand-written streaming kernels (16-byte
    accesses, one pass over mib MiB) on the launch stream: GB/s of bytes read
    (read), written (write) and read + written (copy)."""
    n = mib * (1 << 20)
    with torch.cuda.stream(stream):
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        out = {}
        for name, mode, moved in (("read", mpdc.STREAM_READ, n), ("write", mpdc.STREAM_WRITE, n),
                                  ("copy", mpdc.STREAM_COPY, 2 * n)):
            ms = mpdc.stream_time(mode, b, a, reps, stream=stream)
            out[name] = moved / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def copy_calibration(torch, mib):
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 3}), flush=True)


def coupled_states(torch, mpdc, g, mesh, w, pol, stream, autotune, shapes=None):
    """Dycore (accumulating its mass fluxes) and tracer states of the coupled
    workload; one coupling round is run so the tracer has its fluxes.
    shapes, if given ({"dycore": [[values per lane, group], ...], "tracer":
    [...]}), fixes the launch shapes instead of autotuning them."""
    from paper_2404_08849_amd.inputs import initial as ic
    K, T, n = w["K"], w["T"], w["nsub"]
    s = ic.hdc_jet(mesh, K, seed=2000)
    tr = ic.tracer_solid_body(mesh, K, T, seed=3000)
    dsig = np.diff(ic.sigma_interfaces(K))
    dpi0 = dsig[None, :] * (s["ps"][:, None] - 1000.0)
    dy = mpdc.State(g, mpdc.MODEL_HDC, pol, K=K, dt=w["dt"], sigma=ic.sigma_interfaces(K), accumulate_flux=True)
    dy.state_write(mpdc.FIELD_PS, s["ps"][:, None])
    dy.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
    dy.state_write(mpdc.FIELD_U, s["u"][:, :, None])
    trs = mpdc.State(g, mpdc.MODEL_TRACER, pol, K=K, T=T, dt=n * w["dt"])
    trs.state_write(mpdc.FIELD_TR_DPI, dpi0)
    trs.state_write(mpdc.FIELD_TR_Q, tr["q"])
    if shapes:
        for k, (v, grp) in enumerate(shapes["dycore"]):
            dy.set_kernel_launch(k, v, grp)
        for k, (v, grp) in enumerate(shapes["tracer"]):
            trs.set_kernel_launch(k, v, grp)
    with torch.cuda.stream(stream):
        if autotune and not shapes:
            dy.autotune(stream=stream)
        dy.dycore_step(n, stream=stream)
        trs.couple(dy, stream=stream)
        if autotune and not shapes:
            trs.autotune(stream=stream)
        trs.tracer_step(1, stream=stream)
        torch.cuda.synchronize()
    dy.set_graph(True)
    trs.set_graph(True)
    return dy, trs, s, tr, dpi0


def coupled_step(dy, trs, n, stream):
    dy.dycore_step(n, stream=stream)
    trs.couple(dy, stream=stream)
    trs.tracer_step(1, stream=stream)


def coupled_main(args, torch, mpdc):
    """Coupled dycore + tracer workload: one 'step' is n dycore steps, the
    hand-over of their averaged mass fluxes and one tracer step of n dt."""
    w = WORKLOADS[args.workload]
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    mesh = icosahedral_mesh(w["level"])
    g = mpdc.Mesh(mesh)
    stream = torch.cuda.Stream()
    N, K, T, n = mesh["nCells"], w["K"], w["T"], w["nsub"]
    res = {}
    fixed = json.loads(args.shapes) if args.shapes else {}
    ceil = stream_ceilings(torch, mpdc, stream)
    copy_gbs = ceil["copy"]
    for name in ("MIX", "DBL"):
        pol = getattr(mpdc, "POLICY_" + name)
        dy, trs, s, tr, dpi0 = coupled_states(torch, mpdc, g, mesh, w, pol, stream, not args.no_autotune,
                                              fixed.get(name.lower()))
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                coupled_step(dy, trs, n, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                coupled_step(dy, trs, n, stream)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / max(args.steps, 1)
            # one coupled step under events: n dycore steps, the hand-over, one tracer step
            kd = kernel_times(torch, dy, dict(model="HDC"), n, stream)
            trs.couple(dy, stream=stream)
            kt = kernel_times(torch, trs, dict(model="TRACER"), 1, stream)
            torch.cuda.synchronize()
        bytes_step = n * dy.step_bytes() + trs.step_bytes()
        shapes = {"dycore": [list(dy.get_kernel_launch(k)) for k in range(4)],
                  "tracer": [list(trs.get_kernel_launch(k)) for k in range(3)]}
        del dy, trs
        # accuracy: the workload's coupled steps from the initial state
        dy, trs, s, tr, dpi0 = coupled_states(torch, mpdc, g, mesh, w, pol, stream, False)
        with torch.cuda.stream(stream):
            for _ in range(w["steps"] - 1):
                coupled_step(dy, trs, n, stream)
            torch.cuda.synchronize()
        ps = dy.state_read(mpdc.FIELD_PS)[:, 0]
        dpi_dyn = np.diff(np.arange(K + 1) / K)[None, :] * (ps[:, None] - 1000.0)
        dpi = trs.state_read(mpdc.FIELD_TR_DPI)
        res[name] = dict(sec=sec, kernels={**kd, **kt}, bytes_step=bytes_step, shapes=shapes, ps=ps,
                         q=trs.state_read(mpdc.FIELD_TR_Q),
                         mass_consistency=float(np.abs(dpi - dpi_dyn).max() / np.abs(dpi_dyn).max()),
                         nonfinite=int(dy.diagnostics(mpdc.FIELD_PS, stream=stream, check=False)["nonfinite"] +
                                       trs.diagnostics(mpdc.FIELD_TR_Q, stream=stream, check=False)["nonfinite"]))
        del dy, trs
    mix, dbl = res["MIX"], res["DBL"]
    kt = mix["kernels"]
    dom = max(kt, key=lambda k: kt[k]["ms_in_step"] * kt[k]["launches"])
    ach = kt[dom]["bytes"] / (kt[dom]["ms"] * 1e-3) / 1e9
    from paper_2404_08849_amd.profsum import source_digest
    digest = source_digest()
    family = "tracer" if dom in KERNEL_NAMES["tracer"] else "dycore"
    di = KERNEL_NAMES[family].index(dom)
    fam_shapes = mix["shapes"][family]
    shape = fam_shapes[di] if di < len(fam_shapes) else [0, 0]   # (the vertical step has one shape)
    traffic, traffic_src = recorded_traffic(args.workload, dom, shape, digest)
    gate = {"mix_vs_dbl_l2_ps": rel_l2(mix["ps"], dbl["ps"]), "mix_vs_dbl_l2_q": rel_l2(mix["q"], dbl["q"]),
            "tracer_vs_dycore_layer_mass": {"mix": mix["mass_consistency"], "dbl": dbl["mass_consistency"]},
            "nonfinite": mix["nonfinite"] + dbl["nonfinite"]}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import OracleMesh, oracle_lib
        from paper_2404_08849_amd.inputs import initial as ic
        om = OracleMesh(mesh)
        s = ic.hdc_jet(mesh, K, seed=2000)
        tr = ic.tracer_solid_body(mesh, K, T, seed=3000)
        dpi0 = np.diff(ic.sigma_interfaces(K))[None, :] * (s["ps"][:, None] - 1000.0)
        t0 = time.perf_counter()
        ps_, Th_, u_, q_, dpi_ = s["ps"], s["Theta"], s["u"], tr["q"], dpi0
        ncs = 0
        while ncs == 0 or time.perf_counter() - t0 < 10.0:
            ps_, Th_, u_, Fs, Ms = om.hdc_run_flux(ps_, Th_, u_, w["dt"], n)
            dpi_, q_ = om.tracer_run(Fs / n, dpi_, q_, n * w["dt"], 1, vflux=Ms / n)
            ncs += 1
        el = time.perf_counter() - t0
        cpu = {"value": N * K * n * ncs / el, "unit": "cell-level-steps/s", "cores": oracle_lib().or_num_threads(),
               "kind": "oracle", "sample": "%d coupled steps (each %d dycore steps + one tracer step of %d "
                                           "tracers) on the host (%.1f s)" % (ncs, n, T, el)}
    out = {
        "metric": "cell-level-steps/s (mixed vs all-FP64) at fixed L2 error; HBM GB/s",
        "value": N * K * n / mix["sec"],
        "unit": "cell-level-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mix["sec"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed f32/f64", "data": "synthetic",
        "config": {"workload": w["desc"], "mesh": "G%d" % w["level"], "cells": N, "levels": K, "members": 1,
                   "tracers": T, "dycore_steps_per_step": n, "policy": "MIX", "global_batch": 1, "seq_len": K,
                   "parallelism": "single GPU"},
        "dbl_value": N * K * n / dbl["sec"], "dbl_ms_per_step": dbl["sec"] * 1e3,
        "mix_over_dbl_speedup": dbl["sec"] / mix["sec"],
        "tracer_cell_level_steps_per_s": N * K * T / mix["sec"],
        "hbm_gbs_step": {"mix": mix["bytes_step"] / mix["sec"] / 1e9, "dbl": dbl["bytes_step"] / dbl["sec"] / 1e9},
        "accuracy_gate": gate,
        "kernels_mix": {k: {"ms": v["ms"], "ms_in_step": v["ms_in_step"], "MB": v["bytes"] / 1e6,
                            "GB/s": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in kt.items()},
        "kernels_dbl": {k: {"ms": v["ms"], "ms_in_step": v["ms_in_step"], "MB": v["bytes"] / 1e6,
                            "GB/s": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in dbl["kernels"].items()},
        "launch_shapes": {"mix": mix["shapes"], "dbl": dbl["shapes"]},
        "roofline": roofline_record(kt, dom, ach, traffic, traffic_src, ceil),
        "cpu_baseline": cpu,
        "source_sha256": digest,
    }
    print(json.dumps(out), flush=True)


def roofline_record(kt, dom, ach, traffic, traffic_src, ceil):
    """The dominant kernel's roofline: achieved GB/s (algorithmic bytes of one
    launch / its HIP-event duration) against the 8 TB/s HBM peak, or labelled
    "cache" when that launch's bytes fit the 256 MB MALL; also against the
    library's streaming kernels measured in the same run."""
    bound = "hbm" if kt[dom]["bytes"] > MALL_BYTES else "cache"
    return {"bound": bound, "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
            "bytes_per_launch": kt[dom]["bytes"], "bytes_per_launch_mean": kt[dom]["bytes_mean"],
            "ms_per_launch": kt[dom]["ms"], "ms_per_launch_in_step": kt[dom]["ms_in_step"],
            "timing": "HIP events around back-to-back launches on the launch stream",
            "stream_ceiling_gbs": ceil, "copy_ceiling_gbs": ceil["copy"], "frac_of_copy": ach / ceil["copy"],
            "frac_of_read": ach / ceil["read"],
            "ceiling_source": "the library's streaming kernels (mpdc_stream_time), 2 GiB, 16-byte accesses"}


def stored_reference_gate(torch, mpdc, g, w, st, stream, shapes, case):
    """Both policies for the 10 steps of the stored FP64 oracle results
    (tests/golden, written by make_fullsize_refs.py from the oracle), in the
    timed launch shapes, compared on the stored sample of cells and edges:
    relative max error of the key field (surface pressure, or the tracers)."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize_%s.npz" % case)
    if not os.path.exists(path):
        return None
    ref = dict(np.load(path))
    cells = ref["cells"]
    wl = dict(w, steps=int(ref["nsteps"]))
    out = {"steps": int(ref["nsteps"]), "sample": "%d cells (incl. the 12 pentagons), every level" % len(cells)}
    for name in ("DBL", "MIX"):
        s = make_state(mpdc, g, wl, st, getattr(mpdc, "POLICY_" + name), shapes.get(name.lower()))
        s.set_graph(True)
        with torch.cuda.stream(stream):
            step(s, wl, wl["steps"], stream)
            torch.cuda.synchronize()
        x = s.state_read(key_field(mpdc, w), stream=stream)
        del s
        if w["model"] == "TRACER":
            r = ref["q"]
            x = x[cells]
        elif "members" in ref:
            errs = []
            for j in ref["members"]:
                r = ref["ps_%d" % j]
                errs.append(float(np.abs(x[cells, j] - r).max() / np.abs(r).max()))
            out[name.lower() + "_vs_oracle_linf_ps"] = max(errs)
            continue
        else:
            r = ref["ps"]
            x = x[cells, 0] if x.ndim == 2 else x[cells]
        out[name.lower() + "_vs_oracle_linf_" + ("q" if w["model"] == "TRACER" else "ps")] = \
            float(np.abs(x - r).max() / np.abs(r).max())
    return out


def timed_repeats(torch, s, w, steps, repeats, stream):
    """ms per step of `repeats` further timed runs of `steps` steps each
    (graph replay, continuing the state), and their median."""
    res = []
    with torch.cuda.stream(stream):
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(s, w, steps, stream)
            torch.cuda.synchronize()
            res.append((time.perf_counter() - t0) / max(steps, 1) * 1e3)
    return {"ms_per_step": res, "median_ms_per_step": float(np.median(res)) if res else None}


def secondary_g6(torch, mpdc, stream, args, ceil):
    """The G6 x 30 hydrostatic workload, whose state fits the 256 MB MALL:
    MIX and DBL rates and the dominant kernel's bandwidth, labelled cache."""
    w = WORKLOADS["hdc-g6"]
    mesh, st = build_inputs(w)
    g = mpdc.Mesh(mesh)
    units = mesh["nCells"] * w["K"]
    s_mix, sec_mix = timed_run(torch, mpdc, g, w, st, mpdc.POLICY_MIX, args.steps, args.warmup, stream,
                               not args.no_autotune)
    kt = kernel_times(torch, s_mix, w, args.profile_steps, stream)
    del s_mix
    s_dbl, sec_dbl = timed_run(torch, mpdc, g, w, st, mpdc.POLICY_DBL, args.steps, args.warmup, stream,
                               not args.no_autotune)
    del s_dbl
    dom = max(kt, key=lambda k: kt[k]["ms_in_step"] * kt[k]["launches"])
    ach = kt[dom]["bytes"] / (kt[dom]["ms"] * 1e-3) / 1e9
    rl = roofline_record(kt, dom, ach, None, "not taken for the secondary line", ceil)
    return {"workload": w["desc"], "value": units / sec_mix, "ms_per_step": sec_mix * 1e3,
            "dbl_value": units / sec_dbl, "mix_over_dbl_speedup": sec_dbl / sec_mix,
            "roofline": rl}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(ensemble members and subdomains would be sharded one per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2404_08849_amd.mpdc as mpdc
    if args.copy_calib:
        copy_calibration(torch, args.copy_calib)
        return
    w = WORKLOADS[args.workload]
    if w["model"] == "COUPLED":
        coupled_main(args, torch, mpdc)
        return
    mesh, st = build_inputs(w)
    g = mpdc.Mesh(mesh)
    stream = torch.cuda.Stream()
    N, K, M, T = mesh["nCells"], w["K"], w["M"], w["T"]
    units = N * K * M

    fixed = json.loads(args.shapes) if args.shapes else {}
    ceil = stream_ceilings(torch, mpdc, stream)
    s_mix, sec_mix = timed_run(torch, mpdc, g, w, st, mpdc.POLICY_MIX, args.steps, args.warmup, stream,
                               not args.no_autotune, fixed.get("mix"))
    shapes_mix = s_mix.launch_shapes
    reps = timed_repeats(torch, s_mix, w, args.steps, args.repeats, stream)
    kt = kernel_times(torch, s_mix, w, args.profile_steps, stream)
    step_bytes_mix = s_mix.step_bytes()
    sec_dbl, kt_dbl, step_bytes_dbl, shapes_dbl = None, None, None, None
    if not args.no_dbl:
        s_dbl, sec_dbl = timed_run(torch, mpdc, g, w, st, mpdc.POLICY_DBL, args.steps, args.warmup, stream,
                                   not args.no_autotune, fixed.get("dbl"))
        shapes_dbl = s_dbl.launch_shapes
        kt_dbl = kernel_times(torch, s_dbl, w, args.profile_steps, stream)
        step_bytes_dbl = s_dbl.step_bytes()
        del s_dbl
    # dominant kernel of the mixed step: the largest share of the step time
    dom = max(kt, key=lambda k: kt[k]["ms_in_step"] * kt[k]["launches"])
    ach = kt[dom]["bytes"] / (kt[dom]["ms"] * 1e-3) / 1e9
    acc = accuracy_run(torch, mpdc, g, w, st, stream, {"mix": shapes_mix, "dbl": shapes_dbl})
    from paper_2404_08849_amd.profsum import source_digest
    digest = source_digest()
    names = KERNEL_NAMES["tracer" if w["model"] == "TRACER" else "dycore"]
    di = names.index(dom)
    shape = shapes_mix[di] if di < len(shapes_mix) else [0, 0]   # (the vertical step has one shape)
    traffic, traffic_src = recorded_traffic(args.workload, dom, shape, digest)
    gate = {"mix_vs_dbl_l2": rel_l2(acc["MIX"], acc["DBL"]), "nonfinite": acc["MIX_nonfinite"] + acc["DBL_nonfinite"]}
    if "MIX_mass_drift" in acc:
        gate["mass_drift"] = {"mix": acc["MIX_mass_drift"], "dbl": acc["DBL_mass_drift"]}
    if args.workload in STORED_REFS:
        gate["stored_oracle_10_steps"] = stored_reference_gate(torch, mpdc, g, w, st, stream,
                                                               {"mix": shapes_mix, "dbl": shapes_dbl},
                                                               STORED_REFS[args.workload])

    # mixed-policy variants beside MIX (layered dycores only)
    variants, var_keys = None, {}
    if w["model"] in ("HDC", "NDC", "TRACER") and not args.no_variants:
        variants = {}
        # (the all-FP32 tracer policy has no vertical step)
        names = ((() if w.get("vflux") else ("SGL",)) if w["model"] == "TRACER" else
                 ("MIX_BOX", "MIX_DBL_MASS", "MIX_F32_DIV", "MIX_PGF32", "SGL"))
        for name in names:
            s_v, sec_v = timed_run(torch, mpdc, g, w, st, getattr(mpdc, "POLICY_" + name), args.steps, args.warmup,
                                   stream, not args.no_autotune, fixed.get(name.lower()))
            shp = s_v.launch_shapes
            del s_v
            av = accuracy_run(torch, mpdc, g, w, st, stream, {name.lower(): shp}, names=(name,))
            var_keys[name] = av[name]
            variants[name] = {"value": units / sec_v, "ms_per_step": sec_v * 1e3, "speed_vs_mix": sec_mix / sec_v,
                              "vs_dbl_l2": rel_l2(av[name], acc["DBL"]), "mass_drift": av.get(name + "_mass_drift"),
                              "nonfinite": av[name + "_nonfinite"], "launch_shapes": shp}

    del s_mix
    secondary = None
    if not args.no_secondary and args.workload != "hdc-g6":
        secondary = {"hdc-g6": secondary_g6(torch, mpdc, stream, args, ceil)}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle_lib
        nst = w["steps"] if w["level"] <= 6 else 1
        cores = oracle_lib().or_num_threads()
        key, el, nrun, cores = oracle_baseline(mesh, w, st, nst)
        ref = np.asarray(key)
        gpu_dbl = acc["DBL"] if nst == w["steps"] else None
        if gpu_dbl is not None:
            if w["model"] == "HDC" and M > 1:
                gpu_dbl, gpu_mix = acc["DBL"][:, 0], acc["MIX"][:, 0]
            else:
                gpu_dbl, gpu_mix = acc["DBL"].reshape(ref.shape), acc["MIX"].reshape(ref.shape)
            gate["dbl_vs_oracle_l2"] = rel_l2(gpu_dbl, ref)
            gate["mix_vs_oracle_l2"] = rel_l2(gpu_mix, ref)
            for name, x in var_keys.items():
                xv = x[:, 0] if (w["model"] == "HDC" and M > 1) else x.reshape(ref.shape)
                variants[name]["vs_oracle_l2"] = rel_l2(xv, ref)
        per_member = N * K * (T if w["model"] == "TRACER" else 1)
        # the same oracle on one thread: one step (or the workload's steps on small meshes)
        oracle_lib().or_set_num_threads(1)
        try:
            _, el1, nrun1, _ = oracle_baseline(mesh, w, st, 1 if w["level"] > 5 else nst,
                                               min_seconds=0.0, max_seconds=0.0)
        finally:
            oracle_lib().or_set_num_threads(cores)
        cpu = {"value": per_member * nrun / el, "unit": "cell-level-steps/s" if w["model"] != "TRACER"
               else "cell-level-tracer-steps/s", "cores": cores, "kind": "oracle",
               "sample": "%d step(s) of one member of %s on the host (%.1f s); the first %d are the "
                         "accuracy reference" % (nrun, args.workload, el, nst),
               "value_1_thread": per_member * nrun1 / el1,
               "sample_1_thread": "%d step(s) of one member of %s on one host thread (%.1f s)"
                                  % (nrun1, args.workload, el1)}
    gate["passes"] = bool(gate.get("mix_vs_oracle_l2", gate["mix_vs_dbl_l2"]) <= 1e-5 and gate["nonfinite"] == 0)
    so = gate.get("stored_oracle_10_steps")
    if so:
        key = [k for k in so if k.startswith("mix_vs_oracle")][0]
        gate["passes"] = bool(gate["passes"] and so[key] <= 1e-5)

    value = units / sec_mix
    unit = "cell-level-steps/s"
    out = {
        "metric": "cell-level-steps/s (mixed vs all-FP64) at fixed L2 error; HBM GB/s",
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_mix * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed f32/f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "mesh": "G%d" % w["level"], "cells": N, "levels": K,
                   "members": M, "tracers": T, "policy": "MIX", "global_batch": M, "seq_len": K,
                   "parallelism": "single GPU"},
        "dbl_value": (units / sec_dbl) if sec_dbl else None,
        "dbl_ms_per_step": sec_dbl * 1e3 if sec_dbl else None,
        "mix_over_dbl_speedup": (sec_dbl / sec_mix) if sec_dbl else None,
        "hbm_gbs_step": {"mix": step_bytes_mix / sec_mix / 1e9,
                         "dbl": step_bytes_dbl / sec_dbl / 1e9 if sec_dbl else None},
        "accuracy_gate": gate,
        "variants": variants,
        "kernels_mix": {k: {"ms": v["ms"], "ms_in_step": v["ms_in_step"], "MB": v["bytes"] / 1e6,
                            "GB/s": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in kt.items()},
        "kernels_dbl": ({k: {"ms": v["ms"], "ms_in_step": v["ms_in_step"], "MB": v["bytes"] / 1e6,
                             "GB/s": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in kt_dbl.items()}
                        if kt_dbl else None),
        "launch_shapes": {"mix": shapes_mix, "dbl": shapes_dbl,
                          "note": "(values per lane, cells or threads per work-group) per kernel, autotuned"},
        "repeats": reps,
        "roofline": roofline_record(kt, dom, ach, traffic, traffic_src, ceil),
        "secondary": secondary,
        "cpu_baseline": cpu,
        "source_sha256": digest,
    }
    if w["model"] == "TRACER":
        out["tracer_cell_level_steps_per_s"] = value * T
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
