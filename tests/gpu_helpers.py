"""Shared helpers of the GPU tests: run a workload through the C ABI and
through the FP64 oracle on the same seeded inputs."""
import contextlib

import numpy as np

from paper_2404_08849_amd.inputs import initial as ic


def _stream_ctx(graph):
    """Graph capture needs a non-default stream; plain launches use torch's current one."""
    import torch
    if not graph:
        return contextlib.nullcontext()
    return torch.cuda.stream(torch.cuda.Stream())


def rel_l2(x, r, w=None):
    """Normalised (optionally weighted over the first axis) L2 difference."""
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    if w is None:
        return float(np.sqrt(((x - r) ** 2).sum() / max((r ** 2).sum(), 1e-300)))
    w = np.asarray(w).reshape((-1,) + (1,) * (x.ndim - 1))
    return float(np.sqrt((w * (x - r) ** 2).sum() / max((w * r ** 2).sum(), 1e-300)))


def _gpu_sw_impl(mpdc, gmesh, state, dt, nsteps, policy, graph=False, launch=None):
    st = mpdc.State(gmesh, mpdc.MODEL_SW, policy, K=1, M=1, dt=dt)
    if launch:
        st.set_launch(*launch)
    st.set_graph(graph)
    st.state_write(mpdc.FIELD_H, state["h"])
    st.state_write(mpdc.FIELD_U, state["u"])
    st.state_write(mpdc.FIELD_B, state["b"])
    st.dycore_step(nsteps)
    return st, st.state_read(mpdc.FIELD_H)[:, 0], st.state_read(mpdc.FIELD_U)[:, 0, 0]


def _gpu_hdc_impl(mpdc, gmesh, state, K, dt, nsteps, policy, M=1, graph=False, launch=None, autotune=False):
    st = mpdc.State(gmesh, mpdc.MODEL_HDC, policy, K=K, M=M, dt=dt, sigma=ic.sigma_interfaces(K))
    if launch:
        st.set_launch(*launch)
    st.set_graph(graph)
    ps, Th, u = state["ps"], state["Theta"], state["u"]
    if M == 1:
        ps, Th, u = ps[:, None], Th[:, :, None], u[:, :, None]
    st.state_write(mpdc.FIELD_PS, ps)
    st.state_write(mpdc.FIELD_THETA, Th)
    st.state_write(mpdc.FIELD_U, u)
    if autotune:
        st.autotune()
    st.dycore_step(nsteps)
    out = [st.state_read(f) for f in (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U)]
    if M == 1:
        out = [out[0][:, 0], out[1][:, :, 0], out[2][:, :, 0]]
    return st, out


def _gpu_ndc_impl(mpdc, gmesh, state, K, dt, nsteps, policy, graph=False, launch=None, autotune=False):
    st = mpdc.State(gmesh, mpdc.MODEL_NDC, policy, K=K, M=1, dt=dt, sigma=ic.sigma_interfaces(K))
    if launch:
        st.set_launch(*launch)
    st.set_graph(graph)
    st.state_write(mpdc.FIELD_PS, state["ps"][:, None])
    st.state_write(mpdc.FIELD_THETA, state["Theta"][:, :, None])
    st.state_write(mpdc.FIELD_U, state["u"][:, :, None])
    st.state_write(mpdc.FIELD_W, state["w"][:, :, None])
    st.state_write(mpdc.FIELD_PHI, state["phi"][:, :, None])
    if autotune:
        st.autotune()
    st.dycore_step(nsteps)
    fs = (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U, mpdc.FIELD_W, mpdc.FIELD_PHI)
    out = [st.state_read(f)[..., 0] for f in fs]
    return st, out


def _gpu_tracer_impl(mpdc, gmesh, tr, dt, nsteps, policy, fct=True, graph=False, launch=None, autotune=False):
    K, T = tr["q"].shape[1], tr["q"].shape[2]
    st = mpdc.State(gmesh, mpdc.MODEL_TRACER, policy, K=K, T=T, dt=dt, fct=fct)
    if launch:
        st.set_launch(*launch)
    st.set_graph(graph)
    st.state_write(mpdc.FIELD_TR_FLUX, tr["F"])
    st.state_write(mpdc.FIELD_TR_DPI, tr["dpi"])
    st.state_write(mpdc.FIELD_TR_Q, tr["q"])
    if autotune:
        st.autotune()
    st.tracer_step(nsteps)
    return st, st.state_read(mpdc.FIELD_TR_DPI), st.state_read(mpdc.FIELD_TR_Q)


def gpu_sw(mpdc, gmesh, state, dt, nsteps, policy, graph=False, launch=None):
    with _stream_ctx(graph):
        return _gpu_sw_impl(mpdc, gmesh, state, dt, nsteps, policy, graph, launch)


def gpu_hdc(mpdc, gmesh, state, K, dt, nsteps, policy, M=1, graph=False, launch=None, autotune=False):
    with _stream_ctx(graph):
        return _gpu_hdc_impl(mpdc, gmesh, state, K, dt, nsteps, policy, M, graph, launch, autotune)


def gpu_ndc(mpdc, gmesh, state, K, dt, nsteps, policy, graph=False, launch=None, autotune=False):
    with _stream_ctx(graph):
        return _gpu_ndc_impl(mpdc, gmesh, state, K, dt, nsteps, policy, graph, launch, autotune)


def gpu_tracer(mpdc, gmesh, tr, dt, nsteps, policy, fct=True, graph=False, launch=None, autotune=False):
    with _stream_ctx(graph):
        return _gpu_tracer_impl(mpdc, gmesh, tr, dt, nsteps, policy, fct, graph, launch, autotune)
