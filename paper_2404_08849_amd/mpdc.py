"""Thin ctypes binding of the mpdc C ABI (include/mpdc.h).

Argument marshalling only: every step of the dycore, tracer and diagnostics
runs in the library's HIP kernels.  PyTorch provides the device workspaces
(uint8 tensors) and the stream.  Importing this module loads the in-tree
``libmpdc.so``; if it is missing the import fails loudly -- there is no
CPU fallback.
"""
import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime that libmpdc.so binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpdc.so")

MPDC_OK = 0
ERRORS = {-1: "INVAL", -2: "MESH", -3: "NOMEM", -4: "DEVICE", -5: "NUMERIC", -6: "UNSUPPORTED", -7: "STATE"}

MODEL_SW, MODEL_HDC, MODEL_NDC, MODEL_TRACER = 0, 1, 2, 3
POLICY_DBL, POLICY_MIX, POLICY_MIX_BOX, POLICY_MIX_DBL_MASS, POLICY_MIX_F32_DIV, POLICY_MIX_PGF32, POLICY_SGL = \
    0, 1, 2, 3, 4, 5, 6
POLICY_TERMS = 7
# per-term precision bits of POLICY_TERMS (mpdc.h MPDC_TERM_*)
TERMS = ["mass flux", "divergence", "kinetic energy", "vorticity", "vertex mass", "Coriolis", "theta flux",
         "vertical advection", "column diagnostics", "pressure gradient"]
TERM_BIT = {name: i for i, name in enumerate(TERMS)}
TERMS_MIX = sum(1 << TERM_BIT[t] for t in ("mass flux", "kinetic energy", "vorticity", "Coriolis", "theta flux",
                                            "vertical advection"))
FIELD_H, FIELD_PS, FIELD_THETA, FIELD_U, FIELD_W, FIELD_PHI, FIELD_B = 0, 1, 2, 3, 4, 5, 6
FIELD_TR_FLUX, FIELD_TR_DPI, FIELD_TR_Q, FIELD_TR_VFLUX, FIELD_PHIS, FIELD_VORT = 7, 8, 9, 10, 11, 12
TABLE_CELLS_ON_CELL, TABLE_EDGE_SIGN, TABLE_VERTEX_SIGN = 0, 1, 2
TABLE_TRISK_OFFSET, TABLE_TRISK_EDGE, TABLE_TRISK_WEIGHT, TABLE_HESSIAN = 3, 4, 5, 6

_ip = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class MpdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mpdc error %d (%s): %s" % (code, ERRORS.get(code, "?"), msg))
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("nCells", ctypes.c_int32), ("nEdges", ctypes.c_int32), ("nVertices", ctypes.c_int32),
                ("cells_on_edge", _ip), ("vertices_on_edge", _ip), ("eoc_offset", _ip),
                ("edges_on_cell", _ip), ("vertices_on_cell", _ip), ("cells_on_vertex", _ip),
                ("edges_on_vertex", _ip), ("xCell", _dp), ("xVertex", _dp), ("xEdge", _dp),
                ("dEdge", _dp), ("lEdge", _dp), ("areaCell", _dp), ("areaVertex", _dp),
                ("kiteArea", _dp), ("fVertex", _dp), ("radius", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("policy", ctypes.c_int32), ("K", ctypes.c_int32),
                ("M", ctypes.c_int32), ("T", ctypes.c_int32), ("fct", ctypes.c_int32),
                ("dt", ctypes.c_double), ("grav", ctypes.c_double), ("rd", ctypes.c_double),
                ("cp", ctypes.c_double), ("p0", ctypes.c_double), ("ptop", ctypes.c_double),
                ("sigma", _dp), ("accumulate_flux", ctypes.c_int32), ("forward_backward_off", ctypes.c_int32),
                ("term_fp32", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("mass_tracer", ctypes.c_double * 16), ("min", ctypes.c_double),
                ("max", ctypes.c_double), ("l1", ctypes.c_double), ("l2", ctypes.c_double),
                ("linf", ctypes.c_double), ("nonfinite", ctypes.c_int64), ("cfl_max", ctypes.c_double),
                ("energy", ctypes.c_double), ("tracer_min", ctypes.c_double * 16),
                ("tracer_max", ctypes.c_double * 16)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmpdc.so is not built (run paper_2404_08849_amd.build.build()); "
                          "there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "mpdc_mesh_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(MeshDesc)]),
        "mpdc_mesh_check": (ctypes.c_int, [ctypes.POINTER(MeshDesc)]),
        "mpdc_mesh_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
        "mpdc_mesh_get_table": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_size_t]),
        "mpdc_mesh_table_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int]),
        "mpdc_mesh_destroy": (None, [_vp]),
        "mpdc_state_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.POINTER(Config)]),
        "mpdc_state_create": (ctypes.c_int, [_vp, ctypes.POINTER(Config), _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
        "mpdc_state_write": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_size_t, _vp]),
        "mpdc_state_read": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_size_t, _vp]),
        "mpdc_dycore_step": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
        "mpdc_tracer_step": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
        "mpdc_tracer_couple": (ctypes.c_int, [_vp, _vp, _vp]),
        "mpdc_diagnostics": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(Diag), _vp]),
        "mpdc_set_graph": (ctypes.c_int, [_vp, ctypes.c_int]),
        "mpdc_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
        "mpdc_set_kernel_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "mpdc_get_kernel_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_int)]),
        "mpdc_time_kernel": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double)]),
        "mpdc_kernel_bytes": (ctypes.c_double, [_vp, ctypes.c_int]),
        "mpdc_stage_kernel_bytes": (ctypes.c_double, [_vp, ctypes.c_int, ctypes.c_int]),
        "mpdc_profile_steps": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int)]),
        "mpdc_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p, _vp]),
        "mpdc_step_bytes": (ctypes.c_double, [_vp]),
        "mpdc_error_norms_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_size_t, ctypes.c_size_t,
                                                    ctypes.POINTER(ctypes.c_double), _vp]),
        "mpdc_stream_time": (ctypes.c_int, [ctypes.c_int, _vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp,
                                            ctypes.POINTER(ctypes.c_double)]),
        "mpdc_state_destroy": (None, [_vp]),
        "mpdc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "mpdc_last_error": (ctypes.c_char_p, []),
        "mpdc_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(rc):
    if rc != MPDC_OK:
        raise MpdcError(rc, lib.mpdc_last_error().decode())
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def error_norms_noalloc(x, ref, weight=None, stream=None):
    """mpdc_error_norms_noalloc over the FP64 device tensors x and ref ([n][...])
    and optional weights [n]: (l1, l2, linf, min, max)."""
    out = (ctypes.c_double * 5)()
    n = x.shape[0]
    inner = x.numel() // n if n else 0
    _check(lib.mpdc_error_norms_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
                                        ctypes.c_void_p(weight.data_ptr() if weight is not None else 0), n, inner,
                                        out, _stream(stream)))
    return tuple(out)


STREAM_READ, STREAM_WRITE, STREAM_COPY = 0, 1, 2


def stream_time(mode, dst, src=None, nreps=10, stream=None):
    """mpdc_stream_time: mean duration (ms) of the library's streaming kernel
    (STREAM_READ, STREAM_WRITE or STREAM_COPY) over dst.nbytes bytes of the
    device tensors dst and src."""
    ms = ctypes.c_double()
    _check(lib.mpdc_stream_time(mode, ctypes.c_void_p(dst.data_ptr()),
                                ctypes.c_void_p(src.data_ptr() if src is not None else 0),
                                dst.numel() * dst.element_size(), nreps, _stream(stream), ctypes.byref(ms)))
    return ms.value


class Mesh:
    """mpdc_mesh_create over a mesh dict (connectivity + FP64 geometry)."""

    def __init__(self, mesh, device="cuda", stream=None):
        self._keep = {k: _i32(mesh[k]) for k in ["cells_on_edge", "vertices_on_edge", "eoc_offset", "edges_on_cell",
                                                  "vertices_on_cell", "cells_on_vertex", "edges_on_vertex"]}
        self._keep.update({k: _f64(mesh[k]) for k in ["xCell", "xVertex", "xEdge", "dEdge", "lEdge", "areaCell",
                                                       "areaVertex", "kiteArea", "fVertex"]})
        k = self._keep
        self.N, self.E, self.V = int(mesh["nCells"]), int(mesh["nEdges"]), int(mesh["nVertices"])
        ip = lambda a: a.ctypes.data_as(_ip)
        dp = lambda a: a.ctypes.data_as(_dp)
        self.desc = MeshDesc(self.N, self.E, self.V, ip(k["cells_on_edge"]), ip(k["vertices_on_edge"]),
                             ip(k["eoc_offset"]), ip(k["edges_on_cell"]), ip(k["vertices_on_cell"]),
                             ip(k["cells_on_vertex"]), ip(k["edges_on_vertex"]), dp(k["xCell"]), dp(k["xVertex"]),
                             dp(k["xEdge"]), dp(k["dEdge"]), dp(k["lEdge"]), dp(k["areaCell"]), dp(k["areaVertex"]),
                             dp(k["kiteArea"]), dp(k["fVertex"]), float(mesh["radius"]))
        nbytes = lib.mpdc_mesh_workspace_bytes(ctypes.byref(self.desc))
        if nbytes == 0:
            raise MpdcError(-1, "unusable mesh descriptor")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = _vp()
        _check(lib.mpdc_mesh_create(ctypes.byref(self.desc), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                    _stream(stream), ctypes.byref(h)))
        self.h = h
        self.area = self._keep["areaCell"]
        self.mesh = mesh

    def table(self, table_id):
        n = lib.mpdc_mesh_table_bytes(self.h, table_id)
        dtype = np.int32 if table_id in (TABLE_CELLS_ON_CELL, TABLE_TRISK_OFFSET, TABLE_TRISK_EDGE) else np.float64
        out = np.empty(n // np.dtype(dtype).itemsize, dtype=dtype)
        _check(lib.mpdc_mesh_get_table(self.h, table_id, out.ctypes.data_as(_vp), n))
        return out

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.mpdc_mesh_destroy(self.h)
            self.h = None


class State:
    """mpdc_state_create and the per-state calls (dycore_step, tracer_step, diagnostics, ...)."""

    def __init__(self, mesh, model, policy, K=1, M=1, T=0, dt=1.0, sigma=None, fct=True,
                 grav=9.80616, rd=287.0, cp=1004.5, p0=1.0e5, ptop=1000.0, device="cuda", accumulate_flux=False,
                 forward_backward=True, term_fp32=0):
        self.mesh = mesh
        self.model, self.policy, self.K, self.M, self.T = model, policy, K, M, T
        self.sigma = _f64(np.arange(K + 1) / K if sigma is None else sigma)
        self.cfg = Config(model, policy, K, M, T, int(bool(fct)), dt, grav, rd, cp, p0, ptop,
                          self.sigma.ctypes.data_as(_dp), int(bool(accumulate_flux)), int(not forward_backward),
                          int(term_fp32))
        nbytes = lib.mpdc_state_workspace_bytes(mesh.h, ctypes.byref(self.cfg))
        if nbytes == 0:
            raise MpdcError(-6, lib.mpdc_last_error().decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = _vp()
        _check(lib.mpdc_state_create(mesh.h, ctypes.byref(self.cfg), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                     ctypes.byref(h)))
        self.h = h

    def field_shape(self, f):
        N, E, K, M, T = self.mesh.N, self.mesh.E, self.K, self.M, self.T
        shapes = {FIELD_H: (N, M), FIELD_PS: (N, M), FIELD_THETA: (N, K, M), FIELD_U: (E, K, M),
                  FIELD_W: (N, K + 1, M), FIELD_PHI: (N, K + 1, M), FIELD_B: (N,), FIELD_TR_FLUX: (E, K),
                  FIELD_TR_DPI: (N, K), FIELD_TR_Q: (N, K, T), FIELD_TR_VFLUX: (N, K + 1), FIELD_PHIS: (N,),
                  FIELD_VORT: (self.mesh.V, K, M)}
        return shapes[f]

    def state_write(self, f, data, stream=None):
        if isinstance(data, torch.Tensor):
            t = data.to(torch.float64).contiguous()
            _check(lib.mpdc_state_write(self.h, f, ctypes.c_void_p(t.data_ptr()), 1 if t.is_cuda else 0,
                                        t.numel() * 8, _stream(stream)))
            if t.is_cuda:
                torch.cuda.current_stream().synchronize()
            return
        a = _f64(data)
        _check(lib.mpdc_state_write(self.h, f, a.ctypes.data_as(_vp), 0, a.nbytes, _stream(stream)))

    def state_read(self, f, stream=None):
        out = np.empty(self.field_shape(f), dtype=np.float64)
        _check(lib.mpdc_state_read(self.h, f, out.ctypes.data_as(_vp), 0, out.nbytes, _stream(stream)))
        return out

    def state_read_device(self, f, stream=None):
        out = torch.empty(self.field_shape(f), dtype=torch.float64, device="cuda")
        _check(lib.mpdc_state_read(self.h, f, ctypes.c_void_p(out.data_ptr()), 1, out.numel() * 8, _stream(stream)))
        return out

    def dycore_step(self, nsteps=1, stream=None):
        _check(lib.mpdc_dycore_step(self.h, nsteps, _stream(stream)))

    def tracer_step(self, nsteps=1, stream=None):
        _check(lib.mpdc_tracer_step(self.h, nsteps, _stream(stream)))

    def couple(self, dycore, stream=None):
        """mpdc_tracer_couple: this tracer state takes the dycore state's averaged mass fluxes."""
        _check(lib.mpdc_tracer_couple(self.h, dycore.h, _stream(stream)))

    def diagnostics(self, f, ref=None, stream=None, check=True):
        d = Diag()
        refp = None
        if ref is not None:
            ref = ref.to(torch.float64).contiguous() if isinstance(ref, torch.Tensor) else \
                torch.from_numpy(_f64(ref)).cuda()
            refp = ctypes.c_void_p(ref.data_ptr())
        rc = lib.mpdc_diagnostics(self.h, refp, f, ctypes.byref(d), _stream(stream))
        if rc != MPDC_OK and (check or rc != -5):
            _check(rc)
        nt = max(self.T, 0)
        return dict(mass=d.mass, mass_tracer=list(d.mass_tracer)[:nt], min=d.min, max=d.max,
                    l1=d.l1, l2=d.l2, linf=d.linf, nonfinite=d.nonfinite, cfl_max=d.cfl_max, energy=d.energy,
                    tracer_min=list(d.tracer_min)[:nt], tracer_max=list(d.tracer_max)[:nt], rc=rc)

    def set_graph(self, enable):
        _check(lib.mpdc_set_graph(self.h, int(bool(enable))))

    def set_launch(self, cells_per_block=0, flat_block=0):
        _check(lib.mpdc_set_launch(self.h, cells_per_block, flat_block))

    def set_kernel_launch(self, kernel_id, values_per_lane=0, group=0):
        _check(lib.mpdc_set_kernel_launch(self.h, kernel_id, values_per_lane, group))

    def get_kernel_launch(self, kernel_id):
        v, g = ctypes.c_int(), ctypes.c_int()
        _check(lib.mpdc_get_kernel_launch(self.h, kernel_id, ctypes.byref(v), ctypes.byref(g)))
        return v.value, g.value

    def time_kernel(self, kernel_id, nreps=10, stream=None):
        ms = ctypes.c_double()
        _check(lib.mpdc_time_kernel(self.h, kernel_id, nreps, _stream(stream), ctypes.byref(ms)))
        return ms.value

    def profile_steps(self, nsteps, stream=None):
        """Advance nsteps with HIP events between launches; returns {kernel id: (total ms, launches)}."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int * 4)()
        _check(lib.mpdc_profile_steps(self.h, nsteps, _stream(stream), ms, n))
        return {k: (ms[k], n[k]) for k in range(4) if n[k] > 0}

    def autotune(self, stream=None, cache_path=None):
        """mpdc_autotune; returns the chosen (values per lane, group) per kernel class."""
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib.mpdc_autotune(self.h, path, _stream(stream)))
        return [self.get_kernel_launch(k) for k in range(3 if self.model == MODEL_TRACER else 4)]

    def kernel_bytes(self, kernel_id):
        return lib.mpdc_kernel_bytes(self.h, kernel_id)

    def stage_kernel_bytes(self, kernel_id, stage):
        return lib.mpdc_stage_kernel_bytes(self.h, kernel_id, stage)

    def step_bytes(self):
        return lib.mpdc_step_bytes(self.h)

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.mpdc_state_destroy(self.h)
            self.h = None


# names of the C ABI entry points
def mesh_create(mesh, **kw):
    return Mesh(mesh, **kw)


def state_create(mesh, model, policy, **kw):
    return State(mesh, model, policy, **kw)
