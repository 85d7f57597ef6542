"""ctypes wrapper of the FP64 C oracle (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build_oracle():
    """Compile oracle.c into liboracle.so (gcc, FP64, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
           "-o", _SO + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)


class MeshIn(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("E", ctypes.c_int), ("V", ctypes.c_int),
                ("cells_on_edge", _ip), ("vertices_on_edge", _ip), ("eoc_offset", _ip),
                ("edges_on_cell", _ip), ("vertices_on_cell", _ip), ("cells_on_vertex", _ip),
                ("edges_on_vertex", _ip), ("xCell", _dp), ("xVertex", _dp), ("xEdge", _dp),
                ("dEdge", _dp), ("lEdge", _dp), ("areaCell", _dp), ("areaVertex", _dp),
                ("kiteArea", _dp), ("fVertex", _dp), ("radius", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("T", ctypes.c_int), ("dt", ctypes.c_double),
                ("grav", ctypes.c_double), ("rd", ctypes.c_double), ("cp", ctypes.c_double),
                ("p0", ctypes.c_double), ("ptop", ctypes.c_double), ("sigma", _dp),
                ("fct", ctypes.c_int), ("phis", _dp), ("no_fb", ctypes.c_int)]


def oracle_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_oracle()
        lib = ctypes.CDLL(_SO)
        lib.or_mesh_build.restype = ctypes.c_void_p
        lib.or_mesh_build.argtypes = [ctypes.POINTER(MeshIn)]
        lib.or_mesh_free.argtypes = [ctypes.c_void_p]
        for name in ["or_gradient", "or_divergence", "or_curl", "or_kinetic_energy", "or_vertex_mass",
                     "or_perp_flux", "or_hessian_dir"]:
            getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
        lib.or_coriolis.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
        lib.or_edge_value3.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
        lib.or_edge_value3_formula.argtypes = [ctypes.c_int] + [_dp] * 7
        lib.or_thomas.argtypes = [ctypes.c_int] + [_dp] * 5
        lib.or_iface_advection.argtypes = [ctypes.c_void_p, ctypes.c_int] + [_dp] * 5
        lib.or_table_sizes.argtypes = [ctypes.c_void_p, _ip]
        lib.or_get_cells_on_cell.argtypes = [ctypes.c_void_p, _ip]
        lib.or_get_edge_sign.argtypes = [ctypes.c_void_p, _dp]
        lib.or_get_vertex_sign.argtypes = [ctypes.c_void_p, _dp]
        lib.or_get_trisk.argtypes = [ctypes.c_void_p, _ip, _ip, _dp]
        lib.or_get_hessian.argtypes = [ctypes.c_void_p, _dp]
        lib.or_sw_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, ctypes.c_int]
        lib.or_hdc_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, ctypes.c_int]
        lib.or_ndc_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        lib.or_tracer_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, _dp, ctypes.c_int]
        lib.or_tracer_vertical_column.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double] + [_dp] * 4
        lib.or_hdc_run_flux.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, ctypes.c_int,
                                        _dp, _dp]
        lib.or_ndc_run_flux.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, _dp, _dp,
                                        ctypes.c_int, _dp, _dp]
        lib.or_hdc_tendency.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params)] + [_dp] * 7
        lib.or_hdc_pgf.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp]
        lib.or_nh_column_solve.argtypes = [ctypes.POINTER(Params), ctypes.c_double, _dp, _dp, _dp, _dp]
        lib.or_nh_surface_w.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _dp, _dp, _dp, _dp]
        lib.or_norms.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.or_area_sum.restype = ctypes.c_double
        lib.or_area_sum.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_num_threads.argtypes = [ctypes.c_int]
        lib.or_energy.restype = ctypes.c_double
        lib.or_energy.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_int] + [_dp] * 6
        _lib = lib
    return _lib


def _d(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle needs C-contiguous float64"
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


GRAV, RD, CP, P0, PTOP = 9.80616, 287.0, 1004.5, 1.0e5, 1000.0


class OracleMesh:
    """Oracle tables for one mesh dict (as produced by the mesh generator)."""

    def __init__(self, mesh):
        self.lib = oracle_lib()
        self.mesh = mesh
        keep = {}
        for k in ["cells_on_edge", "vertices_on_edge", "eoc_offset", "edges_on_cell", "vertices_on_cell",
                  "cells_on_vertex", "edges_on_vertex"]:
            keep[k] = np.ascontiguousarray(mesh[k], dtype=np.int32)
        for k in ["xCell", "xVertex", "xEdge", "dEdge", "lEdge", "areaCell", "areaVertex", "kiteArea", "fVertex"]:
            keep[k] = np.ascontiguousarray(mesh[k], dtype=np.float64)
        self._keep = keep
        self.N, self.E, self.V = int(mesh["nCells"]), int(mesh["nEdges"]), int(mesh["nVertices"])
        mi = MeshIn(self.N, self.E, self.V,
                    *[_i(keep[k]) for k in ["cells_on_edge", "vertices_on_edge", "eoc_offset", "edges_on_cell",
                                            "vertices_on_cell", "cells_on_vertex", "edges_on_vertex"]],
                    *[_d(keep[k]) for k in ["xCell", "xVertex", "xEdge", "dEdge", "lEdge", "areaCell",
                                            "areaVertex", "kiteArea", "fVertex"]],
                    float(mesh["radius"]))
        self._mi = mi
        self.h = self.lib.or_mesh_build(ctypes.byref(mi))
        if not self.h:
            raise ValueError("oracle rejected the mesh")

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or_mesh_free(self.h)
            self.h = None

    # ---- tables ----
    def tables(self):
        n = ctypes.c_int()
        self.lib.or_table_sizes(self.h, ctypes.byref(n))
        coc = np.empty(2 * self.E, np.int32)
        sg = np.empty(2 * self.E)
        sv = np.empty(3 * self.V)
        toff = np.empty(self.E + 1, np.int32)
        te = np.empty(n.value, np.int32)
        tw = np.empty(n.value)
        hw = np.empty((2 * self.E, 6))
        self.lib.or_get_cells_on_cell(self.h, _i(coc))
        self.lib.or_get_edge_sign(self.h, _d(sg))
        self.lib.or_get_vertex_sign(self.h, _d(sv))
        self.lib.or_get_trisk(self.h, _i(toff), _i(te), _d(tw))
        self.lib.or_get_hessian(self.h, _d(hw))
        return dict(cells_on_cell=coc, edge_sign=sg, vertex_sign=sv.reshape(self.V, 3), trisk_offset=toff,
                    trisk_edge=te, trisk_weight=tw, hessian=hw)

    # ---- operators: arrays [entity][K] ----
    def _op(self, name, x, nout, K):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.empty((nout, K))
        getattr(self.lib, name)(self.h, K, _d(x), _d(out))
        return out

    @staticmethod
    def _k(x):
        return 1 if x.ndim == 1 else x.shape[1]

    def gradient(self, psi):
        return self._op("or_gradient", psi, self.E, self._k(psi)).reshape(self.E, -1).squeeze()

    def divergence(self, F):
        return self._op("or_divergence", F, self.N, self._k(F)).squeeze()

    def curl(self, u):
        return self._op("or_curl", u, self.V, self._k(u)).squeeze()

    def kinetic_energy(self, u):
        return self._op("or_kinetic_energy", u, self.N, self._k(u)).squeeze()

    def vertex_mass(self, h):
        return self._op("or_vertex_mass", h, self.V, self._k(h)).squeeze()

    def perp_flux(self, F):
        return self._op("or_perp_flux", F, self.E, self._k(F)).squeeze()

    def hessian_dir(self, q):
        return self._op("or_hessian_dir", q, 2 * self.E, self._k(q)).squeeze()

    def coriolis(self, F, qv):
        K = self._k(F)
        F = np.ascontiguousarray(F, dtype=np.float64)
        qv = np.ascontiguousarray(qv, dtype=np.float64)
        out = np.empty((self.E, K))
        self.lib.or_coriolis(self.h, K, _d(F), _d(qv), _d(out))
        return out.squeeze()

    def edge_value3(self, q, F):
        K = self._k(q)
        q = np.ascontiguousarray(q, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.float64)
        out = np.empty((self.E, K))
        self.lib.or_edge_value3(self.h, K, _d(q), _d(F), _d(out))
        return out.squeeze()

    def iface_advection(self, F, dpi, mdot, X):
        """V.grad X + eta_dot dX/deta of the interface field X [N][K+1] (Eqs. 6-7)
        for layer mass fluxes F [E][K], layer masses dpi [N][K] and interface
        vertical mass fluxes mdot [N][K+1]; returns [N][K+1]."""
        F, dpi, mdot, X = [np.ascontiguousarray(a, dtype=np.float64) for a in (F, dpi, mdot, X)]
        K = dpi.shape[1]
        assert F.shape == (self.E, K) and mdot.shape == (self.N, K + 1) and X.shape == (self.N, K + 1)
        out = np.empty((self.N, K + 1))
        self.lib.or_iface_advection(self.h, K, _d(F), _d(dpi), _d(mdot), _d(X), _d(out))
        return out

    # ---- models (copies; inputs untouched) ----
    def params(self, K, dt, T=0, fct=1, sigma=None, phis=None, forward_backward=True):
        if sigma is None:
            sigma = np.arange(K + 1, dtype=np.float64) / K
        self._sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self._phis = None if phis is None else np.ascontiguousarray(phis, dtype=np.float64)
        return Params(K, T, dt, GRAV, RD, CP, P0, PTOP, _d(self._sigma), fct,
                      None if self._phis is None else _d(self._phis), int(not forward_backward))

    def sw_run(self, h, u, b, dt, nsteps, forward_backward=True):
        h, u, b = [np.array(x, dtype=np.float64, order="C") for x in (h, u, b)]
        p = self.params(1, dt, forward_backward=forward_backward)
        self.lib.or_sw_run(self.h, ctypes.byref(p), _d(h), _d(u), _d(b), nsteps)
        return h, u

    def hdc_run(self, ps, Theta, u, dt, nsteps, phis=None, forward_backward=True):
        """phis [N]: surface geopotential (terrain), None for a flat surface;
        forward_backward=False: plain RK3 stages (the PGF from the stage's input)."""
        ps, Theta, u = [np.array(x, dtype=np.float64, order="C") for x in (ps, Theta, u)]
        p = self.params(Theta.shape[1], dt, phis=phis, forward_backward=forward_backward)
        self.lib.or_hdc_run(self.h, ctypes.byref(p), _d(ps), _d(Theta), _d(u), nsteps)
        return ps, Theta, u

    def hdc_run_flux(self, ps, Theta, u, dt, nsteps):
        """hdc_run that also returns the sums of the last-stage mass fluxes
        over the steps: (ps, Theta, u, F_sum [E][K], mdot_sum [N][K+1])."""
        ps, Theta, u = [np.array(x, dtype=np.float64, order="C") for x in (ps, Theta, u)]
        K = Theta.shape[1]
        p = self.params(K, dt)
        Fa, Ma = np.zeros((self.E, K)), np.zeros((self.N, K + 1))
        self.lib.or_hdc_run_flux(self.h, ctypes.byref(p), _d(ps), _d(Theta), _d(u), nsteps, _d(Fa), _d(Ma))
        return ps, Theta, u, Fa, Ma

    def ndc_run_flux(self, ps, Theta, u, w, phi, dt, nsteps):
        """ndc_run that also returns the sums of the last-stage mass fluxes."""
        ps, Theta, u, w, phi = [np.array(x, dtype=np.float64, order="C") for x in (ps, Theta, u, w, phi)]
        K = Theta.shape[1]
        p = self.params(K, dt)
        Fa, Ma = np.zeros((self.E, K)), np.zeros((self.N, K + 1))
        self.lib.or_ndc_run_flux(self.h, ctypes.byref(p), _d(ps), _d(Theta), _d(u), _d(w), _d(phi), nsteps,
                                 _d(Fa), _d(Ma))
        return ps, Theta, u, w, phi, Fa, Ma

    def ndc_run(self, ps, Theta, u, w, phi, dt, nsteps):
        ps, Theta, u, w, phi = [np.array(x, dtype=np.float64, order="C") for x in (ps, Theta, u, w, phi)]
        K = Theta.shape[1]
        if K < 2:
            raise ValueError("the non-hydrostatic column needs K >= 2")
        p = self.params(K, dt)
        self.lib.or_ndc_run(self.h, ctypes.byref(p), _d(ps), _d(Theta), _d(u), _d(w), _d(phi), nsteps)
        return ps, Theta, u, w, phi

    def hdc_pgf(self, ps, Theta, phis=None):
        """Pressure-gradient and gravity term [E][K] of the hydrostatic model at (pi_s, Theta)."""
        ps, Theta = [np.ascontiguousarray(x, dtype=np.float64) for x in (ps, Theta)]
        K = Theta.shape[1]
        p = self.params(K, 1.0, phis=phis)
        out = np.empty((self.E, K))
        self.lib.or_hdc_pgf(self.h, ctypes.byref(p), _d(ps), _d(Theta), _d(out))
        return out

    def hdc_tendency(self, ps, Theta, u):
        """Stage tendencies at a state: (dps, dTheta, du without PGF, mdot)."""
        ps, Theta, u = [np.ascontiguousarray(x, dtype=np.float64) for x in (ps, Theta, u)]
        K = Theta.shape[1]
        p = self.params(K, 1.0)
        dps, dTh = np.empty(self.N), np.empty((self.N, K))
        du, md = np.empty((self.E, K)), np.empty((self.N, K + 1))
        self.lib.or_hdc_tendency(self.h, ctypes.byref(p), _d(ps), _d(Theta), _d(u), _d(dps), _d(dTh), _d(du), _d(md))
        return dps, dTh, du, md

    def nh_column_solve(self, Theta, dpi, wstar, phistar, dts):
        """Implicit vertical step of one column: returns (w, phi) [K+1]."""
        K = len(Theta)
        w = np.array(wstar, dtype=np.float64)
        phi = np.array(phistar, dtype=np.float64)
        Th = np.ascontiguousarray(Theta, dtype=np.float64)
        dp = np.ascontiguousarray(dpi, dtype=np.float64)
        p = self.params(K, dts)
        self.lib.or_nh_column_solve(ctypes.byref(p), dts, _d(Th), _d(dp), _d(w), _d(phi))
        return w, phi

    def nh_surface_w(self, F, dpi, phi):
        """Kinematic surface w [N] (g w_s = V.grad phi_s, Eq. 7 at the surface) for
        layer mass fluxes F [E][K], layer masses dpi [N][K] and phi [N][K+1],
        whose bottom interface is the surface geopotential."""
        F, dpi, phi = [np.ascontiguousarray(a, dtype=np.float64) for a in (F, dpi, phi)]
        K = dpi.shape[1]
        assert F.shape == (self.E, K) and phi.shape == (self.N, K + 1)
        w = np.zeros((self.N, K + 1))
        p = self.params(K, 1.0)
        self.lib.or_nh_surface_w(self.h, ctypes.byref(p), _d(F), _d(dpi), _d(phi), _d(w))
        return w[:, K].copy()

    def energy(self, model, ps, u, Theta=None, w=None, phi=None, b=None, phis=None):
        """Total energy (J): model "SW" (ps = h, b), "HDC" (phis) or "NDC" (w, phi)."""
        mid = {"SW": 0, "HDC": 1, "NDC": 2}[model]
        arr = lambda x: None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        ps, u, Theta, w, phi, b = [arr(x) for x in (ps, u, Theta, w, phi, b)]
        K = 1 if mid == 0 else Theta.shape[1]
        p = self.params(K, 1.0, phis=phis)
        ptr = lambda x: None if x is None else _d(x)
        return self.lib.or_energy(self.h, ctypes.byref(p), mid, ptr(ps), ptr(Theta), ptr(u), ptr(w), ptr(phi),
                                  ptr(b))

    def tracer_run(self, F, dpi, q, dt, nsteps, fct=True, vflux=None):
        """vflux [N][K+1]: vertical mass flux through the interfaces (or None)."""
        F, dpi, q = [np.array(x, dtype=np.float64, order="C") for x in (F, dpi, q)]
        K, T = q.shape[1], q.shape[2]
        p = self.params(K, dt, T=T, fct=int(bool(fct)))
        vf = None if vflux is None else np.ascontiguousarray(vflux, dtype=np.float64)
        self.lib.or_tracer_run(self.h, ctypes.byref(p), _d(F), None if vf is None else _d(vf), _d(dpi), _d(q),
                               nsteps)
        return dpi, q


def norms(area, x, ref):
    """(l1, l2, linf) area-weighted normalised error of x against ref ([n] or [n][K])."""
    lib = oracle_lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float64)
    n = area.shape[0]
    K = x.size // n
    out = np.empty(3)
    lib.or_norms(n, K, _d(area), _d(x), _d(ref), _d(out))
    return out


def area_sum(area, x):
    lib = oracle_lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float64)
    n = area.shape[0]
    return lib.or_area_sum(n, x.size // n, _d(area), _d(x))


def tracer_vertical_column(dpih, m, q, dt):
    """Vertical tracer step of one column: dpih [K], m [K+1], q [K] or [K][T];
    returns (q_new, dpi_new)."""
    lib = oracle_lib()
    dpih = np.ascontiguousarray(dpih, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.float64)
    q = np.array(q, dtype=np.float64, order="C")
    K = len(dpih)
    T = 1 if q.ndim == 1 else q.shape[1]
    dn = np.empty(K)
    lib.or_tracer_vertical_column(K, T, float(dt), _d(dpih), _d(m), _d(q), _d(dn))
    return q, dn


def thomas(sub, diag, sup, rhs):
    lib = oracle_lib()
    sub, diag, sup, rhs = [np.ascontiguousarray(a, dtype=np.float64) for a in (sub, diag, sup, rhs)]
    x = np.empty_like(rhs)
    if lib.or_thomas(len(rhs), _d(sub), _d(diag), _d(sup), _d(rhs), _d(x)):
        raise ZeroDivisionError("zero pivot")
    return x
