"""Pins of the oracle's vertical tracer step and of the dycore-to-tracer mass
flux coupling (CPU).

The tracer equation (Eq. 10) has a vertical flux divergence besides the
horizontal one; the tracer step is time-split from the dycore and its mass
flux is the dycore's, accumulated over the dycore steps and averaged
(Section 2.1, Section 2.3).  Pins:

* vertical step: a constant mixing ratio stays constant for any interface
  flux (including Courant numbers well above 1/2, where the implicit part
  acts); column tracer mass is conserved; no new extrema; zero flux leaves
  the column unchanged; with every Courant number <= 1/2 the step is the
  explicit first-order upwind update (written out here as a plain loop); a
  three-layer through-flow solved by hand; reflection symmetry (flipping the
  column and the flux sign mirrors the result);
* coupling: after n dycore steps, a tracer step of n dt with the averaged
  last-stage fluxes gives layer masses equal to the dycore's
  (sigma_{k+1} - sigma_k)(pi_s - pi_t) to rounding, in the hydrostatic and the
  non-hydrostatic model; a constant tracer stays constant and tracer mass is
  conserved.
"""
import numpy as np
import pytest

from oracle import OracleMesh, area_sum, tracer_vertical_column
from paper_2404_08849_amd.inputs import initial as ic

PTOP = 1000.0


def _column(K, T, cmax, seed, pattern="through"):
    """Random column: layer masses, an interface flux whose largest Courant
    number is about cmax (zero at the lid and the surface), tracers in [0, 1].
    The lid and surface layers are thick so that the new masses stay positive
    under a strong flow through the thin interior layers."""
    r = np.random.default_rng(seed)
    dt = 600.0
    dpih = 1000.0 * (1.0 + r.random(K))
    dpih[0] = dpih[-1] = 1000.0 * (2.0 + cmax)
    U = cmax * 1000.0 / dt * (1.0 if r.random() < 0.5 else -1.0)
    k = np.arange(1, K)
    shape = np.ones(K - 1) if pattern == "through" else np.sin(2.0 * np.pi * k / K)
    m = np.zeros(K + 1)
    m[1:K] = U * shape * (1.0 + 0.02 * r.standard_normal(K - 1))
    q = r.random((K, T))
    return dt, dpih, m, q


def _courant(dt, dpih, m):
    K = len(dpih)
    c = np.zeros(K + 1)
    for k in range(1, K):
        d = dpih[k - 1] if m[k] >= 0 else dpih[k]
        c[k] = dt * abs(m[k]) / d
    return c


# (the two-cell circulation converges and diverges in the thin interior
# layers, so its Courant numbers stay lower there)
@pytest.mark.parametrize("cmax,pattern", [(0.3, "through"), (3.0, "through"), (12.0, "through"),
                                          (0.3, "cells"), (3.0, "cells")])
def test_constant_stays_constant_and_mass_is_conserved(cmax, pattern):
    dt, dpih, m, q = _column(30, 4, cmax, seed=int(cmax * 10), pattern=pattern)
    dn = dpih - dt * (m[1:] - m[:-1])
    assert dn.min() > 0
    if cmax > 1:
        assert _courant(dt, dpih, m).max() > 1.0          # the implicit part is exercised
    qc = np.full_like(q, 0.37)
    qn, dpn = tracer_vertical_column(dpih, m, qc, dt)
    assert np.abs(qn - 0.37).max() <= 1e-14
    assert np.allclose(dpn, dn, rtol=0, atol=1e-12 * dpih.max())
    qn, dpn = tracer_vertical_column(dpih, m, q, dt)
    for t in range(q.shape[1]):
        before = np.dot(dpih, q[:, t])
        after = np.dot(dpn, qn[:, t])
        assert abs(after - before) <= 1e-14 * before
        assert qn[:, t].min() >= q[:, t].min() - 1e-15 and qn[:, t].max() <= q[:, t].max() + 1e-15


def test_zero_flux_is_identity():
    dt, dpih, m, q = _column(12, 3, 1.0, seed=5)
    qn, dpn = tracer_vertical_column(dpih, np.zeros_like(m), q, dt)
    assert np.array_equal(dpn, dpih)
    assert np.allclose(qn, q, rtol=2e-16, atol=0)


def test_small_courant_is_explicit_upwind():
    dt, dpih, m, q = _column(20, 2, 0.3, seed=11, pattern="cells")
    assert _courant(dt, dpih, m).max() <= 0.5
    K = len(dpih)
    qn, dpn = tracer_vertical_column(dpih, m, q, dt)
    ref = np.empty_like(q)
    for t in range(q.shape[1]):
        for k in range(K):
            top = 0.0 if k == 0 else m[k] * (q[k - 1, t] if m[k] >= 0 else q[k, t])
            bot = 0.0 if k == K - 1 else m[k + 1] * (q[k, t] if m[k + 1] >= 0 else q[k + 1, t])
            dnew = dpih[k] - dt * ((0.0 if k == K - 1 else m[k + 1]) - (0.0 if k == 0 else m[k]))
            ref[k, t] = (dpih[k] * q[k, t] - dt * (bot - top)) / dnew
    assert np.allclose(qn, ref, rtol=1e-14, atol=0)


def test_three_layer_through_flow_by_hand():
    # unit layer masses, a downward through-flow with dt m = c at both interior
    # interfaces; c > 1/2 splits into dt mE = 1/2 and dt mI = b = c - 1/2.
    # Layer 0 only loses mass and keeps its mixing ratio; layer 1 keeps its
    # mass: (1 + b) q1 - b q0 = q1h - (q1h - q0h)/2; layer 2 gains c:
    # (1 + c) q2 - b q1 = q2h + q1h/2.
    c, dt = 0.8, 100.0
    b = c - 0.5
    dpih = np.ones(3)
    m = np.array([0.0, c / dt, c / dt, 0.0])
    qh = np.array([0.9, 0.2, 0.5])
    qn, dpn = tracer_vertical_column(dpih, m, qh, dt)
    q0 = qh[0]
    q1 = (0.5 * qh[1] + 0.5 * qh[0] + b * q0) / (1.0 + b)
    q2 = (qh[2] + 0.5 * qh[1] + b * q1) / (1.0 + c)
    assert np.allclose(dpn, [1.0 - c, 1.0, 1.0 + c], rtol=1e-15)
    assert np.allclose(qn, [q0, q1, q2], rtol=1e-14)


def test_reflection_symmetry():
    dt, dpih, m, q = _column(16, 3, 4.0, seed=21, pattern="cells")
    qn, dpn = tracer_vertical_column(dpih, m, q, dt)
    qr, dpr = tracer_vertical_column(dpih[::-1].copy(), -m[::-1].copy(), q[::-1].copy(), dt)
    assert np.allclose(dpr[::-1], dpn, rtol=1e-14)
    assert np.allclose(qr[::-1], qn, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("model", ["HDC", "NDC"])
def test_coupled_tracer_mass_equals_dycore_mass(mesh_cache, model):
    m = mesh_cache(3)
    om = OracleMesh(m)
    K, n, dt = 8, 3, 600.0 if model == "HDC" else 60.0
    sig = ic.sigma_interfaces(K)
    if model == "HDC":
        s = ic.hdc_jet(m, K, seed=2000)
        ps, Th, u, Fs, Ms = om.hdc_run_flux(s["ps"], s["Theta"], s["u"], dt, n)
        ps_plain = om.hdc_run(s["ps"], s["Theta"], s["u"], dt, n)[0]
    else:
        s = ic.nh_warm_bubble(m, K, rh=6.0e5, seed=4000)
        ps, Th, u, w, phi, Fs, Ms = om.ndc_run_flux(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], dt, n)
        ps_plain = om.ndc_run(s["ps"], s["Theta"], s["u"], s["w"], s["phi"], dt, n)[0]
    assert np.array_equal(ps, ps_plain)                  # accumulating does not change the run
    assert np.all(Ms[:, 0] == 0) and np.all(Ms[:, K] == 0)
    dsig = np.diff(sig)
    dpi0 = dsig[None, :] * (s["ps"][:, None] - PTOP)
    dpi_dyn = dsig[None, :] * (ps[:, None] - PTOP)
    r = np.random.default_rng(3)
    q = np.concatenate([np.full((m["nCells"], K, 1), 0.25), r.random((m["nCells"], K, 2))], axis=2)
    dpi_tr, qn = om.tracer_run(Fs / n, dpi0, q, n * dt, 1, vflux=Ms / n)
    err = np.abs(dpi_tr - dpi_dyn).max() / np.abs(dpi_dyn).max()
    assert err <= 1e-13, err
    assert np.abs(qn[:, :, 0] - 0.25).max() <= 1e-13
    for t in range(3):
        before = area_sum(m["areaCell"], dpi0 * q[:, :, t])
        after = area_sum(m["areaCell"], dpi_tr * qn[:, :, t])
        assert abs(after - before) <= 1e-13 * before
    # the vertical flux matters: transporting without it leaves the masses apart
    dpi_h, _ = om.tracer_run(Fs / n, dpi0, q, n * dt, 1)
    assert np.abs(dpi_h - dpi_dyn).max() / np.abs(dpi_dyn).max() > 1e3 * max(err, 1e-16)
