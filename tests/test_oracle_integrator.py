"""Pins of the oracle's predictor-corrector time stepping (paper section
"Time Integration") and of the whole step against the Taylor-Green vortex's
exact solution (paper section "Taylor-Green Vortex").

Facts used: exact integration of constant acceleration by the kick-drift-kick
scheme, its time reversibility when the acceleration depends on positions
only, momentum conservation, periodic wrap, and the analytic energy decay
KE(t) = KE(0) exp(2 b t), b = -8 pi^2 nu / L^2."""
import numpy as np
import pytest

import oracle
import sph_workloads as W


def test_isolated_particles_fall_exactly():
    """Particles far apart (only themselves as neighbours) under gravity:
    x = x0 + u0 t + g t^2 / 2, u = u0 + g t (exact for constant a)."""
    n = 5
    x0 = np.stack([np.linspace(0.1, 0.9, n), np.full(n, 0.5), np.linspace(0.2, 0.8, n)])
    u0 = np.stack([np.linspace(-1, 1, n), np.linspace(0.5, -0.5, n), np.zeros(n)])
    p = W.Params(dim=3, kernel=W.WENDLAND, h=0.04, rho0=1000.0, c0=20.0, nu=1e-3, eta=0.01,
                 dt=1e-3, g=(0.0, 0.0, -9.81), lo=(-1, -1, -1), hi=(2, 2, 2),
                 periodic=(0, 0, 0))
    m = np.full(n, 1e-6)
    steps = 200
    out = oracle.step(p, x0, u0, m, np.zeros(n, np.uint8), steps)
    t = steps * p.dt
    g = np.array(p.g)[:, None]
    # a = g + 0 (only self in the neighbour set)
    assert np.allclose(out["u"], u0 + g * t, rtol=0, atol=1e-12)
    assert np.allclose(out["x"], x0 + u0 * t + 0.5 * g * t * t, rtol=0, atol=1e-12)


def test_time_reversibility_inviscid():
    """With nu = 0 the acceleration depends on positions only and KDK is
    time-reversible: n steps, negate u, n steps returns to x0."""
    p, s = W.taylor_green(16, jitter=0.2, seed=3)
    p = p.replace(nu=0.0)
    n = 20
    f = oracle.step(p, s.x, s.u, s.m, s.ptype, n)
    b = oracle.step(p, f["x"], -f["u"], s.m, s.ptype, n, a=f["a"], prime=False)
    dx = b["x"] - s.x
    dx -= np.round(dx)  # periodic unit box
    assert np.abs(dx).max() < 1e-12
    assert np.abs(-b["u"] - s.u).max() < 1e-11


def test_momentum_conserved_over_steps():
    p, s = W.taylor_green(24, jitter=0.3, seed=5)
    out = oracle.step(p, s.x, s.u, s.m, s.ptype, 30, want_diag=True)
    mom0 = (s.m * s.u).sum(axis=1)
    scale = (s.m * np.abs(s.u)).sum()
    assert np.abs(out["diag"][:, 1:] - mom0).max() < 30 * 1e-14 * scale + 1e-16


def test_positions_stay_in_periodic_box():
    p, s = W.taylor_green(16, jitter=0.45, seed=2)
    out = oracle.step(p, s.x, 3 * s.u + 0.5, s.m, s.ptype, 40)
    assert np.all(out["x"] >= 0.0) and np.all(out["x"] < 1.0)


def test_diagnostics_compensated():
    p, s = W.taylor_green(32)
    d = oracle.diag(p, s.u, s.m)
    assert d[0] == pytest.approx(0.25, rel=1e-12)   # (1/2) * U^2/2 over the unit box
    assert abs(d[1]) < 1e-15 and abs(d[2]) < 1e-15


def test_walls_stay_fixed():
    p, s = W.taylor_green(16, jitter=0.2, seed=8)
    s.ptype[: 40] = W.WALL
    s.u[:, :40] = 0.0
    out = oracle.step(p, s.x, s.u, s.m, s.ptype, 10)
    assert np.array_equal(out["x"][:, :40], s.x[:, :40])
    assert np.all(out["u"][:, :40] == 0.0) and np.all(out["a"][:, :40] == 0.0)


@pytest.mark.parametrize("n_side", [32, 64])
def test_taylor_green_energy_decay(n_side):
    """KE(t) follows KE(0) exp(2 b t), b = -8 pi^2 nu (U = L = 1), within 1%
    pointwise and 2% in the fitted rate, over t <= 0.1.  (Beyond t ~ 0.1 the
    classic scheme's particle arrangement degrades in the vortex stagnation
    regions and its decay departs from the exact one; the paper's own
    Taylor-Green run uses EDAC instead.)"""
    p, s = W.taylor_green(n_side)
    nsteps = int(round(0.1 / p.dt))
    out = oracle.step(p, s.x, s.u, s.m, s.ptype, nsteps, want_diag=True)
    t = (np.arange(nsteps) + 1) * p.dt
    ke = out["diag"][:, 0]
    b = -8 * np.pi ** 2 * p.nu
    exact = 0.25 * np.exp(2 * b * t)
    assert np.abs(ke / exact - 1).max() < 1e-2
    slope = np.polyfit(t, np.log(ke), 1)[0]
    assert abs(slope / (2 * b) - 1) < 2e-2
