"""Pins of the oracle's adjoint (reverse-mode derivative of the
predictor-corrector rollout, for the gradient of the final kinetic energy with
respect to the viscosity and the initial velocities).

Facts used: central finite differences of the oracle's forward map (a
different code path from the hand-written transpose), the dot-product
identity <lam, J w> = <J^T lam, w> for the right-hand side, and the closed
form for isolated particles under gravity: dKE/du0 = m (u0 + g t),
dKE/dnu = 0."""
import numpy as np
import pytest

import oracle
import sph_workloads as W


def _small(jitter=0.25, seed=3, n_side=12):
    p, s = W.taylor_green(n_side, jitter=jitter, seed=seed)
    return p, s


@pytest.mark.parametrize("which", ["x", "v"])
def test_rhs_transpose_dot_product(which):
    """<lam, (A(z + e w) - A(z - e w)) / 2e> equals <(dA/dz)^T lam, w>."""
    p, s = _small()
    rng = np.random.default_rng(17)
    lam = rng.standard_normal(s.x.shape)
    w = rng.standard_normal(s.x.shape)
    lx, lv, _ = oracle.rhs_adjoint(p, s.x, s.u, s.m, s.ptype, lam)
    eps = 1e-7 if which == "x" else 1e-5
    if which == "x":
        ap = oracle.evaluate(p, s.x + eps * w * (1.0 / 12), s.u, s.m, s.ptype)[2]
        am = oracle.evaluate(p, s.x - eps * w * (1.0 / 12), s.u, s.m, s.ptype)[2]
        lhs = np.sum(lam * (ap - am)) / (2 * eps)
        rhs = np.sum(lx * w) / 12
    else:
        ap = oracle.evaluate(p, s.x, s.u + eps * w, s.m, s.ptype)[2]
        am = oracle.evaluate(p, s.x, s.u - eps * w, s.m, s.ptype)[2]
        lhs = np.sum(lam * (ap - am)) / (2 * eps)
        rhs = np.sum(lv * w)
    assert lhs == pytest.approx(rhs, rel=1e-6)


def test_rhs_transpose_nu():
    p, s = _small()
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(s.x.shape)
    _, _, lnu = oracle.rhs_adjoint(p, s.x, s.u, s.m, s.ptype, lam)
    eps = 1e-6
    ap = oracle.evaluate(p.replace(nu=p.nu + eps), s.x, s.u, s.m, s.ptype)[2]
    am = oracle.evaluate(p.replace(nu=p.nu - eps), s.x, s.u, s.m, s.ptype)[2]
    assert np.sum(lam * (ap - am)) / (2 * eps) == pytest.approx(lnu, rel=1e-8)


def test_rhs_transpose_3d_wendland_with_walls():
    p, s = W.periodic_cube(n_side=10, jitter=0.3, sigma_u=0.1, seed=2)
    s.ptype[:50] = W.WALL
    s.u[:, :50] = 0.0
    rng = np.random.default_rng(9)
    lam = rng.standard_normal(s.x.shape)
    w = rng.standard_normal(s.x.shape)
    lx, lv, lnu = oracle.rhs_adjoint(p, s.x, s.u, s.m, s.ptype, lam)
    eps = 1e-8
    ap = oracle.evaluate(p, s.x + eps * w, s.u, s.m, s.ptype)[2]
    am = oracle.evaluate(p, s.x - eps * w, s.u, s.m, s.ptype)[2]
    assert np.sum(lam * (ap - am)) / (2 * eps) == pytest.approx(np.sum(lx * w), rel=1e-5)
    ap = oracle.evaluate(p, s.x, s.u + 1e-5 * w, s.m, s.ptype)[2]
    am = oracle.evaluate(p, s.x, s.u - 1e-5 * w, s.m, s.ptype)[2]
    assert np.sum(lam * (ap - am)) / 2e-5 == pytest.approx(np.sum(lv * w), rel=1e-7)


def test_rollout_gradient_matches_central_differences():
    p, s = _small(n_side=12)
    nsteps = 8
    gu, gnu, ke = oracle.adjoint_ke(p, s.x, s.u, s.m, s.ptype, nsteps)
    assert ke == pytest.approx(oracle.rollout_ke(p, s.x, s.u, s.m, s.ptype, nsteps), rel=1e-15)
    eps = 1e-6
    kp = oracle.rollout_ke(p.replace(nu=p.nu + eps), s.x, s.u, s.m, s.ptype, nsteps)
    km = oracle.rollout_ke(p.replace(nu=p.nu - eps), s.x, s.u, s.m, s.ptype, nsteps)
    assert (kp - km) / (2 * eps) == pytest.approx(gnu, rel=1e-6)
    rng = np.random.default_rng(1)
    w = rng.standard_normal(s.u.shape)
    w /= np.sqrt(np.mean(w * w))
    eps = 1e-5
    kp = oracle.rollout_ke(p, s.x, s.u + eps * w, s.m, s.ptype, nsteps)
    km = oracle.rollout_ke(p, s.x, s.u - eps * w, s.m, s.ptype, nsteps)
    assert (kp - km) / (2 * eps) == pytest.approx(np.sum(gu * w), rel=1e-6)


def test_isolated_particles_closed_form():
    n = 4
    x0 = np.stack([np.linspace(0.1, 0.9, n), np.full(n, 0.5)])
    u0 = np.stack([np.linspace(-1, 1, n), np.linspace(0.5, -0.5, n)])
    p = W.Params(dim=2, kernel=W.CUBIC, h=0.04, rho0=1.0, c0=20.0, nu=1e-2, eta=0.01,
                 dt=1e-3, g=(0.0, -9.81, 0.0), lo=(-1, -1, 0), hi=(2, 2, 0),
                 periodic=(0, 0, 0))
    m = np.array([1.0, 2.0, 0.5, 3.0])
    nsteps = 50
    gu, gnu, _ = oracle.adjoint_ke(p, x0, u0, m, np.zeros(n, np.uint8), nsteps)
    t = nsteps * p.dt
    expect = m * (u0 + np.array(p.g[:2])[:, None] * t)
    assert np.abs(gu - expect).max() < 1e-12
    assert gnu == 0.0
