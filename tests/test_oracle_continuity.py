"""Pins of the oracle's continuity scheme, the paper's worked example: density
rate by the continuity equation (eqn continuity:sph) over all neighbours of a
fluid particle and over fluid neighbours of a solid one, the EOS, the momentum
equation, and the example's Euler stage (u += dt a, then x += dt u with the
new u, rho += dt drho/dt).

Facts used: a uniform velocity field gives no density rate; a solid that sees
only solids has none; a linear compression u = -alpha x gives
drho/dt ~ rho alpha (the continuum rho div u) in the interior; an isolated
particle under gravity follows the closed form of the Euler recurrence; walls
stay put and keep rho0 far from the fluid."""
import numpy as np
import pytest

import oracle
import sph_workloads as W


def test_uniform_velocity_gives_no_density_rate():
    p, s = W.dam_break_2d()
    v = np.empty_like(s.x)
    v[0], v[1] = 0.75, -0.25
    arho = oracle.continuity(p, s.x, v, s.m, s.ptype)
    assert np.all(arho == 0.0)


def test_solids_only_see_fluid_sources():
    """Walls moving against each other but far from the fluid: their rate is
    exactly zero, while a fluid particle among them would see them."""
    p, s = W.dam_break_2d()
    rng = np.random.default_rng(3)
    v = rng.normal(size=s.x.shape)
    arho = oracle.continuity(p, s.x, v, s.m, s.ptype)
    wall = s.ptype == W.WALL
    fluid_x = s.x[:, ~wall]
    R = 2 * p.h
    far = np.array([np.min(np.hypot(*(fluid_x - s.x[:, [i]]))) >= R for i in range(s.n)])
    sel = wall & far
    assert sel.sum() > 100
    assert np.all(arho[sel] == 0.0)
    s2 = s.copy()
    s2.ptype[:] = W.FLUID
    arho2 = oracle.continuity(p, s2.x, v, s2.m, s2.ptype)
    assert np.count_nonzero(arho2[sel]) > 0.9 * sel.sum()


@pytest.mark.parametrize("n_side,tol", [(40, 2e-2), (80, 1e-2)])
def test_linear_compression_rate(n_side, tol):
    """u = -alpha x on a lattice: drho/dt ~ rho0 alpha away from the edges."""
    dx = 1.0 / n_side
    x = W.lattice((n_side, n_side), dx, (0.0, 0.0))
    rho0, h = 1000.0, 1.2 * dx
    p = W.Params(dim=2, kernel=W.CUBIC, h=h, rho0=rho0, c0=10.0, nu=0.0, eta=0.01, dt=1e-4,
                 g=(0, 0, 0), lo=(-0.1, -0.1, 0), hi=(1.1, 1.1, 0), periodic=(0, 0, 0))
    alpha = 0.3
    v = np.zeros_like(x)
    v[0] = -alpha * x[0]
    m = np.full(x.shape[1], rho0 * dx * dx)
    arho = oracle.continuity(p, x, v, m, np.zeros(x.shape[1], np.uint8))
    inner = np.all((x > 0.2) & (x < 0.8), axis=0)
    assert np.abs(arho[inner] - rho0 * alpha).max() < tol * rho0 * alpha


def test_isolated_particles_follow_the_euler_recurrence():
    """No neighbours: u_n = u0 + n g dt and, with x updated by the new u,
    x_n = x0 + n dt u0 + g dt^2 n (n + 1) / 2; rho stays rho0."""
    x = np.array([[0.1, 0.5, 0.9], [0.2, 0.6, 0.3]])
    u0 = np.array([[0.5, -0.25, 0.0], [0.0, 0.125, -0.5]])
    n = x.shape[1]
    p = W.Params(dim=2, kernel=W.CUBIC, h=0.01, rho0=1000.0, c0=10.0, nu=0.0, eta=0.01,
                 dt=1e-3, g=(0.0, -9.81, 0.0), lo=(0, 0, 0), hi=(1, 1, 0), periodic=(0, 0, 0),
                 scheme=W.CONTINUITY)
    steps = 40
    out = oracle.step_continuity(p, x, u0, np.full(n, 1000.0), np.full(n, 0.1),
                                 np.zeros(n, np.uint8), steps)
    g = np.array([[0.0], [-9.81]])
    assert np.abs(out["u"] - (u0 + steps * p.dt * g)).max() < 1e-13
    expect_x = x + steps * p.dt * u0 + g * p.dt ** 2 * steps * (steps + 1) / 2
    assert np.abs(out["x"] - expect_x).max() < 1e-13
    assert np.all(out["rho"] == 1000.0)


def test_dam_break_walls_stay_and_fluid_falls():
    wl = W.workload("dambreak2d")
    p, s = wl.params, wl.state
    out = oracle.step_continuity(p, s.x, s.u, s.rho, s.m, s.ptype, 200)
    wall = s.ptype == W.WALL
    assert np.array_equal(out["x"][:, wall], s.x[:, wall])
    assert np.all(out["u"][:, wall] == 0.0)
    # the column starts to fall: its centre of mass moves down
    assert out["x"][1, ~wall].mean() < s.x[1, ~wall].mean() - 1e-3
    # walls beyond the reach of the fluid keep rho0 exactly
    far = out["x"][1] > 2.5
    assert np.all(out["rho"][wall & far] == p.rho0)
    # the EOS of the last evaluation is the Tait law of the then density
    assert np.all(np.isfinite(out["p"]))


# ---- the continuity scheme under the predictor-corrector integration ----

def test_pc_isolated_particles_are_exact_under_gravity():
    """With a constant acceleration the kick-drift-kick recurrence is exact:
    u_n = u0 + g t_n and x_n = x0 + u0 t_n + g t_n^2 / 2; rho stays rho0."""
    x = np.array([[0.1, 0.5, 0.9], [0.2, 0.6, 0.3]])
    u0 = np.array([[0.5, -0.25, 0.0], [0.0, 0.125, -0.5]])
    n = x.shape[1]
    p = W.Params(dim=2, kernel=W.CUBIC, h=0.01, rho0=1000.0, c0=10.0, nu=0.0, eta=0.01,
                 dt=1e-3, g=(0.0, -9.81, 0.0), lo=(0, 0, 0), hi=(1, 1, 0), periodic=(0, 0, 0),
                 scheme=W.CONTINUITY)
    steps = 40
    out = oracle.step_continuity_pc(p, x, u0, np.full(n, 1000.0), np.full(n, 0.1),
                                    np.zeros(n, np.uint8), steps)
    g = np.array([[0.0], [-9.81]])
    t = steps * p.dt
    assert np.abs(out["u"] - (u0 + g * t)).max() < 1e-13
    assert np.abs(out["x"] - (x + u0 * t + 0.5 * g * t * t)).max() < 1e-13
    assert np.all(out["rho"] == 1000.0)
    assert np.all(out["arho"] == 0.0)


def _order_of_convergence(step, p, s, rho, dt0, nsteps0, halvings=2, ref_div=32):
    """Errors in x at the fixed time nsteps0 dt0 for dt0 / 2^k (k = 0..halvings)
    against a run at dt0 / ref_div; returns the ratios of successive errors."""
    def run(div):
        q = p.replace(dt=dt0 / div)
        return step(q, s.x, s.u, rho, s.m, s.ptype, nsteps0 * div)
    ref = run(ref_div)
    errs = []
    for k in range(halvings + 1):
        d = run(2 ** k)["x"] - ref["x"]
        d -= np.round(d)
        errs.append(np.abs(d).max())
    return [errs[k] / errs[k + 1] for k in range(halvings)], errs


def test_pc_is_second_order_and_euler_first():
    """Halving dt divides the position error at a fixed time by ~4 under the
    predictor-corrector (rho kicked like u) and by ~2 under the Euler stage:
    a rate taken at the wrong state or a kick in the wrong place drops the
    former to first order."""
    p, s = W.taylor_green(16, jitter=0.2, seed=5)
    p = p.replace(scheme=W.CONTINUITY)
    rng = np.random.default_rng(6)
    rho = p.rho0 * (1.0 + rng.uniform(-2e-3, 2e-3, size=s.n))
    dt0 = 2 * p.dt
    pc, e_pc = _order_of_convergence(oracle.step_continuity_pc, p, s, rho, dt0, 8)
    eu, e_eu = _order_of_convergence(oracle.step_continuity, p, s, rho, dt0, 8)
    assert all(3.3 < r < 4.7 for r in pc), (pc, e_pc)
    assert all(1.6 < r < 2.5 for r in eu), (eu, e_eu)


def test_pc_and_euler_share_their_first_rates():
    """Both integrators evaluate the same right-hand side: the rates of a
    primed predictor-corrector call with no steps equal the Euler step's
    rates at the same state."""
    p, s = W.dam_break_2d()
    rng = np.random.default_rng(7)
    f = s.ptype == W.FLUID
    s.u[:, f] = rng.normal(0.0, 0.3, size=(2, int(f.sum())))
    pc = oracle.step_continuity_pc(p, s.x, s.u, s.rho, s.m, s.ptype, 0)
    eu = oracle.step_continuity(p, s.x, s.u, s.rho, s.m, s.ptype, 1)
    assert np.array_equal(pc["a"], eu["a"])
    assert np.array_equal(pc["arho"], eu["arho"])
    assert np.array_equal(pc["arho"], oracle.continuity(p, s.x, s.u, s.m, s.ptype))


def test_dam_break_fixture_is_the_printed_example():
    """Section 3.2.1 prints the example's fluid block: 231 particles, x from
    -1.9 to -0.9, density 1000.  The fixture reproduces them (11 x 21 lattice
    points of spacing 0.1, edges included), on the same lattice as the tank's
    walls, one dx from the floor and the left wall."""
    p, s = W.dam_break_2d()
    fluid = s.ptype == W.FLUID
    assert int(fluid.sum()) == 231
    assert s.x[0, fluid].min() == pytest.approx(-1.9, abs=1e-12)
    assert s.x[0, fluid].max() == pytest.approx(-0.9, abs=1e-12)
    assert s.x[1, fluid].min() == pytest.approx(0.1, abs=1e-12)
    assert s.x[1, fluid].max() == pytest.approx(2.1, abs=1e-12)
    assert np.all(s.rho == 1000.0) and np.all(s.m == pytest.approx(1000.0 * 0.01))
    assert p.h == pytest.approx(0.12) and p.c0 == 10.0 and p.dt == 2e-4
    # every particle on the lattice x = i dx, y = j dx
    assert np.abs(s.x / 0.1 - np.round(s.x / 0.1)).max() < 1e-9
    wall = ~fluid
    gap = lambda k, v: np.abs(s.x[k, wall] - v)
    assert gap(0, -2.0).min() < 1e-12 and gap(1, 0.0).min() < 1e-12
