"""Pins of the oracle's summation density (eq. 2), Tait EOS (eq. eos) and
momentum equation (eq. mom:sph with its pressure and viscous terms).

Facts used: lattice symmetry (equal density everywhere, zero pressure force
under uniform pressure), the EOS special values and numpy's power function,
pairwise antisymmetry (momentum conservation), invariances (Galilean, uniform
velocity, translation), and convergence of the SPH operators to the continuum
derivatives they approximate (nu * Laplacian, -grad p / rho) on smooth fields."""
import numpy as np
import pytest

import oracle
import sph_workloads as W


def test_density_lattice_uniform_and_equals_lattice_sum():
    p, s = W.taylor_green(32)
    rho = oracle.density(p, s.x, s.m)
    assert np.ptp(rho) < 1e-14 * rho.mean()
    # the lattice sum over the 21 offsets with |r| < 2h, from the pinned kernel
    dx = 1.0 / 32
    offs = [(i, j) for i in range(-3, 4) for j in range(-3, 4)
            if (i * i + j * j) * dx * dx < (2 * p.h) ** 2]
    assert len(offs) == 21
    r = np.array([np.hypot(i, j) * dx for i, j in offs])
    expect = s.m[0] * oracle.kernel_w(p, r).sum()
    assert abs(rho[0] - expect) < 1e-14
    # and it approximates rho0 (the integral of W is 1)
    assert abs(rho[0] / p.rho0 - 1) < 1e-3


def test_density_lattice_quintic_equals_lattice_sum():
    """Quintic spline, support 3h with h = dx: the lattice sum over the 25
    offsets with |r| < 3dx (a direct count; exact ties at 3dx excluded)."""
    p, s = W.taylor_green(32, kernel=W.QUINTIC, hdx=1.0)
    rho = oracle.density(p, s.x, s.m)
    assert np.ptp(rho) < 1e-14 * rho.mean()
    dx = 1.0 / 32
    offs = [(i, j) for i in range(-3, 4) for j in range(-3, 4) if i * i + j * j < 9]
    assert len(offs) == 25
    r = np.array([np.hypot(i, j) * dx for i, j in offs])
    expect = s.m[0] * oracle.kernel_w(p, r).sum()
    assert abs(rho[0] - expect) < 1e-14
    assert abs(rho[0] / p.rho0 - 1) < 1e-3


def test_density_3d_lattice_wendland():
    p, s = W.periodic_cube(n_side=12, jitter=0.0, sigma_u=0.1)
    rho = oracle.density(p, s.x, s.m)
    assert np.ptp(rho) < 1e-13 * rho.mean()
    assert abs(rho[0] / p.rho0 - 1) < 2e-2


def test_mass_unchanged_by_sort():
    p, s = W.taylor_green(24, jitter=0.3, seed=5)
    _, perm, _, _ = oracle.bin_sort(p, s.x)
    assert np.sum(s.m[perm]) == pytest.approx(np.sum(s.m), rel=1e-15)
    rho1 = oracle.density(p, s.x, s.m)
    rho2 = oracle.density(p, s.x[:, perm], s.m[perm])
    assert np.abs(rho1[perm] - rho2).max() < 1e-14


def test_eos_special_values_and_power():
    p, _ = W.taylor_green(16)
    B = p.rho0 * p.c0 ** 2 / 7.0
    assert oracle.eos(p, np.array([p.rho0]))[0] == 0.0
    two = 2.0 ** (1.0 / 7.0) * p.rho0
    assert oracle.eos(p, np.array([two]))[0] == pytest.approx(B, rel=1e-14)
    rho = np.random.default_rng(0).uniform(0.9, 1.1, 100) * p.rho0
    ref = B * (np.power(rho / p.rho0, 7.0) - 1.0)
    assert np.abs(oracle.eos(p, rho) - ref).max() < 1e-12 * B


def _eval(p, s, v=None, pr=None):
    rho = oracle.density(p, s.x, s.m)
    if pr is None:
        pr = oracle.eos(p, rho)
    return rho, pr, oracle.momentum(p, s.x, s.u if v is None else v, s.m, s.ptype, rho, pr)


@pytest.mark.parametrize("kernel", [W.CUBIC, W.WENDLAND, W.QUINTIC])
def test_pairwise_antisymmetry_conserves_momentum(kernel):
    """sum_i m_i (a_i - g) = 0 to roundoff: the pair terms are antisymmetric."""
    p, s = W.taylor_green(24, jitter=0.3, seed=2, kernel=kernel)
    p = p.replace(g=(0.3, -1.0, 0.0))
    _, _, a = _eval(p, s)
    g = np.array(p.g[:2])[:, None]
    net = (s.m * (a - g)).sum(axis=1)
    scale = (s.m * np.abs(a - g)).sum()
    assert np.abs(net).max() < 1e-13 * scale


def test_pairwise_antisymmetry_3d():
    p, s = W.periodic_cube(n_side=10, jitter=0.3, sigma_u=0.1, seed=9)
    _, _, a = _eval(p, s)
    net = (s.m * a).sum(axis=1)
    scale = (s.m * np.abs(a)).sum()
    assert np.abs(net).max() < 1e-13 * scale


def test_uniform_velocity_gives_no_viscous_force():
    p, s = W.taylor_green(16, jitter=0.3, seed=1)
    v = np.empty_like(s.u)
    v[0], v[1] = 0.7, -0.2
    _, _, a = _eval(p, s, v=v, pr=np.zeros(s.n))
    assert np.all(a == 0.0)


def test_galilean_and_translation_invariance():
    p, s = W.taylor_green(20, jitter=0.3, seed=4)
    _, _, a0 = _eval(p, s)
    v = s.u + np.array([[0.5], [-0.25]])   # dyadic shift: v_i - v_j exact
    _, _, a1 = _eval(p, s, v=v)
    assert np.abs(a1 - a0).max() < 1e-12 * np.abs(a0).max()
    s2 = s.copy()
    s2.x = np.mod(s.x + np.array([[0.123], [0.456]]), 1.0)
    _, _, a2 = _eval(p, s2)
    assert np.abs(a2 - a0).max() < 1e-9 * np.abs(a0).max()


def test_uniform_pressure_on_lattice_gives_no_force():
    p, s = W.taylor_green(16)
    rho = oracle.density(p, s.x, s.m)
    pr = np.full(s.n, 3.7)
    a = oracle.momentum(p, s.x, np.zeros_like(s.u), s.m, s.ptype, rho, pr)
    assert np.abs(a).max() < 1e-10 * 3.7 / p.h


@pytest.mark.parametrize("n_side,tol", [(32, 1e-2), (64, 3e-3)])
def test_viscous_term_converges_to_laplacian(n_side, tol):
    """With p = 0 the momentum equation reduces to its viscous term, which
    approximates nu * Laplacian(u): on u = (sin 2 pi y, 0), a = -nu (2 pi)^2 u."""
    p, s = W.taylor_green(n_side)
    u = np.zeros_like(s.x)
    u[0] = np.sin(2 * np.pi * s.x[1])
    _, _, a = _eval(p, s, v=u, pr=np.zeros(s.n))
    exact = -p.nu * (2 * np.pi) ** 2 * u[0]
    assert np.abs(a[0] - exact).max() < tol * np.abs(exact).max()
    assert np.abs(a[1]).max() < 1e-12


@pytest.mark.parametrize("n_side,tol", [(32, 1.5e-2), (64, 1.5e-2), (128, 1.5e-2)])
def test_pressure_term_approximates_gradient(n_side, tol):
    """With u = 0 the momentum equation is the pressure term, approximating
    -grad(p)/rho: for p = P0 sin(2 pi x) on a lattice, a_x = -2 pi P0 cos(2 pi x)/rho.
    At fixed h/dx the lattice-sum error of this form does not vanish with dx
    (about 1% at h = 1.3 dx), so the bound is the same at every resolution."""
    p, s = W.taylor_green(n_side)
    rho = oracle.density(p, s.x, s.m)
    P0 = 0.5
    pr = P0 * np.sin(2 * np.pi * s.x[0])
    a = oracle.momentum(p, s.x, np.zeros_like(s.u), s.m, s.ptype, rho, pr)
    exact = -2 * np.pi * P0 * np.cos(2 * np.pi * s.x[0]) / rho
    assert np.abs(a[0] - exact).max() < tol * np.abs(exact).max()


@pytest.mark.parametrize("n_side,tol_visc,tol_pres", [(32, 1.5e-2, 1.5e-2), (64, 1e-2, 3e-3)])
def test_quintic_operators_approximate_derivatives(n_side, tol_visc, tol_pres):
    """Quintic spline (support 3h, h = dx): the viscous term approximates
    nu Laplacian(u) and the pressure term -grad(p)/rho on smooth fields, as
    for the other kernels."""
    p, s = W.taylor_green(n_side, kernel=W.QUINTIC, hdx=1.0)
    rho = oracle.density(p, s.x, s.m)
    u = np.zeros_like(s.x)
    u[0] = np.sin(2 * np.pi * s.x[1])
    a = oracle.momentum(p, s.x, u, s.m, s.ptype, rho, np.zeros(s.n))
    exact = -p.nu * (2 * np.pi) ** 2 * u[0]
    assert np.abs(a[0] - exact).max() < tol_visc * np.abs(exact).max()
    P0 = 0.5
    pr = P0 * np.sin(2 * np.pi * s.x[0])
    a = oracle.momentum(p, s.x, np.zeros_like(s.u), s.m, s.ptype, rho, pr)
    exact = -2 * np.pi * P0 * np.cos(2 * np.pi * s.x[0]) / rho
    assert np.abs(a[0] - exact).max() < tol_pres * np.abs(exact).max()


def test_walls_get_no_acceleration_but_act_as_sources():
    p, s = W.taylor_green(16, jitter=0.2, seed=8)
    s.ptype[: s.n // 2] = W.WALL
    _, _, a = _eval(p, s)
    assert np.all(a[:, : s.n // 2] == 0.0)
    s2 = s.copy()
    s2.ptype[:] = W.FLUID
    _, _, a2 = _eval(p, s2)
    # fluid destinations see the same sources whatever their type
    assert np.array_equal(a[:, s.n // 2:], a2[:, s.n // 2:])


def test_subset_evaluation_matches_full():
    p, s = W.taylor_green(20, jitter=0.3, seed=6)
    rho, pr, a = oracle.evaluate(p, s.x, s.u, s.m, s.ptype)
    sub = W.random_subset(s.n, 37)
    r2, p2, a2 = oracle.eval_subset(p, s.x, s.u, s.m, s.ptype, sub)
    assert np.abs(r2 - rho[sub]).max() < 1e-14
    assert np.abs(a2 - a[:, sub]).max() < 1e-12 * np.abs(a).max()


def _dense(p, s, rho0):
    """The same lattice at reference density rho0: m = rho0 dx^d."""
    p = p.replace(rho0=rho0)
    s = s.copy()
    s.m = s.m * rho0
    return p, s


@pytest.mark.parametrize("n_side,tol", [(32, 1.5e-2), (64, 1.5e-2)])
def test_pressure_term_scales_with_density(n_side, tol):
    """At rho0 = 1000 (m = rho0 dx^2, the dam-break density) the pressure term
    still approximates -grad(p)/rho: the p/rho^2 weighting of eq.
    mom:sph:press and the mass m_j = rho0 dx^2 combine into 1/rho.  A weight
    p/rho instead of p/rho^2 would be off by a factor rho0."""
    p, s = _dense(*W.taylor_green(n_side), 1000.0)
    rho = oracle.density(p, s.x, s.m)
    assert abs(rho.mean() / 1000.0 - 1) < 1e-3
    P0 = 500.0
    pr = P0 * np.sin(2 * np.pi * s.x[0])
    a = oracle.momentum(p, s.x, np.zeros_like(s.u), s.m, s.ptype, rho, pr)
    exact = -2 * np.pi * P0 * np.cos(2 * np.pi * s.x[0]) / rho
    assert np.abs(a[0] - exact).max() < tol * np.abs(exact).max()
    assert np.abs(a[1]).max() < 1e-9 * np.abs(exact).max()


@pytest.mark.parametrize("n_side,tol", [(32, 1e-2), (64, 3e-3)])
def test_viscous_term_independent_of_density(n_side, tol):
    """At rho0 = 1000 the viscous term is still nu Laplacian(u): the
    4 nu/(rho_i + rho_j) prefactor of eq. mom:sph:visc cancels the density
    carried by m_j."""
    p, s = _dense(*W.taylor_green(n_side), 1000.0)
    u = np.zeros_like(s.x)
    u[0] = np.sin(2 * np.pi * s.x[1])
    rho = oracle.density(p, s.x, s.m)
    a = oracle.momentum(p, s.x, u, s.m, s.ptype, rho, np.zeros(s.n))
    exact = -p.nu * (2 * np.pi) ** 2 * u[0]
    assert np.abs(a[0] - exact).max() < tol * np.abs(exact).max()


def _pair(rho, pr, u_i=(0.0, 0.0), nu=0.0, m_j=2.0):
    """Two particles of a cubic-spline run with h = 1: i at the origin, j at
    (1, 0) (q = 1), unit mass for i and m_j for j; rho, pr and the velocity
    of i given; j at rest; no gravity."""
    p = W.Params(dim=2, kernel=W.CUBIC, h=1.0, rho0=1.0, c0=1.0, nu=nu, eta=0.01, dt=1e-3,
                 g=(0.0, 0.0, 0.0), lo=(-10.0, -10.0, 0.0), hi=(10.0, 10.0, 0.0),
                 periodic=(0, 0, 0))
    x = np.array([[0.0, 1.0], [0.0, 0.0]])
    v = np.array([[u_i[0], 0.0], [u_i[1], 0.0]])
    m = np.array([1.0, m_j])
    a = oracle.momentum(p, x, v, m, np.zeros(2, np.uint8), np.asarray(rho, float),
                        np.asarray(pr, float))
    return a[:, 0]


def test_pressure_pair_closed_form():
    """Worked two-particle example of eq. mom:sph:press, by hand: at q = 1 the
    M4 spline has dW/dr = sigma (-3 + 2.25) / h = -0.75 * 10/(7 pi), and
    r_ij = x_i - x_j = (-1, 0), so grad_i W_ij = (0.75 * 10/(7 pi), 0).  With
    p_i = 3, rho_i = 1.5 (P_i = 4/3), p_j = 1, rho_j = 0.5 (P_j = 4), m_j = 2:
    a_i = -m_j (P_i + P_j) grad_i W_ij = (-80/(7 pi), 0), pointing away from j."""
    a = _pair([1.5, 0.5], [3.0, 1.0])
    assert a[0] == pytest.approx(-80.0 / (7.0 * np.pi), rel=1e-14)
    assert a[1] == 0.0


def test_pressure_pair_density_weights():
    """P = p / rho^2: doubling rho_i divides the force of p_i by exactly 4
    and leaves that of p_j alone; doubling rho_j does the converse."""
    base = _pair([1.5, 0.5], [3.0, 0.0])[0]
    assert _pair([3.0, 0.5], [3.0, 0.0])[0] == pytest.approx(base / 4.0, rel=1e-14)
    assert _pair([1.5, 1.0], [3.0, 0.0])[0] == pytest.approx(base, rel=1e-14)
    other = _pair([1.5, 0.5], [0.0, 1.0])[0]
    assert _pair([1.5, 1.0], [0.0, 1.0])[0] == pytest.approx(other / 4.0, rel=1e-14)
    assert _pair([3.0, 0.5], [0.0, 1.0])[0] == pytest.approx(other, rel=1e-14)
    # the two contributions add
    assert _pair([1.5, 0.5], [3.0, 1.0])[0] == pytest.approx(base + other, rel=1e-14)


def test_viscous_pair_closed_form_and_density_sum():
    """Worked two-particle example of eq. mom:sph:visc, by hand: p = 0, i moves
    with u_i = (1, 0) towards j at rest, nu = 0.1, eta = 0.01,
    h = 1, |r| = 1: r_ij . grad_i W_ij = dW/dr |r| = -0.75 * 10/(7 pi), so
    a_i = m_j 4 nu/(rho_i + rho_j) (-0.75 * 10/(7 pi))/(1 + 0.01) v_ij, a drag
    against the relative velocity.  The prefactor depends on rho_i + rho_j
    only: (1, 3), (3, 1) and (2, 2) give the same force."""
    dwdr = -0.75 * 10.0 / (7.0 * np.pi)
    expect = 2.0 * 4.0 * 0.1 / 4.0 * dwdr / 1.01
    for rho in ([1.0, 3.0], [3.0, 1.0], [2.0, 2.0]):
        a = _pair(rho, [0.0, 0.0], u_i=(1.0, 0.0), nu=0.1)
        assert a[0] == pytest.approx(expect, rel=1e-14), rho
        assert a[1] == 0.0
    # a transverse relative velocity gives a transverse drag of the same size
    a = _pair([1.0, 3.0], [0.0, 0.0], u_i=(0.0, 1.0), nu=0.1)
    assert a[0] == 0.0
    assert a[1] == pytest.approx(expect, rel=1e-14)
