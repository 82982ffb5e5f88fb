"""GPU parity of the continuity scheme (density by the continuity equation,
EOS, momentum with gravity; the paper's 2D dam-break example) under both
integrators (the example's Euler stage and the predictor-corrector) against
the FP64 CPU oracle, compared by particle id.

Bars: FP64 state within 1e-12 normwise (max |gpu - ref| / max |ref|), with
the density's departure from rho0 (the part the scheme computes) held to the
same bar against its own scale; mixed precision within 1e-5 for density and
1e-4 for acceleration; different list capacities bitwise equal."""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_04504_amd as sph
import sph_workloads as W
from helpers import normwise, order_by_id

pytestmark = pytest.mark.gpu


def _shuffle(s: W.State, seed: int) -> W.State:
    perm = np.random.default_rng(seed).permutation(s.n)
    return W.State(s.x[:, perm].copy(), s.u[:, perm].copy(), s.m[perm].copy(),
                   s.ptype[perm].copy(), s.pid[perm].copy(), rho=s.rho[perm].copy())


INTEGRATORS = [W.EULER, W.PREDICTOR_CORRECTOR]


def _moving_dam(seed: int = 21, integrator: int = W.EULER):
    """The dam-break example with a random fluid velocity field (walls at
    rest) and a perturbed density, so that every term of the step is live
    from the first step on."""
    p, s = W.dam_break_2d(integrator=integrator)
    rng = np.random.default_rng(seed)
    f = s.ptype == W.FLUID
    s.u[:, f] = rng.normal(0.0, 0.5, size=(2, int(f.sum())))
    s.rho = s.rho * (1.0 + rng.uniform(-2e-3, 2e-3, size=s.n))
    return p, s


def _periodic_continuity(dim: int, seed: int, integrator: int):
    """Periodic jittered fluid with the continuity scheme: the Taylor-Green
    vortex in 2D, the random-velocity cube in 3D, rho0 with a perturbation."""
    if dim == 2:
        p, s = W.taylor_green(40, jitter=0.3, seed=seed)
    else:
        p, s = W.periodic_cube(n_side=12, jitter=0.3, sigma_u=0.1, seed=seed)
    p = p.replace(scheme=W.CONTINUITY, integrator=integrator)
    rng = np.random.default_rng(seed + 100)
    s.rho = p.rho0 * (1.0 + rng.uniform(-1e-3, 1e-3, size=s.n))
    return p, s


def _run(p, s, prec, nsteps, nbr_cap=0, diag=False, splits=None):
    """nsteps on the GPU (primed), in one call or in calls of the sizes in
    splits (the rates carried between calls in a and arho)."""
    prm = sph.make_params(p, prec, nbr_cap)
    dp = sph.DeviceParticles.from_state(s, prec, scheme=sph.CONTINUITY)
    ws = sph.workspace(prm, s.n)
    d = (torch.zeros((nsteps, 1 + p.dim), dtype=torch.float64, device="cuda") if diag
         else None)
    if splits is None:
        sph.step(prm, dp, nsteps, ws, prime=True, diag=d)
    else:
        assert sum(splits) == nsteps and d is None
        for k, ns in enumerate(splits):
            sph.step(prm, dp, ns, ws, prime=k == 0)
    sph.check(ws)
    out = dp.numpy()
    if diag:
        out["diag"] = d.cpu().numpy()
    out["interactions"] = sph.read_interactions(ws)
    return out


def _ref(p, s, nsteps):
    """The oracle's steps, returned in id order (the oracle keeps the input
    order; the library leaves the particles sorted by cell)."""
    if p.integrator == W.EULER:
        r = oracle.step_continuity(p, s.x, s.u, s.rho, s.m, s.ptype, nsteps)
    else:
        r = oracle.step_continuity_pc(p, s.x, s.u, s.rho, s.m, s.ptype, nsteps)
    o = order_by_id(s.pid)
    return {k: v[..., o] for k, v in r.items()}


def _compare_fp64(p, out, ref, tol=1e-12):
    o = order_by_id(out["id"])
    dx = out["x"][:, o] - ref["x"]
    for k in range(p.dim):
        if p.periodic[k]:
            L = p.hi[k] - p.lo[k]
            dx[k] -= L * np.round(dx[k] / L)
    errs = {
        "x": np.abs(dx).max() / np.abs(ref["x"]).max(),
        "u": normwise(out["u"][:, o], ref["u"]),
        "rho": normwise(out["rho"][o], ref["rho"]),
        "drho": normwise(out["rho"][o] - p.rho0, ref["rho"] - p.rho0),
        "a": normwise(out["a"][:, o], ref["a"]),
        "arho": normwise(out["arho"][o], ref["arho"]),
    }
    # p is a difference of nearly equal terms: against its scale B
    B = p.rho0 * p.c0 ** 2 / 7
    errs["p"] = np.abs(out["p"][o] - ref["p"]).max() / B
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("nsteps", [1, 100])
def test_dam_break_trajectory_fp64(nsteps, integrator):
    """The example as stated (fluid at rest, rho = rho0, gravity): nsteps
    steps, state by id within 1e-12; walls never move."""
    p, s = W.dam_break_2d(integrator=integrator)
    s = _shuffle(s, 1)
    ref = _ref(p, s, nsteps)
    out = _run(p, s, sph.FP64, nsteps)
    _compare_fp64(p, out, ref)
    o = order_by_id(out["id"])
    wall = s.ptype[order_by_id(s.pid)] == W.WALL
    x0 = s.x[:, order_by_id(s.pid)]
    assert np.array_equal(out["x"][:, o][:, wall], x0[:, wall])
    assert np.all(out["u"][:, o][:, wall] == 0.0)


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("nsteps", [1, 40])
def test_moving_dam_trajectory_fp64(nsteps, integrator):
    """Every term live (random fluid velocities, perturbed density); the
    diagnostics of each step within 1e-12; one step's interaction count is
    the oracle's sum of neighbour-set sizes (two evaluations, and so twice
    that, when the predictor-corrector is primed)."""
    p, s = _moving_dam(integrator=integrator)
    s = _shuffle(s, 2)
    ref = _ref(p, s, nsteps)
    out = _run(p, s, sph.FP64, nsteps, diag=True)
    _compare_fp64(p, out, ref)
    o = order_by_id(out["id"])
    d = out["diag"][-1]
    m = s.m[order_by_id(s.pid)]
    ke = 0.5 * (ref["u"] ** 2).sum(axis=0) @ m
    mom = ref["u"] @ m
    assert abs(d[0] / ke - 1) < 1e-12
    assert np.abs(d[1:] - mom).max() < 1e-12 * np.abs(mom).max()
    if nsteps == 1 and integrator == W.EULER:
        ro, _ = oracle.neighbors(p, s.x, brute=True)
        assert out["interactions"] == int(ro[-1])
    assert np.all(out["u"][:, o][:, s.ptype[order_by_id(s.pid)] == W.WALL] == 0.0)


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_continuity_fp64(dim, integrator):
    p, s = _periodic_continuity(dim, 31 + dim, integrator)
    s = _shuffle(s, 3)
    nsteps = 10
    ref = _ref(p, s, nsteps)
    out = _run(p, s, sph.FP64, nsteps)
    _compare_fp64(p, out, ref)


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("case", ["dam", "moving_dam", "periodic2d", "periodic3d"])
def test_continuity_mixed_precision(case, integrator):
    """FP32 pair terms, FP64 integration: density (and its departure from
    rho0) within 1e-5, acceleration within 1e-4, after a few steps."""
    if case == "dam":
        p, s = W.dam_break_2d(integrator=integrator)
    elif case == "moving_dam":
        p, s = _moving_dam(22, integrator)
    else:
        p, s = _periodic_continuity(2 if case == "periodic2d" else 3, 41, integrator)
    nsteps = 5
    ref = _ref(p, s, nsteps)
    out = _run(p, s, sph.FP32_MIXED, nsteps)
    o = order_by_id(out["id"])
    e_rho = normwise(out["rho"][o], ref["rho"])
    e_drho = normwise(out["rho"][o] - p.rho0, ref["rho"] - p.rho0)
    e_a = normwise(out["a"][:, o], ref["a"])
    print(case, f"rho {e_rho:.2e} drho {e_drho:.2e} a {e_a:.2e}", flush=True)
    assert e_rho < 1e-5
    assert e_drho < 1e-5
    assert e_a < 1e-4


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32_MIXED])
def test_continuity_list_capacity_paths(prec, integrator):
    """Lists everywhere, cell walks everywhere and a capacity that sends
    about half the particles to the walk give bitwise the same steps."""
    p, s = _moving_dam(23, integrator)
    ro, _ = oracle.neighbors(p, s.x, brute=False)
    split = int(np.median(np.diff(ro)))
    outs = [_run(p, s, prec, 6, cap) for cap in (0, -1, split)]
    for o in outs[1:]:
        for f in ("x", "u", "a", "rho", "p", "arho", "id"):
            assert np.array_equal(o[f], outs[0][f]), f
        assert o["interactions"] == outs[0]["interactions"]


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32_MIXED])
def test_continuity_calls_compose(prec, integrator):
    """Five steps in one call equal calls of 2 + 1 + 2 steps bitwise: the
    predictor-corrector carries its rates between calls in a and arho."""
    p, s = _moving_dam(25, integrator)
    one = _run(p, s, prec, 5)
    split = _run(p, s, prec, 5, splits=(2, 1, 2))
    for f in ("x", "u", "a", "rho", "p", "arho", "id"):
        assert np.array_equal(split[f], one[f]), f


@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32_MIXED])
def test_fine_dam_break_full_size(prec):
    """The benchmark workloads (dam break at dx = 0.1/32, 216,338 particles,
    a grid with more cells than particles; Euler stage in FP64,
    predictor-corrector in mixed precision) in the launch configuration the
    benchmark times: a few steps from the initial state against the oracle,
    every particle by id."""
    wl = W.workload("dambreak2d_fine" if prec == sph.FP64 else "dambreak2d_fine_pc")
    p, s = wl.params, wl.state
    rng = np.random.default_rng(24)
    f = s.ptype == W.FLUID
    s.u[:, f] = rng.normal(0.0, 0.5, size=(2, int(f.sum())))
    nsteps = 3
    ref = _ref(p, s, nsteps)
    out = _run(p, s, prec, nsteps)
    if prec == sph.FP64:
        _compare_fp64(p, out, ref)
    else:
        o = order_by_id(out["id"])
        assert normwise(out["rho"][o], ref["rho"]) < 1e-5
        assert normwise(out["rho"][o] - p.rho0, ref["rho"] - p.rho0) < 1e-5
        assert normwise(out["a"][:, o], ref["a"]) < 1e-4


def test_adjoint_rejects_continuity():
    p, s = W.dam_break_2d()
    prm = sph.make_params(p, sph.FP64)
    dp = sph.DeviceParticles.from_state(s, sph.FP64, scheme=sph.CONTINUITY)
    ws = sph.workspace(prm, s.n, adjoint_k=1)
    lam = torch.zeros(3 * 2 * s.n, dtype=torch.float64, device="cuda")
    lam2 = torch.zeros_like(lam)
    dj = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sph.SphError) as ei:
        sph.step_backward(prm, dp, 1, lam, lam2, dj, ws)
    assert ei.value.code == sph.SPH_EINVAL


@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32_MIXED])
def test_standalone_passes_with_fp64_density(prec):
    """Under the continuity scheme rho is FP64 in both precisions; the
    standalone passes read and write it so: summation density, EOS and
    momentum on a sorted state match the oracle's evaluation."""
    p, s = _moving_dam(26)
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(s, prec, scheme=sph.CONTINUITY)
    assert dp.rho.dtype == torch.float64
    ws = sph.workspace(prm, s.n)
    cs, ce = sph.cell_arrays(prm)
    sph.bin_sort(prm, dp, ws, cs, ce)
    sph.density(prm, dp, cs, ce, ws)
    sph.eos(prm, dp)
    sph.momentum(prm, dp, cs, ce, ws)
    sph.check(ws)
    out = dp.numpy()
    rho, pr, a = oracle.evaluate(p, out["x"], out["u"], out["m"], out["type"])
    tol_rho = 1e-12 if prec == sph.FP64 else 1e-5
    tol_a = 1e-12 if prec == sph.FP64 else 1e-4
    assert normwise(out["rho"], rho) < tol_rho
    B = p.rho0 * p.c0 ** 2 / 7
    assert np.abs(out["p"] - pr).max() / B < 28 * tol_rho
    assert normwise(out["a"], a) < tol_a


@pytest.mark.parametrize("integrator", INTEGRATORS)
@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32_MIXED])
def test_quintic_dam_break(prec, integrator):
    """The dam-break example with the quintic spline (support 3h, its own cell
    grid) and live velocities: 10 steps against the oracle."""
    p, s = W.dam_break_2d(kernel=W.QUINTIC, integrator=integrator)
    rng = np.random.default_rng(27)
    f = s.ptype == W.FLUID
    s.u[:, f] = rng.normal(0.0, 0.5, size=(2, int(f.sum())))
    s = _shuffle(s, 4)
    ref = _ref(p, s, 10)
    out = _run(p, s, prec, 10)
    if prec == sph.FP64:
        _compare_fp64(p, out, ref)
    else:
        o = order_by_id(out["id"])
        assert normwise(out["rho"][o] - p.rho0, ref["rho"] - p.rho0) < 1e-5
        assert normwise(out["a"][:, o], ref["a"]) < 1e-4
