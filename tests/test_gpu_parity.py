"""GPU parity: every C-ABI entry point of the gfx950 library against the FP64
CPU oracle on the same seeded inputs.

Bars: bit-exact for the sort, the permutation, the cell ranges and the
neighbour sets; FP64 fields within 1e-12 normwise (max |gpu - ref| / max |ref|
per component); mixed precision within 1e-5 for density and 1e-4 for
acceleration.  Fixtures for set comparisons drop particles that have a
neighbour within a relative 2e-7 of the support radius in mixed precision
(where positions are quantised to cs / 2^27) and none in FP64; fixtures with
many pairs inside the +-1e-5 band of the FP32 filters, and dyadic lattices
with exact ties at the support radius, check the exact FP64 decision."""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_04504_amd as sph
import sph_workloads as W
from helpers import (NEAR_TIE, drop_near_ties, normwise, order_by_id, shuffled,
                     support_radius, with_near_ties)

pytestmark = pytest.mark.gpu

PRECS = [sph.FP64, sph.FP32_MIXED]
TOL_RHO = {sph.FP64: 1e-12, sph.FP32_MIXED: 1e-5}
TOL_ACC = {sph.FP64: 1e-12, sph.FP32_MIXED: 1e-4}


def make_case(name):
    if name == "tg2d":
        return W.taylor_green(50, jitter=0.3, seed=11)
    if name == "tg2d_cd2":
        return W.taylor_green(50, jitter=0.3, seed=12, cell_div=2)
    if name == "cube3d":
        return W.periodic_cube(n_side=14, jitter=0.3, sigma_u=0.1, seed=13)
    if name == "cube3d_cd2":
        return W.periodic_cube(n_side=14, jitter=0.3, sigma_u=0.1, seed=14, cell_div=2)
    if name == "dam3d":
        p, s = W.dam_break_3d(dx=0.04)
        rng = np.random.default_rng(15)
        s.u[:, s.ptype == 0] = rng.normal(0, 0.3, size=(3, int((s.ptype == 0).sum())))
        return p, s
    if name == "tg2d_quintic":
        return W.taylor_green(50, jitter=0.3, seed=17, kernel=W.QUINTIC, hdx=1.0)
    if name == "cube3d_quintic":
        p, s = W.periodic_cube(n_side=16, jitter=0.3, sigma_u=0.1, seed=18, hdx=1.0)
        return p.replace(kernel=W.QUINTIC), s
    if name == "tg2d_wide":
        # cells of 4 dx: about 16 targets and 144 candidates per cell, so the
        # 2D cooperative build takes each cell's candidates in several
        # passes of 64
        return W.taylor_green(40, jitter=0.3, seed=20, hdx=2.0)
    if name == "tg2d_dense":
        # cells of 6 dx: about 36 targets and 324 candidates per cell
        return W.taylor_green(30, jitter=0.3, seed=21, hdx=3.0)
    if name == "sparse2d":
        # a small jittered patch in a large non-periodic box: more cells than
        # particles, so the list build takes its cells from the sorted slots
        p, s = W.taylor_green(30, jitter=0.3, seed=19)
        p = p.replace(periodic=(0, 0, 0), lo=(-2.0, -2.0, 0), hi=(3.0, 3.0, 0))
        return p, s
    if name == "box2d":
        # non-periodic 2D box with gravity, cubic spline
        p, s = W.taylor_green(40, jitter=0.3, seed=16)
        p = p.replace(periodic=(0, 0, 0), lo=(-0.05, -0.05, 0), hi=(1.05, 1.05, 0),
                      g=(0.0, -9.81, 0.0))
        s.ptype[: s.n // 10] = W.WALL
        s.u[:, : s.n // 10] = 0
        return p, s
    raise KeyError(name)


CASES = ["tg2d", "tg2d_cd2", "cube3d", "cube3d_cd2", "dam3d", "box2d", "tg2d_quintic",
         "cube3d_quintic", "sparse2d", "tg2d_wide", "tg2d_dense"]


def gpu_sorted(p, s, prec):
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(s, prec)
    ws = sph.workspace(prm, s.n)
    cs, ce = sph.cell_arrays(prm)
    sph.bin_sort(prm, dp, ws, cs, ce)
    return prm, dp, ws, cs, ce


@pytest.mark.parametrize("case", CASES)
def test_bin_sort_bit_exact(case):
    p, s = make_case(case)
    s = shuffled(s, seed=1)
    keys, perm, cs_ref, ce_ref = oracle.bin_sort(p, s.x)
    for prec in PRECS:
        prm, dp, ws, cs, ce = gpu_sorted(p, s, prec)
        out = dp.numpy()
        assert np.array_equal(out["id"], s.pid[perm])
        assert np.array_equal(out["x"], s.x[:, perm])
        assert np.array_equal(out["u"], s.u[:, perm])
        assert np.array_equal(out["m"], s.m[perm])
        assert np.array_equal(out["type"], s.ptype[perm])
        assert np.array_equal(cs.cpu().numpy().view(np.uint32), cs_ref)
        assert np.array_equal(ce.cpu().numpy().view(np.uint32), ce_ref)
        sph.check(ws)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_neighbor_sets_bit_exact(case, prec):
    p, s = make_case(case)
    s = drop_near_ties(p, s, NEAR_TIE[prec])
    s = shuffled(s, seed=2)
    prm, dp, ws, cs, ce = gpu_sorted(p, s, prec)
    n = s.n
    offsets = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(sph.SphError) as ei:
        sph.neighbors(prm, dp, cs, ce, 0, offsets, None, ws)
    assert ei.value.code == sph.SPH_ECAPACITY
    total = ei.value.total
    nbr = torch.zeros(total, dtype=torch.int32, device="cuda")
    assert sph.neighbors(prm, dp, cs, ce, total, offsets, nbr, ws) == total
    off = offsets.cpu().numpy()
    idx = nbr.cpu().numpy()
    ids = dp.id.cpu().numpy()
    xs = dp.x.cpu().numpy()
    ro, ri = oracle.neighbors(p, xs, brute=s.n <= 4096)
    assert np.array_equal(off, ro)
    for i in range(n):
        got = np.sort(idx[off[i]:off[i + 1]])
        assert np.array_equal(got, ri[ro[i]:ro[i + 1]]), f"row {i} (id {ids[i]})"


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_density_eos_momentum_parity(case, prec):
    """Standalone density, EOS and momentum calls on a sorted state."""
    p, s = make_case(case)
    s = drop_near_ties(p, s, NEAR_TIE[prec])
    s = shuffled(s, seed=3)
    prm, dp, ws, cs, ce = gpu_sorted(p, s, prec)
    sph.density(prm, dp, cs, ce, ws)
    sph.eos(prm, dp)
    sph.momentum(prm, dp, cs, ce, ws)
    out = dp.numpy()
    rho, pr, a = oracle.evaluate(p, out["x"], out["u"], out["m"], out["type"])
    assert normwise(out["rho"], rho) < TOL_RHO[prec]
    # p is a difference of nearly equal terms: its error is measured against
    # the pressure scale B = rho0 c0^2 / 7
    B = p.rho0 * p.c0 ** 2 / 7
    assert np.abs(out["p"] - pr).max() / B < 7 * TOL_RHO[prec] * 4
    assert normwise(out["a"], a) < TOL_ACC[prec]
    sph.check(ws)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_step_prime_evaluation(case, prec):
    """sph_step with prime and zero steps: the fused density+EOS and momentum
    kernels at the input state, particles left sorted."""
    p, s = make_case(case)
    s = drop_near_ties(p, s, NEAR_TIE[prec])
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(shuffled(s, 4), prec)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    out = dp.numpy()
    rho, pr, a = oracle.evaluate(p, out["x"], out["u"], out["m"], out["type"])
    assert normwise(out["rho"], rho) < TOL_RHO[prec]
    assert normwise(out["a"], a) < TOL_ACC[prec]
    keys = oracle.cell_keys(p, out["x"])
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)


def test_taylor_green_64_trajectory_fp64():
    """50 FP64 predictor-corrector steps of the 64x64 Taylor-Green vortex,
    matched by id: positions, velocities, density, pressure and diagnostics
    within 1e-12 of the oracle.  The acceleration is ill-conditioned in the
    positions (a one-ulp change of x moves it by ~1e-12 relative), so its
    bar is the oracle's own spread under a one-ulp perturbation of x0, and
    never looser than 1e-11."""
    wl = W.workload("tg64")
    p, s = wl.params, wl.state
    ref = oracle.step(p, s.x, s.u, s.m, s.ptype, wl.steps, want_diag=True)
    ref_ulp = oracle.step(p, np.nextafter(s.x, 2.0), s.u, s.m, s.ptype, wl.steps)
    spread = normwise(ref_ulp["a"], ref["a"])
    prm = sph.make_params(p, sph.FP64)
    dp = sph.DeviceParticles.from_state(s, sph.FP64)
    ws = sph.workspace(prm, s.n)
    diag = torch.zeros((wl.steps, 3), dtype=torch.float64, device="cuda")
    sph.step(prm, dp, wl.steps, ws, prime=True, diag=diag)
    out = dp.numpy()
    o = order_by_id(out["id"])
    dx = out["x"][:, o] - ref["x"]
    dx -= np.round(dx)
    assert np.abs(dx).max() < 1e-12
    assert normwise(out["u"][:, o], ref["u"]) < 1e-12
    err_a = normwise(out["a"][:, o], ref["a"])
    assert err_a < max(1e-12, min(1e-11, 4 * spread)), (err_a, spread)
    assert normwise(out["rho"][o], ref["rho"]) < 1e-12
    # pressure against its scale B = rho0 c0^2 / 7 (the EOS amplifies density
    # rounding by 7 B / rho0)
    B = p.rho0 * p.c0 ** 2 / 7
    assert np.abs(out["p"][o] - ref["p"]).max() / B < 1e-12
    d = diag.cpu().numpy()
    assert np.abs(d[:, 0] / ref["diag"][:, 0] - 1).max() < 1e-12
    assert np.abs(d[:, 1:] - ref["diag"][:, 1:]).max() < 1e-12 * 0.25
    sph.check(ws)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_neighbour_list_capacity_paths(case, prec):
    """The pair passes read each particle's neighbours from its list when it
    fits the capacity and walk the cells otherwise: lists everywhere (default
    capacity), walks everywhere (no lists) and a capacity that splits the
    particles between the two give the same fields, and match the oracle."""
    p, s = make_case(case)
    s = drop_near_ties(p, s, NEAR_TIE[prec])
    s = shuffled(s, 5)
    ro, _ = oracle.neighbors(p, s.x, brute=False)
    counts = np.diff(ro)
    split = int(np.median(counts))  # about half the particles above it
    outs = []
    for cap in (0, -1, split):
        prm = sph.make_params(p, prec, cap)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, s.n)
        sph.step(prm, dp, 2, ws, prime=True)
        sph.check(ws)
        outs.append(dp.numpy())
    ref = outs[0]
    for o in outs[1:]:
        for f in ("x", "u", "a", "rho", "p", "id"):
            assert np.array_equal(o[f], ref[f]), f
    # one more evaluation at the final state against the oracle
    rho, _, a = oracle.evaluate(p, ref["x"], ref["u"], ref["m"], ref["type"])
    prm = sph.make_params(p, prec, split)
    dp = sph.DeviceParticles.from_state(W.State(ref["x"], ref["u"], ref["m"], ref["type"],
                                                ref["id"]), prec)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    out = dp.numpy()
    o = order_by_id(out["id"])
    r = order_by_id(ref["id"])
    assert normwise(out["rho"][o], rho[r]) < TOL_RHO[prec]
    assert normwise(out["a"][:, o], a[:, r]) < TOL_ACC[prec]


@pytest.mark.parametrize("case", ["tg2d", "cube3d", "dam3d"])
def test_mixed_precision_few_steps(case):
    p, s = make_case(case)
    nsteps = 5
    ref = oracle.step(p, s.x, s.u, s.m, s.ptype, nsteps)
    prm = sph.make_params(p, sph.FP32_MIXED)
    dp = sph.DeviceParticles.from_state(s, sph.FP32_MIXED)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, nsteps, ws, prime=True)
    out = dp.numpy()
    o = order_by_id(out["id"])
    assert normwise(out["rho"][o], ref["rho"]) < 1e-5
    assert normwise(out["a"][:, o], ref["a"]) < 1e-4
    assert normwise(out["u"][:, o], ref["u"]) < 1e-5


@pytest.mark.parametrize("prec", PRECS)
def test_bitwise_deterministic(prec):
    p, s = make_case("cube3d")
    outs = []
    for _ in range(2):
        prm = sph.make_params(p, prec)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, s.n)
        sph.step(prm, dp, 10, ws, prime=True)
        outs.append(dp.numpy())
    for f in outs[0]:
        assert np.array_equal(outs[0][f], outs[1][f]), f


def test_check_reports_nonfinite_and_outside():
    p, s = make_case("box2d")
    s.x[0, 5] = np.nan
    prm = sph.make_params(p, sph.FP64)
    dp = sph.DeviceParticles.from_state(s, sph.FP64)
    ws = sph.workspace(prm, s.n)
    cs, ce = sph.cell_arrays(prm)
    sph.bin_sort(prm, dp, ws, cs, ce)
    with pytest.raises(sph.SphError) as ei:
        sph.check(ws)
    assert ei.value.code == sph.SPH_ENONFINITE
    sph.check(ws)  # cleared
    p2, s2 = make_case("box2d")
    s2.x[1, 7] = 2.0  # above hi = 1.05 on a non-periodic axis
    dp2 = sph.DeviceParticles.from_state(s2, sph.FP64)
    sph.bin_sort(prm, dp2, ws, cs, ce)
    with pytest.raises(sph.SphError) as ei:
        sph.check(ws)
    assert ei.value.code == sph.SPH_EDOMAIN


def test_single_particle_and_one_cell():
    """Degenerate inputs: one particle (rho = m W(0), a = g); every particle
    inside one cell."""
    p = W.Params(dim=2, kernel=W.CUBIC, h=0.1, rho0=1.0, c0=10.0, nu=0.01, eta=0.01, dt=1e-3,
                 g=(0.0, -1.0, 0.0), lo=(0, 0, 0), hi=(1, 1, 0), periodic=(0, 0, 0))
    s = W.State(np.array([[0.5], [0.5]]), np.zeros((2, 1)), np.array([0.01]),
                np.zeros(1, np.uint8), np.zeros(1, np.int32))
    for prec in PRECS:
        prm = sph.make_params(p, prec)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, 1)
        sph.step(prm, dp, 0, ws, prime=True)
        out = dp.numpy()
        rho, _, a = oracle.evaluate(p, s.x, s.u, s.m, s.ptype)
        assert normwise(out["rho"], rho) < TOL_RHO[prec]
        assert np.array_equal(out["a"][:, 0].astype(np.float64), np.array([0.0, -1.0]))
    rng = np.random.default_rng(5)
    n = 300
    x = 0.5 + rng.uniform(-0.04, 0.04, size=(2, n))
    s = W.State(x, rng.normal(0, 0.1, (2, n)), np.full(n, 1e-4), np.zeros(n, np.uint8),
                np.arange(n, dtype=np.int32))
    for prec in PRECS:
        prm = sph.make_params(p, prec)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, n)
        sph.step(prm, dp, 0, ws, prime=True)
        out = dp.numpy()
        rho, _, a = oracle.evaluate(p, out["x"], out["u"], out["m"], out["type"])
        assert normwise(out["rho"], rho) < TOL_RHO[prec]
        assert normwise(out["a"], a) < TOL_ACC[prec]


def gpu_neighbour_sets(p, s, prec):
    """sph_bin_sort + sph_neighbors; returns the sorted state and CSR lists."""
    prm, dp, ws, cs, ce = gpu_sorted(p, s, prec)
    n = s.n
    offsets = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(sph.SphError) as ei:
        sph.neighbors(prm, dp, cs, ce, 0, offsets, None, ws)
    total = ei.value.total
    nbr = torch.zeros(max(total, 1), dtype=torch.int32, device="cuda")
    assert sph.neighbors(prm, dp, cs, ce, total, offsets, nbr, ws) == total
    sph.check(ws)
    return dp.numpy(), offsets.cpu().numpy(), nbr.cpu().numpy()


def assert_sets_equal(p, out, off, idx):
    ro, ri = oracle.neighbors(p, out["x"], brute=out["x"].shape[1] <= 4096)
    assert np.array_equal(off, ro)
    for i in range(len(off) - 1):
        got = np.sort(idx[off[i]:off[i + 1]])
        assert np.array_equal(got, ri[ro[i]:ro[i + 1]]), f"row {i} (id {out['id'][i]})"
    return ro


def step_interactions(p, s, prec, cap):
    """Sum_i |N(i)| counted by the list build (or, without lists, the density
    walk) of one sph_step evaluation."""
    prm = sph.make_params(p, prec, cap)
    dp = sph.DeviceParticles.from_state(s, prec)
    ws = sph.workspace(prm, s.n)
    sph.read_interactions(ws, reset=True)
    sph.step(prm, dp, 0, ws, prime=True)
    sph.check(ws)
    return sph.read_interactions(ws, reset=True), dp.numpy()


BAND_CASES = ["tg2d", "tg2d_cd2", "cube3d", "cube3d_cd2", "tg2d_quintic", "sparse2d", "box2d",
              "tg2d_wide", "tg2d_dense"]


@pytest.mark.parametrize("case", BAND_CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_near_tie_band_decided_exactly(case, prec):
    """Companion particles at |r|^2 = R^2 (1 +- e), e in [5e-7, 1e-5] (mixed)
    or [1e-12, 1e-5] (FP64): every such pair lies inside the band where the
    FP32 filters of the cell walk and of the list build defer to the FP64
    predicate.  The neighbour sets (sph_neighbors) match brute force exactly,
    and so do the interaction counts of the step's list build and of the
    list-free walk; fields match the oracle."""
    p, s = make_case(case)
    lo = 5e-7 if prec == sph.FP32_MIXED else 1e-12
    s = with_near_ties(p, s, min(400, s.n // 4), lo, 1e-5, seed=21)
    s = drop_near_ties(p, s, NEAR_TIE[prec])
    s = shuffled(s, seed=6)
    # the fixture really holds band pairs
    ro, ri = oracle.neighbors(p, s.x, brute=s.n <= 4096)
    out, off, idx = gpu_neighbour_sets(p, s, prec)
    assert_sets_equal(p, out, off, idx)
    total = int(ro[-1])
    for cap in (0, -1):
        inter, st = step_interactions(p, s, prec, cap)
        assert inter == total, (cap, inter, total)
    rho, _, a = oracle.evaluate(p, st["x"], st["u"], st["m"], st["type"])
    assert normwise(st["rho"], rho) < TOL_RHO[prec]
    assert normwise(st["a"], a) < TOL_ACC[prec]


@pytest.mark.parametrize("dim,cell_div", [(2, 1), (2, 2), (3, 1), (3, 2)])
@pytest.mark.parametrize("prec", PRECS)
def test_exact_ties_on_dyadic_lattice(dim, cell_div, prec):
    """A lattice of spacing dx = 1/64 (2D) or 1/16 (3D) with h = dx: every
    lattice neighbour at distance 2dx = R sits exactly on the support radius,
    and |r|^2 = R^2 is exact in binary.  The predicate is strict, so each
    particle has exactly 9 (2D) or 27 (3D) neighbours, self included: the
    sets of sph_neighbors and the counts of the step's list build and of the
    list-free walk."""
    if dim == 2:
        p, s = W.taylor_green(64, hdx=1.0, cell_div=cell_div)
        K = 9
    else:
        p, s = W.periodic_cube(n_side=16, jitter=0.0, sigma_u=0.1, hdx=1.0, cell_div=cell_div)
        K = 27
    # Fields well conditioned for the 1e-12 bar: on a perfect lattice the
    # pressure terms of a particle cancel exactly in exact arithmetic, so with
    # the lattice density off rho0 (a background pressure) its acceleration
    # is a few ulps of the summed terms, and a smooth velocity field makes the
    # viscous sum a second difference.  Taking rho0 = the lattice density
    # (p = 0) and random velocities leaves sums without cancellation.  Pairs
    # at exactly r = R add W = 0 and grad W = 0, so the fields never see the
    # ties: the neighbour sets and counts below are what this test checks.
    p = p.replace(rho0=float(oracle.density(p, s.x, s.m).mean()))
    s.u = np.random.default_rng(9).normal(0.0, 0.1, s.u.shape)
    s = shuffled(s, seed=7)
    out, off, idx = gpu_neighbour_sets(p, s, prec)
    assert np.all(np.diff(off) == K)
    assert_sets_equal(p, out, off, idx)
    for cap in (0, -1):
        inter, st = step_interactions(p, s, prec, cap)
        assert inter == K * s.n, (cap, inter)
    rho, _, a = oracle.evaluate(p, st["x"], st["u"], st["m"], st["type"])
    assert normwise(st["rho"], rho) < TOL_RHO[prec]
    assert normwise(st["a"], a) < TOL_ACC[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_clamped_particle_lists_match_walks_2d(prec):
    """Particles outside a non-periodic 2D box are clamped into edge cells;
    the cell-cooperative list build (whose FP32 filter hands records far from
    the cell to the exact test) gives the fields of the cell walks, and
    sph_check reports the particles."""
    p, s = make_case("box2d")
    x = s.x.copy()
    fl = np.where(s.ptype == 0)[0]
    R = support_radius(p)
    x[:, fl[0]] = (p.lo[0] - 0.2 * R, p.lo[1] + 0.5)
    x[:, fl[1]] = (p.lo[0] - 0.6 * R, p.lo[1] + 0.5 + 0.1 * R)
    x[:, fl[2]] = (p.hi[0] + 0.3 * R, p.hi[1] + 0.2 * R)
    s = W.State(x, s.u, s.m, s.ptype, s.pid)
    outs = []
    for cap in (0, -1):
        prm = sph.make_params(p, prec, cap)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, s.n)
        sph.step(prm, dp, 0, ws, prime=True)
        with pytest.raises(sph.SphError) as ei:
            sph.check(ws)
        assert ei.value.code == sph.SPH_EDOMAIN
        outs.append(dp.numpy())
    for f in ("a", "rho", "p", "id"):
        assert np.array_equal(outs[0][f], outs[1][f]), f
