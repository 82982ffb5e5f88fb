"""GPU tests of the LDS-tiled 3D mixed-precision passes (sph_params.pair_tiles).

The tiled list build + density, the tiled momentum and their fallback kernels
must give bitwise the fields of the global-list passes (same arithmetic, same
neighbour order), whatever the tile geometry: boxes whose union wraps a
periodic grid onto itself, partial boxes at the grid's edge, boxes whose
union exceeds the staging capacity (every target left to the fallback), and
targets with more neighbours than the list capacity.  The interaction counts
are equal; the diagnostics (summed in another order) agree to 1e-13."""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_04504_amd as sph
import sph_workloads as W
from helpers import NEAR_TIE, drop_near_ties, normwise, order_by_id, shuffled

pytestmark = pytest.mark.gpu

MIXED = sph.FP32_MIXED
ON = 3072          # pair_tiles: tiles wherever they apply, full staging capacity
FIELDS = ("x", "u", "a", "rho", "p", "id")


def case(name):
    if name == "cube_cd1":      # 4 cells per axis: every union wraps onto itself
        return W.periodic_cube(n_side=14, jitter=0.3, sigma_u=0.1, seed=13)
    if name == "cube_cd2":      # 9 cells per axis, boxes of 6 x 6 x 4
        return W.periodic_cube(n_side=14, jitter=0.3, sigma_u=0.1, seed=14, cell_div=2)
    if name == "cube32_cd2":    # 21 cells per axis: partial boxes at the edge
        return W.periodic_cube(n_side=32, jitter=0.2, sigma_u=0.1, seed=21, cell_div=2)
    if name == "quintic_cd1":   # support 3h
        p, s = W.periodic_cube(n_side=16, jitter=0.3, sigma_u=0.1, seed=18, hdx=1.0)
        return p.replace(kernel=W.QUINTIC), s
    if name in ("dam_cd1", "dam_cd2"):
        p, s = W.dam_break_3d(dx=0.04, cell_div=1 if name == "dam_cd1" else 2)
        rng = np.random.default_rng(15)
        s.u[:, s.ptype == 0] = rng.normal(0, 0.3, size=(3, int((s.ptype == 0).sum())))
        return p, s
    raise KeyError(name)


CASES = ["cube_cd1", "cube_cd2", "cube32_cd2", "quintic_cd1", "dam_cd1", "dam_cd2"]


def run_steps(p, s, tiles, nsteps, cap=0):
    """tiles: sph_params.pair_tiles."""
    prm = sph.make_params(p, MIXED, cap, pair_tiles=tiles)
    dp = sph.DeviceParticles.from_state(s, MIXED)
    ws = sph.workspace(prm, s.n)
    diag = torch.zeros((max(nsteps, 1), 4), dtype=torch.float64, device="cuda")
    sph.read_interactions(ws, reset=True)
    sph.step(prm, dp, nsteps, ws, prime=True, diag=diag if nsteps else None)
    sph.check(ws)
    inter = sph.read_interactions(ws, reset=True)
    return dp.numpy(), inter, diag.cpu().numpy()


def assert_same(a, b):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("name", CASES)
def test_tiles_bitwise_equal_to_global_lists(name):
    """Three steps with tiles (forced on), without (global lists) and with a
    staging capacity below every union (all targets on the fallback)."""
    p, s = case(name)
    s = shuffled(s, 3)
    ref, inter_ref, diag_ref = run_steps(p, s, -1, 3)
    for tiles in (ON, 64):
        out, inter, diag = run_steps(p, s, tiles, 3)
        assert_same(out, ref)
        assert inter == inter_ref
        assert np.abs(diag / diag_ref - 1)[:, 0].max() < 1e-13
        assert np.abs(diag - diag_ref)[:, 1:].max() <= 1e-13 * np.abs(diag_ref[:, 0]).max()


@pytest.mark.parametrize("name", ["cube_cd2", "dam_cd2"])
def test_tiles_partial_overflow_and_list_capacity(name):
    """A staging capacity near the median union (some boxes staged, some on
    the fallback) and a list capacity that leaves about half the targets to
    the fallback give the global-list fields."""
    p, s = case(name)
    ref, inter_ref, _ = run_steps(p, s, -1, 2)
    ro, _ = oracle.neighbors(p, s.x, brute=False)
    cnt = np.diff(ro)
    split = int(np.median(cnt)) & ~7
    for tiles, cap in ((900, 0), (ON, split), (900, split)):
        out, inter, _ = run_steps(p, s, tiles, 2, cap)
        assert_same(out, ref)
        assert inter == inter_ref


@pytest.mark.parametrize("name", ["cube_cd2", "dam_cd1", "dam_cd2"])
def test_tiled_standalone_calls(name):
    """sph_density (no EOS) and sph_momentum on a sorted state: tiles against
    global lists, bitwise, then against the oracle."""
    p, s = case(name)
    s = drop_near_ties(p, s, NEAR_TIE[MIXED])
    outs = []
    for tiles in (-1, ON):
        prm = sph.make_params(p, MIXED, 0, pair_tiles=tiles)
        dp = sph.DeviceParticles.from_state(shuffled(s, 4), MIXED)
        ws = sph.workspace(prm, s.n)
        cs, ce = sph.cell_arrays(prm)
        sph.bin_sort(prm, dp, ws, cs, ce)
        sph.density(prm, dp, cs, ce, ws)
        sph.eos(prm, dp)
        sph.momentum(prm, dp, cs, ce, ws)
        sph.check(ws)
        outs.append(dp.numpy())
    assert_same(outs[1], outs[0])
    out = outs[1]
    rho, _, a = oracle.evaluate(p, out["x"], out["u"], out["m"], out["type"])
    assert normwise(out["rho"], rho) < 1e-5
    assert normwise(out["a"], a) < 1e-4


def test_tiles_with_particle_outside_box():
    """A fluid particle clamped into an edge cell from outside the
    non-periodic box walks whole rows (no clipping): same fields as the
    global lists, and sph_check reports it."""
    p, s = case("dam_cd2")
    x = s.x.copy()
    fl = np.where(s.ptype == 0)[0]
    # move two fluid particles next to each other beyond the box's lower x
    # face, inside the support of each other and of the wall
    x[:, fl[0]] = (p.lo[0] - 0.3 * p.h, x[1, fl[0]], x[2, fl[0]])
    x[:, fl[1]] = (p.lo[0] - 0.9 * p.h, x[1, fl[0]] + 0.2 * p.h, x[2, fl[0]])
    s = W.State(x, s.u, s.m, s.ptype, s.pid)
    outs = []
    for tiles in (-1, ON):
        prm = sph.make_params(p, MIXED, 0, pair_tiles=tiles)
        dp = sph.DeviceParticles.from_state(s, MIXED)
        ws = sph.workspace(prm, s.n)
        sph.step(prm, dp, 0, ws, prime=True)
        with pytest.raises(sph.SphError) as ei:
            sph.check(ws)
        assert ei.value.code == sph.SPH_EDOMAIN
        outs.append(dp.numpy())
    for f in ("a", "rho", "p", "id"):
        assert np.array_equal(outs[1][f], outs[0][f]), f


def test_tiled_rollout_gradient_equal():
    """The adjoint recomputes its steps through the tiled passes and rebuilds
    global lists for its own pair passes: the rollout gradient is bitwise
    that of the untiled run.  The kinetic energy comes from the diagnostics,
    whose per-tile partial sums add in another order than the per-block
    ones: equal to 1e-13."""
    from paper_1909_04504_amd.autograd import rollout_ke
    p, s = case("cube_cd2")
    res = []
    for tiles in (-1, ON):
        pp = p
        u0 = torch.tensor(s.u, dtype=torch.float64, device="cuda", requires_grad=True)
        nu = torch.tensor(pp.nu, dtype=torch.float64, requires_grad=True)
        ke = rollout_ke(u0, nu, pp, s.x, s.m, s.ptype, 6, 3, MIXED, pair_tiles=tiles)
        ke.backward()
        res.append((float(ke.detach()), u0.grad.cpu().numpy(), float(nu.grad)))
    assert res[0][0] == pytest.approx(res[1][0], rel=1e-13)
    assert np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]


def test_cube_full_size_tiles_sampled():
    """The 256^3 cube of the benchmark: the tiled priming evaluation against
    the oracle on 1,500 sampled particles."""
    wl = W.workload("cube256")
    p, s = wl.params, wl.state
    prm = sph.make_params(p, MIXED)
    dp = sph.DeviceParticles.from_state(s, MIXED)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    sph.check(ws)
    ids = dp.id.cpu().numpy()
    sub = W.random_subset(s.n, 1500, seed=9)
    slot = np.empty(s.n, np.int64)
    slot[ids] = np.arange(s.n)
    sl = slot[sub]
    rho_g = dp.rho.cpu().numpy()[sl]
    a_g = dp.a.cpu().numpy()[:, sl]
    del dp, ws
    torch.cuda.empty_cache()
    rho, _, a = oracle.eval_subset(p, s.x, s.u, s.m, s.ptype, sub)
    assert normwise(rho_g, rho) < 1e-5
    assert normwise(a_g, a) < 1e-4


def test_default_uses_tiles_on_dense_grids_only():
    """pair_tiles = 0 takes the tiles on a grid with at least one particle
    per cell on average (the periodic cube) and the global lists on a
    sparser one (the dam break's tank)."""
    for name, tiled in (("cube_cd2", True), ("dam_cd2", False)):
        p, s = case(name)
        prm = sph.make_params(p, MIXED)
        dp = sph.DeviceParticles.from_state(s, MIXED)
        ws = sph.workspace(prm, s.n)
        sph.timer_read(reset=True)
        sph.timer_enable(True)
        sph.step(prm, dp, 1, ws, prime=True)
        torch.cuda.synchronize()
        sph.timer_enable(False)
        used = {k for k, (ms, c) in sph.timer_read(reset=True).items() if c > 0}
        assert ("tile_build" in used) == tiled, (name, used)
        assert ("nlist" in used) == (not tiled), (name, used)
