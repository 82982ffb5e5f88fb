"""GPU tests of the Z-order (Morton) cell keys (sph_params.cell_order = 1,
3D): the sort is bit-exact against the oracle's stable sort on the same
keys, the neighbour sets are those of brute force, and every pass gives the
fields of the row-major keys.  A priming evaluation visits each particle's
neighbours in the same order under both keys (same cells in the same order,
the same stable order inside a cell), so its fields are bitwise those of the
row-major run; later steps sort by different keys, so the order inside a
cell can differ and the fields agree to rounding."""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_04504_amd as sph
import sph_workloads as W
from helpers import NEAR_TIE, drop_near_ties, normwise, order_by_id, shuffled

pytestmark = pytest.mark.gpu

PRECS = [sph.FP64, sph.FP32_MIXED]


def case(name):
    if name == "cube_cd1":
        p, s = W.periodic_cube(n_side=14, jitter=0.3, sigma_u=0.1, seed=31)
    elif name == "cube_cd2":
        p, s = W.periodic_cube(n_side=20, jitter=0.3, sigma_u=0.1, seed=32, cell_div=2)
    elif name == "dam_cd2":
        p, s = W.dam_break_3d(dx=0.04, cell_div=2)
        rng = np.random.default_rng(33)
        s.u[:, s.ptype == 0] = rng.normal(0, 0.3, size=(3, int((s.ptype == 0).sum())))
    else:
        raise KeyError(name)
    return p.replace(cell_order=W.Z_ORDER), s


CASES = ["cube_cd1", "cube_cd2", "dam_cd2"]


@pytest.mark.parametrize("name", CASES)
def test_zorder_bin_sort_bit_exact(name):
    p, s = case(name)
    s = shuffled(s, 1)
    keys, perm, cs_ref, ce_ref = oracle.bin_sort(p, s.x)
    for prec in PRECS:
        prm = sph.make_params(p, prec)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, s.n)
        cs, ce = sph.cell_arrays(prm)
        assert cs.numel() == len(cs_ref)
        sph.bin_sort(prm, dp, ws, cs, ce)
        out = dp.numpy()
        assert np.array_equal(out["id"], s.pid[perm])
        assert np.array_equal(out["x"], s.x[:, perm])
        assert np.array_equal(cs.cpu().numpy().view(np.uint32), cs_ref)
        assert np.array_equal(ce.cpu().numpy().view(np.uint32), ce_ref)
        sph.check(ws)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_zorder_neighbour_sets(name, prec):
    p, s = case(name)
    s = drop_near_ties(p, s, NEAR_TIE[prec])
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(shuffled(s, 2), prec)
    ws = sph.workspace(prm, s.n)
    cs, ce = sph.cell_arrays(prm)
    sph.bin_sort(prm, dp, ws, cs, ce)
    offsets = torch.zeros(s.n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(sph.SphError) as ei:
        sph.neighbors(prm, dp, cs, ce, 0, offsets, None, ws)
    total = ei.value.total
    nbr = torch.zeros(total, dtype=torch.int32, device="cuda")
    sph.neighbors(prm, dp, cs, ce, total, offsets, nbr, ws)
    off, idx = offsets.cpu().numpy(), nbr.cpu().numpy()
    ro, ri = oracle.neighbors(p, dp.x.cpu().numpy(), brute=s.n <= 4096)
    assert np.array_equal(off, ro)
    for i in range(s.n):
        assert np.array_equal(np.sort(idx[off[i]:off[i + 1]]), ri[ro[i]:ro[i + 1]]), i


def _run(p, s, prec, nsteps, tiles=0, cap=0):
    prm = sph.make_params(p, prec, cap, pair_tiles=tiles)
    dp = sph.DeviceParticles.from_state(s, prec)
    ws = sph.workspace(prm, s.n)
    sph.read_interactions(ws, reset=True)
    sph.step(prm, dp, nsteps, ws, prime=True)
    sph.check(ws)
    return dp.numpy(), sph.read_interactions(ws, reset=True)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_zorder_prime_bitwise_equal_to_row_major(name, prec):
    p, s = case(name)
    z, inter_z = _run(p, s, prec, 0)
    r, inter_r = _run(p.replace(cell_order=W.ROW_MAJOR), s, prec, 0)
    assert inter_z == inter_r
    oz, orr = order_by_id(z["id"]), order_by_id(r["id"])
    for f in ("a", "rho", "p"):
        assert np.array_equal(z[f][..., oz], r[f][..., orr]), f


@pytest.mark.parametrize("name", CASES)
def test_zorder_steps_paths_and_oracle(name):
    """Mixed precision, four steps: tiles, global lists and cell walks give
    bitwise the same fields under Z-order keys; they match the row-major run
    and the oracle at the mixed-precision bars."""
    p, s = case(name)
    nsteps = 4
    outs = [_run(p, s, sph.FP32_MIXED, nsteps, tiles, cap)
            for tiles, cap in ((3072, 0), (-1, 0), (-1, -1), (64, 0))]
    ref, inter = outs[0]
    for o, i in outs[1:]:
        assert i == inter
        for f in ("x", "u", "a", "rho", "p", "id"):
            assert np.array_equal(o[f], ref[f]), f
    rm, _ = _run(p.replace(cell_order=W.ROW_MAJOR), s, sph.FP32_MIXED, nsteps)
    o1, o2 = order_by_id(ref["id"]), order_by_id(rm["id"])
    assert normwise(ref["rho"][o1], rm["rho"][o2]) < 1e-6
    assert normwise(ref["a"][:, o1], rm["a"][:, o2]) < 1e-5
    orc = oracle.step(p, s.x, s.u, s.m, s.ptype, nsteps)
    assert normwise(ref["rho"][o1], orc["rho"]) < 1e-5
    assert normwise(ref["a"][:, o1], orc["a"]) < 2e-4
