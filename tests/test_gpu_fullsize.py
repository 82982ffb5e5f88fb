"""Parity at the workloads' full sizes, in the launch configuration the bench
times (sph_step), on outputs the oracle can compute: sampled particles for the
3D workloads, whole fields for one step from a shared state for the 2D one."""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_04504_amd as sph
import sph_workloads as W
from helpers import normwise, order_by_id

pytestmark = pytest.mark.gpu

TOL_RHO = {sph.FP64: 1e-12, sph.FP32_MIXED: 1e-5}
TOL_ACC = {sph.FP64: 1e-12, sph.FP32_MIXED: 1e-4}


def _sampled_prime_check(wl, prec, nsample=1500):
    p, s = wl.params, wl.state
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(s, prec)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    sph.check(ws)
    ids = dp.id.cpu().numpy()
    sub_ids = W.random_subset(s.n, nsample, seed=7)
    slot = np.empty(s.n, np.int64)
    slot[ids] = np.arange(s.n)
    sl = slot[sub_ids]
    rho_g = dp.rho.cpu().numpy()[sl].astype(np.float64)
    a_g = dp.a.cpu().numpy()[:, sl].astype(np.float64)
    del dp, ws
    torch.cuda.empty_cache()
    rho_r, _, a_r = oracle.eval_subset(p, s.x, s.u, s.m, s.ptype, sub_ids)
    return rho_g, rho_r, a_g, a_r


@pytest.mark.parametrize("prec", [sph.FP32_MIXED, sph.FP64])
def test_cube256_sampled(prec):
    wl = W.workload("cube256")
    rho_g, rho_r, a_g, a_r = _sampled_prime_check(wl, prec)
    assert normwise(rho_g, rho_r) < TOL_RHO[prec]
    assert normwise(a_g, a_r) < TOL_ACC[prec]


@pytest.mark.parametrize("prec", [sph.FP32_MIXED, sph.FP64])
def test_dambreak3d_sampled(prec):
    wl = W.workload("dambreak3d")
    rho_g, rho_r, a_g, a_r = _sampled_prime_check(wl, prec)
    assert normwise(rho_g, rho_r) < TOL_RHO[prec]
    assert normwise(a_g, a_r) < TOL_ACC[prec]


@pytest.mark.parametrize("prec", [sph.FP32_MIXED, sph.FP64])
def test_tg512_one_step_parity_along_trajectory(prec):
    """Every 100 steps of the 512x512 workload, one step from the GPU's state
    on both sides (whole fields, by id).  The long trajectory itself is
    chaotic at roundoff and is not compared."""
    wl = W.workload("tg512")
    p, s = wl.params, wl.state
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(s, prec)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    for block in range(3):
        if block:
            sph.step(prm, dp, 100, ws, prime=False)
        st = dp.numpy()
        ref = oracle.step(p, st["x"], st["u"], st["m"], st["type"], 1,
                          a=st["a"].astype(np.float64), prime=False)
        probe = dp.clone()
        sph.step(prm, probe, 1, ws, prime=False)
        out = probe.numpy()
        o = order_by_id(out["id"])
        r = order_by_id(st["id"])
        dx = out["x"][:, o] - ref["x"][:, r]
        dx -= np.round(dx)
        assert np.abs(dx).max() < 1e-12
        assert normwise(out["rho"][o], ref["rho"][r]) < TOL_RHO[prec]
        assert normwise(out["a"][:, o], ref["a"][:, r]) < TOL_ACC[prec]
        if prec == sph.FP64:
            assert normwise(out["u"][:, o], ref["u"][:, r]) < 1e-12
        else:
            # u^{n+1} = u^n + dt/2 (a^n + a^{n+1}): bounded by the acceleration bar
            bound = p.dt * TOL_ACC[prec] * np.abs(ref["a"]).max()
            assert np.abs(out["u"][:, o] - ref["u"][:, r]).max() < bound
    sph.check(ws)
