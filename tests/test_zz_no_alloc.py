"""sph_step_noalloc (the static-scratch variant of sph_step) against sph_step
with a caller workspace: two calls in a row, the second on a smaller input,
each bitwise equal to sph_step on the same input (same kernels, same order);
inputs whose workspace exceeds the static scratch are refused."""
import numpy as np
import pytest
import torch

import paper_1909_04504_amd as sph
import sph_workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("x", "u", "a", "rho", "p", "id")


def _case(kind, size):
    if kind == "tg2d":
        return W.taylor_green(size, jitter=0.2, seed=size)
    return W.periodic_cube(n_side=size, jitter=0.3, sigma_u=0.1, seed=size, cell_div=2)


@pytest.mark.parametrize("kind,sizes", [("tg2d", (40, 28)), ("cube3d", (16, 12))])
@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32_MIXED])
def test_step_noalloc_matches_step(kind, sizes, prec):
    nsteps = 3
    for size in sizes:
        p, s = _case(kind, size)
        prm = sph.make_params(p, prec)
        ref = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, s.n)
        d_ref = torch.zeros((nsteps, 1 + p.dim), dtype=torch.float64, device="cuda")
        sph.step(prm, ref, nsteps, ws, prime=True, diag=d_ref)
        got = sph.DeviceParticles.from_state(s, prec)
        d_got = torch.full((nsteps, 1 + p.dim), np.nan, dtype=torch.float64, device="cuda")
        sph.step_noalloc(prm, got, nsteps, prime=True, diag=d_got)
        torch.cuda.synchronize()
        a, b = ref.numpy(), got.numpy()
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (kind, size, f)
        assert torch.equal(d_ref, d_got)


def test_step_noalloc_refuses_large_inputs():
    p, s = W.periodic_cube(n_side=64, jitter=0.2, sigma_u=0.1, seed=3, cell_div=2)
    prm = sph.make_params(p, sph.FP32_MIXED)
    assert sph.workspace_bytes(prm, s.n) > sph.NOALLOC_SCRATCH_BYTES
    dp = sph.DeviceParticles.from_state(s, sph.FP32_MIXED)
    with pytest.raises(sph.SphError) as ei:
        sph.step_noalloc(prm, dp, 1, prime=True)
    assert ei.value.code == sph.SPH_EWORKSPACE
