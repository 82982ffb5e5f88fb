"""GPU adjoint (sph_step_backward, sph_accel_backward, SPHRollout) against the
FP64 CPU oracle's adjoint and against finite differences of the GPU forward."""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_04504_amd as sph
import sph_workloads as W
from helpers import normwise
from paper_1909_04504_amd.autograd import rollout_ke

pytestmark = pytest.mark.gpu


def _grads(p, s, nsteps, k, prec, nbr_cap=0):
    u0 = torch.tensor(s.u, dtype=torch.float64, device="cuda", requires_grad=True)
    nu = torch.tensor(p.nu, dtype=torch.float64, requires_grad=True)
    ke = rollout_ke(u0, nu, p, s.x, s.m, s.ptype, nsteps, k, prec, nbr_cap)
    ke.backward()
    return float(ke), u0.grad.cpu().numpy(), float(nu.grad)


@pytest.mark.parametrize("k,nbr_cap", [(1, 0), (3, 0), (8, 0), (3, -1), (3, 12)])
def test_rollout_gradient_fp64_matches_oracle(k, nbr_cap):
    """nbr_cap: default lists, cell walks only, and lists too short for most
    particles (walked) beside ones that fit."""
    p, s = W.taylor_green(16, jitter=0.25, seed=3)
    nsteps = 8
    ke, gu, gnu = _grads(p, s, nsteps, k, sph.FP64, nbr_cap)
    gu_ref, gnu_ref, ke_ref = oracle.adjoint_ke(p, s.x, s.u, s.m, s.ptype, nsteps)
    assert ke == pytest.approx(ke_ref, rel=1e-12)
    assert normwise(gu, gu_ref) < 1e-10
    assert gnu == pytest.approx(gnu_ref, rel=1e-10)


def test_rollout_gradient_quintic_fp64_and_mixed():
    """Quintic spline (support 3h): the FP64 rollout gradient against the
    oracle adjoint, and the mixed-precision one at the mixed bar."""
    p, s = W.taylor_green(16, jitter=0.25, seed=5, kernel=W.QUINTIC, hdx=1.0)
    nsteps = 6
    gu_ref, gnu_ref, ke_ref = oracle.adjoint_ke(p, s.x, s.u, s.m, s.ptype, nsteps)
    ke, gu, gnu = _grads(p, s, nsteps, 3, sph.FP64)
    assert ke == pytest.approx(ke_ref, rel=1e-12)
    assert normwise(gu, gu_ref) < 1e-10
    assert gnu == pytest.approx(gnu_ref, rel=1e-10)
    ke, gu, gnu = _grads(p, s, nsteps, 3, sph.FP32_MIXED)
    assert normwise(gu, gu_ref) < 1e-3
    assert gnu == pytest.approx(gnu_ref, rel=1e-3)


def test_rollout_gradient_3d_walls_fp64():
    p, s = W.dam_break_3d(dx=0.05)
    rng = np.random.default_rng(4)
    f = s.ptype == 0
    s.u[:, f] = rng.normal(0, 0.2, size=(3, int(f.sum())))
    nsteps = 4
    ke, gu, gnu = _grads(p, s, nsteps, 2, sph.FP64)
    gu_ref, gnu_ref, ke_ref = oracle.adjoint_ke(p, s.x, s.u, s.m, s.ptype, nsteps)
    assert ke == pytest.approx(ke_ref, rel=1e-12)
    assert normwise(gu, gu_ref) < 1e-10
    assert gnu == pytest.approx(gnu_ref, rel=1e-9)
    assert np.all(gu[:, ~f] == 0.0)


def test_mixed_precision_adjoint_at_32_vs_fp64_oracle():
    """Mixed-precision forward and adjoint, 32x32 Taylor-Green, 200 steps,
    checkpoint every 20, against the FP64 CPU adjoint."""
    wl = W.workload("tg32")
    p, s = wl.params, wl.state
    nsteps = 200
    ke, gu, gnu = _grads(p, s, nsteps, 20, sph.FP32_MIXED)
    gu_ref, gnu_ref, ke_ref = oracle.adjoint_ke(p, s.x, s.u, s.m, s.ptype, nsteps)
    assert ke == pytest.approx(ke_ref, rel=1e-5)
    assert normwise(gu, gu_ref) < 1e-3
    assert gnu == pytest.approx(gnu_ref, rel=1e-3)


def test_viscosity_gradient_vs_central_differences_mixed():
    """dKE/dnu of the mixed-precision rollout against a central difference of
    the same forward with an absolute step 1e-4 on nu."""
    p, s = W.taylor_green(64)
    nsteps, k = 50, 10
    _, _, gnu = _grads(p, s, nsteps, k, sph.FP32_MIXED)
    eps = 1e-4

    def ke_at(nu):
        prm = sph.make_params(p.replace(nu=nu), sph.FP32_MIXED)
        dp = sph.DeviceParticles.from_state(s, sph.FP32_MIXED)
        ws = sph.workspace(prm, s.n)
        diag = torch.zeros((nsteps, 3), dtype=torch.float64, device="cuda")
        sph.step(prm, dp, nsteps, ws, prime=True, diag=diag)
        return float(diag[-1, 0])

    fd = (ke_at(p.nu + eps) - ke_at(p.nu - eps)) / (2 * eps)
    assert gnu == pytest.approx(fd, rel=1e-2)


def test_velocity_gradient_directional_fd_fp64():
    p, s = W.taylor_green(20, jitter=0.2, seed=9)
    nsteps = 10
    _, gu, _ = _grads(p, s, nsteps, 4, sph.FP64)
    rng = np.random.default_rng(2)
    w = rng.standard_normal(s.u.shape)
    w /= np.sqrt(np.mean(w * w))
    eps = 1e-6

    def ke_at(u):
        prm = sph.make_params(p, sph.FP64)
        st = W.State(s.x, u, s.m, s.ptype, s.pid)
        dp = sph.DeviceParticles.from_state(st, sph.FP64)
        ws = sph.workspace(prm, s.n)
        diag = torch.zeros((nsteps, 3), dtype=torch.float64, device="cuda")
        sph.step(prm, dp, nsteps, ws, prime=True, diag=diag)
        return float(diag[-1, 0])

    fd = (ke_at(s.u + eps * w) - ke_at(s.u - eps * w)) / (2 * eps)
    assert np.sum(gu * w) == pytest.approx(fd, rel=1e-6)


def test_accel_backward_matches_oracle_transpose():
    p, s = W.periodic_cube(n_side=10, jitter=0.3, sigma_u=0.1, seed=5)
    rng = np.random.default_rng(1)
    lam = rng.standard_normal(s.x.shape)
    for prec, tol, cap in ((sph.FP64, 1e-11, 0), (sph.FP32_MIXED, 2e-4, 0),
                           (sph.FP64, 1e-11, -1), (sph.FP32_MIXED, 2e-4, 40)):
        prm = sph.make_params(p, prec, cap)
        dp = sph.DeviceParticles.from_state(s, prec)
        ws = sph.workspace(prm, s.n, adjoint_k=1)
        la = torch.tensor(lam, dtype=torch.float64, device="cuda")
        lx = torch.zeros_like(la)
        lu = torch.zeros_like(la)
        dJ = torch.zeros(1, dtype=torch.float64, device="cuda")
        sph.accel_backward(prm, dp, la, lx, lu, dJ, ws)
        rx, rv, rnu = oracle.rhs_adjoint(p, s.x, s.u, s.m, s.ptype, lam)
        assert normwise(lx.cpu().numpy(), rx) < tol
        assert normwise(lu.cpu().numpy(), rv) < tol
        assert float(dJ[0]) == pytest.approx(rnu, rel=tol * 10)


def test_adjoint_at_full_size_256_vs_central_differences():
    """The differentiation workload at its stated size: 256x256 Taylor-Green,
    200 mixed-precision steps, checkpoint every 20.  dKE/dnu from the adjoint
    against a central difference of the same forward (absolute step 1e-4 on
    nu), and the directional derivative along a unit-RMS random field w of
    u0 against a central difference with step 1e-4; both within 1e-2."""
    wl = W.workload("tg256")
    p, s = wl.params, wl.state
    nsteps, k, eps = 200, 20, 1e-4
    ke, gu, gnu = _grads(p, s, nsteps, k, sph.FP32_MIXED)

    def ke_at(nu, u):
        prm = sph.make_params(p.replace(nu=nu), sph.FP32_MIXED)
        dp = sph.DeviceParticles.from_state(W.State(s.x, u, s.m, s.ptype, s.pid), sph.FP32_MIXED)
        ws = sph.workspace(prm, s.n)
        diag = torch.zeros((nsteps, 3), dtype=torch.float64, device="cuda")
        sph.step(prm, dp, nsteps, ws, prime=True, diag=diag)
        return float(diag[-1, 0])

    assert ke == pytest.approx(ke_at(p.nu, s.u), rel=1e-12)
    fd_nu = (ke_at(p.nu + eps, s.u) - ke_at(p.nu - eps, s.u)) / (2 * eps)
    assert gnu == pytest.approx(fd_nu, rel=1e-2)
    rng = np.random.default_rng(6)
    w = rng.standard_normal(s.u.shape)
    w /= np.sqrt(np.mean(w * w))
    fd_u = (ke_at(p.nu, s.u + eps * w) - ke_at(p.nu, s.u - eps * w)) / (2 * eps)
    assert np.sum(gu * w) == pytest.approx(fd_u, rel=1e-2)


def test_ke_seed():
    """sph_ke_seed: lam_u = scale m u, lam_x = lam_a = 0, walls zero."""
    for p, s in (W.taylor_green(12, jitter=0.2, seed=1), W.dam_break_3d(dx=0.1)):
        prm = sph.make_params(p, sph.FP64)
        dp = sph.DeviceParticles.from_state(s, sph.FP64)
        d = p.dim
        lam = torch.full((3 * d, s.n), np.nan, dtype=torch.float64, device="cuda")
        sph.ke_seed(prm, dp, 0.75, lam)
        got = lam.cpu().numpy()
        assert np.all(got[:d] == 0) and np.all(got[2 * d:] == 0)
        assert np.array_equal(got[d:2 * d], 0.75 * s.m * s.u)
