"""Host checks of the test fixtures themselves (no GPU): the near-tie helper
places its companions where it says."""
import numpy as np

import sph_workloads as W
from helpers import support_radius, with_near_ties
from test_gpu_parity import make_case


def test_near_tie_fixture_has_band_pairs():
    """The band fixture is what it claims: hundreds of pairs within 1e-5 of R^2."""
    p, s = make_case("cube3d")
    s = with_near_ties(p, s, 400, 5e-7, 1e-5, seed=21)
    R2 = support_radius(p) ** 2
    x = s.x[:, -400:]
    partner = s.x  # brute force distances from each companion
    d = x[:, :, None] - partner[:, None, :]
    L = np.array([p.hi[k] - p.lo[k] for k in range(3)])[:, None, None]
    d -= L * np.round(d / L)
    r2 = (d * d).sum(axis=0) / R2
    band = (np.abs(r2 - 1) < 1e-5) & (np.abs(r2 - 1) >= 5e-7 * 0.99)
    assert band.sum() >= 400


def test_near_tie_fixture_stays_inside_walled_box():
    """On non-periodic axes the companions land inside [lo, hi), so a walled
    fixture never sets the library's out-of-domain flag."""
    for case in ("box2d", "sparse2d"):
        p, s = make_case(case)
        s = with_near_ties(p, s, min(400, s.n // 4), 1e-12, 1e-5, seed=21)
        for k in range(p.dim):
            assert np.all(s.x[k] >= p.lo[k]) and np.all(s.x[k] < p.hi[k]), (case, k)
