"""Pins of the oracle's smoothing kernels (paper Section 2: compact W with
support k h; cubic spline and Wendland C2 with k = 2, the design readings A2,
A3, and the quintic spline with k = 3).  Checked against facts fixed by
mathematics, not against the formulas themselves: unit integral, continuity at
the piece boundaries and at the support edge, and derivatives against finite
differences."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import sph_workloads as W


def _p(dim, kernel, h=0.37):
    return W.Params(dim=dim, kernel=kernel, h=h, rho0=1.0, c0=10.0, nu=0.01, eta=0.01,
                    dt=1e-3, g=(0, 0, 0), lo=(0, 0, 0), hi=(1, 1, 1), periodic=(0, 0, 0))


CASES = [(d, k) for d in (2, 3) for k in (W.CUBIC, W.WENDLAND, W.QUINTIC)]
SUPPORT = {W.CUBIC: 2, W.WENDLAND: 2, W.QUINTIC: 3}  # R = k h


@pytest.mark.parametrize("dim,kernel", CASES)
def test_unit_integral_quadrature(dim, kernel):
    """The integral of W over R^d is 1 (kernel normalisation)."""
    p = _p(dim, kernel)
    L = oracle.lib()
    o = oracle.params(p)
    import ctypes
    w = lambda r: L.orc_kernel_w(ctypes.byref(o), r)
    area = (lambda r: 2 * math.pi * r) if dim == 2 else (lambda r: 4 * math.pi * r * r)
    total = 0.0
    for a, b in [(m * p.h, (m + 1) * p.h) for m in range(SUPPORT[kernel])]:
        val, err = integrate.quad(lambda r: w(r) * area(r), a, b, epsabs=1e-15, epsrel=1e-13,
                                  limit=200)
        total += val
    assert abs(total - 1.0) < 1e-12


@pytest.mark.parametrize("dim,kernel", CASES)
def test_gauss_legendre_unit_integral(dim, kernel):
    """40-point Gauss-Legendre on each polynomial piece integrates it exactly
    (to rounding): the integral must be 1 to 1e-13."""
    p = _p(dim, kernel, h=0.05)
    x, wts = np.polynomial.legendre.leggauss(40)
    total = 0.0
    for a, b in [(m * p.h, (m + 1) * p.h) for m in range(SUPPORT[kernel])]:
        r = 0.5 * (b - a) * x + 0.5 * (b + a)
        f = oracle.kernel_w(p, r) * (2 * math.pi * r if dim == 2 else 4 * math.pi * r * r)
        total += 0.5 * (b - a) * np.dot(wts, f)
    assert abs(total - 1.0) < 1e-13


@pytest.mark.parametrize("dim,kernel", CASES)
def test_compact_support_and_continuity(dim, kernel):
    """W = 0 for r >= R = k h; W and dW/dr continuous at the piece boundaries
    r = h (and 2h) and at r -> R."""
    p = _p(dim, kernel, h=0.5)
    K = SUPPORT[kernel]
    r = np.array([K * p.h, K * p.h + 0.5, 3.0])
    assert np.all(oracle.kernel_w(p, r) == 0.0)
    assert np.all(oracle.kernel_dwdr(p, r) == 0.0)
    eps = 1e-9
    for rb in [m * p.h for m in range(1, K + 1)]:
        wl, wr = oracle.kernel_w(p, [rb - eps, rb + eps])
        dl, dr = oracle.kernel_dwdr(p, [rb - eps, rb + eps])
        assert abs(wl - wr) < 1e-7
        assert abs(dl - dr) < 1e-7
    # monotone decreasing on (0, R)
    rr = np.linspace(1e-6, K * p.h - 1e-6, 500)
    assert np.all(np.diff(oracle.kernel_w(p, rr)) < 0)
    # dW/dr = 0 at the origin (smooth peak)
    assert oracle.kernel_dwdr(p, [0.0])[0] == 0.0


@pytest.mark.parametrize("dim,kernel", CASES)
def test_derivatives_match_finite_differences(dim, kernel):
    p = _p(dim, kernel, h=0.3)
    K = SUPPORT[kernel]
    r = np.linspace(0.01, K * p.h - 0.01, 57)
    for m in range(1, K):
        r = r[np.abs(r - m * p.h) > 1e-3]
    eps = 1e-5
    fd1 = (oracle.kernel_w(p, r + eps) - oracle.kernel_w(p, r - eps)) / (2 * eps)
    d1 = oracle.kernel_dwdr(p, r)
    assert np.abs(fd1 - d1).max() < 1e-7 * np.abs(d1).max()
    fd2 = (oracle.kernel_dwdr(p, r + eps) - oracle.kernel_dwdr(p, r - eps)) / (2 * eps)
    d2 = oracle.kernel_d2wdr2(p, r)
    assert np.abs(fd2 - d2).max() < 1e-6 * np.abs(d2).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_quintic_peak_value(dim):
    """W(0) = sigma w(0) with w(0) = 3^5 - 6 2^5 + 15 = 66, and sigma the
    unit-integral normalisation: the shape integrates to 2 pi (239/7) h^2 in
    2D (the integral of q w(q) over [0, 3] is 239/7) and to 4 pi 30 h^3 in 3D
    (the integral of q^2 w(q) is 30), exact rationals times pi."""
    h = 0.2
    p = _p(dim, W.QUINTIC, h=h)
    expect = (66.0 / (2 * math.pi * 239.0 / 7.0) / h ** 2 if dim == 2
              else 66.0 / (4 * math.pi * 30.0) / h ** 3)
    assert oracle.kernel_w(p, [0.0])[0] == pytest.approx(expect, rel=1e-14)
