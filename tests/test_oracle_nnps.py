"""Pins of the oracle's neighbour search and cell sort (paper section "Nearest
neighbor particle search": uniform cells no smaller than the support radius,
neighbours found in the 3^d surrounding cells; Z-order-style sort of particle
ids by a cell key).

Facts used: exact lattice neighbour counts (tests/golden), strict inequality at
exact ties, symmetry of the predicate, agreement of the O(n^2) definition with
the cell-grid algorithm (two different code paths of the oracle), and the
stable-sort routine of numpy for the sort."""
import os

import numpy as np
import pytest

import oracle
import sph_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lattice_neighbour_counts.txt")


def _golden_counts():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        d, hdx, k = line.split()
        rows.append((int(d), float(hdx), int(k)))
    return rows


def _lattice_case(dim, n_side, hdx, kernel=W.CUBIC, cell_div=1):
    dx = 1.0 / n_side
    x = W.lattice((n_side,) * dim, dx, (0.0,) * dim)
    p = W.Params(dim=dim, kernel=kernel, h=hdx * dx, rho0=1.0, c0=10.0, nu=0.01, eta=0.01,
                 dt=1e-4, g=(0, 0, 0), lo=(0, 0, 0), hi=(1, 1, 1 if dim == 3 else 0),
                 periodic=(1, 1, 1 if dim == 3 else 0), cell_div=cell_div)
    return p, x


@pytest.mark.parametrize("dim,hdx,K", _golden_counts())
def test_lattice_counts(dim, hdx, K):
    """Every particle of a perfect periodic lattice has exactly K neighbours."""
    # dyadic spacings: where R/dx is an integer (hdx = 1.0 in 2D, 1.5 in 3D) the
    # lattice distances equal to R are exact ties, excluded by the strict test
    n_side = 16 if dim == 2 else 10
    if dim == 2 and hdx == 1.0:
        n_side = 64
    if dim == 3 and hdx == 1.5:
        n_side = 16
    p, x = _lattice_case(dim, n_side, hdx)
    off, _ = oracle.neighbors(p, x)
    assert np.all(np.diff(off) == K)
    off_b, _ = oracle.neighbors(p, x, brute=True)
    assert np.all(np.diff(off_b) == K)


def _lattice_count(dim, R_over_dx):
    """Points of the integer lattice with |n|^2 < (R/dx)^2, origin included:
    a direct count, independent of any neighbour search."""
    m = int(np.ceil(R_over_dx))
    g = np.arange(-m, m + 1)
    mesh = np.meshgrid(*([g] * dim), indexing="ij")
    r2 = sum(c.astype(np.int64) ** 2 for c in mesh)
    return int(np.count_nonzero(r2 < R_over_dx ** 2))


@pytest.mark.parametrize("dim,hdx,cell_div", [(2, 1.0, 1), (2, 1.2, 2), (3, 1.0, 1), (3, 0.9, 2)])
def test_lattice_counts_quintic_support(dim, hdx, cell_div):
    """Quintic spline: support R = 3h.  On a perfect periodic lattice every
    particle has the direct lattice count of points within 3h (R/dx = 3 in the
    first 2D case: exact ties at distance 3dx excluded by the strict test)."""
    n_side = 32 if dim == 2 else 16
    p, x = _lattice_case(dim, n_side, hdx, kernel=W.QUINTIC, cell_div=cell_div)
    K = _lattice_count(dim, 3.0 * hdx)
    off, _ = oracle.neighbors(p, x)
    assert np.all(np.diff(off) == K)
    off_b, _ = oracle.neighbors(p, x, brute=True)
    assert np.all(np.diff(off_b) == K)


def _jittered(dim, n_side, jitter, seed, periodic=True, hdx=1.3, cell_div=1):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_side
    x = W.lattice((n_side,) * dim, dx, (0.0,) * dim)
    x = x + rng.uniform(-jitter * dx, jitter * dx, size=x.shape)
    if periodic:
        x = np.mod(x, 1.0)
        lo, hi = (0, 0, 0), (1, 1, 1 if dim == 3 else 0)
    else:
        lo = (-0.1, -0.1, -0.1 if dim == 3 else 0)
        hi = (1.1, 1.1, 1.1 if dim == 3 else 0)
    per = (1, 1, 1 if dim == 3 else 0) if periodic else (0, 0, 0)
    p = W.Params(dim=dim, kernel=W.CUBIC, h=hdx * dx, rho0=1.0, c0=10.0, nu=0.01, eta=0.01,
                 dt=1e-4, g=(0, 0, 0), lo=lo, hi=hi, periodic=per, cell_div=cell_div)
    return p, x


@pytest.mark.parametrize("dim,n_side,periodic,cell_div",
                         [(2, 12, True, 1), (2, 12, False, 1), (2, 16, True, 2),
                          (3, 8, True, 1), (3, 6, False, 1), (3, 8, True, 2)])
def test_cells_equal_brute_force(dim, n_side, periodic, cell_div):
    p, x = _jittered(dim, n_side, 0.45, seed=7 + dim, periodic=periodic, cell_div=cell_div)
    o1, i1 = oracle.neighbors(p, x)
    o2, i2 = oracle.neighbors(p, x, brute=True)
    assert np.array_equal(o1, o2)
    assert np.array_equal(i1, i2)


def test_predicate_symmetric_and_self_included():
    p, x = _jittered(2, 14, 0.4, seed=3)
    off, idx = oracle.neighbors(p, x)
    n = x.shape[1]
    pairs = set()
    for i in range(n):
        row = idx[off[i]:off[i + 1]]
        assert i in row
        pairs.update((i, int(j)) for j in row)
    assert all((j, i) in pairs for (i, j) in pairs)


def test_minimum_image_across_periodic_faces():
    """Two particles near opposite faces of the periodic box are neighbours."""
    p = W.Params(dim=2, kernel=W.CUBIC, h=0.05, rho0=1, c0=10, nu=0.01, eta=0.01, dt=1e-4,
                 g=(0, 0, 0), lo=(0, 0, 0), hi=(1, 1, 0), periodic=(1, 1, 0))
    x = np.array([[0.01, 0.98, 0.5, 0.5], [0.5, 0.5, 0.005, 0.995]])
    off, idx = oracle.neighbors(p, x)
    rows = [set(idx[off[i]:off[i + 1]].tolist()) for i in range(4)]
    assert rows[0] == {0, 1}      # |dx| = 0.03 < 0.1 through the x face
    assert rows[2] == {2, 3}      # |dy| = 0.01 through the y face
    p2 = p.replace(periodic=(0, 0, 0), lo=(-0.1, -0.1, 0), hi=(1.1, 1.1, 0))
    off2, idx2 = oracle.neighbors(p2, x)
    assert set(idx2[off2[0]:off2[1]].tolist()) == {0}


def test_bin_sort_is_numpy_stable_sort():
    p, x = _jittered(2, 20, 0.45, seed=11)
    keys = oracle.cell_keys(p, x)
    ks, perm, cs, ce = oracle.bin_sort(p, x)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(perm, order)
    assert np.array_equal(ks, keys[order])
    assert np.all(np.diff(ks.astype(np.int64)) >= 0)
    assert int((ce.astype(np.int64) - cs).sum()) == x.shape[1]
    # each sorted particle is inside its cell's slot range and its cell's box
    nc, csz = oracle.grid(p)
    for s in range(x.shape[1]):
        k = ks[s]
        assert cs[k] <= s < ce[k]
        i = perm[s]
        cx, cy = k % nc[0], k // nc[0]
        assert cx * csz[0] <= x[0, i] < (cx + 1) * csz[0] + 1e-15
        assert cy * csz[1] <= x[1, i] < (cy + 1) * csz[1] + 1e-15


def test_grid_rejects_short_periodic_axis():
    p = W.Params(dim=2, kernel=W.CUBIC, h=0.2, rho0=1, c0=10, nu=0.01, eta=0.01, dt=1e-4,
                 g=(0, 0, 0), lo=(0, 0, 0), hi=(1, 1, 0), periodic=(1, 1, 0))
    with pytest.raises(ValueError):
        oracle.grid(p)   # floor(1 / 0.4) = 2 < 3 cells


def test_cell_size_at_least_support():
    for cd in (1, 2):
        p, x = _jittered(3, 10, 0.2, seed=1, cell_div=cd)
        nc, cs = oracle.grid(p)
        assert np.all(cs[:3] * cd >= 2 * p.h * (1 - 1e-15))
        assert np.all(nc[:3] == np.floor(1.0 * cd / (2 * p.h)))


def _cell_centres(p, cells):
    """Positions at the centres of the given cells (dim x m integer array)."""
    nc, cs = oracle.grid(p)
    return np.array([p.lo[k] + (cells[k] + 0.5) * cs[k] for k in range(p.dim)], np.float64)


@pytest.mark.parametrize("dim", [2, 3])
def test_z_order_key_recursion(dim):
    """Z-order (Morton) keys follow the curve's recursive definition: the
    cell (2x + a, 2y + b[, 2z + c]) of a grid of 2^k cells per axis has key
    2^dim key(x, y[, z]) + a + 2b[ + 4c] -- the 2^dim children of a cell in
    order x fastest, then y, then z -- and key(0) = 0.  Checked over every
    cell of a 16^dim grid (so the whole bit interleave is pinned)."""
    n = 16
    p = W.Params(dim=dim, kernel=W.CUBIC, h=0.5 / n, rho0=1.0, c0=10.0, nu=0.01, eta=0.01,
                 dt=1e-4, g=(0, 0, 0), lo=(0, 0, 0), hi=(1, 1, 1 if dim == 3 else 0),
                 periodic=(1, 1, 1 if dim == 3 else 0), cell_order=W.Z_ORDER)
    nc, _ = oracle.grid(p)
    assert np.all(nc[:dim] == n)
    cells = np.array(np.meshgrid(*[np.arange(n)] * dim, indexing="ij")).reshape(dim, -1)
    keys = oracle.cell_keys(p, _cell_centres(p, cells)).astype(np.int64)
    key = {tuple(c): k for c, k in zip(cells.T.tolist(), keys.tolist())}
    assert key[(0,) * dim] == 0
    assert sorted(keys.tolist()) == list(range(n ** dim))   # a bijection onto [0, n^dim)
    for c, k in key.items():
        parent = tuple(v // 2 for v in c)
        child = sum((v % 2) << a for a, v in enumerate(c))
        assert k == (key[parent] << dim) + child, (c, k)


def test_z_order_pads_to_a_power_of_two_grid():
    """With nc = 5 cells per axis the keys live in the 8^3 key space of the
    smallest power-of-two grid: cell (4, 4, 4) is the first child of the
    first child of the last octant, key 7 * 64; the sort's cell ranges cover
    the whole key space."""
    p, x = _jittered(3, 10, 0.2, seed=3)
    p = p.replace(h=0.1, cell_order=W.Z_ORDER)   # R = 0.2: 5 cells per axis
    nc, _ = oracle.grid(p)
    assert np.all(nc[:3] == 5)
    k = oracle.cell_keys(p, _cell_centres(p, np.array([[4], [4], [4]])))
    assert int(k[0]) == 7 * 64
    ks, perm, cs, ce = oracle.bin_sort(p, x)
    assert len(cs) == 8 ** 3
    assert int((ce.astype(np.int64) - cs).sum()) == x.shape[1]


@pytest.mark.parametrize("dim", [2, 3])
def test_z_order_bin_sort_is_numpy_stable_sort(dim):
    p, x = _jittered(dim, 18 if dim == 2 else 9, 0.45, seed=12)
    p = p.replace(cell_order=W.Z_ORDER)
    keys = oracle.cell_keys(p, x)
    ks, perm, cs, ce = oracle.bin_sort(p, x)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(perm, order)
    assert np.array_equal(ks, keys[order])
    for s in range(x.shape[1]):
        assert cs[ks[s]] <= s < ce[ks[s]]
    # the order of the sort keys does not change the neighbour sets
    off_r, idx_r = oracle.neighbors(p.replace(cell_order=W.ROW_MAJOR), x)
    off_z, idx_z = oracle.neighbors(p, x)
    assert np.array_equal(off_r, off_z) and np.array_equal(idx_r, idx_z)
