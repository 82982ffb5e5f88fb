"""Helpers shared by the GPU parity tests: fixture shaping and comparisons.
No method arithmetic lives here."""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

import sph_workloads as W


def drop_near_ties(p: W.Params, s: W.State, rel: float) -> W.State:
    """Remove particles with any neighbour at |r^2/R^2 - 1| < rel, so that the
    neighbour sets do not depend on rounding (a well-posed fixture)."""
    R = 2 * p.h
    dim = p.dim
    pts = s.x.T.copy()
    box = None
    if all(p.periodic[k] for k in range(dim)):
        box = np.array([p.hi[k] - p.lo[k] for k in range(dim)])
        pts = np.mod(pts - np.array(p.lo[:dim]), box)
    tree = cKDTree(pts, boxsize=box)
    pairs = tree.query_pairs(R * (1 + 2 * rel), output_type="ndarray")
    if len(pairs) == 0:
        return s
    d = pts[pairs[:, 0]] - pts[pairs[:, 1]]
    if box is not None:
        d -= box * np.round(d / box)
    r2 = (d * d).sum(axis=1)
    bad = np.abs(r2 / (R * R) - 1) < rel
    drop = np.unique(pairs[bad, 0])
    keep = np.ones(s.n, bool)
    keep[drop] = False
    return W.State(s.x[:, keep].copy(), s.u[:, keep].copy(), s.m[keep].copy(),
                   s.ptype[keep].copy(), np.arange(keep.sum(), dtype=np.int32))


def shuffled(s: W.State, seed: int = 0) -> W.State:
    """The same particles in a random order (ids travel with them)."""
    perm = np.random.default_rng(seed).permutation(s.n)
    return W.State(s.x[:, perm].copy(), s.u[:, perm].copy(), s.m[perm].copy(),
                   s.ptype[perm].copy(), s.pid[perm].copy())


def normwise(got: np.ndarray, ref: np.ndarray) -> float:
    """max_i |got - ref| / max_i |ref|, per component, worst component."""
    got = np.atleast_2d(np.asarray(got, np.float64))
    ref = np.atleast_2d(np.asarray(ref, np.float64))
    worst = 0.0
    for g, r in zip(got, ref):
        scale = np.abs(r).max()
        err = np.abs(g - r).max()
        worst = max(worst, err / scale if scale > 0 else err)
    return worst


def order_by_id(ids: np.ndarray) -> np.ndarray:
    """Index array that puts id-labelled rows into id order."""
    return np.argsort(ids, kind="stable")
