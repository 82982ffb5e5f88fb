"""Host-side checks of the benchmark's bookkeeping (no GPU): the refusal of
several GPUs, the count of candidate pairs the list build tests, the roofline
arithmetic and the digest guard on profiled traffic."""
import itertools
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_1909_04504_amd as sph
import sph_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _brute_stencil_tests(prm, x):
    """For every particle, the particles whose cell lies within S cells of its
    own on every axis (periodic axes wrap): counted pair by pair."""
    nc, _ = sph.grid(prm)
    dim, S = prm.dim, prm.cell_div
    cell = np.stack([np.clip(np.floor((x[k] - prm.lo[k]) / ((prm.hi[k] - prm.lo[k]) / nc[k]))
                             .astype(np.int64), 0, nc[k] - 1) for k in range(dim)])
    total = 0
    for i in range(x.shape[1]):
        ok = np.ones(x.shape[1], bool)
        for k in range(dim):
            d = np.abs(cell[k] - cell[k, i])
            if prm.periodic[k]:
                d = np.minimum(d, nc[k] - d)
            ok &= d <= S
        total += int(ok.sum())
    return total


@pytest.mark.parametrize("case", ["periodic2d", "walls2d", "periodic3d_cd2"])
def test_stencil_test_count_matches_brute_force(case):
    if case == "periodic2d":
        p, s = W.taylor_green(24, jitter=0.3, seed=1)
    elif case == "walls2d":
        p, s = W.dam_break_2d(dx=0.2)
    else:
        p, s = W.periodic_cube(n_side=10, jitter=0.3, seed=2, cell_div=2)
    prm = sph.make_params(p, sph.FP32_MIXED)
    assert bench.stencil_tests(sph, prm, s.x) == _brute_stencil_tests(prm, s.x)


def test_roofline_arithmetic():
    """The dominant kernel's algorithmic bytes over its launch time, against
    the peak its intensity selects."""
    wl = W.workload("tg64")
    n, steps = wl.state.n, 10
    inter = 21 * n
    res = {"kernels_us": {"nlist": 10.0, "density": 4.0, "momentum": 6.0},
           "kernels_launches": {"nlist": steps, "density": steps, "momentum": steps},
           "interactions_timed": inter * steps}
    tests = 3 * inter
    rl = bench.roofline(res, wl, sph.FP32_MIXED, steps, tests)
    assert rl["kernel"] == "nlist"
    nbytes = bench.bytes_per_particle("nlist", 2, 4) * n + 4 * inter
    flops = bench.FLOPS_PER_TEST[2] * tests
    assert rl["bytes_per_launch"] == nbytes
    assert flops / nbytes < bench.VALU_PEAK_TFLOPS * 1e12 / (bench.HBM_PEAK_GBS * 1e9)
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s"
    assert rl["achieved"] == pytest.approx(nbytes / 10e-6 / 1e9)
    assert rl["frac"] == pytest.approx(rl["achieved"] / bench.HBM_PEAK_GBS)


def test_bytes_per_particle_counts_each_array_once():
    # 2D mixed precision: record 16 B, key 4, count 4
    assert bench.bytes_per_particle("nlist", 2, 4) == 24
    # FP64 records are 32 B
    assert bench.bytes_per_particle("nlist", 2, 8) == 40
    for k, d, t in itertools.product(("density", "momentum", "cont_momentum", "rank_gather",
                                      "drift_hash", "scatter"), (2, 3), (4, 8)):
        assert bench.bytes_per_particle(k, d, t) > 0
    # the continuity gather also moves rho (in and out), p and (rho, P)
    assert (bench.bytes_per_particle("rank_gather", 2, 4, True)
            - bench.bytes_per_particle("rank_gather", 2, 4)) == 8 + 8 + 4 + 8


def test_profiled_traffic_needs_the_current_source(tmp_path, monkeypatch):
    """Counters taken on other kernel sources are never reported."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"bytes_per_launch": 123.0, "source_digest": bench.source_digest()}
    (prof / "traffic.json").write_text(json.dumps({"nlist/tg512": entry}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: entry["source_digest"])
    assert bench.traffic_from_profile("nlist", "tg512") == 123.0
    assert bench.traffic_from_profile("nlist", "other") is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.traffic_from_profile("nlist", "tg512") is None
