#!/usr/bin/env python3
"""Benchmark of the WCSPH hot path on one MI355X.

Headline workload: the 3D periodic cube of 256^3 = 16,777,216 particles, a
lattice jittered by +-0.2 dx, velocities N(0, 0.1^2) per component, Wendland
C2 with h = 1.5 dx (about 113 neighbours per particle), Tait EOS with
c0 = 10 max|u|, a neighbour rebuild every step.

A step is one full pass of the hot path: half kick + drift + wrap, cell hash,
counting sort with the stable per-cell rank and state gather, neighbour
lists, summation density + EOS, momentum + closing half kick.  Inputs are
resident in device memory before the timed region.

Prints one JSON line.  value = particle-neighbour interactions per second of
the mixed-precision step (pair terms in FP32 on cell-relative offsets, FP64
integration); the full-FP64 step is reported beside it, with the normwise
error of both against the FP64 CPU oracle per field, the 512^2 Taylor-Green
step, the adjoint/forward time ratio and the oracle's own throughput on a
bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s for
# FP64 and for non-packed FP32; the build keeps packed FP32 instructions out of the
# code, so 78.6 TFLOP/s is the FP32 ceiling this code can reach (157.3 packed).
VALU_PEAK_TFLOPS = 78.6

# Algorithmic floating-point operations per accepted neighbour pair (FMA = 2,
# sqrt and reciprocal = 1), from the written kernels: separation (dim),
# squared distance (2 dim - 1), sqrt, q, kernel value or gradient factor, the
# pair terms and the accumulation.
FLOPS_PER_PAIR = {
    ("density", 2): 19, ("density", 3): 20,
    ("momentum", 2): 34, ("momentum", 3): 42,
    # continuity scheme: the momentum pair terms (the viscous one is formed
    # even at nu = 0) plus v_ij . r_ij (2 dim - 1), its product with the
    # gradient factor and the mass, and the accumulation
    ("cont_momentum", 2): 40, ("cont_momentum", 3): 50,
}
PAIR_KERNELS = ("nlist", "density", "momentum", "cont_momentum", "tile_build", "tile_density",
                "tile_momentum")
# bytes per list entry: 32-bit global lists, 16-bit tile lists (union indices)
ENTRY_BYTES = {"nlist": 4, "density": 4, "momentum": 4, "cont_momentum": 4, "tile_build": 2,
               "tile_density": 2, "tile_momentum": 2}
FLOPS_PER_PAIR.update({("tile_density", 3): 20, ("tile_momentum", 3): 42})
KERNEL_NAMES = {0: "cubic spline", 1: "Wendland C2", 2: "quintic spline"}
# Neighbour-list build: per candidate pair tested (every particle of the
# stencil cells of i's cell): the separation (dim), |r|^2 (2 dim - 1).
FLOPS_PER_TEST = {2: 5, 3: 8}


def bytes_per_particle(kernel: str, dim: int, tsize: int, continuity: bool = False) -> int:
    """Algorithmic bytes per particle of each step kernel: every array the
    kernel must touch, read or written once (neighbour re-reads served from
    cache are not algorithmic traffic).  The neighbour lists (4 bytes per
    interaction) are added per pair by the caller."""
    d, T = dim, tsize
    R = 16 if T == 4 else 32  # pair record: int4 offsets + mass / double4
    if kernel == "nlist":
        # in: record, key; out: neighbour count
        return R + 4 + 4
    if kernel == "tile_build":
        # in: record, cell range; out: neighbour count
        return R + 4 + 4
    if kernel == "tile_density":
        # in: record, count; out: rho, p, (rho, P)
        return R + 4 + 2 * T + 2 * T
    if kernel == "tile_momentum":
        # as momentum
        return R + 4 + 4 * T + 2 * T + 1 + 8 * d + d * T + 8 * d + 4
    if kernel == "density":
        # in: record, count; out: rho, p, (rho, P)
        return R + 4 + 2 * T + 2 * T
    if kernel == "momentum":
        # in: record, count, v, (rho, P), type, u (f64); out: a, u (f64), key
        return R + 4 + 4 * T + 2 * T + 1 + 8 * d + d * T + 8 * d + 4
    if kernel == "cont_momentum":
        # in: record, count, v, (rho, P), type, u, x, rho (f64);
        # out: a, u, x, rho (f64), key
        return R + 4 + 4 * T + 2 * T + 1 + 8 * d + 8 * d + 8 + d * T + 8 * d + 8 * d + 8 + 4
    if kernel == "drift_hash":
        # in: x, u (f64), a, type; out: x, v (f64), key, cell count
        return 16 * d + d * T + 1 + 16 * d + 4 + 4
    if kernel == "rank_gather":
        # in: slot, key, cell range, state (x, u, m, type, id); out: state, perm, key,
        # pair records (delta, m) and v
        state = 16 * d + 8 + 1 + 4
        eos = 8 + 8 + T + 2 * T if continuity else 0  # rho in/out, p, (rho, P)
        return 4 + 4 + 8 + 2 * state + 4 + 4 + (d + 1) * T + d * T + eos
    if kernel == "scatter":
        return 4 + 4 + 4 + 4
    return 0


def source_digest() -> str:
    """Digest of the library's device and launch sources (the traffic of a
    profiled kernel is used only while it matches)."""
    h = hashlib.sha256()
    for f in ("sph_kernels.hpp", "sph_tiles.hpp", "sph_adjoint.hpp", "sph_engine.hpp", "sph.hip"):
        with open(os.path.join(ROOT, "paper_1909_04504_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = data.get(f"{kernel}/{workload}")
    if not ent or ent.get("source_digest") != source_digest():
        return None
    return ent.get("bytes_per_launch")


def run_precision(sph, torch, wl, prec, steps, warmup, timing, nbr_cap=0, pair_tiles=0):
    p, s = wl.params, wl.state
    prm = sph.make_params(p, prec, nbr_cap, pair_tiles)
    dp = sph.DeviceParticles.from_state(s, prec, scheme=p.scheme)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    if warmup:
        sph.step(prm, dp, warmup, ws, prime=False)
    torch.cuda.synchronize()
    sph.read_interactions(ws, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sph.step(prm, dp, steps, ws, prime=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inter = sph.read_interactions(ws, reset=True)
    sph.check(ws)
    res = {"seconds": t1 - t0, "ms_per_step": 1e3 * (t1 - t0) / steps,
           "interactions": inter, "interactions_per_s": inter / (t1 - t0)}
    if timing:
        res["pair_tests"] = stencil_tests(sph, prm, dp.x.cpu().numpy())
    if timing:
        # second timed region with every kernel bracketed by HIP events on the
        # library's stream: per-kernel average durations
        sph.timer_read(reset=True)
        sph.timer_enable(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sph.step(prm, dp, steps, ws, prime=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        sph.timer_enable(False)
        kt = sph.timer_read(reset=True)
        res["instrumented_ms_per_step"] = 1e3 * (t3 - t2) / steps
        res["kernels_us"] = {k: 1e3 * ms / max(c, 1) for k, (ms, c) in kt.items()}
        res["kernels_launches"] = {k: c for k, (ms, c) in kt.items()}
        res["interactions_timed"] = sph.read_interactions(ws, reset=True)
    del dp, ws
    torch.cuda.empty_cache()
    return res


def stencil_tests(sph, prm, x) -> int:
    """Candidate pairs the list build tests in one launch: for every particle,
    the particles of the (2S+1)^dim stencil cells of its cell (host count
    from the cell occupancy of positions x)."""
    import numpy as np
    nc, _ = sph.grid(prm)
    dim, S = prm.dim, prm.cell_div
    cells = []
    for k in range(dim):
        cs = (prm.hi[k] - prm.lo[k]) / nc[k]
        c = np.floor((x[k] - prm.lo[k]) / cs).astype(np.int64)
        cells.append(np.clip(c, 0, nc[k] - 1))
    occ = np.zeros(tuple(nc[:dim]), np.int64)
    np.add.at(occ, tuple(cells), 1)
    M = np.zeros_like(occ)
    for off in np.ndindex(*([2 * S + 1] * dim)):
        sh = occ
        for k in range(dim):
            o = off[k] - S
            if o == 0:
                continue
            sh = np.roll(sh, -o, axis=k)  # sh[c] = occ[c + o]
            if not prm.periodic[k]:
                idx = [slice(None)] * dim
                idx[k] = slice(nc[k] - o, nc[k]) if o > 0 else slice(0, -o)
                sh[tuple(idx)] = 0
        M += sh
    return int((occ * M).sum())


def roofline(res, wl, prec, steps, tests=None):
    """Roofline entry of the dominant kernel of the step (the one with the
    largest time per step).  Its algorithmic bytes and flops per launch are
    priced against both HBM (8 TB/s) and the vector ALU (78.6 TFLOP/s); the
    bound is the resource with the larger time floor, i.e. ALU when the
    intensity is at or above the ridge point, and both fractions are kept."""
    kus = res["kernels_us"]
    launches = res["kernels_launches"]
    per_step = {k: kus[k] * launches[k] / steps for k in kus}
    dom = max(per_step, key=per_step.get)
    avg_s = kus[dom] * 1e-6
    dim, n = wl.params.dim, wl.state.n
    tsize = 4 if prec == 1 else 8
    inter_per_launch = res["interactions_timed"] / steps
    nbytes = bytes_per_particle(dom, dim, tsize, wl.params.scheme == 1) * n
    flops = None
    if dom in PAIR_KERNELS:
        # the neighbour lists, written or read once
        nbytes += ENTRY_BYTES[dom] * inter_per_launch
        if dom in ("nlist", "tile_build"):
            # the predicate on every candidate of the (2S+1)^d stencil cells
            # (the tiled build skips the cells beyond the support's reach, so
            # it evaluates fewer)
            flops = FLOPS_PER_TEST[dim] * tests
        else:
            # the momentum passes do no arithmetic for the self pair
            pairs = inter_per_launch if dom in ("density", "tile_density") else inter_per_launch - n
            flops = FLOPS_PER_PAIR[(dom, dim)] * pairs
    hbm_ach = nbytes / avg_s / 1e9
    out = {"kernel": dom, "avg_launch_us": kus[dom], "bytes_per_launch": nbytes,
           "interactions_per_launch": inter_per_launch,
           "hbm": {"achieved": hbm_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": hbm_ach / HBM_PEAK_GBS}}
    ridge = VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if flops is not None:
        alu_ach = flops / avg_s / 1e12
        out["flops_per_launch"] = flops
        out["intensity_flop_per_byte"] = flops / nbytes
        out["alu"] = {"achieved": alu_ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": alu_ach / VALU_PEAK_TFLOPS}
    if flops is not None and flops / nbytes >= ridge:
        out.update({"bound": "alu", **out["alu"]})
    else:
        out.update({"bound": "hbm", **out["hbm"]})
    if dom in ("nlist", "tile_build"):
        out["pair_tests_per_launch"] = tests
    out["traffic"] = traffic_from_profile(dom, wl.name)
    return out


def field_errors(sph, torch, wl, prec, nsample=1500):
    """Normwise error per field (max |f - f_ref| / max |f_ref|, by id) of the
    GPU against the FP64 oracle.
    * 3D workloads: rho, p and a of nsample particles after the priming
      evaluation of the initial state (the oracle evaluates the sample only).
    * 2D Taylor-Green: one whole step from the GPU's state after 100 steps,
      both sides starting from the same state: x, u, rho, p, a of every
      particle."""
    import numpy as np

    import oracle
    import sph_workloads as W

    def nw(g, r):
        g = np.atleast_2d(np.asarray(g, np.float64))
        r = np.atleast_2d(np.asarray(r, np.float64))
        return max(float(np.abs(gg - rr).max() / max(np.abs(rr).max(), 1e-300))
                   for gg, rr in zip(g, r))

    p, s = wl.params, wl.state
    prm = sph.make_params(p, prec)
    dp = sph.DeviceParticles.from_state(s, prec, scheme=p.scheme)
    ws = sph.workspace(prm, s.n)
    sph.step(prm, dp, 0, ws, prime=True)
    if p.dim == 3:
        sph.check(ws)
        ids = dp.id.cpu().numpy()
        sub = W.random_subset(s.n, nsample, seed=7)
        slot = np.empty(s.n, np.int64)
        slot[ids] = np.arange(s.n)
        sl = slot[sub]
        got = {"rho": dp.rho.cpu().numpy()[sl], "p": dp.p.cpu().numpy()[sl],
               "a": dp.a.cpu().numpy()[:, sl]}
        del dp, ws
        torch.cuda.empty_cache()
        rho, pr, a = oracle.eval_subset(p, s.x, s.u, s.m, s.ptype, sub)
        ref = {"rho": rho, "p": pr, "a": a}
        out = {f: nw(got[f], ref[f]) for f in got}
        out["sample"] = f"{len(sub)} particles after the priming evaluation of the initial state"
        return out
    sph.step(prm, dp, 100, ws, prime=False)
    st = dp.numpy()
    sph.step(prm, dp, 1, ws, prime=False)
    sph.check(ws)
    new = dp.numpy()
    del dp, ws
    torch.cuda.empty_cache()
    ref = oracle.step(p, st["x"], st["u"], st["m"], st["type"], 1,
                      a=st["a"].astype(np.float64), prime=False)
    o = np.argsort(new["id"], kind="stable")
    r = np.argsort(st["id"], kind="stable")
    out = {}
    dx = new["x"][:, o] - ref["x"][:, r]
    for k in range(p.dim):
        if p.periodic[k]:
            L = p.hi[k] - p.lo[k]
            dx[k] -= L * np.round(dx[k] / L)
    out["x"] = float(np.abs(dx).max() / np.abs(ref["x"]).max())
    for f in ("u", "rho", "p", "a"):
        out[f] = nw(new[f][..., o], ref[f][..., r])
    out["sample"] = "one whole step from the GPU state after 100 steps (every particle)"
    return out


def adjoint_ratio(sph, torch, steps=200, k=20, reps=2):
    """Backward (recompute + adjoint kernels) time over forward (with the
    checkpoint copies) time of the differentiable rollout on the 256x256
    Taylor-Green workload, mixed precision."""
    import sph_workloads as W
    from paper_1909_04504_amd.autograd import rollout_ke
    wl = W.workload("tg256")
    p, s = wl.params, wl.state
    best = None
    for _ in range(reps + 1):
        u0 = torch.tensor(s.u, dtype=torch.float64, device="cuda", requires_grad=True)
        nu = torch.tensor(p.nu, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ke = rollout_ke(u0, nu, p, s.x, s.m, s.ptype, steps, k, sph.FP32_MIXED)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ke.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        cur = (t1 - t0, t2 - t1)
        if best is None or sum(cur) < sum(best):
            best = cur
    fwd, bwd = best
    return {"workload": f"{wl.name}: {s.n} particles, {steps} steps, checkpoint every {k}",
            "forward_ms": 1e3 * fwd, "backward_ms": 1e3 * bwd, "ratio": bwd / fwd,
            "forward_ms_per_step": 1e3 * fwd / steps}


def _threads_available() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set."""
    k = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        k = min(k, int(env))
    return max(1, k)


def _cube_subblock(wl):
    """The particles of the periodic cube whose lattice sites lie in the
    corner sub-box [0, L/4)^3, as a periodic box of its own: the same
    positions, velocities, masses, smoothing length and neighbour counts
    (jitter never moves a particle across a lattice-cell boundary, so the
    sub-box tiles periodically like the whole), 1/64 of the particles."""
    import numpy as np
    p, s = wl.params, wl.state
    L = p.hi[0] - p.lo[0]
    n_side = round(s.n ** (1.0 / 3.0))
    dx = L / n_side
    site = np.floor((s.x - np.array(p.lo)[:, None]) / dx).astype(np.int64)
    keep = np.all(site < n_side // 4, axis=0)
    sub_hi = tuple(p.lo[k] + (n_side // 4) * dx for k in range(3))
    ps = p.replace(hi=sub_hi)
    import sph_workloads as W
    ss = W.State(s.x[:, keep].copy(), s.u[:, keep].copy(), s.m[keep].copy(),
                 s.ptype[keep].copy(), np.arange(int(keep.sum()), dtype=np.int32))
    return ps, ss


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 CPU oracle on a bounded sample of the same workload, on one
    thread and on every available host thread (the oracle's OpenMP loops over
    destination particles; results are bitwise the same).  value is the
    all-thread rate."""
    import oracle
    p, s = wl.params, wl.state
    if p.scheme == 1:
        return _cpu_baseline_continuity(wl, budget_s)
    if p.dim == 3 and all(p.periodic[:3]) and s.n > 1 << 20:
        p, s = _cube_subblock(wl)
        what = (f"the {s.n}-particle corner sub-box [0, L/4)^3 of {wl.name} as a periodic box "
                f"(same particles, h and neighbour counts)")
    else:
        what = f"{wl.name} ({s.n} particles)"
    off, _ = oracle.neighbors(p, s.x)
    inter = float(off[-1])
    del off
    threads = _threads_available()
    res = {}
    for k in sorted({1, threads}):
        oracle.set_threads(k)
        t0 = time.perf_counter()
        st = oracle.step(p, s.x, s.u, s.m, s.ptype, 0, prime=True)
        t_prime = time.perf_counter() - t0
        nsteps = min(wl.steps, max(1, int(budget_s / max(t_prime, 1e-3))))
        t0 = time.perf_counter()
        oracle.step(p, st["x"], st["u"], s.m, s.ptype, nsteps, a=st["a"], prime=False)
        dt = time.perf_counter() - t0
        res[k] = (nsteps, dt)
    oracle.set_threads(1)
    nsteps, dt = res[threads]
    n1, dt1 = res[1]
    return {"value": inter * nsteps / dt, "unit": "interactions/s", "cores": threads,
            "kind": "oracle", "ms_per_step": 1e3 * dt / nsteps,
            "one_thread": {"value": inter * n1 / dt1, "ms_per_step": 1e3 * dt1 / n1,
                           "steps": n1},
            "sample": f"{nsteps} predictor-corrector step(s) of {what} from the initial state "
                      f"after a priming evaluation, FP64 oracle on {threads} thread(s); "
                      f"interactions counted at the initial rebuild",
            "cpu": _cpu_model()}


def _cpu_baseline_continuity(wl, budget_s):
    import oracle
    p, s = wl.params, wl.state

    def run(nsteps):
        if p.integrator == 1:  # the example's Euler stage
            oracle.step_continuity(p, s.x, s.u, s.rho, s.m, s.ptype, nsteps)
        else:
            oracle.step_continuity_pc(p, s.x, s.u, s.rho, s.m, s.ptype, nsteps)
    off, _ = oracle.neighbors(p, s.x)
    inter = float(off[-1])
    threads = _threads_available()
    res = {}
    for k in sorted({1, threads}):
        oracle.set_threads(k)
        t0 = time.perf_counter()
        run(1)
        t_one = time.perf_counter() - t0
        nsteps = min(wl.steps, max(1, int(budget_s / max(t_one, 1e-3))))
        t0 = time.perf_counter()
        run(nsteps)
        res[k] = (nsteps, time.perf_counter() - t0)
    oracle.set_threads(1)
    nsteps, dt = res[threads]
    n1, dt1 = res[1]
    return {"value": inter * nsteps / dt, "unit": "interactions/s", "cores": threads,
            "kind": "oracle", "ms_per_step": 1e3 * dt / nsteps,
            "one_thread": {"value": inter * n1 / dt1, "ms_per_step": 1e3 * dt1 / n1,
                           "steps": n1},
            "sample": f"{nsteps} of the {wl.steps} steps of {wl.name} ({s.n} particles) from "
                      f"the initial state, FP64 oracle on {threads} thread(s); interactions "
                      f"counted at the first step's rebuild",
            "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


METRIC = ("particle-neighbour interactions/s + ms/step (FP32 vs FP64); "
          "adjoint/forward ratio")


def summary(res):
    """The timing keys of one precision's run (without the per-kernel detail)."""
    if res is None:
        return None
    return {k: res[k] for k in ("ms_per_step", "interactions_per_s", "interactions")
            if k in res}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube256")
    ap.add_argument("--cell-div", type=int, default=0,
                    help="cells per support radius (default: the workload's)")
    ap.add_argument("--cell-order", choices=("row", "z"), default="row",
                    help="sort key of the cells: row-major or Z-order (3D)")
    ap.add_argument("--nbr-cap", type=int, default=0,
                    help="neighbour-list capacity per particle (0: the library default, "
                         "-1: no lists, every pair pass walks the cells)")
    ap.add_argument("--pair-tiles", type=int, default=0,
                    help="LDS-tiled 3D mixed-precision passes: 0 where they apply, -1 never, "
                         "k > 0 at most k staged particles per tile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the per-field errors against the oracle")
    ap.add_argument("--no-tg512", action="store_true",
                    help="skip the 512^2 Taylor-Green step reported beside the headline")
    ap.add_argument("--tg512-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (8 times), to scale the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiled run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs the hot path on one GPU only; "
              "--gpus must be 1 (multi-GPU slab decomposition is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(8):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 8}), flush=True)
        return

    import paper_1909_04504_amd as sph
    import sph_workloads as W

    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    wl = W.workload(args.workload)
    if args.cell_div:
        wl.params = wl.params.replace(cell_div=args.cell_div)
    if args.cell_order == "z":
        wl.params = wl.params.replace(cell_order=W.Z_ORDER)
    note(f"# workload {wl.name}: {wl.description}; n={wl.state.n}")
    mixed = run_precision(sph, torch, wl, sph.FP32_MIXED, args.steps, args.warmup, True,
                          args.nbr_cap, args.pair_tiles)
    note(f"# fp32-mixed: {mixed['ms_per_step']:.4f} ms/step")
    fp64 = None
    if not args.no_fp64:
        fp64 = run_precision(sph, torch, wl, sph.FP64, args.steps, args.warmup, True,
                             args.nbr_cap)
        note(f"# fp64: {fp64['ms_per_step']:.4f} ms/step")
    rl = roofline(mixed, wl, sph.FP32_MIXED, args.steps, mixed["pair_tests"])
    errors = None
    if not args.no_errors and wl.params.scheme == 0:
        errors = {"fp32_mixed": field_errors(sph, torch, wl, sph.FP32_MIXED)}
        if not args.no_fp64:
            errors["fp64"] = field_errors(sph, torch, wl, sph.FP64)
        note(f"# field errors vs oracle: {json.dumps(errors)}")
    tg = None
    if not args.no_tg512 and wl.name != "tg512":
        wl2 = W.workload("tg512")
        tg = {"workload": wl2.name, "description": wl2.description, "particles": wl2.state.n,
              "steps": args.tg512_steps,
              "fp32_mixed": summary(run_precision(sph, torch, wl2, sph.FP32_MIXED,
                                                  args.tg512_steps, 10, False))}
        if not args.no_fp64:
            tg["fp64"] = summary(run_precision(sph, torch, wl2, sph.FP64, args.tg512_steps,
                                               10, False))
        if not args.no_errors:
            tg["errors"] = {"fp32_mixed": field_errors(sph, torch, wl2, sph.FP32_MIXED)}
            if not args.no_fp64:
                tg["errors"]["fp64"] = field_errors(sph, torch, wl2, sph.FP64)
        note(f"# tg512: {tg['fp32_mixed']['ms_per_step']:.4f} ms/step mixed")
        del wl2
    adj = None
    if not args.no_adjoint:
        adj = adjoint_ratio(sph, torch)
        note(f"# adjoint/forward: {adj['ratio']:.2f}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl)
        note(f"# cpu oracle: {cpu['ms_per_step']:.1f} ms/step on {cpu['cores']} thread(s)")

    out = {
        "metric": METRIC,
        "value": mixed["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair terms + f64 integration",
        "data": "synthetic (" + wl.description + ")",
        "config": {"workload": wl.name, "description": wl.description, "particles": wl.state.n,
                   "kernel": KERNEL_NAMES[wl.params.kernel], "h": wl.params.h,
                   "scheme": ("continuity" if wl.params.scheme == 1 else "summation"),
                   "cell_div": wl.params.cell_div,
                   "cell_order": "z-order" if wl.params.cell_order else "row-major",
                   "rebuild": "every step",
                   "nbr_cap": args.nbr_cap, "pair_tiles": args.pair_tiles},
        "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": rl,
        "fp32_mixed": mixed,
        "fp64": fp64,
        "fp64_ms_per_step": fp64["ms_per_step"] if fp64 else None,
        "fp64_interactions_per_s": fp64["interactions_per_s"] if fp64 else None,
        "fp64_vs_mixed_time": (fp64["ms_per_step"] / mixed["ms_per_step"]) if fp64 else None,
        "errors_vs_oracle": errors,
        "tg512": tg,
        "adjoint_forward_ratio": adj["ratio"] if adj else None,
        "adjoint": adj,
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
        "source_digest": source_digest(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
