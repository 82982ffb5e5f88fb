#!/usr/bin/env python3
"""Benchmark of the WCSPH hot path on one MI355X.

Workload: 2D Taylor-Green vortex, 512 x 512 particles on a lattice jittered by
+-0.1 dx, periodic unit box, Re = 100, cubic spline h = 1.3 dx, Tait EOS
c0 = 10 U, predictor-corrector steps with a neighbour rebuild every step.

A step is one full pass of the hot path: half kick + drift + wrap, cell hash,
counting sort with the stable per-cell rank and state gather, summation
density + EOS, momentum + closing half kick.  Inputs are resident in device
memory before the timed region.

Prints one JSON line.  value = particle-neighbour interactions per second of
the mixed-precision step (pair terms in FP32 on cell-relative offsets, FP64
integration); the full-FP64 step is reported beside it.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
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
PAIR_KERNELS = ("nlist", "density", "momentum", "cont_momentum")
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
    h = hashlib.sha256()
    for f in ("paper_1909_04504_amd/csrc/sph_kernels.hpp", "paper_1909_04504_amd/csrc/sph.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
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


def run_precision(sph, torch, wl, prec, steps, warmup, timing, nbr_cap=0):
    p, s = wl.params, wl.state
    prm = sph.make_params(p, prec, nbr_cap)
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
    """Roofline entry of the dominant kernel of the step."""
    kus = res["kernels_us"]
    launches = res["kernels_launches"]
    per_step = {k: kus[k] * launches[k] / steps for k in kus}
    dom = max(per_step, key=per_step.get)
    avg_s = kus[dom] * 1e-6
    dim, n = wl.params.dim, wl.state.n
    tsize = 4 if prec == 1 else 8
    inter_per_launch = res["interactions_timed"] / steps
    nbytes = bytes_per_particle(dom, dim, tsize, wl.params.scheme == 1) * n
    if dom in PAIR_KERNELS:
        nbytes += 4 * inter_per_launch  # the neighbour lists, written or read once
    if dom in PAIR_KERNELS:
        if dom == "nlist":
            flops = FLOPS_PER_TEST[dim] * tests
        else:
            # the momentum passes do no arithmetic for the self pair
            pairs = inter_per_launch if dom == "density" else inter_per_launch - n
            flops = FLOPS_PER_PAIR[(dom, dim)] * pairs
        intensity = flops / nbytes
        ridge = VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        if intensity >= ridge:
            ach = flops / avg_s / 1e12
            out = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TFLOPS,
                   "unit": "TFLOP/s", "frac": ach / VALU_PEAK_TFLOPS}
        else:
            ach = nbytes / avg_s / 1e9
            out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": ach / HBM_PEAK_GBS}
        out["flops_per_launch"] = flops
    else:
        ach = nbytes / avg_s / 1e9
        out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": ach / HBM_PEAK_GBS}
    out["kernel"] = dom
    out["avg_launch_us"] = kus[dom]
    out["bytes_per_launch"] = nbytes
    out["interactions_per_launch"] = inter_per_launch
    if dom == "nlist":
        out["pair_tests_per_launch"] = tests
    out["traffic"] = traffic_from_profile(dom, wl.name)
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


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 CPU oracle, single-threaded, on a bounded sample of the same
    workload: the first steps from the same initial state."""
    import numpy as np

    import oracle
    p, s = wl.params, wl.state
    if p.scheme == 1:
        return _cpu_baseline_continuity(wl, budget_s)
    t0 = time.perf_counter()
    st = oracle.step(p, s.x, s.u, s.m, s.ptype, 0, prime=True)
    t_prime = time.perf_counter() - t0
    nsteps = min(wl.steps, max(1, int(budget_s / max(t_prime, 1e-3))))
    off, _ = oracle.neighbors(p, st["x"])
    t0 = time.perf_counter()
    oracle.step(p, st["x"], st["u"], s.m, s.ptype, nsteps, a=st["a"], prime=False)
    dt = time.perf_counter() - t0
    inter = float(off[-1]) * nsteps
    return {"value": inter / dt, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "ms_per_step": 1e3 * dt / nsteps,
            "sample": f"{nsteps} of the {wl.steps} steps of {wl.name} ({s.n} particles) from "
                      f"the same initial state, FP64 oracle, 1 thread; interactions counted "
                      f"at the first step's rebuild",
            "cpu": _cpu_model()}


def _cpu_baseline_continuity(wl, budget_s):
    import oracle
    p, s = wl.params, wl.state
    def run(nsteps):
        if p.integrator == 1:  # the example's Euler stage
            oracle.step_continuity(p, s.x, s.u, s.rho, s.m, s.ptype, nsteps)
        else:
            oracle.step_continuity_pc(p, s.x, s.u, s.rho, s.m, s.ptype, nsteps)
    t0 = time.perf_counter()
    run(1)
    t_one = time.perf_counter() - t0
    nsteps = min(wl.steps, max(1, int(budget_s / max(t_one, 1e-3))))
    off, _ = oracle.neighbors(p, s.x)
    t0 = time.perf_counter()
    run(nsteps)
    dt = time.perf_counter() - t0
    inter = float(off[-1]) * nsteps
    return {"value": inter / dt, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "ms_per_step": 1e3 * dt / nsteps,
            "sample": f"{nsteps} of the {wl.steps} steps of {wl.name} ({s.n} particles) from "
                      f"the initial state, FP64 oracle, 1 thread; interactions counted at "
                      f"the first step's rebuild",
            "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tg512")
    ap.add_argument("--cell-div", type=int, default=0,
                    help="cells per support radius (default: the workload's)")
    ap.add_argument("--nbr-cap", type=int, default=0,
                    help="neighbour-list capacity per particle (0: the library default, "
                         "-1: no lists, every pair pass walks the cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
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

    wl = W.workload(args.workload)
    if args.cell_div:
        wl.params = wl.params.replace(cell_div=args.cell_div)
    print(f"# workload {wl.name}: {wl.description}; n={wl.state.n}", file=sys.stderr, flush=True)
    mixed = run_precision(sph, torch, wl, sph.FP32_MIXED, args.steps, args.warmup, True,
                          args.nbr_cap)
    print(f"# fp32-mixed: {mixed['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_precision(sph, torch, wl, sph.FP64, args.steps, args.warmup, True,
                             args.nbr_cap)
        print(f"# fp64: {fp64['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    rl = roofline(mixed, wl, sph.FP32_MIXED, args.steps, mixed["pair_tests"])
    adj = None
    if not args.no_adjoint:
        adj = adjoint_ratio(sph, torch)
        print(f"# adjoint/forward: {adj['ratio']:.2f}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl)
        print(f"# cpu oracle: {cpu['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)

    out = {
        "metric": "particle-neighbour interactions/s (mixed precision step)",
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
                   "cell_div": wl.params.cell_div, "rebuild": "every step",
                   "nbr_cap": args.nbr_cap},
        "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": rl,
        "fp32_mixed": mixed,
        "fp64": fp64,
        "fp64_vs_mixed_time": (fp64["ms_per_step"] / mixed["ms_per_step"]) if fp64 else None,
        "adjoint_forward_ratio": adj["ratio"] if adj else None,
        "adjoint": adj,
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
        "source_digest": source_digest(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
