#!/usr/bin/env python3
"""Benchmark of the coupled lattice-Boltzmann / atom step on one MI355X.

Default workload: the 256^3 periodic D3Q19 lattice (tau = 0.55) with 200,000 atoms in ten
20,000-atom globules, FP32 deviation storage.  One timed "step" is one full coupled step
(atom coupling + spreading, neighbour-list binning, the fused stream/collide sweep, atom
forces and integration), all on the GPU with the inputs resident in HBM.

After W untimed warm-up steps, five runs of exactly K steps are timed (HIP events on the
step's stream, device synchronisation on both sides of each run); the reported step time is
their median.  Prints one JSON line: MLUPS (the value), the step's algorithmic HBM GB/s, the
roofline of the dominant kernel (the sweep, timed live with HIP events on its own stream),
and the CPU oracle timed on a bounded sample of the same workload.
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

METRIC = "MLUPS and HBM GB/s (% roofline) of coupled LB step; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
SWEEP_SRC = [os.path.join(ROOT, "paper_2305_05025_amd", "csrc", f)
             for f in ("lb_sweep.hip", "lattice_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_counters.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes_per_site(storage: str, field: bool, q: int = 19) -> int:
    """Algorithmic bytes of one sweep per site: q populations read + q written."""
    s = 4 if storage == "f32" else 2
    return 2 * q * s + (12 if field else 0)


def source_hash() -> str:
    """Hash of the sweep kernel's sources: counter figures taken on other sources are stale."""
    h = hashlib.sha256()
    for f in SWEEP_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str):
    """HBM bytes per sweep launch from committed rocprofv3 counter runs, if they were taken
    on the current sweep source; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    rec = d.get("%s/%s" % (workload, storage))
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_timing(w, steps: int):
    """Seconds the CPU oracle (FP64, its OpenMP loops) takes for `steps` coupled steps of
    workload `w` from the rest state, buffer allocation and first touch included."""
    import numpy as np
    from oracle import oracle as O
    p = O.params_from_workload(w)
    g = np.zeros(O.pop_shape(p))
    t0 = time.perf_counter()
    O.run(p, g, w.x0, w.v0, w.x0, w.bonds, w.body_force, steps)
    return time.perf_counter() - t0


def cpu_baseline(k: int):
    """The CPU oracle on a bounded sample of the workload: coupled steps of one eighth of the
    lattice (half the extent per axis) holding one 20,000-atom globule of the same
    construction and parameters, so the sample has the workload's mix of sites and atoms.  A
    10-step probe (allocation included, so it overestimates a step) sizes the timed run to
    about 15-20 s of the host's work (10 to 400 steps).
    Reported as site updates per second.  Beside it, the oracle on two whole workloads: the
    32^3 tethered ball over its 100 steps and the first 20 of the 96^3 differentiation
    workload's 200 steps."""
    from oracle import oracle as O
    from workloads import make_workload
    from workloads.gen import globule_workload
    w = make_workload(k)
    if w.n_atoms == 0:
        raise ValueError("cpu_baseline needs a workload with atoms")
    Ls = tuple(max(8, l // 2) for l in w.L)
    n_per = min(w.n_atoms, 20000)
    ws = globule_workload(Ls, 1, n_per, seed=k, tau=w.tau, gamma=w.gamma,
                          name="cpu_sample", k_tether=w.k_tether, k_bond=w.k_bond,
                          r0_bond=w.r0_bond, lj_eps=w.lj_eps, lj_sigma=w.lj_sigma,
                          lj_rc=w.lj_rc, lj_exclude_bonded=w.lj_exclude_bonded,
                          bf_kind=0 if w.bf_kind == 3 else w.bf_kind, bf_amp=w.bf_amp,
                          mass=w.mass)
    probe = oracle_timing(ws, 10) / 10
    steps = int(min(400, max(10, round(20.0 / probe))))
    dt = oracle_timing(ws, steps)
    others = []
    for kk, n in ((0, 100), (3, 20)):
        wk = make_workload(kk)
        t = oracle_timing(wk, n)
        others.append({"workload": wk.name, "steps": n, "seconds": round(t, 2),
                       "mlups": round(wk.n_sites * n / t / 1e6, 2)})
    threads = O.num_threads()
    return {"value": round(ws.n_sites * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": "%d coupled steps of a %dx%dx%d lattice with one %d-atom globule, the "
                      "parameters of %s (FP64, %d threads, %.1f s, allocation included)"
                      % (steps, Ls[0], Ls[1], Ls[2], n_per, w.name, threads, dt),
            "whole_workloads": others}


def cpu_baseline_full():
    """The oracle over the full step counts of the 32^3 ball (100), the 128^3 globule (1000)
    and the 96^3 differentiation workload (200), and 20 steps of the 256^3 workload: one JSON
    line per workload.  Takes tens of minutes; not part of the default run."""
    from oracle import oracle as O
    from workloads import make_workload
    for k, n in ((0, 100), (3, 200), (1, 1000), (2, 20)):
        w = make_workload(k)
        t = oracle_timing(w, n)
        print(json.dumps({"cpu_baseline_workload": w.name, "steps": n, "seconds": round(t, 2),
                          "mlups": round(w.n_sites * n / t / 1e6, 3), "kind": "oracle",
                          "cores": O.num_threads(), "cpu": cpu_model()}), flush=True)


def time_steps(sim, steps: int, warmup: int, reps: int = 5):
    """(median ms per step, wall s of the timed runs, the runs' ms per step): `warmup`
    untimed steps, then `reps` runs of exactly `steps` coupled steps, each bracketed by
    device synchronisation and timed by HIP events on the step's stream; no per-phase
    events are queued."""
    import torch
    sim.step(warmup)
    sim.check()
    runs = []
    wall = 0.0
    for _ in range(reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        ev0.record(sim.stream)
        sim.step(steps)
        ev1.record(sim.stream)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t_start
        sim.check()
        runs.append(ev0.elapsed_time(ev1) / steps)
    runs_sorted = sorted(runs)
    return runs_sorted[len(runs) // 2], wall, runs


def adjoint_ratio(dev, config: int = 3, n_steps: int = 200, k: int = 20):
    """Forward and backward (adjoint with checkpoint-and-recompute) times on the
    differentiation workload (by default: 96^3 lattice, one 5,000-atom globule, body-force
    field, 200 steps, checkpoints every 20 steps)."""
    import numpy as np
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import make_workload
    w = make_workload(config)
    sim = CoupledLB.from_workload(w, device=dev)
    fwd_ms = time_steps(sim, n_steps, 20, reps=3)[0]
    sim.close()
    res = []
    for rep in range(2):      # the first pass includes one-off allocation
        sim = CoupledLB.from_workload(w, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ck = sim.run_checkpointed(n_steps, k)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = sim.displacement().double()
        # the loss of the differentiation workload (a workload without a target shift: D = 0)
        D = torch.tensor(w.target_shift if w.target_shift is not None else [0.0, 0.0, 0.0],
                         dtype=torch.float64, device=dev)
        dLdX = (2.0 * (d - D) / w.n_atoms).float()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g = sim.backward(ck, dLdX)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        sim.close()
        res.append(((t1 - t0) * 1e3, (t3 - t2) * 1e3, g))
    ck_ms, bwd_ms, g = res[-1]
    return {"workload": w.name, "steps": n_steps, "k": k,
            "forward_ms": round(fwd_ms * n_steps, 3),
            "forward_with_checkpoints_ms": round(ck_ms, 3),
            "backward_ms": round(bwd_ms, 3),
            "ratio": round(bwd_ms / (fwd_ms * n_steps), 3),
            "dL_dgamma": g["gamma"], "dL_dtau": g["tau"],
            "dL_db_norm": float(torch.linalg.vector_norm(g["body_force"]).item())}


def run(args):
    import torch
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import make_workload

    dev = torch.device("cuda:0")
    t0 = time.time()
    w = make_workload(args.config)
    log("workload %s: lattice %s, %d atoms, built in %.1f s" % (w.name, w.L, w.n_atoms, time.time() - t0))
    flags = (A.LB_FLAG_SINGLE_STREAM if args.single_stream else 0) | \
        (A.LB_FLAG_STEP_GRAPHS if args.graphs else 0)
    sim = CoupledLB.from_workload(w, storage=args.storage, device=dev, flags=flags)
    # the step: K steps with no per-phase events in the queue
    step_ms, wall, runs = time_steps(sim, args.steps, args.warmup)
    # the kernels: K more steps with HIP events around each phase, on the streams the
    # phases run on
    A.lb_timing_begin(sim.ctx, args.steps)
    sim.step(args.steps)
    sweep_ms, atom_ms, nsteps = A.lb_timing_end(sim.ctx)
    sim.check()
    sim.close()
    log("timed 5 x %d steps: median %.4f ms/step (events; runs %s), wall %.3f s; per step in a "
        "further timed run: sweep kernel %.4f ms, atom kernel chains %.4f ms" %
        (args.steps, step_ms, " ".join("%.4f" % r for r in runs), wall, sweep_ms / nsteps,
         atom_ms / nsteps))
    # the other storage formats, same workload and schedule
    storage_ms = {args.storage: round(step_ms, 5)}
    if args.formats:
        for fmt in ("f32", "f16", "bf16"):
            if fmt in storage_ms:
                continue
            s2 = CoupledLB.from_workload(w, storage=fmt, device=dev, flags=flags)
            storage_ms[fmt] = round(time_steps(s2, args.steps, args.warmup)[0], 5)
            s2.close()
            log("storage %s: %.4f ms/step" % (fmt, storage_ms[fmt]))
    # the thermal (fluctuating) lattice: the same workload with noise on the non-conserved
    # modes at kT = 1e-4 (thermal velocity 0.01 per component)
    thermal = None
    if args.formats:
        import dataclasses
        wt = dataclasses.replace(w, kT=1e-4, noise_seed=7)
        s3 = CoupledLB.from_workload(wt, storage=args.storage, device=dev, flags=flags)
        thermal = {"kT": 1e-4, "ms_per_step": round(time_steps(s3, args.steps, args.warmup)[0], 5)}
        s3.close()
        log("thermal: %s" % thermal)
    # the 27-velocity lattice (D3Q27, the higher-order set): same workload, schedule and
    # storage; its sweep moves 27/19 of the bytes, timed live like the main sweep
    d3q27 = None
    if args.formats:
        import dataclasses
        wq = dataclasses.replace(w, velocity_set=27)
        s4 = CoupledLB.from_workload(wq, storage=args.storage, device=dev, flags=flags)
        ms27 = time_steps(s4, args.steps, args.warmup)[0]
        A.lb_timing_begin(s4.ctx, args.steps)
        s4.step(args.steps)
        sw27, _, n27 = A.lb_timing_end(s4.ctx)
        s4.check()
        s4.close()
        bps27 = sweep_bytes_per_site(args.storage, w.bf_kind == 3, 27)
        d3q27 = {"ms_per_step": round(ms27, 5),
                 "mlups": round(w.n_sites / (ms27 * 1e-3) / 1e6, 1),
                 "sweep_ms": round(sw27 / n27, 5), "bytes_per_site": bps27,
                 "sweep_gbs": round(bps27 * w.n_sites / (sw27 / n27 * 1e-3) / 1e9, 1)}
        log("d3q27: %s" % d3q27)
    adj = None
    if args.adjoint:
        adj = adjoint_ratio(dev)
        log("adjoint: %s" % adj)

    S = w.n_sites
    field = w.bf_kind == 3
    bps = sweep_bytes_per_site(args.storage, field)
    mlups = S / (step_ms * 1e-3) / 1e6
    sweep_avg_s = sweep_ms / nsteps * 1e-3
    achieved = bps * S / sweep_avg_s / 1e9
    # whole-step algorithmic bytes: the sweep plus the atom side (positions, velocities,
    # forces read/written, the coupling gather over each atom's 8 nodes counted once per
    # atom-node pair)
    atom_bytes = w.n_atoms * (4 * 3 * 4 * 2 + 8 * 19 * (4 if args.storage == "f32" else 2))
    step_gbs = (bps * S + atom_bytes) / (step_ms * 1e-3) / 1e9
    traffic = measured_traffic(w.name, args.storage)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 5),
        "ms_per_step_runs": [round(r, 5) for r in runs],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.L), "atoms": w.n_atoms,
                   "storage": args.storage, "tau": w.tau, "steps_per_call": args.steps,
                   "streams": streams_used(w, args.single_stream), "graphs": bool(args.graphs)},
        "hbm_gbs_step": round(step_gbs, 1),
        "hbm_frac_step": round(step_gbs / HBM_PEAK_GBS, 4),
        # summed durations of the atom-side kernel chains (binning, coupling, cell sort +
        # force field), which run beside the sweep, and the sweep's share of the step
        "atom_kernels_ms": round(atom_ms / nsteps, 5),
        "sweep_share": round(sweep_ms / nsteps / step_ms, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_sweep<%s>" % args.storage,
                     "bytes_per_site": bps, "sweep_ms": round(sweep_ms / nsteps, 5)},
        "storage_ms_per_step": storage_ms,
        "f16_speedup": (round(storage_ms["f32"] / storage_ms["f16"], 4)
                        if "f32" in storage_ms and "f16" in storage_ms else None),
        "thermal": thermal,
        "d3q27": d3q27,
        "adjoint_forward_ratio": adj["ratio"] if adj else None,
        "adjoint": adj,
    }
    if args.cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(args.config)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def calibrate_copy(args):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 256 * 1024 * 1024  # floats: 1 GiB each way
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "launches": args.steps}), flush=True)


def streams_used(w, single_stream):
    """The library's schedule: the atom work gets a stream of its own unless asked not to, or
    the lattice is small enough that fewer host calls win (LB_ONE_STREAM_MAX_SITES)."""
    from paper_2305_05025_amd import _abi as A
    sites = w.L[0] * w.L[1] * w.L[2]
    small = sites <= A.LB_ONE_STREAM_MAX_SITES and "LBMD_OVERLAP_SMALL" not in os.environ
    return 1 if single_stream or small or w.n_atoms == 0 else 2


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=2, help="workload 0..4 (2 = 256^3, 200k atoms)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="only time the CPU oracle over whole workloads (tens of minutes)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the forward and backward passes (--adjoint-config, "
                         "--adjoint-steps, --adjoint-k) and print them as JSON")
    ap.add_argument("--adjoint-config", type=int, default=3)
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--adjoint-k", type=int, default=20)
    ap.add_argument("--no-formats", dest="formats", action="store_false",
                    help="skip the FP16/BF16 (or FP32) storage, thermal-noise and D3Q27 timings")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="skip the adjoint/forward timing on the differentiation workload")
    ap.add_argument("--single-stream", action="store_true",
                    help="queue every kernel on one stream (no overlap of atom and lattice work)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the steps from captured HIP graphs (LB_FLAG_STEP_GRAPHS)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU (domain-decomposed) path is not "
              "built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args)
    elif args.cpu_baseline_full:
        cpu_baseline_full()
    elif args.adjoint_only:
        import torch
        print(json.dumps(adjoint_ratio(torch.device("cuda:0"), args.adjoint_config,
                                       args.adjoint_steps, args.adjoint_k)), flush=True)
    else:
        run(args)


if __name__ == "__main__":
    main()
