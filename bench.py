"""Benchmark: Liouville cell-updates/s of the coupled Maxwell-Liouville-von
Neumann solver on one MI355X.

One benchmark step = one complete simulation of the three-level ladder
workload (20000 cells, medium on cells [1, 19999), 100000 time steps, pi
Gaussian pulse, Lindblad decay and dephasing): state reset, every time step
(H update, Strang Liouville step, dP/dt, E update, source and boundary) and
the recording (probe every step, E and populations every 10000 steps).
Factor set-up happens once before timing (as in the paper's protocol, which
excludes construction and includes result storage).

Prints ONE JSON line.  Extra keys:
  roofline      dominant kernel (the fused tile kernel): algorithmic FLOP per
                launch / average launch time from HIP events on the launch
                stream, against the FP64 (or FP32) vector peak;
  cpu_baseline  the FP64 oracle on the host cores, bounded sample;
  paper_P       the paper's grid-point metric N_x N_t / t;
  variants      other precisions / routes / sizes timed the same way.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}


def flops_per_update(n):
    """Algorithmic FLOP of one Liouville cell-update in the rotation form:
    merged L1 factor (2 D^2 + D), polarisation (2 D + 1), q 2x2 rotations
    (6 q), Yee updates (7); transcendentals not counted."""
    D, q = n * n - 1, n * (n - 1) // 2
    return 2 * D * D + 3 * D + 6 * q + 8


def time_solver(problem, precision, route, steps, warmup, snap, spl=0, tile=0, per_launch=True):
    import torch
    from paper_1710_09799_amd import mln
    s = mln.Solver(problem, precision=precision, route=route, snap_every=snap,
                   steps_per_launch=spl, tile=tile)
    for _ in range(warmup):
        s.reset()
        s.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.reset()
        s.run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    launch_ms = None
    halo = None
    if per_launch:
        # per-launch kernel time with HIP events on the launch stream
        s.reset()
        from paper_1710_09799_amd.mln import load
        import ctypes
        halo = spl if spl > 0 else 32
        nl = min(200, problem.grid.nt // halo)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nl)]
        for a, b in evs:
            a.record()
            s.step(halo)
            b.record()
        torch.cuda.synchronize()
        launch_ms = sum(a.elapsed_time(b) for a, b in evs) / nl
    s.close()
    return t, launch_ms, halo


def cpu_baseline(seconds_target=15.0):
    import oracle
    from paper_1710_09799_amd import workloads as W
    p = W.three_level()
    nt = 3000
    t0 = time.perf_counter()
    oracle.run(p, nt=nt)
    dt = time.perf_counter() - t0
    ups = p.grid.n_med * nt / dt
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": ups, "unit": "Liouville cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"three-level workload, full 20000-cell grid, first {nt} of 100000 steps, "
                      f"FP64 density-matrix oracle with OpenMP over cells ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--route", default="rotation")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(a 1-D domain decomposition is described in DESIGN.md); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1710_09799_amd import workloads as W
    torch.cuda.init()
    p = W.three_level()
    n_upd = p.grid.n_med * p.grid.nt
    t, launch_ms, halo = time_solver(p, args.precision, args.route, args.steps, args.warmup, snap=10000)
    value = n_upd / t
    fl = flops_per_update(p.medium.n_levels)
    # units one launch processes: medium cells x steps per launch
    per_launch_flop = p.grid.n_med * halo * fl
    achieved = per_launch_flop / (launch_ms * 1e-3)
    peak = PEAK["fp64" if args.precision == "fp64" else "fp32"]
    out = {
        "metric": "Liouville cell-updates/s (three-level ladder, N=3)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}.get(args.precision, args.precision),
        "data": "synthetic",
        "config": {"workload": "three-level ladder N=3, 20000 cells, 100000 steps, pi Gaussian pulse",
                   "nx": p.grid.nx, "nt": p.grid.nt, "n_med": p.grid.n_med,
                   "precision": args.precision, "route": args.route, "steps_per_launch": halo},
        "paper_P": p.grid.nx * p.grid.nt / t,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "fwd_tile_kernel", "launch_ms": launch_ms,
                     "flop_per_update": fl},
    }
    if not args.no_variants:
        var = {}
        for prec in ("fp64", "fp32"):
            if prec == args.precision:
                continue
            tv, lm, _ = time_solver(p, prec, args.route, 1, 1, snap=10000)
            var[f"n3_{prec}"] = {"value": n_upd / tv, "ms": tv * 1e3, "launch_ms": lm}
        out["variants"] = var
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
