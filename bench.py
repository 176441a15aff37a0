"""Benchmark: Liouville cell-updates/s of the coupled Maxwell-Liouville-von
Neumann solver on one MI355X.

One benchmark step = one complete simulation of the three-level ladder
(N = 3: 20000 cells, medium on cells [1, 19999), 100000 time steps, pi
Gaussian pulse, Lindblad decay and dephasing) in compensated single
precision: state reset, every time step (H update, Strang Liouville step,
dP/dt, E update, source and boundary) and the recording (probe every step,
E and populations every 10000 steps, written to device memory).  The factors
are built once before timing; the paper's protocol likewise excludes set-up
and includes result storage.

Prints ONE JSON line.  Keys beyond the common ones:
  roofline      the dominant kernel (four-lanes-per-cell tile kernel, N = 3,
                compensated FP32): algorithmic FLOP per launch (medium cells x
                steps per launch x FLOP per cell-update) / average launch
                duration (HIP events on the launch stream over the timed
                region, divided by the number of launches), against the FP32
                vector peak; traffic = HBM bytes per launch from rocprofv3
                counters when they were taken on the current kernel sources
  cpu_baseline  the FP64 oracle on the host cores and on one thread, bounded
                samples of the two-, three- and six-level workloads, median
                of five each
  paper_P       the paper's grid-point metric N_x N_t / t
  variants      the other precisions, routes and workloads, each the median
                of five timed runs after one warm-up; FP64 also on the shape
                the autotuner picks for it; reduced-precision runs report
                their full-length deviation from the GPU FP64 run; the 2-D
                TMz grid (HBM-bound, GB/s against 8 TB/s)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}
REPS = 5  # repetitions of every variant (the median is reported), as the paper times its runs
CSRC = os.path.join(ROOT, "paper_1710_09799_amd", "csrc")
# sources of the dominant kernel; the committed counter summary records their hash
QUAD_SOURCES = ["fwd_quad.hpp", "fwd_impl.hpp", "fwd_kernels.hpp", "fwd_n3.hip"]
# the four-lanes-per-cell kernel each precision runs fastest on at N = 3
# (measured: the matrix-core product wins with the compensated state)
HEAD_VARIANT = {"fp32": "quad", "fp32c": "quad_mfma", "fp32cf": "quad_mfma", "fp32f": "quad"}
# steps per launch with 128-cell tiles (measured best: the matrix-core form
# amortises its launch cost over the most steps that keep one tile per compute
# unit, 250 tiles of 80 owned cells; the DPP form, FP64 included, runs best
# at 20)
HEAD_K = {"quad": 20, "quad_mfma": 24}
KERNEL_DESC = {"quad": "four lanes per cell, shared-factor product by DPP gathers and FMAs",
               "quad_mfma": "four lanes per cell, shared-factor product on the matrix cores "
                            "(two MFMA 16x16x4 f32 per wavefront and step)"}


def traffic_file(precision):
    return os.path.join(ROOT, "profiles", f"fwd_quad_n3_{precision}_three_level_traffic.txt")


def flops_per_update(n):
    """Algorithmic FLOP of one Liouville cell-update in the rotation form:
    merged L1 factor (2 D^2 + D), polarisation (2 D + 1), q 2x2 rotations
    (6 q), Yee updates (7); transcendentals not counted."""
    D, q = n * n - 1, n * (n - 1) // 2
    return 2 * D * D + 3 * D + 6 * q + 8


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TMZ_SOURCES = ["fwd_tmz.hpp", "fwd_impl.hpp", "fwd_kernels.hpp", "tmz.hip"]
STREAM_SOURCES = ["fwd_stream.hpp", "fwd_impl.hpp", "fwd_kernels.hpp", "stream.hip"]


def measured_traffic(precision, path=None, sources=QUAD_SOURCES):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter
    summary (the headline kernel's by default), or None when it is missing or
    was taken on other kernel sources."""
    try:
        kv = {}
        with open(path or traffic_file(precision)) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != source_hash(sources):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_rate(reps=REPS):
    """Device-to-device copy of 1 GiB (torch copy_): GB/s of bytes read plus
    written, the median of `reps` copies, as a practical reference beside the
    8 TB/s HBM peak."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = _events()
    ts = []
    for _ in range(reps):
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del x, y
    return 2 * (1 << 30) / _median(ts) / 1e9


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def time_solver(problem, steps, warmup, snap, keep=False, mean=False, **kw):
    """Time `steps` complete runs (reset + all time steps).  Returns the
    median wall time per run (the mean with mean=True), the matching GPU time
    per run (HIP events on the launch stream), launches per run and, with
    keep=True, the recorded outputs of the last run."""
    import torch
    from paper_1710_09799_amd import mln
    s = mln.Solver(problem, snap_every=snap, **kw)
    for _ in range(warmup):
        s.reset()
        s.run()
    torch.cuda.synchronize()
    e0, e1 = _events()
    walls, gpus = [], []
    for _ in range(steps):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        s.run()  # from step 0: one HIP graph of the run's launches
        e1.record()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        gpus.append(e0.elapsed_time(e1) * 1e-3)
    k = kw.get("steps_per_launch") or s.config()["steps_per_launch"]
    out = None
    if keep:
        out = {key: (v.cpu().numpy() if v is not None else None) for key, v in s.outputs().items()}
    s.close()
    launches = -(-problem.grid.nt // k)
    if mean:
        return sum(walls) / steps, sum(gpus) / steps, launches, out
    return _median(walls), _median(gpus), launches, out


def tuned_config(problem, precision, trial_steps=256):
    """The kernel shape mln_tune picks for this problem and precision."""
    from paper_1710_09799_amd import mln
    s = mln.Solver(problem, precision=precision)
    cfg = s.tune(trial_steps=trial_steps)
    s.close()
    return dict(variant=cfg["variant"], tile=cfg["tile"], steps_per_launch=cfg["steps_per_launch"])


def rel_err(a, b):
    import numpy as np
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def cpu_baseline(reps=REPS):
    """The oracle (FP64 density matrix, OpenMP over cells) on the host's
    cores and on one thread (the paper's CPU protocol), on bounded samples of
    the two-, three- and six-level workloads: the full grids with the run cut
    to a few steps (the metric is size-normalised), median of `reps`
    repetitions each."""
    import oracle
    from paper_1710_09799_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or (os.cpu_count() or 1)

    def rate(p, nt, nthreads):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.run(p, nt=nt, nthreads=nthreads)
            ts.append(time.perf_counter() - t0)
        return p.grid.n_med * nt / _median(ts), _median(ts)

    cases = (("n2_two_level", W.two_level(), 10000, 1000),
             ("n3_three_level", W.three_level(), 1000, 40),
             ("n6_six_level", W.six_level(), 8, 1))
    per = {}
    for name, p, nt, nt1 in cases:
        v, t = rate(p, nt, threads)
        v1, t1 = rate(p, nt1, 1)
        per[name] = {"value": v, "cores": threads,
                     "sample": f"{p.grid.nx} cells (medium {p.grid.n_med}), first {nt} of {p.grid.nt} steps, "
                               f"median of {reps} ({t:.2f} s each)",
                     "single_thread": {"value": v1, "cores": 1,
                                       "sample": f"first {nt1} steps, median of {reps} ({t1:.2f} s each)"}}
    # the rows beyond the one-component 1-D path (all cores; the oracle's PSTD
    # derivative is a direct DFT, O(nx^2) per step)
    p2d = W.three_level_2d()
    pp, e0, h0 = W.pstd_three_level()
    pc, muy, ay = W.cross_ladder()
    extra = (("tmz_2d_beam", p2d, 2, lambda nt: oracle.run2d(p2d, nt=nt, nthreads=threads)),
             ("pstd_ring", pp, 4, lambda nt: oracle.pstd_run(pp, nt=nt, e_init=e0, h_init=h0, nthreads=threads)),
             ("pol2_cross_ladder", pc, 100, lambda nt: oracle.run_pol2(pc, muy, ay, nt=nt, nthreads=threads)))
    for name, p, nt, fn in extra:
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn(nt)
            ts.append(time.perf_counter() - t0)
        t = _median(ts)
        per[name] = {"value": p.grid.n_med * nt / t, "cores": threads,
                     "sample": f"{p.grid.n_med} medium cells, first {nt} of {p.grid.nt} steps, median of {reps} "
                               f"({t:.2f} s each)"}
    head = per["n3_three_level"]
    return {"value": head["value"], "unit": "Liouville cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "three-level ladder on the full 20000-cell grid, " + head["sample"] +
                      "; FP64 density-matrix oracle, OpenMP over cells",
            "single_thread": head["single_thread"], "per_config": per}


ADJ_KW = dict(precision="fp32c", variant="quad_mfma", tile=128, steps_per_launch=24)


def adjoint_legs(reps):
    """The adjoint workload (three-level ladder, 10000 cells x 50000 steps,
    compensated FP32) with checkpoints every 500 steps (the gradient pass
    recomputes each segment) and with the whole forward tape in device
    memory; medians of `reps` forward runs and gradient passes, against the
    plain forward run."""
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    pa = W.adjoint_case()
    akw = ADJ_KW
    t_plain, _, _, _ = time_solver(pa, reps, 1, 0, record_pop=False, record_e=False, **akw)
    res = {}
    for name, ck in (("adjoint_fp32c", 500), ("adjoint_fp32c_whole_tape", "tape")):
        s = mln.Solver(pa, ckpt_every=ck, **akw)
        s.run()
        s.grad(2 * pa.grid.dt * s.probe.cpu().numpy())  # warm-up (allocates the adjoint buffers)
        tfs, tgs = [], []
        for _ in range(reps):
            s.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = s.run()
            torch.cuda.synchronize()
            tfs.append(time.perf_counter() - t0)
            gp = 2 * pa.grid.dt * out["probe"].cpu().numpy()
            t0 = time.perf_counter()
            s.grad(gp)
            tgs.append(time.perf_counter() - t0)
        s.close()
        tf, tg = _median(tfs), _median(tgs)
        r = {"forward_ms": t_plain * 1e3, ("forward_with_checkpoints_ms" if ck == 500 else "forward_with_tape_ms"):
             tf * 1e3, "grad_ms": tg * 1e3, "grad_over_forward": tg / t_plain, "total_over_forward": (tf + tg) / t_plain}
        if ck == 500:
            r["workload"] = "three-level ladder, 10000 cells, 50000 steps, checkpoint every 500"
        else:
            r["tape_GB"] = 9 * 10048 * pa.grid.nt * 4 / 1e9
            r["workload"] = "three-level ladder, 10000 cells, 50000 steps, whole tape in device memory"
        res[name] = {**r, **akw}
    return res


def variants(p3, ref64, pop64, headline):
    """The other configurations of the metric, one warm-up and one timed run
    each."""
    import numpy as np
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    var = {}
    n3 = p3.grid.n_med * p3.grid.nt
    # N = 3: precisions on the four-lanes-per-cell kernel, and the paper's
    # two routes (and the rotation form) on the one-cell-per-thread kernel
    others = [pr for pr in ("fp32", "fp32c", "fp32cf", "fp32f") if pr != headline]
    for name, kw in tuple((f"n3_{pr}_{HEAD_VARIANT[pr]}", dict(precision=pr, variant=HEAD_VARIANT[pr], tile=128,
                                                                steps_per_launch=HEAD_K[HEAD_VARIANT[pr]]))
                          for pr in others) + (
                     ("n3_fp64_block_rotation", dict(precision="fp64", variant="block", route="rotation",
                                                     tile=256, steps_per_launch=32)),
                     ("n3_fp64_block_diag", dict(precision="fp64", variant="block", route="diag",
                                                 tile=256, steps_per_launch=32)),
                     ("n3_fp64_block_rodrigues", dict(precision="fp64", variant="block", route="rodrigues",
                                                      tile=256, steps_per_launch=32))):
        t, g, nl, out = time_solver(p3, REPS, 1, 10000, keep=True, **kw)
        e = np.concatenate([out["probe"], out["e_snap"].ravel()])
        var[name] = {"value": n3 / t, "ms": t * 1e3, "launch_ms": g * 1e3 / nl,
                     "err_E_vs_fp64": rel_err(e, ref64),
                     "err_pop_vs_fp64": float(np.max(np.abs(out["pop"] - pop64))), **kw}
    # the paper's comparison of the exponential routes (Sec. 5.3): the per-step
    # Pade route against diagonalisation and Rodrigues, and the rotation form,
    # all FP64 on the one-cell-per-thread kernel (tile 256, 32 steps per launch)
    # The paper's own two-level and three-level cases on their printed grid
    # (Sec. 5.1, 5.2: 32768 cells, 24559 steps to 187.5 fs; stand-in density,
    # medium and pulse) are timed too, with the paper's metric P = Nx Nt / t
    # beside the Liouville rate.
    p2 = W.two_level()
    comp = {}
    for lbl, prob in (("n2_two_level", p2), ("n2_sit_paper_grid", W.sit_paper()),
                      ("n3_song_paper_grid", W.song_paper()), ("n3_three_level", p3)):
        nu = prob.grid.n_med * prob.grid.nt
        rates, paper_p = {}, {}
        for route in ("pade", "diag", "rodrigues", "rotation"):
            t, _, _, _ = time_solver(prob, REPS, 1, 0, precision="fp64", variant="block", route=route, tile=256,
                                     steps_per_launch=32, record_pop=False, record_e=False)
            rates[route] = nu / t
            paper_p[route] = prob.grid.nx * prob.grid.nt / t
        comp[lbl] = {"cell_updates_per_s": rates, "paper_P": paper_p,
                     "speedup_vs_pade": {r: rates[r] / rates["pade"] for r in ("diag", "rodrigues", "rotation")}}
    # N = 6 (the paper leaves many-level behaviour open): the six-level grid,
    # a 512-step sample of its run; the Pade route on its one-wavefront-per-
    # cell kernel (tile 128, 8 steps per launch), the others as above with 16
    # steps per launch
    p6s = W.six_level(nt=512)
    nu = p6s.grid.n_med * p6s.grid.nt
    rates = {}
    for route in ("pade", "diag", "rodrigues", "rotation"):
        tk = dict(tile=128, steps_per_launch=8) if route == "pade" else dict(tile=256, steps_per_launch=16)
        t, _, _, _ = time_solver(p6s, REPS, 1, 0, precision="fp64", variant="block", route=route,
                                 record_pop=False, record_e=False, **tk)
        rates[route] = nu / t
    comp["n6_six_level_512_step_sample"] = {
        "cell_updates_per_s": rates,
        "speedup_vs_pade": {r: rates[r] / rates["pade"] for r in ("diag", "rodrigues", "rotation")}}
    comp["paper_speedup_vs_pade_single_cpu_thread"] = {"n2": {"diag": 1.26, "rodrigues": 3.48},
                                                      "n3": {"diag": 1.55, "rodrigues": 7.35}}
    var["route_comparison"] = comp
    # N = 6: six-level region, 50000 cells x 200000 steps.  Rates are the
    # median of REPS runs of a 40000-step sample of the full grid (every
    # launch of the run is alike; the metric is size-normalised); each
    # precision's deviation from FP64 is taken over one full-length run.
    p6 = W.six_level()
    p6t = W.six_level(nt=40000)
    n6 = p6t.grid.n_med * p6t.grid.nt
    ref6 = None
    blk = dict(variant="block", tile=256, steps_per_launch=16)
    cfg6 = tuned_config(W.six_level(nt=2048), "fp64")
    for name, kw in (("n6_fp64", dict(precision="fp64", **blk)),
                     ("n6_fp64_tuned", dict(precision="fp64", **cfg6)),
                     ("n6_fp32", dict(precision="fp32", **blk)),
                     ("n6_fp32c", dict(precision="fp32c", **blk)),
                     ("n6_fp32cf", dict(precision="fp32cf", **blk)),
                     ("n6_bf16x6_mfma", dict(precision="bf16x6", tile=256)),
                     ("n6_bf16x3_mfma", dict(precision="bf16x3", tile=256))):
        t, g, nl, _ = time_solver(p6t, REPS, 1, 0, record_pop=False, record_e=False, **kw)
        rec = {"value": n6 / t, "ms_40000_steps": t * 1e3, "launch_ms": g * 1e3 / nl,
               "tflops": n6 * flops_per_update(6) / g / 1e12, **kw}
        if name != "n6_fp64_tuned":
            _, _, _, out = time_solver(p6, 1, 0, 0, keep=True, record_pop=False, record_e=False, **kw)
            if ref6 is None:
                ref6 = out["probe"]
            else:
                rec["err_E_vs_fp64_full_length"] = rel_err(out["probe"], ref6)
        var[name] = rec
    best64 = max(var["n6_fp64"]["value"], var["n6_fp64_tuned"]["value"])
    var["n6_speedup_vs_best_fp64"] = {k: var[k]["value"] / best64
                                      for k in ("n6_fp32", "n6_fp32c", "n6_fp32cf", "n6_bf16x6_mfma",
                                                "n6_bf16x3_mfma")}
    # N = 2: the two-level 2-pi sech workload (2000 cells x 10000 steps, FP64)
    p2 = W.two_level()
    t, g, nl, _ = time_solver(p2, REPS, 1, 1000, precision="fp64", variant="quad", tile=128)
    var["n2_fp64_two_level"] = {"value": p2.grid.n_med * p2.grid.nt / t, "ms": t * 1e3,
                                "launch_ms": g * 1e3 / nl, "shape": "quad, tile 128, automatic steps per launch"}
    var["n2_large"] = n2_large()
    # batched: 64 independent problems (N = 2 and 3 mixed, 1000..30000 cells,
    # 20000 steps), tiles autotuned on the compensated-FP32 batch, whole run
    # replayed from one HIP graph; every precision at the tuned shape, with
    # its largest deviation from the FP64 batch over all 64 problems
    import torch
    probs = W.batched_sweep()
    nts = probs[0].grid.nt
    nb = sum(p.grid.n_med for p in probs) * nts
    b = mln.Batch(probs, precision="fp32c", snap_every=nts)
    variant, tile, k = b.tune(trial_steps=256)
    b.close()
    bat = {"tuned": {"variant": variant, "tile": tile, "steps_per_launch": k}}
    outs = {}
    for prec in ("fp64", "fp32", "fp32c", "fp32cf", "fp32f"):
        b = mln.Batch(probs, precision=prec, snap_every=nts, variant=variant, tile=tile, steps_per_launch=k)
        b.run()
        tbs = []
        for _ in range(REPS):
            b.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = b.run()
            torch.cuda.synchronize()
            tbs.append(time.perf_counter() - t0)
        tb = _median(tbs)
        outs[prec] = [{kk: (v.cpu().numpy() if v is not None else None) for kk, v in oi.items()} for oi in o]
        bat[prec] = {"value": nb / tb, "ms": tb * 1e3, "workgroups": b.config()["workgroups"]}
        b.close()
        if prec != "fp64":
            eE, eP = [], []
            for oi, ri in zip(outs[prec], outs["fp64"]):
                e = np.concatenate([oi["probe"], oi["e_snap"].ravel()])
                er = np.concatenate([ri["probe"], ri["e_snap"].ravel()])
                eE.append(rel_err(e, er))
                eP.append(float(np.max(np.abs(oi["pop"] - ri["pop"]))))
            bat[prec]["max_err_E_vs_fp64"] = max(eE)
            bat[prec]["max_err_pop_vs_fp64"] = max(eP)
    var["batched_64"] = bat
    var.update(adjoint_legs(REPS))
    return var


def tmz_beam(reps=REPS):
    """Two-dimensional TMz grid (the scheme beyond the paper's 1-D models):
    the three-level ladder on 2048 x 512 cells (medium 1536 x 512), a
    Gaussian beam carrying a 50 fs pi pulse, 4096 steps, one launch per step
    (the Bloch state is streamed from and to HBM every step: the HBM-bound
    form).  GB/s are algorithmic: every cell's E_z, H_x, H_y and every medium
    cell's state read and written once per step; the median of `reps` runs."""
    import numpy as np
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    p = W.three_level_2d()
    g = p.grid
    D = p.medium.n_levels ** 2 - 1
    cells = g.nx * g.ny
    out = {"workload": f"three-level ladder on a {g.nx} x {g.ny} TMz grid (medium {g.mx1 - g.mx0} x "
                       f"{g.my1 - g.my0}), {g.nt} steps, Gaussian beam, 50 fs pi pulse",
           "kernel": "fwd_tmz_kernel (64 x 4 cells per workgroup, one launch per step)"}
    rec = {}
    for prec, rs, rows in (("fp64", 8, D), ("fp32", 4, D), ("fp32c", 4, 2 * D)):
        s = mln.Tmz(p, precision=prec, snap_every=g.nt // 2, record_e=False)
        s.run()
        e0, e1 = _events()
        walls, gpus = [], []
        for _ in range(reps):
            s.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record()
            s.step(g.nt)
            e1.record()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            gpus.append(e0.elapsed_time(e1) * 1e-3)
        s.reset()
        o = s.run()
        rec[prec] = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
        s.close()
        t, gt = _median(walls), _median(gpus)
        byts = (cells * 3 * 2 + g.n_med * rows * 2) * rs
        us = gt / g.nt * 1e6
        out[prec] = {"value": g.n_med * g.nt / t, "paper_P": cells * g.nt / t, "us_per_step": us,
                     "alg_bytes_per_step": byts, "alg_GBps": byts / (us * 1e-6) / 1e9,
                     "hbm_frac": byts / (us * 1e-6) / 8e12}
        tf = os.path.join(ROOT, "profiles", f"fwd_tmz_n3_{prec}_2d_beam_traffic.txt")
        if os.path.exists(tf):
            out[prec]["traffic_bytes_per_step"] = measured_traffic(prec, tf, TMZ_SOURCES)
        if prec != "fp64":
            out[prec]["err_probe_vs_fp64"] = rel_err(rec[prec]["probe"], rec["fp64"]["probe"])
            out[prec]["err_pop_vs_fp64"] = float(np.max(np.abs(rec[prec]["pop"] - rec["fp64"]["pop"])))
    out["speedup_vs_fp64"] = {k: out[k]["value"] / out["fp64"]["value"] for k in ("fp32", "fp32c")}
    return out


def pol2_cross_ladder(reps=REPS):
    """Both transverse field components (mln_pol2_*, FP64): the three-level
    ladder with mu01 on E_z and mu12 on E_y (workloads.cross_ladder), 20000
    cells x 20000 steps; the library's default shape (four lanes per cell,
    automatic steps per launch: 24 here) is the value, beside the blocked
    one-lane kernel and the one-step kernel (one launch per step).  GB/s are
    the one-step kernel's algorithmic traffic: every cell's E_z, H_y, E_y,
    H_z and every medium cell's Bloch vector read and written once per step;
    the median of `reps` runs."""
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    p, muy, amp_y = W.cross_ladder()
    g = p.grid
    D = p.medium.n_levels ** 2 - 1

    def timed(k, lanes):
        s = mln.Pol2(p, muy, amp_y, record_pop=False, record_e=False, steps_per_launch=k, lanes_per_cell=lanes)
        s.run()
        e0, e1 = _events()
        walls, gpus = [], []
        for _ in range(reps):
            s.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record()
            s.step(g.nt)
            e1.record()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            gpus.append(e0.elapsed_time(e1) * 1e-3)
        s.close()
        return _median(walls), _median(gpus)

    t, gt = timed(0, 4)
    tl, gtl = timed(0, 1)
    t1, gt1 = timed(1, 1)
    us, usl, us1 = gt / g.nt * 1e6, gtl / g.nt * 1e6, gt1 / g.nt * 1e6
    byts = (g.nx * 4 * 2 + g.n_med * D * 2) * 8
    return {"workload": f"three-level ladder, mu01 on E_z and mu12 on E_y, {g.nx} cells, {g.nt} steps",
            "kernel": "fwd_pol2_quad_kernel (four lanes per cell, 128-cell windows, 79 owned, "
                      "24 steps per launch)",
            "value": g.n_med * g.nt / t, "us_per_step": us, "dtype": "f64",
            "one_lane_kernel": {"kernel": "fwd_pol2_tile_kernel (one thread per cell, 256-cell windows, "
                                          "127 owned, 64 steps per launch)",
                                "value": g.n_med * g.nt / tl, "us_per_step": usl},
            "one_step_kernel": {"kernel": "fwd_pol2_kernel (one launch per step)",
                                "value": g.n_med * g.nt / t1, "us_per_step": us1,
                                "alg_bytes_per_step": byts, "alg_GBps": byts / (us1 * 1e-6) / 1e9,
                                "hbm_frac": byts / (us1 * 1e-6) / 8e12}}


def pstd_ring():
    """Pseudo-spectral field solver (one workgroup per problem): the
    three-level ladder on a periodic ring of 2048 cells of lambda0/8 (medium
    1024 cells), 8192 steps, alone and as a batch of 256 problems (one per
    compute unit, densities 0.5e24 .. 1.5e24 /m^3); the field-only step time
    (one medium cell) separates the FFT pair from the Liouville step."""
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    p, e0, h0 = W.pstd_three_level()
    g = p.grid

    def timed(s, steps):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    out = {"workload": "three-level ladder on a periodic ring, 2048 cells of lambda0/8 (medium 1024), "
                       "8192 steps, Courant 0.5, pi pulse 50 fs FWHM as the initial field", "precision": "fp64"}
    s = mln.Pstd([p], e_init=e0, h_init=h0, steps_per_launch=256, record_pop=False, record_e=False)
    timed(s, 256)
    t = timed(s, g.nt)
    out["single"] = {"value": g.n_med * g.nt / t, "us_per_step": t / g.nt * 1e6, **s.config()}
    s.close()
    g1 = W.Grid(nx=g.nx, nt=g.nt, dx=g.dx, dt=g.dt, med_begin=1, med_end=2)
    s = mln.Pstd([W.Problem("fields", p.medium, g1, p.source)], e_init=e0, h_init=h0, steps_per_launch=256,
                 record_pop=False, record_e=False)
    timed(s, 256)
    out["single"]["fields_only_us_per_step"] = timed(s, g.nt) / g.nt * 1e6
    s.close()
    n = 256
    probs = [W.Problem(p.name, W.ladder_medium([0.0, W.HBAR * W.OMEGA0, 2.1 * W.HBAR * W.OMEGA0],
                                               [1e-29, 0.8e-29], density=1e24 * (0.5 + i / n),
                                               decay=1e12, dephasing=5e12), g, p.source) for i in range(n)]
    s = mln.Pstd(probs, e_init=e0, h_init=h0, steps_per_launch=256, record_pop=False, record_e=False)
    timed(s, 256)
    nt = 2048
    t = timed(s, nt)
    out["batch_256"] = {"value": n * g.n_med * nt / t, "us_per_step": t / nt * 1e6, "steps": nt}
    s.close()
    return out


def n2_large_problem():
    """The two-level medium and pulse on 2^24 cells (medium: the central
    half), 1000 steps: a shape large enough to fill the chip and to make the
    state's HBM traffic visible."""
    from paper_1710_09799_amd import workloads as W
    return W.two_level(nx=1 << 24, nt=1000, name="two_level_2p24")


def n2_large():
    """Two-level, 2^24 cells, FP64, FP32 and compensated FP32: the streamed
    kernel (one step per launch, one thread per cell, no halo: every launch
    reads and writes the whole state, the HBM-bound form), the one-cell-per-
    thread tile kernel at one step per launch (a 1-cell halo) and temporally
    blocked (16 steps per launch).  GB/s are algorithmic: every medium cell's
    state and every cell's E and H read and written once per launch."""
    p = n2_large_problem()
    out = {"workload": "two-level, 2^24 cells (medium 2^23), 1000 steps"}
    for prec, s, rows in (("fp64", 8, 3), ("fp32", 4, 3), ("fp32c", 4, 6)):
        for name, kw in (("stream", dict(variant="stream")),
                         ("k1", dict(variant="block", tile=256, steps_per_launch=1)),
                         ("k16", dict(variant="block", tile=256, steps_per_launch=16))):
            if prec == "fp32c" and name != "stream":
                continue
            t, g, nl, _ = time_solver(p, REPS, 1, 0, precision=prec, record_pop=False, record_e=False, **kw)
            launch = g / nl
            byts = (p.grid.n_med * rows + p.grid.nx * 2) * s * 2
            out[f"{prec}_{name}"] = {"value": p.grid.n_med * p.grid.nt / t, "launch_us": launch * 1e6,
                                     "alg_GBps": byts / launch / 1e9, "hbm_frac": byts / launch / 8e12,
                                     "alg_bytes_per_launch": byts}
    out["fp64_stream"]["traffic_bytes_per_launch"] = measured_traffic(
        "fp64", os.path.join(ROOT, "profiles", "fwd_stream_n2_two_level_2p24_traffic.txt"), STREAM_SOURCES)
    return out


def calib_copy():
    """A 1 GiB device-to-device copy: reads and writes 2^30 bytes, the
    reference that maps the HBM counters to bytes."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    return x.numel() * 4


# Single workloads for hardware-counter runs: (problem, solver options).  The
# six-level cases run a 1600-step sample of the 200000-step run on the full
# 50000-cell grid (every launch is alike).
PROFILE_CASES = {
    "n2_fp64": ("two_level", {}, dict(precision="fp64", variant="quad", tile=128)),
    "n3_fp64": ("three_level", dict(nt=20000), dict(precision="fp64", variant="quad", tile=128, steps_per_launch=20)),
    "n3_fp32c": ("three_level", dict(nt=20000), dict(precision="fp32c", variant="quad_mfma", tile=128,
                                                   steps_per_launch=24)),
    "n3_fp32c_dpp": ("three_level", dict(nt=20000), dict(precision="fp32c", variant="quad", tile=128,
                                                       steps_per_launch=20)),
    "n6_fp64": ("six_level", dict(nt=1600), dict(precision="fp64", variant="block", tile=256, steps_per_launch=16)),
    "n6_bf16x6": ("six_level", dict(nt=1800), dict(precision="bf16x6", tile=256, steps_per_launch=30)),
    "n6_bf16x3": ("six_level", dict(nt=1800), dict(precision="bf16x3", tile=256, steps_per_launch=30)),
    "n2_large_fp64_stream": ("n2_large", {}, dict(precision="fp64", variant="stream")),
    "n2_large_fp32_stream": ("n2_large", {}, dict(precision="fp32", variant="stream")),
    "n2_large_fp64_k1": ("n2_large", {}, dict(precision="fp64", variant="block", tile=256, steps_per_launch=1)),
    "n2_large_fp64_k16": ("n2_large", {}, dict(precision="fp64", variant="block", tile=256, steps_per_launch=16)),
    "n2_large_fp32_k1": ("n2_large", {}, dict(precision="fp32", variant="block", tile=256, steps_per_launch=1)),
    "n2_large_fp32_k16": ("n2_large", {}, dict(precision="fp32", variant="block", tile=256, steps_per_launch=16)),
    # pseudo-spectral ring (2048 cells, 2048 of its 8192 steps): the problem
    # alone, its field part alone (one medium cell), and 256 problems at once
    # the 64-problem sweep at the shape the autotuner picks (one cell per
    # thread, tile 256, 16 steps per launch), 2048 of its 20000 steps
    "batch64_fp64": ("batch", dict(nt=2048), dict(precision="fp64", variant="block", tile=256, steps_per_launch=16)),
    "batch64_fp32c": ("batch", dict(nt=2048), dict(precision="fp32c", variant="block", tile=256, steps_per_launch=16)),
    # the 2-D TMz beam workload (2048 x 512 cells), 512 of its 4096 steps
    "tmz_fp64": ("tmz", dict(nt=512), dict(precision="fp64")),
    "tmz_fp32": ("tmz", dict(nt=512), dict(precision="fp32")),
    "tmz_fp32c": ("tmz", dict(nt=512), dict(precision="fp32c")),
    # both transverse components (cross-polarised ladder, 20000 cells), 4000 steps
    "pol2_fp64": ("pol2", dict(nt=4000, k=24, lanes=4), {}),
    "pol2_fp64_one_lane": ("pol2", dict(nt=4000, k=64, lanes=1), {}),
    "pol2_fp64_one_step": ("pol2", dict(nt=4000, k=1, lanes=1), {}),
    "pstd_n3_ring": ("pstd", dict(batch=1, med=True), dict(steps_per_launch=256)),
    "pstd_n3_ring_fields": ("pstd", dict(batch=1, med=False), dict(steps_per_launch=256)),
    "pstd_n3_ring_batch256": ("pstd", dict(batch=256, med=True), dict(steps_per_launch=256)),
}


def profile_batch(name, nt, kw, steps, warmup):
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    probs = W.batched_sweep(nt=nt)
    b = mln.Batch(probs, snap_every=0, record_pop=False, record_e=False, graph=False, **kw)
    ts = []
    for r in range(warmup + steps):
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        if r >= warmup:
            ts.append(time.perf_counter() - t0)
    cfg = b.config()
    b.close()
    t = min(ts)
    nu = sum(p.grid.n_med for p in probs) * nt
    print(json.dumps({"profile_case": name, "problems": len(probs), "nt": nt, "cell_updates": nu,
                      "ms_per_run": t * 1e3, "cell_updates_per_s": nu / t, **cfg}))


def profile_pstd(name, batch, med, steps_per_launch, steps, warmup):
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    p, e0, h0 = W.pstd_three_level(nt=2048)
    g = p.grid
    if not med:
        g = W.Grid(nx=g.nx, nt=g.nt, dx=g.dx, dt=g.dt, med_begin=1, med_end=2)
    probs = [W.Problem(p.name, W.ladder_medium([0.0, W.HBAR * W.OMEGA0, 2.1 * W.HBAR * W.OMEGA0],
                                               [1e-29, 0.8e-29], density=1e24 * (0.5 + i / batch),
                                               decay=1e12, dephasing=5e12), g, p.source) for i in range(batch)]
    s = mln.Pstd(probs, e_init=e0, h_init=h0, steps_per_launch=steps_per_launch, record_pop=False,
                 record_e=False)
    ts = []
    for r in range(warmup + steps):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(g.nt)
        torch.cuda.synchronize()
        if r >= warmup:
            ts.append(time.perf_counter() - t0)
    s.close()
    t = min(ts)
    print(json.dumps({"profile_case": name, "nx": g.nx, "nt": g.nt, "n_med": g.n_med, "problems": batch,
                      "launches_per_run": -(-g.nt // steps_per_launch), "ms_per_run": t * 1e3,
                      "us_per_step": t / g.nt * 1e6, "cell_updates_per_s": batch * g.n_med * g.nt / t}))


def profile_tmz(name, nt, precision, steps, warmup):
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    p = W.three_level_2d(nt=nt)
    s = mln.Tmz(p, precision=precision, record_pop=False, record_e=False)
    ts = []
    for r in range(warmup + steps):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(nt)
        torch.cuda.synchronize()
        if r >= warmup:
            ts.append(time.perf_counter() - t0)
    s.close()
    t = _median(ts)
    g = p.grid
    print(json.dumps({"profile_case": name, "nx": g.nx, "ny": g.ny, "nt": nt, "n_med": g.n_med,
                      "launches_per_run": nt, "ms_per_run": t * 1e3, "us_per_step": t / nt * 1e6,
                      "cell_updates_per_s": g.n_med * nt / t, "precision": precision}))


def profile_pol2(name, nt, steps, warmup, k, lanes):
    import torch
    from paper_1710_09799_amd import mln
    from paper_1710_09799_amd import workloads as W
    p, muy, amp_y = W.cross_ladder(nt=nt)
    s = mln.Pol2(p, muy, amp_y, record_pop=False, record_e=False, steps_per_launch=k, lanes_per_cell=lanes)
    ts = []
    for r in range(warmup + steps):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(nt)
        torch.cuda.synchronize()
        if r >= warmup:
            ts.append(time.perf_counter() - t0)
    s.close()
    t = _median(ts)
    g = p.grid
    print(json.dumps({"profile_case": name, "nx": g.nx, "nt": nt, "n_med": g.n_med, "steps_per_launch": k,
                      "lanes_per_cell": lanes,
                      "ms_per_run": t * 1e3, "us_per_step": t / nt * 1e6, "cell_updates_per_s": g.n_med * nt / t}))


def profile_case(name, steps, warmup, calib):
    from paper_1710_09799_amd import workloads as W
    if name == "adjoint":
        print(json.dumps({"profile_case": name, **adjoint_legs(max(steps, 1))}))
        return
    wl, pkw, kw = PROFILE_CASES[name]
    if wl == "tmz":
        profile_tmz(name, pkw["nt"], kw["precision"], steps, warmup)
        if calib:
            calib_copy()
        return
    if wl == "pstd":
        profile_pstd(name, pkw["batch"], pkw["med"], kw["steps_per_launch"], steps, warmup)
        return
    if wl == "pol2":
        profile_pol2(name, pkw["nt"], steps, warmup, pkw["k"], pkw["lanes"])
        return
    if wl == "batch":
        profile_batch(name, pkw["nt"], kw, steps, warmup)
        return
    p = n2_large_problem() if wl == "n2_large" else getattr(W, wl)(**pkw)
    t, g, nl, _ = time_solver(p, steps, warmup, 0, record_pop=False, record_e=False, **kw)
    if calib:
        calib_copy()
    print(json.dumps({"profile_case": name, "nx": p.grid.nx, "nt": p.grid.nt, "n_med": p.grid.n_med,
                      "launches_per_run": nl, "ms_per_run": t * 1e3, "launch_us": g * 1e6 / nl,
                      "cell_updates_per_s": p.grid.n_med * p.grid.nt / t, **kw}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--precision", default="fp32c", choices=["fp32", "fp32c", "fp32cf"],
                    help="precision of the headline run (the others are reported as variants)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--profile-case", choices=sorted(PROFILE_CASES) + ["adjoint"],
                    help="run only this workload (for hardware counters) and print its timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(the 1-D domain decomposition it would use is described in the design notes); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1710_09799_amd import workloads as W
    torch.cuda.init()
    if args.profile_case:
        profile_case(args.profile_case, args.steps, args.warmup, args.calib_copy)
        return
    p = W.three_level()
    n_upd = p.grid.n_med * p.grid.nt
    K = HEAD_K[HEAD_VARIANT[args.precision]]
    kw = dict(precision=args.precision, variant=HEAD_VARIANT[args.precision], tile=128, steps_per_launch=K)
    t, gpu_t, launches, out = time_solver(p, args.steps, args.warmup, 10000, keep=True, mean=True, **kw)
    value = n_upd / t
    fl = flops_per_update(p.medium.n_levels)
    launch_s = gpu_t / launches
    # units one launch processes: every medium cell advanced by K steps
    per_launch_flop = p.grid.n_med * K * fl
    achieved = per_launch_flop / launch_s
    peak = PEAK["fp32"]
    traffic = measured_traffic(args.precision)
    res = {
        "metric": "Liouville cell-updates/s at N=3,6 (FP32/split vs FP64); adjoint/forward cost",
        "value": value,
        "unit": "Liouville cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "three-level ladder N=3, 20000 cells (medium 19998), 100000 steps, "
                               "pi Gaussian pulse 200 fs FWHM, Lindblad decay + dephasing",
                   "nx": p.grid.nx, "nt": p.grid.nt, "n_med": p.grid.n_med,
                   "precision": {"fp32": "fp32 (single precision, deviation form)",
                                 "fp32c": "fp32c (FP32 with compensated float-float state)",
                                 "fp32cf": "fp32cf (compensated state and fields)"}[args.precision],
                   "kernel": KERNEL_DESC[kw["variant"]], "tile": kw["tile"], "steps_per_launch": K,
                   "launches": "one HIP graph per run"},
        "paper_P": p.grid.nx * p.grid.nt / t,
        # the step is a dependency chain (exchange, rotation, gather, shared
        # factor, E update) that a few hundred tiles cannot hide: the kernel
        # is latency-bound; achieved / peak is against the FP32 vector peak,
        # the step time against its measured floor is in step_latency
        "roofline": {"bound": "latency", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "peak_of": "FP32 vector", "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"fwd_quad_kernel<3,float,{args.precision}"
                               + (",mfma>" if kw["variant"] == "quad_mfma" else ">"), "launch_us": launch_s * 1e6,
                     "flop_per_update": fl, "updates_per_launch": p.grid.n_med * K},
    }
    # the latency floor of a step at the headline's launch shape: one LDS
    # exchange and one workgroup barrier, without and with a 128-long chain of
    # dependent FMAs (about the length of the kernel's per-step chain)
    from paper_1710_09799_amd import mln
    wg = -(-p.grid.nx // (kw["tile"] - 2 * K))
    res["step_latency"] = {"kernel_us_per_step": launch_s * 1e6 / K,
                           "floor_exchange_barrier_us": mln.step_floor(wg, 4 * kw["tile"], 4000, 0),
                           "floor_exchange_barrier_chain128_us": mln.step_floor(wg, 4 * kw["tile"], 4000, 128),
                           "launch_shape": f"{wg} workgroups x {4 * kw['tile']} lanes"}
    # the vector FMA rate the kernels can reach (plain instructions, measured)
    res["measured_fma_tflops"] = {"fp32": mln.fma_rate(False), "fp64": mln.fma_rate(True)}
    res["measured_copy_GBps"] = copy_rate()
    if not args.no_variants:
        # FP64 on the headline's launch shape and on the shape mln_tune picks
        # for FP64; the headline precision's own tuned shape beside it
        t64, g64, nl64, out64 = time_solver(p, REPS, 1, 10000, keep=True, precision="fp64", variant="quad",
                                            tile=kw["tile"], steps_per_launch=HEAD_K["quad"])
        import numpy as np
        e32 = np.concatenate([out["probe"], out["e_snap"].ravel()])
        e64 = np.concatenate([out64["probe"], out64["e_snap"].ravel()])
        res["err_vs_fp64"] = {"err_E": rel_err(e32, e64),
                              "err_pop": float(np.max(np.abs(out["pop"] - out64["pop"]))),
                              "note": "full-length deviation from the FP64 GPU path, which matches the "
                                      "oracle to 1e-10 on every parity shape"}
        var = {"n3_fp64_quad": {"value": n_upd / t64, "ms": t64 * 1e3, "launch_ms": g64 * 1e3 / nl64,
                                "tile": kw["tile"], "steps_per_launch": HEAD_K["quad"]}}
        # the headline precision on the other four-lanes-per-cell product
        # (DPP gathers and FMAs against the matrix cores)
        alt = "quad" if kw["variant"] == "quad_mfma" else "quad_mfma"
        ta, ga, nla, _ = time_solver(p, REPS, 1, 10000, precision=args.precision, variant=alt,
                                     tile=kw["tile"], steps_per_launch=HEAD_K[alt])
        var[f"n3_{args.precision}_{alt}"] = {"value": n_upd / ta, "ms": ta * 1e3, "launch_ms": ga * 1e3 / nla,
                                            "variant": alt, "tile": kw["tile"], "steps_per_launch": HEAD_K[alt]}
        cfg64 = tuned_config(W.three_level(nt=4000), "fp64")
        tt, gt, nlt, _ = time_solver(p, REPS, 1, 10000, precision="fp64", **cfg64)
        var["n3_fp64_tuned"] = {"value": n_upd / tt, "ms": tt * 1e3, "launch_ms": gt * 1e3 / nlt, **cfg64}
        cfgh = tuned_config(W.three_level(nt=4000), args.precision)
        th, gh, nlh, _ = time_solver(p, REPS, 1, 10000, precision=args.precision, **cfgh)
        var[f"n3_{args.precision}_tuned"] = {"value": n_upd / th, "ms": th * 1e3, "launch_ms": gh * 1e3 / nlh,
                                             **cfgh}
        best64 = max(var["n3_fp64_quad"]["value"], var["n3_fp64_tuned"]["value"])
        var[f"n3_speedup_{args.precision}_vs_best_fp64"] = value / best64
        var.update(variants(p, e64, out64["pop"], args.precision))
        var["n3_speedup_vs_best_fp64"] = {
            k: var[k]["value"] / best64 for k in var if k.startswith("n3_fp32") and "value" in var[k]}
        var["tmz_2d_beam"] = tmz_beam()
        var["pol2_cross_ladder"] = pol2_cross_ladder()
        var["pstd_ring"] = pstd_ring()
        res["variants"] = var
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline()
    if args.calib_copy:
        res["calib_copy_bytes"] = calib_copy()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
