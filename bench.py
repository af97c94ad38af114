"""Benchmark: WCSPH regional time stepping vs global adaptive stepping on one GPU.

Workload: the 250,000-particle dam break (column 0.5 x 1.0 x 0.5 m at spacing
0.01 m in a 2 x 1 x 1 m box), block levels 0..3, K base steps (default 500).
A step is one base step of the whole path (grid rebuild, block levels, flags,
neighbour search + density, forces, corrector/predictor).

Printed: one JSON line.  ``value`` is RTS particle-steps/s (particles x base
steps / wall seconds, inputs resident in HBM).  The global adaptive
comparator is timed over the same simulated time.  The dominant kernel's
roofline comes from an event-bracketed replay of the same K steps; the CPU
baseline is the FP64 oracle on a bounded window of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, packed FP32 off


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time spent on the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--only-rts", action="store_true",
                    help="time the RTS run only (for profiler runs); prints no JSON line")
    ap.add_argument("--pcisph-steps", type=int, default=200,
                    help="minor steps of the PCISPH double dam break (0: skip it)")
    ap.add_argument("--only-diff", action="store_true",
                    help="run only the differentiable leg (for profiler runs); prints no JSON line")
    ap.add_argument("--only-pcisph", action="store_true",
                    help="run the PCISPH comparison only (for profiler runs); no JSON line")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="base steps of the 64-scene batch and of its sequential runs (0: skip)")
    ap.add_argument("--more-steps", type=int, default=500,
                    help="base steps of the double dam break and block drop legs (0: skip)")
    ap.add_argument("--diff-repeats", type=int, default=3,
                    help="timed forward+backward runs of the differentiable 101k scene (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run an elementwise copy of 256 MiB three times, the "
                         "reference kernel for scaling HBM byte counters")
    return ap.parse_args()


PROFILE_MD = os.path.join(ROOT, "profiles", "wcsph_rts_dam_break_250k_kernels.md")
KERNEL_SOURCES = ("paper_2009_14514_amd/csrc/rts_kernels.hip",
                  "paper_2009_14514_amd/csrc/rts_device.h",
                  "paper_2009_14514_amd/csrc/rts_internal.h")


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(PROFILE_MD).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    m = re.search(r"kernel_sources_sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != h.hexdigest():
        return None
    m = re.search(r"traffic_bytes_per_launch %s: ([0-9.]+)" % re.escape(kernel), text)
    return float(m.group(1)) if m else None


def kernel_traffic(name, n, nb, K, act, inter, cand):
    """Algorithmic bytes and flops per launch of each kernel (averaged over K steps).

    Bytes count the particle state each kernel must read and write plus the
    neighbour bitmasks (one bit per candidate); re-reads of neighbour state
    served by LDS or caches are not counted.  Flops count the float operations
    of the method: 9 per candidate test (3 sub, 1 mul, 2 fma, 1 compare),
    23 per density term (distance 8, sqrt 1, kernel shape 10, compensated
    add 4) and 45 per force term.  ``act``/``inter``/``cand`` are totals over
    the K steps.
    """
    a, i, c = act / K, inter / K, cand / K
    table = {
        "key_hist": (24.0 * n, 10.0 * n),
        "scan": (14.0 * nb, 4.0 * nb),
        "scatter": (16.0 * n, 1.0 * n),
        "cell_gather": (124.0 * n + nb, 16.0 * n),
        "rmin_flags": (12.0 * n + 27.0 * nb, 8.0 * n),
        # own state and flag in; bitmask words, density, p/rho^2, p, count out
        "search_density": (40.0 * a + c / 8.0, 9.0 * c + 23.0 * i),
        # own state, count and bitmask words in; acceleration out
        "force": (52.0 * a + c / 8.0, 45.0 * i),
        "step_stats": (30.0 * nb, 12.0 * nb),
        "correct_predict": (104.0 * n + 16.0 * a, 30.0 * n),
    }
    return table[name]


def run_gpu(args):
    import numpy as np
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.sim import Simulation

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # 256 MiB read and 256 MiB written per launch by one elementwise kernel
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    sc = scenes.dam_break_column()          # 250,000 particles, levels 0..3
    K, W = args.steps, args.warmup
    out = {}

    def timed(sim, steps):
        st = sim.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        sim.advance(steps)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # --- RTS ------------------------------------------------------------------
    rts = Simulation(sc, mode="rts")
    init = rts.save()
    if W:
        rts.advance(W)
        rts.sync()
        rts.load(init)
    ms_rts = timed(rts, K)
    st_rts = rts.sync()
    T = st_rts.time
    print(f"[bench] rts: {K} steps in {ms_rts:.2f} ms, active {st_rts.active_total}, "
          f"err_max {st_rts.err_max_run:.4f}", file=sys.stderr, flush=True)
    if args.only_rts:
        rts.close()
        return None

    # --- global adaptive comparator over the same simulated time ---------------
    ga = Simulation(sc, mode="global_adaptive")
    ga_init = ga.save()
    if W:
        ga.advance(W)
        ga.sync()
        ga.load(ga_init)
    ms_ga = timed(ga, K)
    st_ga = ga.sync()
    while st_ga.time < T * (1.0 - 1e-9):
        ms_ga += timed(ga, 10)
        st_ga = ga.sync()
    print(f"[bench] global adaptive: {st_ga.step} steps in {ms_ga:.2f} ms, "
          f"err_max {st_ga.err_max_run:.4f}", file=sys.stderr, flush=True)

    n = sc.n
    ps_rts = n * K / (ms_rts * 1e-3)
    ps_ga = n * (st_ga.time / st_rts.dt_last) / (ms_ga * 1e-3)
    out.update(
        n=n, nw=sc.nw, K=K, ms_rts=ms_rts, ms_ga=ms_ga, ps_rts=ps_rts, ps_ga=ps_ga,
        sim_time=T, dt_base=st_rts.dt_last,
        rts=dict(active_total=st_rts.active_total, inter_total=st_rts.inter_total,
                 cand_total=st_rts.cand_total, err_max=float(st_rts.err_max_run),
                 level_hist_last=list(st_rts.level_hist)[:4], nbr_max=st_rts.nbr_max),
        ga=dict(steps=st_ga.step, active_total=st_ga.active_total,
                inter_total=st_ga.inter_total, err_max=float(st_ga.err_max_run)),
        nblocks=rts.info["nblocks"],
    )

    # --- per-kernel times: the same K steps, kernels bracketed by HIP events -----
    if not args.no_profile:
        rts.load(init)
        prof = rts.profile(K)
        st_p = rts.sync()
        out["kernels_ms"] = prof
        out["prof_counts"] = dict(active=st_p.active_total, inter=st_p.inter_total,
                                  cand=st_p.cand_total)
    rts.close()
    ga.close()
    return out


def run_pcisph(steps):
    """RTS PCISPH vs standard PCISPH on the 1,000,188-particle double dam break.

    Both arms run the same minor steps from rest (so equal simulated time);
    the correction loop reads its error reductions between iterations, so
    each minor step is timed by wall clock around a completed call.
    """
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.sim import Simulation

    out = {}
    for mode in ("rts", "global_fixed"):
        sc = scenes.double_dam_break()
        sc.params["mode"] = mode
        sim = Simulation(sc)
        sim.advance(1)                       # first major step set-up and lists: warm-up
        sim.sync()
        sim.set_state(sc.pos, sc.vel)        # back to rest
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.advance(steps)
        st = sim.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = dict(n=sc.n, ms=el * 1e3, iters=int(st.pci_iters_total), time=st.time,
                         errmax=float(st.pci_errmax), hist=list(st.level_hist)[:4])
        print(f"[bench] pcisph {mode}: {steps} minor steps in {el * 1e3:.1f} ms, "
              f"{st.pci_iters_total} iterations", file=sys.stderr, flush=True)
        sim.close()
    r, g = out["rts"], out["global_fixed"]
    n = r["n"]
    return {
        "workload": "pcisph_rts_double_dam_break_1m", "n_particles": n, "minor_steps": steps,
        "dt_base_s": 5e-4, "unit": "particle-steps/s",
        "value": n * steps / (r["ms"] * 1e-3), "ms_per_step": r["ms"] / steps,
        "iterations": r["iters"], "density_err_last": r["errmax"],
        "standard_pcisph": {"value": n * steps / (g["ms"] * 1e-3), "ms_per_step": g["ms"] / steps,
                            "iterations": g["iters"], "density_err_last": g["errmax"]},
        "speedup_vs_standard": g["ms"] / r["ms"],
        "adaptive_base_step": run_pcisph_adaptive(steps * 5e-4, r["ms"] / (steps * 5e-4)),
    }


def run_pcisph_adaptive(sim_time, fixed_ms_per_sim_s):
    """Regional PCISPH with the adaptive base step over the same simulated
    time as the fixed-step arms, started from the fixed arms' 5e-4 s and from
    1e-3 s (where fixed-step PCISPH on this scene diverges).  Compared by wall
    time per simulated second, since the steps differ in length."""
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.sim import Simulation

    res = {"sim_time_s": sim_time, "fixed_5e-4_ms_per_sim_s": fixed_ms_per_sim_s}
    for dt0 in (5e-4, 1e-3):
        sc = scenes.double_dam_break(dt_base=dt0)
        sim = Simulation(sc, pci_adapt_dt=1)
        sim.advance(1)
        sim.sync()
        sim.set_state(sc.pos, sc.vel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dts = []
        while True:
            sim.advance(4)
            st = sim.sync()
            dts.append(st.dt_last)
            if st.time >= sim_time * (1.0 - 1e-9):
                break
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[f"from_{dt0:g}"] = dict(
            ms=el * 1e3, sim_time_s=st.time, ms_per_sim_s=el * 1e3 / st.time,
            minor_steps=int(st.step), iterations=int(st.pci_iters_total),
            rollbacks=int(st.pci_rollbacks), dt_min_s=min(dts), dt_max_s=max(dts),
            density_err_last=float(st.pci_errmax),
            speed_vs_fixed_5e_4=fixed_ms_per_sim_s / (el * 1e3 / st.time))
        print(f"[bench] pcisph adaptive from {dt0:g}: {st.time:.4f} s in {el * 1e3:.1f} ms, "
              f"{st.step} steps, {st.pci_iters_total} iterations, {st.pci_rollbacks} roll-backs",
              file=sys.stderr, flush=True)
        sim.close()
    return res


def run_batched(steps):
    """64 dam-break scenes of uneven size advanced together by one graph
    replay per base step (launch shape autotuned), against the same scenes
    run one after another, each by its own context."""
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.sim import Simulation

    sc = scenes.batched_dam_breaks()
    sim = Simulation(sc)
    tune = sim.autotune(steps=3)
    sim.advance(1)
    sim.sync()
    sim.set_state(sc.pos, sc.vel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.advance(steps)
    st = sim.sync()
    ms_batch = (time.perf_counter() - t0) * 1e3
    err = float(st.err_max_run)
    sim.close()
    del sim
    ms_seq = 0.0
    for sub in sc.subscenes:
        one = Simulation(sub)
        one.advance(1)
        one.sync()
        one.set_state(sub.pos, sub.vel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.advance(steps)
        one.sync()
        ms_seq += (time.perf_counter() - t0) * 1e3
        one.close()
    print(f"[bench] batch: {len(sc.subscenes)} scenes, {sc.n} particles, {steps} steps in "
          f"{ms_batch:.1f} ms; sequential {ms_seq:.1f} ms", file=sys.stderr, flush=True)
    return {
        "workload": "wcsph_rts_batch_64_dam_breaks", "n_scenes": len(sc.subscenes),
        "n_particles": sc.n, "base_steps": steps, "unit": "particle-steps/s",
        "value": sc.n * steps / (ms_batch * 1e-3), "ms_per_step": ms_batch / steps,
        "sequential": {"value": sc.n * steps / (ms_seq * 1e-3), "ms_per_step": ms_seq / steps},
        "speedup_vs_sequential": ms_seq / ms_batch, "density_err_max": err,
        "launch_shape": tune,
    }


def run_diff(repeats):
    """Differentiable WCSPH: 101,306-particle dam break (37 x 74 x 37), 16
    substeps of 1e-4 s with checkpoints every 4; forward, then the adjoint
    for L = mean |x(T) - xhat| ^ 2 (gradients in v0, x0, B, alpha)."""
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.diff import DiffRollout

    sc = scenes.diff_scene(counts=(37, 74, 37), box=(2.0, 1.0, 1.0))
    model = DiffRollout(sc, n_sub=16, ckpt_every=4)
    x0 = torch.tensor(sc.pos, dtype=torch.float32, device="cuda")
    v0 = torch.tensor(sc.vel, dtype=torch.float32, device="cuda")
    xT, _ = model.forward(x0, v0, model.B0, model.alpha0)      # nominal run: the target
    xhat = xT + torch.tensor(scenes.target_noise(sc.n, sc.params["target_sigma"]),
                             dtype=torch.float32, device="cuda")
    fw, bw = [], []
    for _ in range(max(repeats, 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xT, _ = model.forward(x0, v0, model.B0, model.alpha0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gx, gv, gB, ga = model.backward(2.0 * (xT - xhat) / sc.n)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fw.append(t1 - t0)
        bw.append(t2 - t1)
    model.close()
    f, b = min(fw) * 1e3, min(bw) * 1e3
    print(f"[bench] differentiable: forward {f:.2f} ms, backward {b:.2f} ms", file=sys.stderr,
          flush=True)
    return {"workload": "wcsph_diff_dam_break_101k_16_substeps", "n_particles": sc.n,
            "substeps": 16, "checkpoint_every": 4, "forward_ms": f, "backward_ms": b,
            "unit": "particle-substeps/s",
            "value": sc.n * 16 / ((f + b) * 1e-3),
            "grad_norms": {"v0": float(gv.norm()), "x0": float(gx.norm()), "B": gB,
                           "alpha": ga}}


def run_more_wcsph(steps):
    """The paper's other WCSPH scenes as synthetic stand-ins: a double dam
    break (256,000 particles) and a dam break with a dropped block (177,000);
    regional vs global adaptive stepping over the same simulated time."""
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.sim import Simulation

    def run(sim, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.advance(k)
        st = sim.sync()
        return (time.perf_counter() - t0) * 1e3, st

    out = {}
    for name, make in (("wcsph_double_dam_break_256k", scenes.wcsph_double_dam_break),
                       ("wcsph_block_drop_177k", scenes.block_drop)):
        sc = make()
        rts = Simulation(sc, mode="rts")
        init = rts.save()
        rts.advance(10)
        rts.sync()
        rts.load(init)
        ms_r, st_r = run(rts, steps)
        ga = Simulation(sc, mode="global_adaptive")
        ms_g, st_g = run(ga, steps)
        while st_g.time < st_r.time * (1.0 - 1e-9):
            m, st_g = run(ga, 10)
            ms_g += m
        out[name] = {"n_particles": sc.n, "base_steps": steps,
                     "value": sc.n * steps / (ms_r * 1e-3), "unit": "particle-steps/s",
                     "density_err_max": float(st_r.err_max_run),
                     "global_adaptive_err_max": float(st_g.err_max_run),
                     "speedup_vs_global_adaptive": ms_g / ms_r}
        print(f"[bench] {name}: rts {ms_r:.1f} ms, global adaptive {ms_g:.1f} ms",
              file=sys.stderr, flush=True)
        rts.close()
        ga.close()
    return out


def run_cpu_baseline(budget_s):
    """FP64 oracle, RTS mode, on the first steps of the same workload."""
    import numpy as np

    import oracle
    from paper_2009_14514_amd import scenes

    sc = scenes.dam_break_column()
    sim = oracle.WCSPH(sc.params, sc.pos.astype(np.float32), walls=sc.walls.astype(np.float32),
                       mode="rts")
    t0 = time.time()
    steps = 0
    while True:
        sim.step()
        steps += 1
        el = time.time() - t0
        if el >= budget_s or steps >= 500:
            break
    return dict(value=sc.n * steps / el, unit="particle-steps/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"first {steps} RTS base steps of the 250,000-particle dam break "
                       f"(FP64, {el:.1f} s)")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU slab decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)
    if args.only_pcisph:
        run_pcisph(args.pcisph_steps)
        return
    if args.only_diff:
        run_diff(args.diff_repeats)
        return
    g = run_gpu(args)
    if g is None:
        return
    K = g["K"]
    line = {
        "metric": "particle-steps/s RTS vs global dt on 1 MI355X at <=1% density error; HBM GB/s",
        "value": g["ps_rts"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": g["ms_rts"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "wcsph_rts_dam_break_250k", "n_particles": g["n"],
                   "n_wall_particles": g["nw"], "spacing_m": 0.01, "h_over_s": 2.0,
                   "levels": 4, "base_steps": K, "dt_base_s": g["dt_base"]},
        "global_adaptive": {"value": g["ps_ga"], "unit": "particle-steps/s",
                            "ms_total": g["ms_ga"], "steps": g["ga"]["steps"],
                            "density_err_max": g["ga"]["err_max"]},
        "speedup_vs_global_adaptive": g["ms_ga"] / g["ms_rts"],
        "density_err_max": g["rts"]["err_max"],
        "active_fraction": g["rts"]["active_total"] / (g["n"] * K),
        "neighbour_interactions_per_s": g["rts"]["inter_total"] / (g["ms_rts"] * 1e-3),
        "simulated_time_s": g["sim_time"],
    }
    if "kernels_ms" in g:
        km = g["kernels_ms"]
        cnt = g["prof_counts"]
        rows = {}
        for name, ms in km.items():
            b, f = kernel_traffic(name, g["n"], g["nblocks"], K, cnt["active"], cnt["inter"],
                                  cnt["cand"])
            avg = ms / K * 1e-3
            rows[name] = {"avg_us": avg * 1e6, "GBps": b / avg / 1e9 if avg > 0 else 0.0,
                          "TFLOPs": f / avg / 1e12 if avg > 0 else 0.0}
        dom = max(km, key=lambda k: km[k])
        d = rows[dom]
        if dom in ("search_density", "force"):
            roof = {"kernel": dom, "bound": "alu", "achieved": d["TFLOPs"],
                    "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": d["TFLOPs"] / FP32_VALU_PEAK_TFLOPS,
                    "traffic": measured_traffic(dom)}
        else:
            roof = {"kernel": dom, "bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": d["GBps"] / HBM_PEAK_GBS,
                    "traffic": measured_traffic(dom)}
        line["roofline"] = roof
        line["kernels"] = rows
        tn = km["key_hist"] + km["scan"] + km["scatter"] + km["cell_gather"]
        tp = km["search_density"] + km["force"]
        tr = km["rmin_flags"] + km["step_stats"]
        ti = km["correct_predict"]
        tot = tn + tp + tr + ti
        line["phase_split"] = {"grid_and_search_share": None,
                               "T_grid": tn / tot, "T_search_density_force": tp / tot,
                               "T_rts_flags": tr / tot, "T_integrate": ti / tot}
    if args.pcisph_steps > 0:
        line["pcisph"] = run_pcisph(args.pcisph_steps)
    if args.batch_steps > 0:
        line["batched"] = run_batched(args.batch_steps)
    if args.more_steps > 0:
        line["more_wcsph"] = run_more_wcsph(args.more_steps)
    if args.diff_repeats > 0:
        line["differentiable"] = run_diff(args.diff_repeats)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = run_cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
