"""Benchmark: WCSPH regional time stepping vs global adaptive stepping on one GPU.

Workload: the 250,000-particle dam break (column 0.5 x 1.0 x 0.5 m at spacing
0.01 m in a 2 x 1 x 1 m box), block levels 0..3 with phase-aligned updates.
A step is one base step of the whole path (grid rebuild, block levels, flags,
neighbour search + density, forces, corrector/predictor).

Equal error: each arm runs at its own sound speed, the smallest (on a grid)
that keeps its max compression at or below 1 % over the whole collapse,
0 -> 0.3 s, through the front's impact on the far wall.

Printed: one JSON line.  ``value`` is RTS particle-steps/s (particles x base
steps / wall seconds, inputs resident in HBM) over K base steps from the
developed state at 0.15 s, the median of the repeats; the global adaptive
comparator is timed over the same simulated window from its own state at
0.15 s.  ``collapse_leg`` times both arms over 0 -> 0.3 s
(``speedup_at_equal_error``).  The dominant kernel's roofline comes from an
event-bracketed run of the same K steps; the CPU baseline is the FP64
oracle on a bounded window of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
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
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats of the K-step window (the median is reported)")
    ap.add_argument("--no-leg", action="store_true",
                    help="skip the 0 -> 0.3 s collapse leg at equal error")
    ap.add_argument("--save-state", default="",
                    help="write the RTS arm's developed state to this file")
    ap.add_argument("--load-state", default="",
                    help="start the RTS arm from this saved state instead of running to it "
                         "(profiler runs: only the timed window is traced)")
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
    ap.add_argument("--more-time", type=float, default=0.3,
                    help="simulated seconds of the double dam break and block drop legs (0: skip)")
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
    neighbour lists (two bytes per entry: the neighbours and the particle
    itself); re-reads of neighbour state served by LDS or caches are not
    counted.  Flops count the float operations
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
        # own state and flag in; list entries, density, p/rho^2, p, count out
        "search_density": (40.0 * a + 2.0 * (i + a), 9.0 * c + 23.0 * i),
        # own state, count and list entries in; acceleration out
        "force": (52.0 * a + 2.0 * (i + a), 45.0 * i),
        "step_stats": (30.0 * nb, 12.0 * nb),
        "correct_predict": (104.0 * n + 16.0 * a, 30.0 * n),
    }
    return table[name]


# Sound speeds c0 = F sqrt(2 g H) of the two arms (H = 1 m column): for each
# arm the smallest F on a grid of step 1-2 whose 0 -> 0.3 s collapse keeps
# the max compression at or below 1 % (calibration sweep measured on one
# MI355X; the collapse leg below re-runs F and the grid point under it).
C0_FACTOR_RTS = 42.0
C0_FACTOR_GA = 39.0
C0_FACTOR_BELOW = {C0_FACTOR_RTS: 40.0, C0_FACTOR_GA: 38.0}
T_DEVELOPED = 0.15     # s: the timed window starts from the state at this time
T_LEG = 0.3            # s: collapse leg, past the front's impact on the far wall
ERR_BOUND = 0.01


def dam_break(factor):
    from paper_2009_14514_amd import scenes
    return scenes.dam_break_column(c0=scenes.sound_speed_for_column(1.0, factor=factor))


def advance_to(sim, t_end, chunk=100):
    """Advances in chunks until the simulated time reaches t_end; returns the
    last stats and the max compression seen up to 0.2 s (before the front
    meets the far wall)."""
    err_pre = 0.0
    while True:
        sim.advance(chunk)
        st = sim.sync()
        if st.time <= 0.2 + 1e-12:
            err_pre = float(st.err_max_run)
        if st.time >= t_end * (1.0 - 1e-12):
            return st, err_pre


def run_leg(mode, factor):
    """0 -> T_LEG of the 250k dam break; wall time per simulated second."""
    import torch

    from paper_2009_14514_amd.sim import Simulation

    sc = dam_break(factor)
    sim = Simulation(sc, mode=mode)
    init = sim.save()
    sim.advance(10)                              # graphs built, caches warm
    sim.sync()
    sim.load(init)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, err_pre = advance_to(sim, T_LEG)
    el = time.perf_counter() - t0
    sim.close()
    r = dict(mode=mode, c0_factor=factor, c0=sc.params["c0"], sim_time_s=st.time,
             steps=int(st.step), wall_ms=el * 1e3, ms_per_sim_s=el * 1e3 / st.time,
             density_err_max=float(st.err_max_run), density_err_max_to_0p2s=err_pre,
             active_fraction=st.active_total / (st.step * sc.n))
    print(f"[bench] leg {mode} F={factor:g}: {st.step} steps to {st.time:.4f} s in "
          f"{el * 1e3:.1f} ms, max compression {st.err_max_run * 100:.3f} %", file=sys.stderr,
          flush=True)
    return r


def run_collapse_leg():
    """Both arms over the whole collapse at their calibrated sound speeds, the
    grid point below each (which must exceed the bound: the calibration is
    the smallest passing one), and both at the common 20 sqrt(2 g H)."""
    legs = {}
    for mode, f in (("rts", C0_FACTOR_RTS), ("global_adaptive", C0_FACTOR_GA)):
        legs[mode] = run_leg(mode, f)
        legs[mode + "_below"] = run_leg(mode, C0_FACTOR_BELOW[f])
    legs["rts_equal_c0"] = run_leg("rts", 20.0)
    legs["global_adaptive_equal_c0"] = run_leg("global_adaptive", 20.0)
    r, g = legs["rts"], legs["global_adaptive"]
    both_ok = r["density_err_max"] <= ERR_BOUND and g["density_err_max"] <= ERR_BOUND
    return {
        "workload": "wcsph_dam_break_250k_collapse_0_to_0.3s",
        "err_bound": ERR_BOUND,
        "speedup_at_equal_error": g["ms_per_sim_s"] / r["ms_per_sim_s"] if both_ok else None,
        "calibration_minimal": {
            "rts": legs["rts_below"]["density_err_max"] > ERR_BOUND,
            "global_adaptive": legs["global_adaptive_below"]["density_err_max"] > ERR_BOUND},
        "speedup_at_equal_c0": (legs["global_adaptive_equal_c0"]["ms_per_sim_s"]
                                / legs["rts_equal_c0"]["ms_per_sim_s"]),
        "runs": legs,
    }


def copy_calibration():
    """Three launches of one elementwise kernel that reads 256 MiB and writes
    256 MiB: the reference for scaling HBM byte counters."""
    import torch

    torch.cuda.set_device(0)
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def run_gpu(args):
    import torch

    from paper_2009_14514_amd.sim import Simulation

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
    K, W, R = args.steps, args.warmup, max(args.repeats, 1)
    out = {}

    def timed(sim, steps):
        # HIP events on the library's stream around `steps` queued steps
        st = sim.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        sim.advance(steps)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def window_error(sim, snap, steps):
        """Max compression over the steps of the window (untimed pass)."""
        sim.load(snap)
        e = 0.0
        for _ in range(steps):
            sim.advance(1)
            e = max(e, float(sim.sync().err_max_last))
        return e

    def developed(mode, factor):
        """A context holding the state at T_DEVELOPED (run untimed from rest),
        saved for the repeats; W warm-up steps from it are run and undone."""
        sc = dam_break(factor)
        sim = Simulation(sc, mode=mode)
        if args.load_state and mode == "rts":
            import numpy as np
            buf = torch.from_numpy(np.fromfile(args.load_state, dtype=np.uint8)).cuda()
            sim.load(buf)
        else:
            advance_to(sim, T_DEVELOPED)
        snap = sim.save()
        if args.save_state and mode == "rts":
            snap.cpu().numpy().tofile(args.save_state)
        if W:
            sim.advance(W)
            sim.sync()
            sim.load(snap)
        return sc, sim, snap

    # --- RTS: K base steps from the developed state, median of R repeats -------
    sc, rts, snap_r = developed("rts", C0_FACTOR_RTS)
    snap_stats_r = rts.sync()
    t_start = snap_stats_r.time
    ms_r = []
    for _ in range(R):
        rts.load(snap_r)
        ms_r.append(timed(rts, K))
    st_r = rts.sync()
    T = st_r.time - t_start
    ms_rts = statistics.median(ms_r)
    print(f"[bench] rts: {K} steps from t = {t_start:.4f} s, median {ms_rts:.3f} ms of "
          f"{R} ({min(ms_r):.3f}-{max(ms_r):.3f}), active {st_r.active_total}, "
          f"err_max {st_r.err_max_last:.4f}", file=sys.stderr, flush=True)
    if args.only_rts:
        if not args.no_profile:
            rts.load(snap_r)
            rts.profile(K)
        rts.close()
        return None

    # --- global adaptive over the same simulated window -------------------------
    _, ga, snap_g = developed("global_adaptive", C0_FACTOR_GA)
    tg0 = ga.sync().time
    steps_g = 0
    while True:                                  # untimed: how many steps cover T
        ga.advance(1)
        steps_g += 1
        if ga.sync().time - tg0 >= T * (1.0 - 1e-12):
            break
    ms_g = []
    for _ in range(R):
        ga.load(snap_g)
        ms_g.append(timed(ga, steps_g))
    st_g = ga.sync()
    T_g = st_g.time - tg0
    ms_ga = statistics.median(ms_g)
    print(f"[bench] global adaptive: {steps_g} steps over {T_g:.3e} s, median {ms_ga:.3f} ms",
          file=sys.stderr, flush=True)

    err_r = window_error(rts, snap_r, K)
    err_g = window_error(ga, snap_g, steps_g)
    n = sc.n
    dtb = st_r.dt_last
    ps_rts = n * K / (ms_rts * 1e-3)
    # base-step equivalents of the comparator's simulated time
    ps_ga = n * (T_g / dtb) / (ms_ga * 1e-3)
    out.update(
        n=n, nw=sc.nw, K=K, R=R, ms_rts=ms_rts, ms_rts_all=ms_r, ms_ga=ms_ga, ms_ga_all=ms_g,
        ps_rts=ps_rts, ps_ga=ps_ga, sim_time=T, t_start=t_start, dt_base=dtb, c0=sc.params["c0"],
        rts=dict(active=st_r.active_total - snap_stats_r.active_total,
                 inter=st_r.inter_total - snap_stats_r.inter_total,
                 err_window=err_r, level_hist_last=list(st_r.level_hist)[:4]),
        ga=dict(steps=steps_g, sim_time=T_g, c0=ga.params["c0"], err_window=err_g),
        nblocks=rts.info["nblocks"],
    )

    # --- per-kernel times: the same K steps, kernels bracketed by HIP events -----
    if not args.no_profile:
        rts.load(snap_r)
        a0 = rts.sync()
        prof = rts.profile(K)
        st_p = rts.sync()
        out["kernels_ms"] = prof
        out["prof_counts"] = dict(active=st_p.active_total - a0.active_total,
                                  inter=st_p.inter_total - a0.inter_total,
                                  cand=st_p.cand_total - a0.cand_total)
    rts.close()
    ga.close()
    return out


def pcisph_arms(make_scene, steps, label):
    """Regional and standard PCISPH over the same minor steps from rest.

    The correction loop reads its error reductions between iterations, so
    each minor step is timed by wall clock around a completed call.  An arm
    that stops with a device status (a particle leaves the domain when the
    step is too long for the spacing) records the status instead of a time.
    """
    import torch

    from paper_2009_14514_amd._rts import RtsError
    from paper_2009_14514_amd.sim import Simulation

    out = {}
    for mode in ("rts", "global_fixed"):
        sc = make_scene()
        sc.params["mode"] = mode
        sim = Simulation(sc)
        sim.advance(1)                       # first major step set-up and lists: warm-up
        sim.sync()
        sim.set_state(sc.pos, sc.vel)        # back to rest
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            sim.advance(steps)
            st = sim.sync()
        except RtsError as e:
            sim.close()
            # untimed rerun one minor step at a time: the step that raised it
            sim = Simulation(sc)
            t_fail = None
            for _ in range(steps):
                t_before = sim.sync(raise_on_error=False).time
                try:
                    sim.advance(1)
                    sim.sync()
                except RtsError:
                    t_fail = t_before
                    break
            out[mode] = dict(n=sc.n, failed=str(e), time=t_fail)
            print(f"[bench] {label} {mode}: stopped in the minor step from t = {t_fail} s ({e})",
                  file=sys.stderr, flush=True)
            sim.close()
            continue
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = dict(n=sc.n, ms=el * 1e3, iters=int(st.pci_iters_total), time=st.time,
                         errmax=float(st.pci_errmax), hist=list(st.level_hist)[:4])
        print(f"[bench] {label} {mode}: {steps} minor steps in {el * 1e3:.1f} ms, "
              f"{st.pci_iters_total} iterations", file=sys.stderr, flush=True)
        sim.close()
    return out


def arm_summary(a, steps):
    if "failed" in a:
        return {"stopped": a["failed"], "stopped_in_step_from_s": a["time"]}
    return {"value": a["n"] * steps / (a["ms"] * 1e-3), "ms_per_step": a["ms"] / steps,
            "iterations": a["iters"], "density_err_last": a["errmax"]}


def run_pcisph(steps):
    """RTS PCISPH vs standard PCISPH on the 1,000,188-particle double dam break,
    and on the same scene at the literal 0.008 m spacing (500,000 particles)
    with base steps of 1e-3 s and 5e-4 s."""
    from paper_2009_14514_amd import scenes

    out = pcisph_arms(scenes.double_dam_break, steps, "pcisph 1M")
    r, g = out["rts"], out["global_fixed"]
    if "failed" in r or "failed" in g:
        raise RuntimeError(f"PCISPH 1M double dam break stopped: {r.get('failed')} {g.get('failed')}")
    n = r["n"]
    literal = {}
    for dt in (1e-3, 5e-4):
        lo = pcisph_arms(lambda: scenes.double_dam_break(spacing=0.008, dt_base=dt), steps,
                         f"pcisph 500k dt={dt:g}")
        e = {"n_particles": lo["rts"]["n"], "spacing_m": 0.008, "dt_base_s": dt,
             "minor_steps": steps, "unit": "particle-steps/s",
             "rts": arm_summary(lo["rts"], steps),
             "standard_pcisph": arm_summary(lo["global_fixed"], steps)}
        if "ms" in lo["rts"] and "ms" in lo["global_fixed"]:
            e["speedup_vs_standard"] = lo["global_fixed"]["ms"] / lo["rts"]["ms"]
        literal[f"dt_{dt:g}"] = e
    return {
        "workload": "pcisph_rts_double_dam_break_1m", "n_particles": n, "minor_steps": steps,
        "dt_base_s": 5e-4, "unit": "particle-steps/s",
        "value": n * steps / (r["ms"] * 1e-3), "ms_per_step": r["ms"] / steps,
        "iterations": r["iters"], "density_err_last": r["errmax"],
        "standard_pcisph": {"value": n * steps / (g["ms"] * 1e-3), "ms_per_step": g["ms"] / steps,
                            "iterations": g["iters"], "density_err_last": g["errmax"]},
        "speedup_vs_standard": g["ms"] / r["ms"],
        "literal_spacing_500k": literal,
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


def run_more_wcsph(t_end):
    """The paper's other WCSPH scenes as synthetic stand-ins: a double dam
    break (256,000 particles) and a dam break with a dropped block (177,000),
    from rest to t_end, each arm at the dam break's calibrated sound speed
    (scaled to the scene's height); wall time per simulated second."""
    import torch

    from paper_2009_14514_amd import scenes
    from paper_2009_14514_amd.sim import Simulation

    out = {}
    for name, make in (("wcsph_double_dam_break_256k", scenes.wcsph_double_dam_break),
                       ("wcsph_block_drop_177k", scenes.block_drop)):
        res = {}
        for mode, f in (("rts", C0_FACTOR_RTS), ("global_adaptive", C0_FACTOR_GA)):
            sc = make()
            # the generators take 20 sqrt(2 g H) for their height H
            sim = Simulation(sc, mode=mode, c0=sc.params["c0"] * f / 20.0)
            init = sim.save()
            sim.advance(10)
            sim.sync()
            sim.load(init)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _ = advance_to(sim, t_end)
            el = (time.perf_counter() - t0) * 1e3
            res[mode] = dict(ms=el, sim_time_s=st.time, steps=int(st.step),
                             ms_per_sim_s=el / st.time, density_err_max=float(st.err_max_run),
                             c0_m_s=sim.params["c0"],
                             active_fraction=st.active_total / (st.step * sc.n))
            sim.close()
        r, g = res["rts"], res["global_adaptive"]
        out[name] = {"n_particles": sc.n, "sim_time_s": t_end,
                     "value": sc.n * r["steps"] / (r["ms"] * 1e-3), "unit": "particle-steps/s",
                     "rts": r, "global_adaptive": g,
                     "speedup_vs_global_adaptive": g["ms_per_sim_s"] / r["ms_per_sim_s"]}
        print(f"[bench] {name}: rts {r['ms']:.1f} ms ({r['density_err_max'] * 100:.2f} %), "
              f"global adaptive {g['ms']:.1f} ms ({g['density_err_max'] * 100:.2f} %)",
              file=sys.stderr, flush=True)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(budget_s):
    """FP64 oracle on the same workload from rest, each arm at its sound
    speed: RTS for about 40 % of the budget, then global adaptive stepping
    over the same simulated time (bounded by the rest of the budget)."""
    import numpy as np

    import oracle

    def arm(mode, factor, t_end, budget):
        sc = dam_break(factor)
        sim = oracle.WCSPH(sc.params, sc.pos.astype(np.float32),
                           walls=sc.walls.astype(np.float32), mode=mode)
        t0 = time.time()
        steps = 0
        while True:
            sim.step()
            steps += 1
            el = time.time() - t0
            if el >= budget or (t_end is not None and sim.t >= t_end * (1.0 - 1e-12)):
                return sc.n, steps, sim.t, el

    n, steps, t_r, el_r = arm("rts", C0_FACTOR_RTS, None, 0.4 * budget_s)
    _, steps_g, t_g, el_g = arm("global_adaptive", C0_FACTOR_GA, t_r, 0.6 * budget_s)
    dtb = t_r / steps
    return dict(value=n * steps / el_r, unit="particle-steps/s", cores=oracle.num_threads(),
                cpu_model=cpu_model(), kind="oracle",
                sample=f"first {steps} RTS base steps ({t_r:.2e} s simulated) of the "
                       f"250,000-particle dam break from rest, FP64, {el_r:.1f} s",
                global_adaptive=dict(value=n * (t_g / dtb) / el_g, steps=steps_g,
                                     sim_time_s=t_g, seconds=el_g,
                                     complete=t_g >= t_r * (1.0 - 1e-12)),
                speedup_vs_global_adaptive=(el_g / t_g) / (el_r / t_r))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU slab decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)
    if args.only_pcisph:
        if args.copy_calibration:
            copy_calibration()
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
                   "levels": 4, "phase_align": 1, "base_steps": K, "dt_base_s": g["dt_base"],
                   "c0_m_s": g["c0"], "c0_factor": C0_FACTOR_RTS,
                   "window_start_s": g["t_start"], "repeats": g["R"], "timing": "median"},
        "ms_per_step_repeats": [m / K for m in g["ms_rts_all"]],
        "global_adaptive": {"value": g["ps_ga"], "unit": "particle-steps/s (base-step equivalents)",
                            "ms_total": g["ms_ga"], "steps": g["ga"]["steps"],
                            "sim_time_s": g["ga"]["sim_time"], "c0_m_s": g["ga"]["c0"],
                            "c0_factor": C0_FACTOR_GA,
                            "density_err_max_window": g["ga"]["err_window"]},
        # wall time per simulated second, comparator over RTS
        "speedup_vs_global_adaptive": g["ps_rts"] / g["ps_ga"],
        "density_err_max_window": g["rts"]["err_window"],
        "active_fraction": g["rts"]["active"] / (g["n"] * K),
        "neighbour_interactions_per_s": g["rts"]["inter"] / (g["ms_rts"] * 1e-3),
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
                          "hbm_frac": b / avg / 1e9 / HBM_PEAK_GBS if avg > 0 else 0.0,
                          "TFLOPs": f / avg / 1e12 if avg > 0 else 0.0,
                          "valu_frac": f / avg / 1e12 / FP32_VALU_PEAK_TFLOPS if avg > 0 else 0.0,
                          "algorithmic_bytes_per_launch": b, "algorithmic_flop_per_launch": f}
        dom = max(km, key=lambda k: km[k])
        d = rows[dom]
        if dom in ("search_density", "force"):
            roof = {"kernel": dom, "bound": "alu", "achieved": d["TFLOPs"],
                    "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": d["TFLOPs"] / FP32_VALU_PEAK_TFLOPS,
                    "traffic": measured_traffic(dom),
                    "hbm_GBps_algorithmic": d["GBps"], "hbm_frac_algorithmic": d["hbm_frac"],
                    "flop_source": "9 flop per candidate test + 23 per density term, "
                                   "counted from the kernel's float operations"}
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
        line["phase_split"] = {"T_grid": tn / tot, "T_search_density_force": tp / tot,
                               "T_rts_flags": tr / tot, "T_integrate": ti / tot}
    if not args.no_leg:
        line["collapse_leg"] = run_collapse_leg()
        line["speedup_at_equal_error"] = line["collapse_leg"]["speedup_at_equal_error"]
    if args.pcisph_steps > 0:
        line["pcisph"] = run_pcisph(args.pcisph_steps)
    if args.batch_steps > 0:
        line["batched"] = run_batched(args.batch_steps)
    if args.more_time > 0:
        line["more_wcsph"] = run_more_wcsph(args.more_time)
    if args.diff_repeats > 0:
        line["differentiable"] = run_diff(args.diff_repeats)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = run_cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
