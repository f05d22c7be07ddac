"""Throughput of the whole critical-curve -> caustic -> crossing-map ->
distance-map path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload n10k]

One step = set_lenses + find_critical_curves (all m+1 rows, with the caustic
image of every root mapped in the same pass) + caustic_crossings +
caustic_distances on one seeded synthetic field whose inputs are already in
HBM.  Prints one JSON line:
  value           roots/s = m * 2N / (seconds per step)
  roofline        the root finder's dominant kernel (the persistent launch
                  that runs every pass, by default): algorithmic FLOP per
                  launch / its HIP-event-timed duration, against the vector
                  peak of each part's precision
  cpu_baseline    the CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FLOP/clk
FP32_VECTOR_PEAK_TFLOPS = 157.3  # packed-FP32 peak; unpacked FP32 issues at the FP64 rate
METRIC = "critical-curve roots/s at N=1e4 stars, % FP64 VALU peak; mixed vs FP64"

WORKLOAD_TEXT = {
    "n10k": "N=10,000 equal-mass stars, kappa_star=0.5, kappa_s=0, gamma=0.3, uniform disk; "
            "20,000 phase steps (20,001 rows x 20,000 roots); caustics; N_cc int32 2048^2 and "
            "FP64 distance map over 40x40 theta_E",
    "n1k": "N=1,000 Salpeter stars on [0.08,1], kappa_star=0.4, kappa_s=0.2, gamma=0.45; "
           "10,000 phase steps (2,000 roots each); caustics; N_cc 1024^2 over 20x20 theta_E",
    "n10k_mixed": "the n10k field and grids in mixed precision: one FP32 Aberth sweep per warm "
                  "row, FP64 Newton polish with an a-posteriori acceptance test and a Vieta row "
                  "check, FP64 sweeps for anything not accepted, FP64 lens mapping",
    "tiny": "N=10 equal-mass stars, kappa_star=0.3, kappa_s=0, gamma=0.3; 1,000 phase steps; "
            "caustics; N_cc 256^2 over 16x16 theta_E",
    "rect": "rectangular field (Sec. 4.2) over the region the n10k source map sees: N=437 "
            "equal-mass stars uniform in [-19.2, 19.2] x [-35.7, 35.7] theta_E, kappa_star=0.5 "
            "(sheet Taylor degree t=87, App. B error 1e-8 within |c|/1.25), kappa_s=0, "
            "gamma=0.3; 20,000 phase steps (20,001 rows x 960 roots); caustics; N_cc int32 "
            "2048^2 and FP64 distance map over 40x40 theta_E",
    "batched": "256 independent fields, N log-uniform in [50, 5000], kappa_star U[0.1, 0.8], "
               "gamma U[0, 0.6], kappa_s=0, Salpeter masses on [0.08,1]; 4,000 phase steps "
               "each; one root-finder call over all fields in mixed precision; caustics",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n10k", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--subchains", type=int, default=0, help="0 = library choice")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: the workload's own (mixed for n10k_mixed)")
    ap.add_argument("--predictor", type=int, default=2, choices=[0, 1, 2],
                    help="warm-row start: 0 previous row, 1 linear, 2 quadratic extrapolation")
    ap.add_argument("--cpu-baseline", dest="cpu_baseline", action="store_true", default=True)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--schedule", default="persistent", choices=["rounds", "persistent"],
                    help="root-finder scheduling: global rounds, or one persistent launch")
    ap.add_argument("--cpu-rows", type=int, default=4,
                    help="warm rows of the oracle timed for the CPU baseline")
    ap.add_argument("--compare", dest="compare", action="store_true", default=True,
                    help="also run the other precision (mixed vs FP64) on the same field")
    ap.add_argument("--no-compare", dest="compare", action="store_false")
    ap.add_argument("--star-sums", dest="star_sums", default="direct", choices=["direct", "fmm"],
                    help="star sums of the FP64 sweeps and the polish: direct, or fast multipole "
                         "(one field per call)")
    ap.add_argument("--multipole", dest="multipole", action="store_true", default=True,
                    help="after the timed run, the same field with fast-multipole star sums (FP64 "
                         "and mixed), reported beside it")
    ap.add_argument("--no-multipole", dest="multipole", action="store_false")
    ap.add_argument("--directional", type=int, default=0, metavar="K",
                    help="after the timed steps, moving-source distance maps of the last step's "
                         "N_cc map for K directions over [0, 180) degrees, with their histograms "
                         "(and by N_cc class at 90 degrees)")
    ap.add_argument("--serial", dest="serial", action="store_true", default=True,
                    help="batched workload: also solve every field alone, one call each")
    ap.add_argument("--no-serial", dest="serial", action="store_false")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (to scale "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path is single-GPU by design "
              "(multi-GPU sharding by phase subchains is described, not built). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8}), flush=True)
        return

    from paper_2506_02121_amd import fields, mlcc

    wl = fields.workload(args.workload, args.seed)
    precision = args.precision or wl.precision
    if wl.fields:
        return bench_batched(args, wl, precision)
    f = wl.field
    if wl.grid is None:
        wl.grid = fields.Grid(0.0, 0.0, 8.0, 8.0, 256, 256)
    m_steps = wl.m_steps
    n = f.n
    dev = torch.device("cuda", 0)
    x = torch.as_tensor(f.x, device=dev)
    y = torch.as_tensor(f.y, device=dev)
    mm = torch.as_tensor(f.m, device=dev)

    def load(c):
        if f.sheet is None:
            c.set_lenses(x, y, mm, f.kappa_s, f.gamma)
        else:
            ks, c1, c2, t = f.sheet
            c.set_lenses_rect(x, y, mm, f.kappa_s, f.gamma, ks, c1, c2, t)

    probe = mlcc.Context(0)
    load(probe)
    n_r = probe.num_roots()   # 2N, or 2N + t - 1 for a rectangular field
    probe.close()
    rows = m_steps + 1
    roots_re = torch.empty((rows, n_r), dtype=torch.float64, device=dev)
    roots_im = torch.empty_like(roots_re)
    w_re = torch.empty_like(roots_re)
    w_im = torch.empty_like(roots_re)
    grid = mlcc.as_grid(wl.grid)
    ncc = torch.empty((grid.ny, grid.nx), dtype=torch.int32, device=dev)
    dist = torch.empty((grid.ny, grid.nx), dtype=torch.float64, device=dev)
    bl = torch.empty((grid.ny, grid.nx), dtype=torch.uint8, device=dev)
    ctx = mlcc.Context(0)
    torch.cuda.synchronize()

    def step(prec):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        load(ctx)
        # roots and, in the same pass, their caustic images
        _, _, _, _, cn, st, _ = ctx.find_critical_curves(
            m_steps, n_subchains=args.subchains, timing=True, caustics=True,
            out=(roots_re, roots_im), caustics_out=(w_re, w_im), precision=prec,
            predictor=args.predictor, schedule=args.schedule, star_sums=args.star_sums)
        ev[1].record()
        ctx.caustic_crossings(w_re, w_im, cn, grid, out=ncc)
        ev[2].record()
        ctx.caustic_distances(grid, ncc, out=(dist, bl))
        ev[3].record()
        st["_events"] = ev
        return st

    def stage_ms(stats):
        """Per-stage GPU time (HIP events on the context's stream), averaged."""
        out = {"lenses_roots_caustics": 0.0, "crossing_map": 0.0, "distance_map": 0.0}
        for s_ in stats:
            ev = s_.pop("_events")
            out["lenses_roots_caustics"] += ev[0].elapsed_time(ev[1]) / len(stats)
            out["crossing_map"] += ev[1].elapsed_time(ev[2]) / len(stats)
            out["distance_map"] += ev[2].elapsed_time(ev[3]) / len(stats)
        return out

    def run(prec, warmup, steps):
        for i in range(warmup):
            t = time.perf_counter()
            step(prec)
            torch.cuda.synchronize()
            log(f"{prec} warmup {i}: {time.perf_counter() - t:.3f} s")
        stats = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ts = time.perf_counter()
            stats.append(step(prec))
            torch.cuda.synchronize()
            log(f"{prec} step {i}: {time.perf_counter() - ts:.3f} s, {stats[-1]['sweeps']} passes / rounds")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return el, stats

    elapsed, stats = run(precision, args.warmup, args.steps)
    ms_per_step = 1e3 * elapsed / args.steps
    roots_per_step = m_steps * n_r
    stages = stage_ms(stats)
    # the standalone lens mapping on a sample of the roots (the step uses the
    # fused mapping): points/s and algorithmic TFLOP/s at 12 N FLOP per point
    n_map = min(rows, max(1, (1 << 26) // n_r))
    zr_s, zi_s = roots_re[:n_map].reshape(-1), roots_im[:n_map].reshape(-1)
    wr_s, wi_s = torch.empty_like(zr_s), torch.empty_like(zi_s)
    load(ctx)
    ctx.map_caustics(zr_s, zi_s, out=(wr_s, wi_s))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    ctx.map_caustics(zr_s, zi_s, out=(wr_s, wi_s))
    ev[1].record()
    torch.cuda.synchronize()
    map_ms = ev[0].elapsed_time(ev[1])
    stages["map_caustics_standalone"] = {
        "points": n_map * n_r, "ms": map_ms, "points_per_s": n_map * n_r / (map_ms * 1e-3),
        "tflops": 12.0 * n * n_map * n_r / (map_ms * 1e-3) / 1e12}
    del zr_s, zi_s, wr_s, wi_s
    value = roots_per_step / (elapsed / args.steps)

    kernels = root_kernels(stats, precision)
    dominant = max(kernels, key=lambda k: k["time_s"])
    s0 = stats[-1]
    updates_per_root_row = (s0["root_updates"] + s0["root_updates_f32"] + s0["polish_updates"]) \
        / float(n_r * (rows + s0["n_subchains"]))
    ncc_h = ncc.cpu().numpy()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "roots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (root-root terms f32)" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "n_stars": n, "roots_per_row": n_r, "phase_steps": m_steps,
                   "grid": [grid.nx, grid.ny], "precision": precision,
                   "predictor": args.predictor, "schedule": args.schedule,
                   "star_sums": args.star_sums, "seed": args.seed},
        "roofline": {
            "bound": "alu",
            "kernel": dominant["kernel"],
            "achieved": dominant["achieved"],
            "peak": dominant["peak"],
            "unit": "TFLOP/s",
            "frac": dominant["frac"],
            "traffic": measured_traffic(dominant["kernel"], args.workload),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_ms": dominant["avg_launch_ms"],
            "launches": dominant["launches"],
            "flop_per_root_update": 29 * n + 10 * (n_r - 1),
            # the headline's "% of the FP64 VALU peak": every algorithmic FLOP
            # of the launch (its FP32 root terms included) over 78.6 TFLOP/s
            "frac_of_fp64_peak": (dominant["achieved"] / FP64_VECTOR_PEAK_TFLOPS
                                  if dominant["achieved"] else None),
            "kernels": kernels,
            "measured_peak": measured_peaks(dominant),
        },
        "stage_ms": stages,
        "root_updates_per_s": (s0_updates(stats[-1])) / (elapsed / args.steps),
        "stats": {"sweeps_per_step": s0["sweeps"], "root_updates_per_step": s0["root_updates"],
                  "root_updates_f32_per_step": s0["root_updates_f32"],
                  "polish_updates_per_step": s0["polish_updates"],
                  "rows_fallback": s0["rows_fallback"],
                  "updates_per_root_per_row": updates_per_root_row,
                  "n_subchains": s0["n_subchains"], "cold_sweeps": s0["cold_sweeps"],
                  "max_row_sweeps": s0["max_row_sweeps"], "match_maxdist": s0["match_maxdist"],
                  "ncc_max": int(ncc_h.max()), "ncc_min": int(ncc_h.min())},
    }
    if args.star_sums == "fmm":
        # the library counts the multipole form's own work: near star terms
        # plus one series evaluation per update; the traffic counters were
        # taken with direct sums
        out["roofline"].update({"traffic": None,
                                "note": "fast-multipole star sums: FLOP = 29 per near star term "
                                        "+ (26 p + 20) per series evaluation + root terms"})
        out["stats"].update({"fmm_near_terms_per_step": s0["fmm_near_terms"],
                             "fmm_far_evals_per_step": s0["fmm_far_evals"]})
    if args.directional > 0:
        out["directional"] = directional_stage(ctx, grid, ncc, args.directional)
    # sampled rows of the timed run: the other runs below report how far their
    # roots lie from these (same sets, any order)
    from scipy.spatial import cKDTree
    sample = np.linspace(0, m_steps, 17).astype(np.int64)
    ref = [(roots_re[j].cpu().numpy(), roots_im[j].cpu().numpy()) for j in sample]

    def distance_to_ref():
        dmax = 0.0
        for j, (a_re, a_im) in zip(sample, ref):
            b = np.stack([roots_re[j].cpu().numpy(), roots_im[j].cpu().numpy()], 1)
            d, _ = cKDTree(b).query(np.stack([a_re, a_im], 1))
            dmax = max(dmax, float(d.max()))
        return dmax

    if args.compare and f.sheet is None:   # a rectangular field is solved in FP64 only
        # the other precision on the same field: throughput and distance
        other = "mixed" if precision == "fp64" else "fp64"
        el2, st2 = run(other, 0, args.steps)
        dmax = distance_to_ref()
        k2 = root_kernels(st2, other)
        out["compare"] = {
            "precision": other, "value": roots_per_step / (el2 / args.steps),
            "ms_per_step": 1e3 * el2 / args.steps, "steps": args.steps,
            "speedup_of_mixed_over_fp64": (el2 / elapsed if other == "fp64" else elapsed / el2),
            "max_root_distance_to_main_run": dmax, "sampled_rows": len(sample),
            "kernels": k2,
            "stats": {k: st2[-1][k] for k in ("sweeps", "root_updates", "root_updates_f32",
                                              "polish_updates", "rows_fallback")},
        }
    if args.multipole and args.star_sums == "direct":
        # the same field with fast-multipole star sums (Sec. 4.1), in each
        # precision the field takes: throughput, its launch's roofline on the
        # method's own FLOP count, and the distance to the timed run's roots
        out["multipole"] = {}
        for prec_m in (["fp64"] if f.sheet is not None else ["fp64", "mixed"]):
            saved = args.star_sums
            args.star_sums = "fmm"
            try:
                el3, st3 = run(prec_m, 1, args.steps)
            except mlcc.MlccError as e:   # reported, not fatal to the timed run's line
                out["multipole"][prec_m] = {"error": str(e)}
                log(f"multipole {prec_m}: {e}")
                continue
            finally:
                args.star_sums = saved
            k3 = root_kernels(st3, prec_m)
            out["multipole"][prec_m] = {
                "value": roots_per_step / (el3 / args.steps), "ms_per_step": 1e3 * el3 / args.steps,
                "steps": args.steps, "warmup": 1,
                "speedup_over_timed_run": elapsed / el3,
                "max_root_distance_to_main_run": distance_to_ref(), "sampled_rows": len(sample),
                "kernels": k3,
                "stats": {k: st3[-1][k] for k in ("n_subchains", "sweeps", "root_updates",
                                                  "root_updates_f32", "polish_updates",
                                                  "fmm_near_terms", "fmm_far_evals")},
            }
            log(f"multipole {prec_m}: {1e3 * el3 / args.steps:.1f} ms per step")
    ctx.close()
    del roots_re, roots_im, w_re, w_im
    torch.cuda.empty_cache()

    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(f, m_steps, args.cpu_rows)
    print(json.dumps(out), flush=True)


def directional_stage(ctx, grid, ncc, k_angles, n_bins=200, d_max=20.0):
    """Moving-source distances (Sec. 5.2, Figs. 5-7) on one N_cc map: for K
    directions over [0, 180) degrees the distance map and its histogram
    P(d | angle); at 90 degrees also P(d | N_cc).  Times the kernels with
    HIP events; algorithmic bytes per pixel and direction: the N_cc map read
    (4 B), the distance (8 B) and border flag (1 B) written."""
    import numpy as np
    import torch

    angles = [np.pi * k / k_angles for k in range(k_angles)]
    dist = torch.empty((grid.ny, grid.nx), dtype=torch.float64, device=ncc.device)
    bl = torch.empty((grid.ny, grid.nx), dtype=torch.uint8, device=ncc.device)
    hist = torch.empty((k_angles, 1, n_bins + 1), dtype=torch.int64, device=ncc.device)
    ctx.caustic_distances_directional(grid, ncc, angles[0], out=(dist, bl))   # warm-up
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for k, a in enumerate(angles):
        ctx.caustic_distances_directional(grid, ncc, a, out=(dist, bl))
        ctx.distance_histogram(dist, bl, n_bins, d_max, out=hist[k])
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    h = hist[:, 0, :].cpu().numpy()
    w = d_max / n_bins

    def median(row):
        c = np.cumsum(row)
        return float((np.searchsorted(c, 0.5 * c[-1]) + 0.5) * w) if c[-1] else None
    med = [median(r) for r in h]
    # by N_cc class at 90 degrees
    ctx.caustic_distances_directional(grid, ncc, np.pi / 2, out=(dist, bl))
    top = int(ncc.max().item())
    by_ncc = ctx.distance_histogram(dist, bl, n_bins, d_max, ncc=ncc, ncc_lo=0,
                                    n_classes=min(top + 1, 8192 // (n_bins + 1))).cpu().numpy()
    npix = grid.nx * grid.ny
    return {
        "angles_deg": [180.0 * a / np.pi for a in angles], "ms_total": ms,
        "ms_per_direction": ms / k_angles,
        "pixels_per_s": npix * k_angles / (ms * 1e-3),
        "algorithmic_gbps": 13.0 * npix * k_angles / (ms * 1e-3) / 1e9,
        "frac_of_hbm": 13.0 * npix * k_angles / (ms * 1e-3) / 8e12,
        "median_distance_by_angle": med, "bins": n_bins, "d_max": d_max,
        "not_border_limited_at_0deg": int(h[0].sum()),
        "median_distance_by_ncc_at_90deg": [median(r) for r in by_ncc],
    }


def s0_updates(st):
    """Root updates of every kind in one call."""
    return st["root_updates"] + st["root_updates_f32"] + st["polish_updates"]


def measured_peaks(k):
    """The device's measured FMA-chain rates beside the published peaks, and
    the dominant kernel's fraction of them (FP64 and FP32 parts each priced
    at their measured rate)."""
    from paper_2506_02121_amd import mlcc
    p64 = mlcc.measure_valu_peak(0, "fp64")
    p32 = mlcc.measure_valu_peak(0, "fp32")
    out = {"fp64_fma_tflops": p64, "fp32_fma_tflops": p32,
           "method": "8 independent FMA chains per lane, 8 waves per SIMD, HIP events"}
    f64 = k.get("flop_f64")
    f32 = k.get("flop_f32")
    if f64 is not None and k["time_s"] > 0:
        t = f64 / (p64 * 1e12) + f32 / (p32 * 1e12)
        out["kernel_frac_of_measured"] = t / k["time_s"]
    return out


def kernel_line(stats, name, flop_key, ms_key, n_key, peak, dtype, f32_key=None):
    """Roofline of one root-finder kernel: algorithmic FLOP of the launches
    that did work over their HIP-event time (with f32_key, FLOP of that key
    run in FP32 and the peak is weighted between `peak` and the FP32 one)."""
    flop = sum(s[flop_key] for s in stats)
    if f32_key:
        f32 = sum(s[f32_key] for s in stats)
        if flop + f32 > 0:
            peak = (flop + f32) / (flop / peak + f32 / FP32_VECTOR_PEAK_TFLOPS)
        flop += f32
    ms = sum(s[ms_key] for s in stats)
    launches = sum(s[n_key] for s in stats)
    achieved = flop / (ms * 1e-3) / 1e12 if ms > 0 else None
    return {"kernel": name, "dtype": dtype, "achieved": achieved, "peak": peak,
            "frac": achieved / peak if achieved else None, "time_s": ms * 1e-3,
            "avg_launch_ms": ms / launches if launches else None, "launches": launches}


def root_kernels(stats, precision):
    if any(s["persistent_launches"] for s in stats):
        # one launch runs every pass kind: its roofline prices the FP64 and
        # the FP32 work each at its own peak
        f64 = sum(s["algorithmic_flop"] + s["algorithmic_flop_polish"] for s in stats)
        f32 = sum(s["algorithmic_flop_f32"] + s["algorithmic_flop_sweep_roots"] for s in stats)
        ms = sum(s["persistent_ms"] for s in stats)
        launches = sum(s["persistent_launches"] for s in stats)
        t_peak = f64 / (FP64_VECTOR_PEAK_TFLOPS * 1e12) + f32 / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
        peak = (f64 + f32) / t_peak / 1e12 if t_peak > 0 else FP64_VECTOR_PEAK_TFLOPS
        achieved = (f64 + f32) / (ms * 1e-3) / 1e12 if ms > 0 else None
        return [{"kernel": "aberth_persistent", "dtype": "f64+f32",
                 "achieved": achieved, "peak": peak,
                 "frac": achieved / peak if achieved else None, "time_s": ms * 1e-3,
                 "avg_launch_ms": ms / launches, "launches": launches,
                 "flop_f64": f64, "flop_f32": f32}]
    ks = [kernel_line(stats, "aberth_sweep_f64", "algorithmic_flop", "sweep_ms",
                      "sweep_launches", FP64_VECTOR_PEAK_TFLOPS, "f64+f32",
                      f32_key="algorithmic_flop_sweep_roots")]
    if precision == "mixed":
        ks.append(kernel_line(stats, "aberth_sweep_f32", "algorithmic_flop_f32", "sweep_f32_ms",
                              "sweep_f32_launches", FP32_VECTOR_PEAK_TFLOPS, "f32"))
        ks.append(kernel_line(stats, "newton_polish_f64", "algorithmic_flop_polish", "polish_ms",
                              "polish_launches", FP64_VECTOR_PEAK_TFLOPS, "f64"))
    return ks


def bench_batched(args, wl, precision):
    """Many independent fields in one root-finder call: roots and caustics of
    every field; value = phase steps x total roots per row / seconds."""
    import numpy as np
    import torch

    from paper_2506_02121_amd import mlcc

    fs = wl.fields
    m_steps = wl.m_steps
    dev = torch.device("cuda", 0)
    off = np.concatenate([[0], np.cumsum([f.n for f in fs])]).astype(np.int64)
    n_tot = int(off[-1])
    x = torch.as_tensor(np.concatenate([f.x for f in fs]), device=dev)
    y = torch.as_tensor(np.concatenate([f.y for f in fs]), device=dev)
    mm = torch.as_tensor(np.concatenate([f.m for f in fs]), device=dev)
    ks = [f.kappa_s for f in fs]
    gs = [f.gamma for f in fs]
    total = (m_steps + 1) * 2 * n_tot
    log(f"{len(fs)} fields, {n_tot} stars, {2 * n_tot} roots per row, "
        f"{4 * total * 8 / 2**30:.1f} GiB of roots and caustics")
    roots_re = torch.empty(total, dtype=torch.float64, device=dev)
    roots_im = torch.empty_like(roots_re)
    w_re = torch.empty_like(roots_re)
    w_im = torch.empty_like(roots_re)
    ctx = mlcc.Context(0)
    torch.cuda.synchronize()

    def step(prec=precision, star_sums=args.star_sums):
        ctx.set_lenses_batched(off, x, y, mm, ks, gs)
        _, _, _, _, cn, st, _ = ctx.find_critical_curves(
            m_steps, n_subchains=args.subchains, timing=True, caustics=True,
            out=(roots_re, roots_im), caustics_out=(w_re, w_im), precision=prec,
            predictor=args.predictor, schedule=args.schedule, star_sums=star_sums)
        return st

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t:.3f} s")
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        stats.append(step())
        torch.cuda.synchronize()
        log(f"step {i}: {time.perf_counter() - ts:.3f} s, {stats[-1]['sweeps']} passes / rounds")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    roots_per_step = m_steps * 2 * n_tot
    kernels = root_kernels(stats, precision)
    dominant = max(kernels, key=lambda k: k["time_s"])
    s0 = stats[-1]
    out = {
        "metric": METRIC, "value": roots_per_step / (elapsed / args.steps), "unit": "roots/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (root-root terms f32)" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {WORKLOAD_TEXT['batched']}", "fields": len(fs),
                   "total_stars": n_tot, "roots_per_row": 2 * n_tot, "phase_steps": m_steps,
                   "precision": precision, "predictor": args.predictor,
                   "schedule": args.schedule, "star_sums": args.star_sums, "seed": args.seed},
        "roofline": {"bound": "alu", "kernel": dominant["kernel"],
                     "achieved": dominant["achieved"], "peak": dominant["peak"],
                     "unit": "TFLOP/s", "frac": dominant["frac"],
                     "traffic": (measured_traffic(dominant["kernel"], "batched")
                                 if args.star_sums == "direct" else None),
                     "avg_launch_ms": dominant["avg_launch_ms"],
                     "launches": dominant["launches"],
                     "frac_of_fp64_peak": (dominant["achieved"] / FP64_VECTOR_PEAK_TFLOPS
                                           if dominant["achieved"] else None),
                     "kernels": kernels},
        "stats": {k: s0[k] for k in ("sweeps", "root_updates", "root_updates_f32",
                                     "polish_updates", "rows_fallback", "n_subchains",
                                     "cold_sweeps", "max_row_sweeps", "match_maxdist")},
    }
    from scipy.spatial import cKDTree
    blocks = ctx.field_blocks(m_steps)
    picks = np.linspace(0, len(fs) - 1, 8).astype(int)
    rows = np.linspace(0, m_steps, 9).astype(np.int64)

    def sample():
        got = []
        for i in picks:
            o, _, n_r = blocks[i]
            for j in rows:
                a = slice(o + j * n_r, o + (j + 1) * n_r)
                got.append(np.stack([roots_re[a].cpu().numpy(), roots_im[a].cpu().numpy()], 1))
        return got
    ref = sample()
    if args.serial:
        # the same fields one call each through the single-field path, same
        # precision, writing their blocks of the same output arrays
        def serial_pass():
            for i, f in enumerate(fs):
                o, _, n_r = blocks[i]
                sl = slice(o, o + (m_steps + 1) * n_r)
                shape = (m_steps + 1, n_r)
                ctx.set_lenses(x[off[i]:off[i + 1]], y[off[i]:off[i + 1]], mm[off[i]:off[i + 1]],
                               f.kappa_s, f.gamma)
                ctx.find_critical_curves(
                    m_steps, caustics=True, precision=precision, predictor=args.predictor,
                    schedule=args.schedule,
                    out=(roots_re[sl].view(shape), roots_im[sl].view(shape)),
                    caustics_out=(w_re[sl].view(shape), w_im[sl].view(shape)))
            torch.cuda.synchronize()
        serial_pass()   # warm-up: buffers grow to the largest field once
        t0 = time.perf_counter()
        serial_pass()
        el_s = time.perf_counter() - t0
        dmax_s = max(float(cKDTree(b).query(a)[0].max()) for a, b in zip(ref, sample()))
        out["serial"] = {
            "what": "every field alone, one find_critical_curves call each (roots and caustics)",
            "value": roots_per_step / el_s, "ms_per_step": 1e3 * el_s,
            "speedup_of_batched": el_s / (elapsed / args.steps),
            "max_root_distance_to_batched_run": dmax_s,
            "sampled": f"{len(picks)} fields x {len(rows)} rows"}
        log(f"serial: {el_s:.3f} s for {len(fs)} calls, max root distance {dmax_s:.2e}")
        step()   # the batched result again, for the comparison below
        ref = sample()
    if args.compare:
        # the other precision on the same fields: throughput, and how far its
        # roots lie from this run's on sampled rows of sampled fields
        other = "mixed" if precision == "fp64" else "fp64"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2 = [step(other) for _ in range(args.steps)]
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t0
        dmax = max(float(cKDTree(b).query(a)[0].max()) for a, b in zip(ref, sample()))
        out["compare"] = {
            "precision": other, "value": roots_per_step / (el2 / args.steps),
            "ms_per_step": 1e3 * el2 / args.steps, "steps": args.steps,
            "speedup_of_mixed_over_fp64": (el2 / elapsed if other == "fp64" else elapsed / el2),
            "max_root_distance_to_main_run": dmax,
            "sampled": f"{len(picks)} fields x {len(rows)} rows",
            "kernels": root_kernels(st2, other),
        }
        log(f"{other}: {1e3 * el2 / args.steps:.0f} ms per step, max root distance {dmax:.2e}")
    if args.multipole and args.star_sums == "direct":
        # the same fields with fast-multipole star sums (a grid per field), in
        # the timed run's precision
        try:
            step(precision, "fmm")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st3 = [step(precision, "fmm") for _ in range(args.steps)]
            torch.cuda.synchronize()
            el3 = time.perf_counter() - t0
        except mlcc.MlccError as e:   # reported, not fatal to the timed run's line
            out["multipole"] = {precision: {"error": str(e)}}
            log(f"multipole {precision}: {e}")
            print(json.dumps(out), flush=True)
            return
        dmax = max(float(cKDTree(b).query(a)[0].max()) for a, b in zip(ref, sample()))
        out["multipole"] = {
            precision: {
                "value": roots_per_step / (el3 / args.steps), "ms_per_step": 1e3 * el3 / args.steps,
                "steps": args.steps, "warmup": 1,
                "speedup_over_timed_run": elapsed / el3,
                "max_root_distance_to_main_run": dmax,
                "sampled": f"{len(picks)} fields x {len(rows)} rows",
                "kernels": root_kernels(st3, precision),
                "stats": {k: st3[-1][k] for k in ("n_subchains", "sweeps", "root_updates",
                                                  "root_updates_f32", "polish_updates",
                                                  "fmm_near_terms", "fmm_far_evals")},
            }
        }
        log(f"multipole {precision}: {1e3 * el3 / args.steps:.0f} ms per step, "
            f"max root distance {dmax:.2e}")
    print(json.dumps(out), flush=True)


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none for this workload or the kernel source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        src = os.path.join(ROOT, vals["kernel_source"])
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if vals.get("workload") != workload or h != vals["source_sha256"]:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(f, m_steps, rows):
    """The oracle as it stands, timed on the host's cores, on a bounded
    sample of the same workload: the centre row of the phase grid cold-started
    from the seeds (not timed), then `rows` warm rows, each seeded with the
    previous row as the paper grows a chain (timed).  roots/s = rows x n_r /
    time (n_r = 2N, + t - 1 for a rectangular field)."""
    import numpy as np

    import oracle
    c = m_steps // 2
    n_r = oracle.num_roots(f)
    log(f"cpu baseline: oracle cold start at row {c}, then {rows} timed warm rows on "
        f"{oracle.num_threads()} threads")
    z, sw0, up0, _ = oracle.aberth_row(f, oracle.phase(c, m_steps))
    t = time.perf_counter()
    ups = 0
    for i in range(1, rows + 1):
        z, sw, up, _ = oracle.aberth_row(f, oracle.phase(c + i, m_steps), z0=z)
        ups += up
    dt = time.perf_counter() - t
    threads = oracle.num_threads()
    # the same oracle on one thread, one more warm row
    oracle.set_num_threads(1)
    t = time.perf_counter()
    _, _, up1, _ = oracle.aberth_row(f, oracle.phase(c + rows + 1, m_steps), z0=z)
    dt1 = time.perf_counter() - t
    oracle.set_num_threads(threads)
    log(f"cpu baseline: {rows * n_r / dt:.3e} roots/s on {threads} threads, "
        f"{n_r / dt1:.3e} on one")
    return {
        "value": rows * n_r / dt,
        "unit": "roots/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{rows} warm rows (phase steps {c + 1}..{c + rows} of {m_steps}, "
                   f"{n_r} roots each, {f.n} stars), each seeded with the previous "
                   f"row, after an untimed cold start at row {c}: {ups} root updates in "
                   f"{dt:.1f} s"),
        "one_thread": {"value": n_r / dt1, "unit": "roots/s",
                       "sample": f"warm row {c + rows + 1}: {up1} root updates in {dt1:.1f} s"},
    }


if __name__ == "__main__":
    main()
