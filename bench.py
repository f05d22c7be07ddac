"""Throughput of the whole critical-curve -> caustic -> crossing-map ->
distance-map path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload n10k]

One step = set_lenses + find_critical_curves (all m+1 rows, with the caustic
image of every root mapped in the same pass) + caustic_crossings +
caustic_distances on one seeded synthetic field whose inputs are already in
HBM, in the paper's double precision.  Prints one JSON line:
  value           roots/s = m * 2N / (seconds per step)
  roofline        the root finder's dominant kernel (the persistent launch
                  that runs every pass, by default): algorithmic FLOP per
                  launch / its HIP-event-timed duration, against the FP64
                  vector peak
  accuracy        the timed run's roots and caustics against oracle rows
  forms           the other forms on the same field, each with its own few
                  steps: FP32 root-root sums in warm rows, mixed precision
                  (chain prediction, and FP32 bulk sweeps without it),
                  multipole star sums; speed-up over the timed run and the
                  error against the same oracle rows
  n1k, batched    (default workload) the 1,000-star workload with its
                  1024^2 crossing map, and 256 fields in one call against
                  one call per field and against FP64
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

# 256 CU x 2.4 GHz x 128 FLOP/clk.  The library is built without packed FP32
# instructions, and an unpacked FP32 FMA issues at the FP64 rate on this
# chip (the 157.3 TFLOP/s FP32 figure counts two FMAs per packed
# instruction), so every algorithmic FLOP, FP64 or FP32, is priced against
# this peak.
FP64_VECTOR_PEAK_TFLOPS = 78.6
METRIC = "critical-curve roots/s at N=1e4 stars, % FP64 VALU peak; mixed vs FP64"

WORKLOAD_TEXT = {
    "n10k": "N=10,000 equal-mass stars, kappa_star=0.5, kappa_s=0, gamma=0.3, uniform disk; "
            "20,000 phase steps (20,001 rows x 20,000 roots); caustics; N_cc int32 2048^2 and "
            "FP64 distance map over 40x40 theta_E",
    "n1k": "N=1,000 Salpeter stars on [0.08,1], kappa_star=0.4, kappa_s=0.2, gamma=0.45; "
           "10,000 phase steps (2,000 roots each); caustics; N_cc 1024^2 over 20x20 theta_E",
    "n10k_mixed": "the n10k field and grids in mixed precision: warm rows polished by FP64 "
                  "Newton steps from the chain prediction and checked by the row identities, "
                  "FP32 Aberth sweeps for cold starts, FP64 lens mapping",
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

DTYPE = {"fp64": "f64", "fp64_r32": "f64 (warm-row root-root terms f32)", "mixed": "f32+f64"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n10k", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--subchains", type=int, default=0, help="0 = library choice")
    ap.add_argument("--precision", default=None, choices=sorted(DTYPE),
                    help="default: the workload's own (mixed for n10k_mixed and batched)")
    ap.add_argument("--predictor", type=int, default=2, choices=[0, 1, 2],
                    help="warm-row start: 0 previous row, 1 linear, 2 quadratic extrapolation")
    ap.add_argument("--cpu-baseline", dest="cpu_baseline", action="store_true", default=True)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--schedule", default="persistent", choices=["rounds", "persistent"],
                    help="root-finder scheduling: global rounds, or one persistent launch")
    ap.add_argument("--cpu-rows", type=int, default=12,
                    help="warm rows of the oracle timed for the CPU baseline")
    ap.add_argument("--star-sums", dest="star_sums", default="direct", choices=["direct", "fmm"],
                    help="star sums of the timed run: direct, or fast multipole")
    ap.add_argument("--forms", dest="forms", action="store_true", default=True,
                    help="after the timed run, the other precisions and the multipole star sums "
                         "on the same field, each for --form-steps steps")
    ap.add_argument("--no-forms", dest="forms", action="store_false")
    ap.add_argument("--form-steps", type=int, default=2)
    ap.add_argument("--oracle-rows", type=int, default=3,
                    help="rows of the phase grid the oracle cold-starts to measure the error of "
                         "every form (0: none)")
    ap.add_argument("--extra", dest="extra", action="store_true", default=True,
                    help="default workload: also the n1k block and the batched block")
    ap.add_argument("--no-extra", dest="extra", action="store_false")
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

    from paper_2506_02121_amd import fields

    wl = fields.workload(args.workload, args.seed)
    precision = args.precision or wl.precision
    if wl.fields:
        blk = batched_block(args, wl, precision, args.steps, args.warmup, serial=args.serial,
                            fp64=args.forms, multipole=args.forms,
                            oracle_fields=4 if args.oracle_rows > 0 else 0)
        out = headline(blk, f"batched: {WORKLOAD_TEXT['batched']}", precision)
        print(json.dumps(out), flush=True)
        return
    blk, field_for_cpu = single_block(args, wl, precision, args.steps, args.warmup,
                                      forms=args.forms, directional=args.directional,
                                      oracle_rows_n=args.oracle_rows)
    out = headline(blk, f"{args.workload}: {WORKLOAD_TEXT[args.workload]}", precision)
    if args.extra and args.workload == "n10k":
        # the other workloads the metric is compared on, each with its own
        # small step count
        n1k = single_block(args, fields.workload("n1k", args.seed), "fp64", 5, 2, forms=False,
                           directional=0, oracle_rows_n=3)[0]
        n1k["config"]["workload"] = f"n1k: {WORKLOAD_TEXT['n1k']}"
        out["n1k"] = n1k
        bat = batched_block(args, fields.workload("batched", args.seed), "mixed", 1, 1,
                            serial=True, fp64=True, multipole=False, oracle_fields=4)
        bat["config"]["workload"] = f"batched: {WORKLOAD_TEXT['batched']}"
        out["batched"] = bat
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(field_for_cpu, wl.m_steps, args.cpu_rows)
    print(json.dumps(out), flush=True)


def headline(blk, workload_text, precision):
    """The contract's JSON line around a block's measurements."""
    out = {
        "metric": METRIC,
        "value": blk["value"],
        "unit": "roots/s",
        "n_gpus": 1,
        "steps": blk["steps"],
        "warmup": blk["warmup"],
        "ms_per_step": blk["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[precision],
        "data": "synthetic",
        "config": dict(workload=workload_text, **blk.pop("config")),
    }
    out.update({k: v for k, v in blk.items() if k not in out})
    return out


# ---------------------------------------------------------------------------
# roofline of the root finder
# ---------------------------------------------------------------------------

def kernel_line(stats, name, flop_keys, ms_key, n_key, dtype):
    """Roofline of one root-finder kernel of the round schedule: algorithmic
    FLOP of the launches that did work over their HIP-event time."""
    flop = sum(sum(s[k] for k in flop_keys) for s in stats)
    ms = sum(s[ms_key] for s in stats)
    launches = sum(s[n_key] for s in stats)
    achieved = flop / (ms * 1e-3) / 1e12 if ms > 0 else None
    return {"kernel": name, "dtype": dtype, "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS if achieved else None,
            "time_s": ms * 1e-3, "avg_launch_ms": ms / launches if launches else None,
            "launches": launches}


def root_kernels(stats):
    """Rooflines of the root finder's launches.  The persistent launch runs
    every pass kind; its FLOP are split by the precision they run in."""
    f64 = sum(s["algorithmic_flop"] + s["algorithmic_flop_polish"] for s in stats)
    f32 = sum(s["algorithmic_flop_f32"] + s["algorithmic_flop_sweep_roots"] for s in stats)
    if any(s["persistent_launches"] for s in stats):
        ms = sum(s["persistent_ms"] for s in stats)
        launches = sum(s["persistent_launches"] for s in stats)
        achieved = (f64 + f32) / (ms * 1e-3) / 1e12 if ms > 0 else None
        return [{"kernel": "aberth_persistent", "dtype": "f64" if f32 == 0 else "f64+f32",
                 "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                 "frac": achieved / FP64_VECTOR_PEAK_TFLOPS if achieved else None,
                 "time_s": ms * 1e-3, "avg_launch_ms": ms / launches, "launches": launches,
                 "flop_per_launch": (f64 + f32) / launches, "flop_f64": f64, "flop_f32": f32,
                 "fp32_share_of_flop": f32 / (f64 + f32) if f64 + f32 else 0.0}]
    ks = [kernel_line(stats, "aberth_sweep_f64",
                      ["algorithmic_flop", "algorithmic_flop_sweep_roots"],
                      "sweep_ms", "sweep_launches", "f64")]
    if any(s["sweep_f32_launches"] for s in stats):
        ks.append(kernel_line(stats, "aberth_sweep_f32", ["algorithmic_flop_f32"], "sweep_f32_ms",
                              "sweep_f32_launches", "f32"))
    if any(s["polish_launches"] for s in stats):
        ks.append(kernel_line(stats, "newton_polish_f64", ["algorithmic_flop_polish"], "polish_ms",
                              "polish_launches", "f64"))
    return ks


def roofline(stats, workload, star_sums):
    kernels = root_kernels(stats)
    d = max(kernels, key=lambda k: k["time_s"])
    out = {
        "bound": "alu", "kernel": d["kernel"], "achieved": d["achieved"], "peak": d["peak"],
        "unit": "TFLOP/s", "frac": d["frac"],
        "traffic": measured_traffic(d["kernel"], workload) if star_sums == "direct" else None,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "avg_launch_ms": d["avg_launch_ms"], "launches": d["launches"],
        "kernels": kernels,
    }
    if star_sums == "fmm":
        out["note"] = ("fast-multipole star sums: FLOP = 29 per near star term + (26 p + 20) per "
                       "series evaluation + root terms")
    return out


def valu_fma_tflops(kind):
    """The device's FP64 ("fp64") or unpacked FP32 ("fp32") FMA-chain rate in
    TFLOP/s from libvalu_probe.so, the measurement aid built beside the
    library (not part of its C-ABI)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2506_02121_amd", "libvalu_probe.so")
    lib = ctypes.CDLL(path)
    lib.valu_probe_fma_tflops.argtypes = [ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.valu_probe_fma_tflops.restype = ctypes.c_int
    out = ctypes.c_double(0.0)
    rc = lib.valu_probe_fma_tflops(0, {"fp64": 0, "fp32": 1}[kind], ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"valu probe failed ({rc})")
    return out.value


def measured_peaks(k):
    """The device's measured FMA-chain rates beside the published peak, and
    the dominant kernel's fraction of them (FP64 and FP32 parts each priced
    at their measured rate)."""
    p64 = valu_fma_tflops("fp64")
    p32 = valu_fma_tflops("fp32")
    out = {"fp64_fma_tflops": p64, "fp32_fma_tflops": p32,
           "method": "8 independent FMA chains per lane, 8 waves per SIMD, HIP events"}
    f64, f32 = k.get("flop_f64"), k.get("flop_f32")
    if f64 is not None and k["time_s"] > 0:
        out["kernel_frac_of_measured"] = (f64 / (p64 * 1e12) + f32 / (p32 * 1e12)) / k["time_s"]
    return out


def s0_updates(st):
    """Root updates of every kind in one call."""
    return st["root_updates"] + st["root_updates_f32"] + st["polish_updates"]


# ---------------------------------------------------------------------------
# error against the oracle
# ---------------------------------------------------------------------------

def oracle_rows(f, m_steps, rows):
    """The oracle's roots and caustics of the given rows, each cold-started
    from the seeds at its phase, with F' at every root (for the tolerance)."""
    import oracle
    refs = []
    t = time.perf_counter()
    for j in rows:
        phi = oracle.phase(int(j), m_steps)
        z, _, _, _ = oracle.aberth_row(f, phi)
        refs.append((int(j), z, oracle.lens_map(f, z), oracle.eval_F(f, phi, z)[1]))
    log(f"oracle: {len(rows)} rows of {len(refs[0][1]) if refs else 0} roots in "
        f"{time.perf_counter() - t:.1f} s")
    return refs


def errors_vs_oracle(f, refs, get_row):
    """Max distance of the GPU's roots and caustics from the oracle's on the
    sampled rows (nearest-neighbour pairing, which must be one-to-one), and
    the max ratio of the root distance to the conditioning-aware tolerance
    1e-9 + 1e-9 / (|1 - kappa_s| |F'(z_ref)|) of the paper's cutoffs."""
    import numpy as np
    from scipy.spatial import cKDTree
    a = abs(1.0 - f.kappa_s)
    wz = ww = ratio = 0.0
    one_to_one = True
    for j, z, w, fp in refs:
        zg, wg = get_row(j)
        d, idx = cKDTree(np.stack([zg.real, zg.imag], 1)).query(np.stack([z.real, z.imag], 1))
        one_to_one &= np.unique(idx).size == z.size
        wz = max(wz, float(d.max()))
        ratio = max(ratio, float((d / (1e-9 + 1e-9 / (a * np.abs(fp)))).max()))
        ww = max(ww, float(np.abs(wg[idx] - w).max()))
    return {"max_root_error": wz, "max_caustic_error": ww, "max_error_over_tolerance": ratio,
            "one_to_one": bool(one_to_one), "rows": [r[0] for r in refs]}


# ---------------------------------------------------------------------------
# one field: the timed run and the other forms on the same field
# ---------------------------------------------------------------------------

def single_block(args, wl, precision, steps, warmup, forms, directional, oracle_rows_n):
    import numpy as np
    import torch

    from paper_2506_02121_amd import fields, mlcc

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

    def step(prec, predictor, star_sums):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        load(ctx)
        # roots and, in the same pass, their caustic images
        _, _, _, _, cn, st, _ = ctx.find_critical_curves(
            m_steps, n_subchains=args.subchains, timing=True, caustics=True,
            out=(roots_re, roots_im), caustics_out=(w_re, w_im), precision=prec,
            predictor=predictor, schedule=args.schedule, star_sums=star_sums)
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

    def run(prec, warmup_, steps_, predictor, star_sums, label):
        for i in range(warmup_):
            t = time.perf_counter()
            step(prec, predictor, star_sums)
            torch.cuda.synchronize()
            log(f"{wl.name} {label} warmup {i}: {time.perf_counter() - t:.3f} s")
        stats = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps_):
            ts = time.perf_counter()
            stats.append(step(prec, predictor, star_sums))
            torch.cuda.synchronize()
            log(f"{wl.name} {label} step {i}: {time.perf_counter() - ts:.3f} s, "
                f"{stats[-1]['sweeps']} passes / rounds")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, stats

    def get_row(j):
        z = roots_re[j].cpu().numpy() + 1j * roots_im[j].cpu().numpy()
        w = w_re[j].cpu().numpy() + 1j * w_im[j].cpu().numpy()
        return z, w

    elapsed, stats = run(precision, warmup, steps, args.predictor, args.star_sums, precision)
    roots_per_step = m_steps * n_r
    stages = stage_ms(stats)
    s0 = stats[-1]
    rf = roofline(stats, wl.name, args.star_sums)
    if rf["kernel"] == "aberth_persistent":
        rf["measured_peak"] = measured_peaks(rf["kernels"][0])
    rf["flop_per_root_update"] = 29 * n + 10 * (n_r - 1)
    ncc_h = ncc.cpu().numpy()
    updates_per_root_row = s0_updates(s0) / float(n_r * (rows + s0["n_subchains"]))
    blk = {
        "value": roots_per_step / (elapsed / steps),
        "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * elapsed / steps,
        "config": {"n_stars": n, "roots_per_row": n_r, "phase_steps": m_steps,
                   "grid": [grid.nx, grid.ny], "precision": precision,
                   "predictor": args.predictor, "schedule": args.schedule,
                   "star_sums": args.star_sums, "seed": args.seed},
        "roofline": rf,
        "stage_ms": stages,
        "root_updates_per_s": s0_updates(s0) / (elapsed / steps),
        "stats": {"sweeps_per_step": s0["sweeps"], "root_updates_per_step": s0["root_updates"],
                  "root_updates_f32_per_step": s0["root_updates_f32"],
                  "polish_updates_per_step": s0["polish_updates"],
                  "rows_fallback": s0["rows_fallback"],
                  "updates_per_root_per_row": updates_per_root_row,
                  "n_subchains": s0["n_subchains"], "cold_sweeps": s0["cold_sweeps"],
                  "max_row_sweeps": s0["max_row_sweeps"], "match_maxdist": s0["match_maxdist"],
                  "cold_restarts": s0["cold_restarts"],
                  "ncc_max": int(ncc_h.max()), "ncc_min": int(ncc_h.min())},
    }
    if args.star_sums == "fmm":
        blk["stats"].update({"fmm_near_terms_per_step": s0["fmm_near_terms"],
                             "fmm_far_evals_per_step": s0["fmm_far_evals"]})
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
    # the map stages against the HBM roof, from their algorithmic bytes:
    # crossing map 32 B of vertices per edge, chain_next, the difference map
    # written and scanned (4 B + 4 B per pixel); distance map 4 B of N_cc
    # in, 8 B of distance and 1 B of mark out per pixel
    npix = grid.nx * grid.ny
    cross_bytes = 32.0 * rows * n_r + 4.0 * n_r + 8.0 * npix
    dist_bytes = 13.0 * npix
    stages["crossing_map_hbm_frac"] = cross_bytes / (stages["crossing_map"] * 1e-3) / 8e12
    stages["distance_map_hbm_frac"] = dist_bytes / (stages["distance_map"] * 1e-3) / 8e12
    if directional > 0:
        blk["directional"] = directional_stage(ctx, grid, ncc, directional)

    refs = []
    if oracle_rows_n > 0:
        rng = np.random.default_rng(2025)
        sample = [0, m_steps // 2] + rng.integers(1, m_steps, size=8).tolist()
        sample = sorted(set(sample[:oracle_rows_n]))
        refs = oracle_rows(f, m_steps, sample)
        blk["accuracy"] = errors_vs_oracle(f, refs, get_row)
        log(f"{wl.name} {precision}: {blk['accuracy']}")

    if forms:
        form_list = [("fp64_r32", args.predictor, "direct"), ("mixed", args.predictor, "direct"),
                     ("mixed", 0, "direct"), ("fp64", args.predictor, "fmm"),
                     ("mixed", args.predictor, "fmm")]
        if f.sheet is not None:   # a rectangular field is solved in the FP64 forms only
            form_list = [q for q in form_list if q[0] != "mixed"]
        blk["forms"] = {}
        fs = max(1, args.form_steps)
        for prec, pred, ss in form_list:
            if (prec, pred, ss) == (precision, args.predictor, args.star_sums):
                continue
            name = prec + ("_predictor0" if pred == 0 else "") + ("_multipole" if ss == "fmm" else "")
            try:
                el, st = run(prec, 1, fs, pred, ss, name)
            except mlcc.MlccError as e:   # reported, not fatal to the timed run's line
                blk["forms"][name] = {"error": str(e)}
                log(f"{name}: {e}")
                continue
            stage_ms(st)
            ks = root_kernels(st)
            dom = max(ks, key=lambda k: k["time_s"])
            entry = {
                "precision": prec, "predictor": pred, "star_sums": ss,
                "value": roots_per_step / (el / fs), "ms_per_step": 1e3 * el / fs,
                "steps": fs, "warmup": 1,
                "speedup_over_timed_run": elapsed / steps / (el / fs),
                "kernel": dom["kernel"], "achieved": dom["achieved"], "frac": dom["frac"],
                "fp32_share_of_flop": dom.get("fp32_share_of_flop"),
                "stats": {k: st[-1][k] for k in ("n_subchains", "sweeps", "root_updates",
                                                 "root_updates_f32", "polish_updates",
                                                 "rows_fallback", "fmm_near_terms",
                                                 "fmm_far_evals")},
            }
            if refs:
                entry["accuracy"] = errors_vs_oracle(f, refs, get_row)
            blk["forms"][name] = entry
            log(f"{name}: {entry['ms_per_step']:.1f} ms per step "
                f"({entry['speedup_over_timed_run']:.2f}x), {entry.get('accuracy')}")
    ctx.close()
    del roots_re, roots_im, w_re, w_im, ncc, dist, bl
    torch.cuda.empty_cache()
    return blk, f


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


# ---------------------------------------------------------------------------
# many fields in one call
# ---------------------------------------------------------------------------

def batched_block(args, wl, precision, steps, warmup, serial, fp64, multipole, oracle_fields):
    """Many independent fields in one root-finder call (roots and caustics
    of every field); value = phase steps x total roots per row / seconds.
    Beside it: every field alone (one call each), the same batch in plain
    FP64, and the error of each against oracle rows of sampled fields."""
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
    log(f"batched: {len(fs)} fields, {n_tot} stars, {2 * n_tot} roots per row, "
        f"{4 * total * 8 / 2**30:.1f} GiB of roots and caustics")
    roots_re = torch.empty(total, dtype=torch.float64, device=dev)
    roots_im = torch.empty_like(roots_re)
    w_re = torch.empty_like(roots_re)
    w_im = torch.empty_like(roots_re)
    ctx = mlcc.Context(0)
    torch.cuda.synchronize()

    def step(prec, star_sums="direct"):
        ctx.set_lenses_batched(off, x, y, mm, ks, gs)
        _, _, _, _, cn, st, _ = ctx.find_critical_curves(
            m_steps, n_subchains=args.subchains, timing=True, caustics=True,
            out=(roots_re, roots_im), caustics_out=(w_re, w_im), precision=prec,
            predictor=args.predictor, schedule=args.schedule, star_sums=star_sums)
        return st

    def timed(prec, warmup_, steps_, star_sums="direct", label=""):
        for i in range(warmup_):
            t = time.perf_counter()
            step(prec, star_sums)
            torch.cuda.synchronize()
            log(f"batched {label or prec} warmup {i}: {time.perf_counter() - t:.3f} s")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = []
        for i in range(steps_):
            ts = time.perf_counter()
            st.append(step(prec, star_sums))
            torch.cuda.synchronize()
            log(f"batched {label or prec} step {i}: {time.perf_counter() - ts:.3f} s")
        return time.perf_counter() - t0, st

    # each field's (roots offset, chain_next offset, n_r) in the flat outputs
    blocks = [((m_steps + 1) * 2 * int(a), 2 * int(a), 2 * int(b - a))
              for a, b in zip(off[:-1], off[1:])]
    order = np.argsort([f.n for f in fs])
    picks = sorted(set(order[np.linspace(0, len(fs) - 1, max(1, oracle_fields)).astype(int)]
                       .tolist())) if oracle_fields else []
    sample_rows = [0, 1234, m_steps // 2]
    refs = {i: oracle_rows(fs[i], m_steps, sample_rows) for i in picks}

    def get_field_row(i):
        o, _, n_r = blocks[i]

        def get(j):
            a = slice(o + j * n_r, o + (j + 1) * n_r)
            return (roots_re[a].cpu().numpy() + 1j * roots_im[a].cpu().numpy(),
                    w_re[a].cpu().numpy() + 1j * w_im[a].cpu().numpy())
        return get

    def accuracy():
        if not picks:
            return None
        per = [errors_vs_oracle(fs[i], refs[i], get_field_row(i)) for i in picks]
        return {"max_root_error": max(p["max_root_error"] for p in per),
                "max_caustic_error": max(p["max_caustic_error"] for p in per),
                "max_error_over_tolerance": max(p["max_error_over_tolerance"] for p in per),
                "one_to_one": all(p["one_to_one"] for p in per),
                "fields": [int(i) for i in picks], "n_stars": [int(fs[i].n) for i in picks],
                "rows": sample_rows}

    star_sums = getattr(args, "star_sums", "direct") if args.workload == "batched" else "direct"
    elapsed, stats = timed(precision, warmup, steps, star_sums=star_sums)
    roots_per_step = m_steps * 2 * n_tot
    s0 = stats[-1]
    blk = {
        "value": roots_per_step / (elapsed / steps), "steps": steps, "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "config": {"fields": len(fs), "total_stars": n_tot, "roots_per_row": 2 * n_tot,
                   "phase_steps": m_steps, "precision": precision, "predictor": args.predictor,
                   "schedule": args.schedule, "star_sums": star_sums, "seed": args.seed},
        "roofline": roofline(stats, "batched", star_sums),
        "stats": {k: s0[k] for k in ("sweeps", "root_updates", "root_updates_f32",
                                     "polish_updates", "rows_fallback", "n_subchains",
                                     "cold_sweeps", "max_row_sweeps", "match_maxdist")},
        "accuracy": accuracy(),
    }
    if serial:
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
                    schedule=args.schedule, star_sums=star_sums,
                    out=(roots_re[sl].view(shape), roots_im[sl].view(shape)),
                    caustics_out=(w_re[sl].view(shape), w_im[sl].view(shape)))
            torch.cuda.synchronize()
        serial_pass()   # warm-up: buffers grow to the largest field once
        t0 = time.perf_counter()
        serial_pass()
        el_s = time.perf_counter() - t0
        blk["serial"] = {
            "what": "every field alone, one find_critical_curves call each (roots and caustics)",
            "value": roots_per_step / el_s, "ms_per_step": 1e3 * el_s,
            "speedup_of_batched": el_s / (elapsed / steps), "accuracy": accuracy()}
        log(f"batched: serial {el_s:.3f} s for {len(fs)} calls")
    if fp64 and precision != "fp64":
        el2, st2 = timed("fp64", 0, 1, star_sums=star_sums)
        ks2 = root_kernels(st2)
        blk["fp64"] = {
            "what": "the same batch in one call, plain FP64",
            "value": roots_per_step / el2, "ms_per_step": 1e3 * el2, "steps": 1,
            "speedup_of_timed_form_over_fp64": el2 / (elapsed / steps),
            "frac": ks2[0]["frac"], "accuracy": accuracy()}
    if multipole and star_sums == "direct":
        try:
            el3, st3 = timed(precision, 1, steps, "fmm", f"{precision} multipole")
            blk["multipole"] = {
                "value": roots_per_step / (el3 / steps), "ms_per_step": 1e3 * el3 / steps,
                "speedup_over_timed_run": elapsed / el3, "accuracy": accuracy(),
                "kernels": root_kernels(st3)}
        except mlcc.MlccError as e:   # reported, not fatal to the timed run's line
            blk["multipole"] = {"error": str(e)}
            log(f"batched multipole: {e}")
    ctx.close()
    del roots_re, roots_im, w_re, w_im
    torch.cuda.empty_cache()
    return blk


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


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(f, m_steps, rows):
    """The oracle as it stands, timed on the host's cores, on a bounded
    sample of the same workload: the centre row of the phase grid cold-started
    from the seeds (not timed), then `rows` warm rows, each seeded with the
    previous row as the paper grows a chain (timed).  roots/s = rows x n_r /
    time (n_r = 2N, + t - 1 for a rectangular field)."""
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
    out = {
        "value": rows * n_r / dt,
        "unit": "roots/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{rows} warm rows (phase steps {c + 1}..{c + rows} of {m_steps}, "
                   f"{n_r} roots each, {f.n} stars), each seeded with the previous "
                   f"row (the paper's warm start, {ups / (rows * n_r):.2f} root updates per "
                   f"root per row; the GPU's chain prediction needs about one), after an "
                   f"untimed cold start at row {c}: {ups} root updates in {dt:.1f} s"),
        "one_thread": {"value": n_r / dt1, "unit": "roots/s",
                       "sample": f"warm row {c + rows + 1}: {up1} root updates in {dt1:.1f} s"},
        # per root update (one pass of a root over the stars and the other
        # roots), the unit that does not depend on how a row is warm-started
        "root_updates_per_s": ups / dt,
    }
    out.update(host_cpu())
    return out


if __name__ == "__main__":
    main()
