"""Benchmark of the mixture-of-media random walk on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-c3] [--no-c4]
                    [--micro] [--lut N [--lut-photons P]] [--layers N [--layers-photons P]]

One step is one pass of the whole path over the 81-wavelength three-medium
workload (81 wavelengths 380-780 nm, per-medium sigma_t log-uniform in
[0.1, 100] mm^-1, alpha uniform in [0.30, 0.999], g uniform in [0, 0.95],
Dirichlet(1,1,1) weights, Fresnel boundary n = 1.4, 2^20 paths per
wavelength, 256 log bins over [1e-3, 50] mm):
    rw_batch_forward (persistent, graph replay, live-path mask) -> rw_finalize ->
    rw_batch_adjoint (path replay of the paths the mask marks, with cotangents
    v_R = 1, v_bins ~ N(0, 1)).
Each step uses a fresh seed.  The metric is path vertices per second over the
forward and the adjoint, counting the vertices actually walked (exact int64
counts from the device): the adjoint replays only the paths that left the top
surface, about a quarter of the forward's vertices, so a step walks fewer
vertices than forward + full replay while giving the same gradient.  The
plain static-grid launches (rw_forward + rw_adjoint, full replay) and the
batched launches with a full replay are timed on the same seeds; the tallies
of one seed are compared across the forms (bit-identical forward sums,
gradients equal to FP64 rounding) for the batched/plain ratio at matched
statistical error.

Extra fields: the batched sweep of 65,536 three-medium sets x 16 wavelengths
at 4,096 paths (one persistent launch) against one plain static launch over
the same units, and its per-set plain launches timed on a subset of sets; the
adjoint sweep (1,024 sets x 81 wavelengths x 2^14 paths, random bin
cotangents); the inverse fit (4,096 targets x 81 wavelengths, 200 Adam steps
at 2^12 paths, by the adjoint and by the LUT route); hero wavelengths on the
two-layer tones and Dwivedi sampling (on the tiny workload's isotropic media
and on the 81-wavelength mixture), each as an efficiency gain over the plain
walk; the autotuned step; the roofline of the dominant kernel (ALU-bound: VALU issue
slots per vertex x vertices / measured kernel time, against the issue peak of
256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz); and the FP64 CPU oracle timed on a
bounded sample of the same workload.

Prints one JSON line.  Inputs are synthetic (seeded); nothing is read from
outside the repository.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC path vertices/s, fwd & adjoint, batched vs plain, at matched stat. error"

# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 instruction
# occupies a SIMD for 4 cycles at full rate)
N_CU, SIMD_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
ISSUE_PEAK = N_CU * SIMD_PER_CU * LANES_PER_SIMD * CLOCK_HZ  # lane-slots / s

# Algorithmic work of one vertex (what the method computes, not loop control),
# in VALU lane-slots: each op weighted by its issue cost relative to a full-rate
# FP32 FMA, as measured by `bench.py --micro` on the MI355X
# (profiles/issue_rates_micro.md).  The counts are those of the compiled
# plain-collision vertex (its draw, then the straight-line step), without
# register moves, draw addressing or the ballot:
#   random numbers: one Philox4x32-10 block = 10 rounds x (2 32x32->64
#     multiply-adds + 2 three-input XORs, one v_bitop3_b32 each);
#   the draw (26): 4 word->float conversions (shift, or, subtract, ~10 ops),
#     the flight's scale, the Henyey-Greenstein inversion (~10 ops), sin(theta)
#     from (1 - mu)(1 + mu) (2), the in-plane components (2); with log, rcp,
#     sqrt, sin and cos;
#   the step (35): flight end depth and the surface and roulette tests (5),
#     position (2), implicit capture (1; the weight product is the roulette
#     test's), the Duff et al. frame and rotation (~20) with the frame's rcp,
#     the renormalisation by one Newton step (7);
#   a surface hit (about 1 vertex in 20): distance rcp + 3 ops, Fresnel ~15 ops
#     + sqrt + rcp.
# The adjoint adds the score bookkeeping: flight-length sum (2), collision
# count (1), g-score fma chain (2).
ALG_MAD64_PER_VERTEX = 20
ALG_XOR3_PER_VERTEX = 20
ALG_FP32_PER_VERTEX = 62          # 26 + 35 + 1/20 of a surface hit's 18
ALG_FP32_ADJ_EXTRA = 5
ALG_TRANS_PER_VERTEX = 6.15       # log, 2 rcp, sqrt, sin, cos + 1/20 x (3 at a surface hit)
# measured issue costs (FMA = 1); a transcendental is priced amid FMA work
COST_MAD64, COST_XOR3, COST_TRANS = 1.19, 1.16, 1.84


# Secondary measure: algorithmic FP32 FLOP per collision vertex, an FMA
# counting 2: 18 FMA, 23 mul, 10 add/sub/min and 6 transcendentals (counted 1
# each) in the flight, capture, Henyey-Greenstein inversion and rotation, plus
# about 1/20 of a surface hit's 15 ops.  Against the FP32 vector peak (which
# assumes packed FMAs) the Philox integer work, which is not FLOPs, keeps this
# low whatever the kernel does.
ALG_FLOP_PER_VERTEX = 76.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


def alg_slots_per_vertex(adjoint: bool) -> float:
    return (ALG_MAD64_PER_VERTEX * COST_MAD64 + ALG_XOR3_PER_VERTEX * COST_XOR3 +
            ALG_FP32_PER_VERTEX + (ALG_FP32_ADJ_EXTRA if adjoint else 0) +
            ALG_TRANS_PER_VERTEX * COST_TRANS)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_27604_amd", "csrc")
    for name in ("rw_device.hpp", "rw_internal.hpp", "rw_kernels.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name: str):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/traffic.json),
    used only while the kernel sources still hash to the measured version."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel_name)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def load_counters(kernel_name: str):
    """rocprofv3 VALU counters of the kernel (profiles/valu_counters.json): VALU
    busy calibrated against a saturating FMA stream x active-lane fraction, used
    only while the kernel sources still hash to the profiled version."""
    path = os.path.join(ROOT, "profiles", "valu_counters.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel_name)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return {k: e[k] for k in ("valu_busy_vs_fma", "active_lane_fraction",
                              "exec_weighted_utilisation", "transcendental_share",
                              "transcendental_rate_fraction")}


def host_cpu():
    """Cores this process may use (at most 16, the host share of one GPU) and
    the CPU model."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, min(cores, 16)), model


def micro(args):
    import ctypes

    import torch

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2606_27604_amd", "librw_micro.so"))
    lib.rw_micro_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.rw_micro_run.restype = ctypes.c_float
    names = ["fma_f32", "mad_u64_u32", "xor3_b32", "log_f32", "sin_f32", "rcp_f32", "sqrt_f32",
             "rsq_f32", "mul_hi_u32", "philox_block", "log_amid_4_fma"]
    grid, iters = N_CU * 16, 4096
    out = torch.zeros(grid * 256, dtype=torch.int32, device="cuda")
    res = {}
    for op, name in enumerate(names):
        lib.rw_micro_run(op, grid, 64, ctypes.c_void_p(out.data_ptr()))  # warm-up
        ms = min(lib.rw_micro_run(op, grid, iters, ctypes.c_void_p(out.data_ptr())) for _ in range(3))
        per = 1 if name == "philox_block" else (16 if name == "mad_u64_u32" else 8)
        rate = grid * 256.0 * iters * per / (ms * 1e-3)
        res[name] = rate
    fma = res["fma_f32"]
    rep = {k: {"lane_ops_per_s": v, "issue_cost_vs_fma": fma / v} for k, v in res.items()}
    # groups of four FMAs and one log: the log's own cost is the group's less four
    rep["log_amid_4_fma"]["issue_cost_vs_fma"] -= 4.0
    rep["issue_peak_lane_slots_per_s"] = ISSUE_PEAK
    rep["fma_fraction_of_issue_peak"] = fma / ISSUE_PEAK
    print(json.dumps(rep, indent=1))


def cpu_baseline(wl, seed, max_seconds=30.0):
    """The FP64 oracle on the host on a bounded sample of the same workload: all
    81 wavelengths, forward + adjoint, at a path count doubled from 2^16 until one
    pass takes 8 s (or reaches the workload's 2^20)."""
    from oracle import oracle as O

    cores, model = host_cpu()
    paths = 1 << 16
    geo = O.Geometry(n_media=3, n_rel=wl.n_rel, n_bins=wl.n_bins)
    total_v, total_t = 0, 0.0
    rng = np.random.default_rng(99)
    cot_B = rng.standard_normal((wl.n_units, wl.n_bins + 2))
    while True:
        t0 = time.perf_counter()
        _, _, vert = O.forward(geo, wl.sigma_t, wl.albedo, wl.g, wl.weight, paths, seed,
                               n_threads=cores)
        O.adjoint(geo, wl.sigma_t, wl.albedo, wl.g, wl.weight, paths, seed,
                  cot_R=np.ones(wl.n_units), cot_bins=cot_B, n_threads=cores)
        dt = time.perf_counter() - t0
        total_v, total_t = 2 * int(vert.sum()), dt
        if dt > 8.0 or paths >= wl.paths_per_unit or dt * 2 > max_seconds:
            break
        paths *= 2
    return {"value": total_v / total_t, "unit": "vertices/s", "cores": cores, "kind": "oracle",
            "per_core": total_v / total_t / cores, "cpu_model": model,
            "sample": f"81 wavelengths x {paths} paths (forward + adjoint), FP64, "
                      f"{total_v} vertices in {total_t:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--c3-sets", type=int, default=65536)
    ap.add_argument("--c3-plain-sets", type=int, default=512)
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-hero", action="store_true")
    ap.add_argument("--no-dwivedi", action="store_true")
    ap.add_argument("--dwivedi-paths", type=int, default=1 << 20)
    ap.add_argument("--hero-tones", type=int, default=64)
    ap.add_argument("--hero-photons", type=int, default=1 << 16)
    ap.add_argument("--c5-targets", type=int, default=4096)
    ap.add_argument("--c5-iters", type=int, default=200)
    ap.add_argument("--c5-lut", type=int, default=800)
    ap.add_argument("--c5-lut-photons", type=int, default=1 << 16)
    ap.add_argument("--c4-sets", type=int, default=1024)
    ap.add_argument("--micro", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run an elementwise copy of 256 MiB in / 256 MiB out (reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the headline legs themselves (the default run adds a separate "
                         "autotuned leg)")
    ap.add_argument("--no-autotune-leg", action="store_true")
    ap.add_argument("--lut", type=int, default=0,
                    help="instead of the step benchmark, time the generation of an N x N "
                         "(alpha, g) lookup table (Sec. 4.2) and print its own JSON line")
    ap.add_argument("--lut-photons", type=int, default=1 << 14)
    ap.add_argument("--lut-cells-per-launch", type=int, default=1 << 17)
    ap.add_argument("--layers", type=int, default=0,
                    help="instead of the step benchmark, time the two-layer tissue walk over N "
                         "synthetic tones x 81 wavelengths and print its own JSON line")
    ap.add_argument("--layers-photons", type=int, default=1 << 16)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the walk would shard by unit with no "
              "communication, but no multi-GPU path is built; --gpus above 1 is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_27604_amd import api, rw, workloads

    if args.micro:
        micro(args)
        return
    if args.lut:
        lut_generation(rw, torch, args)
        return
    if args.layers:
        layered_tones(rw, torch, args)
        return
    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ctx = rw.Context(0)
    stream = torch.cuda.current_stream()
    wl = workloads.config2()
    media = rw.Media.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.n_sets, wl.n_wl)
    geom = rw.Geometry(n_media=3, n_rel=wl.n_rel, n_bins=wl.n_bins, r_min_mm=wl.r_min_mm,
                       r_max_mm=wl.r_max_mm)
    n, P = wl.n_units, wl.paths_per_unit
    rng = np.random.default_rng(2024)
    cot_R = torch.ones(n, dtype=torch.float32, device="cuda")
    cot_B = torch.from_numpy(rng.standard_normal((n, wl.n_bins + 2)).astype(np.float32)).cuda()
    tally = rw.Tally(n, wl.n_bins)
    R_mean = torch.empty(n, dtype=torch.float64, device="cuda")
    R_se, Rr, Rr_se, Pd = (torch.empty_like(R_mean), torch.empty((n, wl.n_bins), dtype=torch.float64,
                                                                  device="cuda"), None, None)
    Rr_se = torch.empty_like(Rr)
    Pd = torch.empty_like(Rr)
    grad = torch.empty((n, 12), dtype=torch.float64, device="cuda")
    sumsq = torch.empty_like(grad)
    avert = torch.empty(n, dtype=torch.int64, device="cuda")
    aflags = torch.zeros(1, dtype=torch.int32, device="cuda")
    mask = rw.new_path_mask(n, P)

    cur = {"ctx": ctx, "tune": args.autotune}

    def step(seed, batched, ev=None, skip=True):
        pm = mask if (batched and skip) else None
        c = cur["ctx"]
        if ev:
            ev[0].record(stream)
        if batched:
            rw.rw_batch_forward(c, media, geom, None, P, seed, tally, autotune=cur["tune"],
                                stream=stream, path_mask=pm)
        else:
            rw.rw_forward(c, media, geom, P, seed, tally, stream=stream)
        if ev:
            ev[1].record(stream)
        rw.rw_finalize(c, geom, n, None, P, tally, R_mean, R_se, Rr, Rr_se, Pd, stream=stream)
        if ev:
            ev[2].record(stream)
        if batched:
            rw.rw_batch_adjoint(c, media, geom, None, P, seed, cot_R, cot_B, grad, sumsq, avert,
                                aflags, autotune=cur["tune"], stream=stream, path_mask=pm)
        else:
            rw.rw_adjoint(c, media, geom, P, seed, cot_R, cot_B, grad, sumsq, avert, aflags,
                          stream=stream)
        if ev:
            ev[3].record(stream)

    def run(batched, seed0, skip=True):
        for i in range(args.warmup):
            step(seed0 + 1000 + i, batched, skip=skip)
        # the per-step vertex sums below, once untimed: torch loads its
        # reduction kernel on first use (about 25 ms, which would stall the
        # first timed step's launch)
        tally.vertices.sum(), avert.sum()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        verts = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(seed0 + i, batched, evs[i], skip=skip)
            verts.append((tally.vertices, avert))
            # vertex counts of this step (device int64), summed without a sync
            verts[-1] = (tally.vertices.sum(), avert.sum())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fwd_ms = [e[0].elapsed_time(e[1]) for e in evs]
        fin_ms = [e[1].elapsed_time(e[2]) for e in evs]
        adj_ms = [e[2].elapsed_time(e[3]) for e in evs]
        vf = [int(a.item()) for a, _ in verts]
        va = [int(b.item()) for _, b in verts]
        return dict(wall=wall, fwd_ms=fwd_ms, fin_ms=fin_ms, adj_ms=adj_ms, vf=vf, va=va)

    bat = run(True, 1)
    flags = rw.rw_check(ctx, tally.flags) | rw.rw_check(ctx, aflags)
    plain = None if args.no_plain else run(False, 1)
    full = None if args.no_plain else run(True, 1, skip=False)

    def outputs(batched, skip):
        step(77, batched, skip=skip)
        torch.cuda.synchronize()
        return tally.R.clone(), tally.bins.clone(), tally.vertices.clone(), grad.clone()

    def matched():
        """The same seed through every launch form: forward sums bit for bit,
        gradients to FP64 rounding (summed in another order)."""
        ref = outputs(True, True)
        res = {}
        for name, b, sk in (("plain", False, False), ("batched_full_replay", True, False)):
            o = outputs(b, sk)
            g0, g1 = ref[3].double(), o[3].double()
            rel = float(((g0 - g1).abs() / (g1.abs() + g1.abs().max(0).values + 1e-300)).max())
            res[name] = {"tallies_bit_identical": bool(torch.equal(ref[0], o[0]) and
                                                       torch.equal(ref[1], o[1]) and
                                                       torch.equal(ref[2], o[2])),
                         "gradient_max_rel_diff": rel}
        return res

    total_v = sum(bat["vf"]) + sum(bat["va"])
    value = total_v / bat["wall"]
    ms_per_step = 1e3 * bat["wall"] / args.steps
    fwd_avg = float(np.mean(bat["fwd_ms"]))
    adj_avg = float(np.mean(bat["adj_ms"]))
    vf_avg = float(np.mean(bat["vf"]))
    va_avg = float(np.mean(bat["va"]))
    if adj_avg >= fwd_avg:
        dom, dom_ms, dom_v = "walk_kernel<3, adjoint>", adj_avg, va_avg
    else:
        # the forward that sets the live-path mask (its own instantiation)
        dom, dom_ms, dom_v = "walk_kernel<3, forward, marked>", fwd_avg, vf_avg
    slots = alg_slots_per_vertex(dom.endswith("adjoint>"))
    achieved = slots * dom_v / (dom_ms * 1e-3) / 1e12
    peak = ISSUE_PEAK / 1e12
    traffic = load_traffic(dom)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded parameter draws; no dataset or trained weights)",
        "config": {"workload": "mixture3-81wl: 81 wavelengths x 2^20 paths, K=3, n=1.4, "
                               "256 log bins [1e-3, 50] mm; step = batched forward + finalize + "
                               "batched adjoint (path replay), fresh seed per step",
                   "units": n, "paths_per_unit": P, "parallelism": "single GPU"},
        "forward_ms": fwd_avg,
        "adjoint_ms": adj_avg,
        "adjoint_replays": "paths that left the top surface (live-path mask of the forward)",
        "adjoint_vertices_per_step": va_avg,
        "forward_vertices_per_step": vf_avg,
        "finalize_ms": float(np.mean(bat["fin_ms"])),
        "forward_vertices_per_s": vf_avg / (fwd_avg * 1e-3),
        "adjoint_vertices_per_s": va_avg / (adj_avg * 1e-3),
        "vertices_per_step": vf_avg + va_avg,
        "spectra_per_s": wl.n_sets * args.steps / bat["wall"],
        "device_flags": flags,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": traffic, "kernel": dom,
                     "slots_per_vertex": slots, "counters": load_counters(dom),
                     "secondary": {
                         "measure": "algorithmic FP32 FLOP/s over the FP32 vector peak",
                         "flop_per_vertex": ALG_FLOP_PER_VERTEX,
                         "achieved_tflops": ALG_FLOP_PER_VERTEX * dom_v / (dom_ms * 1e-3) / 1e12,
                         "peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
                         "frac": ALG_FLOP_PER_VERTEX * dom_v / (dom_ms * 1e-3) / 1e12
                                 / FP32_VECTOR_PEAK_TFLOPS},
                     "note": "achieved = algorithmic VALU lane-slots (ops x measured issue cost) "
                             "per second against 256 CU x 4 SIMD x 16 lanes x 2.4 GHz; traffic = "
                             "HBM bytes per launch from FETCH_SIZE/WRITE_SIZE (copy-calibrated); "
                             "counters = rocprofv3 SQ counters of the same kernel (exec-weighted "
                             "VALU utilisation = VALU busy, calibrated against a saturating FMA "
                             "stream, x active-lane fraction; transcendental lane-ops/s over "
                             "their measured peak)"},
    }
    if plain is not None:
        for name, r in (("plain", plain), ("batched_full_replay", full)):
            rv = sum(r["vf"]) + sum(r["va"])
            out[name] = {"ms_per_step": 1e3 * r["wall"] / args.steps,
                         "vertices_per_s": rv / r["wall"],
                         "forward_ms": float(np.mean(r["fwd_ms"])),
                         "adjoint_ms": float(np.mean(r["adj_ms"])),
                         "adjoint_vertices_per_step": float(np.mean(r["va"]))}
        out["batched_over_plain_speedup"] = plain["wall"] / bat["wall"]
        out["batched_full_replay_over_plain_speedup"] = plain["wall"] / full["wall"]
        m = matched()
        out["matched_statistical_error"] = all(v["tallies_bit_identical"] and
                                               v["gradient_max_rel_diff"] < 1e-9
                                               for v in m.values())
        out["matched_statistical_error_check"] = m
    if not args.no_autotune_leg:
        out["autotuned"] = autotuned_leg(rw, torch, cur, run, bat, args)
    del tally, grad, sumsq
    torch.cuda.empty_cache()

    if not args.no_c3:
        out["batched_sweep"] = c3(ctx, rw, api, workloads, torch, args)
    if not args.no_c4:
        out["adjoint_sweep"] = c4(ctx, rw, workloads, torch, args)
    if not args.no_hero:
        out["hero_wavelengths"] = hero_leg(ctx, rw, api, workloads, torch, args)
    if not args.no_dwivedi:
        out["dwivedi"] = dwivedi_leg(ctx, rw, api, workloads, torch, args)
    if not args.no_c5:
        out["inverse_fit"] = c5(torch, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, seed=5)
    print(json.dumps(out), flush=True)


def autotuned_leg(rw, torch, cur, run, bat, args):
    """The headline step with autotune = 1 on a fresh context: its first
    forward and adjoint calls time the candidate shapes (paths per work item,
    waves per workgroup, wave occupancy) and cache the fastest; the timed steps
    then run with them.  Reports the shapes chosen, read back from the cache
    file, next to the untuned step."""
    import tempfile

    path = os.path.join(tempfile.mkdtemp(prefix="rw_tune_"), "cache.txt")
    old = os.environ.get("RW_AUTOTUNE_CACHE")
    os.environ["RW_AUTOTUNE_CACHE"] = path
    try:
        saved = dict(cur)
        cur["ctx"], cur["tune"] = rw.Context(0), True
        t0 = time.perf_counter()
        r = run(True, 1)  # the warm-up steps include the tuning
        tuned_wall = time.perf_counter() - t0
        cur.update(saved)
    finally:
        if old is None:
            os.environ.pop("RW_AUTOTUNE_CACHE", None)
        else:
            os.environ["RW_AUTOTUNE_CACHE"] = old
    chosen = {}
    with open(path) as f:
        for line in f:
            key, _, val = line.strip().partition("|")
            c, w, o = (int(x) for x in val.split())
            chosen[key] = {"chunk": c, "paths_per_lane_per_item": c // 64, "waves_per_wg": w,
                           "wgs_per_cu": o if o > 0 else "occupancy limit"}
    return {"ms_per_step": 1e3 * r["wall"] / args.steps,
            "forward_ms": float(np.mean(r["fwd_ms"])), "adjoint_ms": float(np.mean(r["adj_ms"])),
            "untuned_ms_per_step": 1e3 * bat["wall"] / args.steps,
            "tuning_and_warmup_s": tuned_wall - r["wall"],
            "same_vertices_as_untuned": r["vf"] == bat["vf"],
            "chosen": chosen,
            "default": {"chunk": 2048, "waves_per_wg": 4, "wgs_per_cu": "occupancy limit"}}


def hero_leg(ctx, rw, api, workloads, torch, args):
    """Hero wavelengths on the two-layer tones: the per-wavelength walk
    (rw_layered_forward, N photons per wavelength) against groups of C
    neighbouring wavelengths sharing N photons per group
    (rw_layered_hero_forward), on the same tones.  Reported per form: the
    launch time, the walked vertices, the median relative standard error of R,
    and the efficiency gain, the median over wavelengths of
    (SE^2 x time) of the per-wavelength walk over that of the hero walk."""
    wl = workloads.layered_tones(args.hero_tones, paths=args.hero_photons)
    L = rw.Layers.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.thickness_mm, wl.n_rel_bottom)
    geom = rw.Geometry(n_media=2, n_rel=wl.n_rel, n_bins=wl.n_bins)
    N = args.hero_photons
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()  # warm-up
        torch.cuda.synchronize()
        e0.record(s)
        r = fn()
        e1.record(s)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    plain, t_plain = timed(lambda: api.layered_forward(ctx, L, geom, N, 3, stream=s))
    se_p = (plain.R_se / plain.R).cpu().numpy()
    res = {"workload": f"two-layer tones: {args.hero_tones} tones x 81 wavelengths, "
                       f"{N} photons per wavelength (per-wavelength walk) or per group",
           "per_wavelength": {"ms": t_plain, "vertices": int(plain.vertices.sum()),
                              "median_rel_se": float(np.median(se_p))}}
    for C in (3, 9):
        h, t_h = timed(lambda: api.layered_hero_forward(ctx, L, geom, C, N - N % C, 3, stream=s))
        assert rw.rw_check(ctx, h.tally.flags) == 0
        se_h = (h.R_se / h.R).cpu().numpy()
        gain = (se_p ** 2 * t_plain) / (se_h ** 2 * t_h)
        res[f"hero_{C}"] = {"ms": t_h, "vertices": int(h.vertices.sum()),
                            "median_rel_se": float(np.median(se_h)),
                            "efficiency_gain_median": float(np.median(gain)),
                            "efficiency_gain_p10_p90": [float(np.quantile(gain, 0.1)),
                                                        float(np.quantile(gain, 0.9))]}
    return res


def dwivedi_leg(ctx, rw, api, workloads, torch, args):
    """Dwivedi sampling (rw_dwivedi_forward) against the plain batched walk at
    the same paths per unit: on the tiny workload's isotropic, index-matched
    half-spaces (16 albedos in [0.5, 0.99], sigma_t = 1) with technique
    probability 1, and on the 81-wavelength mixture (anisotropic, Fresnel
    n = 1.4) with probability 0.2.  Per form: the launch time, the walked
    vertices, per unit the efficiency gain (SE^2 x time of the plain walk over
    that of the Dwivedi walk), median and 10-90 % range, and the z-scores of
    the two estimates of R (heavy-tailed weights show as a low bias there: the
    sample SE then understates the error), and per unit the weight balance
    (R + T + A) / (paths x (1 - F(0))), which is 1 in expectation and falls
    short when the sample misses the weights' tail."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()  # warm-up
        torch.cuda.synchronize()
        e0.record(s)
        r = fn()
        e1.record(s)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    res = {}
    for name, wl, q in (("isotropic_half_spaces", workloads.config1(paths=args.dwivedi_paths), 1.0),
                        ("mixture3_81wl", workloads.config2(paths=args.dwivedi_paths), 0.2)):
        m = rw.Media.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.n_units, 1)
        geom = rw.Geometry(n_media=wl.n_media, n_rel=wl.n_rel, n_bins=wl.n_bins)
        N = wl.paths_per_unit
        plain, t_p = timed(lambda: api.forward(ctx, m, geom, N, 21, stream=s))
        dw, t_d = timed(lambda: api.dwivedi_forward(ctx, m, geom, N, 21, q, stream=s))
        assert rw.rw_check(ctx, dw.tally.flags) == 0
        se_p = plain.R_se.cpu().numpy()
        se_d = dw.R_se.cpu().numpy()
        gain = (se_p ** 2 * t_p) / (se_d ** 2 * t_d)
        z = (dw.R - plain.R).cpu().numpy() / np.hypot(se_p, se_d)
        f0 = ((wl.n_rel - 1.0) / (wl.n_rel + 1.0)) ** 2
        sums = dw.tally.R.cpu().numpy()
        balance = (sums[:, 0] + sums[:, 2] + sums[:, 3]) / (N * (1.0 - f0))
        res[name] = {"units": wl.n_units, "paths_per_unit": N, "q": q,
                     "plain_ms": t_p, "dwivedi_ms": t_d,
                     "plain_vertices": int(plain.vertices.sum()),
                     "dwivedi_vertices": int(dw.vertices.sum()),
                     "efficiency_gain_median": float(np.median(gain)),
                     "efficiency_gain_p10_p90": [float(np.quantile(gain, 0.1)),
                                                 float(np.quantile(gain, 0.9))],
                     "R_z_vs_plain_median_abs": float(np.median(np.abs(z))),
                     "R_z_vs_plain_max_abs": float(np.max(np.abs(z))),
                     "weight_balance_median": float(np.median(balance)),
                     "weight_balance_min": float(np.min(balance))}
    return res


def c5(torch, args):
    """The inverse fit: 4,096 target spectra (81 wavelengths, the forward
    walk's R(lambda) and R(r, lambda) at random three-medium parameters, 2^18
    paths, 1 % noise), each refit from a random start by Adam over the 11
    parameters per wavelength for 200 steps, through the batched forward and
    the path-replay adjoint at 2^12 paths per evaluation; then the paper's LUT
    route (an 800 x 800 table from the walk, the fused LUT-fit kernel) on the
    same targets.  Both are scored by the walk at 2^18 paths: spectral RMSE
    against the noise-free targets and parameter recovery up to component
    permutation (median absolute errors)."""
    from paper_2606_27604_amd import fit, lut

    print(f"c5: targets for {args.c5_targets} spectra", file=sys.stderr, flush=True)
    prob = fit.make_problem(args.c5_targets, 1 << 18)
    print(f"c5: targets ready ({prob.target_seconds:.1f} s); mc fit", file=sys.stderr, flush=True)
    mc = fit.run_fit(iters=args.c5_iters, paths=1 << 12, problem=prob, log_every=20, progress=True)
    print(f"c5: mc fit {mc['fit_seconds']:.1f} s; lut table", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    table = lut.generate(prob.ctx, args.c5_lut, args.c5_lut, args.c5_lut_photons)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    print(f"c5: table {t_table:.1f} s; lut fit", file=sys.stderr, flush=True)
    lf = fit.run_lut_fit(iters=args.c5_iters, problem=prob, table=table)
    lf["lut_seconds"] = t_table
    return {"workload": f"inverse fit: {args.c5_targets} targets x 81 wavelengths (K=3, n=1.4), "
                        f"{args.c5_iters} Adam steps; targets from the walk at 2^18 paths + 1 % "
                        f"noise; scored by the walk at 2^18 paths",
            "mc_adjoint_route": mc, "lut_route": lf}


def c3(ctx, rw, api, workloads, torch, args):
    """65,536 sets x 16 wavelengths x 4,096 paths: one persistent launch, and
    per-set plain launches timed on a subset of sets (same seeds, same estimates)."""
    wl = workloads.config3(n_sets=args.c3_sets)
    media = rw.Media.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.n_sets, wl.n_wl)
    geom = rw.Geometry(n_media=3, n_rel=wl.n_rel, n_bins=wl.n_bins)
    n, P = wl.n_units, wl.paths_per_unit
    tally = rw.Tally(n, wl.n_bins)
    s = torch.cuda.current_stream()
    rw.rw_batch_forward(ctx, media, geom, None, P, 7, tally, stream=s)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    rw.rw_batch_forward(ctx, media, geom, None, P, 7, tally, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    full_ms = e0.elapsed_time(e1)
    full_v = int(tally.vertices.sum().item())
    res = {"workload": f"batched-{wl.n_sets}x16: K=3, n=1.4, 4096 paths per unit",
           "units": n, "batched_ms": full_ms, "batched_vertices_per_s": full_v / (full_ms * 1e-3),
           "spectra_per_s": wl.n_sets / (full_ms * 1e-3)}
    slots = alg_slots_per_vertex(False)
    achieved = slots * full_v / (full_ms * 1e-3) / 1e12
    key = f"walk_kernel<3, forward>@batched-{wl.n_sets}x16"
    res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": ISSUE_PEAK / 1e12,
                       "unit": "Tslot/s", "frac": achieved / (ISSUE_PEAK / 1e12),
                       "kernel": "walk_kernel<3, forward>", "slots_per_vertex": slots,
                       "counters": load_counters(key), "traffic": load_traffic(key)}
    # matched shape: one plain static launch (rw_forward) over all the units,
    # same seed, same estimates
    stat = rw.Tally(n, wl.n_bins)
    rw.rw_forward(ctx, media, geom, P, 7, stat, stream=s)
    torch.cuda.synchronize()
    e0.record(s)
    rw.rw_forward(ctx, media, geom, P, 7, stat, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    st_ms = e0.elapsed_time(e1)
    res.update({"plain_static_ms": st_ms,
                "plain_static_vertices_per_s": full_v / (st_ms * 1e-3),
                "plain_static_over_batched_time": st_ms / full_ms,
                "plain_static_tallies_bit_identical": bool(
                    torch.equal(stat.R, tally.R) and torch.equal(stat.bins, tally.bins) and
                    torch.equal(stat.vertices, tally.vertices))})
    del stat
    # secondary: per-set plain launches (16 units each) vs one batched launch,
    # on a subset of sets
    S = min(args.c3_plain_sets, wl.n_sets)
    U = S * wl.n_wl
    sub_media = media.unit_range(0, U)
    sub_tally_b = rw.Tally(U, wl.n_bins)
    sub_tally_p = rw.Tally(U, wl.n_bins)
    rw.rw_batch_forward(ctx, sub_media, geom, None, P, 7, sub_tally_b, stream=s)
    torch.cuda.synchronize()
    e0.record(s)
    rw.rw_batch_forward(ctx, sub_media, geom, None, P, 7, sub_tally_b, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    sub_b_ms = e0.elapsed_time(e1)
    per_set = [(media.unit_range(i * wl.n_wl, wl.n_wl), sub_tally_p.view(i * wl.n_wl, wl.n_wl))
               for i in range(S)]
    for m_i, t_i in per_set[:8]:
        rw.rw_forward(ctx, m_i, geom, P, 7, t_i, stream=s)
    torch.cuda.synchronize()
    e0.record(s)
    for m_i, t_i in per_set:
        rw.rw_forward(ctx, m_i, geom, P, 7, t_i, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    sub_p_ms = e0.elapsed_time(e1)
    same = bool(torch.equal(sub_tally_b.vertices, sub_tally_p.vertices) and
                torch.allclose(sub_tally_b.R, sub_tally_p.R, rtol=1e-12, atol=0))
    res.update({"subset_sets": S, "subset_batched_ms": sub_b_ms, "subset_per_set_plain_ms": sub_p_ms,
                "per_set_over_batched_time": sub_p_ms / sub_b_ms,
                "same_estimates_as_batched": same})
    return res


def c4(ctx, rw, workloads, torch, args):
    """Adjoint sweep: 1,024 three-medium sets x 81 wavelengths x 2^14 paths,
    cotangents v_R = 1 and v_bins ~ N(0, 1): one batched path-replay launch
    (after its forward), timed with HIP events on the launch stream."""
    wl = workloads.config4(n_sets=args.c4_sets)
    media = rw.Media.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.n_sets, wl.n_wl)
    geom = rw.Geometry(n_media=3, n_rel=wl.n_rel, n_bins=wl.n_bins)
    n, P = wl.n_units, wl.paths_per_unit
    cot_R = torch.from_numpy(wl.extra["cot_R"]).cuda()
    cot_B = torch.from_numpy(wl.extra["cot_bins"]).cuda()
    grad = torch.empty((n, 12), dtype=torch.float64, device="cuda")
    sq = torch.empty_like(grad)
    vert = torch.empty(n, dtype=torch.int64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    tally = rw.Tally(n, wl.n_bins)
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for rep in range(2):  # first repetition warms up (graph build)
        ev[0].record(s)
        rw.rw_batch_forward(ctx, media, geom, None, P, 41 + rep, tally, stream=s)
        ev[1].record(s)
        rw.rw_batch_adjoint(ctx, media, geom, None, P, 41 + rep, cot_R, cot_B, grad, sq, vert,
                            flags, stream=s)
        ev[2].record(s)
        torch.cuda.synchronize()
    fwd_ms, adj_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    v = int(vert.sum().item())
    return {"workload": f"adjoint-{wl.n_sets}x81: K=3, n=1.4, {P} paths per unit, v_R = 1, "
                        "v_bins ~ N(0, 1)",
            "units": n, "forward_ms": fwd_ms, "adjoint_ms": adj_ms,
            "adjoint_vertices_per_s": v / (adj_ms * 1e-3),
            "forward_vertices_per_s": int(tally.vertices.sum().item()) / (fwd_ms * 1e-3),
            "device_flags": int(flags.item()) | int(tally.flags.item())}


def lut_generation(rw, torch, args):
    """Lookup-table generation (Sec. 4.2): an N x N grid over (alpha, g) at
    sigma_t = 1, n = 1.4, one K = 1 unit per cell, through the batched forward
    walk in launches of --lut-cells-per-launch cells.  The paper's table is
    800 x 800 at 10^6 photons per cell; the time at 10^6 photons is projected
    linearly from the measured per-photon rate (every photon costs the same in
    expectation).  The FP64 oracle is timed on 256 seeded random cells."""
    from paper_2606_27604_amd import lut

    ctx = rw.Context(0)
    s = torch.cuda.current_stream()
    N, P = args.lut, args.lut_photons
    nb, r_min, r_max = lut.LUT_BINS, lut.LUT_R_MIN, lut.LUT_R_MAX
    # warm-up: a small table (library set-up, graph build)
    lut.generate(ctx, 8, 8, 1024, n_bins=nb, r_min=r_min, r_max=r_max, stream=s)
    torch.cuda.synchronize()
    evs, verts, flags = [], [], []

    def on_batch(b, e, res):
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        evs.append(ev)
        verts.append(res.vertices.sum())
        flags.append(res.tally.flags)
        ev.synchronize()  # progress per finished launch (the next one is enqueued after it)
        print(f"lut: cells {b}..{e} of {N * N} done, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)

    e0 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    t0 = time.perf_counter()
    table = lut.generate(ctx, N, N, P, n_bins=nb, r_min=r_min, r_max=r_max,
                         max_units_per_call=args.lut_cells_per_launch, stream=s,
                         on_batch=on_batch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in zip([e0] + evs[:-1], evs)]
    v = [int(x.item()) for x in verts]
    fl = 0
    for f in flags:
        fl |= rw.rw_check(ctx, f)
    gpu_s = sum(ms) * 1e-3
    total_v = sum(v)
    slots = alg_slots_per_vertex(False)
    achieved = slots * total_v / gpu_s / 1e12
    peak = ISSUE_PEAK / 1e12
    paths = N * N * P
    out = {
        "metric": "LUT generation: MC path vertices/s (forward walk, K = 1 per cell)",
        "value": total_v / gpu_s, "unit": "vertices/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32",
        "data": "synthetic (uniform alpha/g grid)",
        "config": {"workload": f"lut-{N}x{N}: alpha in [0, 0.999], g in [0, 0.99], sigma_t = 1, "
                               f"n = 1.4, {P} photons per cell, {nb} log bins "
                               f"[{r_min:g}, {r_max:g}] mm",
                   "cells": N * N, "photons_per_cell": P,
                   "cells_per_launch": args.lut_cells_per_launch},
        "seconds": gpu_s, "wall_seconds": wall, "launches": len(ms),
        "vertices": total_v, "vertices_per_photon": total_v / paths,
        "photons_per_s": paths / gpu_s,
        "projected_seconds_800x800_at_1e6_photons": 800 * 800 * 1e6 * (gpu_s / paths),
        "device_flags": fl,
        "R_range": [float(table.R.min()), float(table.R.max())],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": load_traffic("walk_kernel<1, forward>"),
                     "counters": load_counters("walk_kernel<1, forward>"),
                     "kernel": "walk_kernel<1, forward>", "slots_per_vertex": slots},
    }
    del table
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = lut_cpu_baseline(N)
    print(json.dumps(out), flush=True)


def layered_tones(rw, torch, args):
    """The two-layer tissue walk (Sec. 3 geometry, rw_layered_forward, then its
    adjoint rw_layered_adjoint) over N synthetic tones x 81 wavelengths at
    --layers-photons photons per (tone, wavelength), n = 1.4 in both layers,
    each timed with HIP events on the launch stream (second of two calls).  The paper generates 30,000 tones x
    376 wavelengths at 10^6 photons; the time for that is projected linearly
    from the measured per-photon rate of these tones.  The FP64 oracle is
    timed on a bounded sample of the same units."""
    from paper_2606_27604_amd import workloads

    ctx = rw.Context(0)
    s = torch.cuda.current_stream()
    P = args.layers_photons
    wl = workloads.layered_tones(n_tones=args.layers, paths=P)
    layers = rw.Layers.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.thickness_mm, wl.n_rel_bottom)
    geom = rw.Geometry(n_media=2, n_rel=wl.n_rel, n_bins=wl.n_bins, r_min_mm=wl.r_min_mm,
                       r_max_mm=wl.r_max_mm)
    tally = rw.Tally(wl.n_units, wl.n_bins)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for rep in range(2):  # the first call builds the graph
        ev[0].record(s)
        rw.rw_layered_forward(ctx, layers, geom, None, P, 100 + rep, tally, stream=s)
        ev[1].record(s)
        torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    flags = rw.rw_check(ctx, tally.flags)
    v = int(tally.vertices.sum().item())
    paths = wl.n_units * P
    slots = alg_slots_per_vertex(False)
    achieved = slots * v / (ms * 1e-3) / 1e12
    peak = ISSUE_PEAK / 1e12
    out = {
        "metric": "two-layer tissue walk: MC path vertices/s (forward)",
        "value": v / (ms * 1e-3), "unit": "vertices/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic two-layer tones (no chromophore spectra)",
        "config": {"workload": f"layered-{args.layers}x81: top layer 0.05-0.35 mm over a "
                               f"semi-infinite bottom layer, n = 1.4, {P} photons per "
                               "(tone, wavelength), 256 log bins [1e-3, 50] mm",
                   "units": wl.n_units, "photons_per_unit": P},
        "ms": ms, "vertices": v, "vertices_per_photon": v / paths,
        "photons_per_s": paths / (ms * 1e-3), "spectra_per_s": args.layers / (ms * 1e-3),
        "projected_hours_30000_tones_x_376_wl_at_1e6_photons":
            30000 * 376 * 1e6 * (ms * 1e-3 / paths) / 3600.0,
        "device_flags": flags,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak,
                     "traffic": load_traffic("walk_kernel<2, forward, layered>"),
                     "counters": load_counters("walk_kernel<2, forward, layered>"),
                     "kernel": "walk_kernel<2, forward, layered>", "slots_per_vertex": slots,
                     "note": "slot model of the mixture forward vertex; the ~1 % of vertices "
                             "that cross the interface, reflect or leave are priced as "
                             "collisions"},
    }
    # the adjoint replay of the same walk (rw_layered_adjoint), R and bin cotangents
    n = wl.n_units
    cot_R = torch.ones(n, dtype=torch.float32, device="cuda")
    cot_bins = torch.randn((n, wl.n_bins + 2), generator=torch.Generator().manual_seed(1)).cuda()
    grad = torch.empty((n, 8), dtype=torch.float64, device="cuda")
    sumsq = torch.empty_like(grad)
    avert = torch.empty(n, dtype=torch.int64, device="cuda")
    aflags = torch.zeros(1, dtype=torch.int32, device="cuda")
    for rep in range(2):
        ev[0].record(s)
        rw.rw_layered_adjoint(ctx, layers, geom, None, P, 100 + rep, cot_R, cot_bins, grad, sumsq,
                              avert, aflags, stream=s)
        ev[1].record(s)
        torch.cuda.synchronize()
    ams = ev[0].elapsed_time(ev[1])
    av = int(avert.sum().item())
    aslots = alg_slots_per_vertex(True)
    a_ach = aslots * av / (ams * 1e-3) / 1e12
    out["adjoint"] = {"ms": ams, "vertices_per_s": av / (ams * 1e-3), "vertices": av,
                      "device_flags": rw.rw_check(ctx, aflags),
                      "roofline": {"bound": "alu", "achieved": a_ach, "peak": peak,
                                   "unit": "Tslot/s", "frac": a_ach / peak,
                                   "kernel": "walk_kernel<2, adjoint, layered>",
                                   "slots_per_vertex": aslots}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = layered_cpu_baseline(wl)
    print(json.dumps(out), flush=True)


def layered_cpu_baseline(wl, max_seconds=30.0):
    """The FP64 oracle on the first tone's 81 wavelengths, at a photon count
    doubled from 2^10 until one pass takes 8 s."""
    from oracle import oracle as O

    cores, model = host_cpu()
    sub = wl.subset(np.arange(wl.n_wl))
    geo = O.Geometry(n_media=2, n_rel=float(np.float32(wl.n_rel)), n_bins=wl.n_bins)
    paths = 1 << 10
    while True:
        t0 = time.perf_counter()
        _, _, vert = O.layered_forward(geo, sub.sigma_t, sub.albedo, sub.g, sub.thickness_mm,
                                       float(np.float32(wl.n_rel_bottom)), paths, 17,
                                       n_threads=cores)
        dt = time.perf_counter() - t0
        if dt > 8.0 or dt * 2 > max_seconds:
            break
        paths *= 2
    return {"value": float(vert.sum()) / dt, "unit": "vertices/s", "cores": cores, "kind": "oracle",
            "per_core": float(vert.sum()) / dt / cores, "cpu_model": model,
            "sample": f"one tone x 81 wavelengths x {paths} photons, FP64, "
                      f"{int(vert.sum())} vertices in {dt:.2f} s"}


def lut_cpu_baseline(N, n_cells=256, max_seconds=30.0):
    """The FP64 oracle on 256 seeded random cells of the same grid, at a photon
    count doubled from 2^10 until one pass takes 8 s."""
    from oracle import oracle as O

    cores, model = host_cpu()
    rng = np.random.default_rng(123)
    ia, ig = rng.integers(0, N, n_cells), rng.integers(0, N, n_cells)
    al = np.float32(np.linspace(0.0, 0.999, N, dtype=np.float32)[ia])[None].astype(np.float64)
    gg = np.float32(np.linspace(0.0, 0.99, N, dtype=np.float32)[ig])[None].astype(np.float64)
    from paper_2606_27604_amd import lut

    geo = O.Geometry(n_media=1, n_rel=float(np.float32(1.4)), n_bins=lut.LUT_BINS,
                     r_min_mm=lut.LUT_R_MIN, r_max_mm=lut.LUT_R_MAX)
    one = np.ones((1, n_cells))
    paths = 1 << 10
    while True:
        t0 = time.perf_counter()
        _, _, vert = O.forward(geo, one, al, gg, one, paths, 17, n_threads=cores)
        dt = time.perf_counter() - t0
        if dt > 8.0 or dt * 2 > max_seconds:
            break
        paths *= 2
    return {"value": float(vert.sum()) / dt, "unit": "vertices/s", "cores": cores, "kind": "oracle",
            "per_core": float(vert.sum()) / dt / cores, "cpu_model": model,
            "sample": f"{n_cells} random cells of the {N}x{N} grid x {paths} photons, FP64, "
                      f"{int(vert.sum())} vertices in {dt:.2f} s"}


if __name__ == "__main__":
    main()
