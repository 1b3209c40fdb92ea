"""Benchmark of the line-by-line + ray-march hot path on one MI355X.

Headline workload: the large axisymmetric configuration at full shape
(512 x 256 cells, 11 species, the 4M-line generator, a 2^22-point grid over
1000-100000 cm^-1 in bands of 131,072, 256 wall points x 1024 directions).
One step = the whole path (lrt_solve_ranges: per-cell populations and scales,
candidate ranges, the Voigt accumulation of every cell, the march of every
traced ray with the fused trapezoid, the wall sums) over a fixed stratified
spectral slice: 16 ranges of 1,024 points, one at a seeded position in each
sixteenth of the grid, every cell, line and ray at full shape.  The slice's
Voigt evaluations per second are measured directly; the whole configuration
(256 such slices of points) is extrapolated from it and labelled so.

Beside it, outside the timed region: one double-precision step of the same
slice; the stagnation line (400 cells, 2.2M lines, 2^21 points, 17 rays) and
the 256 x 128-cell axisymmetric case as whole solves; cost legs of the march
variants, continuum, full Lorentz width and QSS-CR populations; the serving
stream (closed loop, then open loop at 0.5 and 0.8 of saturation); measured
unit peaks (lrt_probe); and the oracle on the host's cores.

Prints one JSON line on stdout (progress goes to stderr).
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Voigt line-pt evals/s + q_rad solves/s (FP32-comp vs FP64, 1 GPU); p99 latency"

# MI355X nominal figures: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.
CLOCK_HZ = 2.4e9
LANE_ISSUE = 256 * 64 * CLOCK_HZ          # non-packed VALU lane-instructions per s (39.3e12)
PEAK_FP32_TFLOPS = 157.3                   # packed FP32 vector peak (FMA = 2 flops)
PEAK_FP32_NONPACKED_TFLOPS = 78.6          # one FMA per lane per cycle
HBM_PEAK = 8.0e12
# Algorithmic work of one Whiting-Voigt evaluation, counted from the profile's
# formula (Sec. 2.2.1): 6 transcendentals (the two exponentials, the log and
# exp of x^2.25, two reciprocals) and about 20 other single-precision
# operations (offset, scale, squares, arguments, the three-term combination,
# the eta and kappa products and their compensated updates).
OPS_PER_EVAL = 26
# Issue slots of one evaluation in the form the kernel evaluates, one slot per
# VALU instruction (y = (nu - nu0)/gamma_V):
#   wing point (|dnu| > 25 HWHM, both exponentials exactly zero in single
#   precision): offset 2 (sub, fma), 1 + y^2 1, |y|^2.25 3 (log, scale, exp),
#   1 + 0.1 x^2.25 1, reciprocal of the product 2, numerator 2, product 1,
#   two accumulating FMAs 2 = 14;
#   core point: + exponent and exp for each of the two exponentials (4) and
#   their two FMAs = 20.
SLOTS_CORE = 20
SLOTS_WING = 14

SLICE_RANGES = 16
RANGE_POINTS = 1024
SLICE_SEED = 11864


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--workload", default="axi_large", choices=["axi_large", "stagnation", "slab", "axi"],
                    help="axi_large: the stratified slice of the large axisymmetric case (headline); "
                         "the others: whole solves")
    ap.add_argument("--band", type=int, default=None,
                    help="time one band alone (coefficients of every cell, then the march of every "
                         "ray), print its own JSON line and exit")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true",
                    help="skip every leg outside the timed steps (FP64 step aside), so that a profiler "
                         "sees the timed path only")
    ap.add_argument("--serving-requests", type=int, default=500,
                    help="requests per open-loop rate (closed loop: 2/5 of it); 0 skips serving")
    ap.add_argument("--peak", action="store_true", help="only run the unit throughput probes and exit")
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the serving stream (--serving-requests per open-loop rate) and exit")
    ap.add_argument("--no-full-count", action="store_true",
                    help="skip the whole-configuration term count (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy 3 times (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = (2 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read_per_copy": a.numel() * 4,
                      "bytes_written_per_copy": a.numel() * 4, "copies": 3}), flush=True)


def peaks():
    """Measured unit throughputs (lrt_probe) against the nominal peaks."""
    from paper_2604_11856_amd import lrt
    out = {}
    for k in ("fma_f32", "fma_f64", "exp_f32", "log_f32", "rcp_f32", "mix_f32", "copy"):
        rate, ms = lrt.probe(k)
        if k == "copy":
            out[k] = {"GB_per_s": rate / 1e9, "frac_of_hbm_peak": rate / HBM_PEAK, "ms": ms}
        else:
            out[k] = {"lane_ops_per_s": rate, "frac_of_lane_issue": rate / LANE_ISSUE, "ms": ms}
    out["fma_f32"]["TFLOP_s"] = 2 * out["fma_f32"]["lane_ops_per_s"] / 1e12
    out["fma_f64"]["TFLOP_s"] = 2 * out["fma_f64"]["lane_ops_per_s"] / 1e12
    out["nominal"] = {"lane_issue_per_s": LANE_ISSUE, "fp32_TFLOPs_packed": PEAK_FP32_TFLOPS,
                      "fp32_TFLOPs_nonpacked": PEAK_FP32_NONPACKED_TFLOPS, "hbm_GB_s": HBM_PEAK / 1e9}
    return out


def workload(name):
    from paper_2604_11856_amd import synth
    if name == "stagnation":
        wl = synth.config_stagnation()
        desc = ("stagnation-line: 400 cells x 0.01 cm, 11 species, 200k atomic + 2M rovibronic "
                "lines, 2^21-point grid 1000-100000 cm^-1, 17 rays (wall normal + 16 GL)")
    elif name == "slab":
        wl = synth.config_slab()
        desc = "slab: 64 cells x 0.05 cm, 2000 N/O lines, 200,000-point grid 5000-80000 cm^-1, 1 ray"
    elif name == "axi":
        wl = synth.config_axi()
        desc = ("axisymmetric: 256x128 cells, 11 species, 1M lines, 2^20-point grid in 16 bands, "
                "64 wall points x (16 GL x 16 azimuth) rays")
    else:
        wl = synth.config_axi_large()
        desc = ("large axisymmetric: 512x256 cells, 11 species, %d lines (4M generator: 1M atomic + 3M "
                "rovibronic, lines off the grid rejected), 2^22-point grid 1000-100000 cm^-1 in 32 bands "
                "of 131072, 256 wall points x (32 GL x 32 azimuth) directions" % wl.lines.n)
    return wl, desc


def slice_ranges(n_points):
    """The stratified slice: one RANGE_POINTS-point range at a seeded position
    in each of SLICE_RANGES equal strata of the grid."""
    rng = np.random.Generator(np.random.PCG64(SLICE_SEED))
    stratum = n_points // SLICE_RANGES
    kf = np.array([j * stratum + int(rng.integers(0, stratum - RANGE_POINTS + 1))
                   for j in range(SLICE_RANGES)], np.int64)
    return kf, np.full(SLICE_RANGES, RANGE_POINTS, np.int64)


def band_bench(args):
    """One band of a workload timed alone: the single-precision coefficients of
    every cell, then the march of every ray through them with the band's
    trapezoid sum (no per-point intensity kept), HIP events per kernel."""
    import torch
    from paper_2604_11856_amd import lrt
    wl, desc = workload(args.workload)
    ctx = lrt.Context(0).load(wl)
    sz = ctx.sizes()
    b = args.band
    if not 0 <= b < sz["n_bands"]:
        print("band %d out of range [0, %d)" % (b, sz["n_bands"]), file=sys.stderr)
        sys.exit(2)
    n_terms, n_core = ctx.count_terms(b, core=True)
    nb = ctx.band_len(b)
    n_seg = ctx.segment_count()
    eta = torch.empty((sz["n_cells"], nb), dtype=torch.float32, device="cuda:0")
    kap = torch.empty_like(eta)
    esc = torch.zeros((sz["n_cells"], 2), dtype=torch.int32, device="cuda:0")
    I_int = torch.empty((sz["n_rays"],), dtype=torch.float64, device="cuda:0")

    def once():
        ctx.coeffs(b, lrt.LRT_FP32_COMP, eta, kap, esc)
        ctx.march(b, lrt.LRT_FP32_COMP, eta, kap, esc, None, I_int)

    for _ in range(args.warmup):
        once()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = {k: ctx.profile_read(k) for k in lrt.KERNELS}
    ctx.profile(False)
    acc_s = prof["accum"][0] / 1e3 / max(1, prof["accum"][1])
    mar_s = prof["march"][0] / 1e3 / max(1, prof["march"][1])
    slots = n_core * SLOTS_CORE + (n_terms - n_core) * SLOTS_WING
    seg_pts = n_seg * nb
    print(json.dumps({
        "metric": "one band alone: Voigt line-pt evals/s, march row GB/s", "workload": desc,
        "band": b, "band_points": nb, "cells": sz["n_cells"], "rays": sz["n_rays"],
        "steps": args.steps, "warmup": args.warmup, "ms_per_band": dt * 1e3,
        "terms": n_terms, "core_fraction": n_core / max(1, n_terms), "evals_per_s": n_terms / dt,
        "accum_ms": acc_s * 1e3, "accum_evals_per_s": n_terms / acc_s,
        "accum_frac_of_fp32_peak": OPS_PER_EVAL * n_terms / acc_s / (PEAK_FP32_TFLOPS * 1e12),
        "accum_issue_occupancy": slots / acc_s / LANE_ISSUE,
        "march_ms": mar_s * 1e3, "segment_points": seg_pts,
        "march_row_GB_per_s": seg_pts * 8 / mar_s / 1e9,
        "kernels_ms": {k: v[0] / args.steps for k, v in prof.items()}}), flush=True)
    ctx.close()


# Sources of the accumulation and march kernels; a committed counter summary
# records the sha256 of its kernel's sources (in this order).
ACCUM_SOURCES = ("lrt_accum.hip", "lrt_device.h", "lrt_internal.h")
MARCH_SOURCES = ("lrt_march.hip", "lrt_device.h", "lrt_internal.h")


def sources_sha256(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2604_11856_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counter_summary(summary, sources):
    """The machine-readable fields of a committed counter summary, provided it
    was taken with the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    fields = {}
    for ln in open(path):
        if ":" in ln:
            k, v = ln.split(":", 1)
            fields[k.strip().strip("-* ")] = v.strip()
    if fields.get("kernel_source_sha256") != sources_sha256(sources) or "traffic_bytes_per_launch" not in fields:
        return None
    return fields


def counter_traffic(summary, sources=ACCUM_SOURCES):
    """HBM bytes per launch from a committed counter summary taken with the
    current kernel sources; otherwise None."""
    f = counter_summary(summary, sources)
    return None if f is None else float(f["traffic_bytes_per_launch"])


def serving(n_open, budget_gb=64, slots=64):
    """Serving stream on the resident 1M-line list and 2^20-point grid:
    closed-loop saturation X_sat (all requests at t = 0), then Poisson
    arrivals at 0.5 and 0.8 X_sat; latency = submit -> result on the host."""
    from paper_2604_11856_amd import lrt, synth
    wl = synth.config_axi()
    ctx = lrt.Context(0)
    ctx.set_species(wl.species)
    ctx.set_lines(wl.lines)
    ctx.set_grid(wl.grid)
    srv = lrt.Server(ctx, budget_gb << 30, slots)
    # warm the kernels with one small request
    srv.wait(srv.submit(synth.serving_requests(1, wl.grid.n_points, max_cells=32, max_win=20000,
                                               seed=1)[0]))
    n_closed = max(16, (2 * n_open) // 5)
    reqs = synth.serving_requests(n_closed, wl.grid.n_points, seed=11859)
    # (cell, grid point) pairs whose coefficients the closed loop computes and marches
    cell_points = sum(int(r.cells.n) * int(r.n_window) for r in reqs)
    t0 = time.perf_counter()
    res = [srv.wait(t) for t in [srv.submit(r) for r in reqs]]
    t_closed = time.perf_counter() - t0
    ok = all(x["status"] == 0 for x in res)
    x_sat = n_closed / t_closed
    log("serving: closed loop %d requests in %.1f s" % (n_closed, t_closed))
    open_loop = {}
    for frac, seed in ((0.5, 11861), (0.8, 11865)):
        rate = frac * x_sat
        reqs = synth.serving_requests(n_open, wl.grid.n_points, rate_hz=rate, seed=seed)
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            dt = t0 + r.arrival - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(r))
        res = [srv.wait(t) for t in tickets]
        t_open = time.perf_counter() - t0
        ok = ok and all(x["status"] == 0 for x in res)
        lat = np.array([x["latency_ms"] for x in res])
        open_loop["%.1f_x_sat" % frac] = {
            "requests": n_open, "rate_hz": rate, "seconds": t_open, "solves_per_s": n_open / t_open,
            "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
            "max_latency_ms": float(lat.max()),
            "p50_queue_ms": float(np.percentile([x["queue_ms"] for x in res], 50))}
        log("serving: open loop at %.1f X_sat, %d requests in %.1f s" % (frac, n_open, t_open))
    info = srv.info()
    srv.stop()
    ctx.close()
    return {"resident": "1M lines (250k atomic + 750k rovibronic), 2^20-point grid 1000-100000 cm^-1",
            "requests": "cells logU[16, 2048], window logU[1e4, 1e6] points, mixed species subsets",
            "budget_GB": budget_gb, "slots": slots, "all_ok": ok,
            "closed_loop": {"requests": n_closed, "seconds": t_closed, "solves_per_s": x_sat,
                            "cell_points": cell_points, "cell_points_per_s": cell_points / t_closed},
            "open_loop": open_loop, "epochs": info["epochs"]}


def compare_march_schemes(ctx, lrt, torch, sz, reps=3):
    """Band 0 in single precision: the march (a5 + a6) with the cell-constant
    scheme and with the linear-j segment scheme over LOS nodes, on the same
    eta/kappa; per-launch time from HIP events and the spread of I_int."""
    eta, kap, esc = ctx.coeffs_torch(0, lrt.LRT_FP32_COMP)
    Ii = torch.zeros(sz["n_rays"], dtype=torch.float64, device="cuda:0")
    out = {}
    res = {}
    for name, scheme in (("cell", lrt.LRT_MARCH_CELL), ("linear_j", lrt.LRT_MARCH_LINEAR_J)):
        ctx.set_march(scheme)
        ctx.march(0, lrt.LRT_FP32_COMP, eta, kap, esc, None, Ii)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.march(0, lrt.LRT_FP32_COMP, eta, kap, esc, None, Ii)
        torch.cuda.synchronize()
        ms, n = ctx.profile_read("march")
        ctx.profile(False)
        out[name + "_ms_per_launch"] = ms / max(1, n)
        res[name] = Ii.cpu().numpy().copy()
    ctx.set_march(lrt.LRT_MARCH_CELL)
    out["band"] = 0
    out["I_int_rel_diff_linear_vs_cell_max"] = float(np.max(np.abs(res["linear_j"] - res["cell"]) /
                                                           np.abs(res["cell"])))
    del eta, kap, esc
    torch.cuda.empty_cache()
    return out


def continuum_cost(ctx, wl, lrt, torch, reps=2):
    """Band 0 in single precision: accumulation time without and with the
    atomic continuum (bound-free + free-free of N and O, added per point in the
    accumulation's epilogue)."""
    from paper_2604_11856_amd import synth
    cont = synth.air_continuum(wl.species)
    if not cont:
        return None
    out = {}
    for name, rec in (("lines_only", None), ("with_continuum", cont)):
        ctx.set_continuum(rec)
        eta, kap, esc = ctx.coeffs_torch(0, lrt.LRT_FP32_COMP)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.coeffs(0, lrt.LRT_FP32_COMP, eta, kap, esc)
        torch.cuda.synchronize()
        ms, n = ctx.profile_read("accum")
        ctx.profile(False)
        out[name + "_accum_ms"] = ms / max(1, n)
        del eta, kap, esc
    ctx.set_continuum(None)
    torch.cuda.empty_cache()
    out["band"] = 0
    out["thresholds"] = int(sum(int((r.sigma0 > 0).sum()) for r in cont))
    return out


def lorentz_cost(ctx, wl, lrt, torch, reps=2):
    """Band 0 in single precision: accumulation with the uniform Lorentz law of
    the workload against the full per-line width of the atomic lines (natural
    + Stark + van der Waals, Sec. 2.2.1).  The windows follow the widths, so
    the in-window term counts differ; each is counted."""
    from paper_2604_11856_amd import synth
    E = synth.air_ionization_energies(wl.species)
    out = {"band": 0}
    for name, e in (("uniform", None), ("full", E)):
        ctx.set_lorentz(e)
        terms = ctx.count_terms(0)
        eta, kap, esc = ctx.coeffs_torch(0, lrt.LRT_FP32_COMP)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.coeffs(0, lrt.LRT_FP32_COMP, eta, kap, esc)
        torch.cuda.synchronize()
        ms, n = ctx.profile_read("accum")
        ctx.profile(False)
        t = ms / max(1, n)
        out[name] = {"accum_ms": t, "terms": int(terms), "evals_per_s": terms / (t / 1e3)}
        del eta, kap, esc
    ctx.set_lorentz(None)
    torch.cuda.empty_cache()
    return out


def cr_cost(wl, lrt, torch, reps=2, scale_cells=32768):
    """QSS collisional-radiative populations of N and O (Sec. 2.1) on the
    workload with its atomic lines put on level pairs (synth.with_cr): whole
    single-precision solves with those lines and the bound-free absorption
    taking their populations from the per-(cell, atom) CR solve, against the
    same line list with Boltzmann populations; then the CR solve alone on
    scale_cells cells (one wave per (cell, atom) system)."""
    from paper_2604_11856_amd import synth
    cw = synth.with_cr(wl)
    if not cw.cr.species:
        return None
    ctx = lrt.Context(0).load(cw)

    def timed_solves():
        ctx.solve(lrt.LRT_FP32_COMP)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            q, _, _ = ctx.solve(lrt.LRT_FP32_COMP)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        prof = {k: ctx.profile_read(k) for k in ("cr", "accum")}
        ctx.profile(False)
        return q, dt, prof

    q_cr, dt_cr, p_cr = timed_solves()
    ctx.set_cr(None)
    q_b, dt_b, p_b = timed_solves()
    ctx.close()
    torch.cuda.empty_cache()
    out = {"atoms": [wl.species[r.species].name for r in cw.cr.species],
           "levels_solved": [int(r.n_model) for r in cw.cr.species],
           "lines_on_levels": int((cw.line_levels[:, 0] >= 0).sum()),
           "systems": wl.cells.n * len(cw.cr.species),
           "ms_per_step": dt_cr * 1e3, "ms_per_step_boltzmann": dt_b * 1e3,
           "cr_ms_per_solve": p_cr["cr"][0] / max(1, p_cr["cr"][1]),
           "accum_ms_per_launch": p_cr["accum"][0] / max(1, p_cr["accum"][1]),
           "accum_ms_per_launch_boltzmann": p_b["accum"][0] / max(1, p_b["accum"][1]),
           "q_rad_ratio_cr_over_boltzmann": [float(a / b) if b and np.isfinite(a / b) else None
                                             for a, b in zip(q_cr, q_b)]}
    # the CR solve alone at a larger cell count (the axisymmetric grid's)
    sw = synth.with_cr(synth.stagnation_line(n_cells=scale_cells, n_atomic=64, n_rovib=0, n_points=4096,
                                             n_mu=0))
    c2 = lrt.Context(0).load(sw)
    c2.solve(lrt.LRT_FP64)
    torch.cuda.synchronize()
    c2.profile(True)
    for _ in range(reps):
        c2.solve(lrt.LRT_FP64)
    torch.cuda.synchronize()
    ms, n = c2.profile_read("cr")
    c2.profile(False)
    c2.close()
    t = ms / max(1, n)
    out["scaled"] = {"cells": scale_cells, "systems": scale_cells * len(sw.cr.species), "cr_ms": t,
                     "systems_per_s": scale_cells * len(sw.cr.species) / (t / 1e3)}
    return out


def timed(ctx, lrt, torch, fn, steps, warmup):
    """Mean seconds per call of fn() over `steps` calls after `warmup`, with
    a device synchronisation on both sides, and the per-kernel HIP-event
    totals of the timed calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = {k: ctx.profile_read(k) for k in lrt.KERNELS}
    ctx.profile(False)
    return dt, out, prof


def whole_solve_leg(name, lrt, torch, steps, fp64_steps, side):
    """A configuration's whole solve (every band): FP32-comp steps, one FP64
    step, and on the stagnation line the cost legs of the path's variants."""
    wl, desc = workload(name)
    ctx = lrt.Context(0).load(wl)
    sz = ctx.sizes()
    counts = [ctx.count_terms(b, core=True) for b in range(sz["n_bands"])]
    n_terms = sum(c[0] for c in counts)
    dt, (q, I, _), prof = timed(ctx, lrt, torch, lambda: ctx.solve(lrt.LRT_FP32_COMP), steps, 1)
    out = {"workload": desc, "steps": steps, "ms_per_step": dt * 1e3, "evals_per_s": n_terms / dt,
           "voigt_terms_per_step": n_terms, "terms_per_band": [int(c[0]) for c in counts],
           "core_terms_per_band": [int(c[1]) for c in counts], "q_rad_solves_per_s": sz["n_wall"] / dt,
           "los_solves_per_s": sz["n_rays"] / dt,
           "accum_ms_per_step": prof["accum"][0] / steps, "march_ms_per_step": prof["march"][0] / steps}
    if fp64_steps > 0:
        dt64, (q64, I64, _), _ = timed(ctx, lrt, torch, lambda: ctx.solve(lrt.LRT_FP64), fp64_steps, 0)
        out["fp64"] = {"ms_per_step": dt64 * 1e3, "speedup_fp32c_over_fp64": dt64 / dt,
                       "rel_err_fp32c_vs_fp64": {
                           "I_int_max": float(np.max(np.abs(I - I64) / np.maximum(np.abs(I64), 1e-300))),
                           "q_max": float(np.max(np.abs(q - q64) / np.abs(q64)))}}
    if side and name == "stagnation":
        out["march_schemes"] = compare_march_schemes(ctx, lrt, torch, sz)
        out["continuum"] = continuum_cost(ctx, wl, lrt, torch)
        out["lorentz"] = lorentz_cost(ctx, wl, lrt, torch)
        out["cr"] = cr_cost(wl, lrt, torch)
    ctx.close()
    torch.cuda.empty_cache()
    return out


def generated_lines_leg(lrt, torch, steps=2):
    """The stagnation line with its molecular lines generated on the device
    (lrt_gen_rovib_lines) from the four air band systems (30 x 30 bands each,
    J up to 150) instead of the stored synthetic list: generation time, the
    list set from device memory, then whole single-precision solves."""
    from paper_2604_11856_amd import synth
    wl = synth.config_stagnation()
    ctx = lrt.Context(0)
    ctx.set_species(wl.species)
    sy = synth.air_band_systems(nv=30, J_max=150)
    ctx.gen_rovib_lines(sy, wl.grid.nu_min, wl.grid.nu_max)    # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gen = ctx.gen_rovib_lines(sy, wl.grid.nu_min, wl.grid.nu_max)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    atom = np.isin(wl.lines.species, [i for i, sp in enumerate(wl.species) if sp.kind == synth.KIND_ATOM])
    dev = {k: torch.cat([torch.as_tensor(np.asarray(getattr(wl.lines, k))[atom], dtype=torch.float64,
                                         device="cuda:0"), gen[k]]) for k in lrt.LINE_FIELDS}
    dev["species"] = torch.cat([torch.as_tensor(np.asarray(wl.lines.species)[atom], dtype=torch.int32,
                                                device="cuda:0"), gen["species"]])
    t0 = time.perf_counter()
    ctx.set_lines_device(dev)
    t_set = time.perf_counter() - t0
    ctx.set_grid(wl.grid)
    ctx.set_cells(wl.cells)
    ctx.set_rays(wl.geometry)
    n_terms = ctx.count_terms(0)
    dt, (q, _, _), prof = timed(ctx, lrt, torch, lambda: ctx.solve(lrt.LRT_FP32_COMP), steps, 1)
    out = {"atomic_lines": int(atom.sum()), "generated_lines": int(gen["nu0"].shape[0]),
           "generation_ms": t_gen * 1e3, "generated_lines_per_s": gen["nu0"].shape[0] / t_gen,
           "set_lines_from_device_ms": t_set * 1e3, "solve_ms_per_step": dt * 1e3,
           "evals_per_s": n_terms / dt, "voigt_terms_per_step": n_terms, "q_rad_W_cm2": [float(x) for x in q]}
    ctx.close()
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, ks_all):
    """The oracle's coefficients (its plain FP64 loops, as committed) on a
    bounded sample of the workload: seeded cells x a 32-point cluster of the
    slice, every line; first single-threaded, then on the host's CPU share.
    The sample grows until one run takes a few seconds."""
    import oracle as O
    from paper_2604_11856_amd import synth
    rng = np.random.Generator(np.random.PCG64(7))
    ks = np.asarray(ks_all[:32], np.int64)
    order = rng.permutation(wl.cells.n)
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    # a GPU machine allots 16 host CPUs to its one GPU
    threads_all = max(1, min(affinity, 16))

    def run(n_cells, threads):
        idx = np.sort(order[:n_cells])
        sub = synth.Cells(wl.cells.T_tr[idx], wl.cells.T_v[idx], np.ascontiguousarray(wl.cells.N[idx]),
                          wl.cells.n_e[idx])
        t = time.perf_counter()
        _, _, n_terms = O.coeffs(wl.species, wl.lines, sub, wl.grid, ks, threads=threads)
        return n_terms, time.perf_counter() - t

    out = {}
    for label, threads, target in (("single_thread", 1, 8.0), ("all", threads_all, 10.0)):
        n = 8 * threads
        n_terms, dt = run(n, threads)
        while dt < 1.0 and n < wl.cells.n:
            n = min(wl.cells.n, n * 4)
            n_terms, dt = run(n, threads)
        if dt < target and n < wl.cells.n:
            n = min(wl.cells.n, int(n * target / max(dt, 1e-3)))
            n_terms, dt = run(n, threads)
        out[label] = {"value": n_terms / dt, "threads": threads, "cells": n, "terms": n_terms,
                      "seconds": dt}
        log("cpu baseline %s: %d cells, %.2e terms in %.1f s" % (label, n, n_terms, dt))
    a = out["all"]
    return {"value": a["value"], "unit": "Voigt line-pt evals/s", "cores": a["threads"], "kind": "oracle",
            "sample": "%d seeded cells x 32 grid points (%d-%d) of the large axisymmetric case, all %d lines: "
                      "%d terms in %.2f s on %d threads" % (a["cells"], ks[0], ks[-1], wl.lines.n, a["terms"],
                                                            a["seconds"], a["threads"]),
            "single_thread": out["single_thread"], "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "cpu_model": cpu_model()}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.peak:
        print(json.dumps({"metric": "unit throughput probes", "peaks": peaks()}), flush=True)
        return
    if args.band is not None:
        band_bench(args)
        return
    if args.serving_only:
        print(json.dumps({"metric": "serving stream", "serving": serving(max(1, args.serving_requests))}), flush=True)
        return
    import torch
    from paper_2604_11856_amd import lrt

    if args.workload != "axi_large":
        leg = whole_solve_leg(args.workload, lrt, torch, args.steps, args.fp64_steps, not args.no_side)
        print(json.dumps({"metric": METRIC, "value": leg["evals_per_s"], "unit": "Voigt line-pt evals/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": leg["ms_per_step"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic", "config": {"workload": leg["workload"]}, "leg": leg}),
              flush=True)
        return

    t_start = time.perf_counter()
    wl, desc = workload("axi_large")
    ctx = lrt.Context(0).load(wl)
    sz = ctx.sizes()
    log("loaded %s in %.1f s" % (desc, time.perf_counter() - t_start))
    kf, npt = slice_ranges(sz["n_points"])
    n_slice_pts = int(npt.sum())
    n_terms, n_core = ctx.count_terms_ranges(kf, npt, core=True)
    terms_per_range = [int(ctx.count_terms_ranges(kf[j:j + 1], npt[j:j + 1])) for j in range(SLICE_RANGES)]
    n_seg = ctx.segment_count()
    log("slice: %d terms, %d segments" % (n_terms, n_seg))

    dt32, (q32, I32, qr32), prof32 = timed(ctx, lrt, torch,
                                           lambda: ctx.solve_ranges(lrt.LRT_FP32_COMP, kf, npt),
                                           args.steps, args.warmup)
    log("timed %d steps: %.1f ms per step" % (args.steps, dt32 * 1e3))
    fp64 = {}
    if args.fp64_steps > 0:
        dt64, (q64, I64, _), prof64 = timed(ctx, lrt, torch, lambda: ctx.solve_ranges(lrt.LRT_FP64, kf, npt),
                                            args.fp64_steps, 0)
        fp64 = {"ms_per_step": dt64 * 1e3, "evals_per_s": n_terms / dt64,
                "accum_ms_per_step": prof64["accum"][0] / args.fp64_steps,
                "speedup_fp32c_over_fp64": dt64 / dt32,
                "rel_err_fp32c_vs_fp64": {
                    "I_int_max": float(np.max(np.abs(I32 - I64) / np.maximum(np.abs(I64), 1e-300))),
                    "q_max": float(np.max(np.abs(q32 - q64) / np.abs(q64))),
                    "q_median": float(np.median(np.abs(q32 - q64) / np.abs(q64)))}}
        log("fp64 step: %.1f ms" % (dt64 * 1e3))
    # the whole configuration: the slice is 1/256 of the points; the
    # accumulation also scaled by the exact term counts of every band
    ratio = sz["n_points"] / n_slice_pts
    acc_step = prof32["accum"][0] / 1e3 / args.steps
    t_full_pts = dt32 * ratio
    if args.no_full_count:
        n_terms_full = int(n_terms * ratio)
        t_full_terms = t_full_pts
    else:
        t_full_count = time.perf_counter()
        n_terms_full = sum(ctx.count_terms(b) for b in range(sz["n_bands"]))
        log("whole-configuration term count %.3e in %.1f s" % (n_terms_full, time.perf_counter() - t_full_count))
        t_full_terms = acc_step * n_terms_full / n_terms + (dt32 - acc_step) * ratio
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    acc_launch_s = prof32["accum"][0] / 1e3 / max(1, prof32["accum"][1])
    terms_per_launch = n_terms / SLICE_RANGES
    flops_per_launch = OPS_PER_EVAL * terms_per_launch
    slots_per_launch = (n_core * SLOTS_CORE + (n_terms - n_core) * SLOTS_WING) / SLICE_RANGES
    mar_launch_s = prof32["march"][0] / 1e3 / max(1, prof32["march"][1])
    march_bytes_per_launch = n_seg * RANGE_POINTS * 8.0
    march_traffic = counter_traffic("march_f32_axi_large_slice_pmc.md", MARCH_SOURCES)
    line = {
        "metric": METRIC,
        "value": n_terms / dt32,
        "unit": "Voigt line-pt evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc + "; one step = the whole path over a stratified spectral slice of "
                   "%d x %d points (one range at a seeded position in each sixteenth of the grid) with every "
                   "cell, line and traced ray; whole-configuration time and q_rad wall-point solves/s are "
                   "EXTRAPOLATED from the slice (x%d in points, accumulation by exact term counts)"
                   % (SLICE_RANGES, RANGE_POINTS, int(round(ratio))),
                   "precision": "fp32 profile evaluation, per-point sums over 64-line blocks merged with Kahan "
                   "compensation; populations, widths, windows, march state and quadrature in f64",
                   "cells": sz["n_cells"], "lines": wl.lines.n, "grid_points": sz["n_points"],
                   "slice_ranges": [[int(a), int(b)] for a, b in zip(kf, npt)],
                   "traced_rays": sz["n_rays"], "wall_points": sz["n_wall"], "segments": n_seg,
                   "voigt_terms_per_step": n_terms, "voigt_terms_per_range": terms_per_range},
        "whole_config_extrapolated": {
            "ms_by_points": t_full_pts * 1e3, "ms_by_terms": t_full_terms * 1e3,
            "voigt_terms": n_terms_full, "q_rad_solves_per_s": sz["n_wall"] / t_full_terms,
            "evals_per_s": n_terms_full / t_full_terms},
        "q_rad_solves_per_s": sz["n_wall"] / t_full_terms,
        "q_rad_W_cm2_over_slice": {"min": float(q32.min()), "max": float(q32.max())},
        "fp64": fp64,
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in prof32.items()},
        "roofline": {"bound": "alu", "kernel": "accum_f32",
                     "achieved": flops_per_launch / acc_launch_s / 1e12, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops_per_launch / acc_launch_s / (PEAK_FP32_TFLOPS * 1e12),
                     "traffic": counter_traffic("accum_f32_axi_large_slice_pmc.md"),
                     "ops_per_eval": OPS_PER_EVAL, "evals_per_launch": terms_per_launch,
                     "avg_launch_ms": acc_launch_s * 1e3,
                     "frac_of_nonpacked_fp32": flops_per_launch / acc_launch_s / (PEAK_FP32_NONPACKED_TFLOPS * 1e12),
                     "issue_occupancy": slots_per_launch / acc_launch_s / LANE_ISSUE,
                     "core_fraction": n_core / max(1, n_terms),
                     "slots_per_eval": slots_per_launch / max(1.0, terms_per_launch)},
        "march_roofline": {"bound": "hbm", "kernel": "march_f32",
                           "achieved": march_bytes_per_launch / mar_launch_s / 1e9, "peak": HBM_PEAK / 1e9,
                           "unit": "GB/s", "frac": march_bytes_per_launch / mar_launch_s / HBM_PEAK,
                           "traffic": march_traffic, "row_bytes_per_launch": march_bytes_per_launch,
                           "hbm_GB_per_s_from_counters": (march_traffic / mar_launch_s / 1e9
                                                          if march_traffic else None),
                           "avg_launch_ms": mar_launch_s * 1e3},
        "p50_latency_ms": None, "p99_latency_ms": None,
    }
    if not args.no_side:
        line["measured_peaks"] = peaks()
        log("peaks done")
        line["stagnation"] = whole_solve_leg("stagnation", lrt, torch, 3, 1, True)
        log("stagnation leg done")
        line["stagnation_generated_lines"] = generated_lines_leg(lrt, torch)
        log("generated-lines leg done")
        line["axisymmetric"] = whole_solve_leg("axi", lrt, torch, 1, 0, False)
        log("axisymmetric leg done")
        if args.serving_requests > 0:
            sv = serving(args.serving_requests)
            line["serving"] = sv
            line["p50_latency_ms"] = sv["open_loop"]["0.5_x_sat"]["p50_latency_ms"]
            line["p99_latency_ms"] = sv["open_loop"]["0.5_x_sat"]["p99_latency_ms"]
            line["serving_solves_per_s"] = sv["open_loop"]["0.5_x_sat"]["solves_per_s"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, np.arange(kf[3], kf[3] + npt[3]))
    line["bench_seconds"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
