"""Benchmark of the line-by-line + ray-march hot path on one MI355X.

One step = the whole path over one batch of resident synthetic input:
per-cell populations and scales, per-(cell, line) setup, line-to-grid Voigt
accumulation of eta/kappa for every cell, march of every ray and the spectral
+ angular quadrature to the wall flux (lrt_solve).  Default workload: the 1-D
stagnation line with 400 cells, 11 species, 200k atomic + 2M rovibronic lines,
a 2^21-point grid over 1000-100000 cm^-1 and 17 rays (wall normal + 16
Gauss-Legendre directions), in the compensated single-precision form.  The
double-precision form is timed beside it for the speedup and the error.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Voigt line-pt evals/s + q_rad solves/s (FP32-comp vs FP64, 1 GPU); p99 latency"

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz -> non-packed FP32 VALU lane-op
# issue rate (one wave64 instruction per SIMD every 4 cycles).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Issue slots of one profile evaluation in the form the kernel evaluates, one
# slot per VALU instruction, transcendentals included (v_exp/v_log/v_rcp issue
# in one slot; the transcendental unit behind them runs at half rate, which
# instruction counters show overlapping with other VALU issue rather than
# adding a second slot).  In y = (nu - nu0)/gamma_V:
#   wing point (|dnu| > 25 HWHM, both exponentials exactly zero in single
#   precision): offset 2 (sub, fma), 1 + y^2 1, |y|^2.25 3 (log, scale, exp),
#   1 + 0.1 x^2.25 1, reciprocal of the product 2, numerator 2, product 1,
#   two accumulating FMAs 2 = 14;
#   core point: + exponent and exp for each of the two exponentials (4) and
#   their two FMAs = 20.
SLOTS_CORE = 20
SLOTS_WING = 14
# Issue slots of one (ray, segment, grid point) update of the single-precision
# cell-constant march: tau = kappa ds 1, exponent scale 1, exp 1, the thin-
# segment polynomial of F 5, (1 - e)/tau 3 (sub, rcp, mul), branch-free pick
# of the two 2 (compare, select), eta F 1 and its conversion and scale to
# double 2, conversion of e^-tau 1, the FP64 update of I 1 = 18.
SLOTS_MARCH = 18
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--workload", default="stagnation", choices=["stagnation", "slab", "axi", "axi_large"])
    ap.add_argument("--band", type=int, default=None,
                    help="time one band alone (coefficients of every cell, then the march of every "
                         "ray), print its own JSON line and exit")
    ap.add_argument("--cpu-points", type=int, default=1536, help="grid points of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the side measurements (march schemes, continuum, QSS-CR), so that a "
                         "profiler sees only the timed steps")
    ap.add_argument("--serving-requests", type=int, default=48,
                    help="requests per serving phase (closed loop, then open loop); 0 skips")
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
        desc = ("large axisymmetric: 512x256 cells, 11 species, 4M-line generator, 2^22-point grid "
                "in 32 bands of 131072, 256 wall points x (32 GL x 32 azimuth) rays")
    return wl, desc


def band_bench(args):
    """One band of a workload timed alone: the single-precision coefficients of
    every cell, then the march of every ray through them with the band's
    trapezoid sum (no per-point intensity kept), HIP events per kernel.  A
    whole step of the large axisymmetric case is 32 such bands."""
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
    n_seg = sum(len(ctx.ray(r)[0]) for r in range(sz["n_rays"]))
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
        "accum_ms": acc_s * 1e3, "accum_frac_of_valu_issue": slots / acc_s / PEAK_LANE_OPS,
        "march_ms": mar_s * 1e3, "segment_points": seg_pts,
        "march_row_GB_per_s": seg_pts * 8 / mar_s / 1e9,
        "march_frac_of_valu_issue": seg_pts * SLOTS_MARCH / mar_s / PEAK_LANE_OPS,
        "kernels_ms": {k: v[0] / args.steps for k, v in prof.items()}}), flush=True)
    ctx.close()


# Sources of the accumulation kernel; the committed counter summary records
# their sha256 (in this order).
ACCUM_SOURCES = ("lrt_accum.hip", "lrt_device.h", "lrt_internal.h")


def counter_traffic(workload_name):
    """HBM bytes per accumulation launch from the committed counter summary, if
    it was taken on the stagnation workload with the current kernel sources;
    otherwise None."""
    import hashlib
    if workload_name != "stagnation":
        return None
    path = os.path.join(ROOT, "profiles", "accum_f32_stagnation_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for ln in open(path):
        if ":" in ln:
            k, v = ln.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ACCUM_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2604_11856_amd", "csrc", f), "rb").read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch"])


def serving(n_closed, n_open, budget_gb=64, slots=64):
    """Serving stream on the resident 1M-line list and 2^20-point grid:
    closed-loop saturation (all requests at t = 0), then Poisson arrivals at
    half that rate; latency = submit -> result on the host."""
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
    reqs = synth.serving_requests(n_closed, wl.grid.n_points, seed=11859)
    # (cell, grid point) pairs whose coefficients the closed loop computes and marches
    cell_points = sum(int(r.cells.n) * int(r.n_window) for r in reqs)
    t0 = time.perf_counter()
    res = [srv.wait(t) for t in [srv.submit(r) for r in reqs]]
    t_closed = time.perf_counter() - t0
    x_sat = n_closed / t_closed
    rate = 0.5 * x_sat
    reqs = synth.serving_requests(n_open, wl.grid.n_points, rate_hz=rate, seed=11861)
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        dt = t0 + r.arrival - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(r))
    res = [srv.wait(t) for t in tickets]
    t_open = time.perf_counter() - t0
    ok = all(x["status"] == 0 for x in res)
    lat = np.array([x["latency_ms"] for x in res])
    info = srv.info()
    srv.stop()
    ctx.close()
    return {"resident": "1M lines (250k atomic + 750k rovibronic), 2^20-point grid 1000-100000 cm^-1",
            "requests": "cells logU[16, 2048], window logU[1e4, 1e6] points, mixed species subsets",
            "budget_GB": budget_gb, "slots": slots, "all_ok": ok,
            "closed_loop": {"requests": n_closed, "seconds": t_closed, "solves_per_s": x_sat,
                            "cell_points": cell_points, "cell_points_per_s": cell_points / t_closed},
            "open_loop": {"requests": n_open, "rate_hz": rate, "seconds": t_open,
                          "solves_per_s": n_open / t_open,
                          "p50_latency_ms": float(np.percentile(lat, 50)),
                          "p99_latency_ms": float(np.percentile(lat, 99)),
                          "max_latency_ms": float(lat.max())},
            "epochs": info["epochs"]}


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


def cpu_baseline(wl, n_points):
    import oracle as O
    from paper_2604_11856_amd import synth
    threads = min(os.cpu_count() or 1, 16)
    ks = synth.sample_points(wl.grid, wl.lines, n_points, seed=1)
    t = time.perf_counter()
    _, _, n_terms = O.coeffs(wl.species, wl.lines, wl.cells, wl.grid, ks, threads=threads)
    dt = time.perf_counter() - t
    return {"value": n_terms / dt, "unit": "Voigt line-pt evals/s", "cores": threads,
            "kind": "oracle",
            "sample": "all %d cells x %d grid points (%d-point clusters), all %d lines: %d terms in %.2f s"
                      % (wl.cells.n, ks.size, 32, wl.lines.n, n_terms, dt)}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.band is not None:
        band_bench(args)
        return
    import torch
    from paper_2604_11856_amd import lrt

    wl, desc = workload(args.workload)
    ctx = lrt.Context(0).load(wl)
    sz = ctx.sizes()
    counts = [ctx.count_terms(b, core=True) for b in range(sz["n_bands"])]
    n_terms = sum(c[0] for c in counts)
    n_core = sum(c[1] for c in counts)
    seg_pts = sum(len(ctx.ray(r)[0]) for r in range(sz["n_rays"])) * sz["n_points"]

    def run(prec, steps, warmup):
        for _ in range(warmup):
            ctx.solve(prec)
        torch.cuda.synchronize()
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for _ in range(steps):
            out = ctx.solve(prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        prof = {k: ctx.profile_read(k) for k in lrt.KERNELS}
        ctx.profile(False)
        return dt, out, prof

    dt32, (q32, I32, _), prof32 = run(lrt.LRT_FP32_COMP, args.steps, args.warmup)
    res = {}
    if args.fp64_steps > 0:
        dt64, (q64, I64, _), prof64 = run(lrt.LRT_FP64, args.fp64_steps, 0)
        res = {"ms_per_step": dt64 * 1e3, "evals_per_s": n_terms / dt64,
               "accum_ms_per_launch": prof64["accum"][0] / max(1, prof64["accum"][1]),
               "speedup_fp32c_over_fp64": dt64 / dt32,
               "rel_err_fp32c_vs_fp64": {
                   "I_int_max": float(np.max(np.abs(I32 - I64) / np.maximum(np.abs(I64), 1e-300))),
                   "q": [float(abs(a - b) / abs(b)) if b != 0 else 0.0 for a, b in zip(q32, q64)]}}

    march_schemes = continuum = cr = lorentz = None
    if not args.no_side:
        march_schemes = compare_march_schemes(ctx, lrt, torch, sz)
        continuum = continuum_cost(ctx, wl, lrt, torch)
        lorentz = lorentz_cost(ctx, wl, lrt, torch)
        cr = cr_cost(wl, lrt, torch) if args.workload == "stagnation" else None

    acc_ms, acc_n = prof32["accum"]
    acc_s = acc_ms / 1e3 / max(1, acc_n)
    terms_per_launch = n_terms / sz["n_bands"]
    slots_per_launch = (n_core * SLOTS_CORE + (n_terms - n_core) * SLOTS_WING) / sz["n_bands"]
    achieved = slots_per_launch / acc_s
    mar_ms, mar_n = prof32["march"]
    mar_s = mar_ms / 1e3 / max(1, mar_n)
    march_bytes = seg_pts * 8 / sz["n_bands"]
    march_slots = seg_pts * SLOTS_MARCH / sz["n_bands"]
    unique_bytes = sz["n_cells"] * sz["n_points"] * 8 / sz["n_bands"]

    line = {
        "metric": METRIC,
        "value": n_terms / dt32,
        "unit": "Voigt line-pt evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "precision": "fp32 profile evaluation, per-point sums over 64-line "
                   "blocks merged with Kahan compensation; populations, widths, windows, march "
                   "state and quadrature in f64",
                   "cells": sz["n_cells"], "lines": wl.lines.n, "grid_points": sz["n_points"],
                   "bands": sz["n_bands"], "rays": sz["n_rays"], "wall_points": sz["n_wall"],
                   "voigt_terms_per_step": n_terms},
        "q_rad_solves_per_s": sz["n_wall"] / dt32,
        "los_solves_per_s": sz["n_rays"] / dt32,
        "q_rad_W_cm2": [float(x) for x in q32],
        "fp64": res,
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in prof32.items()},
        "roofline": {"bound": "alu", "kernel": "accum_f32",
                     "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T lane-op/s (FP32 VALU issue slots, one per instruction)",
                     "frac": achieved / PEAK_LANE_OPS, "traffic": counter_traffic(args.workload),
                     "evals_per_launch": terms_per_launch,
                     "core_fraction": n_core / max(1, n_terms),
                     "slots_per_eval": slots_per_launch / max(1.0, terms_per_launch),
                     "avg_launch_ms": acc_s * 1e3},
        "march_schemes": march_schemes,
        "continuum": continuum,
        "lorentz": lorentz,
        "cr": cr,
        # every ray of a wall point re-reads the rows of the cells it crosses, so
        # the march does an exp per (ray, segment, point) on 8 B that the rays
        # share through the caches: it is bound by VALU issue, not by HBM
        "march_roofline": {"bound": "alu", "kernel": "march_f32",
                           "achieved": march_slots / mar_s / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                           "unit": "T lane-op/s (VALU issue slots, one per instruction)",
                           "frac": march_slots / mar_s / PEAK_LANE_OPS, "avg_launch_ms": mar_s * 1e3,
                           "segment_points_per_launch": seg_pts / sz["n_bands"],
                           "slots_per_segment_point": SLOTS_MARCH,
                           "row_bytes_per_launch": march_bytes,
                           "row_GB_per_s": march_bytes / mar_s / 1e9,
                           "unique_bytes_per_launch": unique_bytes,
                           "unique_frac_of_hbm_peak": unique_bytes / mar_s / HBM_PEAK},
        "p50_latency_ms": None, "p99_latency_ms": None,
    }
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if args.serving_requests > 0:
        sv = serving(args.serving_requests, args.serving_requests)
        line["serving"] = sv
        line["p50_latency_ms"] = sv["open_loop"]["p50_latency_ms"]
        line["p99_latency_ms"] = sv["open_loop"]["p99_latency_ms"]
        line["serving_solves_per_s"] = sv["open_loop"]["solves_per_s"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_points)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
