"""Throughput of the ISM chemistry + cooling source step on one MI355X.

The metric workload (default, `--workload pts512`): the 512^3 lognormal-GRF grid with 2 pc
cells, 16 point sources (maps made once from the initial state), a per-cell CR map, Z' = 1 and
one step of dt = 1e4 yr.  A step is one pass of the hot path: six-ray columns, then the source
step of every cell; the cell state is restored from a device copy before each step, so every
step does the same work.  Three forms are measured in the same run:

  f64        plain method, FP64 everywhere                       (columns F64 + step F64)
  mixed      plain method, FP32 evaluation, FP64 update/sums     (columns MIXED + step MIXED)
  surrogate  FP32 + learned surrogate with certification and
             fallback to the mixed step                          (columns MIXED + surrogate step)

`value` is the cell-updates/s of `--path` (default f64) over K steps (W untimed steps first,
synchronisations around the K), inputs resident in HBM; `paths` reports all three forms with
their substep statistics, per-field error against the FP64 oracle on the 64^3 subsample, the
surrogate's fallback fraction and the speedups.  `cpu_baseline` times the oracle on a bounded
sample of the same workload, in one process and over the host's cores.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--path f64|mixed|surrogate] [--no-cpu]

Other workloads (`--workload`): grf128, the 128^3 GRF grid (4 pc cells, CR attenuation by
N_eff); pts256, the 256^3 grid with 16 point sources and ten successive mixed steps (`--maps
lc|art`: straight-line maps or the adaptive ray trace, which also measures the flux trace and the
radiation force); train, the surrogate's Adam steps.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3           # packed FP32 (two lanes per instruction)
FP32_ISSUE_PEAK_TFLOPS = 78.6      # what the library's code can issue: packed FP32 is kept out of it
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_CELL = 2 * (10 * 128 + 2 * 128 * 128 + 128 * 3)
FIELDS = ("T", "xH2", "xHp", "xe", "xCp", "xCO")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", choices=("f64", "mixed", "surrogate"), default="f64")
    ap.add_argument("--workload", choices=("grf128", "pts256", "pts512", "train"), default="pts512",
                    help="pts512: the metric workload, 512^3 with 16 point sources, K steps of each form; grf128: the "
                         "128^3 GRF grid; pts256: 256^3 with 16 point sources, ten successive steps (mixed form); "
                         "train: surrogate training, one Adam step of batch 65,536 per step (use --steps of a few "
                         "hundred)")
    ap.add_argument("--pts512-stride", type=int, default=8,
                    help="pts512: error report on every s-th cell along each axis (8: a 64^3 subsample)")
    ap.add_argument("--maps", choices=("lc", "art"), default="lc",
                    help="pts256 point-source maps: lc straight-line 1/r^2 exp(-tau) with the Stromgren cap (the "
                         "configuration's recipe), art adaptive ray tracing (Sec. 5.1)")
    ap.add_argument("--pts256-order", choices=("previous", "temperature"), default="previous",
                    help="pts256 processing order of steps 2-10: by the previous step's substep counts (order_cells 2) "
                         "or by temperature (order_cells 1); the first step is always by temperature")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the error report")
    ap.add_argument("--cpu-cells", type=int, default=65536)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a cache-cold 1 GiB buffer (the known-size kernel that scales HBM counters)")
    return ap.parse_args()


def _code_only(src):
    """C++ source without its comments, its tokens joined by single spaces (string and character
    literals kept)."""
    import re
    pat = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'', re.S)
    code = pat.sub(lambda m: "" if m.group(0).startswith("/") else m.group(0), src)
    return " ".join(code.split())


def kernel_source_hash():
    """SHA-256 over the code of the library's HIP sources (comments left out): traffic counters
    stay valid only while the code they were taken on is unchanged."""
    import hashlib
    d = os.path.join(ROOT, "paper_2210_08024_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(_code_only(open(os.path.join(d, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def measured_counters(kernel, workload="grf128"):
    """Counters per launch of `kernel` from the committed summary of `workload`, if it was taken on
    the current sources: HBM bytes (FETCH_SIZE x fetch factor + WRITE_SIZE x write factor, KiB ->
    bytes), VALU wave instructions and lane utilisation.  None when absent or stale."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    rows, meta = {}, {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, val = line.partition("=")
        key = key.strip()
        if key in ("src_sha", "fetch_factor", "write_factor"):
            meta[key] = val.strip()
        else:
            rows[key] = [float(v) for v in val.split()]
    if meta.get("src_sha") != kernel_source_hash() or kernel not in rows:
        return None
    v = rows[kernel]
    out = {"bytes": 1024.0 * (v[0] * float(meta["fetch_factor"]) + v[1] * float(meta["write_factor"]))}
    if len(v) >= 4:
        out["valu_insts"], out["lane_util"] = v[2], v[3]
    return out


def measured_traffic(kernel):
    c = measured_counters(kernel)
    return None if c is None else c["bytes"]


def calibrate_copy():
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    c = torch.empty_like(a)
    c.fill_(2.0)  # a second GiB written after a evicts it from L2 and the Infinity Cache
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": a.numel() * 4}), flush=True)


def copy_bandwidth(reps=3):
    """Achievable HBM bandwidth: best of `reps` timed device copies of 1 GiB (read + write), GB/s."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(reps + 1):
        ev[0].record()
        b.copy_(a)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / best / 1e9


def cpu_baseline(state, cfg, ncell_sample, par_o):
    """The CPU oracle on the same workload: its vectorised six-ray columns over the whole 128^3 grid,
    then its step on a seeded sample of the cells; cell-updates/s = 1 / (columns time per grid cell +
    step time per sampled cell)."""
    from oracle import columns as ocol
    from oracle import step as ostep
    from oracle.constants import PC, YR
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(state["n"].size, ncell_sample, replace=False))
    t0 = time.perf_counter()
    rc = ocol.columns6(state["n"], state["xH2"], None, cfg["dx_pc"] * PC, par_o)
    t1 = time.perf_counter()
    sel = lambda a: np.ascontiguousarray(np.asarray(a).ravel()[idx])
    rad = dict(chi_PE=sel(rc["chi_PE"]), chi_LW=sel(rc["chi_LW"]), chi_H2=sel(rc["chi_H2"]), chi_C=sel(rc["chi_C"]),
               phi=np.zeros(len(idx)), xi=sel(rc["xi"]), Neff=sel(rc["N_eff"]))
    ref = ostep.chem_cool_step(sel(state["n"]), sel(state["T"]), sel(state["xH2"]), sel(state["xHp"]), rad,
                               cfg["dt_yr"] * YR, par_o)
    t2 = time.perf_counter()
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    base = {"value": 1.0 / ((t1 - t0) / state["n"].size + (t2 - t1) / ncell_sample), "unit": "cell-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"the oracle's vectorised six-ray columns over the 128^3 grid ({t1 - t0:.1f} s) + its step on "
                      f"{ncell_sample} seeded random cells ({t2 - t1:.1f} s), numpy single-threaded; host has "
                      f"{threads} threads"}
    return base, idx, ref, rad


def cpu_parallel(pool, procs, state, cfg, idx, rad, par_o, chunk=4096):
    """The oracle over the pool of worker processes: its vectorised six-ray columns over eight 64^3
    sub-boxes of the grid (the same work per cell as the whole grid), then its step on the sampled
    cells in chunks of `chunk`; cell-updates/s = 1 / (columns time per cell + step time per cell)."""
    from oracle.constants import PC, YR
    m = 64
    boxes = _sub_boxes(state["n"].shape, m, 8)
    box = lambda o, k: np.ascontiguousarray(state[k][o[0]:o[0] + m, o[1]:o[1] + m, o[2]:o[2] + m])
    dx, dt = cfg["dx_pc"] * PC, cfg["dt_yr"] * YR
    t0 = time.perf_counter()
    ncol = sum(pool.map(_oracle_columns_box, [(box(o, "n"), box(o, "xH2"), dx, par_o) for o in boxes]))
    t_col = time.perf_counter() - t0
    sel = lambda a, i, j: np.ascontiguousarray(np.asarray(a).ravel()[idx[i:j]])
    jobs = [(sel(state["n"], i, i + chunk), sel(state["T"], i, i + chunk), sel(state["xH2"], i, i + chunk),
             sel(state["xHp"], i, i + chunk), {k: v[i:i + chunk] for k, v in rad.items()}, dt, par_o)
            for i in range(0, len(idx), chunk)]
    t0 = time.perf_counter()
    pool.map(_oracle_chunk, jobs)
    t_step = time.perf_counter() - t0
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / (t_col / ncol + t_step / len(idx)), "unit": "cell-updates/s", "cores": procs,
            "kind": "oracle",
            "sample": f"columns over 8 sub-boxes of 64^3 ({t_col:.2f} s) + the step of the same {len(idx)} cells in "
                      f"chunks of {chunk} ({t_step:.1f} s), {procs} worker processes; CPU {model}"}


def conservation(res, xCt, xOt):
    """Element budgets of a step's output.  x_H, x_C and x_O are formed from the closure
    relations (x_H = 1 - 2 x_H2 - x_H+, x_C = x_C,tot - x_C+ - x_CO, x_O = x_O,tot - x_CO - x_O+
    with x_O+ = x_O,tot x_H+), so each sum holds exactly; what can fail is the remainder going
    negative.  Reported: the largest excess of each sum over its total (0 = conserved with every
    species >= 0) and the smallest abundance."""
    xH2, xHp = res["xH2"].astype(np.float64), res["xHp"].astype(np.float64)
    xCp, xCO = res["xCp"].astype(np.float64), res["xCO"].astype(np.float64)
    return {"H_excess_max": float(np.max(np.maximum(2.0 * xH2 + xHp - 1.0, 0.0))),
            "C_excess_max": float(np.max(np.maximum((xCp + xCO) / xCt - 1.0, 0.0))),
            "O_excess_max": float(np.max(np.maximum(xCO / xOt + xHp - 1.0, 0.0))),
            "min_abundance": float(min(xH2.min(), xHp.min(), xCp.min(), xCO.min()))}


def device_conservation(xH2, xHp, xCp, xCO, par_o):
    """conservation() over whole device arrays, with reductions on the device."""
    cp, co = xCp.double(), xCO.double()
    xCt, xOt = par_o.xCtot, par_o.xOtot
    return {"H_excess_max": float((2.0 * xH2 + xHp - 1.0).clamp_min(0.0).max()),
            "C_excess_max": float(((cp + co) / xCt - 1.0).clamp_min(0.0).max()),
            "O_excess_max": float((co / xOt + xHp - 1.0).clamp_min(0.0).max()),
            "min_abundance": float(min(xH2.min(), xHp.min(), cp.min(), co.min()))}


def field_errors(out, ref, idx, xCt, cells=None):
    """Per-field max / p99 relative error at the sampled cells (floors: 1e-7 for abundances, carbon
    species relative to x_C,tot), the fraction of sampled cells over 1e-3 in any field and, with
    `cells` (the grid index of each sampled cell), the grid indices of the first 8 such cells."""
    rep, worst = {}, np.zeros(len(idx))
    for k in FIELDS:
        fl = 0.0 if k == "T" else 1e-7 * (xCt if k in ("xCp", "xCO") else 1.0)
        a = out[k][idx].astype(np.float64)
        b = ref[k]
        e = np.abs(a - b) / np.maximum(np.abs(b), fl)
        rep[k] = {"max": float(e.max()), "p99": float(np.percentile(e, 99))}
        worst = np.maximum(worst, e)
    rep["frac_cells_over_1e-3"] = float((worst > 1e-3).mean())
    if cells is not None:
        rep["cells_over_1e-3"] = [int(cells[i]) for i in np.nonzero(worst > 1e-3)[0][:8]]
    return rep


def bench_pts256(args):
    """256^3, 2 pc cells, 16 point sources (maps once: straight-line 1/r^2 exp(-tau) maps, or
    with --maps art the adaptive ray tracing of Sec. 5.1), CR map, ten successive mixed steps of
    1e4 yr with x_C fed back into the columns; value = cell-updates/s over the ten steps, the
    one-time point-source maps included."""
    import torch
    from paper_2210_08024_amd import ism, workloads
    from oracle.census import substep_census
    from oracle.constants import Params as OParams
    s, cfg = workloads.make("pts256")
    shape = s["n"].shape
    N = s["n"].size
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ism.init(0)
    par = ism.Params(Zg=1.0, Zd=1.0, cr_mode=2)
    # steps after the first: cells grouped by the previous step's substep counts (in outs["nsub"])
    par_next = ism.Params(Zg=1.0, Zd=1.0, cr_mode=2, order_cells=2 if args.pts256_order == "previous" else 1)
    dx = cfg["dx_pc"] * workloads.PC
    dt = cfg["dt_yr"] * workloads.YR
    stream = torch.cuda.current_stream()
    init = {k: torch.from_numpy(np.ascontiguousarray(s[k]).ravel()).to(dev) for k in ("n", "T", "xH2", "xHp")}
    xi = torch.from_numpy(s["xi"].ravel()).to(dev, torch.float32)
    n = init["n"].view(shape)
    T, xH2, xHp = (torch.empty_like(init[k]) for k in ("T", "xH2", "xHp"))
    f32 = lambda: torch.empty(N, dtype=torch.float32, device=dev)
    maps = {k: f32() for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")}
    rad = {k: f32() for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
    outs = {"xCp": f32(), "xCO": f32(), "xe": f32(), "nsub": torch.empty(N, dtype=torch.int32, device=dev),
            "status": torch.empty(N, dtype=torch.uint8, device=dev)}
    xC = torch.empty(N, dtype=torch.float64, device=dev)
    xCt = OParams(Zg=1.0).xCtot
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    times = {"maps": [], "columns": [], "step": []}
    tot_sub = []

    def run(record):
        T.copy_(init["T"])
        xH2.copy_(init["xH2"])
        xHp.copy_(init["xHp"])
        for v in maps.values():
            v.zero_()
        ev[0].record(stream)
        if args.maps == "art":
            ism.ray_trace(n, xH2.view(shape), xHp.view(shape), None, dx, par, ism.MIXED, cfg["sources"],
                          {k: v.view(shape) for k, v in maps.items()})
        else:
            ism.point_sources(n, xH2.view(shape), None, dx, par, ism.MIXED, cfg["sources"],
                              {k: v.view(shape) for k, v in maps.items()})
        ev[1].record(stream)
        if record:
            torch.cuda.synchronize()
            times["maps"].append(ev[0].elapsed_time(ev[1]) * 1e-3)
        for step in range(cfg["steps"]):
            rad["xi"].copy_(xi)
            ev[2].record(stream)
            ism.columns6(n, xH2.view(shape), None if step == 0 else xC.view(shape), dx, par, ism.MIXED,
                         out={k: v.view(shape) for k, v in rad.items()})
            for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C"):
                rad[k].add_(maps[k])
            r = dict(rad)
            r["phi"] = maps["phi"]
            ev[3].record(stream)
            ism.chem_cool_step(init["n"], T, xH2, xHp, r, dt, par if step == 0 else par_next, ism.MIXED, out=outs)
            ev[0].record(stream)
            torch.sub(xCt, outs["xCp"].double() + outs["xCO"].double(), out=xC).clamp_(min=0.0)
            if record:
                torch.cuda.synchronize()
                times["columns"].append(ev[2].elapsed_time(ev[3]) * 1e-3)
                times["step"].append(ev[3].elapsed_time(ev[0]) * 1e-3)
                tot_sub.append(int(outs["nsub"].to(torch.int64).sum().item()))

    for _ in range(args.warmup):
        run(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(False)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    run(True)
    # for reference, outside the timed job: the other way of making the maps
    other = {k: torch.zeros_like(v) for k, v in maps.items()}
    ev[0].record(stream)
    if args.maps == "art":
        ism.point_sources(n, init["xH2"].view(shape), None, dx, par, ism.MIXED, cfg["sources"],
                          {k: v.view(shape) for k, v in other.items()})
    else:
        ism.ray_trace(n, init["xH2"].view(shape), init["xHp"].view(shape), None, dx, par, ism.MIXED,
                      cfg["sources"], {k: v.view(shape) for k, v in other.items()})
    ev[1].record(stream)
    torch.cuda.synchronize()
    other_ms = ev[0].elapsed_time(ev[1])
    force = None
    if args.maps == "art":
        force = bench_radiation_force(ism, par, n, init, shape, dx, cfg["sources"], stream, ev)
    how = ("adaptive ray tracing (Sec. 5.1)" if args.maps == "art" else
           "straight-line 1/r^2 exp(-tau) maps with the Stromgren cap")
    arith, trans = substep_census(OParams())
    t_step = float(np.sum(times["step"]))
    achieved = float(np.sum(tot_sub)) * (arith + trans) / t_step / 1e12
    out = {
        "metric": "cell-updates/s per chem+cool step (columns6 + source step)",
        "value": N * cfg["steps"] / wall, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / cfg["steps"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "pts256: 256^3 lognormal GRF (2 pc cells, 512 pc box), 16 point sources (Q 1.24e50 s^-1, "
                               "L_FUV 1.36e6 L_sun; maps once by " + how + "), chi0 = 1 six-ray, xi_cr log-uniform [1e-17, 1e-15], "
                               "Z' = 1, ten successive steps of 1e4 yr", "cells": N, "path": "mixed",
                   "maps": args.maps, "job": "point-source maps once + ten (columns6 + step)",
                   "order": "steps 2-10 by the previous step's substep counts" if args.pts256_order == "previous"
                   else "by temperature"},
        "roofline": {"bound": "alu", "kernel": "step_queue_kernel", "achieved": achieved, "peak": FP32_ISSUE_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_ISSUE_PEAK_TFLOPS,
                     "traffic": None, "work": f"{int(np.sum(tot_sub))} substeps over ten steps x ({arith} + {trans})"},
        "detail": {"maps_ms": times["maps"][0] * 1e3,
                   ("maps_long_characteristics_ms" if args.maps == "art" else "maps_ray_tracing_ms"): other_ms, "columns_ms_mean": float(np.mean(times["columns"])) * 1e3,
                   "step_ms_mean": float(np.mean(times["step"])) * 1e3,
                   "step_ms_each": [round(t * 1e3, 3) for t in times["step"]],
                   "nsub_mean_each": [round(x / N, 3) for x in tot_sub],
                   "status_nonzero_last": int(((outs["status"] & 0xEF) != 0).sum().item()),
                   "conservation_last": device_conservation(xH2, xHp, outs["xCp"], outs["xCO"], OParams(Zg=1.0))},
    }
    if force is not None:
        out["radiation_force"] = force
    print(json.dumps(out), flush=True)


# Algorithmic bytes per cell of radiation_force_kernel on the mixed path: reads the 9 float
# flux components and n, T, x_H2, x_H+ (double), writes 3 float force components and the
# grain-destruction byte.
FORCE_BYTES_MIXED = 9 * 4 + 4 * 8 + 3 * 4 + 1


def bench_radiation_force(ism, par, n, init, shape, dx, sources, stream, ev, reps=20):
    """Outside the timed job: the ray trace with the flux estimator (Eq. e:Frad) on the initial
    state, and the radiation force with the grain-destruction switch (Sec. 6.2) from it."""
    import torch
    N = n.numel()
    fx = {k: torch.zeros(shape, dtype=torch.float32, device="cuda") for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")}
    fx["flux"] = torch.zeros((9,) + tuple(shape), dtype=torch.float32, device="cuda")
    xH2, xHp, T = init["xH2"].view(shape), init["xHp"].view(shape), init["T"].view(shape)
    ev[0].record(stream)
    ism.ray_trace(n, xH2, xHp, None, dx, par, ism.MIXED, sources, fx)
    ev[1].record(stream)
    torch.cuda.synchronize()
    trace_ms = ev[0].elapsed_time(ev[1])
    f_rad = torch.empty((3,) + tuple(shape), dtype=torch.float32, device="cuda")
    off = torch.empty(tuple(shape), dtype=torch.uint8, device="cuda")
    ism.radiation_force(n, T, xH2, xHp, fx["flux"], par, ism.MIXED, f_rad=f_rad, dust_off=off)
    ev[2].record(stream)
    for _ in range(reps):
        ism.radiation_force(n, T, xH2, xHp, fx["flux"], par, ism.MIXED, f_rad=f_rad, dust_off=off)
    ev[3].record(stream)
    torch.cuda.synchronize()
    force_ms = ev[2].elapsed_time(ev[3]) / reps
    gbs = N * FORCE_BYTES_MIXED / (force_ms * 1e-3) / 1e9
    copy = copy_bandwidth()
    return {"ray_trace_with_flux_ms": trace_ms, "radiation_force_ms": force_ms,
            "dust_off_fraction": float(off.double().mean().item()),
            "roofline": {"bound": "hbm", "kernel": "radiation_force_kernel", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                         "work": f"{FORCE_BYTES_MIXED} B/cell x {N} cells per launch",
                         "copy_GBs_measured": copy, "frac_of_copy": gbs / copy}}


# Per training sample: forward 2 (10 x 128 + 2 x 128 x 128 + 128 x 3) FLOP, backward (error
# signal and weight gradients) twice that.
TRAIN_FLOP_PER_SAMPLE = 3 * 68864
# HBM bytes per training sample as the kernels move them: the forward stores the FP32
# pre-activations (3 x 128) and BF16 layer inputs (16 + 3 x 128) and reads X, Y (13 floats); the
# backward reads the pre-activations and writes the error signals over them (2 x 3 x 128 FP32);
# the weight gradients read the error signals (3 x 128 FP32 + 3) and the layer inputs again.
TRAIN_BYTES_PER_SAMPLE = (3 * 128 * 4 + (16 + 3 * 128) * 2 + 13 * 4) + 2 * 3 * 128 * 4 + \
    (3 * 128 * 4 + 3 * 4 + (16 + 3 * 128) * 2)


def bench_train(args):
    """Surrogate training: K timed Adam steps (forward with stored activations, backward, per-chunk
    weight gradients, ordered reduction, Adam on FP32 masters) of batch 65,536 on seeded standard
    normal pairs of the network's shapes (10 inputs, 3 outputs; the checkpoint itself is trained
    by surrogate_train.py on pairs from the plain FP64 step).  HIP events on the launch stream."""
    import torch
    from paper_2210_08024_amd import ism
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    ism.init(0)
    B = 65536
    g = torch.Generator(device="cuda").manual_seed(11)
    X = torch.randn((16 * B, 10), device="cuda", generator=g)
    Y = torch.randn((16 * B, 3), device="cuda", generator=g)
    sur = ism.Surrogate(seed=0)
    sur.set_norm([0.0] * 10, [1.0] * 10, [0.0] * 3, [1.0] * 3)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(k):
        b = k % 16
        sur.train_step(X[b * B:(b + 1) * B], Y[b * B:(b + 1) * B], 1e-3, loss)

    for k in range(args.warmup):
        step(k)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        step(k)
    ev[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t = ev[0].elapsed_time(ev[1]) * 1e-3
    tf = TRAIN_FLOP_PER_SAMPLE * B * args.steps / t / 1e12
    gbs = TRAIN_BYTES_PER_SAMPLE * B * args.steps / t / 1e9
    out = {"metric": "surrogate training samples/s", "value": B * args.steps / t, "unit": "samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3 / max(args.steps, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32",
           "data": "synthetic",
           "config": {"workload": "train: 10 -> 128 -> 128 -> 128 -> 3 SiLU network, batch 65,536, Adam; seeded "
                                  "standard normal pairs", "wall_ms_per_step": wall * 1e3 / max(args.steps, 1),
                      "final_loss": float(loss.item())},
           "roofline": {"bound": "mfma", "kernel": "training step (5 kernels)", "achieved": tf,
                        "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / BF16_PEAK_TFLOPS, "traffic": None,
                        "work": f"{TRAIN_FLOP_PER_SAMPLE} FLOP/sample x {B} samples per step"},
           "roofline_hbm": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": gbs / HBM_PEAK_GBS,
                            "work": f"{TRAIN_BYTES_PER_SAMPLE} B/sample of stored activations moved per step"}}
    print(json.dumps(out), flush=True)


def _oracle_chunk(job):
    """One chunk of the oracle step (a worker of the error report and of the parallel CPU baseline)."""
    from oracle import step as ostep
    n, T, xH2, xHp, rad, dt, par = job
    return ostep.chem_cool_step(n, T, xH2, xHp, rad, dt, par)


def _oracle_columns_box(job):
    """The oracle's vectorised six-ray columns over one sub-box (a worker of the parallel CPU baseline)."""
    from oracle import columns as ocol
    n, xH2, dx, par = job
    ocol.columns6(n, xH2, None, dx, par)
    return n.size


def _sub_boxes(shape, m, k):
    """k corner offsets of m^3 sub-boxes spread over the grid (deterministic)."""
    offs = []
    for q in range(k):
        offs.append(tuple(((q * 7 + a * 3) % max(1, (d - m) // m + 1)) * m for a, d in enumerate(shape)))
    return offs


def bench_pts512(args):
    """512^3, 2 pc cells, 16 point sources, CR map, one step of 1e4 yr on each form (plain F64, plain
    mixed, FP32 + surrogate with the plain mixed step as fallback).  A step of a form is six-ray
    columns + source step with the state restored from a device copy first.  The point-source
    maps are computed once from the initial state (in double; the mixed forms take them rounded to
    float) and are not part of the step.  value = cell-updates/s of --path (default f64) over K
    timed steps.  Errors: every form against the FP64 oracle step on the stride-s subsample (s = 8:
    64^3 cells), fed the GPU's FP64 radiation at those cells; the oracle runs in a pool of worker
    processes forked before the GPU is touched."""
    import multiprocessing as mp
    try:
        ncores = len(os.sched_getaffinity(0))
    except Exception:
        ncores = os.cpu_count() or 1
    procs = max(1, min(16, ncores))
    pool = None if args.no_cpu else mp.get_context("fork").Pool(procs)
    import torch
    from paper_2210_08024_amd import ism, workloads, surrogate_train
    from oracle.census import substep_census
    from oracle.constants import Params as OParams
    t_gen = time.perf_counter()
    s, cfg = workloads.make("pts512")
    t_gen = time.perf_counter() - t_gen
    shape = s["n"].shape
    N = s["n"].size
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ism.init(0)
    par = ism.Params(Zg=1.0, Zd=1.0, cr_mode=2)
    par_o = OParams(Zg=1.0, Zd=1.0, cr_mode=2)
    dx = cfg["dx_pc"] * workloads.PC
    dt = cfg["dt_yr"] * workloads.YR
    stream = torch.cuda.current_stream()
    init = {k: torch.from_numpy(np.ascontiguousarray(s[k]).ravel()).to(dev) for k in ("n", "T", "xH2", "xHp")}
    xi64 = torch.from_numpy(s["xi"].ravel()).to(dev)
    n = init["n"]
    T, xH2, xHp = (torch.empty_like(init[k]) for k in ("T", "xH2", "xHp"))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    # point-source maps once, in double
    maps64 = {k: torch.zeros(N, dtype=torch.float64, device=dev) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")}
    ev[0].record(stream)
    if args.maps == "art":
        ism.ray_trace(n.view(shape), init["xH2"].view(shape), init["xHp"].view(shape), None, dx, par, ism.F64,
                      cfg["sources"], {k: v.view(shape) for k, v in maps64.items()})
    else:
        ism.point_sources(n.view(shape), init["xH2"].view(shape), None, dx, par, ism.F64, cfg["sources"],
                          {k: v.view(shape) for k, v in maps64.items()})
    ev[1].record(stream)
    torch.cuda.synchronize()
    maps_ms = ev[0].elapsed_time(ev[1])
    maps32 = {k: v.float() for k, v in maps64.items()}
    sur = surrogate_train.load()
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)

    def buffers(rd):
        rad = {k: torch.empty(N, dtype=rd, device=dev) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
        outs = {"xCp": torch.empty(N, dtype=rd, device=dev), "xCO": torch.empty(N, dtype=rd, device=dev),
                "xe": torch.empty(N, dtype=rd, device=dev), "nsub": torch.empty(N, dtype=torch.int32, device=dev),
                "status": torch.empty(N, dtype=torch.uint8, device=dev)}
        return rad, outs

    bufs = {torch.float64: buffers(torch.float64), torch.float32: buffers(torch.float32)}

    def one_step(path, evs=None):
        """One step of a form; evs = four events recorded before the columns, after the columns,
        after the point-source maps are added (before the step) and after the step (on the launch
        stream; no synchronisation here)."""
        f64 = path == "f64"
        prec = ism.F64 if f64 else ism.MIXED
        rad, outs = bufs[torch.float64 if f64 else torch.float32]
        maps = maps64 if f64 else maps32
        T.copy_(init["T"])
        xH2.copy_(init["xH2"])
        xHp.copy_(init["xHp"])
        rad["xi"].copy_(xi64)
        if evs:
            evs[0].record(stream)
        ism.columns6(n.view(shape), xH2.view(shape), None, dx, par, prec, out={k: v.view(shape) for k, v in rad.items()})
        if evs:
            evs[1].record(stream)
        for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C"):
            rad[k].add_(maps[k])
        r = dict(rad)
        r["phi"] = maps["phi"]
        if evs:
            evs[2].record(stream)
        if path == "surrogate":
            ism.chem_cool_step_surrogate(sur, n, T, xH2, xHp, r, dt, par, out=outs, n_fallback=nfb)
        else:
            ism.chem_cool_step(n, T, xH2, xHp, r, dt, par, prec, out=outs)
        if evs:
            evs[3].record(stream)

    def run_form(p, K, W):
        """W untimed steps, then K steps bracketed by synchronisations; per-step HIP events."""
        for _ in range(W):
            one_step(p)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            one_step(p, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        med = lambda a, b: float(np.median([e[a].elapsed_time(e[b]) * 1e-3 for e in evs]))
        return wall, med(0, 1), med(1, 2), med(2, 3)

    # the subsample: every s-th cell along each axis
    st = args.pts512_stride
    kk, jj, ii = np.meshgrid(np.arange(0, shape[0], st), np.arange(0, shape[1], st), np.arange(0, shape[2], st),
                             indexing="ij")
    idx = (ii + shape[2] * (jj + shape[1] * kk)).ravel()
    tid = torch.from_numpy(idx).to(dev)
    order = [args.path] + [p for p in ("f64", "mixed", "surrogate") if p != args.path]
    paths, rad_sample, walls = {}, None, {}
    for p in order:
        wall, tc, tm, ts = run_form(p, args.steps, args.warmup)
        walls[p] = wall
        rad, outs = bufs[torch.float64 if p == "f64" else torch.float32]
        if p == "f64":
            rad_sample = {k: rad[k][tid].double().cpu().numpy() for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "xi")}
            rad_sample["Neff"] = rad["N_eff"][tid].double().cpu().numpy()
            rad_sample["phi"] = maps64["phi"][tid].cpu().numpy()
        res = {"T": T[tid].cpu().numpy(), "xH2": xH2[tid].cpu().numpy(), "xHp": xHp[tid].cpu().numpy()}
        res.update({k: outs[k][tid].double().cpu().numpy() for k in ("xCp", "xCO", "xe")})
        nsub = outs["nsub"].to(torch.int64)
        q = torch.quantile(nsub[::64].double(), torch.tensor([0.5, 0.99], dtype=torch.float64, device=dev))
        paths[p] = {"ms_per_step": wall / args.steps * 1e3, "columns_ms": tc * 1e3, "maps_add_ms": tm * 1e3,
                    "step_ms": ts * 1e3, "cell_updates_per_s": N / (wall / args.steps),
                    "step_only_cell_updates_per_s": N / ts,
                    "nsub_mean": float(nsub.double().mean()), "nsub_p50": float(q[0]), "nsub_p99": float(q[1]),
                    "nsub_max": int(nsub.max()), "substeps": int(nsub.sum()),
                    "status_nonzero": int(((outs["status"] & 0xEF) != 0).sum()), "_res": res}
        paths[p]["conservation"] = device_conservation(xH2, xHp, outs["xCp"], outs["xCO"], OParams(Zg=1.0))
        if p == "surrogate":
            paths[p]["fallback_fraction"] = nfb.item() / N
            paths[p]["accepted_cells"] = int(N - nfb.item())
    for p in ("mixed", "surrogate"):
        paths[p]["speedup_vs_f64"] = paths["f64"]["ms_per_step"] / paths[p]["ms_per_step"]
    paths["surrogate"]["speedup_vs_mixed"] = paths["mixed"]["ms_per_step"] / paths["surrogate"]["ms_per_step"]
    # inference kernel alone (network inputs built once, then timed forwards) on 2^24 cells
    rad32, _ = bufs[torch.float32]
    B = 1 << 24
    X, _ = ism.surrogate_pairs(n[:B], init["T"][:B], init["xH2"][:B], init["xHp"][:B],
                               {k: v[:B] for k, v in rad32.items()}, dt, par, ism.MIXED)
    Y = torch.empty((B, 3), dtype=torch.float32, device=dev)
    sur.forward(X, Y)
    ev[0].record(stream)
    for _ in range(10):
        sur.forward(X, Y)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_mlp = ev[0].elapsed_time(ev[1]) * 1e-3 / 10
    mlp_tf = MLP_FLOP_PER_CELL * B / t_mlp / 1e12
    del X, Y
    hbm_copy = copy_bandwidth()

    # the FP64 oracle on the subsample, fed the GPU's FP64 radiation there (worker pool): the error
    # report, and the parallel leg of the CPU baseline's step
    cpu = None
    if not args.no_cpu:
        sel = lambda a: np.ascontiguousarray(a.ravel()[idx])
        st0 = {k: sel(s[k]) for k in ("n", "T", "xH2", "xHp")}
        chunk = 4096
        jobs = [tuple(st0[k][a:a + chunk] for k in ("n", "T", "xH2", "xHp")) +
                ({k: v[a:a + chunk] for k, v in rad_sample.items()}, dt, par_o) for a in range(0, len(idx), chunk)]
        t0 = time.perf_counter()
        parts = pool.map(_oracle_chunk, jobs)
        t_or_par = time.perf_counter() - t0
        ref = {k: np.concatenate([q[k] for q in parts]) for k in FIELDS}
        xCt = par_o.xCtot
        ar = np.arange(len(idx))
        for p in paths:
            paths[p]["error_vs_oracle"] = field_errors(paths[p]["_res"], ref, ar, xCt, cells=idx)
        cpu = cpu_baseline_pts512(pool, procs, s, dx, par_o, st0, rad_sample, dt, t_or_par, len(idx))
        pool.close()
        pool.join()
    for p in paths:
        paths[p].pop("_res")

    arith, trans = substep_census(par_o)
    vp = paths[args.path]
    kname = "step_queue_kernel<double>" if args.path == "f64" else "step_queue_kernel<float>"
    achieved = vp["substeps"] * (arith + trans) / (vp["step_ms"] * 1e-3) / 1e12
    peak = FP64_PEAK_TFLOPS if args.path == "f64" else FP32_ISSUE_PEAK_TFLOPS
    cnt = measured_counters(kname, "pts512")
    cols_bytes = N * (72 if args.path == "f64" else 48)
    how = ("adaptive ray tracing (Sec. 5.1)" if args.maps == "art" else
           "straight-line 1/r^2 exp(-tau) maps with the Stromgren cap")
    out = {
        "metric": "cell-updates/s per chem+cool step: FP64 plain vs FP32+surrogate at <=1e-3 rel err",
        "value": vp["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": vp["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f64": "f64", "mixed": "f32+f64", "surrogate": "bf16+f32+f64"}[args.path],
        "data": "synthetic",
        "config": {"workload": "pts512: 512^3 lognormal GRF (2 pc cells, 1024 pc box), 16 point sources (Q 1.24e50 s^-1, "
                               "L_FUV 1.36e6 L_sun; maps once by " + how + "), chi0 = 1 six-ray, xi_cr log-uniform "
                               "[1e-17, 1e-15], Z' = 1, one step of 1e4 yr (six-ray columns + source step)",
                   "cells": N, "path": args.path, "maps": args.maps},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None if cnt is None else cnt["bytes"],
                     "traffic_algorithmic": N * (133 if args.path == "f64" else 97),
                     "work": f"{vp['substeps']} substeps x ({arith} flops + {trans} transcendentals counted as 1) "
                             f"per launch (census of the oracle's substep); time = the step call (cell ordering + "
                             f"step kernel) between HIP events on the launch stream"},
        "roofline_issue": issue_roofline(kname, vp["step_ms"] * 1e-3, "pts512"),
        "roofline_columns": {"bound": "hbm", "kernel": "columns6 (all passes)", "achieved": cols_bytes / (vp["columns_ms"] * 1e-3) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": cols_bytes / (vp["columns_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "traffic": columns_traffic(args.path, "pts512"),
                             "work": f"{N} cells x {72 if args.path == 'f64' else 48} B (n, x_H2, x_C in; chi_PE, chi_LW, "
                                     f"chi_H2, chi_C, N_eff, xi out)"},
        "roofline_mlp": {"bound": "mfma", "kernel": "mlp_fwd_kernel", "achieved": mlp_tf, "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": mlp_tf / BF16_PEAK_TFLOPS, "ms": t_mlp * 1e3,
                         "work": f"{MLP_FLOP_PER_CELL} FLOP/cell x {B} cells per launch"},
        "paths": paths,
        "detail": {"maps_ms": maps_ms, "generate_s": t_gen, "subsample_cells": int(len(idx)),
                   "hbm_copy_GBs_measured": hbm_copy,
                   "fp32_peak_note": "FP32 vector peak the build can issue: 78.6 TFLOP/s (packed FP32 instructions "
                                     "are kept out of the generated code; 157.3 is the packed rate)"},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def cpu_baseline_pts512(pool, procs, s, dx, par_o, st0, rad_sample, dt, t_step_par, nsample):
    """The CPU oracle as it stands on a bounded sample of the 512^3 workload: its vectorised six-ray
    columns over sub-boxes of the grid plus its step on subsample cells (fed the GPU's FP64
    radiation).  One process: one 128^3 sub-box and the whole subsample (about 6 s); all cores: 16
    sub-boxes of 96^3 over the pool and the whole subsample (the error report's run).
    cell-updates/s = 1 / (columns time per cell + step time per cell)."""
    from oracle import columns as ocol
    from oracle import step as ostep
    m, m1 = 96, 128
    shape = s["n"].shape
    boxes = _sub_boxes(shape, m, 16)
    box = lambda o, k, e=m: np.ascontiguousarray(s[k][o[0]:o[0] + e, o[1]:o[1] + e, o[2]:o[2] + e])
    b1 = _sub_boxes(shape, m1, 1)[0]
    t0 = time.perf_counter()
    ocol.columns6(box(b1, "n", m1), box(b1, "xH2", m1), None, dx, par_o)
    t_col1 = time.perf_counter() - t0
    ns = nsample
    t0 = time.perf_counter()
    ostep.chem_cool_step(st0["n"][:ns], st0["T"][:ns], st0["xH2"][:ns], st0["xHp"][:ns],
                         {k: v[:ns] for k, v in rad_sample.items()}, dt, par_o)
    t_step1 = time.perf_counter() - t0
    jobs = [(box(o, "n"), box(o, "xH2"), dx, par_o) for o in boxes]
    t0 = time.perf_counter()
    ncol = sum(pool.map(_oracle_columns_box, jobs))
    t_colp = time.perf_counter() - t0
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    one = 1.0 / (t_col1 / m1 ** 3 + t_step1 / ns)
    par_v = 1.0 / (t_colp / ncol + t_step_par / nsample)
    return {"value": one, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the oracle (numpy, FP64) on the 512^3 workload, one process: vectorised six-ray columns over a "
                      f"{m1}^3 sub-box ({t_col1:.2f} s) + the step of {ns} subsample cells ({t_step1:.1f} s); "
                      f"CPU {model}",
            "parallel": {"value": par_v, "unit": "cell-updates/s", "cores": procs, "kind": "oracle",
                         "sample": f"columns over 16 sub-boxes of 96^3 ({t_colp:.2f} s) + the step of the "
                                   f"{nsample}-cell subsample in chunks of 4,096 ({t_step_par:.1f} s), "
                                   f"{procs} worker processes"}}


# VALU issue slots: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
# (full-rate FP32 and FP64 FMA; transcendental and FP64 helper instructions take longer, so this
# is an upper bound on the instructions a kernel can issue).
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def issue_roofline(kernel, t_launch, workload="grf128"):
    """VALU wave instructions per second of the kernel (counters from the committed summary over
    the measured launch time) against the chip's issue rate; None when the counters are stale."""
    c = measured_counters(kernel, workload)
    if c is None or "valu_insts" not in c:
        return None
    rate = c["valu_insts"] / t_launch
    return {"bound": "alu-issue", "kernel": kernel, "achieved": rate, "peak": VALU_ISSUE_PEAK,
            "unit": "wave64 VALU instructions/s", "frac": rate / VALU_ISSUE_PEAK, "lane_util": c["lane_util"],
            "counters": f"SQ_INSTS_VALU per launch from profiles/traffic_{workload}.txt"}


def columns_traffic(path, workload):
    """HBM bytes of one columns6 call (all its kernels) from the committed counters, or None."""
    names = ("columns_tilesum_kernel", "columns_offsets_kernel",
             "columns_tile_kernel<double>" if path == "f64" else "columns_tile_kernel<float>")
    cs = [measured_counters(k, workload) for k in names]
    return None if any(c is None for c in cs) else sum(c["bytes"] for c in cs)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "train":
        return bench_train(args)
    if args.workload in ("pts256", "pts512"):
        if args.gpus != 1:
            print(json.dumps({"error": "the library runs on one GPU; --gpus above 1 is not supported"}))
            sys.exit(2)
        return bench_pts256(args) if args.workload == "pts256" else bench_pts512(args)
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus above 1 is not supported "
                                   "(the source step is per-cell independent; see the sharding notes)"}))
        sys.exit(2)
    pool, procs = None, 0
    if not args.no_cpu:
        # the oracle's worker processes are forked before torch is imported and the GPU touched
        import multiprocessing as mp
        try:
            procs = max(1, min(16, len(os.sched_getaffinity(0))))
        except Exception:
            procs = max(1, min(16, os.cpu_count() or 1))
        pool = mp.get_context("fork").Pool(procs)
    import torch
    from paper_2210_08024_amd import ism, workloads, surrogate_train
    from oracle.census import substep_census
    from oracle.constants import Params as OParams

    state, cfg = workloads.make("grf128")
    shape = state["n"].shape
    N = state["n"].size
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ism.init(0)
    par = ism.Params(Zg=cfg["Zg"], Zd=cfg["Zg"], cr_mode=cfg["cr_mode"])
    dx = cfg["dx_pc"] * workloads.PC
    dt = cfg["dt_yr"] * workloads.YR
    init = {k: torch.from_numpy(np.ascontiguousarray(state[k]).ravel()).to(dev) for k in ("n", "T", "xH2", "xHp")}
    n = init["n"]
    T, xH2, xHp = (torch.empty_like(init[k]) for k in ("T", "xH2", "xHp"))
    sur = surrogate_train.load()
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def buffers(rd):
        rad = {k: torch.empty(N, dtype=rd, device=dev) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
        outs = {"xCp": torch.empty(N, dtype=rd, device=dev), "xCO": torch.empty(N, dtype=rd, device=dev),
                "xe": torch.empty(N, dtype=rd, device=dev), "nsub": torch.empty(N, dtype=torch.int32, device=dev),
                "status": torch.empty(N, dtype=torch.uint8, device=dev)}
        return rad, outs

    bufs = {torch.float64: buffers(torch.float64), torch.float32: buffers(torch.float32)}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def one_step(path, times=None):
        prec = ism.F64 if path == "f64" else ism.MIXED
        rad, outs = bufs[torch.float64 if path == "f64" else torch.float32]
        T.copy_(init["T"])
        xH2.copy_(init["xH2"])
        xHp.copy_(init["xHp"])
        if times is not None:
            ev[0].record(stream)
        ism.columns6(n.view(shape), xH2.view(shape), None, dx, par, prec, out={k: v.view(shape) for k, v in rad.items()})
        if times is not None:
            ev[1].record(stream)
        r = dict(rad)
        r["phi"] = None
        if path == "surrogate":
            ism.chem_cool_step_surrogate(sur, n, T, xH2, xHp, r, dt, par, out=outs, n_fallback=nfb)
        else:
            ism.chem_cool_step(n, T, xH2, xHp, r, dt, par, prec, out=outs)
        if times is not None:
            ev[2].record(stream)
            torch.cuda.synchronize()
            times["columns"].append(ev[0].elapsed_time(ev[1]) * 1e-3)
            times["step"].append(ev[1].elapsed_time(ev[2]) * 1e-3)

    def measure(path, reps=5):
        one_step(path)
        times = {"columns": [], "step": []}
        for _ in range(reps):
            one_step(path, times)
        rad, outs = bufs[torch.float64 if path == "f64" else torch.float32]
        res = {"T": T.cpu().numpy(), "xH2": xH2.cpu().numpy(), "xHp": xHp.cpu().numpy()}
        res.update({k: v.cpu().numpy() for k, v in outs.items()})
        return float(np.median(times["columns"])), float(np.median(times["step"])), res

    # timed region: K steps of the selected form
    for _ in range(args.warmup):
        one_step(args.path)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(args.path)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    paths = {}
    for p in ("f64", "mixed", "surrogate"):
        tc, ts, res = measure(p)
        nsub = res["nsub"].astype(np.int64)
        paths[p] = {"ms_per_step": (tc + ts) * 1e3, "columns_ms": tc * 1e3, "step_ms": ts * 1e3,
                    "cell_updates_per_s": N / (tc + ts), "step_only_cell_updates_per_s": N / ts, "_res": res,
                    "conservation": conservation(res, OParams(Zg=cfg["Zg"]).xCtot, OParams(Zg=cfg["Zg"]).xOtot),
                    "nsub_mean": float(nsub.mean()), "nsub_p50": float(np.percentile(nsub, 50)),
                    "nsub_p99": float(np.percentile(nsub, 99)), "nsub_max": int(nsub.max()),
                    "status_nonzero": int(((res["status"] & 0xEF) != 0).sum())}
        if p == "surrogate":
            paths[p]["fallback_fraction"] = nfb.item() / N
            paths[p]["accepted_cells"] = int(N - nfb.item())
    for p in ("mixed", "surrogate"):
        paths[p]["speedup_vs_f64"] = paths["f64"]["ms_per_step"] / paths[p]["ms_per_step"]
    paths["surrogate"]["speedup_vs_mixed"] = paths["mixed"]["ms_per_step"] / paths["surrogate"]["ms_per_step"]

    # inference kernel alone (network inputs built once, then timed forwards)
    rad32, _ = bufs[torch.float32]
    X, _ = ism.surrogate_pairs(n, init["T"], init["xH2"], init["xHp"], rad32, dt, par, ism.MIXED)
    Y = torch.empty((N, 3), dtype=torch.float32, device=dev)
    sur.forward(X, Y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        sur.forward(X, Y)
    e1.record(stream)
    torch.cuda.synchronize()
    t_mlp = e0.elapsed_time(e1) * 1e-3 / 10
    mlp_tf = MLP_FLOP_PER_CELL * N / t_mlp / 1e12

    # dominant kernel of the selected form: the persistent step kernel
    tot_sub = int(paths[args.path]["_res"]["nsub"].astype(np.int64).sum())
    arith, trans = substep_census(OParams())
    flops = float(tot_sub) * (arith + trans)
    peak = FP64_PEAK_TFLOPS if args.path == "f64" else FP32_ISSUE_PEAK_TFLOPS
    t_step = paths[args.path]["step_ms"] * 1e-3
    achieved = flops / t_step / 1e12
    ms = wall / args.steps * 1e3
    out = {
        "metric": "cell-updates/s per chem+cool step (columns6 + source step)",
        "value": N / (wall / args.steps),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "mixed": "f32+f64", "surrogate": "bf16+f32+f64"}[args.path],
        "data": "synthetic",
        "config": {"workload": "grf128: 128^3 lognormal GRF (sigma_ln 1.5, 2 pc smoothing), 4 pc cells, "
                               "P/k = 3e3 K cm^-3, Z' = 1, chi0 = 1 six-ray, xi_cr0 = 2e-16 attenuated by N_eff, "
                               "dt = 1e4 yr", "cells": N, "path": args.path},
        "roofline": {"bound": "alu", "kernel": "step_queue_kernel", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic("step_queue_kernel<double>" if args.path == "f64"
                                                 else "step_queue_kernel<float>"),
                     "traffic_algorithmic": N * (133 if args.path == "f64" else 97),
                     "work": f"{tot_sub} substeps x ({arith} flops + {trans} transcendentals counted as 1) "
                             f"per launch; census of the oracle's substep"},
        "roofline_issue": issue_roofline(
            "step_queue_kernel<double>" if args.path == "f64" else "step_queue_kernel<float>", t_step),
        "roofline_mlp": {"bound": "mfma", "kernel": "mlp_fwd_kernel", "achieved": mlp_tf, "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": mlp_tf / BF16_PEAK_TFLOPS, "ms": t_mlp * 1e3,
                         "work": f"{MLP_FLOP_PER_CELL} FLOP/cell x {N} cells per launch"},
        "paths": paths,
        "detail": {"hbm_copy_GBs_measured": copy_bandwidth(),
                   "columns_hbm_GBs_algorithmic_f64": N * 72 / (paths["f64"]["columns_ms"] * 1e-3) / 1e9,
                   "columns_hbm_GBs_algorithmic_mixed": N * 48 / (paths["mixed"]["columns_ms"] * 1e-3) / 1e9},
    }
    if not args.no_cpu:
        par_cpu = OParams(Zg=1.0, Zd=1.0, cr_mode=1)
        base, idx, ref, rad_cpu = cpu_baseline(state, cfg, args.cpu_cells, par_cpu)
        base["parallel"] = cpu_parallel(pool, procs, state, cfg, idx, rad_cpu, par_cpu)
        pool.close()
        pool.join()
        out["cpu_baseline"] = base
        xCt = OParams(Zg=1.0, Zd=1.0).xCtot
        for p in paths:
            paths[p]["error_vs_oracle"] = field_errors(paths[p]["_res"], ref, idx, xCt)
    for p in paths:
        paths[p].pop("_res")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
