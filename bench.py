"""Throughput of the GSIS kinetic hot path on one MI355X.

A step is one iteration of the whole hot path on one batch of synthetic
input.  The headline workload is the largest single-GPU configuration: the
Mach-5 flow past a 16^3-cell solid block in 96x64x64 cells with 40^3
velocity nodes on [-12, 12]^3 (source iteration, no GSIS correction), in
FP64, where a step is a kinetic pass (parameter build, boundary densities,
implicit upwind sweep, moment reduction) and the residual; the FP32 path
runs beside it with the field difference at equal passes.  The 48^3-cell,
32^3-node cavity at Kn = 0.01 with full GSIS (kinetic pass, GSIS-II
correction with 300 inner iterations, residual) and its time to
convergence, the second-order right-hand side and the 64-cavity batch are
reported as extra keys.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c3r", "c3t", "c4", "c5"],
                   help="headline workload (c5 runs only the 64-cavity batch)")
    p.add_argument("--no-gsis-extras", action="store_true",
                   help="skip the c2 GSIS step, convergence and second-order runs beside a c3/c4 headline")
    p.add_argument("--gsis", action="store_true",
                   help="GSIS steps (kinetic pass + correction + residual) on the headline workload")
    p.add_argument("--no-umesh", action="store_true",
                   help="skip the block flow on the tetrahedral spatial mesh beside a c3 headline")
    p.add_argument("--no-refined", action="store_true",
                   help="skip the passes of the block flow on the refined velocity mesh beside a c3 headline")
    p.add_argument("--dtype", default=None, choices=["fp64", "fp32"])
    p.add_argument("--macro-iters", type=int, default=None)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp32", action="store_true")
    p.add_argument("--tile", default=None, help="tx,ty,tz,block")
    p.add_argument("--no-converge", action="store_true", help="skip the time-to-convergence runs")
    p.add_argument("--no-batch", action="store_true", help="skip the 64-cavity batched run")
    p.add_argument("--batch-iters", type=int, default=50)
    p.add_argument("--precondition", default="1000,10",
                   help="macro_steps,kinetic_steps of the initial field (Alg. 1) for an extra time-to-convergence "
                        "run; 'none' skips it")
    p.add_argument("--second-order", default="1",
                   help="Venkatakrishnan K of the extra second-order-RHS runs (c2: step and convergence), "
                        "'none' to skip them, a negative K for no limiter")
    p.add_argument("--stretch", type=float, default=0.0,
                   help="non-uniform velocity grid: the same node counts clustered at the origin by a sinh map "
                        "of this strength (0: the workload's uniform grid)")
    p.add_argument("--copy-calib-mib", type=int, default=0,
                   help="after the run, copy a buffer of this many MiB three times (HBM counter calibration)")
    return p.parse_args()


# the sources the box sweep kernel is built from: its counter summary holds while they hash the same
SWEEP_SOURCES = ("paper_2310_18916_amd/csrc/k_sweep.hip", "paper_2310_18916_amd/csrc/gsis_common.h",
                 "paper_2310_18916_amd/csrc/gsis_sweep_math.h")


def sweep_traffic(dtype, tile, workload_name):
    """HBM bytes per sweep pass from the committed rocprofv3 counter summary, or
    None when that summary was taken on other kernel sources or has no entry
    for this tile."""
    import hashlib
    tag = {"c2": "c2", "c3": "c3"}.get(workload_name)
    if tag is None:
        return None
    path = os.path.join(ROOT, "profiles", f"{tag}_{dtype}_sweep_pmc.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    key = "tile " + ",".join(map(str, tile))
    if kv.get("source_sha256") != h.hexdigest() or f"{key} fetch_bytes_per_pass" not in kv:
        return None
    return float(kv[f"{key} fetch_bytes_per_pass"]) + float(kv[f"{key} write_bytes_per_pass"])


def workload(name):
    from paper_2310_18916_amd import inputs as I
    return {"c1": I.c1, "c2": I.c2, "c3": I.c3, "c3r": I.c3r, "c3t": I.c3t, "c4": I.c4}[name]()


def run_gpu(case, dtype, steps, warmup, macro_iters, tile):
    import torch
    from paper_2310_18916_amd.gsis import Solver
    s = Solver(case, dtype, tile=tile)
    s.init_maxwellian()
    tune = None
    if tile is None and case.inv_dt == 0.0 and case.mesh is None:
        tune = sorted(s.autotune(reps=2), key=lambda r: r[1])   # untimed set-up: one pass

    def step():
        s.kinetic_step(1)
        if case.gsis:
            s.gsis_correct(macro_iters)
        return s.residual()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s.profile_read(reset=True)
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eps = None
    for _ in range(steps):
        eps = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.profile(False)
    prof = s.profile_read(reset=True)
    return {"seconds": t1 - t0, "prof": prof, "eps": [float(x) for x in eps], "solver": s, "tune": tune,
            "tile": s.get_tile(), "moments": s.moments()}


def converge(case, dtype, tile, tol=1e-6, max_iters=200, pre=None, full=True):
    """GSIS iterations from the initial state until the convergence criterion of
    Sec. 5 holds, max(eps_rho, eps_u, eps_T) < tol (full=True; the iteration where
    eps_rho and eps_T alone first fell below tol, the workload's own stopping
    rule, is reported beside it), or until eps_rho, eps_T < tol (full=False);
    returns iterations, wall time and the moments at the stop.
    pre = (macro_steps, kinetic_steps): the initial field of Alg. 1 first
    (inside the timed region)."""
    import torch
    from paper_2310_18916_amd.gsis import Solver
    s = Solver(case, dtype, tile=tuple(tile))
    s.init_maxwellian()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if pre is not None:
        s.precondition(*pre)
        s.residual()            # the preconditioned state becomes the reference of the first change
    it, eps = 0, None
    rho_T = None
    while it < max_iters:
        s.kinetic_step(1)
        s.gsis_correct(case.macro_iters)
        eps = s.residual()
        it += 1
        if rho_T is None and eps[0] < tol and eps[2] < tol:
            rho_T = {"iterations": it, "seconds": time.perf_counter() - t0, "eps": [float(x) for x in eps]}
            if not full:
                break
        if max(eps) < tol:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {"criterion": "max(eps_rho, eps_u, eps_T) < tol (Sec. 5)", "iterations": it, "seconds": dt,
           "eps": [float(x) for x in eps], "converged": bool(max(eps) < tol),
           "rho_T_criterion": rho_T}
    if not full:
        res = dict(rho_T or {"iterations": it, "seconds": dt, "eps": [float(x) for x in eps]},
                   criterion="eps_rho, eps_T < tol")
    return res, s.moments()


def second_order(case, k, steps, warmup, macro, out, converge_too=True):
    """The same step with the second-order right-hand side (Sec. 3.2), FP64 and
    FP32, on the tiles the first-order runs chose; the reconstruction's
    algorithmic bytes per pass: the limiter reads f and writes phi, the source
    reads f and phi and writes the sweep's per-point term (5 elements per
    point and VDF); the sweep then reads that term and writes f."""
    import dataclasses
    c2 = dataclasses.replace(case, order=2, limiter_k=k)
    pts = c2.nfluid * c2.nvel
    nvdf = 2 if c2.species == 1 else 1
    res = {"limiter_k": k}
    for dt in ("fp64", "fp32"):
        tile = out["sweep_tile"] if dt == "fp64" else out.get("fp32", {}).get("sweep_tile", out["sweep_tile"])
        r = run_gpu(c2, dt, steps, warmup, macro, tuple(tile))
        prof = r["prof"]
        esz = 8 if dt == "fp64" else 4
        rec_ms, rec_n = prof["recon"]
        sw_ms, sw_n = prof["sweep"]
        recon_gbs = pts * nvdf * esz * 5 / (rec_ms / rec_n * 1e-3) / 1e9
        res[dt] = {"value": pts * steps / r["seconds"], "ms_per_step": r["seconds"] / steps * 1e3,
                   "sweep_tile": r["tile"], "phases_ms_per_step": {kk: v[0] / steps for kk, v in prof.items()},
                   "recon_gbs": recon_gbs,
                   "sweep_gbs": pts * nvdf * esz * 2 / (sw_ms / sw_n * 1e-3) / 1e9,
                   # the dominant phase of a second-order pass: limiter + source, per pass
                   "roofline": {"bound": "hbm", "kernel": "k_recon_limiter + k_recon_source",
                                "achieved": recon_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": recon_gbs / HBM_PEAK_GBS, "traffic": None,
                                "algorithmic_bytes": pts * nvdf * esz * 5}}
        del r
    if converge_too and case.gsis:
        c1st, m1st = converge(case, "fp64", out["sweep_tile"], full=False)
        c2nd, m2nd = converge(c2, "fp64", out["sweep_tile"], full=False)
        res["converged_fp64"] = c2nd
        res["converged_fp64_first_order"] = c1st
        res["second_vs_first_order_max_rel_diff"] = field_diff(m2nd, m1st)
    return res


def field_diff(a, b):
    """max relative difference of rho, T and u (u relative to max |u|)."""
    import numpy as np
    return {"rho": float(np.abs(a[:, 0] - b[:, 0]).max() / np.abs(b[:, 0]).max()),
            "T": float(np.abs(a[:, 4] - b[:, 4]).max() / np.abs(b[:, 4]).max()),
            "u": float(np.abs(a[:, 1:4] - b[:, 1:4]).max() / max(np.abs(b[:, 1:4]).max(), 1e-300))}


def batched(iters):
    """The 64-cavity workload as one batch (FP32 VDF, captured GSIS iteration,
    autotuned tile) against the plain path: each cavity alone in FP64."""
    import torch
    from paper_2310_18916_amd import inputs as I
    from paper_2310_18916_amd.gsis import Batch, Solver
    cases = I.c5()
    pts = sum(c.nfluid * c.nvel for c in cases)
    out = {"workload": "c5_64_cavities", "cases": len(cases), "points_per_pass": pts, "iterations": iters}
    res = {}
    for dtype in ("fp32", "fp64"):
        b = Batch(cases, dtype)
        b.init_maxwellian()
        tune = sorted(b.autotune(reps=1), key=lambda r: r[1])
        b.run(1, cases[0].macro_iters, graph=True)      # capture + first replay
        b.synchronize()
        t0 = time.perf_counter()
        b.run(iters, cases[0].macro_iters, graph=True)
        b.synchronize()
        dt = time.perf_counter() - t0
        res[dtype] = {"seconds": dt, "ms_per_iteration": dt / iters * 1e3, "value": pts * iters / dt,
                      "tile": list(b.get_tile()), "device_ms": b.last_run_ms(),
                      "eps_last_max": [float(x) for x in b.residuals()[-1].max(axis=0)],
                      "moments": [b[i].moments() for i in range(len(cases))], "tune_best": tune[0]}
        b.close()
        del b
        torch.cuda.empty_cache()
    # a closed box's steady states form a family along its total mass, which the
    # kinetic passes do not conserve on the way: the two precisions reach members
    # a path-dependent mass apart, so the fields are compared with the density
    # divided by its mean, and that mass offset is reported beside them
    def normalised(m):
        m = m.copy()
        m[:, 0] /= m[:, 0].mean()
        return m
    diffs = [field_diff(normalised(a), normalised(c)) for a, c in zip(res["fp32"]["moments"], res["fp64"]["moments"])]
    worst = {k: max(d[k] for d in diffs) for k in ("rho", "T", "u")}
    mass_offset = max(abs(a[:, 0].mean() / c[:, 0].mean() - 1.0)
                      for a, c in zip(res["fp32"]["moments"], res["fp64"]["moments"]))
    # plain path: every cavity alone, FP64, direct launches; per-iteration time measured
    # over 2 iterations after one warm iteration, scaled to the batch's iteration count
    plain = 0.0
    for c in cases:
        s = Solver(c, "fp64")
        s.init_maxwellian()
        s.kinetic_step(1)
        s.gsis_correct(c.macro_iters)
        s.residual()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            s.kinetic_step(1)
            s.gsis_correct(c.macro_iters)
            s.residual()
        torch.cuda.synchronize()
        plain += (time.perf_counter() - t0) / 2
        del s
    for k in ("fp32", "fp64"):
        res[k].pop("moments")
    out.update({"fp32": res["fp32"], "fp64": res["fp64"],
                "fp32_vs_fp64_batch_max_rel_diff": worst,
                "fp32_vs_fp64_total_mass_offset": mass_offset,
                "plain_fp64_single_ms_per_iteration": plain * 1e3,
                "speedup_fp32_batch_vs_plain_fp64": plain / (res["fp32"]["seconds"] / iters),
                "speedup_fp64_batch_vs_plain_fp64": plain / (res["fp64"]["seconds"] / iters)})
    return out


def cpu_baseline(case, budget_s=12.0):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: the same
    velocity grid and gas on a 16^3-cell cavity, kinetic passes repeated until about
    budget_s seconds of CPU work have run."""
    from oracle.oracle import Oracle, build
    from paper_2310_18916_amd import inputs as I
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        build()
    if case.solid is None:
        n = 16
        sample = I.cavity(n, case.nv[0], case.Kn, lid=case.bcs[5].u[0], vmax=case.vmax[0], omega=case.omega)
        shape = f"a {n}^3-cell cavity"
    else:
        sample = I.block_flow(16, 12, 12, ((6, 10), (4, 8), (4, 8)), case.nv[0], case.vmax[0], case.Kn,
                              species=case.species, omega=case.omega)
        shape = "a 16x12x12-cell block flow"
    o = Oracle(sample)
    o.init_maxwellian()
    passes = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or passes >= 50:
            break
    pts = sample.ncell * sample.nvel * passes
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": pts / dt, "unit": "cell-updates/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": f"{passes} FP64 kinetic passes of the oracle on {shape} x {sample.nv[0]}^3 nodes "
                      f"(same velocity grid, gas and Kn), {dt:.2f} s"}


def copy_calibration(mib):
    """A plain device-to-device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"bytes_read": n * 8, "bytes_written": n * 8, "copies": 3}


def hbm_rates(gib=4):
    """Achievable HBM rates of plain streaming on this GPU (torch's own kernels on
    gib-GiB FP64 buffers, best of three): read (sum), write (fill), copy."""
    import torch
    n = gib * (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        ms = []
        for _ in range(3):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return min(ms) * 1e-3

    nbytes = n * 8
    out = {"read_gbs": nbytes / best(lambda: a.sum()) / 1e9,
           "write_gbs": nbytes / best(lambda: b.fill_(2.0)) / 1e9,
           "copy_gbs": 2 * nbytes / best(lambda: b.copy_(a)) / 1e9,
           "buffer_gib": gib, "how": "torch sum / fill_ / copy_, best of 3, device events"}
    del a, b
    torch.cuda.empty_cache()
    return out


def gsis_extras(a, steps, warmup):
    """The cavity with full GSIS (48^3 cells, 32^3 nodes, Kn = 0.01): the step
    (kinetic pass + GSIS-II correction with 300 inner iterations + residual) in
    FP64 and FP32, the time to convergence under the criterion of Sec. 5 in
    both precisions (and with the initial field of Alg. 1), and the
    second-order right-hand side."""
    case = workload("c2")
    macro = case.macro_iters
    pts = case.nfluid * case.nvel
    out = {"workload": case.name, "cells": case.ncell, "nodes": case.nvel, "Kn": case.Kn, "macro_iters": macro,
           "step": "kinetic pass + gsis_correct + residual"}
    for dt in ("fp64", "fp32"):
        r = run_gpu(case, dt, steps, warmup, macro, None)
        out[dt] = {"value": pts * steps / r["seconds"], "ms_per_step": r["seconds"] / steps * 1e3,
                   "sweep_tile": r["tile"], "phases_ms_per_step": {k: v[0] / steps for k, v in r["prof"].items()},
                   "kinetic_only_updates_per_s": pts * steps / ((r["prof"]["prep"][0] + r["prof"]["sweep"][0]
                                                                 + r["prof"]["moments"][0]) * 1e-3)}
        del r
    out["speedup_fp32_vs_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    # the Grad-13 wall flux of the correction (gsis_set_wall_flux): its step
    g13 = dataclasses.replace(case, wall_flux=1)
    r = run_gpu(g13, "fp64", steps, warmup, macro, out["fp64"]["sweep_tile"])
    out["fp64_g13_wall_flux"] = {"value": pts * steps / r["seconds"], "ms_per_step": r["seconds"] / steps * 1e3,
                                 "phases_ms_per_step": {k: v[0] / steps for k, v in r["prof"].items()}}
    del r
    if not a.no_converge:
        c64, m64 = converge(case, "fp64", out["fp64"]["sweep_tile"], max_iters=100)
        c32, m32 = converge(case, "fp32", out["fp32"]["sweep_tile"], max_iters=100)
        out["converged"] = {"tol": 1e-6, "fp64": c64, "fp32": c32,
                            "fp32_vs_fp64_max_rel_diff": field_diff(m32, m64),
                            "speedup_fp32_vs_fp64_time_to_converge": c64["seconds"] / c32["seconds"]}
        cg, mg = converge(g13, "fp64", out["fp64"]["sweep_tile"], max_iters=100)
        out["converged"]["fp64_g13_wall_flux"] = cg
        out["converged"]["g13_vs_maxwell_wall_flux_max_rel_diff"] = field_diff(mg, m64)
        if a.precondition != "none":
            pre = tuple(int(x) for x in a.precondition.split(","))
            cp, mp = converge(case, "fp64", out["fp64"]["sweep_tile"], pre=pre, max_iters=100)
            cp["initial_field"] = {"euler_macro_steps": pre[0], "kinetic_steps": pre[1]}
            out["converged"]["fp64_preconditioned"] = cp
            out["converged"]["preconditioned_vs_plain_max_rel_diff"] = field_diff(mp, m64)
    if a.second_order != "none":
        out["second_order"] = second_order(case, float(a.second_order), steps, warmup, macro,
                                           {"sweep_tile": out["fp64"]["sweep_tile"],
                                            "fp32": {"sweep_tile": out["fp32"]["sweep_tile"]}},
                                           converge_too=not a.no_converge)
    return out


def refined_mesh(steps, warmup):
    """Kinetic passes of the c3 block flow on the refined velocity mesh of
    Sec. 3.1 (a node list: per-node tables and direct-sum kernels), FP64 and
    FP32, with the phase times and the sweep's and moments' HBM rates."""
    import torch
    case = workload("c3r")
    pts = case.nfluid * case.nvel
    res = {"workload": case.name, "nodes": case.nvel, "cells": case.ncell}
    for dtype in ("fp64", "fp32"):
        r = run_gpu(case, dtype, steps, warmup, 0, None)
        esz = 8 if dtype == "fp64" else 4
        prof = r["prof"]
        sweep_ms, n = prof["sweep"]
        mom_ms, _ = prof["moments"]
        res[dtype] = {"value": pts * steps / r["seconds"], "ms_per_pass": r["seconds"] / steps * 1e3,
                      "phases_ms_per_pass": {k: v[0] / steps for k, v in prof.items() if v[1]},
                      "sweep_gbs": pts * esz / (sweep_ms / n * 1e-3) / 1e9,
                      "moments_gbs": pts * esz / (mom_ms / n * 1e-3) / 1e9, "sweep_tile": r["tile"]}
        del r
        torch.cuda.empty_cache()
    return res


def unstructured_mesh(steps, warmup):
    """Kinetic passes of the block flow on an unstructured spatial mesh (291,840
    tetrahedra, the refined velocity mesh of c3r): the level-by-level sweep
    over velocity classes, FP64 and FP32, with the phase times and the
    sweep's and moments' HBM rates (algorithmic bytes: every point written
    once by the sweep and read once by the moment kernel); then the GSIS step
    on the same mesh."""
    import torch
    case = workload("c3t")
    pts = case.nfluid * case.nvel
    res = {"workload": case.name, "cells": case.mesh.ncell, "faces": case.mesh.nface, "nodes": case.nvel}
    for dtype in ("fp64", "fp32"):
        r = run_gpu(case, dtype, steps, warmup, 0, None)
        esz = 8 if dtype == "fp64" else 4
        prof = r["prof"]
        sweep_ms, n = prof["sweep"]
        mom_ms, _ = prof["moments"]
        res[dtype] = {"value": pts * steps / r["seconds"], "ms_per_pass": r["seconds"] / steps * 1e3,
                      "phases_ms_per_pass": {k: v[0] / steps for k, v in prof.items() if v[1]},
                      "sweep_gbs": pts * esz / (sweep_ms / n * 1e-3) / 1e9,
                      "moments_gbs": pts * esz / (mom_ms / n * 1e-3) / 1e9}
        del r
        torch.cuda.empty_cache()
    # the GSIS step on the same mesh: kinetic pass + GSIS-II correction (300 inner
    # iterations on the tetrahedra) + residual
    import dataclasses
    gcase = dataclasses.replace(case, gsis=True, macro_iters=300)
    res["gsis"] = {"macro_iters": 300, "step": "kinetic pass + gsis_correct + residual"}
    for dtype in ("fp64", "fp32"):
        r = run_gpu(gcase, dtype, max(2, steps // 2), 1, 300, None)
        ns = max(2, steps // 2)
        res["gsis"][dtype] = {"value": pts * ns / r["seconds"], "ms_per_step": r["seconds"] / ns * 1e3,
                              "phases_ms_per_step": {k: v[0] / ns for k, v in r["prof"].items() if v[1]},
                              "eps": r["eps"]}
        del r
        torch.cuda.empty_cache()
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the path is single-GPU by design",
              file=sys.stderr)
        sys.exit(2)
    if a.workload == "c5":
        print(json.dumps({"batched": batched(a.batch_iters)}), flush=True)
        return
    case = workload(a.workload)
    if a.gsis:
        import dataclasses
        case = dataclasses.replace(case, gsis=True)
    if a.stretch > 0:
        from paper_2310_18916_amd import inputs as I
        case = I.with_nodes(case, [I.stretched_nodes(case.nv[k], max(-case.vmin[k], case.vmax[k]), a.stretch)
                                   for k in range(3)])
        case.name += f"_stretch{a.stretch:g}"
    dtype = a.dtype or "fp64"
    macro = a.macro_iters if a.macro_iters is not None else case.macro_iters
    tile = tuple(int(x) for x in a.tile.split(",")) if a.tile else None
    r = run_gpu(case, dtype, a.steps, a.warmup, macro, tile)
    pts = case.nfluid * case.nvel
    steps = a.steps
    seconds = r["seconds"]
    value = pts * steps / seconds
    prof = r["prof"]
    esz = 8 if dtype == "fp64" else 4
    sweep_ms, sweep_n = prof["sweep"]
    mom_ms, mom_n = prof["moments"]
    nvdf = 2 if case.species == 1 else 1                                # the diatomic gas carries f0 and f1
    sweep_bytes = pts * nvdf * esz * (2 if case.inv_dt != 0 else 1)   # write f^{n+1/2} (+ read f^n if 1/dt != 0)
    mom_bytes = pts * nvdf * esz                                       # read f^{n+1/2}
    sweep_gbs = sweep_bytes / (sweep_ms / sweep_n * 1e-3) / 1e9
    mom_gbs = mom_bytes / (mom_ms / mom_n * 1e-3) / 1e9
    dominant = "sweep" if sweep_ms >= mom_ms else "moments"
    ach = sweep_gbs if dominant == "sweep" else mom_gbs
    traffic = sweep_traffic(dtype, r["tile"], a.workload) if dominant == "sweep" else None
    head_moments = r["moments"]
    tune_top = [[list(c), round(ms, 4)] for c, ms in (r["tune"] or [])[:6]]
    eps_head, tile_head = r["eps"], r["tile"]
    del r
    import torch
    torch.cuda.empty_cache()
    out = {
        "metric": "phase-space cell-updates/s (cells x velocities); FP32 vs FP64 at equal accuracy",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": seconds / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": case.ncell, "fluid_cells": case.nfluid, "nodes": case.nvel,
                   "Kn": case.Kn, "gsis": case.gsis, "macro_iters": macro if case.gsis else 0,
                   "step": "kinetic pass + gsis_correct + residual" if case.gsis else "kinetic pass + residual"},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": dominant,
                     "per": "one sweep pass (all hyperplane launches)",
                     "algorithmic_bytes": sweep_bytes if dominant == "sweep" else mom_bytes},
        "phases_ms_per_step": {k: v[0] / steps for k, v in prof.items()},
        "kinetic_only_updates_per_s": pts * steps / ((prof["prep"][0] + sweep_ms + mom_ms) * 1e-3),
        "kinetic_pass_gbs": (sweep_bytes + mom_bytes) / ((sweep_ms + mom_ms) / sweep_n * 1e-3) / 1e9,
        "sweep_gbs": sweep_gbs,
        "moments_gbs": mom_gbs,
        "final_eps": eps_head,
        "sweep_tile": tile_head,
        "autotune_top": tune_top,
    }
    rates = hbm_rates()
    # the sweep's algorithmic bytes are writes, the moments' reads
    ceiling = rates["write_gbs"] if dominant == "sweep" else rates["read_gbs"]
    out["roofline"]["measured_ceiling"] = ceiling
    out["roofline"]["frac_of_measured"] = ach / ceiling
    out["hbm_measured"] = rates
    if not a.no_fp32:
        other = "fp32" if dtype == "fp64" else "fp64"
        ro = run_gpu(case, other, steps, a.warmup, macro, None)
        vo = pts * steps / ro["seconds"]
        fluid = ~case.solid_mask().astype(bool)
        out[other] = {"value": vo, "speedup_fp32_vs_fp64": vo / value if other == "fp32" else value / vo,
                      "sweep_tile": ro["tile"], "phases_ms_per_step": {k: v[0] / steps for k, v in ro["prof"].items()},
                      "autotune_top": [[list(c), round(ms, 4)] for c, ms in (ro["tune"] or [])[:6]],
                      # the two precisions after the same passes from the same initial state
                      "max_rel_diff_vs_" + dtype: field_diff(ro["moments"][fluid], head_moments[fluid])}
        del ro
        torch.cuda.empty_cache()
    if a.workload == "c2":
        if a.second_order != "none":
            out["second_order"] = second_order(case, float(a.second_order), steps, a.warmup, macro, out,
                                               converge_too=not a.no_converge)
        if not a.no_converge and case.gsis and dtype == "fp64":
            c64, m64 = converge(case, "fp64", out["sweep_tile"], max_iters=100)
            c32, m32 = converge(case, "fp32", out["fp32"]["sweep_tile"] if "fp32" in out else out["sweep_tile"],
                                max_iters=100)
            out["converged"] = {"tol": 1e-6, "fp64": c64, "fp32": c32,
                                "fp32_vs_fp64_max_rel_diff": field_diff(m32, m64),
                                "speedup_fp32_vs_fp64_time_to_converge": c64["seconds"] / c32["seconds"]}
    elif not a.no_gsis_extras:
        out["gsis_c2"] = gsis_extras(a, steps, a.warmup)
    if a.workload == "c3" and not a.no_refined:
        out["refined_velocity_mesh"] = refined_mesh(max(3, steps // 4), 2)
    if a.workload == "c3" and not a.no_umesh:
        out["unstructured_mesh"] = unstructured_mesh(max(3, steps // 4), 2)
    if not a.no_batch:
        out["batched"] = batched(a.batch_iters)
    if a.copy_calib_mib > 0:
        out["copy_calibration"] = copy_calibration(a.copy_calib_mib)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
