#!/usr/bin/env python3
"""Benchmark of the MORE-Stress hot path on one MI355X.

Default (--mode c5): one step = the global stage of one 200x200 TSV array
(40,000 cells of 15x15x50 um, each meshed 20x20x40 hexes with a Cu via of
5 um and a 0.5 um SiO2 liner, cubic face interpolation, n = 168,
dT = -250 K) whose six outer faces carry a seeded smooth displacement field
(8 Fourier modes, 0.1 um): reduced assembly, lifting, Chronopoulos-Gear PCG
with FP64 refinement, and every element's centroid von Mises stress
reconstructed into a device buffer.  The record is the plain FP64 path; the
mixed-precision path (FP32 PCG, FP64 refinement, BF16-split reconstruction)
is measured the same way and reported beside it with its von Mises error
against the FP64 path.  The one-shot local stage (cell assembly, basis,
projection) runs before the clock, as the paper reports it apart from the
global stage.  The same line carries the oracle's throughput on the host
(the global stage of 20x20 sub-arrays of the same cell with a field of the
same kind) with the GPU's error against it on that sub-array, and two extra
legs: a batch of 128 independent 16x16 arrays (16x16x32 cells) and a Poisson
request stream served with continuous batching.

--mode batch: the batch of 128 16x16 arrays alone, with the oracle's global
stage on the first arrays (at least 10 s) and every one of those arrays
compared with the GPU's result (u and von Mises).

--mode single --workload c3: one 64x64 array with 10% dummy cells;
--workload bump: a 100x100 micro-bump layer (40x40x20 um blocks, 16^3 hexes,
a SnAg column with Cu pads in underfill, both faces clamped, 5% empty sites);
--workload hex120: a 64x64 TSV array on a 120-degree lattice (rhombic blocks
of 15 um spacing, 16x14x32 hexes, 10% dummy blocks, bottom clamped).

--mode plane: the paper's evaluation grid (100 x 100 points on each cell's
mid-height plane) for the 16x16 array, FP64 and mixed, with the normalised
MAE of the mixed field against the FP64 one.

--mode convergence: Table 3's sweep of interpolation orders (2..6)^3 on a
20x20 array: local- and global-stage times, iterations, self-convergence.

--mode serve: a Poisson stream of requests (mean 200 /s; N ~ U{4..48},
pitch ~ U{10,15,20} um, dT ~ U[-300,-150] K, 10% dummy cells) served with
continuous batching in mixed precision; reports TSV-cells/s and p50/p99 of
completion minus arrival.  --rates runs the stream at several rates.

Prints one JSON line.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TSV-cells/s (solve+stress recon) at ≤1e-3 rel err vs FP64; p50/p99 latency"
TIME_EVERY = 16
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
# Vector passes over the reduced DoFs per PCG iteration that the method
# itself needs (read the preconditioned residual, x, r, p, s and the
# diagonal; write x, r, p, s), as counted for the roofline of the update.
PCG_PASSES = 10


def quiet_gc():
    """Collect now and move every live object out of the collector's reach,
    so that no full collection (tens of ms with torch loaded) lands inside a
    timed region."""
    gc.collect()
    gc.freeze()


def per_iteration_work(kernel, mos, n, n_cells, n_dofs, mixed):
    """Algorithmic work of one PCG iteration of one problem in a kernel
    class: the cell GEMM's 2 n^2 flops per cell, or the update's vector
    passes over the problem's reduced DoFs.  The cell-major copies of u and
    K_r u that the GEMM and the update exchange are a cost of the two-launch
    design, not of the method, and are not counted."""
    w = 4 if mixed else 8
    if kernel == mos.MOS_K_CELL_GEMM:
        return 2.0 * n * n * n_cells
    if kernel == mos.MOS_K_PCG_UPDATE:
        return float(PCG_PASSES * n_dofs * w)
    raise ValueError(kernel)


KERNEL_INFO = {  # kernel id -> (name, bound, unit, note)
    1: ("k_bgemm", "mfma", "TFLOP/s", "2 n^2 flops per cell and iteration (K_r GEMM of the PCG matvec)"),
    2: ("k_cg_scalars", "latency", "us", "per-problem fixed-order reductions and CG step"),
    3: ("k_cgstep", "hbm", "GB/s", f"{PCG_PASSES} vector passes x reduced DoFs x word size per iteration "
                                   "(the method's vectors only; the cell-layout copies are not counted)"),
    4: ("k_recon", "mfma", "TFLOP/s", "2*6*n_elem*n flops per cell (stress GEMM; the BF16 form issues 3x "
                                      "these on MFMA for its hi/lo split)"),
}
KERNELS = (1, 2, 3, 4)


def kernel_source(path, name):
    """Text of the definition of kernel (or device function) `name` in a HIP
    source file: from the template line (if any) before its `__global__` /
    `__device__` line to the closing brace of its body; None when it is not
    found."""
    try:
        lines = open(path).read().split("\n")
    except OSError:
        return None
    for i, ln in enumerate(lines):
        if ("__global__" in ln or "__device__" in ln) and f" {name}(" in ln:
            start = i - 1 if i > 0 and lines[i - 1].lstrip().startswith("template") else i
            text = "\n".join(lines[start:])
            depth, seen = 0, False
            for j, ch in enumerate(text):
                if ch == "{":
                    depth += 1
                    seen = True
                elif ch == "}":
                    depth -= 1
                    if seen and depth == 0:
                        return text[:j + 1]
            return None
    return None


def recorded_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or
    None when no record matches or the kernel's definition has changed since
    the counters were taken (SHA-256 of its source text)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    for e in rec.get("entries", []):
        if (e["kernel"], e["workload"], e["precision"]) != (kernel, workload, precision):
            continue
        funs, want = e.get("functions"), e.get("functions_sha256")
        if not funs or not want:
            return None
        texts = [kernel_source(os.path.join(ROOT, e.get("source", "")), f) for f in funs]
        if any(t is None for t in texts):
            return None
        if hashlib.sha256("\n".join(texts).encode()).hexdigest() != want:
            return None
        return e.get("traffic_bytes_per_launch")
    return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def oracle_solve(case, oroms, field_dofs=None):
    """The oracle's global stage of one array: abstract mesh, constraints
    (clamped faces, or the case's field on every outer face at the oracle's
    own node coordinates), assembly + lifting + direct solve, centroid
    stress.  Returns (u, von Mises)."""
    from oracle import array as oarray
    from oracle import fem as ofem
    import numpy as np
    sp = case.specs[0]
    mesh = oarray.AbstractMesh(case.nx_cells, case.ny_cells, sp.interp, sp.pitch_x, sp.pitch_y, sp.height)
    pd, pv = (), ()
    if case.field is not None:
        outer = np.nonzero(mesh.outer_node_mask())[0]
        pd = (3 * outer[:, None] + np.arange(3)[None, :]).ravel()
        pv = case.field(mesh.coords[outer]).ravel()
    dofs, vals = oarray.constrained_dofs(mesh, case.clamp_bottom, case.clamp_top, pd, pv)
    u = oarray.solve_mor(mesh, case.cell_type, oroms, case.delta_T, dofs, vals)
    vm = ofem.von_mises(oarray.reconstruct(mesh, case.cell_type, oroms, u, case.delta_T))
    return u, vm


def cpu_baseline(cases, min_seconds=10.0):
    """The oracle's global stage on consecutive arrays of the workload, on
    the host cores, until at least `min_seconds` of timed work (or all of
    them), then the first array once more with its BLAS pools held to one
    thread (`value_1_thread`); the host's CPU model is recorded beside.
    Each distinct cell's local stage is run first and not timed.  Returns
    the record and the oracle's (u, von Mises) of every array solved."""
    from oracle import mor as omor
    roms = {}
    elapsed, cells, refs = 0.0, 0, []
    for case in cases:
        for s in case.specs:
            if s not in roms:
                roms[s] = omor.local_stage(s)
        t0 = time.perf_counter()
        refs.append(oracle_solve(case, [roms[s] for s in case.specs]))
        elapsed += time.perf_counter() - t0
        cells += case.n_cells
        if elapsed >= min_seconds:
            break
    c0 = cases[0]
    bc = "its field on all outer faces" if c0.field is not None else "bottom clamped"
    out = {"value": round(cells / elapsed, 3), "unit": "TSV-cells/s", "cores": int(blas_threads()),
           "kind": "oracle",
           "sample": f"full global stage of {len(refs)} {c0.nx_cells}x{c0.ny_cells} arrays of the workload's "
                     f"cell ({cells} cells, {elapsed:.2f} s; {bc}): assembly, lifting, direct solve, centroid "
                     f"stress of every element; host has {os.cpu_count()} logical CPUs",
           "cpu_model": cpu_model()}
    # The first array once more with the BLAS pools held to one thread.
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle_solve(c0, [roms[s] for s in c0.specs])
            out["value_1_thread"] = round(c0.n_cells / (time.perf_counter() - t0), 3)
    except ImportError:
        pass
    return out, refs


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def rel_max(a, b):
    import numpy as np
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return float(np.abs(a - b).max() / np.abs(b).max())


def outer_prescribed(mos, ctx, rom, case, np):
    """Prescribed reduced DoFs for a displacement field on all six outer
    faces, evaluated at the library's own reduced-node coordinates."""
    coords, _, _, _ = mos.mos_array_layout(ctx, case.nx_cells, case.ny_cells, rom)
    sp = case.specs[0]
    L = np.array([case.nx_cells * sp.pitch_x, case.ny_cells * sp.pitch_y, sp.height])
    tol = 1e-9 * L
    outer = np.nonzero(np.any((np.abs(coords) <= tol) | (np.abs(coords - L) <= tol), axis=1))[0]
    vals = case.field(coords[outer])
    dofs = (3 * outer[:, None] + np.arange(3)[None, :]).ravel()
    return dofs.astype(np.int64), vals.ravel()


def kernel_totals(mos, ctx, run):
    """Every launch of each kernel class over one run, timed with events:
    (launches, total ms) per class."""
    out = {}
    for k in KERNELS:
        mos.mos_timing_start(ctx, k, 1)
        run()
        launches, ms, _ = mos.mos_timing_stop(ctx)
        out[k] = (launches, ms)
    return out


def class_rooflines(mos, totals, n, n_cells, n_elem, n_dofs, iters, mixed, runs=1):
    """Achieved rate of each kernel class over `runs` runs (from the totals
    pass, every launch timed) against its bound."""
    out = {}
    w_gemm = per_iteration_work(mos.MOS_K_CELL_GEMM, mos, n, n_cells, n_dofs, mixed) * iters
    w_upd = per_iteration_work(mos.MOS_K_PCG_UPDATE, mos, n, n_cells, n_dofs, mixed) * iters
    w_rec = 2.0 * 6 * n_elem * n * n_cells
    for k, work, peak, scale in ((mos.MOS_K_CELL_GEMM, w_gemm, PEAK_FP32_TFLOPS if mixed else PEAK_FP64_TFLOPS,
                                  1e12),
                                 (mos.MOS_K_PCG_UPDATE, w_upd, PEAK_HBM_GBS, 1e9),
                                 (mos.MOS_K_RECON, w_rec, PEAK_BF16_TFLOPS if mixed else PEAK_FP64_TFLOPS, 1e12)):
        launches, ms = totals[k]
        if ms <= 0:
            continue
        a = work * runs / (ms / 1e3) / scale
        out[KERNEL_INFO[k][0]] = {"ms_per_solve": round(ms / runs, 4), "launches_per_solve": launches / runs,
                                  "achieved": round(a, 3), "unit": KERNEL_INFO[k][2], "peak": peak,
                                  "frac": round(a / peak, 4)}
    return out


def solve_leg(args, mos, torch, np, ctx, roms, case, prec, kw, workload_key):
    """One array through an engine sized for it, in one precision: warm-up,
    a pass that times every launch of each kernel class, then the timed
    solves (each: submit, PCG to convergence, reconstruction of every
    element's von Mises stress) with one launch in TIME_EVERY of the dominant
    kernel carrying HIP events on the library's stream.  Returns the record
    and the last von Mises field (host, float64)."""
    mixed = prec == "mixed"
    n = roms[0].query(mos.MOS_Q_N)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    coords, _, _, _ = mos.mos_array_layout(ctx, case.nx_cells, case.ny_cells, roms[0])
    n_dofs = 3 * coords.shape[0]
    n_dofs_pad = -(-n_dofs // 768) * 768
    n_cells = case.n_cells
    w = 4 if mixed else 8
    budget = int((n_dofs_pad * 160 + n_cells * 16 * 176 * (2 * w + 24)) * 1.3) + (256 << 20)
    eng = mos.Engine(ctx, roms, mixed=mixed, device_bytes=budget, gemm=args.cell_gemm, precond=args.precond)
    if args.gemm_split is not None:
        eng.option(mos.MOS_OPT_GEMM_SPLIT, args.gemm_split)
    vm = torch.empty((n_cells, n_elem), dtype=torch.float32 if mixed else torch.float64, device="cuda")

    def run():
        tk = eng.submit(case.nx_cells, case.ny_cells, case.cell_type, case.delta_T, vm=vm, **kw)
        while tk not in eng.progress(args.chunk):
            pass
        return eng.result(tk)

    for _ in range(args.warmup):
        run()
    totals = kernel_totals(mos, ctx, run)
    dominant = max((k for k in totals if k != mos.MOS_K_PCG_SCALARS), key=lambda k: totals[k][1])
    every = 1 if dominant == mos.MOS_K_RECON else TIME_EVERY
    mos.mos_timing_start(ctx, dominant, every)
    quiet_gc()
    torch.cuda.synchronize()
    res, lat = [], []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        res.append(run())
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t1) / args.steps
    launches, k_ms, seen = mos.mos_timing_stop(ctx)
    st, rel, iters, sweeps = res[-1]
    # Condition estimate of the preconditioned reduced system, from the
    # first sweep's PCG coefficients of one more (untimed) solve.
    tk = eng.submit(case.nx_cells, case.ny_cells, case.cell_type, case.delta_T, vm=vm, **kw)
    while tk not in eng.progress(args.chunk):
        pass
    kappa, kappa_steps = eng.cond_estimate(tk)
    eng.result(tk)
    if st != 0:
        raise RuntimeError(f"{prec} solve failed with status {st}: {eng.last_error}")
    name, bound, unit, note = KERNEL_INFO[dominant]
    if dominant == mos.MOS_K_RECON:
        work = 2.0 * 6 * n_elem * n * n_cells * args.steps
        peak = PEAK_BF16_TFLOPS if mixed else PEAK_FP64_TFLOPS
    else:
        work = per_iteration_work(dominant, mos, n, n_cells, n_dofs, mixed) * sum(r[2] for r in res)
        peak = (PEAK_FP32_TFLOPS if mixed else PEAK_FP64_TFLOPS) if bound == "mfma" else PEAK_HBM_GBS
    avg_s = k_ms / max(launches, 1) / 1e3
    achieved = work / max(seen, 1) / avg_s / (1e12 if unit == "TFLOP/s" else 1e9)
    rec = {
        "value": round(n_cells / wall, 2), "ms_per_solve": round(wall * 1e3, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "pcg_iters": iters, "refinement_sweeps": sweeps, "rel_residual": rel,
        "cond_estimate": {"kappa": round(kappa, 3), "lanczos_steps": kappa_steps},
        "roofline": {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 5), "traffic": recorded_traffic(name, workload_key, prec),
                     "traffic_unit": "bytes/launch", "kernel": name, "avg_launch_us": round(avg_s * 1e6, 3),
                     "timed_launches": int(launches), "launches": int(seen), "timed_every": every,
                     "work_per_launch": round(work / max(seen, 1), 1), "work_note": note,
                     "kernel_share_of_solve": round(avg_s * seen / args.steps * 1e3 / (wall * 1e3), 4)},
        "kernel_classes": class_rooflines(mos, totals, n, n_cells, n_elem, n_dofs, iters, mixed),
        "kernels_ms_per_solve": {KERNEL_INFO[k][0]: round(v[1], 4) for k, v in totals.items()},
    }
    out_vm = vm.double().cpu().numpy()
    eng.close()
    del vm
    torch.cuda.empty_cache()
    return rec, out_vm, n_dofs


def subarray_check(mos, torch, np, ctx, roms, case, ref):
    """The GPU's FP64 and mixed results on a sub-array the oracle solved:
    u (FP64) and von Mises (both) against the oracle's."""
    u_ref, vm_ref = ref
    kw = dict(clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top)
    if case.field is not None:
        kw["prescribed_dofs"], kw["prescribed_values"] = outer_prescribed(mos, ctx, roms[0], case, np)
    out = {"array": f"{case.nx_cells}x{case.ny_cells}"}
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    for prec in ("fp64", "mixed"):
        mixed = prec == "mixed"
        sol = mos.mos_solve_array(ctx, roms, case.nx_cells, case.ny_cells, case.cell_type, case.delta_T,
                                  mixed=mixed, **kw)
        vm = torch.empty((case.n_cells, n_elem), dtype=torch.float32 if mixed else torch.float64, device="cuda")
        mos.mos_reconstruct(ctx, sol, vm=vm)
        u, res, it = mos.mos_get_solution(sol)
        out[prec] = {"rel_err_u_vs_oracle": rel_max(u, u_ref),
                     "rel_err_vm_vs_oracle": rel_max(vm.double().cpu().numpy(), vm_ref),
                     "normalized_mae_vm_vs_oracle": float(np.abs(vm.double().cpu().numpy() - vm_ref).mean()
                                                          / np.abs(vm_ref).max()),
                     "pcg_iters": it, "rel_residual": res}
        del sol, vm
    return out


def c5_mode(args, mos, torch, np, W):
    """The 200x200 array with a liner and a Fourier field on all outer faces:
    FP64 record, mixed beside it, the oracle on 20x20 sub-arrays of the same
    cell, and the batch and served legs."""
    case = W.case_c5(args.seed)
    ctx = mos.Context(0)
    torch.cuda.reset_peak_memory_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in case.specs]
    torch.cuda.synchronize()
    local_ms = (time.perf_counter() - t0) * 1e3
    n = roms[0].query(mos.MOS_Q_N)
    kw = dict(clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top)
    pd, pv = outer_prescribed(mos, ctx, roms[0], case, np)
    # The boundary data is resident in HBM before the clock starts (the
    # library reads the device list at set-up).
    kw["prescribed_dofs"], kw["prescribed_values"] = torch.as_tensor(pd, device="cuda"), torch.as_tensor(
        pv, device="cuda")
    paths, vms = {}, {}
    for prec in ("fp64", "mixed"):
        paths[prec], vms[prec], n_dofs = solve_leg(args, mos, torch, np, ctx, roms, case, prec, kw,
                                                   "single_c5")
        print(f"[bench] c5 {prec}: {paths[prec]['ms_per_solve']} ms per solve", file=sys.stderr, flush=True)
    # The same FP64 solve with the boundary list handed over in host memory
    # (copied to the device at every submission): the PCIe-inclusive rate.
    hargs = argparse.Namespace(**vars(args))
    hargs.steps, hargs.warmup = 3, 1
    hkw = dict(kw, prescribed_dofs=pd, prescribed_values=pv)
    hrec, _, _ = solve_leg(hargs, mos, torch, np, ctx, roms, case, "fp64", hkw, "single_c5")
    host_list = {"value": hrec["value"], "ms_per_solve": hrec["ms_per_solve"], "prescribed_entries": int(pd.size),
                 "bytes_per_solve": int(pd.size * 16)}
    err = rel_max(vms["mixed"], vms["fp64"])
    nmae = float(np.abs(vms["mixed"] - vms["fp64"]).mean() / np.abs(vms["fp64"]).max())
    peak_gb = round(torch.cuda.max_memory_allocated() / 2**30, 3)
    cpu, check = None, None
    if not args.no_cpu_baseline:
        subs = [W.case_c5(args.seed + k, n=args.sub) for k in range(8)]
        cpu, refs = cpu_baseline(subs)
        check = subarray_check(mos, torch, np, ctx, roms, subs[0], refs[0])
        print(f"[bench] cpu baseline {cpu['value']} cells/s; sub-array check {json.dumps(check)}",
              file=sys.stderr, flush=True)
    sp = case.specs[0]
    head = paths["fp64"]
    mx = paths["mixed"]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "TSV-cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "200x200 TSV array (C5): 20x20x40-hex cells with a 0.5 um SiO2 liner, cubic faces, "
                               "seeded Fourier displacement field on all six outer faces",
                   "array": f"{case.nx_cells}x{case.ny_cells}", "cells": case.n_cells,
                   "cell_um": [sp.pitch_x, sp.pitch_y, sp.height], "cell_mesh": list(sp.mesh),
                   "tsv_diameter_um": sp.tsv_diameter, "liner_um": sp.liner_thickness, "interp": list(sp.interp),
                   "n": n, "reduced_dofs": int(n_dofs), "delta_T": case.delta_T,
                   "bc": "Fourier field (8 modes, 0.1 um) on all outer faces", "seed": args.seed,
                   "precision": "fp64 (record); mixed beside it", "pcg_chunk": args.chunk,
                   "preconditioner": "jacobi" if args.precond == 0 else "jacobi + aggregate coarse correction"},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "latency_is": "per array: submission to completion of solve + reconstruction",
        "pcg_iters": head["pcg_iters"],
        "refinement_sweeps": head["refinement_sweeps"],
        "rel_residual": head["rel_residual"],
        "cond_estimate": head["cond_estimate"],
        "roofline": head["roofline"],
        "kernel_classes": head["kernel_classes"],
        "kernels_ms_per_solve": head["kernels_ms_per_solve"],
        "cpu_baseline": cpu,
        "mixed_side_by_side": {
            "value": mx["value"], "unit": "TSV-cells/s", "ms_per_solve": mx["ms_per_solve"],
            "dtype": "f32+bf16+f64", "p50_ms": mx["p50_ms"], "p99_ms": mx["p99_ms"], "pcg_iters": mx["pcg_iters"],
            "refinement_sweeps": mx["refinement_sweeps"], "rel_residual": mx["rel_residual"],
            "cond_estimate": mx["cond_estimate"], "max_rel_err_vm_vs_fp64": err, "normalized_mae_vm_vs_fp64": nmae,
            "roofline": mx["roofline"], "kernel_classes": mx["kernel_classes"],
            "kernels_ms_per_solve": mx["kernels_ms_per_solve"]},
        "accuracy_vs_oracle": check,
        "host_list_fp64": host_list,
        "local_stage_ms": round(local_ms, 1),
        "peak_hbm_gb": peak_gb,
    }
    del roms
    gc.collect()
    torch.cuda.empty_cache()
    if not args.no_legs:
        bargs = argparse.Namespace(**vars(args))
        bargs.no_single = True
        b64, _ = batch_leg(bargs, mos, torch, np, W, "fp64")
        bmx, _ = batch_leg(bargs, mos, torch, np, W, "mixed")
        out["batch_c2"] = {p: {k: r[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "pcg_iters_mean",
                                                  "cond_estimate", "dtype", "roofline")}
                           | {"config": r["config"]["workload"]}
                           for p, r in (("fp64", b64), ("mixed", bmx))}
        print(f"[bench] batch legs {b64['value']} / {bmx['value']} cells/s", file=sys.stderr, flush=True)
        sv = serve_leg(args, mos, torch, np, W, args.rate)
        out["served_c4"] = {k: sv[k] for k in ("value", "p50_ms", "p99_ms", "offered_cells_per_s", "rate_hz",
                                               "requests", "max_rel_err_vm_vs_fp64_sampled", "dtype",
                                               "busy_fraction")}
        print(f"[bench] served {sv['value']} cells/s p50 {sv['p50_ms']} p99 {sv['p99_ms']}", file=sys.stderr,
              flush=True)
    print(json.dumps(out))


def batch_leg(args, mos, torch, np, W, precision, with_cpu=False):
    """One precision of the batch workload (B independent 16x16 arrays);
    returns its JSON record and the oracle's results of the arrays it
    solved for the CPU baseline (when it ran)."""
    B = args.batch
    mixed = precision == "mixed"
    cases = [W.case_c2(args.seed + i) for i in range(B)]
    diam = [4.0, 5.0, 6.0]
    spec0 = cases[0].specs[0]
    gc.collect()
    torch.cuda.empty_cache()
    ctx = mos.Context(0)
    torch.cuda.reset_peak_memory_stats()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, W.CellSpec(tsv_diameter=d))) for d in diam]
    torch.cuda.synchronize()
    local_ms = (time.perf_counter() - t0) * 1e3 / len(diam)
    n = roms[0].query(mos.MOS_Q_N)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    n_cells = cases[0].n_cells
    X = 16 * 3 + 1
    n_nodes = X * X * 4 - n_cells * 2 * 2 * 2
    n_dofs = 3 * n_nodes
    n_dofs_pad = -(-n_dofs // 768) * 768
    eng = mos.Engine(ctx, roms, mixed=mixed, device_bytes=int(B * (n_dofs_pad * 140 + n_cells * 16 * 176 * 34)
                                                             * 1.3) + (64 << 20), gemm=args.cell_gemm,
                     precond=args.precond, graph=args.graph)
    precond = 1 if args.precond is None else args.precond
    if args.gemm_split is not None:
        eng.option(mos.MOS_OPT_GEMM_SPLIT, args.gemm_split)
    vms = [torch.empty((n_cells, n_elem), dtype=torch.float32 if mixed else torch.float64, device="cuda")
           for _ in range(B)]
    us = [torch.empty((n_dofs,), dtype=torch.float64, device="cuda") for _ in range(B)]
    types = [np.full(n_cells, diam.index(c.specs[0].tsv_diameter), dtype=np.uint8) for c in cases]
    host = {"submit_s": 0.0, "progress_calls": 0, "steps": 0}

    def step(record=None, kappa=None):
        tks = {}
        ts = time.perf_counter()
        for i, c in enumerate(cases):
            tks[eng.submit(c.nx_cells, c.ny_cells, types[i], c.delta_T, vm=vms[i], u=us[i])] = i
        if record is not None:
            host["submit_s"] += time.perf_counter() - ts
            host["steps"] += 1
        left = set(tks)
        info = {}
        while left:
            if record is not None:
                host["progress_calls"] += 1
            for tk in eng.progress(args.chunk):
                if kappa is not None:
                    kappa.append(eng.cond_estimate(tk))
                st, rel, it, sw = eng.result(tk)
                if st != 0:
                    raise RuntimeError(f"array {tks[tk]} failed with status {st}: {eng.last_error}")
                info[tks[tk]] = (time.perf_counter() - ts, it, sw, rel)
                left.discard(tk)
        if record is not None:
            record.append(info)
        return info

    for _ in range(args.warmup):
        step()
    totals = kernel_totals(mos, ctx, step)
    dominant = max((k for k in totals if k != mos.MOS_K_PCG_SCALARS), key=lambda k: totals[k][1])

    # Timed region: one launch in TIME_EVERY of the dominant kernel carries
    # dispatch-stamped HIP events on its stream (stamping every launch adds
    # host work to the step being measured).  With graph replay of the
    # iteration chunks the timed region runs unsampled (a sampled kernel
    # keeps its chunk out of the graph) and the kernel is sampled in a
    # separate pass of the same steps afterwards.
    # Reconstruction launches once per cell type and step: every one is sampled.
    every = 1 if dominant == mos.MOS_K_RECON else TIME_EVERY
    if not args.graph:
        mos.mos_timing_start(ctx, dominant, every)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    recs = []
    quiet_gc()
    torch.cuda.synchronize()
    ev[0].record(stream)
    for s in range(args.steps):
        step(recs)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    sampled = recs
    if args.graph:
        sampled = []
        mos.mos_timing_start(ctx, dominant, every)
        for s in range(max(2, args.steps // 2)):
            step(sampled)
        torch.cuda.synchronize()
    launches, k_ms, seen = mos.mos_timing_stop(ctx)
    total_ms = ev[0].elapsed_time(ev[-1])
    ms_per_step = total_ms / args.steps
    lat = np.array([v[0] * 1e3 for r in recs for v in r.values()])
    iters = [v[1] for r in recs for v in r.values()]
    sweeps = [v[2] for r in recs for v in r.values()]
    iters_sampled = [v[1] for r in sampled for v in r.values()]

    name, bound, unit, note = KERNEL_INFO[dominant]
    if dominant == mos.MOS_K_RECON:
        work = 2.0 * 6 * n_elem * n * n_cells * B * len(sampled)
        peak = PEAK_BF16_TFLOPS if mixed else PEAK_FP64_TFLOPS
    else:
        work = per_iteration_work(dominant, mos, n, n_cells, n_dofs, mixed) * sum(iters_sampled)
        if bound == "mfma":
            peak = PEAK_FP32_TFLOPS if mixed else PEAK_FP64_TFLOPS
        else:
            peak = PEAK_HBM_GBS
    avg_s = k_ms / max(launches, 1) / 1e3
    work_per_launch = work / max(seen, 1)
    achieved = work_per_launch / avg_s / (1e12 if unit == "TFLOP/s" else 1e9)
    roofline = {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 5),
                "traffic": recorded_traffic(name, f"batch{B}_c2", precision), "traffic_unit": "bytes/launch",
                "kernel": name,
                "avg_launch_us": round(avg_s * 1e6, 3), "timed_launches": int(launches), "launches": int(seen),
                "timed_every": every, "work_per_launch": round(work_per_launch, 1), "work_note": note,
                "kernel_share_of_step": round(avg_s * seen / len(sampled) * 1e3 / ms_per_step, 4),
                "kernels_ms_per_step": {KERNEL_INFO[k][0]: round(v[1], 4) for k, v in totals.items()}}

    # Single-array latency (batch of one), for reference.
    single = []
    for s in range(0 if args.no_single else 3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tk = eng.submit(16, 16, types[0], cases[0].delta_T, vm=vms[0], u=us[0])
        while tk not in eng.progress(args.chunk):
            pass
        eng.result(tk)
        torch.cuda.synchronize()
        single.append((time.perf_counter() - t1) * 1e3)

    # Condition estimates of the batch's arrays, from one more (untimed) step.
    kappa = []
    step(kappa=kappa)
    kv = np.array([k for k, _ in kappa])
    cond = {"median": round(float(np.median(kv)), 3), "min": round(float(kv.min()), 3),
            "max": round(float(kv.max()), 3), "lanczos_steps_median": int(np.median([n for _, n in kappa]))}

    cpu, refs, check = None, None, None
    if with_cpu and not args.no_cpu_baseline:
        cpu, refs = cpu_baseline(cases)
        step()
        torch.cuda.synchronize()
        eu = [rel_max(us[i].cpu().numpy(), r[0]) for i, r in enumerate(refs)]
        ev_ = [rel_max(vms[i].double().cpu().numpy(), r[1]) for i, r in enumerate(refs)]
        nm = [float(np.abs(vms[i].double().cpu().numpy() - r[1]).mean() / np.abs(r[1]).max())
              for i, r in enumerate(refs)]
        check = {"arrays_compared": len(refs), "max_rel_err_u": max(eu), "max_rel_err_vm": max(ev_),
                 "max_normalized_mae_vm": max(nm)}

    out = {
        "metric": METRIC,
        "value": round(B * n_cells / (ms_per_step / 1e3), 2),
        "unit": "TSV-cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {B} independent 16x16 TSV arrays (16x16x32-hex cells, one C2-shaped run "
                               f"per seed)",
                   "arrays_per_step": B, "cells_per_step": B * n_cells, "array": "16x16",
                   "cell_um": [spec0.pitch_x, spec0.pitch_y, spec0.height], "cell_mesh": list(spec0.mesh),
                   "tsv_diameter_um": "per array from {4,5,6}", "interp": list(spec0.interp), "n": n,
                   "reduced_dofs_per_array": int(n_dofs), "delta_T": -250.0, "bc": "bottom clamped",
                   "precision": precision, "seed": args.seed, "pcg_chunk": args.chunk,
                   "gemm_split": args.gemm_split if args.gemm_split is not None else "tuned",
                   "preconditioner": "jacobi" if precond == 0 else "jacobi + aggregate coarse correction",
                   "chunk_launch": "graph replay" if args.graph else "direct"},
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "step_ms": [round(ev[s].elapsed_time(ev[s + 1]), 3) for s in range(args.steps)],
        "latency_is": "per array, submission to completion of solve + reconstruction",
        "single_array_ms": round(float(np.median(single)), 4) if single else None,
        "pcg_iters_mean": round(float(np.mean(iters)), 1),
        "refinement_sweeps_mean": round(float(np.mean(sweeps)), 2),
        "cond_estimate": cond,
        "local_stage_ms_per_cell_type": round(local_ms, 2),
        "host": {"submit_ms_per_step": round(host["submit_s"] * 1e3 / max(host["steps"], 1), 3),
                 "progress_calls_per_step": round(host["progress_calls"] / max(host["steps"], 1), 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": check,
        "peak_hbm_gb": round(torch.cuda.max_memory_allocated() / 2**30, 3),
    }
    eng.close()
    return out, refs


def batch_mode(args, mos, torch, np, W):
    """The batch workload in one precision, or (default) the plain FP64 path
    as the record with the mixed-precision path measured beside it; every
    array the oracle solved for the CPU baseline is compared with the GPU's
    result in both precisions."""
    if args.precision is not None:
        out, _ = batch_leg(args, mos, torch, np, W, args.precision, with_cpu=True)
        print(json.dumps(out))
        return
    out, refs = batch_leg(args, mos, torch, np, W, "fp64", with_cpu=True)
    mx, _ = batch_leg(args, mos, torch, np, W, "mixed", with_cpu=refs is not None)
    r = mx["roofline"] or {}
    out["mixed_side_by_side"] = {
        "value": mx["value"], "unit": mx["unit"], "ms_per_step": mx["ms_per_step"], "dtype": mx["dtype"],
        "p50_ms": mx["p50_ms"], "p99_ms": mx["p99_ms"], "single_array_ms": mx["single_array_ms"],
        "pcg_iters_mean": mx["pcg_iters_mean"], "refinement_sweeps_mean": mx["refinement_sweeps_mean"],
        "cond_estimate": mx["cond_estimate"], "accuracy_vs_oracle": mx["accuracy_vs_oracle"],
        "peak_hbm_gb": mx["peak_hbm_gb"],
        "roofline": {k: r.get(k) for k in ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                                           "avg_launch_us", "kernels_ms_per_step")},
    }
    print(json.dumps(out))


def single_mode(args, mos, torch, np, W):
    """One large array (C3- or C5-shaped, a 64x64 array on a 120-degree
    lattice, or a 100x100 micro-bump layer) through the engine, plain FP64 and mixed precision side by side, each
    with its dominant kernel's roofline."""
    if args.workload == "c5":
        args.no_legs = True
        return c5_mode(args, mos, torch, np, W)
    bump = args.workload == "bump"
    case = {"bump": W.case_bump, "hex120": W.case_hex}.get(args.workload, W.case_c3)(args.seed)
    key = "single_" + args.workload
    ctx = mos.Context(0)
    torch.cuda.reset_peak_memory_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in case.specs]
    torch.cuda.synchronize()
    local_ms = (time.perf_counter() - t0) * 1e3
    n = roms[0].query(mos.MOS_Q_N)
    kw = dict(clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top)
    paths, vms = {}, {}
    for prec in ("fp64", "mixed"):
        paths[prec], vms[prec], n_dofs = solve_leg(args, mos, torch, np, ctx, roms, case, prec, kw, key)
    err = rel_max(vms["mixed"], vms["fp64"])
    sp = case.specs[0]
    head = paths["fp64"]
    out = {
        "metric": METRIC, "value": head["value"], "unit": "bump-cells/s" if bump else "TSV-cells/s", "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": case.name, "array": f"{case.nx_cells}x{case.ny_cells}", "cells": case.n_cells,
                   "cell_um": [sp.pitch_x, sp.pitch_y, sp.height], "skew": sp.skew, "cell_mesh": list(sp.mesh),
                   "interp": list(sp.interp), "n": n, "reduced_dofs": int(n_dofs),
                   "dummy_cells": int((case.cell_type != 0).sum()),
                   "bc": "bottom and top clamped" if case.clamp_top else "bottom clamped",
                   "delta_T": case.delta_T, "seed": args.seed, "precision": "fp64 (record); mixed beside it"},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "pcg_iters": head["pcg_iters"],
        "refinement_sweeps": head["refinement_sweeps"], "rel_residual": head["rel_residual"],
        "cond_estimate": head["cond_estimate"],
        "roofline": head["roofline"], "kernel_classes": head["kernel_classes"],
        "mixed_side_by_side": paths["mixed"], "max_rel_err_vm_mixed_vs_fp64": err,
        "local_stage_ms_total": round(local_ms, 1),
        "peak_hbm_gb": round(torch.cuda.max_memory_allocated() / 2**30, 3),
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def plane_mode(args, mos, torch, np, W):
    """The paper's evaluation (Sec. 5.1): von Mises on a g x g grid (default
    100 x 100) of points on every cell's mid-height plane, for the 16x16 array
    of 16x16x32 cells with cubic faces, from an FP64 and a mixed-precision
    solution.  Times the plane reconstruction (one GEMM per cell type over a
    stress basis built at the sample points) and reports the paper's error
    measure, the normalised MAE, of the mixed field against the FP64 one."""
    case = W.case_c2(args.seed)
    g = args.grid
    ctx = mos.Context(0)
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in case.specs]
    n = roms[0].query(mos.MOS_Q_N)
    n_cells = case.n_cells
    paths, fields = {}, {}
    for prec in ("fp64", "mixed"):
        mixed = prec == "mixed"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol = mos.mos_solve_array(ctx, roms, case.nx_cells, case.ny_cells, case.cell_type, case.delta_T,
                                  clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top, mixed=mixed)
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t0) * 1e3
        vm = torch.empty((n_cells, g * g), dtype=torch.float32 if mixed else torch.float64, device="cuda")
        t0 = time.perf_counter()
        mos.mos_reconstruct_plane(ctx, sol, g, vm)       # first call also builds the plane basis
        first_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            mos.mos_reconstruct_plane(ctx, sol, g, vm)
        mos.mos_timing_start(ctx, mos.MOS_K_RECON, 1)
        quiet_gc()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            mos.mos_reconstruct_plane(ctx, sol, g, vm)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t1) / args.steps
        launches, k_ms, seen = mos.mos_timing_stop(ctx)
        work = 2.0 * 6 * g * g * n * n_cells * args.steps        # algorithmic flops of the timed calls
        kern_s = k_ms / 1e3 / max(launches, 1) * max(seen, 1)      # kernel time of the timed calls
        peak = PEAK_BF16_TFLOPS if mixed else PEAK_FP64_TFLOPS
        achieved = work / kern_s / 1e12
        paths[prec] = {
            "cells_per_s": round(n_cells / wall, 1), "points_per_s": round(n_cells * g * g / wall, 1),
            "ms_per_call": round(wall * 1e3, 4), "first_call_ms_with_basis": round(first_ms, 2),
            "solve_ms": round(solve_ms, 2), "pcg_iters": sol.query(mos.MOS_Q_ITERS),
            "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(achieved / peak, 5), "kernel": "k_recon (plane basis)",
                         "avg_launch_us": round(k_ms * 1e3 / max(launches, 1), 3),
                         "launches_per_call": round(seen / args.steps, 2),
                         "work_note": "2 * 6 g^2 n flops per cell"},
        }
        fields[prec] = vm.double().cpu().numpy()
        del sol, vm
    ref, mx = fields["fp64"], fields["mixed"]
    sp = case.specs[0]
    out = {
        "mode": "plane",
        "metric": "evaluation-plane cells/s (von Mises on the mid-height grid)",
        "value": paths["fp64"]["cells_per_s"],
        "unit": "TSV-cells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": paths["fp64"]["ms_per_call"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "array": f"{case.nx_cells}x{case.ny_cells}", "cells": n_cells,
                   "cell_mesh": list(sp.mesh), "interp": list(sp.interp), "n": n, "grid": [g, g],
                   "points_per_cell": g * g, "plane": "z = h/2", "delta_T": case.delta_T, "seed": args.seed},
        "fp64": paths["fp64"],
        "mixed": paths["mixed"],
        "normalized_mae_mixed_vs_fp64": float(np.mean(np.abs(mx - ref)) / np.abs(ref).max()),
        "max_rel_err_mixed_vs_fp64": float(np.abs(mx - ref).max() / np.abs(ref).max()),
        "max_vm_mpa": float(ref.max()),
    }
    print(json.dumps(out))


def convergence_mode(args, mos, torch, np, W):
    """The interpolation-order sweep of Table 3 on one GPU: a 20x20 array of
    15x15x50 um cells (16x16x32 hexes, d = 5 um, dT = -250 K, bottom clamped)
    at orders (2,2,2) ... (6,6,6).  Per order: the one-shot local stage
    (mos_build_cell + mos_reduce), the global stage of one array call
    (mos_solve_array + centroid reconstruction) in FP64 and mixed precision,
    PCG iterations, and the normalised MAE of the plane von Mises (100 x 100
    per cell) against the (6,6,6) FP64 field -- a self-convergence measure,
    since the paper's reference (a commercial solver on its own mesh) is not
    available."""
    import dataclasses
    base = W.CellSpec()
    N = 20
    cell_type = np.zeros(N * N, dtype=np.uint8)
    g = args.grid
    ctx = mos.Context(0)
    rows, planes = [], {}
    for k in (2, 3, 4, 5, 6):
        spec = dataclasses.replace(base, interp=(k, k, k))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
        torch.cuda.synchronize()
        local_ms = (time.perf_counter() - t0) * 1e3
        n = rom.query(mos.MOS_Q_N)
        n_elem = rom.query(mos.MOS_Q_CELL_ELEMS)
        row = {"interp": [k, k, k], "n": n, "local_stage_ms": round(local_ms, 2)}
        for prec in ("fp64", "mixed"):
            mixed = prec == "mixed"
            dt = torch.float32 if mixed else torch.float64
            vm = torch.empty((N * N, n_elem), dtype=dt, device="cuda")

            def run():
                sol = mos.mos_solve_array(ctx, [rom], N, N, cell_type, -250.0, clamp_bottom=True, mixed=mixed)
                mos.mos_reconstruct(ctx, sol, vm=vm)
                return sol

            for _ in range(args.warmup):
                run()
            quiet_gc()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                sol = run()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t1) / args.steps
            vp = torch.empty((N * N, g * g), dtype=dt, device="cuda")
            mos.mos_reconstruct_plane(ctx, sol, g, vp)
            planes[(k, prec)] = vp.double().cpu().numpy()
            row[prec] = {"global_stage_ms": round(wall * 1e3, 3), "cells_per_s": round(N * N / wall, 1),
                         "pcg_iters": sol.query(mos.MOS_Q_ITERS), "refinement_sweeps": sol.query(mos.MOS_Q_REFINES)}
            del sol, vm, vp
        rows.append(row)
        del rom
        torch.cuda.empty_cache()
    ref = planes[(6, "fp64")]
    for row in rows:
        k = row["interp"][0]
        for prec in ("fp64", "mixed"):
            v = planes[(k, prec)]
            row[prec]["plane_nmae_vs_order6_fp64"] = float(np.mean(np.abs(v - ref)) / np.abs(ref).max())
    head = rows[2]["fp64"]
    out = {
        "mode": "convergence",
        "metric": METRIC,
        "value": head["cells_per_s"],
        "unit": "TSV-cells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["global_stage_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "20x20 TSV array, 16x16x32 hex cells, interpolation orders 2..6",
                   "array": f"{N}x{N}", "cell_um": [base.pitch_x, base.pitch_y, base.height],
                   "cell_mesh": list(base.mesh), "tsv_diameter_um": base.tsv_diameter, "delta_T": -250.0,
                   "bc": "bottom clamped", "plane_grid": [g, g], "value_is": "order (4,4,4), FP64"},
        "orders": rows,
    }
    print(json.dumps(out))


def calib_mode(args, torch):
    """A plain device copy of known size (1 GiB read, 1 GiB written per
    launch): the reference that scales the FETCH_SIZE / WRITE_SIZE counters
    of the profiled kernels into HBM bytes, and the sustained copy and fill
    rates (event-timed after a warm-up copy) that the bandwidth-bound
    kernels are compared with."""
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    rates = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 8 * n), ("fill", lambda: y.fill_(2.0), 4 * n)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        rates[name] = round(nbytes * args.steps / (e0.elapsed_time(e1) * 1e6), 1)
    print(json.dumps({"mode": "calib", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "launches": args.steps + 1, "copy_GBps": rates["copy"], "fill_GBps": rates["fill"]}))




def serve_leg(args, mos, torch, np, W, rate, n_requests=None, ctx=None, roms=None):
    """A Poisson stream of requests at `rate` per second served by one mixed
    engine with continuous batching: requests are submitted as they arrive,
    admitted by the device budget, advanced together, and stamped complete
    when the engine reports them (after their reconstruction has finished on
    the device).  Returns the record."""
    n_requests = n_requests or args.requests
    reqs = W.request_stream(seed=args.seed, n_requests=n_requests, rate_hz=rate)
    pitches = [10.0, 15.0, 20.0]
    ctx = ctx or mos.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if roms is None:
        specs = []
        for p in pitches:
            s = W.CellSpec(pitch_x=p, pitch_y=p)
            specs += [s, s.dummy()]
        roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in specs]
    torch.cuda.synchronize()
    local_ms = (time.perf_counter() - t0) * 1e3
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    eng = mos.Engine(ctx, roms, mixed=True, device_bytes=int(args.budget_gb * (1 << 30)), precond=args.precond)
    cases = [W.request_case(r) for r in reqs]
    types = []
    for r, c in zip(reqs, cases):
        base = 2 * pitches.index(r.pitch)
        types.append((base + c.cell_type).astype(np.uint8))
    out_vm = {}
    arrival, done_t, cells = {}, {}, 0
    i = 0
    tickets = {}
    busy = 0.0
    quiet_gc()
    torch.cuda.synchronize()
    start = time.perf_counter()
    while len(done_t) < len(reqs):
        now = time.perf_counter() - start
        while i < len(reqs) and reqs[i].arrival_s <= now:
            c = cases[i]
            vm = torch.empty((c.n_cells, n_elem), dtype=torch.float32, device="cuda")
            tk = eng.submit(c.nx_cells, c.ny_cells, types[i], c.delta_T, vm=vm)
            tickets[tk] = i
            out_vm[i] = vm
            arrival[i] = reqs[i].arrival_s
            i += 1
        st = eng.stats()
        if st["active"] == 0 and st["queued"] == 0:
            if i < len(reqs):
                time.sleep(max(0.0, min(reqs[i].arrival_s - (time.perf_counter() - start), 0.002)))
            continue
        tb = time.perf_counter()
        for tk in eng.progress(args.chunk):
            k = tickets.pop(tk)
            status, rel, it, sw = eng.result(tk)
            if status != 0:
                raise RuntimeError(f"request {k} failed with status {status}: {eng.last_error}")
            done_t[k] = time.perf_counter() - start
            cells += cases[k].n_cells
            if k % 50 != 0:
                out_vm.pop(k, None)
        busy += time.perf_counter() - tb
    lat = np.array([(done_t[k] - arrival[k]) * 1e3 for k in range(len(reqs))])
    span = max(done_t.values()) - reqs[0].arrival_s
    eng.close()
    # Accuracy: sampled requests against the FP64 GPU path.
    errs = []
    for k in sorted(out_vm)[:4]:
        c = cases[k]
        base = 2 * pitches.index(reqs[k].pitch)
        sub = [roms[base], roms[base + 1]]
        sol = mos.mos_solve_array(ctx, sub, c.nx_cells, c.ny_cells, c.cell_type, c.delta_T)
        ref = torch.empty((c.n_cells, n_elem), dtype=torch.float64, device="cuda")
        mos.mos_reconstruct(ctx, sol, vm=ref)
        r = ref.cpu().numpy()
        errs.append(float(np.abs(out_vm[k].double().cpu().numpy() - r).max() / np.abs(r).max()))
    return {
        "value": round(cells / span, 2), "unit": "TSV-cells/s", "dtype": "f32+bf16+f64",
        "rate_hz": rate, "requests": len(reqs),
        "offered_cells_per_s": round(sum(c.n_cells for c in cases) / (reqs[-1].arrival_s + 1e-9), 1),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "span_s": round(span, 3),
        "busy_fraction": round(busy / span, 3),
        "local_stage_ms_total": round(local_ms, 1),
        "max_rel_err_vm_vs_fp64_sampled": max(errs) if errs else None,
    }


def serve_mode(args, mos, torch, np, W):
    """The request stream at 200 /s (or each rate of --rates, sharing the
    cached bases), TSV-cells/s and p50/p99 of completion minus arrival."""
    ctx = mos.Context(0)
    torch.cuda.reset_peak_memory_stats()
    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    pitches = [10.0, 15.0, 20.0]
    specs = []
    for p in pitches:
        s = W.CellSpec(pitch_x=p, pitch_y=p)
        specs += [s, s.dummy()]
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in specs]
    rows = []
    for r in rates:
        rows.append(serve_leg(args, mos, torch, np, W, r, ctx=ctx, roms=roms))
        print(f"[serve] rate {r:g}/s: {rows[-1]['value']} cells/s p50 {rows[-1]['p50_ms']} p99 {rows[-1]['p99_ms']} "
              f"busy {rows[-1]['busy_fraction']}", file=sys.stderr, flush=True)
    head = rows[0]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "TSV-cells/s",
        "n_gpus": 1,
        "steps": head["requests"],
        "warmup": 0,
        "ms_per_step": round(head["span_s"] * 1e3 / head["requests"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16+f64",
        "data": "synthetic",
        "config": {"workload": "Poisson request stream, continuous batching (C4-shaped)",
                   "requests": args.requests, "rate_hz": rates[0], "N": "U{4..48}", "pitch_um": pitches,
                   "delta_T": "U[-300,-150]", "dummy_fraction": 0.1, "cell_mesh": [16, 16, 32],
                   "interp": [4, 4, 4], "precision": "mixed", "budget_gb": args.budget_gb,
                   "pcg_chunk": args.chunk,
                   "preconditioner": "jacobi" if args.precond == 0 else "jacobi + aggregate coarse correction"},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "rates": rows,
        "peak_hbm_gb": round(torch.cuda.max_memory_allocated() / 2**30, 3),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=["c5", "batch", "serve", "single", "calib", "plane", "convergence"],
                    default="c5")
    ap.add_argument("--grid", type=int, default=100, help="plane mode: sample points per cell along x and y")
    ap.add_argument("--workload", choices=["c3", "c5", "bump", "hex120"], default="c3",
                    help="single mode: C3, C5, a 100x100 micro-bump layer, or a 64x64 120-degree array")
    ap.add_argument("--sub", type=int, default=20, help="c5 mode: sub-array size the oracle solves on the host")
    ap.add_argument("--no-legs", action="store_true", help="c5 mode: skip the batch and served legs")
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="batch mode: run this precision only (default: the FP64 record with the "
                         "mixed-precision path measured beside it)")
    ap.add_argument("--gemm-split", type=int, default=None,
                    help="fixed slot blocks per wave of the cell GEMM (default: tuned online)")
    ap.add_argument("--cell-gemm", type=int, choices=[0, 1, 2, 3], default=None,
                    help="cell GEMM variant (0 rows with the operand path tuned, 1 tiles, 2 K_r-stationary rows, "
                         "3 rows with the operand tile in LDS; "
                         "default: the engine's)")
    ap.add_argument("--precond", type=int, choices=[0, 1], default=None,
                    help="PCG preconditioner (0 Jacobi, 1 Jacobi plus the aggregate coarse correction; "
                         "default: the engine's)")
    ap.add_argument("--no-single", action="store_true",
                    help="batch mode: skip the single-array latency pass (for counter runs that average over "
                         "every launch of the process)")
    ap.add_argument("--chunk", type=int, default=16)
    ap.add_argument("--graph", type=int, choices=[0, 1], default=0,
                    help="batch mode: replay each chunk of PCG iterations from a captured HIP graph (1) or launch "
                         "its kernels directly (0, default)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0, help="served leg: mean request rate per second")
    ap.add_argument("--rates", type=str, default=None, help="serve mode: comma-separated request rates")
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the hot path runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2411_12690_amd import mos
    torch.cuda.set_device(0)
    if args.mode == "calib":
        calib_mode(args, torch)
    elif args.mode == "c5":
        c5_mode(args, mos, torch, np, W)
    elif args.mode == "batch":
        batch_mode(args, mos, torch, np, W)
    elif args.mode == "single":
        single_mode(args, mos, torch, np, W)
    elif args.mode == "plane":
        plane_mode(args, mos, torch, np, W)
    elif args.mode == "convergence":
        convergence_mode(args, mos, torch, np, W)
    else:
        serve_mode(args, mos, torch, np, W)


if __name__ == "__main__":
    main()
