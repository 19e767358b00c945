"""Benchmark: matrix-free Q2 viscous operator (vmult) throughput on one MI355X.

Workload (the 64^3 sinker configuration): unit cube, 64^3 uniform cells,
Q2 velocity (6,440,067 dofs), 8 seeded sinkers (centre seed 2), viscosity
contrast 1e4, operator applied to a seeded uniform[-1, 1] vector (seed 42).
One step = 100 FP32 operator applications (the configuration's 100
repetitions); `value` = velocity dofs processed per second over the timed
steps, in GDoF/s.  Also reported beside it (not part of `value`): the FP64
operator, one FP32/FP64 V-cycle, and the Stokes solve to 1e-8 with the FP32
and the FP64 V-cycle inside FP64 FGMRES.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-solve] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

REPS = 100                      # operator applications per step
PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector (packed FMA), published
PEAK_HBM_GBS = 8000.0
# Algorithmic work of the cell kernel per cell (sum factorisation as built,
# counting an FMA as 2 flops): 810 (interpolation) + 972 (gradients) + 297
# (stress) + 1215 (transposed gradients) + 729 (transposed interpolation)
FLOP_PER_CELL = 4023


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-solve", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--level", type=int, default=6, help="cells per edge = 2^level (default 6: 64^3)")
    p.add_argument("--solve-workload", choices=["adaptive32p2", "uniform128p1"], default=None,
                   help="instead of the operator benchmark, compare the Stokes solves on this workload")
    p.add_argument("--max-iter", type=int, default=3000, help="FGMRES iteration cap of --solve-workload")
    p.add_argument("--variants", default=None,
                   help="solves of --solve-workload, comma separated from fp64, fp32, fp32_learned, fp32_gmres, "
                        "fp32_idr2, fp64_idr2, fp32_diag (default: all on adaptive32p2; on uniform128p1 all but "
                        "fp32_idr2, which stalls near 1e-5 there, and fp32_diag, which needs ~4x the iterations)")
    p.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                   help="turn the counter_collection.csv files of a FETCH_SIZE and a WRITE_SIZE pass over "
                        "--counter-probe into profiles/vmult_counters_sinker64.json (no GPU needed)")
    p.add_argument("--counter-probe", action="store_true",
                   help="only launch the operator (mfgmg_vmult, FP32: brick + halo kernels) and a plain copy of "
                        "known size, 20 times each, for hardware-counter runs")
    return p.parse_args()


COPY_BYTES = 256 << 20          # the calibration copy: 256 MiB read + 256 MiB written


def counter_probe(s, L, x32, y32):
    """Kernels for a rocprofv3 --pmc pass: 20 operator applications (FP32) and
    20 copies of COPY_BYTES, so that FETCH_SIZE / WRITE_SIZE per dispatch of
    the operator's kernels can be scaled by what the same counters read for a
    copy of known size."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=x32.device)
    b = torch.empty_like(a)
    for _ in range(20):
        s.vmult(L, x32, y32)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counter_probe": True, "copy_bytes": COPY_BYTES, "vmult_launches": 20}), flush=True)


def cpu_baseline(level, centres, dr, seconds=12.0):
    """The CPU oracle's cellwise FP64 operator on the same workload: applied
    repeatedly to the same vector until about `seconds` have elapsed."""
    from oracle import mesh as om, operators as ops
    from paper_1907_06696_amd import inputs
    lev, ijk = om.uniform_leaves(level)
    m = om.LevelMesh(lev, ijk, level + 1)
    X = ops.gauss_points_of_cells(m).reshape(-1, 3)
    mu = ops.harmonic_cell_viscosity(inputs.sinker_mu(X, centres, dr).reshape(-1, 27))
    A = ops.CellwiseA(m, mu)
    x = inputs.uniform_vector(m.n_u, 42)
    A.matvec(x)
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < seconds or reps < 2:
        A.matvec(x)
        reps += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": m.n_u * reps / dt / 1e9, "unit": "GDoF/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} FP64 applications of the oracle's cellwise operator (numpy BLAS, "
                      f"{threads} threads) on the full {1 << level}^3 mesh, {dt:.1f} s"}


WEIGHTS = os.path.join(ROOT, "paper_1907_06696_amd", "data", "mlp_sinker32.npz")
COUNTERS = os.path.join(ROOT, "profiles", "vmult_counters_sinker64.json")
KERNEL_SOURCES = ("brick_kernel.h", "cell_kernel.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1907_06696_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(level):
    """HBM bytes per operator application from the committed FETCH_SIZE /
    WRITE_SIZE passes (scaled by the calibration copy), or None when the
    counters were taken on other kernel sources or another workload."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_hash") != kernel_source_hash() or c.get("level") != level:
        return None
    return {"bytes": int(c["bytes_per_application"]), "source": os.path.relpath(COUNTERS, ROOT)}


# outer-solver variants of Sec. 3.4 (V-cycle precision, options): plain GMRES
# and IDR(2) with the fixed Chebyshev Schur map (IDR also with the FP64
# V-cycle: its short recurrences can stall on the FP32 one), FGMRES with the
# block-diagonal P_D;
# vectors = FP64 block vectors the Krylov method keeps (FGMRES 2m + 1, GMRES
# m + 2, IDR(s) 3s + 2, each plus b, x, r, w)
SOLVER_VARIANTS = {
    "fp32_gmres": ("fp32", dict(krylov="gmres", schur="cheb")),
    "fp32_idr2": ("fp32", dict(krylov="idr", schur="cheb", idr_s=2)),
    "fp64_idr2": ("fp64", dict(krylov="idr", schur="cheb", idr_s=2)),
    "fp32_diag": ("fp32", dict(block="diagonal")),
}


def krylov_vectors(kw, restart):
    k = kw.get("krylov", "fgmres")
    if k == "gmres":
        return restart + 2 + 4
    if k == "idr":
        return 3 * kw.get("idr_s", 2) + 2 + 4
    return 2 * restart + 1 + 4


def solve_compare(s, qp, centres, max_iter=3000, verbose=0, restart=50,
                  variants=("fp64", "fp32", "fp32_learned", "fp32_gmres", "fp32_idr2", "fp64_idr2", "fp32_diag")):
    """Stokes solve to 1e-8 (FP64 FGMRES): plain FP64 V-cycle, FP32 V-cycle,
    and FP32 V-cycle with the learned smoother scaling (installed with its
    guard; a failed learned solve is redone plain and both costs counted);
    then the outer-solver variants in SOLVER_VARIANTS."""
    import torch
    from paper_1907_06696_amd import inputs
    info = s.info()
    L = info["L"]
    n = info["n_u"][L]
    rhs = torch.empty(n, dtype=torch.float64, device="cuda")
    s.assemble_rhs(inputs.sinker_force(qp, centres).reshape(-1, 27, 3), rhs)
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    p = torch.empty(info["n_p"], dtype=torch.float64, device="cuda")

    def one(prec, scaled, **kw):
        if verbose:
            print(f"[solve] {prec}{' + learned scaling' if scaled else ''} {kw}", file=sys.stderr, flush=True)
        st = s.solve_stokes(rhs, u, p, vcycle_prec=prec, use_scaling=int(scaled), raise_on_noconv=False,
                            max_iter=max_iter, verbose=verbose, restart=restart, **kw)
        return {"seconds": round(st["seconds"], 3), "iterations": st["iterations"],
                "rel_residual": st["rel_residual"], "inner_cg": st["inner_cg_iterations"],
                "converged": bool(st["converged"]), "vectors": krylov_vectors(kw, restart)}

    out = {"restart": restart}
    if "fp64" in variants:
        out["fp64"] = one("fp64", False)
    if "fp32" in variants or "fp32_learned" in variants:
        out["fp32"] = one("fp32", False)
    for name, (prec, kw) in SOLVER_VARIANTS.items():
        if name in variants:
            out[name] = one(prec, False, **kw)
    if "fp32_learned" not in variants:
        return out
    w = torch.tensor(np.load(WEIGHTS)["weights"], device="cuda")
    t0 = time.perf_counter()
    used, fac = s.apply_mlp(w, guard=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    lrn = one("fp32", True) if used else dict(out["fp32"])
    if used and not lrn["converged"]:
        again = one("fp32", False)
        lrn = dict(again, seconds=round(lrn["seconds"] + again["seconds"], 3),
                   iterations=lrn["iterations"] + again["iterations"], fallback=True)
    lrn.update({"learned_used": used, "setup_s": round(t_setup, 3),
                "vcycle_factor_plain": round(float(fac[0]), 5), "vcycle_factor_learned": round(float(fac[1]), 5)})
    out["fp32_learned"] = lrn
    if "fp64" in out:
        out["speedup_fp32_learned_vs_fp64"] = round(out["fp64"]["seconds"] / max(lrn["seconds"], 1e-9), 3)
    for lv in range(2, L + 1):
        s.set_scaling(lv, None)
    return out


def solve_workload(name, variants, max_iter=3000):
    """The adaptive 32^3 + 2 (16 sinkers, DR 1e6) and the 128^3 + 1
    (32 sinkers, DR 1e6) sinker solves; one JSON line each.  FGMRES restarts
    every 100 iterations here: at this contrast and sinker count restarts
    every 50 stall (the 32^3 + 2 case stagnates near 4e-6 for thousands of
    iterations; 60 needs twice the iterations), and 100 was the fastest of
    80, 100 and 120 over both workloads."""
    import torch
    from paper_1907_06696_amd import inputs, mfgmg
    cfg = inputs.CONFIGS[name]
    centres = inputs.sinker_centres(cfg["sinkers"], cfg["centre_seed"])
    t0 = time.perf_counter()
    s = mfgmg.Solver(cfg["base_level"])
    cells = inputs.refinement_cells(cfg["base_level"], centres, cfg["dr"], cfg["refine_percentile"])
    s.refine(cells, cfg["refine_levels"])
    s.finalize_mesh()
    info = s.info()
    L = info["L"]
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    s.set_viscosity(inputs.sinker_mu(qp, centres, cfg["dr"]).reshape(-1, 27))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"[{name}] L={L} cells={info['n_cells'][L]} n_u={info['n_u'][L]} n_p={info['n_p']} "
          f"hanging={info['n_hanging'][L]} setup {t_setup:.1f} s", flush=True)
    res = solve_compare(s, qp, centres, verbose=100, restart=100, variants=variants, max_iter=max_iter)
    print(json.dumps({"workload": name, "cells": info["n_cells"][L], "velocity_dofs": info["n_u"][L],
                      "pressure_dofs": info["n_p"], "levels": L, "setup_s": round(t_setup, 2),
                      "stokes_solve_1e-8": res}), flush=True)
    s.close()


def summarize_counters(fetch_csv, write_csv, level=6):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the operator's two
    kernels at the 2^level mesh, each scaled by bytes / counter of the
    calibration copy (the largest copy dispatches, COPY_BYTES read and
    written)."""
    import csv
    n = 1 << level
    out = {"level": level, "kernel_source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES}
    total = 0.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        gmax = max(int(r["Grid_Size"]) for r in copies)
        cal = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == gmax]
        cal_kib = sorted(cal)[len(cal) // 2]
        scale = COPY_BYTES / (cal_kib * 1024.0)
        per = {}
        for tag in ("k_vmult_brick<float", "k_brick_halo_add<float"):
            v = [float(r["Counter_Value"]) for r in rows if tag in r["Kernel_Name"] and int(r["Grid_Size"]) == n ** 3]
            per[tag.split("<")[0]] = {"dispatches": len(v), "kib_per_dispatch": sum(v) / max(len(v), 1)}
        bytes_ = sum(d["kib_per_dispatch"] for d in per.values()) * 1024.0 * scale
        out[name] = {"calibration_kib": cal_kib, "scale_bytes_per_counted_byte": scale, "kernels": per,
                     "bytes_per_application": bytes_}
        total += bytes_
    out["bytes_per_application"] = total
    with open(COUNTERS, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)
    if args.solve_workload:
        variants = args.variants
        if variants is None:
            skip = ("fp32_idr2", "fp32_diag") if args.solve_workload == "uniform128p1" else ()
            variants = ",".join(["fp64", "fp32", "fp32_learned"] + [v for v in SOLVER_VARIANTS if v not in skip])
        solve_workload(args.solve_workload, variants.split(","), args.max_iter)
        return
    import torch
    from paper_1907_06696_amd import inputs, mfgmg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = inputs.CONFIGS["uniform64"]
    level = args.level
    centres = inputs.sinker_centres(cfg["sinkers"], cfg["centre_seed"])
    dr = cfg["dr"]

    t_setup = time.perf_counter()
    s = mfgmg.Solver(level)
    s.finalize_mesh()
    info = s.info()
    L = info["L"]
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    mu_qp = inputs.sinker_mu(qp, centres, dr).reshape(-1, 27)
    t_mesh = time.perf_counter() - t_setup
    t0 = time.perf_counter()
    s.set_viscosity(mu_qp)
    torch.cuda.synchronize()
    t_assemble = time.perf_counter() - t0
    n = info["n_u"][L]
    ncell = info["n_cells"][L]
    x64 = torch.tensor(inputs.uniform_vector(n, cfg["vector_seed"]), dtype=torch.float64, device=dev)
    x32 = x64.float()
    y32 = torch.empty_like(x32)
    y64 = torch.empty_like(x64)
    if args.counter_probe:
        counter_probe(s, L, x32, y32)
        s.close()
        return

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    def step32():
        for _ in range(REPS):
            s.vmult(L, x32, y32)

    def step64():
        for _ in range(REPS):
            s.vmult(L, x64, y64)

    # the timed region: K steps of 100 FP32 operator applications
    t32 = timed(step32, args.steps, args.warmup)
    ms_per_step = t32 / args.steps * 1e3
    value = n * REPS * args.steps / t32 / 1e9
    t64 = timed(step64, max(2, args.steps // 4), 1)
    gdofs64 = n * REPS * max(2, args.steps // 4) / t64 / 1e9
    # roofline of the operator application timed above (one mfgmg_vmult call =
    # the owner-computes brick kernel + the halo-add kernel, HIP events on the
    # stream they are launched on)
    vmult_call_s = t32 / (REPS * args.steps)
    kernel_s = vmult_call_s
    flops = FLOP_PER_CELL * ncell
    alg_bytes = 2 * 4 * n + 4 * ncell        # read x, write y, cell viscosity (FP32)
    achieved_tflops = flops / kernel_s / 1e12
    traffic = measured_traffic(level)

    # V-cycles
    vc = {}
    for name, xx in (("fp32", x32), ("fp64", x64)):
        out = torch.empty_like(xx)
        tv = timed(lambda: s.vcycle(xx, out), 10, 2)
        vc[name] = tv / 10 * 1e3

    result = {
        "metric": "Q2 viscous vmult GDoF/s",
        "value": round(value, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sinker {1 << level}^3 uniform Q2 vmult, 8 sinkers, DR 1e4",
                   "cells": ncell, "velocity_dofs": n, "reps_per_step": REPS},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
                     "traffic": traffic["bytes"] if traffic else None,
                     "kernel": "k_vmult_brick<float,8,8,4> + k_brick_halo_add<float,8,8,4> (one mfgmg_vmult)",
                     "kernel_us": round(kernel_s * 1e6, 2),
                     "flop_per_launch": flops, "alg_bytes_per_launch": alg_bytes,
                     "hbm_frac_algorithmic": round(alg_bytes / kernel_s / 1e9 / PEAK_HBM_GBS, 4),
                     "traffic_source": traffic["source"] if traffic else "none for this kernel source"},
        "vmult_fp64_gdofs": round(gdofs64, 3),
        "vmult_call_us_fp32": round(vmult_call_s * 1e6, 2),
        "vcycle_ms": {k: round(v, 3) for k, v in vc.items()},
        "setup_s": {"mesh": round(t_mesh, 2), "assemble": round(t_assemble, 2)},
    }

    if not args.no_solve:
        result["stokes_solve_1e-8"] = solve_compare(s, qp, centres)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(level, centres, dr)
    s.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
