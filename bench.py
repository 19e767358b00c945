"""Benchmark: matrix-free Q2 viscous operator throughput and Stokes solves on one MI355X.

Operator workload (the 64^3 sinker configuration): unit cube, 64^3 uniform
cells, Q2 velocity (6,440,067 dofs), 8 seeded sinkers (centre seed 2),
viscosity contrast 1e4, operator applied to seeded uniform[-1, 1] vectors
(seeds 42, 43, ...).  One step = 100 FP64 operator applications (the
configuration's 100 repetitions), cycling through 6 (x, y) vector pairs
(618 MB, more than the 256 MB last-level cache, so every application reads x
and writes y in HBM); `value` = velocity dofs processed per second over the
timed steps, in GDoF/s.  Reported beside it (not part of `value`): the same
with one pair (cache-warm), the FP32 operator (cold and warm), the cell loop
alone, one FP32/FP64 V-cycle, and the Stokes solves to 1e-8 (FP64 FGMRES with
the FP64 V-cycle, the FP32 V-cycle, and the FP32 V-cycle with the learned
smoother scaling) on the 64^3 workload and on the adaptive 32^3 + 2 workload
(16 sinkers, contrast 1e6).  The CPU leg times the oracle's operator and
recomputes the FP64 residual of every solve with the oracle's cellwise
operators.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-solve] [--no-adaptive] [--no-cpu]
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
ROTATE = {"f64": 6, "f32": 8}   # (x, y) pairs cycled through: 618 MB / 412 MB > 256 MB cache
PEAK_FP64_TFLOPS = 78.6         # MI355X FP64 vector, published
PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector (packed FMA), published
PEAK_FP32_UNPACKED_TFLOPS = 78.6   # the rate without packed FP32 instructions, which this build does not use
PEAK_HBM_GBS = 8000.0
# Algorithmic work of the cell kernel per cell (sum factorisation as built,
# counting an FMA as 2 flops): 810 (interpolation) + 972 (gradients) + 297
# (stress) + 1215 (transposed gradients) + 729 (transposed interpolation)
FLOP_PER_CELL = 4023
# The Q3-Q2 operator (k = 2) per cell: 36 one-dimensional contractions of 64
# values with 4 terms each (9 interpolation, 9 derivative, 9 transposed
# derivative, 9 transposed interpolation sweeps; 4 multiplies + 3 adds),
# 768 for the symmetric stress (6 sums, 6 scalings per point) and 384 for
# summing the three transposed derivatives of each component
Q3_FLOP_PER_CELL = 36 * 64 * 7 + 768 + 384


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-solve", action="store_true", help="skip every Stokes solve")
    p.add_argument("--no-adaptive", action="store_true", help="skip the adaptive 32^3 + 2 solves")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU leg (oracle timing and residual checks)")
    p.add_argument("--no-q3", action="store_true", help="skip the Q3-Q2 (k = 2) section")
    p.add_argument("--q3-level", type=int, default=5, help="Q3-Q2 section: 2^level cells per edge (default 5: 32^3)")
    p.add_argument("--q3-only", action="store_true", help="run the Q3-Q2 section alone (for profiling)")
    p.add_argument("--level", type=int, default=6, help="cells per edge = 2^level (default 6: 64^3)")
    p.add_argument("--solve-workload", choices=["adaptive32p2", "uniform128p1"], default=None,
                   help="instead of the operator benchmark, compare the Stokes solves on this workload")
    p.add_argument("--max-iter", type=int, default=3000, help="FGMRES iteration cap of --solve-workload")
    p.add_argument("--variants", default=None,
                   help="solves of --solve-workload, comma separated from fp64, fp32, fp32_learned, fp64_local, "
                        "fp32_local, fp32_gmres, fp32_idr2, fp64_idr2, fp32_diag (default: all on adaptive32p2; "
                        "on uniform128p1 all but fp32_diag, which needs ~4x the iterations)")
    p.add_argument("--oracle-residual", action="store_true",
                   help="with --solve-workload: recompute every solve's FP64 residual with the oracle")
    p.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                   help="turn the counter_collection.csv files of a FETCH_SIZE and a WRITE_SIZE pass over "
                        "--counter-probe into profiles/vmult_counters_sinker64.json (no GPU needed)")
    p.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV", default=None,
                   help="print a markdown table of a rocprofv3 kernel trace: per kernel and grid, calls, mean, "
                        "median and total duration, registers and LDS (no GPU needed)")
    p.add_argument("--counter-probe", action="store_true",
                   help="only launch the operator (mfgmg_vmult: brick + halo kernels) 20 times in FP64 and 20 "
                        "times in FP32 on rotating vector pairs, and a plain copy of known size 20 times, for "
                        "hardware-counter runs")
    return p.parse_args()


COPY_BYTES = 256 << 20          # the calibration copy: 256 MiB read + 256 MiB written


def counter_probe(s, L, pairs):
    """Kernels for a rocprofv3 --pmc pass: 20 operator applications per
    precision on rotating pairs (as timed) and 20 copies of COPY_BYTES, so that
    FETCH_SIZE / WRITE_SIZE per dispatch of the operator's kernels can be
    scaled by what the same counters read for a copy of known size."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for prec in ("f64", "f32"):
        xs, ys = pairs[prec]
        for r in range(20):
            s.vmult(L, xs[r % len(xs)], ys[r % len(xs)])
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counter_probe": True, "copy_bytes": COPY_BYTES, "vmult_launches_per_precision": 20}),
          flush=True)


WEIGHTS = os.path.join(ROOT, "paper_1907_06696_amd", "data", "mlp_sinker32.npz")
COUNTERS = os.path.join(ROOT, "profiles", "vmult_counters_sinker64.json")
KERNEL_SOURCES = ("brick_kernel.h", "cell_kernel.h")
KERNEL_TAGS = {"f64": ("k_vmult_brick<double", "k_brick_halo_add<double"),
               "f32": ("k_vmult_brick<float", "k_brick_halo_add<float")}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1907_06696_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(level, prec):
    """HBM bytes per operator application from the committed FETCH_SIZE /
    WRITE_SIZE passes (scaled by the calibration copy), or None when the
    counters were taken on other kernel sources or another workload."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_hash") != kernel_source_hash() or c.get("level") != level or prec not in c:
        return None
    return {"bytes": int(c[prec]["bytes_per_application"]), "source": os.path.relpath(COUNTERS, ROOT)}


# the local-smoothing hierarchy (level meshes of one refinement level, the
# multigrid of Sec. 2.2.1's reference) with the FP64 and the FP32 V-cycle;
# outer-solver variants of Sec. 3.4 (V-cycle precision, options): plain GMRES
# and IDR(2) with the fixed Chebyshev Schur map (IDR also with the FP64
# V-cycle: its short recurrences can stall on the FP32 one), FGMRES with the
# block-diagonal P_D;
# vectors = FP64 block vectors the Krylov method keeps (FGMRES 2m + 1, GMRES
# m + 2, IDR(s) 3s + 2, each plus b, x, r, w)
SOLVER_VARIANTS = {
    "fp64_local": ("fp64", dict(hierarchy="local")),
    "fp32_local": ("fp32", dict(hierarchy="local")),
    "fp32_gmres": ("fp32", dict(krylov="gmres", schur="cheb")),
    "fp32_idr2": ("fp32", dict(krylov="idr", schur="cheb", idr_s=2)),
    "fp64_idr2": ("fp64", dict(krylov="idr", schur="cheb", idr_s=2)),
    "fp32_diag": ("fp32", dict(block="diagonal")),
    # the inner pressure-mass CG to 1e-6 instead of the default 1e-2
    "fp32_schur1e-6": ("fp32", dict(schur_rtol=1e-6)),
}


def q3_section(level, centres, dr, timed, solves=True):
    """The Q3-Q2 pair (k = 2 of Sec. 2.1) on the same sinker field (8
    sinkers, DR 1e4): operator throughput, FP64 and FP32, on rotating vector
    pairs larger than the last-level cache (one mfgmg_vmult: the output
    initialisation and the wavefront-per-cell kernel), V-cycles, and the
    Stokes solves to 1e-8 with the FP64 and the FP32 V-cycle (FGMRES(50))."""
    import torch
    from paper_1907_06696_amd import inputs, mfgmg
    t0 = time.perf_counter()
    s = mfgmg.Solver(level)
    s.set_element(2)
    s.finalize_mesh()
    info = s.info()
    L = info["L"]
    n, ncell = info["n_u"][L], info["n_cells"][L]
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    s.set_viscosity(inputs.sinker_mu(qp, centres, dr).reshape(-1, 64))
    torch.cuda.synchronize()
    out = {"workload": f"sinker {1 << level}^3 uniform Q3-Q2, 8 sinkers, DR 1e4", "cells": ncell,
           "velocity_dofs": n, "pressure_dofs": info["n_p"], "setup_s": round(time.perf_counter() - t0, 2)}
    print(f"[q3] {out['workload']}: {n} velocity dofs, setup {out['setup_s']} s", file=sys.stderr, flush=True)
    reps = 20
    flops = Q3_FLOP_PER_CELL * ncell
    ops = {}
    first = {}
    for prec, dt, word, peak in (("f64", torch.float64, 8, PEAK_FP64_TFLOPS), ("f32", torch.float32, 4,
                                                                                PEAK_FP32_TFLOPS)):
        npairs = max(2, int(np.ceil(320e6 / (2 * word * n))))
        xs = [torch.tensor(inputs.uniform_vector(n, 42 + i), dtype=dt, device="cuda") for i in range(npairs)]
        ys = [torch.empty_like(x) for x in xs]
        k = [0]

        def step():
            for r in range(reps):
                i = (k[0] + r) % npairs
                s.vmult(L, xs[i], ys[i])
            k[0] += reps
        t = timed(step, 5, 1) / (5 * reps)
        ach = flops / t / 1e12
        ops[prec] = {"gdofs": round(n / t / 1e9, 3), "call_us": round(t * 1e6, 2), "pairs": npairs,
                     "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                     "flop_per_launch": flops, "alg_bytes_per_launch": 2 * word * n + word * ncell,
                     "hbm_frac_algorithmic": round((2 * word * n + word * ncell) / t / 1e9 / PEAK_HBM_GBS, 4)}
        first[prec] = xs[0]
        del ys
    ops["kernel"] = "k_vmult_q3 + k_q3_halo_add (one mfgmg_vmult)"
    out["operator"] = ops
    vc = {}
    for name, key in (("fp32", "f32"), ("fp64", "f64")):
        xx = first[key]
        yy = torch.empty_like(xx)
        vc[name] = round(timed(lambda: s.vcycle(xx, yy), 10, 2) / 10 * 1e3, 3)
    out["vcycle_ms"] = vc
    print(f"[q3] operator {json.dumps({p: ops[p]['gdofs'] for p in ('f64', 'f32')})} GDoF/s, "
          f"V-cycle {vc} ms", file=sys.stderr, flush=True)
    if solves:
        rhs = torch.empty(n, dtype=torch.float64, device="cuda")
        s.assemble_rhs(inputs.sinker_force(qp, centres).reshape(-1, 64, 3), rhs)
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        p = torch.empty(info["n_p"], dtype=torch.float64, device="cuda")
        sol = {}
        for prec in ("fp64", "fp32"):
            st = s.solve_stokes(rhs, u, p, vcycle_prec=prec, raise_on_noconv=False, max_iter=3000)
            sol[prec] = {"seconds": round(st["seconds"], 3), "iterations": st["iterations"],
                         "rel_residual": st["rel_residual"], "inner_cg": st["inner_cg_iterations"],
                         "converged": bool(st["converged"])}
        out["stokes_solve_1e-8"] = sol
        print(f"[q3] solves {json.dumps(sol)}", file=sys.stderr, flush=True)
    s.close()
    return out


def krylov_vectors(kw, restart):
    k = kw.get("krylov", "fgmres")
    if k == "gmres":
        return restart + 2 + 4
    if k == "idr":
        return 3 * kw.get("idr_s", 2) + 2 + 4
    return 2 * restart + 1 + 4


def solve_compare(s, qp, centres, max_iter=3000, verbose=0, restart=50, keep=None,
                  variants=("fp64", "fp32", "fp32_learned", "fp32_gmres", "fp32_idr2", "fp64_idr2", "fp32_diag")):
    # (on a uniform mesh the local-smoothing cycle is the global one: not repeated)
    """Stokes solve to 1e-8 (FP64 FGMRES): plain FP64 V-cycle, FP32 V-cycle,
    and FP32 V-cycle with the learned smoother scaling (installed behind its
    guard, estimated with the FP64 V-cycle; a failed learned solve is redone
    plain and both costs counted); then the outer-solver variants in
    SOLVER_VARIANTS.  keep: dict that receives each solution (u, p) on the
    host, for the oracle's residual check."""
    import torch
    from paper_1907_06696_amd import inputs
    info = s.info()
    L = info["L"]
    n = info["n_u"][L]
    rhs = torch.empty(n, dtype=torch.float64, device="cuda")
    s.assemble_rhs(inputs.sinker_force(qp, centres).reshape(-1, 27, 3), rhs)
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    p = torch.empty(info["n_p"], dtype=torch.float64, device="cuda")

    def one(name, prec, scaled, **kw):
        if verbose:
            print(f"[solve] {name}: {prec}{' + learned scaling' if scaled else ''} {kw}", file=sys.stderr, flush=True)
        st = s.solve_stokes(rhs, u, p, vcycle_prec=prec, use_scaling=int(scaled), raise_on_noconv=False,
                            max_iter=max_iter, verbose=verbose, restart=restart, **kw)
        if keep is not None:
            keep[name] = (u.cpu().numpy(), p.cpu().numpy())
        rec = {"seconds": round(st["seconds"], 3), "iterations": st["iterations"],
               "rel_residual": st["rel_residual"], "inner_cg": st["inner_cg_iterations"],
               "converged": bool(st["converged"]), "vectors": krylov_vectors(kw, restart)}
        if st["fp64_from"] >= 0:   # a stalled FP32 IDR run went on with the FP64 V-cycle
            rec["fp64_from_iteration"] = st["fp64_from"]
        return rec

    out = {"restart": restart}
    if "fp64" in variants:
        out["fp64"] = one("fp64", "fp64", False)
    if "fp32" in variants or "fp32_learned" in variants:
        out["fp32"] = one("fp32", "fp32", False)
    for name, (prec, kw) in SOLVER_VARIANTS.items():
        if name in variants:
            out[name] = one(name, prec, False, **kw)
    if "fp32_learned" not in variants:
        return out
    w = torch.tensor(np.load(WEIGHTS)["weights"], device="cuda")
    t0 = time.perf_counter()
    used, fac = s.apply_mlp(w, guard="fp64")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    if used:
        lrn = one("fp32_learned", "fp32", True)
        if not lrn["converged"]:
            again = one("fp32_learned", "fp32", False)
            lrn = dict(again, seconds=round(lrn["seconds"] + again["seconds"], 3),
                       iterations=lrn["iterations"] + again["iterations"], fallback=True)
    else:
        lrn = dict(out["fp32"])
        if keep is not None and "fp32" in keep:
            keep["fp32_learned"] = keep["fp32"]
    lrn.update({"learned_used": used, "setup_s": round(t_setup, 3),
                "seconds_with_setup": round(lrn["seconds"] + t_setup, 3),
                "vcycle_factor_plain": round(float(fac[0]), 5), "vcycle_factor_learned": round(float(fac[1]), 5)})
    out["fp32_learned"] = lrn
    if "fp64" in out:
        out["speedup_fp32_vs_fp64"] = round(out["fp64"]["seconds"] / max(out["fp32"]["seconds"], 1e-9), 3)
        out["speedup_fp32_learned_vs_fp64"] = round(out["fp64"]["seconds"] / max(lrn["seconds_with_setup"], 1e-9), 3)
    out["speedup_fp32_learned_vs_fp32"] = round(out["fp32"]["seconds"] / max(lrn["seconds_with_setup"], 1e-9), 3)
    for lv in range(2, L + 1):
        s.set_scaling(lv, None)
    return out


def adaptive_solver(name):
    """Library context of an adaptive workload with its viscosity set."""
    import torch
    from paper_1907_06696_amd import inputs, mfgmg
    cfg = inputs.CONFIGS[name]
    centres = inputs.sinker_centres(cfg["sinkers"], cfg["centre_seed"])
    t0 = time.perf_counter()
    s = mfgmg.Solver(cfg["base_level"])
    cells = inputs.refinement_cells(cfg["base_level"], centres, cfg["dr"], cfg["refine_percentile"])
    s.refine(cells, cfg["refine_levels"])
    s.finalize_mesh()
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    s.set_viscosity(inputs.sinker_mu(qp, centres, cfg["dr"]).reshape(-1, 27))
    torch.cuda.synchronize()
    return s, qp, centres, cells, time.perf_counter() - t0


def solve_workload(name, variants, max_iter=3000, verbose=100, oracle_check=False):
    """The adaptive 32^3 + 2 (16 sinkers, DR 1e6) and the 128^3 + 1
    (32 sinkers, DR 1e6) sinker solves.  FGMRES restarts every 100 iterations
    here: at this contrast and sinker count restarts every 50 stall (the
    32^3 + 2 case stagnates near 4e-6 for thousands of iterations; 60 needs
    twice the iterations), and 100 was the fastest of 80, 100 and 120 over
    both workloads."""
    s, qp, centres, cells, t_setup = adaptive_solver(name)
    info = s.info()
    L = info["L"]
    print(f"[{name}] L={L} cells={info['n_cells'][L]} n_u={info['n_u'][L]} n_p={info['n_p']} "
          f"hanging={info['n_hanging'][L]} setup {t_setup:.1f} s", file=sys.stderr, flush=True)
    keep = {} if oracle_check else None
    res = solve_compare(s, qp, centres, verbose=verbose, restart=100, variants=variants, max_iter=max_iter, keep=keep)
    out = {"workload": name, "cells": info["n_cells"][L], "velocity_dofs": info["n_u"][L],
           "pressure_dofs": info["n_p"], "levels": L, "setup_s": round(t_setup, 2), "stokes_solve_1e-8": res}
    keys = (s.support_points(L, 0), s.support_points(L, 1))
    s.close()
    return out, keep, keys, cells, centres


# ------------------------------------------------------------------- CPU leg
def oracle_operator_timing(level, centres, dr, seconds=12.0):
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


def oracle_residuals(lev, ijk, centres, dr, keys, sols):
    """FP64 relative residual ||b - K x|| / ||b|| of each device solution,
    recomputed by the oracle's cellwise operators on its own mesh, viscosity
    and right-hand side (vectors matched by canonical node keys)."""
    from oracle import mesh as om, operators as ops
    from paper_1907_06696_amd import inputs
    t0 = time.perf_counter()
    lev, ijk = om.morton_sort(np.asarray(lev, np.int64), np.asarray(ijk, np.int64))
    m = om.LevelMesh(lev, ijk, int(lev.max()) + 1, with_pressure=True)
    print(f"[oracle] leaf mesh: {m.ncell} cells, {m.n_u} velocity dofs, {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    X = ops.gauss_points_of_cells(m).reshape(-1, 3)
    mu = ops.harmonic_cell_viscosity(inputs.sinker_mu(X, centres, dr).reshape(-1, 27))
    b_u = ops.assemble_rhs(m, inputs.sinker_force(X, centres).reshape(-1, 27, 3))
    ku, kp = keys
    node = np.searchsorted(m.keys, ku)
    pnode = np.searchsorted(m.pkeys, kp)
    assert np.array_equal(m.keys[node], ku) and np.array_equal(m.pkeys[pnode], kp)
    dof = (3 * node[:, None] + np.arange(3)[None, :]).ravel()
    AB = (ops.CellwiseA(m, mu), ops.CellwiseB(m))
    out = {}
    for name, (u_lib, p_lib) in sols.items():
        u = np.empty(m.n_u)
        u[dof] = u_lib
        p = np.empty(m.npnode)
        p[pnode] = p_lib
        out[name] = ops.stokes_residual(m, mu, b_u, u, p, ops_AB=AB)
        print(f"[oracle] residual of {name}: {out[name]:.3e}, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    return out, time.perf_counter() - t0


def adaptive_leaves(cfg, cells):
    from oracle import mesh as om
    lev, ijk = om.uniform_leaves(cfg["base_level"])
    mask = np.isin(om.cell_code(lev, ijk), om.cell_code(cells[:, 0], cells[:, 1:]))
    lev, ijk = om.refine(lev, ijk, mask, cfg["refine_levels"])
    return om.balance(lev, ijk)


def cpu_leg(level, centres, dr, checks):
    """The CPU baseline: the oracle's operator timed on the host cores, and
    the oracle's FP64 residual of every device solution (not timed)."""
    res = oracle_operator_timing(level, centres, dr)
    out = {}
    for name, (lev, ijk, cen, d, keys, sols) in checks.items():
        r, dt = oracle_residuals(lev, ijk, cen, d, keys, sols)
        out[name] = {k: float(f"{v:.3e}") for k, v in r.items()}
        out[name]["oracle_seconds"] = round(dt, 1)
    res["oracle_fp64_residual_of_device_solutions"] = out
    return res


def summarize_counters(fetch_csv, write_csv, level=6):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the operator's two
    kernels at the 2^level mesh, per precision, each scaled by bytes / counter
    of the calibration copy (the largest copy dispatches, COPY_BYTES read and
    written)."""
    import csv
    out = {"level": level, "kernel_source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES,
           "note": "operator applications on rotating vector pairs (618 MB FP64, 412 MB FP32)"}
    scale = {}
    rows = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows[name] = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
        copies = [r for r in rows[name] if "copyBuffer" in r["Kernel_Name"]]
        gmax = max(int(r["Grid_Size"]) for r in copies)
        cal = sorted(float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == gmax)
        scale[name] = (cal[len(cal) // 2], COPY_BYTES / (cal[len(cal) // 2] * 1024.0))
    for prec, tags in KERNEL_TAGS.items():
        entry = {}
        total = 0.0
        for name in ("FETCH_SIZE", "WRITE_SIZE"):
            per = {}
            for tag in tags:
                # the probe's 20 applications: the last 20 dispatches at the leaf's
                # grid, the kernel's largest (set-up also applies the leaf operator,
                # to estimate lambda, and the lower levels' operators)
                mine = [r for r in rows[name] if tag in r["Kernel_Name"]]
                gmax = max((int(r["Grid_Size"]) for r in mine), default=0)
                v = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in mine
                           if int(r["Grid_Size"]) == gmax)[-20:]
                per[tag.split("<")[0]] = {"dispatches": len(v), "kib_per_dispatch": sum(c for _, c in v) / max(len(v), 1)}
            b = sum(d["kib_per_dispatch"] for d in per.values()) * 1024.0 * scale[name][1]
            entry[name] = {"calibration_kib": scale[name][0], "scale_bytes_per_counted_byte": scale[name][1],
                           "kernels": per, "bytes_per_application": b}
            total += b
        entry["bytes_per_application"] = total
        out[prec] = entry
    with open(COUNTERS, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def summarize_trace(path, top=14):
    """Markdown table of a rocprofv3 kernel trace grouped by (kernel, grid)."""
    import csv
    groups = {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"] or "(unnamed)"
        name = name.replace("void ", "").replace("(anonymous namespace)::", "").replace("mfgmg::", "").split("(")[0]
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        g = groups.setdefault((name, grid), {"d": [], "vgpr": r["VGPR_Count"], "agpr": r["Accum_VGPR_Count"],
                                             "lds": r["LDS_Block_Size"]})
        g["d"].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print("| kernel | grid | calls | mean us | median us | total ms | VGPR(+AGPR) | LDS B |")
    print("|---|---|---|---|---|---|---|---|")
    for (name, grid), g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["d"]))[:top]:
        d = sorted(g["d"])
        print(f"| {name} | {grid} | {len(d)} | {sum(d) / len(d):.2f} | {d[len(d) // 2]:.2f} | {sum(d) / 1e3:.2f} | "
              f"{g['vgpr']}+{g['agpr']} | {g['lds']} |")


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)
    if args.solve_workload:
        variants = args.variants
        if variants is None:
            skip = ("fp32_diag",) if args.solve_workload == "uniform128p1" else ()
            variants = ",".join(["fp64", "fp32", "fp32_learned"] + [v for v in SOLVER_VARIANTS
                                                                       if v not in skip and "schur" not in v])
        out, keep, keys, cells, centres = solve_workload(args.solve_workload, variants.split(","), args.max_iter,
                                                         oracle_check=args.oracle_residual)
        if args.oracle_residual:
            from paper_1907_06696_amd import inputs
            cfg = inputs.CONFIGS[args.solve_workload]
            lev, ijk = adaptive_leaves(cfg, cells)
            r, dt = oracle_residuals(lev, ijk, centres, cfg["dr"], keys, keep)
            out["oracle_fp64_residual"] = {k: float(f"{v:.3e}") for k, v in r.items()}
            out["oracle_seconds"] = round(dt, 1)
        print(json.dumps(out), flush=True)
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

    if args.q3_only:
        print(json.dumps({"q3q2": q3_section(args.q3_level, centres, dr, timed, solves=not args.no_solve)}),
              flush=True)
        return

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
    pairs = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        xs = [torch.tensor(inputs.uniform_vector(n, cfg["vector_seed"] + i), dtype=dt, device=dev)
              for i in range(ROTATE[prec])]
        pairs[prec] = (xs, [torch.empty_like(xs[0]) for _ in xs])
    if args.counter_probe:
        counter_probe(s, L, pairs)
        s.close()
        return

    def op_step(prec, rotate, add=False):
        xs, ys = pairs[prec]
        k = [0]
        f = s.vmult_add if add else s.vmult

        def step():
            for r in range(REPS):
                i = (k[0] + r) % len(xs) if rotate else 0
                f(L, xs[i], ys[i])
            k[0] += REPS
        return step

    # the timed region: K steps of 100 FP64 operator applications on rotating pairs
    t64 = timed(op_step("f64", True), args.steps, args.warmup)
    ms_per_step = t64 / args.steps * 1e3
    value = n * REPS * args.steps / t64 / 1e9
    sub = max(2, args.steps // 4)
    times = {("f64", "cold"): t64 / (REPS * args.steps)}
    times[("f64", "warm")] = timed(op_step("f64", False), sub, 1) / (REPS * sub)
    times[("f32", "cold")] = timed(op_step("f32", True), sub, 1) / (REPS * sub)
    times[("f32", "warm")] = timed(op_step("f32", False), sub, 1) / (REPS * sub)
    # the cell loop alone (mfgmg_vmult_add: one brick-kernel launch per call)
    cell_loop = {p: timed(op_step(p, True, add=True), sub, 1) / (REPS * sub) for p in ("f64", "f32")}

    flops = FLOP_PER_CELL * ncell

    def roof(prec, peak, extra=None):
        """Roofline of one operator application (brick kernel + halo-add
        kernel, HIP events on the stream they are launched on), cold."""
        call = times[(prec, "cold")]
        word = 8 if prec == "f64" else 4
        alg_bytes = 2 * word * n + word * ncell        # read x, write y, cell viscosity
        ach = flops / call / 1e12
        tr = measured_traffic(level, prec)
        # brick shape of the level (8 x 8 x 4 cells from 64 per edge up, 8 x 4 x 4 below)
        tname = f"{'double' if prec == 'f64' else 'float'}, 8, {8 if (1 << level) >= 64 else 4}, 4"
        out = {"bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
               "frac": round(ach / peak, 4), "traffic": tr["bytes"] if tr else None,
               "kernel": f"k_vmult_brick<{tname}> + k_brick_halo_add<{tname}> (one mfgmg_vmult)",
               "call_us": round(call * 1e6, 2), "cell_loop_us": round(cell_loop[prec] * 1e6, 2),
               "cell_loop_frac": round(flops / cell_loop[prec] / 1e12 / peak, 4),
               "flop_per_launch": flops, "alg_bytes_per_launch": alg_bytes,
               "hbm_frac_algorithmic": round(alg_bytes / call / 1e9 / PEAK_HBM_GBS, 4),
               "hbm_frac_measured": round(tr["bytes"] / call / 1e9 / PEAK_HBM_GBS, 4) if tr else None,
               "traffic_source": tr["source"] if tr else "none for this kernel source"}
        out.update(extra or {})
        return out

    # V-cycles
    vc = {}
    for name, xx in (("fp32", pairs["f32"][0][0]), ("fp64", pairs["f64"][0][0])):
        out = torch.empty_like(xx)
        tv = timed(lambda: s.vcycle(xx, out), 10, 2)
        vc[name] = tv / 10 * 1e3
    # the same V-cycle captured once as a graph and replayed (as the solves
    # run it: no host launch per kernel); every replay checked against the
    # eager V-cycle
    vcg = {}
    for name, xx in (("fp32", pairs["f32"][0][0]), ("fp64", pairs["f64"][0][0])):
        ref = torch.empty_like(xx)
        out = torch.empty_like(xx)
        s.vcycle(xx, ref)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s.vcycle(xx, out)
        tv = timed(g.replay, 10, 2)
        err = float((out - ref).norm() / ref.norm())
        tol = 1e-5 if name == "fp32" else 1e-12
        if not err <= tol:
            raise RuntimeError(f"graph-replayed {name} V-cycle differs from the eager one ({err:.2e})")
        vcg[name] = round(tv / 10 * 1e3, 3)
        del g

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sinker {1 << level}^3 uniform Q2 vmult, 8 sinkers, DR 1e4, FP64, "
                               f"{ROTATE['f64']} rotating vector pairs",
                   "cells": ncell, "velocity_dofs": n, "reps_per_step": REPS},
        "roofline": roof("f64", PEAK_FP64_TFLOPS),
        "vmult_gdofs": {f"{p}_{c}": round(n / t / 1e9, 3) for (p, c), t in times.items()},
        "roofline_fp32": roof("f32", PEAK_FP32_TFLOPS, {
            "frac_unpacked_peak": round(flops / times[("f32", "cold")] / 1e12 / PEAK_FP32_UNPACKED_TFLOPS, 4),
            "unpacked_peak": PEAK_FP32_UNPACKED_TFLOPS}),
        "vcycle_ms": {k: round(v, 3) for k, v in vc.items()},
        "vcycle_graph_ms": vcg,
        "setup_s": {"mesh": round(t_mesh, 2), "assemble": round(t_assemble, 2)},
    }
    print(f"[bench] operator done: {json.dumps(result['vmult_gdofs'])}", file=sys.stderr, flush=True)

    checks = {}
    if not args.no_solve:
        keep = {} if not args.no_cpu else None
        result["stokes_solve_1e-8"] = solve_compare(s, qp, centres, keep=keep)
        if keep is not None:
            from oracle import mesh as om
            lev, ijk = om.uniform_leaves(level)
            checks[f"uniform{1 << level}"] = (lev, ijk, centres, dr, (s.support_points(L, 0),
                                                                       s.support_points(L, 1)), keep)
        print("[bench] 64^3 solves done", file=sys.stderr, flush=True)
    s.close()
    if not args.no_solve and not args.no_adaptive:
        out, keep, keys, cells, cen = solve_workload("adaptive32p2", ("fp64", "fp32", "fp32_learned", "fp64_local",
                                                                      "fp32_local"),
                                                     verbose=0, oracle_check=not args.no_cpu)
        result["adaptive32p2"] = out
        if keep is not None:
            acfg = inputs.CONFIGS["adaptive32p2"]
            lev, ijk = adaptive_leaves(acfg, cells)
            checks["adaptive32p2"] = (lev, ijk, cen, acfg["dr"], keys, keep)
        print("[bench] adaptive 32^3+2 solves done", file=sys.stderr, flush=True)

    if not args.no_q3:
        result["q3q2"] = q3_section(args.q3_level, centres, dr, timed, solves=not args.no_solve)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_leg(level, centres, dr, checks)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
