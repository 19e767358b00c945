"""Learned smoother scaling: training-data generation, training, evaluation.

Orchestration of C-ABI calls only (every step runs in the library's kernels):

* ``generate``: for each seeded sinker field on a uniform 2^base mesh, the
  library fits per-cell targets on every smoothed level (``fit_targets``) and
  computes the cell features; pairs stay on the device;
* ``train``: ``mlp_train`` (mean-squared error, Adam, mini-batches);
* ``evaluate``: on held-out fields, the FP64 FGMRES Stokes solve to 1e-8 with
  the FP32 V-cycle, plain Chebyshev-Jacobi vs the learned scaling (installed
  by ``apply_mlp`` with its guard), iterations and wall seconds.

    python -m paper_1907_06696_amd.learn --fields 256 --eval 0 --weights-out w.npz
    python -m paper_1907_06696_amd.learn --weights-in w.npz --eval 32 --json eval.json
"""
import argparse
import json
import time

import numpy as np

from . import inputs, mfgmg


def solver_for(base, centres, dr, refine_cells=None, levels_up=1):
    s = mfgmg.Solver(base)
    if refine_cells is not None and len(refine_cells):
        s.refine(refine_cells, levels_up)
    s.finalize_mesh()
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    s.set_viscosity(inputs.sinker_mu(qp, centres, dr).reshape(-1, 27))
    return s, qp


def init_weights(seed=0):
    """He-uniform weights, zero biases (numpy default generator), FP32."""
    g = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((27, 64), (64, 64), (64, 3)):
        lim = np.sqrt(6.0 / fi)
        parts.append(g.uniform(-lim, lim, (fo, fi)).ravel())
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def _log(msg):
    print(msg, flush=True)


def generate(base=5, seeds=range(10000, 10256), steps=30, lr=0.05, log=_log):
    """Device tensors (features [N, 27], targets [N, 3]) over all smoothed
    levels of all fields."""
    import torch
    feats, targets = [], []
    t0 = time.time()
    seeds = list(seeds)
    for i, seed in enumerate(seeds):
        centres, dr = inputs.learned_field(seed)
        s, _ = solver_for(base, centres, dr)
        L = s.info()["L"]
        for ell in range(2, L + 1):
            feats.append(s.features(ell))
            y, hist = s.fit_targets(ell, steps=steps, lr=lr)
            targets.append(y)
        s.close()
        if log and (i % 8 == 0 or i == len(seeds) - 1):
            log(f"[generate] field {i + 1}/{len(seeds)} seed {seed} ({len(centres)} sinkers, DR {dr:.1e}) "
                f"finest-level J {hist[0]:.3f} -> {hist[-1]:.3f}, {time.time() - t0:.1f} s")
    return torch.cat(feats).contiguous(), torch.cat(targets).contiguous()


def train(feats, targets, epochs=20, batch=4096, lr=1e-3, seed=0, init_seed=0):
    """Returns (weights device tensor [6147], per-epoch loss)."""
    import torch
    w = torch.tensor(init_weights(init_seed), device=feats.device)
    hist = mfgmg.mlp_train(w, feats, targets, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return w, hist


def evaluate(w, base=6, seeds=range(20000, 20032), prec="fp32", log=_log, max_iter=1000):
    """Per-field FGMRES iterations and seconds to 1e-8: plain vs learned."""
    import torch
    rows = []
    for seed in seeds:
        centres, dr = inputs.learned_field(seed)
        s, qp = solver_for(base, centres, dr)
        info = s.info()
        L = info["L"]
        n = info["n_u"][L]
        rhs = torch.empty(n, dtype=torch.float64, device="cuda")
        s.assemble_rhs(inputs.sinker_force(qp, centres).reshape(-1, 27, 3), rhs)
        u = torch.empty_like(rhs)
        p = torch.empty(info["n_p"], dtype=torch.float64, device="cuda")
        plain = s.solve_stokes(rhs, u, p, vcycle_prec=prec, use_scaling=0, raise_on_noconv=False,
                               max_iter=max_iter)
        t0 = time.perf_counter()
        used, fac = s.apply_mlp(w, guard="fp64")
        t_apply = time.perf_counter() - t0
        lrn = s.solve_stokes(rhs, u, p, vcycle_prec=prec, use_scaling=1, raise_on_noconv=False,
                             max_iter=max_iter) if used else plain
        fallback = bool(used and not lrn["converged"])
        if fallback:  # a learned solve that fails is redone with the plain smoother
            again = s.solve_stokes(rhs, u, p, vcycle_prec=prec, use_scaling=0, raise_on_noconv=False,
                                   max_iter=max_iter)
            lrn = dict(again, iterations=lrn["iterations"] + again["iterations"],
                       seconds=lrn["seconds"] + again["seconds"])
        row = {"seed": seed, "sinkers": len(centres), "dr": dr,
               "plain_its": plain["iterations"], "plain_s": plain["seconds"], "plain_res": plain["rel_residual"],
               "learned_used": used, "factor_plain": fac[0], "factor_learned": fac[1],
               "learned_its": lrn["iterations"], "learned_s": lrn["seconds"], "learned_res": lrn["rel_residual"],
               "apply_s": t_apply, "learned_s_with_setup": lrn["seconds"] + t_apply, "fallback": fallback, "plain_converged": bool(plain["converged"])}
        rows.append(row)
        s.close()
        if log:
            log(f"[evaluate] seed {seed}: plain {plain['iterations']} its {plain['seconds']:.2f} s | "
                f"learned(used={used}) {lrn['iterations']} its {lrn['seconds']:.2f} s | "
                f"factor {fac[0]:.3f} -> {fac[1]:.3f}")
    return rows


def summarize(rows):
    pi = np.array([r["plain_its"] for r in rows])
    li = np.array([r["learned_its"] for r in rows])
    ps = np.array([r["plain_s"] for r in rows])
    ls = np.array([r["learned_s"] for r in rows])
    lt = np.array([r["learned_s_with_setup"] for r in rows])
    return {"fields": len(rows), "median_plain_its": float(np.median(pi)), "median_learned_its": float(np.median(li)),
            "median_plain_s": float(np.median(ps)), "median_learned_s": float(np.median(ls)),
            "median_learned_s_with_setup": float(np.median(lt)),
            "total_plain_s": float(ps.sum()), "total_learned_s_with_setup": float(lt.sum()),
            "used": int(sum(r["learned_used"] for r in rows)),
            "fields_fewer_its": int((li < pi).sum()), "fields_more_its": int((li > pi).sum())}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--fields", type=int, default=256, help="training fields (0: skip training)")
    ap.add_argument("--eval", type=int, default=32, help="held-out evaluation fields (0: skip)")
    ap.add_argument("--base", type=int, default=5, help="training mesh 2^base cells per axis")
    ap.add_argument("--eval-base", type=int, default=6)
    ap.add_argument("--steps", type=int, default=30, help="Adam steps of the target fit")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=2000)
    ap.add_argument("--weights-in", default=None, help="evaluate these weights (.npz) instead of training")
    ap.add_argument("--weights-out", default=None)
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    import torch
    cfg = inputs.CONFIGS["learned"]
    res = {}
    if a.weights_in:
        w = torch.tensor(np.load(a.weights_in)["weights"], device="cuda")
    else:
        t0 = time.time()
        feats, targets = generate(a.base, range(cfg["train_seed0"], cfg["train_seed0"] + a.fields), a.steps)
        res["generate_s"] = time.time() - t0
        res["pairs"] = int(feats.shape[0])
        _log(f"[train] {feats.shape[0]} pairs")
        t0 = time.time()
        w, hist = train(feats, targets, epochs=a.epochs, batch=a.batch, lr=a.lr)
        res["train_s"] = time.time() - t0
        res["loss"] = [float(v) for v in hist]
        _log(f"[train] loss {hist[0]:.4f} -> {hist[-1]:.4f} in {res['train_s']:.1f} s")
        if a.weights_out:
            np.savez(a.weights_out, weights=w.cpu().numpy(), loss=hist)
    if a.eval:
        rows = evaluate(w, a.eval_base, range(cfg["eval_seed0"], cfg["eval_seed0"] + a.eval), max_iter=a.max_iter)
        res["summary"] = summarize(rows)
        res["rows"] = rows
        _log(json.dumps(res["summary"]))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
