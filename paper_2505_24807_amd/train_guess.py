"""Train the learned Davidson starting space on the GPU and evaluate it.

    python -m paper_2505_24807_amd.train_guess [--train 2000] [--epochs 30]
        [--out paper_2505_24807_amd/guess_net.bin] [--eval 50] [--report path.json]

Training set: synthetic.molecules.guess_training_molecule(seed) for seeds
0 .. train-1 (polyenes and water clusters, 10-80 atoms).  Their 10 lowest CIS
roots come from the library's own batched Davidson (FP64 products); the
network is trained on them by the library's kernels (seqx_mlp_train) and saved
with seqx_mlp_save.  Evaluation: held-out molecules guess_eval_molecule(100000
+ s) (200-600 atoms), CIS, 10 roots, FP64, with three starting spaces: the 2K
smallest-gap unit vectors, the 4K smallest-gap pairs (P-space) and the 4K
best-scored pairs (learned P-space).  Reported per molecule: Davidson
iterations, solve time, and the time after which all 10 roots stay within
1e-4 eV of the converged values.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2505_24807_amd import seqx  # noqa: E402
from synthetic import molecules, params  # noqa: E402

K = 10


def time_to(t, om, ref, thr=1e-4):
    ok = np.all(np.abs(om - ref[None, :]) <= thr, axis=1)
    bad = np.nonzero(~ok)[0]
    first = 0 if bad.size == 0 else int(bad[-1]) + 1
    return float(t[first]) if first < len(t) else None


def evaluate(ctx, seeds, log=print):
    rows = []
    names = {seqx.GUESS_GAP: "gap", seqx.GUESS_GAP_PSPACE: "gap_pspace", seqx.GUESS_LEARNED: "learned_pspace"}
    for s in seeds:
        mol = molecules.guess_eval_molecule(s)
        job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
        n, o, v = job.dims()
        row = {"seed": s, "atoms": int(mol.natoms), "nov": o * v}
        runs = {}
        for g in (seqx.GUESS_GAP, seqx.GUESS_GAP_PSPACE, seqx.GUESS_LEARNED):
            job.solve(theory=seqx.CIS, nroots=K, tol=1e-6, max_iter=400, guess=g)
            st = job.stats()
            t, om = job.history()
            runs[g] = (job.results().omega_eV, st.dav_iterations, st.t_davidson_s, t, om, st.n_sigma)
        ref = runs[seqx.GUESS_GAP][0]
        for g, (om_f, it, ts, t, om, ns) in runs.items():
            row[names[g]] = {"iterations": it, "seconds": round(ts, 4), "n_sigma": ns,
                             "time_to_1e-4_eV": time_to(t, om, ref),
                             "max_abs_dev_eV": float(np.abs(om_f - ref).max())}
        job.free()
        rows.append(row)
        log(json.dumps(row), flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=2505)
    ap.add_argument("--out", default=os.path.join(HERE, "guess_net.bin"))
    ap.add_argument("--eval", type=int, default=50)
    ap.add_argument("--eval-only", action="store_true", help="load --out instead of training")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    ctx = seqx.Context(0)
    ctx.set_params(*seqx.params_table(params.load()))
    report = {}
    if not args.eval_only:
        t0 = time.time()
        mols = [molecules.guess_training_molecule(s) for s in range(args.train)]
        natoms, Z, xyz = molecules.concat(mols)
        print(f"[train] {len(mols)} molecules, {int(natoms.sum())} atoms: prepare", flush=True)
        job = ctx.prepare(list(natoms), Z, xyz)
        t1 = time.time()
        print(f"[train] prepared in {t1 - t0:.1f} s; batched CIS K={K}", flush=True)
        job.solve(theory=seqx.CIS, nroots=K, tol=1e-5, max_iter=400, precision=seqx.FP64, batched=True)
        st = job.stats()
        t2 = time.time()
        print(f"[train] labels in {t2 - t1:.1f} s ({st.dav_iterations} iterations, {st.n_sigma} sigma vectors)",
              flush=True)
        log = job.mlp_train(epochs=args.epochs, batch=args.batch, lr=args.lr, seed=args.seed, init=True)
        job.free()
        print(f"[train] {args.epochs} epochs in {log['seconds']:.1f} s; loss {log['loss'][0]:.4f} -> "
              f"{log['loss'][-1]:.4f}", flush=True)
        ctx.mlp_save(args.out)
        report["training"] = {"molecules": len(mols), "prepare_s": round(t1 - t0, 2), "labels_s": round(t2 - t1, 2),
                              "label_iterations": st.dav_iterations, "train_s": round(log["seconds"], 2),
                              "loss": [round(x, 5) for x in log["loss"]]}
    else:
        ctx.mlp_load(args.out)
    if args.eval > 0:
        rows = evaluate(ctx, [100000 + s for s in range(args.eval)])
        agg = {}
        for key in ("gap", "gap_pspace", "learned_pspace"):
            its = [r[key]["iterations"] for r in rows]
            tt = [r[key]["time_to_1e-4_eV"] for r in rows if r[key]["time_to_1e-4_eV"] is not None]
            agg[key] = {"mean_iterations": float(np.mean(its)), "mean_seconds": float(np.mean([r[key]["seconds"] for r in rows])),
                        "mean_time_to_1e-4_eV": float(np.mean(tt)) if tt else None,
                        "max_abs_dev_eV": max(r[key]["max_abs_dev_eV"] for r in rows)}
        report["evaluation"] = {"molecules": len(rows), "summary": agg, "rows": rows}
        print(json.dumps({"summary": agg}), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
