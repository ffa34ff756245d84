"""Train and evaluate the learned warm start on the GPU.

Data: densities are K in {4..12} Gaussian-blob mixtures on 128^3 grids over
[-1,1]^3 (training seeds 10000.., held-out seeds 20000..); targets are the
potentials of the damped solver run to convergence in FP64 (1500 substeps,
residual checked), restricted to 64^3.  Training: Adam on the mean-squared
error of the scaled correction to the coarse cue and of dphi/dt (target 0),
plus a weighted squared 7-point Laplacian of the correction's error (the
residual the solver starts from); the weight is chosen on validation seeds
15000.. among the values given.
Evaluation: substeps of the damped FP32 solver to R_b < 1e-4 from the zero
start, the coarse cue alone, the learned start (zero start as fallback) and the
restricted exact solution (the best any 64^3 predictor prolonged to 128^3 can
do).  Writes the weights (.npz) and a JSON report.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print(*a, flush=True)


def densities(seeds, n, device):
    import torch

    import workloads

    return [workloads.blob_density_torch(n, workloads.warmstart_blobs(s), device, torch.float32) for s in seeds]


def build(seeds, n, feats, device, chunk, target_steps):
    """(planar inputs, coarse phi at n/2, scale, exact phi at n/2, exact phi at n (fp32), residuals)."""
    import torch

    from paper_1602_05700_amd import hgs, warmstart as ws

    P, C, S, E2, E1, R = [], [], [], [], [], []
    for i in range(0, len(seeds), chunk):
        rho = torch.stack(densities(seeds[i:i + chunk], n, device))
        planar, phi2c, scale = feats.inputs(rho)
        phis, res = ws.converged_phi(list(rho), n, device, steps=target_steps)
        ex = torch.stack([p.float() for p in phis])
        ex2 = torch.empty_like(phi2c)
        hgs.nn_restrict2(ex, ex2)
        P.append(planar)
        C.append(phi2c)
        S.append(scale)
        E2.append(ex2)
        E1.append(ex)
        R.extend(res)
        log(f"[data] {min(i + chunk, len(seeds))}/{len(seeds)} samples, max R_b of targets {max(res):.2e}")
    return (torch.cat(P), torch.cat(C), torch.cat(S), torch.cat(E2), torch.cat(E1), R)


def train(net, P, tgt, args, lap_w, dev, log_prefix=""):
    """Adam over shuffled mini-batches with a cosine learning-rate schedule;
    loss = mean-squared error + lap_w * squared Laplacian of the phi error."""
    import torch

    from paper_1602_05700_amd import hgs, warmstart as ws

    loss_dev = torch.zeros(1, dtype=torch.float64, device=dev)
    parts = torch.empty(hgs.NN_MSE_PARTIALS, dtype=torch.float64, device=dev)
    B = args.batch
    scratch = torch.empty(B * P[0, 0].numel(), dtype=torch.float32, device=dev)
    wsb = None
    curve = []
    g = torch.Generator().manual_seed(1)
    steps = 0
    t1 = time.time()
    for ep in range(args.epochs):
        perm = torch.randperm(P.shape[0], generator=g)
        lr = args.lr * 0.5 * (1 + np.cos(np.pi * ep / args.epochs))
        tot = 0.0
        for i in range(0, P.shape[0] - B + 1, B):
            idx = perm[i:i + B].to(dev)
            x = ws.pack(P[idx].contiguous())
            acts = net.forward(x)
            grad = torch.empty_like(x)
            hgs.nn_lapmse(acts[-1], tgt[idx].contiguous(), grad, loss_dev, parts, scratch, ch=0, w=lap_w)
            grads, wsb = net.backward(acts, grad, wsb)
            net.adam_step(grads, lr)
            tot += loss_dev.item() / (B * ws.OUT_CH * x[0, ..., 0].numel())
            steps += 1
        curve.append(tot / (P.shape[0] // B))
        log(f"[train{log_prefix}] epoch {ep} lr {lr:.2e} loss {curve[-1]:.4e}")
    torch.cuda.synchronize()
    return {"epochs": args.epochs, "batch": B, "steps": steps, "seconds": time.time() - t1, "loss_curve": curve,
            "lap_w": lap_w}


def evaluate(net, data, seeds, n, feats, args, dev, controls=True, tag="eval", criteria=()):
    """Substeps to R_b < tol from the zero start, the coarse cue alone, the
    learned start (zero start as fallback) and the restricted exact solution.
    criteria: further criteria ("R_f" in FP64 storage, whose FP32 floor at
    128^3 lies above 1e-4; "E" against the converged target) whose substep
    counts from the zero and the learned start are recorded as well."""
    import torch

    from paper_1602_05700_amd import hgs, warmstart as ws

    Pt, Ct, St, E2t, E1t, _ = data
    rows = []
    for i, seed in enumerate(seeds):
        rho = densities([seed], n, dev)[0]
        exact = E1t[i]
        nrm = exact.double().norm().item()
        zero = ws.steps_to_tolerance(rho, n, args.tol)
        phi, pd = ws.predict_fine(net, Pt[i:i + 1].contiguous(), Ct[i:i + 1].contiguous(), St[i:i + 1], n)
        learned = ws.steps_to_tolerance(rho, n, args.tol, start=(phi[0], pd[0]))
        fallback = not learned[3]  # start_solver fell back to the zero start
        e = lambda f: float((f.double() - exact.double()).norm().item() / nrm)
        row = {"seed": seed, "zero": zero[0], "learned": learned[0],
               "learned_raw": learned[0], "fallback": bool(fallback),
               "R0": {"zero": zero[1], "learned": learned[1]}, "E0": {"learned": e(phi[0])}}
        if controls:
            # coarse cue alone (non-learned control)
            pc = torch.empty((1, n, n, n), dtype=torch.float32, device=dev)
            hgs.nn_prolong2(Ct[i:i + 1].contiguous(), pc)
            coarse = ws.steps_to_tolerance(rho, n, args.tol, start=(pc[0], torch.zeros_like(pc[0])))
            # ideal 2x-coarse predictor: restricted exact solution, prolonged
            pi = torch.empty((1, n, n, n), dtype=torch.float32, device=dev)
            hgs.nn_prolong2(E2t[i:i + 1].contiguous(), pi)
            ideal = ws.steps_to_tolerance(rho, n, args.tol, start=(pi[0], torch.zeros_like(pi[0])))
            row.update({"coarse": coarse[0], "ideal": ideal[0]})
            row["R0"].update({"coarse": coarse[1], "ideal": ideal[1]})
            row["E0"].update({"coarse": e(pc[0]), "ideal": e(pi[0])})
        for crit in criteria:
            kw = {"storage": "f64"} if crit == "R_f" else {}
            kw.update({"metric": crit, "ref": exact if crit == "E" else None})
            z_c = ws.steps_to_tolerance(rho, n, args.tol, **kw)
            l_c = ws.steps_to_tolerance(rho, n, args.tol, start=(phi[0], pd[0]), **kw)
            row[f"zero_{crit}"], row[f"learned_{crit}"] = z_c[0], l_c[0]
            row["R0"].update({f"zero_{crit}": z_c[1], f"learned_{crit}": l_c[1]})
        rows.append(row)
        log(f"[{tag}] seed {seed}: zero {zero[0]} learned {learned[0]}{' (fallback)' if fallback else ''}"
            + (f" coarse {row['coarse']} ideal {row['ideal']}" if controls else "")
            + f"; R0 learned {learned[1]:.2e}, E0 learned {row['E0']['learned']:.2e}")
    return rows


def summarise(rows, cc):
    def stats(key, extra=0.0):
        v = np.array([r[key] for r in rows], dtype=float) + extra
        return {"median": float(np.median(v)), "q25": float(np.percentile(v, 25)),
                "q75": float(np.percentile(v, 75))}

    z = stats("zero")
    out = {"samples": len(rows), "steps_zero": z, "steps_learned": stats("learned", cc),
           "ratio_learned": z["median"] / stats("learned", cc)["median"],
           "fallback_rate": float(np.mean([r["fallback"] for r in rows])),
           "R0_median": {k: float(np.median([r["R0"][k] for r in rows])) for k in rows[0]["R0"]},
           "E0_median": {k: float(np.median([r["E0"][k] for r in rows])) for k in rows[0]["E0"]}}
    if "coarse" in rows[0]:
        out.update({"steps_coarse": stats("coarse", cc), "steps_ideal": stats("ideal"),
                    "ratio_coarse": z["median"] / stats("coarse", cc)["median"],
                    "ratio_ideal": z["median"] / stats("ideal")["median"]})
    for crit in ("R_f", "E"):
        if f"zero_{crit}" in rows[0]:
            zc, lc = stats(f"zero_{crit}"), stats(f"learned_{crit}", cc)
            out[f"criterion_{crit}"] = {"steps_zero": zc, "steps_learned": lc,
                                        "ratio": zc["median"] / lc["median"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=2048)
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lap-w", default="8",
                    help="comma-separated Laplacian loss weights; the best on the validation seeds is kept")
    ap.add_argument("--coarse-steps", type=int, default=200)
    ap.add_argument("--coarse", choices=("direct", "relax"), default="direct",
                    help="coarse cue: direct Poisson solve, or coarse-steps damped substeps")
    ap.add_argument("--target-steps", type=int, default=1500)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1602_05700_amd", "warmstart_weights.npz"))
    ap.add_argument("--report", default="warmstart_report.json")
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--criteria", default="R_f,E",
                    help="criteria besides R_b counted on the held-out densities (comma-separated, or empty)")
    args = ap.parse_args()

    import torch

    from paper_1602_05700_amd import warmstart as ws

    dev = torch.device("cuda:0")
    n = args.n
    feats = ws.Features(n, dev, coarse_steps=args.coarse_steps, coarse=args.coarse)
    cc = feats.coarse_cost_fine_steps
    t0 = time.time()
    report = {"n": n, "tol": args.tol, "coarse_steps": args.coarse_steps, "coarse_cost_fine_steps": cc,
              "args": vars(args)}
    if not args.eval_only:
        train_seeds = list(range(10000, 10000 + args.train))
        P, C, S, E2, _, R = build(train_seeds, n, feats, dev, args.chunk, args.target_steps)
        report["target_max_Rb"] = float(max(R))
        corr = (E2 - C) / S.view(-1, 1, 1, 1)
        out_scale = float(1.0 / corr.std().item())
        tgt = torch.zeros((P.shape[0], ws.OUT_CH) + tuple(P.shape[2:]), dtype=torch.float32, device=dev)
        tgt[:, 0] = corr * out_scale
        del C, E2, corr
        log(f"[train] {P.shape[0]} samples, out_scale {out_scale:.3e}, data {time.time() - t0:.1f} s")
        val_seeds = list(range(15000, 15000 + args.val))
        val = build(val_seeds, n, feats, dev, args.chunk, args.target_steps)
        best = None
        report["sweep"] = []
        for w in [float(v) for v in args.lap_w.split(",")]:
            net = ws.Net.create(dev, seed=0)
            net.out_scale = out_scale
            net.coarse_steps = args.coarse_steps
            info = train(net, P, tgt, args, w, dev, log_prefix=f" w={w:g}")
            vs = summarise(evaluate(net, val, val_seeds, n, feats, args, dev, controls=False, tag=f"val w={w:g}"),
                           cc)
            info["val"] = vs
            report["sweep"].append(info)
            log(f"[val] w={w:g}: median learned steps {vs['steps_learned']['median']:.1f}, "
                f"zero {vs['steps_zero']['median']}, ratio {vs['ratio_learned']:.2f}x")
            if best is None or vs["steps_learned"]["median"] < best[0]:
                best = (vs["steps_learned"]["median"], w, net)
        report["chosen_lap_w"] = best[1]
        best[2].save(args.weights)
        del P, S, tgt
    net = ws.Net.load(args.weights, dev)

    # ---- held-out evaluation
    test_seeds = list(range(20000, 20000 + args.test))
    data = build(test_seeds, n, feats, dev, args.chunk, args.target_steps)
    crits = tuple(c for c in args.criteria.split(",") if c)
    rows = evaluate(net, data, test_seeds, n, feats, args, dev, controls=True, criteria=crits)
    ev = summarise(rows, cc)
    ev["target_max_Rb"] = float(max(data[5]))
    ev["rows"] = rows
    report["eval"] = ev
    report["seconds"] = time.time() - t0
    os.makedirs(os.path.dirname(os.path.abspath(args.report)), exist_ok=True)
    json.dump(report, open(args.report, "w"), indent=1)
    log(f"[eval] median steps: zero {ev['steps_zero']['median']} coarse {ev['steps_coarse']['median']:.1f} "
        f"learned {ev['steps_learned']['median']:.1f} ideal {ev['steps_ideal']['median']}; "
        f"gain learned {ev['ratio_learned']:.2f}x coarse {ev['ratio_coarse']:.2f}x ideal {ev['ratio_ideal']:.2f}x; "
        f"fallback {ev['fallback_rate']:.2f}")
    for crit in crits:
        c = ev[f"criterion_{crit}"]
        log(f"[eval] {crit} < {args.tol:g}: median steps zero {c['steps_zero']['median']} "
            f"learned {c['steps_learned']['median']:.1f}, gain {c['ratio']:.2f}x")


if __name__ == "__main__":
    main()
