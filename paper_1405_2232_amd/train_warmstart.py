"""Train the warm-start network on solver trajectories and evaluate it.

    python -m paper_1405_2232_amd.train_warmstart --out DIR [--physical]
        [--stage all|train|eval] [--weights FILE] [--init-weights FILE]

(defaults: 64 x 64 cases with 1-3 droplets, 1024 training solves to a
1e-7 residual, 120 epochs, 64 held-out cases evaluated at 1e-8; with
--physical every solve, screen and evaluation starts at rest in the
forcing scheme's velocity; --stage train stops after writing the
parameters, --stage eval evaluates given parameters)

Steps (all on the GPU):
  1. solve the training cases (seeds 0..train-1) to the residual target in
     batches (FP64 storage);
  2. train the U-Net on (initial fields -> steady fields);
  3. solve the held-out cases (seeds 100000..) cold and warm (prediction
     screened by its one-step residual, cold start where rejected), and
     report steps and wall time to the target for both, the warm time
     including the network's inference.
Writes DIR/warmstart_<n>.npz (the trained parameters; the benchmark loads
paper_1405_2232_amd/warmstart_64.npz) and DIR/warmstart_eval.json.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--train", type=int, default=1024)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--batch-solve", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--target", type=float, default=1e-8, help="residual target of the evaluation")
    ap.add_argument("--train-target", type=float, default=1e-7, help="residual target of the training solves")
    ap.add_argument("--cap", type=int, default=600000)
    ap.add_argument("--train-cap", type=int, default=400000)
    ap.add_argument("--max-drops", type=int, default=3)
    ap.add_argument("--out", default="gpurun_out")
    ap.add_argument("--physical", action="store_true",
                    help="solve, screen and evaluate from the start at rest in the forcing scheme's "
                         "velocity (stored momentum -F/2) instead of zero stored momentum")
    ap.add_argument("--factor", type=float, default=1.0,
                    help="the screen keeps a prediction whose one-step residual is at most this "
                         "multiple of the cold start's")
    ap.add_argument("--stage", choices=("all", "train", "eval"), default="all")
    ap.add_argument("--weights", default=None, help="trained parameters for --stage eval")
    ap.add_argument("--init-weights", default=None,
                    help="start training from these parameters (the network is convolutional, so "
                         "parameters trained on one box size serve another) instead of a fresh init")
    args = ap.parse_args(argv)

    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.warmstart import WarmStart, load_params, solve

    os.makedirs(args.out, exist_ok=True)
    t_all = time.perf_counter()
    test_cases = [inputs.warmstart_case(100000 + s, n=args.n, max_drops=args.max_drops) for s in range(args.test)]
    if args.stage == "eval":
        ws = WarmStart(args.n, params=load_params(args.weights))
        res = {"n": args.n, "weights": args.weights}
        return _evaluate(args, ws, test_cases, res, t_all)
    train_cases = [inputs.warmstart_case(s, n=args.n, max_drops=args.max_drops) for s in range(args.train)]

    # 1. training trajectories
    steady, keep = [], []
    t0 = time.perf_counter()
    for k in range(0, len(train_cases), args.batch_solve):
        part = train_cases[k:k + args.batch_solve]
        r = solve(part, target=args.train_target, cap=args.train_cap, physical=args.physical, log=log)
        for i, st in enumerate(r["steps"]):
            if st is not None:
                keep.append(k + i)
                steady.append(r["fields"][i])
        log("solved %d/%d training cases, %d converged, %.1f s" % (
            min(k + args.batch_solve, len(train_cases)), len(train_cases), len(keep), time.perf_counter() - t0))
    gen_s = time.perf_counter() - t0

    # 2. training
    ws = WarmStart(args.n, params=load_params(args.init_weights) if args.init_weights else None)
    data = ws.dataset([train_cases[i] for i in keep], steady)
    t0 = time.perf_counter()
    hist = ws.train(data, epochs=args.epochs, lr=args.lr, log=log)
    train_s = time.perf_counter() - t0
    del data
    np.savez(os.path.join(args.out, "warmstart_%d.npz" % args.n), **{
        k: v.astype(np.float32) for k, v in ws.net.get_params().items()})

    res = {"n": args.n, "train_cases": args.train, "train_converged": len(keep),
           "train_target": args.train_target, "train_cap": args.train_cap, "max_drops": args.max_drops,
           "epochs": args.epochs, "loss": hist, "data_generation_s": round(gen_s, 1),
           "training_s": round(train_s, 1), "physical": args.physical, "init_weights": args.init_weights}
    if args.stage == "train":
        with open(os.path.join(args.out, "warmstart_train.json"), "w") as fp:
            json.dump(res, fp, indent=1)
        log(json.dumps(res))
        return 0
    return _evaluate(args, ws, test_cases, res, t_all)


def _evaluate(args, ws, test_cases, res, t_all):
    """Held-out evaluation: cold, then warm (inference and screening timed
    in), then every prediction unscreened; all from the same kind of start."""
    import time
    from paper_1405_2232_amd.warmstart import screen, solve
    ph = args.physical
    cold = solve(test_cases, target=args.target, cap=args.cap, keep=False, physical=ph, log=log)
    t0 = time.perf_counter()
    preds = ws.predict(test_cases)
    inits, rp, rc = screen(test_cases, preds, factor=args.factor, physical=ph)
    infer_s = time.perf_counter() - t0
    log("screened: %d of %d predictions kept" % (sum(p is not None for p in inits), len(inits)))
    warm = solve(test_cases, inits=inits, target=args.target, cap=args.cap, keep=False, physical=ph, log=log)
    raw = solve(test_cases, inits=preds, target=args.target, cap=args.cap, keep=False, physical=ph, log=log)
    both = [i for i in range(len(test_cases)) if cold["steps"][i] is not None and warm["steps"][i] is not None]
    cs = np.array([cold["steps"][i] for i in both], dtype=float)
    wsteps = np.array([warm["steps"][i] for i in both], dtype=float)
    capped = lambda st: int(sum(args.cap if s is None else s for s in st))  # noqa: E731
    res.update({
        "test_cases": args.test, "target": args.target, "cap": args.cap, "physical": ph,
        "screen_factor": args.factor,
        "accepted_predictions": int(sum(p is not None for p in inits)),
        "cold": {"converged": int(sum(s is not None for s in cold["steps"])), "wall_s": round(cold["wall_s"], 2),
                 "steps_capped_total": capped(cold["steps"]),
                 "mean_steps_on_both": float(cs.mean()) if len(cs) else None},
        "warm": {"converged": int(sum(s is not None for s in warm["steps"])),
                 "wall_s": round(warm["wall_s"] + infer_s, 2), "inference_and_screen_s": round(infer_s, 2),
                 "steps_capped_total": capped(warm["steps"]),
                 "mean_steps_on_both": float(wsteps.mean()) if len(wsteps) else None},
        "step_ratio_warm_over_cold_on_both": float(wsteps.sum() / cs.sum()) if len(cs) else None,
        "unscreened": {"converged": int(sum(s is not None for s in raw["steps"])),
                       "wall_s": round(raw["wall_s"], 2), "steps_capped_total": capped(raw["steps"]),
                       "invalid_predictions": raw["invalid_inits"]},
        "cold_steps": cold["steps"], "warm_steps": warm["steps"], "unscreened_steps": raw["steps"],
        "predicted_residual": rp, "cold_residual": rc,
        "total_s": round(time.perf_counter() - t_all, 1),
    })
    with open(os.path.join(args.out, "warmstart_eval.json"), "w") as fp:
        json.dump(res, fp, indent=1)
    log(json.dumps({k: v for k, v in res.items() if not k.endswith("_steps") and k not in
                    ("predicted_residual", "cold_residual", "loss")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
