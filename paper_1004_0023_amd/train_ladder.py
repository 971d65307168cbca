"""Generate training data, train and evaluate the ladder network on the GPU.

    python -m paper_1004_0023_amd.train_ladder scan [--from 0 --to 4096]
    python -m paper_1004_0023_amd.train_ladder fit
    python -m paper_1004_0023_amd.train_ladder eval

Instances are drawn like the batched workload (N ~ U[32,512], d-regular with
d ~ U{4..8}, M in {32,64,128}, R in {16,32,64}, T in [0.1, 3.0], Gamma = 1) from their
own seeds: training instances 0 .. 4095, held-out instances 4096 .. 4351.

scan: the sampler measures round trips per sweep of every training instance under each
      constant Trotter-coupling mixing lambda (see ladder.py); results accumulate in
      the scan file, so the scan can be split over several runs.
fit:  per-instance target lambda from the scan, the same target at all 64 knots; the
      network is fitted with the library's FP32 kernels and saved.
eval: held-out instances under the geometric ladder, the learned ladders and the best
      single constant lambda of the training scan, all for the same number of sweeps;
      the report gives measured round trips per sweep (with paired bootstrap intervals),
      swap-rate-predicted round trips and minimum pair acceptance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1004_0023_amd import ladder as L  # noqa: E402

CONFIG_ID = 5
K = 10
N_TRAIN = 4096
N_HELD = 256
SEED0 = 0x10040023_00000000 + CONFIG_ID
DATA = os.path.join(HERE, "data")
SCAN_FILE = os.path.join(DATA, "ladder_scan.npz")
MODEL_FILE = os.path.join(DATA, "ladder_mlp.npz")
REPORT_FILE = os.path.join(DATA, "ladder_eval.json")


def log(msg):
    print(f"[train_ladder {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def draw(idx_from: int, count: int):
    import workloads as W
    return [W.config3_instance(i, config=CONFIG_ID) for i in range(idx_from, idx_from + count)]


def heldout(count: int = N_HELD):
    return draw(N_TRAIN, count)


def load_scan(path: str):
    if not os.path.exists(path):
        return (np.full((N_TRAIN, len(L.SCAN_LAMBDAS)), np.nan), 0)
    with np.load(path, allow_pickle=False) as f:
        if tuple(f["lams"]) != tuple(L.SCAN_LAMBDAS):
            raise ValueError(f"{path} was scanned with other lambdas")
        return f["rates"].copy(), int(f["sweeps"])


def phase_scan(args):
    rates, sweeps = load_scan(args.scan_file)
    if sweeps and sweeps != args.scan_sweeps:
        raise ValueError(f"{args.scan_file} holds scans of {sweeps} sweeps")
    cycles = args.scan_sweeps // K
    t0 = time.time()
    for off in range(args.idx_from, args.idx_to, args.chunk):
        n = min(args.chunk, args.idx_to - off)
        chunk = draw(off, n)
        rates[off:off + n] = L.scan(chunk, SEED0 + off, K, cycles)
        os.makedirs(os.path.dirname(args.scan_file), exist_ok=True)
        np.savez(args.scan_file, rates=rates, lams=np.asarray(L.SCAN_LAMBDAS),
                 sweeps=np.int64(args.scan_sweeps))
        log(f"scanned instances {off}..{off + n - 1} ({time.time() - t0:.0f} s); "
            f"mean rates {np.round(rates[off:off + n].mean(0) * 1e4, 3)} x1e-4")


def targets_from_scan(rates: np.ndarray) -> np.ndarray:
    return np.array([L.target_lambda(r) for r in rates])


def phase_fit(args):
    rates, sweeps = load_scan(args.scan_file)
    if np.isnan(rates).any():
        raise ValueError(f"{args.scan_file} is incomplete")
    lam = targets_from_scan(rates)
    log(f"targets: mean {lam.mean():.3f}, std {lam.std():.3f} from {sweeps}-sweep scans")
    feats = np.stack([L.features(i) for i in draw(0, N_TRAIN)])
    Q = np.repeat(lam[:, None], L.N_KNOTS, axis=1)
    model = L.train(feats, Q, steps=args.steps, log=log)
    os.makedirs(os.path.dirname(args.model), exist_ok=True)
    model.save(args.model)
    pred = model.knots(draw(0, N_TRAIN)).mean(axis=1)
    log(f"saved {args.model}; train fit: rms(pred - target) {np.sqrt(((pred - lam) ** 2).mean()):.4f}, "
        f"corr {np.corrcoef(pred, lam)[0, 1]:.3f}")


def paired(a, b, rng):
    d = a - b
    boots = [d[rng.integers(0, len(d), len(d))].mean() for _ in range(2000)]
    return {"mean_difference": float(d.mean()), "ratio_of_means": float(a.mean() / b.mean()),
            "ci95": [float(np.percentile(boots, 2.5)), float(np.percentile(boots, 97.5))],
            "better": int((d > 0).sum()), "worse": int((d < 0).sum())}


def phase_eval(args):
    rates, sweeps = load_scan(args.scan_file)
    best_c = int(np.argmax(np.nanmean(rates, axis=0)))
    lam_const = float(L.SCAN_LAMBDAS[best_c])
    model = L.LadderModel.load(args.model)
    held = heldout(args.heldout)
    cycles = args.eval_sweeps // K
    seed = SEED0 + 0x5EED
    t0 = time.time()
    runs = {
        "geometric": L.evaluate(held, [0.0] * len(held), seed, K, cycles),
        "learned": L.evaluate(held, model.rung_lambdas(held), seed, K, cycles),
        "best_constant": L.evaluate(held, [lam_const] * len(held), seed, K, cycles),
    }
    log(f"evaluated {len(held)} held-out instances x 3 ladders x {cycles * K} sweeps "
        f"in {time.time() - t0:.0f} s")
    rng = np.random.default_rng(1)

    def by_R(a):
        return {str(R): float(a[[i.R == R for i in held]].mean()) for R in (16, 32, 64)}

    rt = {k: v[0] for k, v in runs.items()}
    lam_learned = model.knots(held).mean(axis=1)
    report = {
        "train_instances": N_TRAIN, "heldout_instances": len(held),
        "scan_lambdas": list(L.SCAN_LAMBDAS), "scan_sweeps": sweeps,
        "sweeps_per_instance": cycles * K, "sweeps_per_exchange": K,
        "best_constant_lambda": lam_const,
        "learned_lambda": {"mean": float(lam_learned.mean()), "min": float(lam_learned.min()),
                           "max": float(lam_learned.max())},
        "measured_round_trips_per_sweep": {
            **{k: float(v.mean()) for k, v in rt.items()},
            "by_R": {k: by_R(v) for k, v in rt.items()},
            "learned_vs_geometric": paired(rt["learned"], rt["geometric"], rng),
            "learned_vs_best_constant": paired(rt["learned"], rt["best_constant"], rng)},
        "predicted_round_trips_per_exchange": {k: float(v[1].mean()) for k, v in runs.items()},
        "min_pair_acceptance": {k: float(v[2].mean()) for k, v in runs.items()},
        "count_by_R": {str(R): int(sum(i.R == R for i in held)) for R in (16, 32, 64)},
    }
    os.makedirs(os.path.dirname(args.report), exist_ok=True)
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(report))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("phase", choices=["scan", "fit", "eval"])
    ap.add_argument("--from", dest="idx_from", type=int, default=0)
    ap.add_argument("--to", dest="idx_to", type=int, default=N_TRAIN)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--scan-sweeps", type=int, default=40000)
    ap.add_argument("--eval-sweeps", type=int, default=100000)
    ap.add_argument("--heldout", type=int, default=N_HELD)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--scan-file", default=SCAN_FILE)
    ap.add_argument("--model", default=MODEL_FILE)
    ap.add_argument("--report", default=REPORT_FILE)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    {"scan": phase_scan, "fit": phase_fit, "eval": phase_eval}[args.phase](args)


if __name__ == "__main__":
    main()
