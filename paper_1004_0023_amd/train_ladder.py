"""Generate training data, train and evaluate the ladder network on the GPU.

    python -m paper_1004_0023_amd.train_ladder scan [--from 0 --to 4096] [--slope S]
    python -m paper_1004_0023_amd.train_ladder fit
    python -m paper_1004_0023_amd.train_ladder eval

Instances are drawn like the batched workload (N ~ U[32,512], d-regular with
d ~ U{4..8}, M in {32,64,128}, R in {16,32,64}, T in [0.1, 3.0], Gamma = 1) from their
own seeds: training instances 0 .. 4095, held-out instances 4096 .. 4351.

scan: the sampler measures round trips per sweep of every training instance under each
      linear Trotter-coupling mixing profile of the scan grid (levels x slopes, see
      ladder.py); results accumulate in the scan file and finished cells are skipped,
      so the scan can be split over several runs.
fit:  per-instance target profile from the scan, evaluated at the 64 knots; the network
      is fitted with the library's FP32 kernels and saved.
eval: held-out instances under the geometric ladder, the learned ladders, the best
      single constant lambda and the best single profile of the training scan, all for
      the same number of sweeps; the report gives measured round trips per sweep (with
      paired bootstrap intervals), swap-rate-predicted round trips and minimum pair
      acceptance.
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
    """rates[instance][slope][level] (NaN where not yet scanned) and the sweeps per
    measurement.  A file from before the slope axis holds the slope-0 cells only."""
    shape = (N_TRAIN, len(L.SCAN_SLOPES), len(L.SCAN_LAMBDAS))
    rates = np.full(shape, np.nan)
    if not os.path.exists(path):
        return rates, 0
    with np.load(path, allow_pickle=False) as f:
        if tuple(f["lams"]) != tuple(L.SCAN_LAMBDAS):
            raise ValueError(f"{path} was scanned with other levels")
        slopes = tuple(f["slopes"]) if "slopes" in f else (0.0,)
        stored = f["rates"].reshape(N_TRAIN, len(slopes), len(L.SCAN_LAMBDAS))
        for j, sl in enumerate(slopes):
            if sl not in L.SCAN_SLOPES:
                raise ValueError(f"{path} holds slope {sl}, not one of {L.SCAN_SLOPES}")
            rates[:, L.SCAN_SLOPES.index(sl)] = stored[:, j]
        return rates, int(f["sweeps"])


def save_scan(path: str, rates: np.ndarray, sweeps: int):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, rates=rates, lams=np.asarray(L.SCAN_LAMBDAS),
             slopes=np.asarray(L.SCAN_SLOPES), sweeps=np.int64(sweeps))


def phase_scan(args):
    rates, sweeps = load_scan(args.scan_file)
    if sweeps and sweeps != args.scan_sweeps:
        raise ValueError(f"{args.scan_file} holds scans of {sweeps} sweeps")
    cycles = args.scan_sweeps // K
    slopes = L.SCAN_SLOPES if args.slope is None else (args.slope,)
    t0 = time.time()
    for sl in slopes:
        j = L.SCAN_SLOPES.index(sl)
        for off in range(args.idx_from, args.idx_to, args.chunk):
            n = min(args.chunk, args.idx_to - off)
            if np.all(np.isfinite(rates[off:off + n, j])):
                continue
            rates[off:off + n, j] = L.scan(draw(off, n), SEED0 + off, K, cycles, slope=sl)
            save_scan(args.scan_file, rates, args.scan_sweeps)
            log(f"slope {sl}: scanned instances {off}..{off + n - 1} ({time.time() - t0:.0f} s); "
                f"mean rates {np.round(rates[off:off + n, j].mean(0) * 1e4, 3)} x1e-4")


def targets_from_scan(rates: np.ndarray) -> np.ndarray:
    """Per instance (level, slope) of the target profile."""
    return np.array([L.target_profile(r) for r in rates])


def phase_fit(args):
    rates, sweeps = load_scan(args.scan_file)
    if np.isnan(rates).any():
        raise ValueError(f"{args.scan_file} is incomplete")
    tgt = targets_from_scan(rates)
    log(f"targets from {sweeps}-sweep scans: level mean {tgt[:, 0].mean():.3f} "
        f"std {tgt[:, 0].std():.3f}; slope counts "
        f"{ {float(sl): int((tgt[:, 1] == sl).sum()) for sl in L.SCAN_SLOPES} }")
    feats = np.stack([L.features(i) for i in draw(0, N_TRAIN)])
    Q = np.stack([L.profile(a, sl, L.N_KNOTS) for a, sl in tgt])
    model = L.train(feats, Q, steps=args.steps, log=log)
    os.makedirs(os.path.dirname(args.model), exist_ok=True)
    model.save(args.model)
    pred = model.knots(draw(0, N_TRAIN))
    lvl, q_lvl = pred.mean(axis=1), Q.mean(axis=1)
    log(f"saved {args.model}; train fit: rms(pred - target) over knots "
        f"{np.sqrt(((pred - Q) ** 2).mean()):.4f}, corr of mean level "
        f"{np.corrcoef(lvl, q_lvl)[0, 1]:.3f}, mean slope (last - first knot) "
        f"{(pred[:, -1] - pred[:, 0]).mean():.3f} vs target {(Q[:, -1] - Q[:, 0]).mean():.3f}")


def paired(a, b, rng):
    d = a - b
    boots = [d[rng.integers(0, len(d), len(d))].mean() for _ in range(2000)]
    return {"mean_difference": float(d.mean()), "ratio_of_means": float(a.mean() / b.mean()),
            "ci95": [float(np.percentile(boots, 2.5)), float(np.percentile(boots, 97.5))],
            "better": int((d > 0).sum()), "worse": int((d < 0).sum())}


def phase_eval(args):
    rates, sweeps = load_scan(args.scan_file)
    mean = np.nanmean(rates, axis=0)                         # [slope][level]
    lam_const = float(L.SCAN_LAMBDAS[int(np.argmax(mean[L.SCAN_SLOPES.index(0.0)]))])
    j_s, j_l = np.unravel_index(int(np.argmax(mean)), mean.shape)
    best_profile = (float(L.SCAN_LAMBDAS[j_l]), float(L.SCAN_SLOPES[j_s]))
    model = L.LadderModel.load(args.model)
    held = heldout(args.heldout)
    cycles = args.eval_sweeps // K
    seed = SEED0 + 0x5EED
    t0 = time.time()
    runs = {
        "geometric": L.evaluate(held, [0.0] * len(held), seed, K, cycles),
        "learned": L.evaluate(held, model.rung_lambdas(held), seed, K, cycles),
        "best_constant": L.evaluate(held, [lam_const] * len(held), seed, K, cycles),
        "best_profile": L.evaluate(held, [L.profile(*best_profile, i.R) for i in held], seed,
                                   K, cycles),
    }
    log(f"evaluated {len(held)} held-out instances x {len(runs)} ladders x {cycles * K} sweeps "
        f"in {time.time() - t0:.0f} s")
    rng = np.random.default_rng(1)

    def by_R(a):
        return {str(R): float(a[[i.R == R for i in held]].mean()) for R in (16, 32, 64)}

    rt = {k: v[0] for k, v in runs.items()}
    kn = model.knots(held)
    lam_learned = kn.mean(axis=1)
    report = {
        "train_instances": N_TRAIN, "heldout_instances": len(held),
        "scan_lambdas": list(L.SCAN_LAMBDAS), "scan_slopes": list(L.SCAN_SLOPES),
        "scan_sweeps": sweeps, "scan_mean_rates": mean.tolist(),
        "sweeps_per_instance": cycles * K, "sweeps_per_exchange": K,
        "best_constant_lambda": lam_const,
        "best_profile": {"level": best_profile[0], "slope": best_profile[1]},
        "learned_lambda": {"mean": float(lam_learned.mean()), "min": float(lam_learned.min()),
                           "max": float(lam_learned.max()),
                           "slope_last_minus_first_knot": float((kn[:, -1] - kn[:, 0]).mean())},
        "measured_round_trips_per_sweep": {
            **{k: float(v.mean()) for k, v in rt.items()},
            "by_R": {k: by_R(v) for k, v in rt.items()},
            "learned_vs_geometric": paired(rt["learned"], rt["geometric"], rng),
            "learned_vs_best_constant": paired(rt["learned"], rt["best_constant"], rng),
            "learned_vs_best_profile": paired(rt["learned"], rt["best_profile"], rng)},
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
    ap.add_argument("--slope", type=float, default=None,
                    help="scan only this slope of the grid (default: every slope)")
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
