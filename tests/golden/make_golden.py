"""Write the stored end-of-run digests of the oracle for the long parity cases.

    python tests/golden/make_golden.py [config3 | config4 | config2 | all] [--threads T]

Each case runs the CPU oracle (and nothing else: the inputs come from the seeded
generators in ``workloads``) over the problem shapes of the paper's workloads at the
lengths the GPU parity tests use, and stores, per instance, a SHA-256 digest of the final
state: spins [R][M][N] by replica slot, E_cl, C, the permutation, labels, swap counts,
round trips, per-rung accumulators and visit counts, and the counters t, e, n_acc.  The
digest only serialises the state; it holds none of the sampler's arithmetic.

    config3  all 512 instances of the batched workload, 16 PT cycles of 10 sweeps (one
             replay of the 16-cycle graph that pt_run captures)
    config4  the 8x8x16 lattice (N=1024, M=256, R=64), 100 cycles of 10 sweeps
    config2  N=128, M=64, R=32, 1000 cycles of 10 sweeps

A config-4 run takes about 20 minutes on one core, config 3 about 50 core-minutes
(spread over threads: the oracle's calls release the GIL).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# observables in digest order (sumCt is left out: these cases run without correlations)
DIGEST_KEYS = ("E_cl", "C", "rung_of", "replica_of", "acc", "att", "roundtrips", "label",
               "sumE", "sumC", "sumE2", "sumC2", "nup", "ndown")

CASES = {
    "config3": dict(config=3, cycles=16),
    "config4": dict(config=4, cycles=100),
    "config2": dict(config=2, cycles=1000),
}


def state_digest(spins: np.ndarray, obs: dict) -> str:
    """SHA-256 of a final state: spins as int8 bytes, then every observable in
    DIGEST_KEYS as little-endian int64, then t, e and n_acc."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(spins, dtype=np.int8).tobytes())
    for k in DIGEST_KEYS:
        h.update(np.asarray(obs[k]).astype("<i8").tobytes())
    h.update(np.asarray([obs["t"], obs["e"], obs["n_acc"]], dtype="<i8").tobytes())
    return h.hexdigest()


def golden_path(case: str) -> str:
    return os.path.join(HERE, f"{case}_digests.json")


def load_golden(case: str) -> dict:
    with open(golden_path(case)) as f:
        return json.load(f)


def instances_of(config: int):
    import workloads as W
    return {2: lambda: [W.config2()], 3: W.config3, 4: lambda: [W.config4()]}[config]()


def run_case(case: str, threads: int) -> dict:
    import oracle
    import workloads as W
    spec = CASES[case]
    config, cycles = spec["config"], spec["cycles"]
    insts = instances_of(config)
    seed = W.sampler_seed(config)
    k = W.sweeps_per_exchange(config)
    digests = [None] * len(insts)
    summary = [None] * len(insts)

    def one(n):
        ref = oracle.OracleChain(insts[n], seed, index=n)
        ref.run(k, cycles)
        obs = ref.observables()
        digests[n] = state_digest(ref.s, obs)
        summary[n] = {"roundtrips": int(np.sum(obs["roundtrips"])),
                      "acc": int(np.sum(obs["acc"])), "E_cl_min": int(np.min(obs["E_cl"]))}

    t0 = time.time()
    # largest instances first, so the pool ends together
    order = sorted(range(len(insts)), key=lambda n: -insts[n].flips_per_sweep)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(one, order))
    return {"case": case, "config": config, "seed": seed, "sweeps_per_exchange": k,
            "cycles": cycles, "instances": len(insts),
            "note": "written by tests/golden/make_golden.py from the CPU oracle",
            "oracle_seconds": round(time.time() - t0, 1),
            "digests": digests, "summary": summary}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=list(CASES) + ["all"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    import oracle
    oracle.lib()  # builds the oracle if it is missing or older than its source
    for case in (CASES if args.case == "all" else [args.case]):
        rec = run_case(case, args.threads)
        with open(golden_path(case), "w") as f:
            json.dump(rec, f, indent=0)
            f.write("\n")
        print(f"{case}: {rec['instances']} instances in {rec['oracle_seconds']} s", flush=True)


if __name__ == "__main__":
    main()
