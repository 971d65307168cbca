"""Benchmark: spin-flip attempts per second of the parallel-tempering sampler on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3] [--encoding int8|bitpack]

A step is one PT cycle over the whole batch: sweeps_per_exchange Metropolis sweeps of
every replica of every instance (with the energy bookkeeping of each replica), then one
replica-exchange step with its statistics, round-trip labels and accumulators.  All
state is resident in device memory when the timed region starts.  Prints one JSON line.

The default workload is the batched one (512 instances of uneven size in one launch),
the configuration whose sweep kernel the roofline target refers to; --config 1, 2 or 4
selects the single-instance workloads.  --encoding int8 keeps one byte per spin,
--encoding bitpack 32 replica slots per 32-bit word (the same chain either way); the
default is bitpack for configs 3 and 4 and int8 for configs 1 and 2.

    python bench.py --copy-calibration BYTES

runs a plain device-to-device copy of BYTES bytes (used to scale the HBM counters of a
profiler run; prints one JSON line and nothing else).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 compute units, each with 4 SIMDs of 16 lanes (64 lanes of 32-bit integer
# work per clock), at a 2.4 GHz peak engine clock.
CUS, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
PEAK_INT_OPS = CUS * LANES_PER_CU * CLOCK_HZ  # 3.93e13 32-bit VALU lane-ops/s

# Committed HBM-traffic records (profiler counters, scaled by a copy calibration) per
# (kernel, workload), each with the source file whose SHA-256 it was measured on.
_CSRC = os.path.join(ROOT, "paper_1004_0023_amd", "csrc")
TRAFFIC_RECORDS = {
    ("sweep_fast_kernel", 3): (os.path.join(ROOT, "profiles", "sweep_fast_kernel_config3_traffic.json"),
                               os.path.join(_CSRC, "pt_kernels.hip")),
    ("oct_tile_kernel", 3): (os.path.join(ROOT, "profiles", "oct_tile_kernel_config3_traffic.json"),
                             os.path.join(_CSRC, "pt_octet.hip")),
}
# The encoding each workload runs in unless --encoding says otherwise: the lattice is
# specified bit-packed; the batch runs in whichever encoding is faster on it (bit-packed,
# measured); the single small instances are specified as bytes.
DEFAULT_ENCODING = {1: "int8", 2: "int8", 3: "bitpack", 4: "bitpack"}


def ops_per_flip(avg_degree: float) -> float:
    """Algorithmic 32-bit VALU lane-operations of one Metropolis attempt in the byte-SWAR
    formulation (four same-parity slices of a site per 32-bit word, one Philox call per
    word):
      Philox4x32-10, a quarter of a call: 10 rounds x (2 products + 2 three-input xors) / 4 = 10
      local field: per neighbour one byte lookup and one add, shared by 4 slices     = d / 2
      time field: one byte-align and one add per word                                 = 0.5
      threshold index 3V + tau: five operations per word                              = 1.25
      per attempt: index extraction, comparison, flip-bit merge                       = 3
      spin update: one xor per word                                                   = 0.25
    """
    return 10.0 + avg_degree / 2.0 + 0.5 + 1.25 + 3.0 + 0.25


def workload(config: int):
    import workloads as W
    if config == 1:
        insts = [W.config1()]
        desc = "config1: N=8 3-regular, M=16, R=8, T in [0.1,2.0], Gamma=1, 1 instance"
    elif config == 2:
        insts = [W.config2()]
        desc = ("config2: N=128 6-regular, J in +-{1,2,3}, h=0, M=64, R=32, T in [0.05,3.0], "
                "Gamma=1, 1 instance")
    elif config == 3:
        insts = W.config3()
        desc = ("config3: 512 instances in one launch, N~U[32,512], d~U{4..8}, M in "
                "{32,64,128}, R in {16,32,64}, T in [0.1,3.0], Gamma=1")
    elif config == 4:
        insts = [W.config4()]
        desc = "config4: 8x8x16 periodic cubic N=1024, J=+-1, h=0, M=256, R=64, Gamma=1.5"
    else:
        raise SystemExit(f"unknown config {config}")
    return insts, desc


def cpu_baseline(insts, seed, k, budget_s=2.0, max_threads=16):
    """The oracle as it stands on the host's cores, on a bounded sample.  As in the
    paper's multi-core design (independent chains from a work pool, Figures 4-5), each
    host thread runs whole PT cycles of its own instance (the first instances of the
    workload, batch indices 0..threads-1) for about budget_s; the oracle's ctypes calls
    release the GIL.  Rate = all attempts / wall time of the parallel section."""
    import threading
    import oracle
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(max_threads, ncpu, len(insts)))
    flips = [0] * threads

    def work(n):
        inst = insts[n]
        ref = oracle.OracleChain(inst, seed, index=n)
        t0 = time.perf_counter()
        ref.run(k, 1)
        one = time.perf_counter() - t0
        cycles = max(0, int(budget_s / max(one, 1e-6)) - 1)
        if cycles:
            ref.run(k, cycles)
        flips[n] = (cycles + 1) * k * inst.flips_per_sweep

    pool = [threading.Thread(target=work, args=(n,)) for n in range(threads)]
    t0 = time.perf_counter()
    for th in pool:
        th.start()
    for th in pool:
        th.join()
    dt = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": sum(flips) / dt, "unit": "spin-flip attempts/s", "cores": threads,
            "kind": "oracle",
            "sample": f"instances 0..{threads - 1} of the workload, one per host thread, whole "
                      f"cycles of {k} sweeps + exchange for about {budget_s:.0f} s each; "
                      f"{sum(flips):.3e} attempts in {dt:.1f} s wall; host {model}, "
                      f"{ncpu} CPUs available"}


def traffic_per_launch(kernel: str = "sweep_fast_kernel", config: int = 3):
    """HBM bytes per launch of `kernel` on workload `config` from the committed profiler
    record, or None when there is none or the kernel source has changed since the
    counters were taken."""
    ent = TRAFFIC_RECORDS.get((kernel, config))
    if ent is None:
        return None
    try:
        with open(ent[0]) as f:
            rec = json.load(f)
        with open(ent[1], "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_calibration(nbytes: int):
    import torch
    torch.cuda.set_device(0)
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-bytes", type=int, default=0)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0)
    ap.add_argument("--encoding", choices=["int8", "bitpack"], default=None,
                    help="spin encoding (default: bitpack for configs 3 and 4, int8 otherwise)")
    ap.add_argument("--work-queue", action="store_true",
                    help="bit-packed whole octets: workgroups take octets from the device work queues")
    ap.add_argument("--device-scope-records", action="store_true",
                    help="resident octet slice blocks: records through device-scope operations")
    ap.add_argument("--no-latency-path", action="store_true",
                    help="byte tiles of small batches: sweep without forming next items ahead")
    ap.add_argument("--tau-corr", action="store_true",
                    help="also accumulate imaginary-time correlations at every exchange step "
                         "(byte encoding only; the default encoding then is int8)")
    args = ap.parse_args()
    if args.tau_corr and args.encoding == "bitpack":
        ap.error("--tau-corr needs the byte encoding (--encoding int8)")
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}). "
              "Instances and replicas are independent between exchanges, so a multi-GPU run "
              "would shard them, but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1004_0023_amd import ptqmc

    if args.encoding is None:
        args.encoding = "int8" if args.tau_corr else DEFAULT_ENCODING.get(args.config, "int8")
    torch.cuda.set_device(0)
    insts, desc = workload(args.config)
    k = W.sweeps_per_exchange(args.config)
    seed = W.sampler_seed(args.config)
    default_steps = {1: 10_000, 2: 10_000, 3: 1_000, 4: 2_000}[args.config]
    steps = args.steps if args.steps is not None else default_steps
    print(f"bench: {desc}; {steps} steps of {k} sweeps + exchange", file=sys.stderr, flush=True)

    encoding = ptqmc.PT_BITPACK32 if args.encoding == "bitpack" else ptqmc.PT_INT8
    flags = (ptqmc.PT_FLAG_TAU_CORR if args.tau_corr else 0) | (
        ptqmc.PT_FLAG_WORK_QUEUE if args.work_queue else 0) | (
        ptqmc.PT_FLAG_NO_LATENCY_PATH if args.no_latency_path else 0) | (
        ptqmc.PT_FLAG_DEVICE_SCOPE_RECORDS if args.device_scope_records else 0)
    s = ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, flags=flags,
                      tile_bytes=args.tile_bytes, block_threads=args.block_threads,
                      encoding=encoding)
    # Untimed set-up: without a launch shape given, the first sweep calls time the candidate
    # shapes (three rounds of 15); run cycles until that is done, whatever W is, so that
    # neither the warm-up nor the timed steps include tuning.  Then the W warm-up cycles.
    for _ in range(64):
        if s.info()["tuned"]:
            break
        s.run(1)
    if not s.info()["tuned"]:
        raise RuntimeError("launch-shape tuning did not finish in 64 cycles")
    s.run(args.warmup)
    s.sync()
    torch.cuda.synchronize()
    # The timed region is pt_run's own route (graph replays, or multi-cycle launches when
    # every instance fits one tile), with no events inside it.  The K steps run as five
    # equal segments, each closed by a synchronisation, so the spread of the rate is
    # visible; the reported value is all K steps over the whole time.
    n_seg = 5 if steps >= 5 else 1
    bounds = [steps * j // n_seg for j in range(n_seg + 1)]
    seg_s = []
    t0 = time.perf_counter()
    for j in range(n_seg):
        ts = time.perf_counter()
        s.run(bounds[j + 1] - bounds[j])
        s.sync()
        seg_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info = s.info()
    flips_per_step = k * int(info["flips_per_sweep"])
    value = steps * flips_per_step / elapsed
    seg_rates = [(bounds[j + 1] - bounds[j]) * flips_per_step / seg_s[j] for j in range(n_seg)]
    route = "multi-cycle launches" if info["multi_launches"] > 0 else "graph replays"

    # Calibration pass, right after the timed region on the same context: timing switched
    # on, pt_run launches cycle by cycle with HIP events on the library's stream around
    # every sweep call (one launch per occupancy class of whole-replica tiles; slice
    # blocks: one resident launch per call, or one per sweep; packed: one per colour
    # class) and every exchange launch; multi-cycle launches are timed whole.  The
    # roofline is quoted per launch of the dominant kernel: the call's algorithmic work
    # and event time divided by its launch count, so the mean launch duration is the one
    # a kernel trace of the timed route reports.
    multi = info["multi_launches"] > 0
    cal_cycles = 4096 if multi else max(1, min(steps, 100))
    s.timing_reset()
    pre = s.info()
    s.timing_enable(True)
    s.run(cal_cycles)
    s.sync()
    cal = s.info()
    s.timing_enable(False)
    # the launch counts of multi-cycle launches run on; keep this pass's
    cal["multi_launches"] -= pre["multi_launches"]
    cal["multi_cycles"] -= pre["multi_cycles"]
    blocked = cal["block_tiles"] > 0
    packed = encoding == ptqmc.PT_BITPACK32
    if multi:
        kernel = "sweep_fast_kernel"
        cycles_per_launch = cal["multi_cycles"] / max(1, cal["multi_launches"])
        launch_s = cal["multi_ms"] / max(1, cal["multi_launches"]) / 1e3
        calls_per_launch = cycles_per_launch
        launches_per_call = 1.0 / cycles_per_launch
        avg_sweep_s = launch_s / cycles_per_launch  # one cycle, its exchange included
    else:
        avg_sweep_s = cal["sweep_ms"] / max(1, cal["sweep_launches"]) / 1e3
        if (packed and cal["oct_blocks"] > 0 and cal["oct_tiles"] == 0 and
                cal["class_launches"] == 0 and cal["oct_resident"]):
            # octet slice blocks, all resident: one launch per call
            kernel = "oct_resident_kernel"
            launches_per_call = 1
        elif packed and cal["oct_blocks"] > 0 and cal["oct_tiles"] == 0 and cal["class_launches"] == 0:
            # octet slice blocks: one launch per parity of every sweep
            kernel = "oct_phase_kernel"
            launches_per_call = 2 * k
        elif packed and cal["oct_tiles"] > 0 and cal["oct_blocks"] == 0 and cal["class_launches"] == 0:
            # whole octets: one launch per call and workgroup size
            kernel = "oct_tile_kernel"
            launches_per_call = max(1, cal["oct_tile_launches"])
        elif packed:
            # one launch per colour class and sweep, plus the two energy launches of the call
            kernel = "bp_sweep_kernel"
            launches_per_call = k * max(1, cal["class_launches"])
        elif blocked:
            kernel = "sweep_block_kernel"
            launches_per_call = 1 if cal["block_resident"] else k
        else:
            kernel = "sweep_fast_kernel"
            launches_per_call = max(1, cal["sweep_groups"])
        launch_s = avg_sweep_s / launches_per_call
        calls_per_launch = 1.0 / launches_per_call
    ops_call = 0.0
    for inst in insts:
        ops_call += k * inst.flips_per_sweep * ops_per_flip(2.0 * inst.n_edges / inst.N)
    ops_launch = ops_call * calls_per_launch
    achieved = ops_launch / launch_s / 1e12 if launch_s > 0 else 0.0
    peak = PEAK_INT_OPS / 1e12
    if packed:
        desc += "; bit-packed spins (32 replica slots per 32-bit word)"
    if args.tau_corr:
        desc += "; imaginary-time correlations accumulated at every exchange step"
    out = {
        "metric": "spin-flip attempts/s",
        "value": value,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if packed else "u8",
        "data": "synthetic",
        "config": {"workload": desc, "instances": len(insts), "sweeps_per_exchange": k,
                   "flips_per_step": flips_per_step, "tiles": info["n_tiles"],
                   "tile_bytes": info["tile_bytes"], "block_threads": info["block_threads"],
                   "lds_bytes": info["lds_bytes"], "timed_route": route,
                   "encoding": args.encoding,
                   "tau_corr": bool(args.tau_corr),
                   "work_queue": bool(info["oct_queue"]) if packed else None,
                   "fused_exchange": bool(info["oct_fused"]) if packed else None,
                   "ring_xcd": bool(info["oct_ring_xcd"]) if packed else None,
                   "latency_path": None if packed else bool(info["latency_path"]),
                   "lane_words": None if packed else info["lane_words"],
                   "block_resident": (bool(cal["block_resident"]) if blocked else
                                      bool(cal["oct_resident"]) if packed and cal["oct_blocks"] > 0
                                      else None),
                   "segment_rates": {"segments": n_seg,
                                     "mean": statistics.mean(seg_rates),
                                     "std": statistics.pstdev(seg_rates),
                                     "median": statistics.median(seg_rates)},
                   "calibration": {"cycles": cal_cycles,
                                   "sweep_call_ms": avg_sweep_s * 1e3,
                                   "sweep_kernel_flips_per_s": flips_per_step / avg_sweep_s
                                   if avg_sweep_s else None,
                                   "exchange_kernel_ms": cal["exchange_ms"] / max(1, cal["exchange_launches"]),
                                   "launches_per_call": launches_per_call,
                                   "mean_launch_ms": launch_s * 1e3,
                                   "ops_per_launch": ops_launch}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic_per_launch(kernel, args.config),
                     "kernel": kernel},
    }
    s.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(insts, seed, k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
