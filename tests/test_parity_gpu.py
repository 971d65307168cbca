"""Parity of the HIP path with the CPU oracle, through the C ABI.

Everything is integer or decided by identical IEEE operations, so the bar is bit
equality: spins, integer energies, the replica permutation, labels, swap counts, round
trips and accumulators.  The oracle runs one instance at a time with that instance's
batch index.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden as golden  # noqa: E402  (digests written from the oracle)

pytestmark = pytest.mark.gpu

KEYS = ("E_cl", "C", "rung_of", "replica_of", "acc", "att", "roundtrips", "label", "sumE",
        "sumC", "sumE2", "sumC2", "nup", "ndown")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ptqmc():
    import torch
    from paper_1004_0023_amd import ptqmc as P
    torch.cuda.set_device(0)
    P.lib()
    return P


def assert_same(sampler, n, ref, what=""):
    got = sampler.observables(n)
    want = ref.observables()
    for k in KEYS:
        assert np.array_equal(np.asarray(got[k]), np.asarray(want[k])), f"{what} inst {n}: {k}"
    assert (got["t"], got["e"], got["n_acc"]) == (want["t"], want["e"], want["n_acc"]), what
    assert np.array_equal(sampler.spins(n), ref.s), f"{what} inst {n}: spins"


def edge_batch():
    """Small instances covering the degenerate shapes: a lone spin, ragged N, classical
    M=1, M=2, R=2 and odd R, a colouring that is not contiguous, large couplings and
    fields, and a dense graph with many colours."""
    rng = np.random.default_rng([1004, 23])
    out = [
        W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                        np.array([1], np.int8), 4, [0.5, 1.0, 2.0], 1.0, name="lone"),
        W.random_small_instance(rng, 5, 6, 3, d=2, jmax=2, hmax=2, name="ragged"),
        W.random_small_instance(rng, 10, 1, 4, d=3, jmax=3, hmax=1, name="classical"),
        W.random_small_instance(rng, 7, 2, 2, d=2, jmax=1, hmax=0, name="m2r2"),
        W.random_small_instance(rng, 13, 8, 5, d=4, jmax=7, hmax=5, relabel=False,
                                name="noncontig"),
        W.random_small_instance(rng, 12, 4, 6, d=11, jmax=1, hmax=1, name="dense"),
        W.random_small_instance(rng, 33, 10, 7, d=3, jmax=120, hmax=100, t_min=2.0,
                                t_max=60.0, name="bigfield"),
    ]
    return out


def fast_batch():
    """Shapes the byte-SWAR kernel takes (M a power-of-two multiple of 8, fields up to
    20): ragged N, a lone spin, the largest field the byte lanes hold, M = 256, odd R,
    colours that are not contiguous label ranges, and general integer couplings."""
    rng = np.random.default_rng([1004, 24])
    lone = W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                           np.array([-1], np.int8), 8, [0.4, 0.9, 1.7], 1.0, name="lone8")
    # F = 20: a 5-regular graph with |J| = 4 and h = 0
    N = 10
    edges = W.random_regular_graph(N, 5, rng)
    J = rng.choice(np.array([-4, 4], np.int8), size=edges.shape[0])
    maxf = W.make_instance(N, edges, J, np.zeros(N, np.int8), 16, [0.5, 1.0, 3.0, 9.0], 1.0,
                           name="F20")
    assert maxf.F() == 20
    return [
        lone,
        W.random_small_instance(rng, 5, 8, 3, d=2, jmax=2, hmax=2, name="ragged8"),
        maxf,
        W.random_small_instance(rng, 7, 256, 2, d=2, jmax=1, hmax=1, name="m256"),
        W.random_small_instance(rng, 13, 16, 5, d=4, jmax=3, hmax=2, relabel=False,
                                name="noncontig16"),
        W.random_small_instance(rng, 9, 32, 7, d=8, jmax=1, hmax=1, name="dense32"),
        W.random_small_instance(rng, 30, 8, 6, d=3, jmax=3, hmax=0, t_min=0.2, t_max=5.0,
                                name="general8"),
    ]


def oracle_batch(insts, seed, k, cycles, extra_sweeps=0):
    refs = []
    for n, inst in enumerate(insts):
        r = oracle.OracleChain(inst, seed, index=n)
        r.run(k, cycles)
        if extra_sweeps:
            r.sweep(extra_sweeps)
        refs.append(r)
    return refs


def test_device_threshold_bitwise(ptqmc):
    say("case: device threshold rule vs oracle")
    rng = np.random.default_rng(5)
    xs = np.concatenate([np.linspace(-5, 40, 50001), rng.random(50000) * 45 - 2,
                         [0.0, 1e-300, 5e-324, 22.18070977791825, 32.0, 1e6, -1e6]])
    got = ptqmc.threshold_device(xs)
    want = np.array([oracle.metropolis_threshold(float(x)) for x in xs], dtype=np.uint32)
    assert np.array_equal(got, want)


def test_init_matches_oracle(ptqmc):
    say("case: init, edge and fast batches")
    insts = edge_batch() + fast_batch()
    seed = 0xABCDEF0123456789
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=1) as s:
        for n, inst in enumerate(insts):
            assert_same(s, n, oracle.OracleChain(inst, seed, index=n), "init")


@pytest.mark.parametrize("block_threads", [0, 256])
def test_config1_full_run(ptqmc, block_threads):
    """Config 1 for 10^4 sweeps with an exchange after every sweep.  With the tuner on
    (block_threads 0) the one run() call stays on per-cycle launches; with the shape
    fixed (tuner off) the same call runs as multi-cycle launches, each workgroup doing
    its instance's exchange steps itself."""
    inst = W.config1()
    seed = W.sampler_seed(1)
    say(f"case: config 1, 10^4 sweeps, exchange every sweep, block_threads={block_threads}")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=1, block_threads=block_threads) as s:
        s.run(10_000)
        ref = oracle.OracleChain(inst, seed)
        ref.run(1, 10_000)
        assert_same(s, 0, ref, "config1")
        info = s.info()
        if block_threads:
            assert info["multi_launches"] >= 10 and info["multi_cycles"] == 10_000
        # a second call after tuning has ended takes the multi-cycle launches either way
        before = info["multi_launches"]
        s.run(300)
        ref.run(1, 300)
        assert_same(s, 0, ref, "config1 second call")
        assert s.info()["multi_launches"] > before


@pytest.mark.parametrize("shape,latency", [((0, 0), None), ((1, 1024), 1), ((1, 512), 0)])
def test_config2_long_run_digest(ptqmc, shape, latency):
    """Config 2 (N=128, M=64, R=32, exchange every 10 sweeps) for 1000 cycles (10^4
    sweeps): the final state's digest equals the oracle's stored one.  With the tuned
    launch shape, with 1024 threads per replica (the pipelined latency path: the largest
    step of class k of parity 0 with class k - 1 of parity 1 holds 72 sites x 8 lanes) and
    with 512 threads (too few for it: classes one by one)."""
    gold = golden.load_golden("config2")
    inst = W.config2()
    seed = W.sampler_seed(2)
    assert gold["seed"] == seed and gold["sweeps_per_exchange"] == 10
    say(f"case: config 2, {gold['cycles']} cycles of 10 sweeps, shape {shape}, "
        f"against the stored digest")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, tile_replicas=shape[0],
                       block_threads=shape[1]) as s:
        if latency is not None:
            assert s.info()["latency_path"] == latency
        s.run(gold["cycles"])
        got = golden.state_digest(s.spins(0), s.observables(0))
    assert got == gold["digests"][0]


def test_config2_truncated(ptqmc):
    inst = W.config2()
    seed = W.sampler_seed(2)
    say("case: config 2, 40 cycles of 10 sweeps")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10) as s:
        s.run(40)
        ref = oracle.OracleChain(inst, seed)
        ref.run(10, 40)
        assert_same(s, 0, ref, "config2")


@pytest.mark.parametrize("two_words", [False, True])
@pytest.mark.parametrize("batch", ["edge", "fast", "mixed"])
@pytest.mark.parametrize("tile_replicas,block_threads",
                         [(0, 0), (1, 64), (3, 512), (2, 1024), (4, 192), (0, 320)])
def test_batch_launch_shapes(ptqmc, batch, tile_replicas, block_threads, two_words):
    """Every launch shape, at the lane width the library picks for these small batches
    (one four-slice word per lane) and with two words per lane forced."""
    insts = {"edge": edge_batch, "fast": fast_batch,
             "mixed": lambda: fast_batch()[:4] + edge_batch()[:4]}[batch]()
    seed = 0x10040023
    k, cycles = 3, 25
    say(f"case: {batch} batch, tile_replicas={tile_replicas} block_threads={block_threads} "
        f"two_words={two_words}")
    refs = oracle_batch(insts, seed, k, cycles)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, tile_replicas=tile_replicas,
                       block_threads=block_threads,
                       flags=ptqmc.PT_FLAG_TWO_WORD_LANES if two_words else 0) as s:
        assert s.info()["lane_words"] == (2 if two_words else 1)
        s.run(cycles)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], f"shape({tile_replicas},{block_threads})")


@pytest.mark.parametrize("tile_replicas,block_threads", [(0, 0), (2, 256)])
def test_four_slice_lanes(ptqmc, tile_replicas, block_threads):
    """The fast path with one four-slice word per lane instead of two: the same chain."""
    insts = fast_batch()
    seed = 0x4F0E5
    k, cycles = 2, 20
    say(f"case: fast batch, four-slice lanes, tile_replicas={tile_replicas} "
        f"block_threads={block_threads}")
    refs = oracle_batch(insts, seed, k, cycles)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, tile_replicas=tile_replicas,
                       block_threads=block_threads, flags=ptqmc.PT_FLAG_FOUR_SLICE_LANES) as s:
        s.run(cycles)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "four-slice lanes")


@pytest.mark.parametrize("batch,two_words,no_latency",
                         [("fast", False, False), ("fast", True, False), ("mixed", False, False),
                          ("fast", False, True)])
def test_latency_path_matches_oracle(ptqmc, batch, two_words, no_latency):
    """Small batches at one replica and 1024 threads per workgroup, where the classes of
    most tiles fit the pipelined latency path (one step per class: class k of parity 0
    with class k - 1 of parity 1); the lone-spin instance has one class and sweeps class
    by class in the same launch.  The same with the path switched off."""
    insts = {"fast": fast_batch, "mixed": lambda: fast_batch()[:4] + edge_batch()[:4]}[batch]()
    seed = 0x1A7E
    k, cycles = 3, 20
    flags = (ptqmc.PT_FLAG_TWO_WORD_LANES if two_words else 0) | (
        ptqmc.PT_FLAG_NO_LATENCY_PATH if no_latency else 0)
    say(f"case: latency path, {batch} batch, two_words={two_words} off={no_latency}")
    refs = oracle_batch(insts, seed, k, cycles)
    # one replica per tile, so that pt_run does not take the multi-cycle launches of
    # whole-instance tiles
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, tile_replicas=1, block_threads=1024,
                       flags=flags) as s:
        assert s.info()["latency_path"] == (0 if no_latency else 1)
        s.run(cycles)
        s.sweep(5)
        for n in range(len(insts)):
            refs[n].sweep(5)
            assert_same(s, n, refs[n], "latency path")


@pytest.mark.parametrize("encoding", ["int8", "bitpack"])
def test_more_than_64_replicas(ptqmc, encoding):
    """Instances of 65, 96 and 130 replicas: the exchange step of instances of at most 64
    replicas runs in one wave, these take its general form (and the bit-packed encoding
    a third, partly filled 32-slot word group).  Every cycle's state is the oracle's."""
    rng = np.random.default_rng([1004, 28])
    insts = [W.random_small_instance(rng, 6, 8, 65, d=2, jmax=1, hmax=1, t_min=0.2, t_max=4.0,
                                     name="r65"),
             W.random_small_instance(rng, 10, 16, 96, d=3, jmax=1, hmax=1, t_min=0.3, t_max=3.0,
                                     name="r96"),
             W.random_small_instance(rng, 4, 8, 130, d=2, jmax=1, hmax=0, t_min=0.1, t_max=5.0,
                                     name="r130")]
    seed = 0x65A
    k, cycles = 2, 12
    enc = ptqmc.PT_BITPACK32 if encoding == "bitpack" else ptqmc.PT_INT8
    say(f"case: R = 65, 96, 130, {encoding}")
    refs = oracle_batch(insts, seed, k, cycles)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, encoding=enc) as s:
        s.run(cycles)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], f"R={insts[n].R}")


def spread_colours(inst):
    """The same instance with colour c renamed 2c: every odd colour class is empty."""
    import dataclasses
    return dataclasses.replace(inst, color=np.ascontiguousarray(2 * np.asarray(inst.color)),
                               n_colors=2 * inst.n_colors, name=inst.name + "_spread")


@pytest.mark.parametrize("mode", ["latency", "classes", "bitpack"])
def test_empty_colour_classes(ptqmc, mode):
    """Colourings with empty classes between the used ones (colour c renamed 2c): the
    byte kernel's latency path (which pairs class k of parity 0 with class k - 1 of parity
    1, here often an empty one), its class-by-class sweep, and the bit-packed encoding
    follow the oracle."""
    rng = np.random.default_rng([1004, 29])
    if mode == "bitpack":
        base = [W.random_small_instance(rng, 24, 16, 12, d=4, jmax=1, hmax=1, name="oct"),
                W.random_small_instance(rng, 9, 8, 40, d=8, jmax=1, hmax=0, name="oct8")]
    else:
        base = fast_batch()[1:]
    insts = [spread_colours(i) for i in base]
    seed = 0xE3C
    k, cycles = 3, 10
    flags = ptqmc.PT_FLAG_NO_LATENCY_PATH if mode == "classes" else 0
    enc = ptqmc.PT_BITPACK32 if mode == "bitpack" else ptqmc.PT_INT8
    shape = {} if mode == "bitpack" else dict(tile_replicas=1, block_threads=1024)
    say(f"case: empty colour classes, {mode}")
    refs = oracle_batch(insts, seed, k, cycles)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, flags=flags, encoding=enc,
                       **shape) as s:
        if mode != "bitpack":
            assert s.info()["latency_path"] == (1 if mode == "latency" else 0)
        s.run(cycles)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], f"{mode} {insts[n].name}")


def test_sixteen_bit_entries_in_small_batch(ptqmc):
    """A lone large regular +-1 instance (N = 512, M = 128, degree 8: a replica of more
    than half a compute unit's LDS, so its neighbour entries are 16 bits) with two
    replicas: too few lanes for two words each, yet the batch keeps two-word lanes, which
    are the only ones that read 16-bit entries."""
    rng = np.random.default_rng([1004, 27])
    inst = W.random_small_instance(rng, 512, 128, 2, d=8, jmax=1, hmax=1, name="ent16")
    seed = 0x16E
    k, cycles = 2, 3
    say("case: 16-bit entries, N=512 M=128 R=2")
    refs = oracle_batch([inst], seed, k, cycles)
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=k) as s:
        info = s.info()
        assert info["ent16_instances"] == 1 and info["lane_words"] == 2
        s.run(cycles)
        assert_same(s, 0, refs[0], "16-bit entries")


def test_split_calls_graph_and_eager_agree(ptqmc):
    insts = edge_batch()[:4]
    seed = 77
    say("case: pt_run graph vs eager vs split sweep/exchange")
    refs = oracle_batch(insts, seed, 2, 40, extra_sweeps=3)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2) as a, \
            ptqmc.Sampler(insts, seed, sweeps_per_exchange=2, flags=ptqmc.PT_FLAG_NO_GRAPH) as b, \
            ptqmc.Sampler(insts, seed, sweeps_per_exchange=2) as c:
        a.run(40)          # graph path (>= 16 cycles)
        b.run(40)          # eager
        for _ in range(40):
            c.sweep(1)
            c.sweep(1)
            c.exchange()
        for s in (a, b, c):
            s.sweep(3)
        for n in range(len(insts)):
            for s, tag in ((a, "graph"), (b, "eager"), (c, "split")):
                assert_same(s, n, refs[n], tag)


def test_checkpoint_resume(ptqmc):
    insts = edge_batch()[1:5]
    seed = 2025
    say("case: save/load resume")
    refs = oracle_batch(insts, seed, 2, 30)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2) as a:
        a.run(13)
        blob = a.save()
        with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2) as b:
            b.load(blob)
            b.run(17)
            for n in range(len(insts)):
                assert_same(b, n, refs[n], "resumed")
        with ptqmc.Sampler(insts, seed + 1, sweeps_per_exchange=2) as other:
            with pytest.raises(ptqmc.PTError):
                other.load(blob)
        # the host-side checks accept the real checkpoint; an all-zero state (rung_of is
        # then no permutation) is refused before anything reaches the device
        ptqmc.checkpoint_validate(insts, seed, blob, sweeps_per_exchange=2)
        with pytest.raises(ptqmc.PTError) as e:
            a.load(blob[:40] + bytes(len(blob) - 40))
        assert e.value.code == ptqmc.PT_ESTATE


def test_set_spins_recomputes_energies(ptqmc):
    inst = W.config1()
    say("case: set_spins")
    rng = np.random.default_rng(0)
    s_new = rng.choice(np.array([-1, 1], np.int8), size=(inst.R, inst.M, inst.N))
    with ptqmc.Sampler([inst], 5) as s:
        s.set_spins(0, s_new)
        assert np.array_equal(s.spins(0), s_new)
        ref = oracle.OracleChain(inst, 5)
        E, Cc = ref.energies(s_new)
        obs = s.observables(0)
        assert np.array_equal(obs["E_cl"], E) and np.array_equal(obs["C"], Cc)
        with pytest.raises(ptqmc.PTError):
            s.set_spins(0, np.zeros_like(s_new))


def test_injected_launch_failure_falls_back(ptqmc):
    insts = edge_batch()[4:6]
    seed = 31
    say("case: injected out-of-resources fallback")
    refs = oracle_batch(insts, seed, 2, 10)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2, tile_replicas=4,
                       flags=ptqmc.PT_FLAG_INJECT_LAUNCH_OOR_ONCE) as s:
        s.run(10)
        assert s.info()["fallbacks"] >= 1
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "fallback")


@pytest.fixture(scope="module")
def config3_batch():
    return W.config3()


# (tile bytes, block threads): 64 KiB x 1024 is the shape the tuner picks on an MI355X for
# this batch (the benchmark records the shape it ran); the others are the rest of the
# tuner's range, and (0, 0) runs the tuner itself, whose first ten calls each use a
# different candidate shape.
CONFIG3_SHAPES = [(65536, 1024), (131072, 1024), (32768, 512), (16384, 1024), (8192, 256),
                  (65536, 256), (0, 0)]


@pytest.mark.parametrize("tile_bytes,block_threads", CONFIG3_SHAPES)
def test_config3_full_batch_digests(ptqmc, config3_batch, tile_bytes, block_threads):
    """All 512 instances of the batched workload for 16 PT cycles (160 sweeps) as one
    pt_run call, i.e. one replay of the captured 16-cycle graph (the benchmark's route):
    every instance's final state (spins, energies, permutation, labels, swap counts,
    round trips, accumulators, counters) has the digest of the oracle's run of that
    instance, stored by tests/golden/make_golden.py.  With the tuner on (0, 0) the cycles
    run as 16 calls, each timing another candidate shape."""
    gold = golden.load_golden("config3")
    insts = config3_batch
    seed = W.sampler_seed(3)
    k, cycles = gold["sweeps_per_exchange"], gold["cycles"]
    assert gold["seed"] == seed and gold["instances"] == len(insts) == 512
    say(f"case: config 3, 512 instances, {cycles} cycles of {k} sweeps, "
        f"tile_bytes={tile_bytes} block_threads={block_threads}")
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, tile_bytes=tile_bytes,
                       block_threads=block_threads) as s:
        if tile_bytes:
            s.run(cycles)   # one replay of the 16-cycle graph
        else:
            for _ in range(cycles):
                s.run(1)    # tuning: each call a different candidate shape
        info = s.info()
        if tile_bytes:
            assert info["tile_bytes"] == tile_bytes and info["block_threads"] == block_threads
        bad = [n for n in range(len(insts))
               if golden.state_digest(s.spins(n), s.observables(n)) != gold["digests"][n]]
    assert not bad, f"{len(bad)} instances differ from the oracle, first {bad[:8]}"


@pytest.mark.parametrize("block_threads,queue", [(1024, False), (256, True), (0, False)])
def test_config3_bitpack_digests(ptqmc, config3_batch, block_threads, queue):
    """The batched workload in the bit-packed encoding (every instance whole octets) for
    the stored 16 cycles, a PT cycle one launch with the exchange run by the octet that
    completes each instance: workgroups in list order (the benchmark's route at its tuned
    1024 threads, and under the tuner) and taking octets from the device work queues.
    Every instance's final state has the oracle's digest."""
    gold = golden.load_golden("config3")
    insts = config3_batch
    seed = W.sampler_seed(3)
    k, cycles = gold["sweeps_per_exchange"], gold["cycles"]
    flags = ptqmc.PT_FLAG_WORK_QUEUE if queue else 0
    say(f"case: config 3 bit-packed, {cycles} cycles, block_threads={block_threads} queue={queue}")
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, encoding=ptqmc.PT_BITPACK32,
                       block_threads=block_threads, flags=flags) as s:
        info = s.info()
        assert info["oct_tiles"] > 0 and info["oct_blocks"] == 0 and info["class_launches"] == 0
        assert info["oct_fused"] == 1 and info["oct_queue"] == (1 if queue else 0)
        if block_threads:
            s.run(cycles)
        else:
            for _ in range(cycles):
                s.run(1)
        bad = [n for n in range(len(insts))
               if golden.state_digest(s.spins(n), s.observables(n)) != gold["digests"][n]]
    assert not bad, f"{len(bad)} instances differ from the oracle, first {bad[:8]}"


@pytest.mark.parametrize("per_sweep", [False, True])
@pytest.mark.parametrize("tile_bytes,block_threads", [(0, 256), (4096, 1024)])
def test_slice_blocks_match_oracle(ptqmc, tile_bytes, block_threads, per_sweep):
    """Replicas forced into slice blocks reproduce the oracle's trajectory, both with all
    blocks resident in one launch per call (halos passed between blocks in device memory)
    and with one launch per sweep (halos from boundary records)."""
    insts = fast_batch() + [W.config1()]
    seed = 0xB10C
    k, cycles = 3, 12
    flags = ptqmc.PT_FLAG_SLICE_BLOCKS | (ptqmc.PT_FLAG_BLOCK_LAUNCH_PER_SWEEP if per_sweep else 0)
    say(f"case: slice blocks, tile_bytes={tile_bytes} block_threads={block_threads} "
        f"per_sweep={per_sweep}")
    refs = oracle_batch(insts, seed, k, cycles)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, tile_bytes=tile_bytes,
                       block_threads=block_threads, flags=flags) as s:
        s.run(cycles)
        assert s.info()["block_resident"] == (0 if per_sweep else 1)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "blocks")


@pytest.mark.parametrize("k", [3, 10])
def test_resident_split_blocks_match_oracle(ptqmc, k):
    """Resident slice blocks of eight groups (M = 256) run the split sweep order.  With at
    most one site per thread the next sweep's halos are loaded into registers at the end
    of a sweep: N = 200 leaves threads past N (they load site N - 1 and keep it unused),
    N = 256 fills the workgroup, and N = 300 exceeds it, so those blocks wait and load
    their halos before the edge slots instead.  Calls of k sweeps, then of one and of
    seven sweeps (a one-sweep call fetches halos it never uses)."""
    rng = np.random.default_rng([1004, 26])
    insts = [W.random_small_instance(rng, N, 256, 3, d=4, jmax=2, hmax=1, name=f"split{N}")
             for N in (200, 256, 300)]
    seed = 0x5B117
    cycles = 4
    say(f"case: resident split slice blocks, N in 200/256/300, M=256, k={k}")
    refs = oracle_batch(insts, seed, k, cycles, extra_sweeps=8)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, tile_bytes=0, block_threads=256,
                       flags=ptqmc.PT_FLAG_SLICE_BLOCKS) as s:
        s.run(cycles)
        s.sweep(1)
        s.sweep(7)
        assert s.info()["block_resident"] == 1
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "split blocks")


def test_config2_slice_blocks(ptqmc):
    inst = W.config2()
    seed = W.sampler_seed(2)
    say("case: config 2 in slice blocks, 6 cycles of 10 sweeps")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, tile_bytes=8192,
                       block_threads=512, flags=ptqmc.PT_FLAG_SLICE_BLOCKS) as s:
        s.run(6)
        ref = oracle.OracleChain(inst, seed)
        ref.run(10, 6)
        assert_same(s, 0, ref, "config2 blocks")


@pytest.mark.parametrize("mode", ["resident", "resident_device_scope", "per_sweep", "bitpack",
                                  "bitpack_device_scope"])
def test_config4_long_run_digest(ptqmc, mode):
    """The 8x8x16 lattice (N=1024, M=256, R=64) for 100 cycles of 10 sweeps (10^3
    sweeps): resident slice blocks, slice blocks launched once per sweep, and the
    bit-packed encoding all end in the state whose digest the oracle stored, with no call
    recovered.  Resident blocks run with every ring of blocks on one XCD (a replica's 4
    byte blocks, an octet's 32), records through that XCD's L2, and with records through
    device-scope operations."""
    gold = golden.load_golden("config4")
    inst = W.config4()
    seed = W.sampler_seed(4)
    assert gold["seed"] == seed
    flags = ptqmc.PT_FLAG_BLOCK_LAUNCH_PER_SWEEP if mode == "per_sweep" else 0
    if mode.endswith("device_scope"):
        flags |= ptqmc.PT_FLAG_DEVICE_SCOPE_RECORDS
    enc = ptqmc.PT_BITPACK32 if mode.startswith("bitpack") else ptqmc.PT_INT8
    say(f"case: config 4, {gold['cycles']} cycles of 10 sweeps, {mode}, against the stored digest")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, flags=flags, encoding=enc) as s:
        s.run(gold["cycles"])
        info = s.info()
        if mode.startswith("bitpack"):
            assert info["oct_resident"] == 1
            assert info["oct_ring_xcd"] == (1 if mode == "bitpack" else 0)
        else:
            assert info["block_resident"] == (0 if mode == "per_sweep" else 1)
            assert info["block_ring_xcd"] == (1 if mode == "resident" else 0)
        got = golden.state_digest(s.spins(0), s.observables(0))
        assert s.info()["recoveries"] == 0
    assert got == gold["digests"][0]


@pytest.mark.parametrize("per_sweep", [False, True])
def test_config4_lattice_one_cycle(ptqmc, per_sweep):
    """The 8x8x16 lattice (N=1024, M=256, R=64): a replica (256 KiB) exceeds one
    workgroup's LDS, so it always runs in slice blocks.  One full cycle (10 sweeps and an
    exchange) against the oracle, with resident blocks and with one launch per sweep."""
    inst = W.config4()
    seed = W.sampler_seed(4)
    flags = ptqmc.PT_FLAG_BLOCK_LAUNCH_PER_SWEEP if per_sweep else 0
    say(f"case: config 4, 1 cycle of 10 sweeps, per_sweep={per_sweep}")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, tile_bytes=131072,
                       block_threads=1024, flags=flags) as s:
        s.run(1)
        assert s.info()["block_resident"] == (0 if per_sweep else 1)
        ref = oracle.OracleChain(inst, seed)
        ref.run(10, 1)
        assert_same(s, 0, ref, "config4")


def test_resident_block_wait_timeout_recovers(ptqmc):
    """Resident slice blocks bound their neighbour waits.  Forced from the host (every
    block waits for a progress count no block ever publishes, under a poll bound of 16),
    each wait gives up and every workgroup still exits; the next synchronising call
    restores the state of the last clean synchronisation, replays the calls since with a
    launch per sweep and succeeds: the state is the oracle's, one recovery is counted,
    and the calls that follow run without resident launches."""
    inst = W.config4()
    seed = 7
    say("case: resident slice blocks, forced wait timeout (config 4), recovery")
    ref = oracle.OracleChain(inst, seed)
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, tile_bytes=131072, block_threads=1024,
                       flags=ptqmc.PT_FLAG_TEST_BLOCK_WAIT_TIMEOUT | ptqmc.PT_FLAG_NO_GRAPH) as s:
        s.run(1)
        assert s.info()["block_resident"] == 1
        s.sweep(3)
        s.exchange()
        s.sync()
        ref.run(10, 1)
        ref.sweep(3)
        ref.exchange()
        info = s.info()
        assert info["recoveries"] == 1
        assert_same(s, 0, ref, "recovered")
        s.run(1)
        ref.run(10, 1)
        assert s.info()["block_resident"] == 0
        assert_same(s, 0, ref, "after recovery")
        assert s.info()["recoveries"] == 1


def test_maximum_sizes(ptqmc):
    """The largest slice count (M = 4096), a large whole-replica tile (N = 4095 at M = 8,
    about 90 KiB of LDS) and a replica whose rows need offsets beyond 16 bits (N = 4096,
    M = 64, run as slice blocks) reproduce the oracle."""
    rng = np.random.default_rng([1004, 25])
    insts = [W.random_small_instance(rng, 3, 4096, 2, d=2, name="m4096"),
             W.random_small_instance(rng, 4095, 8, 2, d=2, name="n4095"),
             W.random_small_instance(rng, 4096, 64, 2, d=3, name="wide_rows")]
    seed = 0x3A5
    k, cycles = 2, 3
    say("case: maximum sizes (M=4096; N=4095 at M=8; N=4096 at M=64 in slice blocks)")
    refs = oracle_batch(insts, seed, k, cycles)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k) as s:
        s.run(cycles)
        assert s.info()["block_tiles"] > 0
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "max sizes")


def test_replica_too_large_is_refused(ptqmc):
    """A replica that no kernel can hold in one workgroup's LDS is refused at pt_init with
    the reason, and nothing is left allocated."""
    rng = np.random.default_rng([1004, 26])
    inst = W.random_small_instance(rng, 65535, 2, 2, d=2, name="too_large")
    say("case: N=65535, M=2 replica refused")
    with pytest.raises(ptqmc.PTError) as ei:
        ptqmc.Sampler([inst], 1, sweeps_per_exchange=1)
    assert ei.value.code == ptqmc.PT_EINVAL and "does not fit" in str(ei.value)


def whole_tile_batch():
    """Instances that each fit one whole-replica fast tile (R a power of two), so that
    pt_run takes its multi-cycle launches: a lone spin, ragged N, the largest byte field,
    M = 256, and config 1."""
    f = fast_batch()
    rng = np.random.default_rng([1004, 27])
    lone = W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                           np.array([1], np.int8), 8, [0.4, 0.9, 1.7, 2.5], 1.0, name="lone8r4")
    return [lone,
            W.random_small_instance(rng, 5, 8, 2, d=2, jmax=2, hmax=2, name="ragged8r2"),
            f[2],  # F = 20, R = 4
            f[3],  # M = 256, R = 2
            W.random_small_instance(rng, 9, 32, 8, d=8, jmax=1, hmax=1, name="dense32r8"),
            W.config1()]


@pytest.mark.parametrize("mode", ["tiles", "whole_tiles", "slice_blocks", "bitpack", "tau"])
def test_every_graph_replay_matches_oracle(ptqmc, mode):
    """pt_run replays a captured graph of 16 cycles.  Three replays, with eager
    pt_sweep / pt_exchange calls and synchronisations between them, each checked against
    the oracle: whole-replica tiles of one replica each (fused cycles), resident slice
    blocks, the packed encoding, and the correlation accumulators.  With every instance
    in one tile (whole_tiles: R a power of two) a run(16) is instead one launch of 16
    cycles, each workgroup doing its instance's exchange steps itself; the test checks
    that those launches ran."""
    insts = whole_tile_batch() if mode == "whole_tiles" else fast_batch()[:5]
    seed = 0x6A7
    k = 2
    flags = {"tiles": 0, "whole_tiles": 0, "slice_blocks": ptqmc.PT_FLAG_SLICE_BLOCKS,
             "bitpack": 0, "tau": ptqmc.PT_FLAG_TAU_CORR}[mode]
    enc = ptqmc.PT_BITPACK32 if mode == "bitpack" else ptqmc.PT_INT8
    keys = KEYS + (("sumCt",) if mode == "tau" else ())
    say(f"case: graph replays, {mode}")
    refs = [oracle.OracleChain(inst, seed, index=n) for n, inst in enumerate(insts)]
    # a fixed block size turns the launch-shape tuner off, so every run(16) is a replay
    # (or, for whole_tiles, one multi-cycle launch); one replica per tile keeps "tiles" on
    # the graph path
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, flags=flags, encoding=enc,
                       block_threads=256, tile_replicas=1 if mode == "tiles" else 0) as s:
        for rep in range(3):
            s.run(16)  # one replay of the captured 16-cycle graph
            s.sync()
            for r in refs:
                r.run(k, 16)
            for n in range(len(insts)):
                got, want = s.observables(n), refs[n].observables()
                for key in keys:
                    assert np.array_equal(np.asarray(got[key]), np.asarray(want[key])), (mode, rep, n, key)
                assert np.array_equal(s.spins(n), refs[n].s), (mode, rep, n)
            if mode == "whole_tiles":
                info = s.info()
                assert info["multi_launches"] == rep + 1 and info["multi_cycles"] == 16 * (rep + 1)
            # eager work between replays
            s.sweep(1)
            s.exchange()
            for r in refs:
                r.sweep(1)
                r.exchange()
        if mode == "slice_blocks":
            assert s.info()["block_resident"] == 1
