"""The bit-packed spin encoding (PT_BITPACK32) against the CPU oracle, through the C ABI.

Packing 32 replica slots per word changes only where the spins live: every attempt
still draws its own Philox word and reads its own rung's threshold table, so the
trajectory must be the oracle's bit for bit -- the same bar as the byte encoding.  The
cases add replica counts above 32 and not multiples of 32 (a partly filled last word)
to the degenerate shapes of the byte-encoding tests.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

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


def batch():
    """Degenerate shapes (a lone spin, ragged N, M = 1, M = 2, R = 2, odd R, a colouring
    that is not contiguous, a dense graph, large couplings and fields, M not a multiple of
    8) and replica counts 33, 40 and 65 (two or three words, the last partly filled)."""
    rng = np.random.default_rng([1004, 26])
    return [
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
        W.random_small_instance(rng, 20, 16, 33, d=3, jmax=1, hmax=1, name="r33"),
        W.random_small_instance(rng, 9, 12, 40, d=4, jmax=2, hmax=1, name="r40"),
        W.random_small_instance(rng, 16, 32, 65, d=5, jmax=1, hmax=1, name="r65"),
    ]


def oracle_batch(insts, seed, k, cycles):
    refs = []
    for n, inst in enumerate(insts):
        r = oracle.OracleChain(inst, seed, index=n)
        r.run(k, cycles)
        refs.append(r)
    return refs


def test_init_matches_oracle(ptqmc):
    say("case: bit-packed init, mixed batch")
    insts = batch()
    seed = 0x5EED0B17
    with ptqmc.Sampler(insts, seed, encoding=ptqmc.PT_BITPACK32) as s:
        assert s.info()["encoding"] == ptqmc.PT_BITPACK32
        for n, inst in enumerate(insts):
            assert_same(s, n, oracle.OracleChain(inst, seed, index=n), "init")


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(ptqmc, graph):
    """Sweeps and exchanges over the mixed batch, eagerly and from the captured graph."""
    insts = batch()
    seed = 0xB17B17
    k, cycles = 3, 20
    say(f"case: bit-packed mixed batch, {cycles} cycles of {k} sweeps, graph={graph}")
    refs = oracle_batch(insts, seed, k, cycles)
    flags = 0 if graph else ptqmc.PT_FLAG_NO_GRAPH
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, encoding=ptqmc.PT_BITPACK32,
                       flags=flags) as s:
        s.run(cycles)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "bitpack")


def test_same_chain_as_byte_encoding(ptqmc):
    """The two encodings run the same chain: split pt_sweep / pt_exchange calls under
    each end in identical observables and spins (config 2's instance, 64 sweeps)."""
    inst = W.config2()
    seed = W.sampler_seed(2)
    say("case: bit-packed vs byte encoding, config 2, 64 sweeps")
    out = []
    for enc in (ptqmc.PT_INT8, ptqmc.PT_BITPACK32):
        with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, encoding=enc) as s:
            for _ in range(8):
                s.sweep(8)
                s.exchange()
            obs = s.observables(0)
            out.append(({k: np.asarray(obs[k]).copy() for k in KEYS}, s.spins(0).copy()))
    (oa, sa), (ob, sb) = out
    for k in KEYS:
        assert np.array_equal(oa[k], ob[k]), k
    assert np.array_equal(sa, sb)


def test_config1_run(ptqmc):
    inst = W.config1()
    seed = W.sampler_seed(1)
    say("case: bit-packed config 1, 2000 sweeps, exchange every sweep")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=1, encoding=ptqmc.PT_BITPACK32) as s:
        s.run(2000)
        ref = oracle.OracleChain(inst, seed)
        ref.run(1, 2000)
        assert_same(s, 0, ref, "config1")


@pytest.mark.parametrize("per_sweep", [False, True])
def test_config4_lattice_one_cycle(ptqmc, per_sweep):
    """The 8x8x16 lattice with its 64 replicas in two words per spin position: one cycle
    of 10 sweeps and an exchange against the oracle, with the octet slice blocks resident
    for the call and launched per parity of every sweep."""
    inst = W.config4()
    seed = W.sampler_seed(4)
    flags = ptqmc.PT_FLAG_BLOCK_LAUNCH_PER_SWEEP if per_sweep else 0
    say(f"case: bit-packed config 4, 1 cycle of 10 sweeps, per_sweep={per_sweep}")
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, encoding=ptqmc.PT_BITPACK32,
                       flags=flags) as s:
        s.run(1)
        info = s.info()
        # octet slice blocks (a whole octet, N * M bytes, exceeds half a unit's LDS)
        assert info["oct_blocks"] > 0 and info["oct_tiles"] == 0 and info["class_launches"] == 0
        assert info["oct_resident"] == (0 if per_sweep else 1)
        ref = oracle.OracleChain(inst, seed)
        ref.run(10, 1)
        assert_same(s, 0, ref, "config4")


def test_octet_resident_wait_timeout_recovers(ptqmc):
    """Resident octet slice blocks bound their neighbour waits.  Forced from the host
    (every block waits for a progress count no block publishes, under a poll bound of 16),
    each wait gives up and every workgroup still exits; the next synchronising call
    restores the state of the last clean synchronisation and replays the calls since with
    per-parity launches: the state is the oracle's and one recovery is counted."""
    inst = W.config4()
    seed = 7
    say("case: resident octet slice blocks, forced wait timeout (config 4), recovery")
    ref = oracle.OracleChain(inst, seed)
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, encoding=ptqmc.PT_BITPACK32,
                       flags=ptqmc.PT_FLAG_TEST_BLOCK_WAIT_TIMEOUT) as s:
        assert s.info()["oct_resident"] == 1
        s.run(2)
        s.sweep(1)
        s.sync()
        ref.run(10, 2)
        ref.sweep(1)
        info = s.info()
        assert info["recoveries"] == 1 and info["oct_resident"] == 0
        assert_same(s, 0, ref, "recovered")
        s.run(1)
        ref.run(10, 1)
        assert_same(s, 0, ref, "after recovery")
        assert s.info()["recoveries"] == 1


@pytest.mark.parametrize("encoding", ["bitpack", "int8"])
def test_xcd_mismatch_recovers(ptqmc, encoding):
    """Resident slice blocks whose rings share an XCD pass their records through its L2,
    which is only right while the launch's workgroups keep to round-robin XCDs.  A launch
    that reports a mismatch (forced from the host) fails the call; the next synchronising
    call restores the last clean state and replays the calls with per-sweep launches: the
    state is the oracle's, one recovery is counted, and the error word named the cause."""
    inst = W.config4()
    seed = 11
    enc = ptqmc.PT_BITPACK32 if encoding == "bitpack" else ptqmc.PT_INT8
    say(f"case: forced XCD mismatch of resident slice blocks (config 4, {encoding}), recovery")
    ref = oracle.OracleChain(inst, seed)
    # the byte encoding at its tuned shape (4 resident blocks per replica), so that no
    # tuner candidate runs first
    shape = {} if encoding == "bitpack" else dict(tile_bytes=131072, block_threads=1024)
    with ptqmc.Sampler([inst], seed, sweeps_per_exchange=10, encoding=enc,
                       flags=ptqmc.PT_FLAG_TEST_XCD_MISMATCH, **shape) as s:
        info = s.info()
        assert (info["oct_ring_xcd"] if encoding == "bitpack" else info["block_ring_xcd"]) == 1
        s.run(2)
        s.sync()
        ref.run(10, 2)
        info = s.info()
        assert info["recoveries"] == 1 and info["last_device_error"] & 8
        assert_same(s, 0, ref, "recovered")
        s.run(1)
        ref.run(10, 1)
        assert_same(s, 0, ref, "after recovery")
        assert s.info()["recoveries"] == 1


def octet_batch():
    """Instances the octet kernels take (+-1 couplings, |h| <= 1, one degree, M a
    power-of-two multiple of 8): the smallest M (8), degree 8 with fields (nine adder-tree
    inputs), replica counts that leave a word's last octet partly filled (9, 24 + 1 of a
    second word), config 1, and one octet too large for a workgroup's share of LDS
    (N = 600, M = 128), which runs as slice blocks; plus an instance with |J| = 2 that
    goes to the per-class kernel."""
    rng = np.random.default_rng([1004, 28])
    return [
        W.random_small_instance(rng, 6, 8, 9, d=3, jmax=1, hmax=1, name="m8r9"),
        W.random_small_instance(rng, 31, 16, 33, d=8, jmax=1, hmax=1, name="d8r33"),
        W.random_small_instance(rng, 50, 64, 16, d=4, jmax=1, hmax=1, name="n50"),
        W.config1(),
        W.random_small_instance(rng, 600, 128, 12, d=4, jmax=1, hmax=1, t_min=0.5,
                                name="blocks"),
        W.random_small_instance(rng, 12, 16, 6, d=3, jmax=2, hmax=1, name="generic"),
    ]


@pytest.mark.parametrize("graph,per_sweep", [(False, False), (True, False), (True, True)])
def test_octet_kernels_match_oracle(ptqmc, graph, per_sweep):
    """Whole octets resident for a call, octet slice blocks (resident for the call, or
    launched per parity of every sweep) and the per-class kernel for the rest, in one
    batch, against the oracle."""
    insts = octet_batch()
    seed = 0x0C7E7
    k, cycles = 3, 18
    say(f"case: bit-packed octet batch, {cycles} cycles of {k} sweeps, graph={graph}, "
        f"per_sweep={per_sweep}")
    refs = oracle_batch(insts, seed, k, cycles)
    flags = (0 if graph else ptqmc.PT_FLAG_NO_GRAPH) | (
        ptqmc.PT_FLAG_BLOCK_LAUNCH_PER_SWEEP if per_sweep else 0)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, encoding=ptqmc.PT_BITPACK32,
                       flags=flags) as s:
        info = s.info()
        assert info["oct_tiles"] > 0 and info["oct_blocks"] > 0 and info["class_launches"] > 0
        assert info["oct_resident"] == (0 if per_sweep else 1)
        s.run(cycles)
        s.sweep(2)  # a call of another length (the blocks sum the energies at its end)
        s.sweep(1)  # and of one sweep
        for r in refs:
            r.sweep(2)
            r.sweep(1)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "octets")


@pytest.mark.parametrize("queue", [True, False])
def test_whole_octet_cycles_match_oracle(ptqmc, queue):
    """A batch whose instances are all whole octets: a PT cycle is one launch, the octet
    that completes an instance running its exchange step, with workgroups in list order
    and taking octets from the device work queues.  Three replays of the 16-cycle graph
    with eager sweeps and exchanges between them, each against the oracle."""
    insts = octet_batch()[:4]
    seed = 0x0C7E8
    k = 2
    flags = ptqmc.PT_FLAG_WORK_QUEUE if queue else 0
    say(f"case: whole octets, graph replays, queue={queue}")
    refs = [oracle.OracleChain(inst, seed, index=n) for n, inst in enumerate(insts)]
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=k, encoding=ptqmc.PT_BITPACK32,
                       flags=flags, block_threads=256) as s:
        info = s.info()
        assert info["oct_tiles"] > 0 and info["oct_blocks"] == 0 and info["class_launches"] == 0
        assert info["oct_queue"] == (1 if queue else 0) and info["oct_fused"] == 1
        for rep in range(3):
            s.run(16)
            s.sync()
            for r in refs:
                r.run(k, 16)
            for n in range(len(insts)):
                assert_same(s, n, refs[n], f"replay {rep}")
            s.sweep(1)
            s.exchange()
            s.run(1)
            for r in refs:
                r.sweep(1)
                r.exchange()
                r.run(k, 1)
        for n in range(len(insts)):
            assert_same(s, n, refs[n], "after eager calls")


def test_checkpoint_and_spins(ptqmc):
    """Save / load resume under the packed encoding, a checkpoint of the other encoding
    refused, and set_spins / spins round trips with energies recomputed."""
    insts = batch()[7:]
    seed = 77
    say("case: bit-packed checkpoint resume and set_spins")
    refs = oracle_batch(insts, seed, 2, 25)
    with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2, encoding=ptqmc.PT_BITPACK32) as a:
        a.run(11)
        blob = a.save()
        with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2, encoding=ptqmc.PT_BITPACK32) as b:
            b.load(blob)
            b.run(14)
            for n in range(len(insts)):
                assert_same(b, n, refs[n], "resumed")
        with ptqmc.Sampler(insts, seed, sweeps_per_exchange=2) as other:
            with pytest.raises(ptqmc.PTError):
                other.load(blob)
        rng = np.random.default_rng(3)
        inst = insts[2]
        s_new = rng.choice(np.array([-1, 1], np.int8), size=(inst.R, inst.M, inst.N))
        a.set_spins(2, s_new)
        assert np.array_equal(a.spins(2), s_new)
        E, Cc = oracle.OracleChain(inst, seed, index=2, init=False).energies(s_new)
        obs = a.observables(2)
        assert np.array_equal(obs["E_cl"], E) and np.array_equal(obs["C"], Cc)
