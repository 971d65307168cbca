"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every check here would fail under a plausible mistake in the oracle: a wrong Philox
round, a wrong exponential, a wrong sign in the action change, a wrong neighbour or
slice index in the local field, a wrong swap formula, a wrong label rule, or a wrong
estimator.  The references are (i) published known-answer vectors and an independent
Philox implementation (rocRAND's engine, compiled on the host), (ii) libm, (iii)
brute-force recomputation of the action from its definition, (iv) exact transition
matrices, (v) exact enumeration and transfer matrices, and (vi) exact diagonalisation
of the transverse-field Hamiltonian.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
TWO32 = 4294967296.0


# ------------------------------------------------------------------ brute force helpers

def slice_energy(inst, s_k):
    """E(s) = sum_edges J s_i s_j + sum_i h s_i for one slice (int)."""
    e = 0
    if inst.n_edges:
        e += int(np.sum(inst.J.astype(np.int64) * s_k[inst.edges[:, 0]] * s_k[inst.edges[:, 1]]))
    e += int(np.sum(inst.h.astype(np.int64) * s_k))
    return e


def replica_terms(inst, s):
    """(E_cl, C) of one replica s[M][N] straight from the definitions."""
    s = s.astype(np.int64)
    E = sum(slice_energy(inst, s[k]) for k in range(inst.M))
    C = 0
    if inst.M >= 2:
        C = int(sum(np.sum(s[k] * s[(k + 1) % inst.M]) for k in range(inst.M)))
    return E, C


def action(inst, s, rung):
    E, C = replica_terms(inst, s)
    K = inst.K[rung] if inst.M >= 2 else 0.0
    return inst.b[rung] * E - K * C


def classes(inst):
    """Update classes in sweep order: (p, g) -> list of (k, i)."""
    P = 2 if inst.M >= 2 else 1
    out = []
    for p in range(P):
        for g in range(inst.n_colors):
            out.append([(k, i) for k in range(p, inst.M, P) for i in range(inst.N)
                        if inst.color[i] == g])
    return out


# ------------------------------------------------------------------ Philox

def _read_kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = _read_kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


def test_philox_matches_rocrand_engine(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "philox_x")
    subprocess.check_call([hipcc, "-O1", "-o", exe,
                           os.path.join(HERE, "native", "philox_rocrand_xcheck.cpp")],
                          cwd=str(tmp_path))
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(300):
        key = rng.integers(0, 2 ** 32, size=2)
        ctr = rng.integers(0, 2 ** 32, size=4)
        ctr[1] %= 2 ** 30  # the engine is positioned through a 64-bit offset 4*(c1:c0)
        cases.append((key, ctr))
    cases.append((np.array([0, 0]), np.array([0, 0, 0, 0])))
    inp = "\n".join(f"{k[0]} {k[1]} {c[0]} {c[1]} {c[2]} {c[3]}" for k, c in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    assert len(lines) == len(cases)
    for (key, ctr), line in zip(cases, lines):
        want = [int(x) for x in line.split()]
        got = [int(x) for x in oracle.philox4x32_10(ctr, key)]
        assert got == want


def test_draw_words_follow_counter_layout():
    # flip word: slice k = 2m + p; word (m & 3) of
    # Philox(((2i + p) * ceil((M/2)/4) + m // 4, t, c, n), (lo, hi ^ 0))
    seed = 0x0123456789ABCDEF
    n, c, t = 5, 3, 77
    for M in (1, 2, 6, 16):
        Mh = M // 2 if M >= 2 else 1
        G = (Mh + 3) // 4
        for k in range(M):
            p, m = (k % 2, k // 2) if M >= 2 else (0, 0)
            for i in range(7):
                w = oracle.philox4x32_10([(2 * i + p) * G + m // 4, t, c, n],
                                         [seed & 0xFFFFFFFF, seed >> 32])
                assert oracle.flip_word(seed, n, M, c, t, k, i) == int(w[m & 3])
                w = oracle.philox4x32_10([(2 * i + p) * G + m // 4, 0, c, n],
                                         [seed & 0xFFFFFFFF, (seed >> 32) ^ 0x494E4954])
                assert oracle.init_spin(seed, n, M, c, k, i) == (1 if int(w[m & 3]) >> 31 else -1)
    w = oracle.philox4x32_10([6, 11, 0, n], [seed & 0xFFFFFFFF, (seed >> 32) ^ 0x53574150])
    assert oracle.swap_word(seed, n, 6, 11) == int(w[0])


def test_every_draw_uses_a_distinct_counter():
    """Within one sweep of one replica every (slice, site) attempt reads a different
    (counter, word) pair of the oracle's draw layout, so no random number is reused."""
    seed = 99
    for N, M in ((5, 1), (6, 2), (7, 6), (9, 16), (3, 40)):
        words = [oracle.flip_word(seed, 0, M, 0, 0, k, i) for k in range(M) for i in range(N)]
        # 32-bit words from distinct counters collide with probability ~ n^2 / 2^33
        assert len(set(words)) == len(words)


# ------------------------------------------------------------------ exp and thresholds

def test_exp_det_close_to_libm():
    xs = np.concatenate([np.linspace(-32.0, 0.0, 20001),
                         -np.random.default_rng(1).random(20000) * 32.0,
                         -np.logspace(-300, 1.5, 2000)])
    worst = 0.0
    for x in xs:
        want = math.exp(float(x))
        got = oracle.exp_det(float(x))
        worst = max(worst, abs(got - want) / want)
    assert worst < 1e-15
    assert oracle.exp_det(0.0) == 1.0
    assert oracle.exp_det(-32.5) == 0.0


def test_threshold_is_quantised_metropolis():
    assert oracle.metropolis_threshold(0.0) == 0xFFFFFFFF
    assert oracle.metropolis_threshold(-3.0) == 0xFFFFFFFF
    prev = 0xFFFFFFFF
    for dS in np.concatenate([np.linspace(1e-12, 40.0, 40001), [1e-300, 5e-17, 22.18, 23.0]]):
        thr = oracle.metropolis_threshold(float(dS))
        p = (thr + 1) / TWO32
        want = math.exp(-float(dS))
        assert p >= 1.0 / TWO32
        assert abs(p - want) <= 1.0 / TWO32 or (want < 1.0 / TWO32 and thr == 0)
        if dS > 1e-12 and dS < 40.0:
            assert thr <= prev or prev == 0xFFFFFFFF
            prev = thr


def test_swap_threshold_symmetry():
    # P(accept x<->y) / P(accept y<->x) = exp(D) up to the 2^-32 quantisation
    for D in np.linspace(-20.0, 20.0, 4001):
        fwd = (oracle.metropolis_threshold(-D) + 1) / TWO32
        bwd = (oracle.metropolis_threshold(D) + 1) / TWO32
        assert abs(fwd - math.exp(D) * bwd) <= (1 + math.exp(D)) / TWO32


# ------------------------------------------------------------------ single-site kernel

@pytest.mark.parametrize("M", [1, 2, 4])
def test_single_site_kernel_detailed_balance(M):
    """Exact transition probabilities of every single-site update of a 2-site system
    (states enumerated) satisfy detailed balance w.r.t. exp(-S) to 2^-32."""
    rng = np.random.default_rng(3)
    inst = W.make_instance(2, np.array([[0, 1]]), np.array([2], np.int8),
                           np.array([1, -1], np.int8), M, [0.7], 1.3)
    n = 2 * M
    S = np.zeros(2 ** n)
    for x in range(2 ** n):
        s = np.array([1 if (x >> b) & 1 else -1 for b in range(n)], np.int8).reshape(M, 2)
        S[x] = action(inst, s, 0)
    pi = np.exp(-(S - S.min()))
    pi /= pi.sum()
    worst = 0.0
    for x in range(2 ** n):
        for b in range(n):
            y = x ^ (1 << b)
            pxy = (oracle.metropolis_threshold(S[y] - S[x]) + 1) / TWO32
            pyx = (oracle.metropolis_threshold(S[x] - S[y]) + 1) / TWO32
            worst = max(worst, abs(pi[x] * pxy - pi[y] * pyx))
    assert worst <= 2.0 / TWO32
    del rng


# ------------------------------------------------------------------ brute-force trajectory

def brute_force_sweeps(inst, seed, index, s, rung_of, t0, n_sweeps):
    """Reference sweep: every attempted flip's change of E_cl and C is recomputed from
    the definitions over the whole replica (no local fields)."""
    s = s.copy()
    for t in range(t0, t0 + n_sweeps):
        for cls in classes(inst):
            for c in range(inst.R):
                rung = rung_of[c]
                for (k, i) in cls:
                    E0, C0 = replica_terms(inst, s[c])
                    s[c, k, i] = -s[c, k, i]
                    E1, C1 = replica_terms(inst, s[c])
                    s[c, k, i] = -s[c, k, i]
                    K = inst.K[rung] if inst.M >= 2 else 0.0
                    dS = inst.b[rung] * float(E1 - E0) - K * float(C1 - C0)
                    thr = oracle.metropolis_threshold(dS)
                    u = oracle.flip_word(seed, index, inst.M, c, t, k, i)
                    if u <= thr:
                        s[c, k, i] = -s[c, k, i]
    return s


@pytest.mark.parametrize("N,M,R,d", [(5, 4, 2, 2), (6, 2, 3, 3), (4, 1, 2, 3), (7, 6, 2, 2)])
def test_sweep_matches_brute_force(N, M, R, d):
    rng = np.random.default_rng([11, N, M, R])
    inst = W.random_small_instance(rng, N, M, R, d=d, jmax=2, hmax=2, t_min=0.4, t_max=2.0)
    seed = 0xDEADBEEF12345678
    o = oracle.OracleChain(inst, seed, index=3)
    # scramble the permutation so rung lookups are exercised
    perm = rng.permutation(R).astype(np.int32)
    o.replica_of[:] = perm
    o.rung_of[perm] = np.arange(R, dtype=np.int32)
    s0 = o.s.copy()
    o.sweep(3)
    ref = brute_force_sweeps(inst, seed, 3, s0, o.rung_of.copy(), 0, 3)
    assert np.array_equal(o.s, ref)
    E, Cc = zip(*[replica_terms(inst, o.s[c]) for c in range(R)])
    assert np.array_equal(o.E, np.array(E)) and np.array_equal(o.C, np.array(Cc))
    assert o.t == 3


def paired_order_sweeps(inst, seed, index, s, rung_of, t0, n_sweeps):
    """Sweeps in the order of the paired-class kernels: a step takes colour class g of
    the even slices of sweep t together with class g - 1 of the odd slices (class
    n_colors - 1 of sweep t - 1 when g = 0), and a last step finishes the odd slices of
    the last sweep.  Every decision of a step is taken from the state at the step's
    start, as concurrent lanes see it; the flips are applied after."""
    s = s.copy()
    nc = inst.n_colors

    def members(p, g):
        return [(k, i) for k in range(p, inst.M, 2) for i in range(inst.N) if inst.color[i] == g]

    t_end = t0 + n_sweeps
    for t in range(t0, t_end + 1):
        for g in range(nc if t < t_end else 1):
            parts = []
            if t < t_end:
                parts.append((t, members(0, g)))
            if g > 0 or t > t0:
                parts.append((t if g > 0 else t - 1, members(1, g - 1 if g > 0 else nc - 1)))
            flips = []
            for c in range(inst.R):
                rung = rung_of[c]
                K = inst.K[rung]
                E0, C0 = replica_terms(inst, s[c])
                for (tt, cls) in parts:
                    for (k, i) in cls:
                        s[c, k, i] = -s[c, k, i]
                        E1, C1 = replica_terms(inst, s[c])
                        s[c, k, i] = -s[c, k, i]
                        dS = inst.b[rung] * float(E1 - E0) - K * float(C1 - C0)
                        u = oracle.flip_word(seed, index, inst.M, c, tt, k, i)
                        if u <= oracle.metropolis_threshold(dS):
                            flips.append((c, k, i))
            for (c, k, i) in flips:
                s[c, k, i] = -s[c, k, i]
    return s


@pytest.mark.parametrize("N,M,R,d", [(6, 4, 2, 2), (7, 6, 2, 3), (9, 8, 2, 4)])
def test_paired_class_order_keeps_the_trajectory(N, M, R, d):
    """Class g of the even slices and class g - 1 of the odd slices share no site, and
    an update reads the other parity only at its own site: taking them as one step of
    simultaneous decisions reproduces the plain order (all even-slice classes, then all
    odd-slice classes) spin for spin.  Instances with two to four colour classes."""
    rng = np.random.default_rng([12, N, M, R, d])
    inst = W.random_small_instance(rng, N, M, R, d=d, jmax=2, hmax=2, t_min=0.4, t_max=2.0)
    assert inst.n_colors >= 2
    seed = 0x5EED0000A11CE5
    o = oracle.OracleChain(inst, seed, index=5)
    s0 = o.s.copy()
    rung_of = o.rung_of.copy()
    o.sweep(3)
    assert not np.array_equal(o.s, s0)
    assert np.array_equal(paired_order_sweeps(inst, seed, 5, s0, rung_of, 0, 3), o.s)


def test_simultaneous_step_over_neighbouring_classes_changes_the_trajectory():
    """The same simultaneous step taken over two classes of one parity (neighbouring sites
    of one slice) does change the trajectory on a small ferromagnet: the test above is not
    passing for want of interactions."""
    rng = np.random.default_rng([13])
    inst = W.random_small_instance(rng, 6, 2, 1, d=2, jmax=1, hmax=0, t_min=0.3, t_max=0.3)
    seed = 0x5EED0000B0B
    o = oracle.OracleChain(inst, seed, index=1)
    s0 = o.s.copy()
    rung_of = o.rung_of.copy()
    o.sweep(4)
    s = s0.copy()
    for t in range(4):
        for p in range(2):
            # all classes of the parity as one simultaneous step
            cls = [(k, i) for k in range(p, inst.M, 2) for i in range(inst.N)]
            flips = []
            for c in range(inst.R):
                rung = rung_of[c]
                E0, C0 = replica_terms(inst, s[c])
                for (k, i) in cls:
                    s[c, k, i] = -s[c, k, i]
                    E1, C1 = replica_terms(inst, s[c])
                    s[c, k, i] = -s[c, k, i]
                    dS = inst.b[rung] * float(E1 - E0) - inst.K[rung] * float(C1 - C0)
                    if oracle.flip_word(seed, 1, inst.M, c, t, k, i) <= oracle.metropolis_threshold(dS):
                        flips.append((c, k, i))
            for (c, k, i) in flips:
                s[c, k, i] = -s[c, k, i]
    assert not np.array_equal(s, o.s)


def test_init_spins_and_energies_from_definition():
    rng = np.random.default_rng(5)
    inst = W.random_small_instance(rng, 9, 4, 3, d=2, jmax=3, hmax=2)
    seed = 42
    o = oracle.OracleChain(inst, seed, index=2)
    for c in range(3):
        for k in range(4):
            for i in range(9):
                assert o.s[c, k, i] == oracle.init_spin(seed, 2, 4, c, k, i)
        assert (o.E[c], o.C[c]) == replica_terms(inst, o.s[c])
    assert list(o.replica_of) == [0, 1, 2] and list(o.rung_of) == [0, 1, 2]
    assert list(o.label) == [oracle.LABEL_UP, oracle.LABEL_NONE, oracle.LABEL_NONE]


# ------------------------------------------------------------------ exchange

def test_swap_log_ratio_formula():
    """(b_r - b_{r+1})(E_x - E_y) - (K_r - K_{r+1})(C_x - C_y) equals the log ratio of the
    product measure after/before exchanging x and y (from the definitions)."""
    rng = np.random.default_rng(9)
    inst = W.random_small_instance(rng, 6, 4, 2, d=3, jmax=2, hmax=1)
    for _ in range(50):
        x = rng.choice(np.array([-1, 1], np.int8), size=(4, 6))
        y = rng.choice(np.array([-1, 1], np.int8), size=(4, 6))
        direct = (action(inst, x, 0) + action(inst, y, 1)) - (action(inst, y, 0) + action(inst, x, 1))
        Ex, Cx = replica_terms(inst, x)
        Ey, Cy = replica_terms(inst, y)
        D = (inst.b[0] - inst.b[1]) * float(Ex - Ey) - (inst.K[0] - inst.K[1]) * float(Cx - Cy)
        assert abs(D - direct) <= 1e-12 * max(1.0, abs(direct))


def reference_exchange(inst, seed, index, E, C, replica_of, label, rt, e):
    R = inst.R
    replica_of = replica_of.copy()
    label = label.copy()
    rt = rt.copy()
    acc = np.zeros(R - 1, np.uint64)
    att = np.zeros(R - 1, np.uint64)
    for r in range(e % 2, R - 1, 2):
        x, y = replica_of[r], replica_of[r + 1]
        K = inst.K if inst.M >= 2 else np.zeros(R)
        D = (inst.b[r] - inst.b[r + 1]) * float(E[x] - E[y]) - (K[r] - K[r + 1]) * float(C[x] - C[y])
        att[r] += 1
        if oracle.swap_word(seed, index, r, e) <= oracle.metropolis_threshold(-D):
            replica_of[r], replica_of[r + 1] = y, x
            acc[r] += 1
    cold, hot = replica_of[0], replica_of[R - 1]
    if label[cold] == oracle.LABEL_DOWN:
        rt[cold] += 1
        label[cold] = oracle.LABEL_UP
    elif label[cold] == oracle.LABEL_NONE:
        label[cold] = oracle.LABEL_UP
    if label[hot] == oracle.LABEL_UP:
        label[hot] = oracle.LABEL_DOWN
    nup = np.array([label[replica_of[r]] == oracle.LABEL_UP for r in range(R)], np.uint64)
    ndown = np.array([label[replica_of[r]] == oracle.LABEL_DOWN for r in range(R)], np.uint64)
    return replica_of, label, rt, acc, att, nup, ndown


def test_exchange_matches_reference_step():
    rng = np.random.default_rng(21)
    inst = W.random_small_instance(rng, 6, 4, 7, d=3, jmax=1, hmax=1, t_min=0.5, t_max=1.5)
    seed = 99
    o = oracle.OracleChain(inst, seed, index=1)
    acc_tot = np.zeros(6, np.uint64)
    att_tot = np.zeros(6, np.uint64)
    up_tot = np.zeros(7, np.uint64)
    down_tot = np.zeros(7, np.uint64)
    for step in range(40):
        o.sweep(1)
        E = o.E.copy(); Cc = o.C.copy()
        want = reference_exchange(inst, seed, 1, E, Cc, o.replica_of, o.label, o.rt, o.e)
        sums_before = o.sumE.copy()
        o.exchange()
        assert np.array_equal(o.replica_of, want[0])
        assert np.array_equal(o.label, want[1])
        assert np.array_equal(o.rt, want[2])
        acc_tot += want[3]; att_tot += want[4]
        up_tot += want[5]; down_tot += want[6]
        assert np.array_equal(o.acc, acc_tot) and np.array_equal(o.att, att_tot)
        assert np.array_equal(o.nup, up_tot) and np.array_equal(o.ndown, down_tot)
        assert np.array_equal(o.rung_of[o.replica_of], np.arange(7))
        assert np.array_equal(o.sumE - sums_before, E[o.replica_of])
    assert o.e == 40 and o.n_acc == 40


def test_equal_rungs_always_swap():
    rng = np.random.default_rng(2)
    inst = W.random_small_instance(rng, 5, 4, 4, d=2)
    inst = inst.with_ladder(np.full(4, inst.b[1]), np.full(4, inst.K[1]))
    o = oracle.OracleChain(inst, 5)
    o.run(2, 30)
    assert np.array_equal(o.acc[:3], o.att[:3]) and o.att[:3].sum() > 0


def test_round_trip_counting_on_forced_walk():
    """With all rungs equal every attempted swap succeeds, so the replica permutation is
    a deterministic even/odd shuffle; count round trips by following the walk."""
    rng = np.random.default_rng(4)
    inst = W.random_small_instance(rng, 4, 2, 4, d=2)
    inst = inst.with_ladder(np.full(4, 0.3), np.full(4, 0.5))
    o = oracle.OracleChain(inst, 17)
    pos = np.arange(4)  # rung of each replica
    label = np.array([1, 0, 0, 0])
    rt = np.zeros(4, int)
    for e in range(40):
        o.sweep(1)
        o.exchange()
        for r in range(e % 2, 3, 2):
            a, b = np.where(pos == r)[0][0], np.where(pos == r + 1)[0][0]
            pos[a], pos[b] = r + 1, r
        cold, hot = np.where(pos == 0)[0][0], np.where(pos == 3)[0][0]
        if label[cold] == 2:
            rt[cold] += 1
            label[cold] = 1
        elif label[cold] == 0:
            label[cold] = 1
        if label[hot] == 1:
            label[hot] = 2
    assert np.array_equal(o.rung_of, pos)
    assert np.array_equal(o.rt.astype(int), rt) and rt.sum() > 0


# ------------------------------------------------------------------ metamorphic

def test_metamorphic_relations():
    rng = np.random.default_rng(8)
    inst = W.random_small_instance(rng, 11, 6, 3, d=3, jmax=2, hmax=1)
    a = oracle.OracleChain(inst, 1234)
    b = oracle.OracleChain(inst, 1234)
    c = oracle.OracleChain(inst, 1234)
    for _ in range(5):
        a.sweep(4)
        for _ in range(4):
            b.sweep(1)
        c.sweep(4, shuffle_seed=987654321)
        a.exchange(); b.exchange(); c.exchange()
    for n in oracle.OracleChain.ARRAYS:
        assert np.array_equal(getattr(a, n), getattr(b, n)), n
        assert np.array_equal(getattr(a, n), getattr(c, n)), n
    # checkpoint / resume
    snap = a.snapshot()
    a.run(3, 5)
    d = oracle.OracleChain(inst, 1234, init=False)
    d.restore(snap)
    d.run(3, 5)
    for n in oracle.OracleChain.ARRAYS:
        assert np.array_equal(getattr(a, n), getattr(d, n)), n


def test_zero_couplings_keep_classical_energy_flat():
    inst = W.make_instance(6, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                           np.zeros(6, np.int8), 4, [0.5, 1.0], 1.0)
    o = oracle.OracleChain(inst, 3)
    o.run(1, 20)
    assert np.all(o.E == 0) and np.all(o.sumE == 0)


# ------------------------------------------------------------------ exact distributions

def batch_mean_error(x, n_batches=20):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // n_batches
    bm = x[: m * n_batches].reshape(n_batches, m).mean(axis=1)
    return bm.std(ddof=1) / math.sqrt(n_batches)


def run_series(o, k, n_cycles, burn):
    """Per-rung series of (E_cl, C) sampled after every exchange step."""
    o.run(k, burn)
    Es, Cs = [], []
    for _ in range(n_cycles):
        o.run(k, 1)
        Es.append(o.E[o.replica_of].copy())
        Cs.append(o.C[o.replica_of].copy())
    return np.array(Es, dtype=np.float64), np.array(Cs, dtype=np.float64)


def test_classical_pt_matches_exact_enumeration():
    """M = 1: per-rung mean energy and energy histogram of the PT chain against the
    exact Boltzmann distribution of all 2^N states."""
    rng = np.random.default_rng([31, 10])
    inst = W.random_small_instance(rng, 10, 1, 4, d=3, jmax=1, hmax=1, t_min=0.6, t_max=3.0)
    o = oracle.OracleChain(inst, 77)
    Es, _ = run_series(o, 1, 40000, 2000)
    states = np.array([[1 if (x >> b) & 1 else -1 for b in range(10)] for x in range(1024)],
                      dtype=np.int64)
    energies = np.array([slice_energy(inst, s) for s in states], dtype=np.float64)
    for r in range(inst.R):
        w = np.exp(-inst.b[r] * (energies - energies.min()))
        w /= w.sum()
        mean_exact = float(np.sum(w * energies))
        err = batch_mean_error(Es[:, r])
        assert abs(Es[:, r].mean() - mean_exact) < 5 * err + 1e-9, (r, Es[:, r].mean(), mean_exact, err)
        # histogram of energy levels
        levels = np.unique(energies)
        p_exact = np.array([w[energies == L].sum() for L in levels])
        p_emp = np.array([(Es[:, r] == L).mean() for L in levels])
        assert np.max(np.abs(p_emp - p_exact)) < 0.02


def transfer_matrix_exact(inst, rung):
    """Exact <E_cl>/M and <C>/M of the M-slice Suzuki-Trotter chain at one rung, from
    the 2^N x 2^N transfer matrix (no sampling)."""
    N, M = inst.N, inst.M
    b, K = inst.b[rung], inst.K[rung]
    states = np.array([[1 if (x >> q) & 1 else -1 for q in range(N)] for x in range(2 ** N)],
                      dtype=np.float64)
    E = np.array([slice_energy(inst, s.astype(np.int64)) for s in states], dtype=np.float64)
    overlap = states @ states.T  # sum_i s_i s'_i
    T = np.exp(K * overlap)
    V = np.exp(-0.5 * b * (E - E.min()))
    Wm = V[:, None] * T * V[None, :]
    lam, U = np.linalg.eigh(Wm)
    lam_s = lam / np.abs(lam).max()
    WM1 = (U * lam_s ** (M - 1)) @ U.T
    WM = (U * lam_s ** M) @ U.T
    Z = np.trace(WM)
    e_mean = np.sum(np.diag(WM) * E) / Z
    c_mean = np.sum((V[:, None] * (T * overlap) * V[None, :]) * WM1.T) / (Z * np.abs(lam).max())
    return e_mean, c_mean


@pytest.mark.parametrize("N,M", [(1, 8), (5, 8)])
def test_st_pt_matches_transfer_matrix(N, M):
    """Quantum (M >= 2) chains: per-rung <E_cl>/M and <C>/M against the exact transfer-
    matrix values of the same finite-M action."""
    rng = np.random.default_rng([41, N, M])
    inst = W.random_small_instance(rng, N, M, 4, d=2, jmax=1, hmax=1, t_min=0.4, t_max=2.0,
                                   Gamma=1.0)
    o = oracle.OracleChain(inst, 555)
    Es, Cs = run_series(o, 1, 30000, 2000)
    for r in range(inst.R):
        e_ex, c_ex = transfer_matrix_exact(inst, r)
        e_err = batch_mean_error(Es[:, r] / M)
        c_err = batch_mean_error(Cs[:, r] / M)
        assert abs(Es[:, r].mean() / M - e_ex) < 5 * e_err + 1e-9, (r, Es[:, r].mean() / M, e_ex, e_err)
        assert abs(Cs[:, r].mean() / M - c_ex) < 5 * c_err + 1e-9, (r, Cs[:, r].mean() / M, c_ex, c_err)


def free_spin_closed_form(b, K, h, M):
    """Single spin, M slices, field h: Z = lam+^M + lam-^M with
    lam+- = e^K cosh(bh) +- sqrt(e^{2K} sinh^2(bh) + e^{-2K}).  Returns
    (<s^k s^{k+1}>, <s^k>) from central differences of ln Z in K and in h."""
    def lnZ(K_, h_):
        a = math.exp(K_) * math.cosh(b * h_)
        r = math.sqrt(math.exp(2 * K_) * math.sinh(b * h_) ** 2 + math.exp(-2 * K_))
        return math.log((a + r) ** M + (a - r) ** M)
    d = 1e-6
    corr = (lnZ(K + d, h) - lnZ(K - d, h)) / (2 * d) / M
    mag = -(lnZ(K, h + d) - lnZ(K, h - d)) / (2 * d) / (M * b)
    return corr, mag


def test_free_spin_closed_form_exact():
    """N=1, h=0: a periodic Ising ring in imaginary time,
    <s^k s^{k+1}> = (tanh K + tanh^{M-1} K)/(1 + tanh^M K), and the thermodynamic
    estimator equals -Gamma tanh(beta Gamma) at every M (no sampling)."""
    for M in (2, 4, 16):
        inst = W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                               np.zeros(1, np.int8), M, [0.5, 1.0], 1.0)
        for r in range(2):
            th = math.tanh(inst.K[r])
            corr = (th + th ** (M - 1)) / (1 + th ** M)
            e_ex, c_ex = transfer_matrix_exact(inst, r)
            assert abs(c_ex - corr) < 1e-12
            assert abs(free_spin_closed_form(inst.b[r], inst.K[r], 0, M)[0] - corr) < 1e-8
            beta = 1.0 / inst.T[r]
            obs = dict(n_acc=1, sumE=np.array([0] * 2), sumC=np.array([corr * M] * 2))
            _, H = oracle.energy_estimators(obs, inst)
            assert abs(H[r] + math.tanh(beta * inst.Gamma)) < 1e-12


def test_free_spin_in_field_sampled():
    """N=1 with h=1: sampled <s^k s^{k+1}> and <s^k> of the PT chain against the
    two-state transfer-matrix closed form.  (At h = 0 a lone spin is a decoupled
    zero-field ring, on which the Metropolis rule with a fixed update order is
    reducible -- see test_fixed_order_metropolis_reducible_on_free_ring.)"""
    M = 8
    inst = W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                           np.ones(1, np.int8), M, [0.5, 1.0], 1.0)
    o = oracle.OracleChain(inst, 8)
    Es, Cs = run_series(o, 1, 30000, 1000)
    for r in range(2):
        corr, mag = free_spin_closed_form(inst.b[r], inst.K[r], 1.0, M)
        c_err = batch_mean_error(Cs[:, r] / M)
        m_err = batch_mean_error(Es[:, r] / M)  # E_cl/M = h <s>
        assert abs(Cs[:, r].mean() / M - corr) < 5 * c_err + 1e-9
        assert abs(Es[:, r].mean() / M - mag) < 5 * m_err + 1e-9


def test_fixed_order_metropolis_reducible_on_free_ring():
    """A known property of the Metropolis rule (downhill and level moves always taken)
    under a fixed update order: on a lone zero-field spin the M-slice ring splits into
    closed classes, so the sampled <s^k s^{k+1}> is biased.  The oracle must show it
    (a heat-bath rule, or a wrong always-accept test, would not)."""
    M = 4
    inst = W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                           np.zeros(1, np.int8), M, [0.5, 1.0], 1.0)
    o = oracle.OracleChain(inst, 8)
    _, Cs = run_series(o, 1, 20000, 1000)
    th = math.tanh(inst.K[0])
    corr = (th + th ** (M - 1)) / (1 + th ** M)
    assert abs(Cs[:, 0].mean() / M - corr) > 0.03


def tfim_ed(inst, beta):
    """Exact <H> and <H_P> of H = sum J sz sz + sum h sz - Gamma sum sx (dense ED)."""
    N = inst.N
    dim = 2 ** N
    states = np.array([[1 if (x >> q) & 1 else -1 for q in range(N)] for x in range(dim)])
    diag = np.array([slice_energy(inst, s.astype(np.int64)) for s in states], dtype=np.float64)
    H = np.diag(diag)
    for q in range(N):
        idx = np.arange(dim)
        H[idx, idx ^ (1 << q)] -= inst.Gamma
    lam, U = np.linalg.eigh(H)
    w = np.exp(-beta * (lam - lam.min()))
    Z = w.sum()
    Hm = float(np.sum(w * lam) / Z)
    HP = float(np.sum(w * np.einsum("ij,i,ij->j", U, diag, U)) / Z)
    return Hm, HP


def test_trotter_limit_approaches_exact_diagonalisation():
    """The finite-M Suzuki-Trotter estimator (exact, via transfer matrices) converges to
    the ED value of the 8-spin transverse-field Ising model of the first workload as
    1/M^2, and is within 1e-2 relative at M = 256."""
    base = W.config1()
    for T in (0.5, 1.0):
        beta = 1.0 / T
        H_ed, HP_ed = tfim_ed(base, beta)
        errs = []
        for M in (16, 32, 64, 256):
            inst = W.make_instance(base.N, base.edges, base.J, base.h, M, [T], base.Gamma,
                                   relabel=False)
            e_ex, c_ex = transfer_matrix_exact(inst, 0)
            obs = dict(n_acc=1, sumE=np.array([e_ex * M]), sumC=np.array([c_ex * M]))
            _, H = oracle.energy_estimators(obs, inst)
            errs.append(abs(H[0] - H_ed))
        assert errs[-1] / abs(H_ed) < 1e-2
        # quadratic convergence: halving 1/M reduces the error about fourfold
        assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0


def test_sampled_estimator_near_exact_diagonalisation():
    """The oracle's sampled thermodynamic estimator at M = 64 agrees with ED of the
    8-spin model within the Trotter error plus sampling error."""
    base = W.config1()
    T = 1.0
    M = 64
    inst = W.make_instance(base.N, base.edges, base.J, base.h, M, [0.9, 1.0, 1.1],
                           base.Gamma, relabel=False)
    o = oracle.OracleChain(inst, 2024)
    Es, Cs = run_series(o, 2, 6000, 300)
    x = inst.Gamma / (T * M)
    Hs = Es[:, 1] / M - inst.N * inst.Gamma / math.tanh(2 * x) + (inst.Gamma / M) * Cs[:, 1] / math.sinh(2 * x)
    H_ed, _ = tfim_ed(base, 1.0 / T)
    e_ex, c_ex = transfer_matrix_exact(inst, 1)
    H_tm = e_ex - inst.N * inst.Gamma / math.tanh(2 * x) + (inst.Gamma / M) * c_ex * M / math.sinh(2 * x)
    err = batch_mean_error(Hs)
    assert abs(Hs.mean() - H_tm) < 5 * err
    assert abs(Hs.mean() - H_ed) < 5 * err + abs(H_tm - H_ed) + 1e-3 * abs(H_ed)
