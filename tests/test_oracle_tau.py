"""Pins of the oracle's imaginary-time correlation accumulators (CPU only).

Ct_l = sum_k sum_i s_i^k s_i^{(k + lag_l) mod M} of the replica at each rung is added to
sumCt[r][l] at every exchange step, with lag_l = max(1, floor((l + 1) M / 16)).  Pinned
against: closed forms on special configurations; the per-rung bookkeeping replayed
step by step; the exact expectation of the M-slice Suzuki-Trotter chain (2^N x 2^N
transfer matrices, no sampling) against the oracle's sampled averages; and that exact
finite-M expectation against the quantum imaginary-time correlation of the transverse-
field Ising model from exact diagonalisation, converging as 1/M^2 -- the correlation
whose decay gives the gap that the paper's application computes.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def slice_energy(inst, s_k):
    e = 0
    if inst.n_edges:
        e += int(np.sum(inst.J.astype(np.int64) * s_k[inst.edges[:, 0]] * s_k[inst.edges[:, 1]]))
    return e + int(np.sum(inst.h.astype(np.int64) * s_k))


def batch_mean_error(x, n_batches=20):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // n_batches
    bm = x[: m * n_batches].reshape(n_batches, m).mean(axis=1)
    return bm.std(ddof=1) / math.sqrt(n_batches)


def states_of(N):
    return np.array([[1 if (x >> q) & 1 else -1 for q in range(N)] for x in range(2 ** N)],
                    dtype=np.float64)


def tau_corr_transfer_matrix(inst, rung):
    """Exact <Ct_l> of the M-slice chain at one rung: with W = V T V the symmetric
    transfer matrix (T = exp(K s.s'), V = exp(-b E / 2)),
    <s_i^0 s_i^d> = Tr[Z_i W^d Z_i W^(M-d)] / Tr[W^M] and <Ct> = M sum_i <s_i^0 s_i^d>."""
    N, M = inst.N, inst.M
    b, K = inst.b[rung], inst.K[rung]
    S = states_of(N)
    E = np.array([slice_energy(inst, s.astype(np.int64)) for s in S], dtype=np.float64)
    T = np.exp(K * (S @ S.T))
    V = np.exp(-0.5 * b * (E - E.min()))
    Wm = V[:, None] * T * V[None, :]
    lam, U = np.linalg.eigh(Wm)
    lam = lam / np.abs(lam).max()

    def power(p):
        return (U * lam ** p) @ U.T

    Z = np.trace(power(M))
    out = np.zeros(oracle.TAU_LAGS)
    for l in range(oracle.TAU_LAGS):
        d = oracle.tau_lag(M, l) % M
        Pd, Prest = power(d), power(M - d)
        tot = 0.0
        for i in range(N):
            zi = S[:, i]
            tot += np.trace((zi[:, None] * Pd) @ (zi[:, None] * Prest))
        out[l] = M * tot / Z
    return out


def tau_corr_ed(inst, beta, taus):
    """(1/N) sum_i <sigma^z_i(tau) sigma^z_i(0)> of H = E(sigma^z) - Gamma sum sigma^x
    (dense exact diagonalisation), and the spectrum."""
    N = inst.N
    dim = 2 ** N
    S = states_of(N)
    diag = np.array([slice_energy(inst, s.astype(np.int64)) for s in S], dtype=np.float64)
    H = np.diag(diag)
    for q in range(N):
        idx = np.arange(dim)
        H[idx, idx ^ (1 << q)] -= inst.Gamma
    lam, U = np.linalg.eigh(H)
    lam0 = lam - lam.min()
    Z = np.exp(-beta * lam0).sum()
    out = []
    for tau in taus:
        g = 0.0
        for i in range(N):
            A = U.T @ (S[:, i][:, None] * U)   # sigma^z_i in the eigenbasis
            g += np.sum(np.exp(-(beta - tau) * lam0)[:, None] * A ** 2 *
                        np.exp(-tau * lam0)[None, :]) / Z
        out.append(g / N)
    return np.array(out), lam


def test_tau_lags():
    assert [oracle.tau_lag(16, l) for l in range(8)] == list(range(1, 9))
    assert [oracle.tau_lag(256, l) for l in range(8)] == [16 * (l + 1) for l in range(8)]
    assert [oracle.tau_lag(24, l) for l in range(8)] == [1, 3, 4, 6, 7, 9, 10, 12]
    for M in (1, 2, 4, 8):
        assert all(oracle.tau_lag(M, l) >= 1 for l in range(8))
        assert oracle.tau_lag(M, 7) == max(1, M // 2)


def test_tau_corr_special_configurations():
    inst = W.random_small_instance(np.random.default_rng(3), 5, 12, 2, d=2)
    o = oracle.OracleChain(inst, 1)
    N, M = inst.N, inst.M
    up = np.ones((inst.R, M, N), np.int8)
    assert np.all(o.tau_corr(up) == N * M)
    # alternating in imaginary time: s^k = (-1)^k, so every product is (-1)^lag
    alt = np.ones((inst.R, M, N), np.int8)
    alt[:, 1::2, :] = -1
    want = np.array([N * M * (-1) ** oracle.tau_lag(M, l) for l in range(8)])
    assert np.all(o.tau_corr(alt) == want)
    # one flipped spin enters two products of every lag
    one = up.copy()
    one[0, 0, 3] = -1
    assert np.all(o.tau_corr(one)[0] == N * M - 4) and np.all(o.tau_corr(one)[1] == N * M)
    # a random configuration against the rolled sum
    rng = np.random.default_rng(9)
    s = rng.choice(np.array([-1, 1], np.int8), size=(inst.R, M, N))
    got = o.tau_corr(s)
    for c in range(inst.R):
        for l in range(8):
            d = oracle.tau_lag(M, l)
            assert got[c, l] == int(np.sum(s[c].astype(np.int64) * np.roll(s[c], -d, axis=0)))


def test_tau_accumulated_per_rung_at_every_exchange():
    """sumCt[r] grows at each exchange step by Ct of the replica then at rung r."""
    inst = W.random_small_instance(np.random.default_rng(4), 6, 8, 4, d=2)
    o = oracle.OracleChain(inst, 2)
    want = np.zeros((inst.R, 8), np.int64)
    for _ in range(12):
        o.sweep(2)
        o.exchange()
        ct = o.tau_corr()
        want += ct[o.replica_of]
    assert np.array_equal(o.sumCt, want)
    assert o.n_acc == 12


@pytest.mark.parametrize("N,M", [(3, 8), (4, 16)])
def test_tau_sampled_matches_transfer_matrix(N, M):
    """The oracle chain's per-rung averages of Ct_l against the exact transfer-matrix
    expectation of the same finite-M action."""
    rng = np.random.default_rng([61, N, M])
    inst = W.random_small_instance(rng, N, M, 3, d=2, jmax=1, hmax=1, t_min=0.5, t_max=2.0,
                                   Gamma=1.0)
    o = oracle.OracleChain(inst, 99)
    o.run(1, 2000)
    prev = o.sumCt.copy()
    series = []
    for _ in range(20000):
        o.run(1, 1)
        series.append(o.sumCt - prev)
        prev = o.sumCt.copy()
    series = np.array(series, dtype=np.float64)  # [step][rung][lag]
    for r in range(inst.R):
        exact = tau_corr_transfer_matrix(inst, r)
        for l in range(8):
            err = batch_mean_error(series[:, r, l])
            assert abs(series[:, r, l].mean() - exact[l]) < 5 * err + 1e-9, (r, l, exact[l], err)


def test_tau_trotter_limit_approaches_exact_diagonalisation():
    """<Ct_l>/(N M) at lag_l = (l+1) M/16, i.e. imaginary time (l+1) beta/16, converges
    to the ED correlation of the 8-spin transverse-field Ising model of the first
    workload as 1/M^2, within 1e-2 at M = 256."""
    base = W.config1()
    for T in (0.5, 1.0):
        beta = 1.0 / T
        taus = [(l + 1) * beta / 16 for l in range(8)]
        g_ed, _ = tau_corr_ed(base, beta, taus)
        errs = []
        for M in (16, 32, 64, 256):
            inst = W.make_instance(base.N, base.edges, base.J, base.h, M, [T], base.Gamma,
                                   relabel=False)
            g_st = tau_corr_transfer_matrix(inst, 0) / (base.N * M)
            errs.append(np.max(np.abs(g_st - g_ed)))
        assert errs[-1] < 1e-2
        assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0
