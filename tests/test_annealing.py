"""Hamiltonian-parameter (annealing) ladders and the gap fit (CPU).

A rung at (beta, s) of H(s) = -A(s) sum sigma^x + B(s) H_P is the temperature rung of the
transverse-field model at T' = 1 / (beta B), Gamma' = A / B: both give the same (b, K),
which pins the mapping against the temperature form the rest of the package uses.  The
gap fit is pinned on exact imaginary-time correlations -- from exact diagonalisation and
from the finite-M transfer matrix -- of ferromagnetic rings at weak transverse field,
where the two lowest states form an avoided crossing carrying sigma^z's weight (the
situation of the paper's application, Section 1).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_1004_0023_amd import annealing as AN
from test_oracle_tau import states_of, slice_energy, tau_corr_transfer_matrix


def ring(N, M):
    edges = np.array([[i, (i + 1) % N] for i in range(N)])
    edges.sort(axis=1)
    return W.make_instance(N, edges, -np.ones(N, np.int8), np.zeros(N, np.int8), M, [1.0], 1.0,
                           relabel=False)


def ed(inst, A, B):
    """Spectrum and sigma^z_i matrices (eigenbasis) of -A sum sx + B H_P."""
    N = inst.N
    dim = 2 ** N
    S = states_of(N)
    diag = np.array([slice_energy(inst, s.astype(np.int64)) for s in S], dtype=np.float64)
    H = B * np.diag(diag)
    for q in range(N):
        idx = np.arange(dim)
        H[idx, idx ^ (1 << q)] -= A
    lam, U = np.linalg.eigh(H)
    Z = [U.T @ (S[:, i][:, None] * U) for i in range(N)]
    return lam, Z


def ed_corr(lam, Z, beta, taus):
    e = lam - lam.min()
    Zs = np.exp(-beta * e).sum()
    return np.array([sum(np.sum(np.exp(-(beta - t) * e)[:, None] * z ** 2 * np.exp(-t * e)[None, :])
                         for z in Z) / (len(Z) * Zs) for t in taus])


def test_rungs_equal_the_temperature_mapping():
    beta, M = 7.0, 32
    s = np.array([0.2, 0.45, 0.7, 0.9])
    b, K = AN.annealing_rungs(s, beta, M)
    A, B = 1 - s, s
    for r in range(len(s)):
        bt, Kt = W.st_rungs([1.0 / (beta * B[r])], A[r] / B[r], M)
        assert b[r] == pytest.approx(bt[0], rel=1e-14) and K[r] == pytest.approx(Kt[0], rel=1e-12)


def test_rungs_closed_forms_and_limits():
    beta, M = 3.0, 16
    b, K = AN.annealing_rungs([0.0, 0.5], beta, M)
    assert b[0] == 0.0 and K[0] == pytest.approx(-0.5 * np.log(np.tanh(beta / M)))
    assert b[1] == pytest.approx(beta * 0.5 / M)
    assert np.all(AN.annealing_rungs([0.3, 0.6], beta, 1)[1] == 0)  # classical: no K
    with pytest.raises(ValueError):
        AN.annealing_rungs([1.0], beta, M)  # A = 0 decouples the slices
    inst = AN.with_annealing_ladder(ring(4, 8), [0.6, 0.5, 0.4], 10.0)
    assert inst.R == 3 and inst.b.shape == (3,) and inst.K.shape == (3,)


def test_correlation_curve():
    obs = dict(n_acc=4, sumCt=np.full((2, AN.TAU_LAGS), 4 * 3 * 32 // 2))
    taus, G = AN.correlation_curve(obs, 3, 32, 8.0)
    assert np.allclose(taus, [(l + 1) * 2 * 8.0 / 32 for l in range(8)])
    assert np.allclose(G, 0.5)
    assert [AN.tau_lag(24, l) for l in range(8)] == [oracle.tau_lag(24, l) for l in range(8)]


@pytest.mark.parametrize("N", [4, 5, 6])
def test_fit_recovers_gap_from_exact_correlations(N):
    """Ferromagnetic rings at A/B = 0.6 .. 0.9: the fit to the ED correlation at the
    lags' imaginary times (beta = 20) gives E1 - E0 within 3 %."""
    A, B, beta = {4: 0.6, 5: 0.8, 6: 0.9}[N], 1.0, 20.0
    lam, Z = ed(ring(N, 16), A, B)
    taus = [(l + 1) * beta / 16 for l in range(8)]
    g = ed_corr(lam, Z, beta, taus)
    gap = lam[1] - lam[0]
    assert AN.fit_gap(taus[1:], g[1:], beta) == pytest.approx(gap, rel=0.03)


def test_fit_on_finite_trotter_chain_near_exact_gap():
    """The exact M = 128 Suzuki-Trotter correlation (transfer matrix, the chain the
    sampler runs) at an annealing rung gives the ED gap of H(s) within 5 %."""
    beta, M, s = 40.0, 128, 0.6
    base = ring(4, M)
    inst = AN.with_annealing_ladder(base, [s, 0.5], beta)
    ct = tau_corr_transfer_matrix(inst, 0)
    taus, G = AN.correlation_curve(dict(n_acc=1, sumCt=ct[None, :]), inst.N, M, beta)
    lam, _ = ed(base, 1 - s, s)
    assert AN.fit_gap(taus[1:], G[0, 1:], beta) == pytest.approx(lam[1] - lam[0], rel=0.05)
