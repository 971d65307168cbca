"""Hamiltonian-parameter (annealing) ladders and gap estimates.

The paper's application (Section 1: Adiabatic QUantum Algorithms, AQUA) computes the
minimum gap between the two lowest states of an adiabatic evolution with this sampler.
The evolution is H(s) = -A(s) sum_i sigma^x_i + B(s) H_P(sigma^z), with H_P = E the
instance's Ising energy.  At inverse temperature beta with M Trotter slices a value of
s is a rung (b, K) of the sampler (its ladders are data, Section 2):

    b = beta B(s) / M,      K = -1/2 ln tanh(beta A(s) / M).

With PT_FLAG_TAU_CORR the sampler accumulates per rung the imaginary-time spin
correlations Ct_l at lags lag_l = max(1, floor((l + 1) M / 16)) slices, i.e. at
tau_l = lag_l beta / M.  G(tau) = Ct / (N M) estimates (1/N) sum_i <sigma^z_i(tau)
sigma^z_i(0)>, which on the periodic imaginary-time interval [0, beta] behaves as
c + a cosh(Delta (beta/2 - tau)) when one excitation Delta above the ground state carries
sigma^z's spectral weight (as at an avoided crossing of the two lowest states).
`fit_gap` fits that form; it needs beta * Delta well above 1.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Sequence, Tuple

import numpy as np

TAU_LAGS = 8


def linear_schedule(s):
    """A(s) = 1 - s, B(s) = s."""
    s = np.asarray(s, dtype=np.float64)
    return 1.0 - s, s


def annealing_rungs(s_values: Sequence[float], beta: float, M: int,
                    schedule: Callable = linear_schedule) -> Tuple[np.ndarray, np.ndarray]:
    """(b_r, K_r) of the rungs s_values (rung 0 first) at inverse temperature beta."""
    A, B = schedule(np.asarray(s_values, dtype=np.float64))
    A = np.broadcast_to(np.asarray(A, dtype=np.float64), np.shape(s_values))
    B = np.broadcast_to(np.asarray(B, dtype=np.float64), np.shape(s_values))
    if np.any(B < 0):
        raise ValueError("B(s) must be >= 0")
    b = beta * B / M
    if M == 1:
        return b, np.zeros_like(b)
    if np.any(A <= 0):
        raise ValueError("A(s) must be > 0 for M >= 2 (the slices decouple at A = 0)")
    K = -0.5 * np.log(np.tanh(beta * A / M))
    return b, K


def with_annealing_ladder(inst, s_values: Sequence[float], beta: float,
                          schedule: Callable = linear_schedule):
    """A copy of a workloads.Instance whose rungs are the values s_values at beta."""
    b, K = annealing_rungs(s_values, beta, inst.M, schedule)
    return dataclasses.replace(inst, R=len(b), b=b, K=K, T=np.full(len(b), 1.0 / beta))


def tau_lag(M: int, l: int) -> int:
    return max(1, (l + 1) * M // 16)


def correlation_curve(obs, N: int, M: int, beta: float) -> Tuple[np.ndarray, np.ndarray]:
    """(tau_l, G[r][l]): imaginary times of the lags and the per-rung averages
    sumCt / (n_acc N M) from the observables of one instance."""
    n = int(obs["n_acc"])
    if n == 0:
        raise ValueError("no exchange steps accumulated")
    taus = np.array([tau_lag(M, l) * beta / M for l in range(TAU_LAGS)])
    G = np.asarray(obs["sumCt"], dtype=np.float64) / (n * N * M)
    return taus, G


def fit_gap(taus: Sequence[float], G: Sequence[float], beta: float) -> float:
    """Delta of the least-squares fit G(tau) = c + a cosh(Delta (beta/2 - tau)); for
    each Delta the pair (c, a) is linear, so the search is one-dimensional (a log grid
    over beta Delta in [0.05, 60], then a bounded refinement)."""
    from scipy.optimize import minimize_scalar
    t = np.asarray(taus, dtype=np.float64)
    g = np.asarray(G, dtype=np.float64)

    def resid(D):
        X = np.stack([np.ones_like(t), np.cosh(D * (beta / 2 - t))], axis=1)
        coef, *_ = np.linalg.lstsq(X, g, rcond=None)
        return float(np.sum((X @ coef - g) ** 2))

    grid = np.geomspace(0.05 / beta, 60.0 / beta, 400)
    r = np.array([resid(D) for D in grid])
    j = int(np.argmin(r))
    lo, hi = grid[max(j - 1, 0)], grid[min(j + 1, len(grid) - 1)]
    res = minimize_scalar(resid, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12})
    return float(res.x)
