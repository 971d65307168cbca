"""FP64 estimators of the sampler's observables, per rung, from its integer accumulators.

The sampler accumulates integers on the device (per rung: sums of E_cl, C and their
squares at every exchange step; per pair: attempted and accepted swaps; per replica:
completed round trips; per rung: steps with an UP / DOWN replica there), and the host
turns them into FP64 estimates, as the paper accumulates in double precision on the
host (Section 5).  Nothing here touches the Markov chain.

A rung is the pair (b, K) of the replica action S = b E_cl - K C, with
E_cl = sum_k E(s^k) and C = sum_k sum_i s_i^k s_i^{k+1} over the M Trotter slices.  For
H = B H_P - A sum_i sigma^x_i at inverse temperature beta the Suzuki-Trotter rung is
b = beta B / M and K = -1/2 ln tanh(x) with x = beta A / M (a temperature ladder at
transverse field Gamma has B = 1, A = Gamma).  Differentiating the Trotter partition
function Z_M = (sinh(2x)/2)^(N M / 2) sum exp(-S) gives, at every M, the estimators

    <H_P>            = <E_cl> / M
    <sum sigma^x>    = N coth(2x) - (<C> / M) / sinh(2x)
    <H>              = B <H_P> - A <sum sigma^x>

with tanh(x) = exp(-2K), so coth(2x) = (1 + t^2) / (2t) and 1/sinh(2x) = (1 - t^2) / (2t)
for t = exp(-2K).  They converge to the quantum values with error O(1/M^2).
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np


def rung_estimators(obs: Dict, N: int, M: int, b: Sequence[float], K: Sequence[float],
                    beta: Optional[Sequence[float]] = None) -> Dict[str, np.ndarray]:
    """Per-rung estimates from one instance's observables (the dict of
    ``Sampler.observables``: sumE, sumC, sumE2, sumC2, n_acc, acc, att, roundtrips, nup,
    ndown, t).

    b, K: the rung constants the instance was built with.  beta: the inverse temperature
    of each rung; omitted, the ladder is taken as a temperature ladder (B = 1, so
    beta = M b and A = x / b = Gamma).

    Returns arrays by rung: H_P, sigma_x, H, E_mean (<E_cl>/M), E_var (variance of
    E_cl/M over the accumulated samples), C_mean (<C>/M), C_var, up_fraction
    (nup / (nup + ndown), NaN where neither was seen); by pair: swap_rate (acc / att);
    and the scalars roundtrip_rate (completed round trips per sweep, summed over
    replicas) and samples (n_acc)."""
    n = int(obs["n_acc"])
    if n < 1:
        raise ValueError("no accumulated samples (run at least one exchange step)")
    b = np.asarray(b, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    M = int(M)
    sumE = np.asarray(obs["sumE"], dtype=np.float64)
    sumC = np.asarray(obs["sumC"], dtype=np.float64)
    # second moments from the int64 sums (exact integers; FP64 from here on)
    sumE2 = np.asarray(obs["sumE2"], dtype=np.float64)
    sumC2 = np.asarray(obs["sumC2"], dtype=np.float64)
    E_mean = sumE / (n * M)
    C_mean = sumC / (n * M)
    E_var = (sumE2 / n - (sumE / n) ** 2) / (M * M)
    C_var = (sumC2 / n - (sumC / n) ** 2) / (M * M)
    if beta is None:
        beta = M * b
    beta = np.asarray(beta, dtype=np.float64)
    B = b * M / beta
    if M >= 2:
        t = np.exp(-2.0 * K)                 # tanh(x)
        coth2x = (1.0 + t * t) / (2.0 * t)
        csch2x = (1.0 - t * t) / (2.0 * t)
        x = np.arctanh(t)
        A = x * M / beta
        sigma_x = N * coth2x - C_mean * csch2x
    else:
        A = np.zeros_like(b)
        sigma_x = np.zeros_like(b)
    H_P = E_mean
    H = B * H_P - A * sigma_x
    acc = np.asarray(obs["acc"], dtype=np.float64)
    att = np.asarray(obs["att"], dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        swap_rate = np.where(att > 0, acc / np.maximum(att, 1.0), np.nan)
        nup = np.asarray(obs["nup"], dtype=np.float64)
        ndown = np.asarray(obs["ndown"], dtype=np.float64)
        up_fraction = np.where(nup + ndown > 0, nup / np.maximum(nup + ndown, 1.0), np.nan)
    t_sweeps = int(obs["t"])
    rt = float(np.sum(np.asarray(obs["roundtrips"], dtype=np.float64)))
    return {"H_P": H_P, "sigma_x": sigma_x, "H": H, "E_mean": E_mean, "E_var": E_var,
            "C_mean": C_mean, "C_var": C_var, "up_fraction": up_fraction,
            "swap_rate": swap_rate,
            "roundtrip_rate": rt / t_sweeps if t_sweeps > 0 else float("nan"),
            "samples": n}


def instance_estimators(obs: Dict, inst) -> Dict[str, np.ndarray]:
    """rung_estimators for an instance record with N, M, b, K and, when it has them,
    temperatures T (beta = 1/T) -- the records of the ``workloads`` module."""
    T = getattr(inst, "T", None)
    beta = None if T is None else 1.0 / np.asarray(T, dtype=np.float64)
    return rung_estimators(obs, inst.N, inst.M, inst.b, inst.K, beta)
