"""Learned ladders.

The sampler takes a ladder as data: per-rung (b_r, K_r) of the Suzuki-Trotter action
S_r = b_r E_cl - K_r C (Section 2).  Ladder selection is outside the Markov chain (the
paper defers it to its reference [7]); rung 0 carries the target ensemble and every
other rung is an auxiliary distribution, so a ladder can never change what rung 0
samples, only how fast replicas travel between the ends.

Parametrisation.  Temperatures stay geometric on [T_min, T_max].  At fixed Gamma the
Trotter coupling K = -1/2 ln tanh(Gamma/(M T)) grows with T, so hot rungs have stiff
world lines whose single-slice flips are rarely accepted.  The learned part softens
that: with u = r/(R-1) and a per-rung mixing lambda(u) in [0, 1],
    K_r = K_geo,r^(1 - lambda(u_r)) * K_0^lambda(u_r),        b_r = 1/(M T_r),
i.e. a transverse field Gamma_r that rises with T (a temperature/Hamiltonian-parameter
ladder).  lambda = 0 is the geometric ladder, the fallback; rung 0 is unchanged for
every lambda.  The network's 64 outputs are logits of lambda at the knots
u_j = j/63, interpolated linearly to the rungs.

Training data.  For each training instance the sampler itself measures replica round
trips per sweep under linear profiles lambda(u) = clip(a + s (u - 1/2), 0, 1): a small
set of levels a for each of a few slopes s.  Per slope, the best level is the maximiser
of a quadratic fitted to the measured rates (the best measured level when the fit is
not concave), clipped to the scanned range; the target profile is the slope whose
fitted peak is higher, at its best level.  The network (32 -> 128 -> 128 -> 64 FP32,
trained with the library's own kernels, per-output logistic cross entropy) maps
instance features to that profile at the knots.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

N_FEATURES = 32
N_KNOTS = 64
SCAN_LAMBDAS = (0.1, 0.2, 0.3, 0.4, 0.55)   # profile levels a
SCAN_SLOPES = (0.0, 0.25)                   # profile slopes s


# ----------------------------------------------------------------------------- features

def features(inst) -> np.ndarray:
    """32 FP32 instance features: sizes, degree statistics, coupling and field
    histograms, field bound, colours, transverse field, temperature range and the
    Trotter couplings at both ends of the geometric ladder."""
    N, M, R = inst.N, inst.M, inst.R
    deg = np.zeros(N)
    if inst.n_edges:
        np.add.at(deg, inst.edges[:, 0], 1)
        np.add.at(deg, inst.edges[:, 1], 1)
    J = inst.J.astype(np.float64) if inst.n_edges else np.zeros(1)
    h = inst.h.astype(np.float64)
    absJ = np.abs(J)
    T = np.asarray(inst.T, dtype=np.float64)
    t_min, t_max = float(np.nanmin(T)), float(np.nanmax(T))
    _, Kends = st_rungs([t_min, t_max], inst.Gamma, M)
    f = [
        N / 512.0, M / 128.0, R / 64.0, math.log(N), math.log(M), math.log(R),
        deg.min() / 8.0, deg.mean() / 8.0, deg.max() / 8.0, deg.std(),
        float((J < 0).mean()), float((J > 0).mean()), absJ.mean(), absJ.max() / 4.0,
        float((h < 0).mean()), float((h == 0).mean()), float((h > 0).mean()),
        np.abs(h).mean(), absJ.sum() / N, inst.F() / 20.0, inst.n_colors / 8.0,
        inst.Gamma, math.log(t_min), math.log(t_max), math.log(t_max / t_min),
        inst.Gamma / t_min / M, inst.Gamma / t_max / M, math.log(N * M * R),
        float(Kends[0]), float(Kends[1]), math.log(t_max / t_min) / (R - 1),
        math.log(N * M),
    ]
    assert len(f) == N_FEATURES
    return np.asarray(f, dtype=np.float32)


# ----------------------------------------------------------------------------- ladders

def geometric(t_min: float, t_max: float, R: int) -> np.ndarray:
    return t_min * (t_max / t_min) ** (np.arange(R) / (R - 1))


def st_rungs(T: Sequence[float], Gamma: float, M: int) -> Tuple[np.ndarray, np.ndarray]:
    """(b_r, K_r) of the Suzuki-Trotter action: b = 1/(M T), K = -1/2 ln tanh(Gamma/(M T))."""
    T = np.asarray(T, dtype=np.float64)
    b = 1.0 / (M * T)
    K = np.zeros_like(b) if M == 1 else -0.5 * np.log(np.tanh(Gamma / (M * T)))
    return b, K


def knots_to_rungs(lam_knots: Sequence[float], R: int) -> np.ndarray:
    """Per-rung lambda from its values at the knots u_j = j/(n-1)."""
    lam_knots = np.asarray(lam_knots, dtype=np.float64)
    n = lam_knots.shape[0]
    return np.interp(np.arange(R) / (R - 1), np.arange(n) / (n - 1), lam_knots)


def profile(level: float, slope: float, n: int) -> np.ndarray:
    """The linear profile lambda(u) = clip(level + slope (u - 1/2), 0, 1) at u = j/(n-1),
    j = 0 .. n-1 (the rungs of an n-rung ladder, or the knots when n = N_KNOTS)."""
    u = np.arange(n) / (n - 1)
    return np.clip(level + slope * (u - 0.5), 0.0, 1.0)


def coupling_ladder(inst, lam) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(T, b, K) of the geometric-temperature ladder with Trotter-coupling mixing lam
    (a scalar or one value per rung)."""
    T = geometric(float(inst.T[0]), float(inst.T[-1]), inst.R)
    b, K = st_rungs(T, inst.Gamma, inst.M)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), K.shape)
    if inst.M > 1:
        K0 = K[0]
        K = K ** (1.0 - lam) * K0 ** lam
        K[0] = K0                        # the target rung, bit for bit
    return T, b, K


def with_ladder(inst, lam):
    T, b, K = coupling_ladder(inst, lam)
    return dataclasses.replace(inst, b=b, K=K, T=T)


def _quadratic_peak(lams, rates) -> Tuple[float, float]:
    """(x, y) at the maximum of a least-squares quadratic through (lams, rates), x clipped
    to the scanned range; the best measured point when the fit is not concave; the
    middle of the range with rate 0 when nothing was measured."""
    x = np.asarray(lams, dtype=np.float64)
    y = np.asarray(rates, dtype=np.float64)
    if not np.any(y > 0):
        return float(np.median(x)), 0.0
    best = int(np.argmax(y))
    c2, c1, c0 = np.polyfit(x, y, 2)
    if c2 >= 0:
        return float(x[best]), float(y[best])
    xp = float(np.clip(-c1 / (2 * c2), x.min(), x.max()))
    return xp, float(np.polyval([c2, c1, c0], xp))


def target_lambda(rates: Sequence[float], lams: Sequence[float] = SCAN_LAMBDAS) -> float:
    """The level that maximises a least-squares quadratic through (lams, rates), clipped
    to the scanned range; the best scanned level when the fit is not concave."""
    return _quadratic_peak(lams, rates)[0]


def target_profile(rates, lams: Sequence[float] = SCAN_LAMBDAS,
                   slopes: Sequence[float] = SCAN_SLOPES) -> Tuple[float, float]:
    """(level, slope) of the target profile from rates[slope][level]: for each slope the
    quadratic peak over the levels; the slope whose fitted peak is highest wins (the
    first of equal peaks)."""
    rates = np.asarray(rates, dtype=np.float64).reshape(len(slopes), len(lams))
    peaks = [_quadratic_peak(lams, r) for r in rates]
    j = int(np.argmax([p[1] for p in peaks]))
    return peaks[j][0], float(slopes[j])


def deo_round_trip_rate(acc: np.ndarray, att: np.ndarray) -> float:
    """Round trips per exchange step predicted from swap rates for deterministic even/odd
    swaps, 1 / (2 + 2 sum_r rho_r/(1 - rho_r)) with rho_r the rejection rate of pair
    (r, r+1) (Syed, Bouchard-Cote, Deligiannidis & Doucet, JRSS B 84, 2022).  It assumes
    the rung index moves without memory, which the measured rate does not."""
    acc = np.asarray(acc, dtype=np.float64)
    att = np.asarray(att, dtype=np.float64)
    a = np.clip(acc / np.maximum(att, 1), 1e-9, 1.0)
    return float(1.0 / (2.0 + 2.0 * np.sum((1.0 - a) / a)))


def up_fraction(nup: np.ndarray, ndown: np.ndarray) -> np.ndarray:
    """f(r) = nup/(nup + ndown): the fraction of visits to rung r made by replicas whose
    last end was the coldest rung (Katzgraber, Trebst, Huse & Troyer, J. Stat. Mech.
    P03018, 2006); NaN where a rung had no labelled visit."""
    nup = np.asarray(nup, dtype=np.float64)
    tot = nup + np.asarray(ndown, dtype=np.float64)
    return np.where(tot > 0, nup / np.maximum(tot, 1), np.nan)


# ----------------------------------------------------------------------------- sampler runs

def run_batch(instances, seed: int, k: int, burn_cycles: int, cycles: int):
    """Run the sampler on a batch and return per-instance counts accumulated over the
    measurement cycles only (differences after burn-in)."""
    from . import ptqmc
    with ptqmc.Sampler(instances, seed, sweeps_per_exchange=k) as s:
        s.run(burn_cycles)
        before = [s.observables(n) for n in range(len(instances))]
        s.run(cycles)
        after = [s.observables(n) for n in range(len(instances))]
    out = []
    for a, b in zip(after, before):
        out.append(dict(
            nup=(a["nup"] - b["nup"]).astype(np.int64),
            ndown=(a["ndown"] - b["ndown"]).astype(np.int64),
            roundtrips=int((a["roundtrips"] - b["roundtrips"]).astype(np.int64).sum()),
            acc=(a["acc"] - b["acc"]).astype(np.int64),
            att=(a["att"] - b["att"]).astype(np.int64)))
    return out


def evaluate(instances, lams, seed: int, k: int, cycles: int, burn_cycles: int = 0):
    """Per instance: measured round trips per sweep, swap-rate-predicted round trips per
    exchange step and minimum pair acceptance, under per-instance mixing lams."""
    obs = run_batch([with_ladder(i, l) for i, l in zip(instances, lams)], seed, k,
                    burn_cycles, cycles)
    rt = np.array([o["roundtrips"] / (cycles * k) for o in obs])
    pred = np.array([deo_round_trip_rate(o["acc"], o["att"]) for o in obs])
    amin = np.array([float((o["acc"] / np.maximum(o["att"], 1)).min()) for o in obs])
    return rt, pred, amin


def scan(instances, seed: int, k: int, cycles: int, lams: Sequence[float] = SCAN_LAMBDAS,
         slope: float = 0.0):
    """Measured round trips per sweep of every instance under the profiles of each level
    in lams at one slope: array [len(instances)][len(lams)]."""
    out = np.zeros((len(instances), len(lams)))
    for c, lam in enumerate(lams):
        rt, _, _ = evaluate(instances, [profile(lam, slope, i.R) for i in instances], seed, k,
                            cycles)
        out[:, c] = rt
    return out


# ----------------------------------------------------------------------------- network

def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-np.asarray(z, dtype=np.float64)))


@dataclasses.dataclass
class LadderModel:
    params: np.ndarray      # flat FP32 network parameters
    mean: np.ndarray        # feature standardisation
    std: np.ndarray

    def standardise(self, feats: np.ndarray) -> np.ndarray:
        return ((np.asarray(feats, np.float32) - self.mean) / self.std).astype(np.float32)

    def logits(self, feats: np.ndarray) -> np.ndarray:
        from . import ptqmc
        net = ptqmc.LadderNet(self.params)
        return net.forward(self.standardise(feats)).cpu().numpy()

    def knots(self, instances) -> np.ndarray:
        """lambda at the 64 knots for every instance: array [n][64]."""
        return _sigmoid(self.logits(np.stack([features(i) for i in instances])))

    def rung_lambdas(self, instances) -> List[np.ndarray]:
        return [knots_to_rungs(kn, i.R) for kn, i in zip(self.knots(instances), instances)]

    def save(self, path: str):
        np.savez(path, params=self.params, mean=self.mean, std=self.std)

    @staticmethod
    def load(path: str) -> "LadderModel":
        with np.load(path, allow_pickle=False) as f:
            return LadderModel(f["params"].astype(np.float32), f["mean"].astype(np.float32),
                               f["std"].astype(np.float32))


def train(feats: np.ndarray, targets: np.ndarray, steps: int = 3000, batch: int = 256,
          lr: float = 1e-3, seed: int = 0, log=None) -> LadderModel:
    """Fit the network to per-knot targets in [0, 1] with the library's FP32 kernels
    (logistic cross entropy, Adam)."""
    from . import ptqmc
    feats = np.asarray(feats, np.float32)
    mean = feats.mean(axis=0)
    std = feats.std(axis=0)
    std = np.where(std > 1e-6 * np.maximum(np.abs(mean), 1.0), std, 1.0)
    X = ((feats - mean) / std).astype(np.float32)
    Q = np.asarray(targets, np.float32)
    q0 = float(np.clip(Q.mean(), 1e-3, 1 - 1e-3))
    net = ptqmc.LadderNet(ptqmc.init_ladder_params(seed, out_bias=math.log(q0 / (1 - q0))))
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    for step in range(steps):
        idx = rng.choice(n, size=min(batch, n), replace=False)
        loss = net.loss_grad(X[idx], Q[idx], ptqmc.MLP_LOSS_SIGMOID)
        net.adam(lr)
        if log and (step % 500 == 0 or step == steps - 1):
            log(f"step {step} loss {loss:.5f}")
    return LadderModel(net.numpy_params(), mean.astype(np.float32), std.astype(np.float32))
