"""Ladder helpers (CPU): the Trotter-coupling ladder family, targets from scans, the
swap-rate prediction, features and the stored model/scan files."""
import math
import os

import numpy as np
import pytest

import workloads as W
from paper_1004_0023_amd import ladder as L

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(os.path.dirname(HERE), "paper_1004_0023_amd", "data")


@pytest.fixture(scope="module")
def inst():
    return W.config3_instance(7, config=5)


def test_lambda_zero_is_geometric(inst):
    T, b, K = L.coupling_ladder(inst, 0.0)
    Tg = L.geometric(float(inst.T[0]), float(inst.T[-1]), inst.R)
    bg, Kg = L.st_rungs(Tg, inst.Gamma, inst.M)
    assert np.array_equal(T, Tg) and np.array_equal(b, bg) and np.allclose(K, Kg, rtol=0, atol=0)


@pytest.mark.parametrize("lam", [0.2, 0.5, 1.0])
def test_coupling_family_keeps_rung0_and_interpolates(inst, lam):
    _, b, K = L.coupling_ladder(inst, lam)
    _, bg, Kg = L.coupling_ladder(inst, 0.0)
    assert np.array_equal(b, bg)                     # temperatures never move
    assert K[0] == Kg[0]                             # the target rung is untouched
    assert np.all(K >= Kg[0] - 1e-15) and np.all(K <= Kg + 1e-15)
    # log K is the lam-weighted mean of log K_geo and log K_0
    assert np.allclose(np.log(K), (1 - lam) * np.log(Kg) + lam * np.log(Kg[0]), atol=1e-12)
    if lam == 1.0:
        assert np.allclose(K, Kg[0])                 # Gamma_r proportional to T_r


def test_coupling_family_classical_case():
    i = W.random_small_instance(np.random.default_rng(3), N=16, M=1, R=4)
    _, _, K = L.coupling_ladder(i, 0.4)
    assert np.all(K == 0)


def test_knots_to_rungs():
    kn = np.linspace(0.0, 1.0, L.N_KNOTS)
    for R in (2, 16, 64, 100):
        lam = L.knots_to_rungs(kn, R)
        assert lam.shape == (R,)
        assert np.allclose(lam, np.arange(R) / (R - 1))
    assert np.allclose(L.knots_to_rungs(np.full(L.N_KNOTS, 0.3), 17), 0.3)


def test_target_lambda():
    lams = np.array(L.SCAN_LAMBDAS)
    # exact concave quadratic: the peak is recovered
    assert abs(L.target_lambda(-(lams - 0.33) ** 2 + 1.0) - 0.33) < 1e-9
    # a peak outside the range is clipped
    assert L.target_lambda(lams) == pytest.approx(lams.max())
    # a convex fit falls back to the best measured candidate
    assert L.target_lambda([3.0, 1.0, 0.5, 1.0, 2.0]) == lams[0]
    # no round trips at all: the middle of the scan
    assert L.target_lambda([0, 0, 0, 0, 0]) == float(np.median(lams))


def test_deo_round_trip_rate_closed_forms():
    # every swap accepted: 1/2 round trip per exchange step
    assert L.deo_round_trip_rate(np.full(7, 10), np.full(7, 10)) == pytest.approx(0.5)
    # R-1 pairs with acceptance a: 1/(2 + 2 (R-1)(1-a)/a)
    a, n = 0.25, 9
    want = 1.0 / (2 + 2 * n * (1 - a) / a)
    assert L.deo_round_trip_rate(np.full(n, 25), np.full(n, 100)) == pytest.approx(want)


def test_up_fraction():
    f = L.up_fraction([5, 3, 0, 0], [0, 1, 4, 0])
    assert f[0] == 1 and f[1] == 0.75 and f[2] == 0 and np.isnan(f[3])


def test_features_shape_and_determinism(inst):
    f = L.features(inst)
    assert f.shape == (L.N_FEATURES,) and f.dtype == np.float32
    assert np.all(np.isfinite(f))
    assert np.array_equal(f, L.features(W.config3_instance(7, config=5)))
    # the Trotter couplings at both ends
    _, Kg = L.st_rungs([inst.T[0], inst.T[-1]], inst.Gamma, inst.M)
    assert f[28] == pytest.approx(Kg[0]) and f[29] == pytest.approx(Kg[1])


def test_model_save_load(tmp_path):
    rng = np.random.default_rng(0)
    m = L.LadderModel(rng.random(28992).astype(np.float32), rng.random(32).astype(np.float32),
                      rng.random(32).astype(np.float32) + 0.5)
    p = str(tmp_path / "m.npz")
    m.save(p)
    m2 = L.LadderModel.load(p)
    for a, b in ((m.params, m2.params), (m.mean, m2.mean), (m.std, m2.std)):
        assert np.array_equal(a, b)


def test_profile():
    # the knots of a linear profile, clipped to [0, 1]
    assert np.allclose(L.profile(0.3, 0.25, 5), [0.175, 0.2375, 0.3, 0.3625, 0.425])
    assert np.array_equal(L.profile(0.9, 0.5, 3), [0.65, 0.9, 1.0])
    assert np.array_equal(L.profile(0.05, 0.4, 3), [0.0, 0.05, 0.25])
    # slope 0 is the constant ladder bit for bit, so the slope-0 scan is the constant scan
    i = W.config3_instance(3, config=5)
    assert np.array_equal(L.coupling_ladder(i, L.profile(0.3, 0.0, i.R))[2],
                          L.coupling_ladder(i, 0.3)[2])
    # the profile at the knots interpolates to the profile at the rungs
    for R in (16, 33, 64):
        assert np.allclose(L.knots_to_rungs(L.profile(0.3, 0.25, L.N_KNOTS), R),
                           L.profile(0.3, 0.25, R), atol=1e-12)


def test_target_profile():
    lams = np.array(L.SCAN_LAMBDAS)
    flat = -(lams - 0.33) ** 2 + 1.0
    # the slope whose fitted peak is higher wins, at its own best level
    a, s = L.target_profile([flat, -(lams - 0.21) ** 2 + 1.5])
    assert abs(a - 0.21) < 1e-9 and s == L.SCAN_SLOPES[1]
    a, s = L.target_profile([flat, -(lams - 0.21) ** 2 + 0.5])
    assert abs(a - 0.33) < 1e-9 and s == L.SCAN_SLOPES[0]
    # the fitted peak, not the best measured point, decides
    a, s = L.target_profile([[1.0, 2.0, 2.9, 3.0, 1.0], [1.0, 2.9, 2.95, 2.9, 1.0]])
    assert s == L.SCAN_SLOPES[1]
    # equal peaks: the first slope
    assert L.target_profile([flat, flat])[1] == L.SCAN_SLOPES[0]


def test_stored_scan_and_model_files():
    with np.load(os.path.join(DATA, "ladder_scan.npz"), allow_pickle=False) as f:
        assert tuple(f["lams"]) == tuple(L.SCAN_LAMBDAS)
        assert tuple(f["slopes"]) == tuple(L.SCAN_SLOPES)
        rates = f["rates"]
        assert rates.shape == (4096, len(L.SCAN_SLOPES), len(L.SCAN_LAMBDAS))
        assert np.all(np.isfinite(rates)) and np.all(rates >= 0)
    path = os.path.join(DATA, "ladder_mlp.npz")
    if not os.path.exists(path):
        pytest.skip("no trained model stored")
    m = L.LadderModel.load(path)
    assert m.params.shape == (28992,) and m.mean.shape == (32,) and np.all(m.std > 0)
    # the network's lambda at the knots, evaluated on the CPU with the FP64 statement
    from oracle import mlp
    x = m.standardise(np.stack([L.features(W.config3_instance(4096 + n, config=5))
                                for n in range(8)]))
    z, _ = mlp.forward(m.params.astype(np.float64), x.astype(np.float64))
    lam = 1 / (1 + np.exp(-z))
    assert np.all((lam > 0.05) & (lam < 0.8))
