"""The product's FP64 estimators (paper_1004_0023_amd.estimators) against closed forms,
exact transfer-matrix expectations, exact diagonalisation and the oracle's statement of
the same estimator; no GPU."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1004_0023_amd import annealing
from paper_1004_0023_amd import estimators as est
from test_oracle_pins import tfim_ed, transfer_matrix_exact


def _obs(R, n, sumE, sumC, sumE2=None, sumC2=None, t=1):
    z = np.zeros(R, np.int64)
    return dict(n_acc=n, sumE=np.asarray(sumE), sumC=np.asarray(sumC),
                sumE2=z if sumE2 is None else np.asarray(sumE2),
                sumC2=z if sumC2 is None else np.asarray(sumC2),
                acc=np.zeros(R - 1, np.uint64), att=np.ones(R - 1, np.uint64),
                roundtrips=np.zeros(R, np.uint64), nup=np.zeros(R, np.uint64),
                ndown=np.zeros(R, np.uint64), t=t)


def test_free_spin_no_trotter_error():
    """A lone spin at h = 0 has H_P = 0, so the estimator with the exact imaginary-time
    bond <s^k s^{k+1}> = (tanh K + tanh^{M-1} K)/(1 + tanh^M K) equals the quantum value
    -Gamma tanh(beta Gamma) at every M."""
    for M in (2, 4, 16, 128):
        for Gamma in (0.5, 1.0, 1.5):
            inst = W.make_instance(1, np.zeros((0, 2), np.int32), np.zeros(0, np.int8),
                                   np.zeros(1, np.int8), M, [0.3, 1.0, 2.5], Gamma)
            th = np.tanh(inst.K)
            corr = (th + th ** (M - 1)) / (1 + th ** M)
            obs = _obs(3, 1, [0, 0, 0], corr * M)
            e = est.instance_estimators(obs, inst)
            want = -Gamma * np.tanh(Gamma / np.asarray(inst.T))
            assert np.allclose(e["H"], want, rtol=0, atol=1e-12)
            assert np.allclose(e["sigma_x"], np.tanh(Gamma / np.asarray(inst.T)), atol=1e-12)


def test_exact_chain_expectations_converge_to_diagonalisation():
    """Fed the exact finite-M expectations of the 8-spin model of the first workload
    (transfer matrices), the estimator of <H> converges to exact diagonalisation as
    1/M^2 and is within 1e-2 relative at M = 256; <H_P> likewise approaches
    Tr(H_P e^{-beta H})/Z."""
    base = W.config1()
    T = 1.0
    H_ed, HP_ed = tfim_ed(base, 1.0 / T)
    errs = []
    for M in (16, 32, 64, 256):
        inst = W.make_instance(base.N, base.edges, base.J, base.h, M, [T], base.Gamma,
                               relabel=False)
        e_ex, c_ex = transfer_matrix_exact(inst, 0)
        obs = _obs(1, 1, [e_ex * M], [c_ex * M])
        e = est.instance_estimators(obs, inst)
        errs.append(abs(e["H"][0] - H_ed))
        if M == 256:
            assert abs(e["H_P"][0] - HP_ed) < 2e-2 * abs(HP_ed)
    assert errs[-1] < 1e-2 * abs(H_ed)
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0


def test_matches_oracle_statement_on_sampled_accumulators():
    """On accumulators of real oracle runs (quantum and classical instances) the product
    estimator equals the oracle's FP64 statement of it."""
    rng = np.random.default_rng([1004, 40])
    insts = [W.config1(),
             W.random_small_instance(rng, 10, 8, 5, d=3, jmax=2, hmax=1, name="q"),
             W.random_small_instance(rng, 9, 1, 4, d=2, jmax=1, hmax=1, name="classical")]
    for n, inst in enumerate(insts):
        o = oracle.OracleChain(inst, 77, index=n)
        o.run(2, 300)
        obs = o.observables()
        hp_o, H_o = oracle.energy_estimators(obs, inst)
        e = est.instance_estimators(obs, inst)
        assert np.allclose(e["H_P"], hp_o, rtol=1e-13, atol=1e-12)
        assert np.allclose(e["H"], H_o, rtol=1e-13, atol=1e-12)


def test_moments_rates_and_fractions():
    """Variances from the squared sums, swap rates acc/att, up fractions and the round-trip
    rate per sweep, on accumulators whose values are known."""
    M, R = 4, 3
    Es = np.array([[-8, 4, 0], [-4, 8, 4], [-12, 0, 8]], np.int64)  # samples x rungs
    Cs = np.array([[16, 0, 4], [12, 4, -4], [16, 8, 0]], np.int64)
    obs = _obs(R, 3, Es.sum(0), Cs.sum(0), (Es ** 2).sum(0), (Cs ** 2).sum(0), t=30)
    obs["acc"] = np.array([3, 1], np.uint64)
    obs["att"] = np.array([6, 4], np.uint64)
    obs["roundtrips"] = np.array([2, 0, 1], np.uint64)
    obs["nup"] = np.array([3, 1, 0], np.uint64)
    obs["ndown"] = np.array([0, 3, 0], np.uint64)
    e = est.rung_estimators(obs, N=2, M=M, b=[0.5, 0.25, 0.125], K=[0.3, 0.5, 0.8])
    assert np.allclose(e["E_mean"], Es.mean(0) / M)
    assert np.allclose(e["E_var"], Es.var(0) / M ** 2)
    assert np.allclose(e["C_mean"], Cs.mean(0) / M)
    assert np.allclose(e["C_var"], Cs.var(0) / M ** 2)
    assert np.allclose(e["swap_rate"], [0.5, 0.25])
    assert e["up_fraction"][0] == 1.0 and e["up_fraction"][1] == 0.25
    assert math.isnan(e["up_fraction"][2])
    assert e["roundtrip_rate"] == pytest.approx(3 / 30)
    with pytest.raises(ValueError):
        est.rung_estimators(dict(obs, n_acc=0), N=2, M=M, b=[0.5] * 3, K=[0.3] * 3)


def test_annealing_rung_scales_by_B():
    """A rung of H(s) = -A(s) sum sigma^x + B(s) H_P at inverse temperature beta is the
    temperature rung at T' = 1/(beta B), Gamma' = A/B: the estimator given beta returns
    B times the one given beta' = beta B (the same accumulators)."""
    beta, M = 20.0, 64
    s_vals = [0.3, 0.45, 0.6]
    b, K = annealing.annealing_rungs(s_vals, beta, M)
    rng = np.random.default_rng(3)
    obs = _obs(3, 5, rng.integers(-400, 0, 3), rng.integers(0, 300, 3))
    A = np.array([1 - s for s in s_vals])
    B = np.array(s_vals)
    e_s = est.rung_estimators(obs, 6, M, b, K, beta=[beta] * 3)
    e_t = est.rung_estimators(obs, 6, M, b, K, beta=beta * B)
    assert np.allclose(e_s["H"], B * e_t["H"], rtol=1e-12)
    # and the transverse magnetisation depends on K alone
    assert np.allclose(e_s["sigma_x"], e_t["sigma_x"], rtol=1e-12)
    assert np.allclose(e_s["H"], B * e_s["H_P"] - A * e_s["sigma_x"], rtol=1e-12)
