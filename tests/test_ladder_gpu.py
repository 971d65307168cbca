"""The trained ladder network against the geometric ladder on held-out instances, at
equal sweeps (GPU).  Both runs use the same instances, seeds and sweep count; the only
difference is the (b_r, K_r) data the network proposes, so the round-trip gain is what
the network adds over the plain method."""
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL = os.path.join(os.path.dirname(HERE), "paper_1004_0023_amd", "data", "ladder_mlp.npz")
N_TRAIN = 4096   # training instances are 0 .. 4095; held-out instances follow


@pytest.fixture(scope="module")
def ptq():
    import torch
    from paper_1004_0023_amd import ptqmc
    torch.cuda.set_device(0)
    ptqmc.lib()
    return ptqmc


@pytest.mark.gpu
def test_learned_ladder_beats_geometric_and_best_constant_on_heldout(ptq):
    """64 held-out instances, 10^5 sweeps each, the same seeds for every ladder: the
    learned ladder gives at least 1.5x the geometric ladder's round trips (better on three
    instances for every one worse), and at least the round trips of the best constant
    coupling mix of the training scan (lambda = 0.3, the same for every instance and
    rung) -- the part of the gain that the network's per-instance choice adds on top of
    the ladder family.  The chain is deterministic for a seed, so the counts are too."""
    from paper_1004_0023_amd import ladder as L
    if not os.path.exists(MODEL):
        pytest.skip("no trained model stored")
    n, k, cycles = 64, 10, 10_000
    best_const = 0.3  # best constant of the training scan (data/ladder_eval.json)
    held = [W.config3_instance(N_TRAIN + 128 + j, config=5) for j in range(n)]
    print(f"case: learned vs geometric vs constant ladder, {n} held-out instances, "
          f"{k * cycles} sweeps", flush=True)
    model = L.LadderModel.load(MODEL)
    lam = model.rung_lambdas(held)
    for x, i in zip(lam, held):
        assert x.shape == (i.R,) and np.all((x >= 0) & (x <= 1))
    seed = 0x1ADDE5
    rt_geo, _, _ = L.evaluate(held, [0.0] * n, seed, k, cycles)
    rt_cst, _, _ = L.evaluate(held, [best_const] * n, seed, k, cycles)
    rt_lrn, _, _ = L.evaluate(held, lam, seed, k, cycles)
    d = rt_lrn - rt_geo
    print(f"round trips per sweep: geometric {rt_geo.mean():.3e}, constant {rt_cst.mean():.3e}, "
          f"learned {rt_lrn.mean():.3e}; learned better than geometric on {(d > 0).sum()}, "
          f"worse on {(d < 0).sum()} of {n}; better than constant on "
          f"{(rt_lrn > rt_cst).sum()}, worse on {(rt_lrn < rt_cst).sum()}", flush=True)
    assert rt_lrn.sum() >= 1.5 * rt_geo.sum()
    assert (d > 0).sum() >= 3 * (d < 0).sum()
    assert rt_lrn.sum() >= rt_cst.sum()


@pytest.mark.gpu
def test_learned_ladder_keeps_target_rung(ptq):
    """Rung 0 gets the geometric ladder's (b_0, K_0) bit for bit, so the coldest rung
    samples the same ensemble with or without the network."""
    from paper_1004_0023_amd import ladder as L
    if not os.path.exists(MODEL):
        pytest.skip("no trained model stored")
    held = [W.config3_instance(N_TRAIN + j, config=5) for j in range(16)]
    model = L.LadderModel.load(MODEL)
    for i, lam in zip(held, model.rung_lambdas(held)):
        _, b, K = L.coupling_ladder(i, lam)
        _, bg, Kg = L.coupling_ladder(i, 0.0)
        assert b[0] == bg[0] and K[0] == Kg[0]
