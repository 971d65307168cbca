"""The product's estimators on accumulators the GPU sampler produced: <H> of the 8-spin
transverse-field model of the first workload at M = 64 against exact diagonalisation,
within the Trotter error (known exactly from transfer matrices) plus sampling error."""
import sys

import numpy as np
import pytest

import workloads as W
from paper_1004_0023_amd import estimators as est
from test_oracle_pins import tfim_ed, transfer_matrix_exact

pytestmark = pytest.mark.gpu


def test_gpu_estimator_near_exact_diagonalisation():
    import torch
    from paper_1004_0023_amd import ptqmc
    torch.cuda.set_device(0)
    base = W.config1()
    M, T = 64, 1.0
    inst = W.make_instance(base.N, base.edges, base.J, base.h, M, [0.9, 1.0, 1.1],
                           base.Gamma, relabel=False)
    copies, burn, cycles = 16, 2000, 20000
    print(f"case: estimators, {copies} copies of the 8-spin model at M={M}, "
          f"{burn}+{cycles} cycles", flush=True)
    sys.stdout.flush()
    with ptqmc.Sampler([inst] * copies, 0xE57, sweeps_per_exchange=2, block_threads=256) as s:
        s.run(burn)
        first = [s.observables(n) for n in range(copies)]
        s.run(cycles)
        last = [s.observables(n) for n in range(copies)]
    Hs = []
    for a, b in zip(first, last):
        d = {k: (np.asarray(b[k]) - np.asarray(a[k])) if isinstance(b[k], np.ndarray)
             else b[k] - a[k] for k in b}
        e = est.instance_estimators(d, inst)
        assert e["samples"] == cycles
        Hs.append(e["H"][1])  # the rung at T = 1
    Hs = np.asarray(Hs)
    mean, se = Hs.mean(), Hs.std(ddof=1) / np.sqrt(copies)
    H_ed, _ = tfim_ed(base, 1.0 / T)
    e_ex, c_ex = transfer_matrix_exact(inst, 1)
    exact = est.rung_estimators(dict(n_acc=1, sumE=np.array([e_ex * M]),
                                     sumC=np.array([c_ex * M]), sumE2=np.zeros(1),
                                     sumC2=np.zeros(1), acc=np.zeros(0), att=np.zeros(0),
                                     roundtrips=np.zeros(1), nup=np.zeros(1),
                                     ndown=np.zeros(1), t=1),
                                N=inst.N, M=M, b=[inst.b[1]], K=[inst.K[1]], beta=[1.0 / T])
    H_tm = exact["H"][0]
    print(f"<H>: sampled {mean:.5f} +- {se:.5f}, finite-M exact {H_tm:.5f}, ED {H_ed:.5f}",
          flush=True)
    assert abs(mean - H_tm) < 5 * se
    assert abs(mean - H_ed) < 5 * se + abs(H_tm - H_ed) + 1e-3 * abs(H_ed)
