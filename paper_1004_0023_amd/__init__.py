"""MI355X-native parallel-tempering quantum Monte Carlo sampler.

The hot path -- Metropolis sweeps of Suzuki-Trotter replicas and replica exchange
(Karimi, Dickson & Hamze, arXiv:1004.0023, Sections 2, 5, 6) -- lives in the HIP library
``_lib/libptqmc.so`` behind the C ABI of ``include/ptqmc.h``; ``python -m
paper_1004_0023_amd.build`` compiles it for gfx950.

    import workloads as W
    from paper_1004_0023_amd import ptqmc
    insts = W.config3()                       # the 512-instance batch; any Instance list works
    with ptqmc.Sampler(insts, seed=1, sweeps_per_exchange=10) as s:
        s.run(1000)                           # 1000 x (10 sweeps + one exchange step)
        obs = s.observables(0)                # energies, permutation, swap and round-trip counts

Options: ``encoding=ptqmc.PT_BITPACK32`` keeps 32 replica slots per 32-bit word (the same
chain, 8x less device memory); ``flags=ptqmc.PT_FLAG_TAU_CORR`` accumulates imaginary-time
spin correlations per rung (``observables(n)["sumCt"]``).

``ptqmc`` is the binding (argument marshalling only; torch provides device memory and
streams).  ``ladder`` proposes per-instance ladders with the trained network
(``data/ladder_mlp.npz``) and ``train_ladder`` regenerates its training data, weights
and evaluation on the GPU.  ``annealing`` builds ladders over the parameter s of an
adiabatic evolution H(s) = -A(s) sum sigma^x + B(s) H_P and estimates the gap per rung
from the correlations:

    from paper_1004_0023_amd import annealing
    inst = annealing.with_annealing_ladder(base, s_values, beta)   # rung 0 = s_values[0]
    with ptqmc.Sampler([inst], seed=1, sweeps_per_exchange=10,
                       flags=ptqmc.PT_FLAG_TAU_CORR) as s:
        s.run(100_000)
        taus, G = annealing.correlation_curve(s.observables(0), inst.N, inst.M, beta)
    gap0 = annealing.fit_gap(taus[1:], G[0, 1:], beta)
"""

__all__ = ["ptqmc", "build", "ladder", "train_ladder", "annealing"]
