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

``ptqmc`` is the binding (argument marshalling only; torch provides device memory and
streams).  ``ladder`` proposes per-instance ladders with the trained network
(``data/ladder_mlp.npz``) and ``train_ladder`` regenerates its training data, weights
and evaluation on the GPU.
"""

__all__ = ["ptqmc", "build", "ladder", "train_ladder"]
