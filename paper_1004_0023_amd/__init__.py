"""MI355X-native parallel-tempering quantum Monte Carlo sampler.

The hot path -- Metropolis sweeps of Suzuki-Trotter replicas and replica exchange --
lives in the HIP library ``_lib/libptqmc.so`` behind the C ABI of ``include/ptqmc.h``.
Import ``paper_1004_0023_amd.ptqmc`` for the binding (it imports torch, which provides
device memory and streams).
"""

__all__ = ["ptqmc", "build"]
