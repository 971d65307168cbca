"""The C ABI used from C alone: tests/native/abi_run.c links libptqmc directly (no Python,
no torch; library-owned workspace and stream), runs a PT job from an instance file and
prints its observables.  On the CPU it must compile and link against include/ptqmc.h; on
the GPU its output must equal the oracle's trajectory bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "abi_run.c")
LIBDIR = os.path.join(ROOT, "paper_1004_0023_amd", "_lib")


def build_driver(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libptqmc.so")):
        pytest.skip("library not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "abi_run")
    subprocess.check_call([cc, "-O2", "-std=c99", "-Wall", "-Wextra", "-Werror",
                           "-I", os.path.join(ROOT, "include"), SRC, "-L", LIBDIR, "-lptqmc",
                           f"-Wl,-rpath,{LIBDIR}", "-o", exe])
    return exe


def write_instance(inst, path):
    with open(path, "w") as f:
        f.write(f"{inst.N} {inst.M} {inst.R} {inst.n_edges} {inst.n_colors}\n")
        for (i, j), J in zip(inst.edges, inst.J):
            f.write(f"{int(i)} {int(j)} {int(J)}\n")
        f.write(" ".join(str(int(x)) for x in inst.h) + "\n")
        f.write(" ".join(str(int(x)) for x in inst.color) + "\n")
        f.write(" ".join(float(x).hex() for x in inst.b) + "\n")
        f.write(" ".join(float(x).hex() for x in inst.K) + "\n")


def test_driver_compiles_against_the_header(tmp_path):
    exe = build_driver(tmp_path)
    assert os.access(exe, os.X_OK)


@pytest.mark.gpu
@pytest.mark.parametrize("encoding,flags", [(0, 0), (1, 0), (0, 0x80)])
def test_c_driver_matches_oracle(tmp_path, encoding, flags):
    """Byte and bit-packed encodings, and the correlation accumulators (flag 0x80,
    PT_FLAG_TAU_CORR), all through the C ABI alone."""
    exe = build_driver(tmp_path)
    rng = np.random.default_rng([1004, 27])
    for n, inst in enumerate([W.config1(),
                              W.random_small_instance(rng, 13, 8, 5, d=4, jmax=3, hmax=2)]):
        seed, k, cycles = 0xC0FFEE + n, 3, 40
        path = str(tmp_path / f"inst{n}.txt")
        write_instance(inst, path)
        print(f"case: C driver, instance {n} (N={inst.N} M={inst.M} R={inst.R}), "
              f"encoding {encoding}, flags {flags:#x}", flush=True)
        out = subprocess.run([exe, path, str(seed), str(k), str(cycles), str(encoding),
                              str(flags)], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0, out.stderr
        got = {}
        for line in out.stdout.splitlines():
            key, *vals = line.split()
            got[key] = np.array([int(v) for v in vals], dtype=np.int64)
        ref = oracle.OracleChain(inst, seed, index=0)
        ref.run(k, cycles)
        want = ref.observables()
        for key in ("E_cl", "C", "rung_of", "replica_of", "acc", "att", "roundtrips", "label",
                    "sumE", "sumC", "sumE2", "sumC2", "nup", "ndown"):
            assert np.array_equal(got[key], np.asarray(want[key]).astype(np.int64)), key
        assert tuple(got["counters"]) == (want["t"], want["e"], want["n_acc"])
        assert np.array_equal(got["spins"], ref.s.reshape(-1).astype(np.int64))
        if flags & 0x80:
            assert np.array_equal(got["sumCt"], want["sumCt"].reshape(-1))
