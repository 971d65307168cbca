"""Python access to the plain-C CPU oracle (``ptoracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is imported by the test-suite, by the smoke check
and by the CPU-baseline leg of the benchmark, never by the product library.  It is an
independent, slow, obviously-correct statement of what the sampler computes: Philox
draws, the deterministic exponential, Metropolis single-spin sweeps in colour-class
order, even/odd replica exchange, round-trip labels and per-rung accumulators
(including the imaginary-time spin correlations at TAU_LAGS Trotter lags).

The oracle handles one instance at a time; the instance number ``index`` enters every
random counter, so instance n of a batch is reproduced by passing ``index = n``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ptoracle.c")
TAU_LAGS = 8  # imaginary-time correlation lags per rung (OR_TAU_LAGS)
_LIB = os.path.join(_HERE, "libptoracle.so")

LABEL_NONE, LABEL_UP, LABEL_DOWN = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Inst(C.Structure):
    _fields_ = [("index", C.c_int32), ("N", C.c_int32), ("M", C.c_int32), ("R", C.c_int32),
                ("n_edges", C.c_int32), ("n_colors", C.c_int32),
                ("edge_i", C.c_void_p), ("edge_j", C.c_void_p), ("edge_J", C.c_void_p),
                ("h", C.c_void_p), ("color", C.c_void_p), ("b", C.c_void_p), ("K", C.c_void_p)]


class _State(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("s", "rung_of", "replica_of", "E", "C", "label", "rt",
                                          "acc", "att", "sumE", "sumC", "sumE2", "sumC2",
                                          "nup", "ndown", "counters", "sumCt")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.or_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_exp_det.argtypes = [C.c_double]
        L.or_exp_det.restype = C.c_double
        L.or_metropolis_threshold.argtypes = [C.c_double]
        L.or_metropolis_threshold.restype = C.c_uint32
        L.or_flip_word.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                   C.c_int32, C.c_int32]
        L.or_flip_word.restype = C.c_uint32
        L.or_swap_word.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_uint64]
        L.or_swap_word.restype = C.c_uint32
        L.or_init_spin.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_int32]
        L.or_init_spin.restype = C.c_int8
        L.or_energies.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_init.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64]
        L.or_sweep.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32]
        L.or_sweep.restype = C.c_int
        L.or_sweep_ordered.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_uint64]
        L.or_sweep_ordered.restype = C.c_int
        L.or_exchange.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64]
        L.or_run.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32]
        L.or_run.restype = C.c_int
        L.or_tau_lag.argtypes = [C.c_int32, C.c_int32]
        L.or_tau_lag.restype = C.c_int32
        L.or_tau_corr.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def tau_lag(M: int, l: int) -> int:
    """Lag l of the imaginary-time correlations, in slices (or_tau_lag)."""
    return int(lib().or_tau_lag(int(M), int(l)))


def exp_det(x: float) -> float:
    return lib().or_exp_det(float(x))


def metropolis_threshold(dS: float) -> int:
    return int(lib().or_metropolis_threshold(float(dS)))


def flip_word(seed, n, M, c, t, k, i) -> int:
    """Word of the flip attempt at (instance n, slot c, sweep t, slice k, site i)."""
    return int(lib().or_flip_word(seed, n, M, c, t, k, i))


def swap_word(seed, n, r, e) -> int:
    return int(lib().or_swap_word(seed, n, r, e))


def init_spin(seed, n, M, c, k, i) -> int:
    return int(lib().or_init_spin(seed, n, M, c, k, i))


class OracleChain:
    """Oracle state of one instance: spins [R][M][N] by replica slot plus the
    permutation, counters, labels, swap statistics and per-rung accumulators."""

    ARRAYS = ("s", "rung_of", "replica_of", "E", "C", "label", "rt", "acc", "att",
              "sumE", "sumC", "sumE2", "sumC2", "nup", "ndown", "counters", "sumCt")

    def __init__(self, inst, seed: int, index: int = 0, init: bool = True):
        self.inst = inst
        self.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        self.index = int(index)
        N, M, R = inst.N, inst.M, inst.R
        self._keep = dict(
            ei=np.ascontiguousarray(inst.edges[:, 0], dtype=np.int32) if inst.n_edges else np.zeros(1, np.int32),
            ej=np.ascontiguousarray(inst.edges[:, 1], dtype=np.int32) if inst.n_edges else np.zeros(1, np.int32),
            J=np.ascontiguousarray(inst.J, dtype=np.int8) if inst.n_edges else np.zeros(1, np.int8),
            h=np.ascontiguousarray(inst.h, dtype=np.int8),
            color=np.ascontiguousarray(inst.color, dtype=np.uint8),
            b=np.ascontiguousarray(inst.b, dtype=np.float64),
            K=np.ascontiguousarray(inst.K, dtype=np.float64))
        k = self._keep
        self._inst = _Inst(self.index, N, M, R, inst.n_edges, inst.n_colors, _p(k["ei"]),
                           _p(k["ej"]), _p(k["J"]), _p(k["h"]), _p(k["color"]), _p(k["b"]),
                           _p(k["K"]))
        self.s = np.zeros((R, M, N), dtype=np.int8)
        self.rung_of = np.zeros(R, dtype=np.int32)
        self.replica_of = np.zeros(R, dtype=np.int32)
        self.E = np.zeros(R, dtype=np.int64)
        self.C = np.zeros(R, dtype=np.int64)
        self.label = np.zeros(R, dtype=np.int8)
        self.rt = np.zeros(R, dtype=np.uint64)
        self.acc = np.zeros(max(R - 1, 1), dtype=np.uint64)
        self.att = np.zeros(max(R - 1, 1), dtype=np.uint64)
        self.sumE = np.zeros(R, dtype=np.int64)
        self.sumC = np.zeros(R, dtype=np.int64)
        self.sumE2 = np.zeros(R, dtype=np.int64)
        self.sumC2 = np.zeros(R, dtype=np.int64)
        self.nup = np.zeros(R, dtype=np.uint64)
        self.ndown = np.zeros(R, dtype=np.uint64)
        self.counters = np.zeros(3, dtype=np.uint64)
        self.sumCt = np.zeros((R, TAU_LAGS), dtype=np.int64)
        self._bind()
        if init:
            lib().or_init(C.byref(self._inst), C.byref(self._state), self.seed)

    def _bind(self):
        self._state = _State(*[_p(getattr(self, n)) for n in self.ARRAYS])

    # --- dynamics
    def sweep(self, n: int = 1, shuffle_seed: int = 0):
        if shuffle_seed:
            rc = lib().or_sweep_ordered(C.byref(self._inst), C.byref(self._state), self.seed,
                                        int(n), int(shuffle_seed))
        else:
            rc = lib().or_sweep(C.byref(self._inst), C.byref(self._state), self.seed, int(n))
        if rc:
            raise MemoryError("oracle sweep failed")

    def exchange(self):
        lib().or_exchange(C.byref(self._inst), C.byref(self._state), self.seed)

    def run(self, k: int, n_cycles: int):
        if lib().or_run(C.byref(self._inst), C.byref(self._state), self.seed, int(k),
                        int(n_cycles)):
            raise MemoryError("oracle run failed")

    def energies(self, spins: np.ndarray = None):
        s = self.s if spins is None else np.ascontiguousarray(spins, dtype=np.int8)
        E = np.zeros(self.inst.R, dtype=np.int64)
        Cc = np.zeros(self.inst.R, dtype=np.int64)
        lib().or_energies(C.byref(self._inst), _p(s), _p(E), _p(Cc))
        return E, Cc

    # --- state access
    @property
    def t(self) -> int:
        return int(self.counters[0])

    @property
    def e(self) -> int:
        return int(self.counters[1])

    @property
    def n_acc(self) -> int:
        return int(self.counters[2])

    def snapshot(self) -> Dict[str, np.ndarray]:
        return {n: getattr(self, n).copy() for n in self.ARRAYS}

    def restore(self, snap: Dict[str, np.ndarray]):
        for n in self.ARRAYS:
            getattr(self, n)[...] = snap[n]

    def observables(self) -> Dict[str, np.ndarray]:
        R = self.inst.R
        return dict(E_cl=self.E.copy(), C=self.C.copy(), rung_of=self.rung_of.copy(),
                    replica_of=self.replica_of.copy(), acc=self.acc[:R - 1].copy(),
                    att=self.att[:R - 1].copy(), roundtrips=self.rt.copy(),
                    label=self.label.copy(), sumE=self.sumE.copy(), sumC=self.sumC.copy(),
                    sumE2=self.sumE2.copy(), sumC2=self.sumC2.copy(), nup=self.nup.copy(),
                    ndown=self.ndown.copy(), sumCt=self.sumCt.copy(), t=self.t, e=self.e,
                    n_acc=self.n_acc)

    def tau_corr(self, spins: np.ndarray = None) -> np.ndarray:
        """Ct_l of every replica slot [R][TAU_LAGS] (or_tau_corr)."""
        s = self.s if spins is None else np.ascontiguousarray(spins, dtype=np.int8)
        out = np.zeros((self.inst.R, TAU_LAGS), dtype=np.int64)
        per = self.inst.M * self.inst.N
        for c in range(self.inst.R):
            lib().or_tau_corr(C.byref(self._inst), _p(s.reshape(-1)[c * per:]), _p(out[c]))
        return out


def energy_estimators(obs, inst):
    """Host FP64 estimators per rung from the accumulators (Suzuki-Trotter
    thermodynamic estimator, x = beta*Gamma/M):
        <H_P> = sumE/(n*M)
        <H>   = sumE/(n*M) - N*Gamma*coth(2x) + (Gamma/M) * (sumC/n) / sinh(2x)."""
    n = obs["n_acc"]
    M = inst.M
    beta = 1.0 / np.asarray(inst.T, dtype=np.float64)
    hp = obs["sumE"].astype(np.float64) / (n * M)
    if M == 1:
        return hp, hp.copy()
    x = beta * inst.Gamma / M
    cbar = obs["sumC"].astype(np.float64) / n
    H = hp - inst.N * inst.Gamma / np.tanh(2 * x) + (inst.Gamma / M) * cbar / np.sinh(2 * x)
    return hp, H
