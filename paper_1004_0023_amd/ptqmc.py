"""ctypes binding of libptqmc (include/ptqmc.h): argument marshalling only.

Every step of the sampler runs in the HIP library; PyTorch supplies the device
workspace and the stream.  The binding fails loudly when the library is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np
import torch  # loaded before libptqmc so both share torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libptqmc.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EHIP, PT_ELAUNCH, PT_ESTATE = 0, -1, -2, -3, -4, -5
PT_INT8, PT_BITPACK32 = 0, 1
PT_FLAG_TIMING, PT_FLAG_NO_GRAPH, PT_FLAG_INJECT_LAUNCH_OOR_ONCE = 0x1, 0x2, 0x4
PT_FLAG_FOUR_SLICE_LANES = 0x10
PT_FLAG_BLOCK_LAUNCH_PER_SWEEP = 0x20
PT_FLAG_TEST_BLOCK_WAIT_TIMEOUT = 0x40
PT_FLAG_TAU_CORR = 0x80
PT_FLAG_WORK_QUEUE = 0x100
PT_FLAG_TWO_WORD_LANES = 0x200
PT_FLAG_NO_LATENCY_PATH = 0x400
PT_FLAG_DEVICE_SCOPE_RECORDS = 0x800
PT_FLAG_TEST_XCD_MISMATCH = 0x1000
TAU_LAGS = 8  # PT_TAU_LAGS
PT_FLAG_SLICE_BLOCKS = 0x8
LABEL_NONE, LABEL_UP, LABEL_DOWN = 0, 1, 2
MLP_LOSS_SOFTMAX, MLP_LOSS_SIGMOID = 0, 1

EXPORTS = ["pt_workspace_bytes", "pt_init", "pt_sweep", "pt_exchange", "pt_run", "pt_sync",
           "pt_observables", "pt_get_spins", "pt_set_spins", "pt_save", "pt_load",
           "pt_checkpoint_validate", "pt_get_info", "pt_timing_reset", "pt_timing_enable",
           "pt_free",
           "pt_strerror", "pt_last_error",
           "pt_threshold", "pt_threshold_device", "pt_mlp_param_count",
           "pt_mlp_workspace_bytes", "pt_mlp_forward", "pt_mlp_forward_static",
           "pt_mlp_loss_grad", "pt_mlp_adam"]
MLP_STATIC_MAX_BATCH = 4096  # PT_MLP_STATIC_MAX_BATCH


class PTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class _Instance(C.Structure):
    _fields_ = [("N", C.c_int32), ("M", C.c_int32), ("R", C.c_int32), ("n_edges", C.c_int32),
                ("n_colors", C.c_int32), ("edge_i", C.c_void_p), ("edge_j", C.c_void_p),
                ("edge_J", C.c_void_p), ("h", C.c_void_p), ("color", C.c_void_p),
                ("rung_b", C.c_void_p), ("rung_K", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("sweeps_per_exchange", C.c_int32),
                ("encoding", C.c_int32), ("flags", C.c_uint32), ("tile_replicas", C.c_int32),
                ("tile_bytes", C.c_int32), ("block_threads", C.c_int32)]


class _Obs(C.Structure):
    _fields_ = [("E_cl", C.c_void_p), ("C", C.c_void_p), ("rung_of", C.c_void_p),
                ("replica_of", C.c_void_p), ("acc", C.c_void_p), ("att", C.c_void_p),
                ("roundtrips", C.c_void_p), ("label", C.c_void_p), ("sumE", C.c_void_p),
                ("sumC", C.c_void_p), ("sumE2", C.c_void_p), ("sumC2", C.c_void_p),
                ("nup", C.c_void_p), ("ndown", C.c_void_p),
                ("t", C.c_uint64), ("e", C.c_uint64), ("n_acc", C.c_uint64),
                ("sumCt", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("n_tiles", C.c_int32), ("block_threads", C.c_int32),
                ("lds_bytes", C.c_int32), ("max_tile_replicas", C.c_int32),
                ("fallbacks", C.c_int32), ("encoding", C.c_int32), ("device_cus", C.c_int32),
                ("tile_bytes", C.c_int32), ("tuned", C.c_int32),
                ("flips_per_sweep", C.c_uint64), ("sweep_ms", C.c_double),
                ("sweep_launches", C.c_int64), ("exchange_ms", C.c_double),
                ("exchange_launches", C.c_int64), ("sweep_groups", C.c_int32),
                ("block_tiles", C.c_int32), ("block_resident", C.c_int32),
                ("class_launches", C.c_int32), ("multi_launches", C.c_int64),
                ("multi_cycles", C.c_int64), ("multi_ms", C.c_double),
                ("oct_tiles", C.c_int32), ("oct_blocks", C.c_int32),
                ("oct_tile_launches", C.c_int32), ("oct_resident", C.c_int32),
                ("oct_queue", C.c_int32), ("oct_fused", C.c_int32), ("oct_ring_xcd", C.c_int32),
                ("block_ring_xcd", C.c_int32),
                ("recoveries", C.c_int64),
                ("lane_words", C.c_int32), ("ent16_instances", C.c_int32),
                ("last_device_error", C.c_uint32), ("latency_path", C.c_int32)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def lib():
    """Load libptqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_1004_0023_amd.build`)")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        L.pt_workspace_bytes.argtypes = [vp, i32, vp, C.POINTER(C.c_size_t)]
        L.pt_init.argtypes = [C.POINTER(vp), vp, i32, vp, vp, vp, C.c_size_t]
        L.pt_sweep.argtypes = [vp, i32]
        L.pt_exchange.argtypes = [vp]
        L.pt_run.argtypes = [vp, i32]
        L.pt_sync.argtypes = [vp]
        L.pt_observables.argtypes = [vp, i32, vp]
        L.pt_get_spins.argtypes = [vp, i32, vp]
        L.pt_set_spins.argtypes = [vp, i32, vp]
        L.pt_save.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.pt_load.argtypes = [vp, vp, C.c_size_t]
        L.pt_checkpoint_validate.argtypes = [vp, i32, vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.pt_get_info.argtypes = [vp, vp]
        L.pt_timing_reset.argtypes = [vp]
        L.pt_timing_enable.argtypes = [vp, i32]
        L.pt_free.argtypes = [vp]
        L.pt_free.restype = None
        L.pt_strerror.argtypes = [C.c_int]
        L.pt_strerror.restype = C.c_char_p
        L.pt_last_error.argtypes = []
        L.pt_last_error.restype = C.c_char_p
        L.pt_threshold.argtypes = [C.c_double]
        L.pt_threshold.restype = C.c_uint32
        L.pt_threshold_device.argtypes = [vp, vp, i32, vp]
        L.pt_mlp_param_count.argtypes = []
        L.pt_mlp_workspace_bytes.argtypes = [i32]
        L.pt_mlp_workspace_bytes.restype = C.c_size_t
        L.pt_mlp_forward.argtypes = [vp, vp, vp, i32, vp, vp]
        L.pt_mlp_forward_static.argtypes = [vp, vp, vp, i32, vp]
        L.pt_mlp_loss_grad.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
        L.pt_mlp_adam.argtypes = [vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float,
                                  C.c_float, i32, vp]
        for name in EXPORTS:
            if name not in ("pt_free", "pt_strerror", "pt_last_error", "pt_threshold",
                            "pt_mlp_workspace_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PT_OK:
        msg = lib().pt_last_error().decode(errors="replace")
        raise PTError(rc, f"{lib().pt_strerror(rc).decode()}: {msg}")


def threshold(dS: float) -> int:
    """Host-side acceptance threshold used to build the library's tables."""
    return int(lib().pt_threshold(float(dS)))


def threshold_device(dS: Sequence[float]) -> np.ndarray:
    """The same rule evaluated by the library's device code (swap decisions)."""
    x = torch.as_tensor(np.asarray(dS, dtype=np.float64), device="cuda")
    out = torch.empty(x.numel(), dtype=torch.int32, device="cuda")  # holds uint32 words
    stream = torch.cuda.current_stream().cuda_stream
    _check(lib().pt_threshold_device(x.data_ptr(), out.data_ptr(), x.numel(), stream))
    return out.cpu().numpy().view(np.uint32).copy()


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _records(instances: Sequence):
    """pt_instance records of the instances, and the arrays they point into (which must
    be kept alive while the records are used)."""
    keep: List[np.ndarray] = []
    recs = (_Instance * len(instances))()
    for n, inst in enumerate(instances):
        E = int(inst.edges.shape[0])
        ei = _arr(inst.edges[:, 0] if E else np.zeros(1), np.int32)
        ej = _arr(inst.edges[:, 1] if E else np.zeros(1), np.int32)
        J = _arr(inst.J if E else np.zeros(1), np.int8)
        h = _arr(inst.h, np.int8)
        col = _arr(inst.color, np.uint8)
        b = _arr(inst.b, np.float64)
        K = _arr(inst.K, np.float64)
        keep += [ei, ej, J, h, col, b, K]
        recs[n] = _Instance(inst.N, inst.M, inst.R, E, inst.n_colors, ei.ctypes.data,
                            ej.ctypes.data, J.ctypes.data, h.ctypes.data, col.ctypes.data,
                            b.ctypes.data, K.ctypes.data)
    return recs, keep


def _options(seed, sweeps_per_exchange=1, encoding=PT_INT8, flags=0, tile_replicas=0,
             tile_bytes=0, block_threads=0) -> _Options:
    return _Options(int(seed) & 0xFFFFFFFFFFFFFFFF, int(sweeps_per_exchange), int(encoding),
                    int(flags), int(tile_replicas), int(tile_bytes), int(block_threads))


def checkpoint_size(instances: Sequence, seed: int, **options) -> int:
    """Bytes of a checkpoint of these instances and options (pt_checkpoint_validate with
    no buffer; no GPU needed)."""
    recs, _keep = _records(list(instances))
    opt = _options(seed, **options)
    need = C.c_size_t(0)
    _check(lib().pt_checkpoint_validate(C.cast(recs, C.c_void_p), len(recs), C.byref(opt),
                                        None, 0, C.byref(need)))
    return int(need.value)


def checkpoint_validate(instances: Sequence, seed: int, blob: bytes, **options):
    """Raise PTError unless pt_load would accept blob for these instances and options
    (no GPU needed)."""
    recs, _keep = _records(list(instances))
    opt = _options(seed, **options)
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _check(lib().pt_checkpoint_validate(C.cast(recs, C.c_void_p), len(recs), C.byref(opt),
                                        C.cast(buf, C.c_void_p), len(blob), None))


class Sampler:
    """A batch of instances sampled by the library (one pt_ctx).

    instances: objects with N, M, R, edges [E,2], J, h, color, n_colors, b, K (see the
    workloads module).  Instance n of the batch uses n in its random counters.
    """

    def __init__(self, instances: Iterable, seed: int, sweeps_per_exchange: int = 1,
                 encoding: int = PT_INT8, flags: int = 0, tile_replicas: int = 0,
                 block_threads: int = 0, tile_bytes: int = 0,
                 stream: Optional[torch.cuda.Stream] = None,
                 torch_workspace: bool = True):
        self.instances = list(instances)
        recs, self._keep = _records(self.instances)
        self._recs = recs
        self.opt = _options(seed, sweeps_per_exchange, encoding, flags, tile_replicas,
                            tile_bytes, block_threads)
        L = lib()
        nbytes = C.c_size_t(0)
        _check(L.pt_workspace_bytes(C.cast(recs, C.c_void_p), len(self.instances),
                                    C.byref(self.opt), C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        ws_ptr, ws_len = None, 0
        self._ws = None
        if torch_workspace:
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            ws_ptr = (base + 255) // 256 * 256
            ws_len = self.workspace_bytes
        ctx = C.c_void_p()
        _check(L.pt_init(C.byref(ctx), C.cast(recs, C.c_void_p), len(self.instances),
                         C.byref(self.opt), C.c_void_p(self._stream.cuda_stream),
                         C.c_void_p(ws_ptr) if ws_ptr else None, ws_len))
        self._ctx = ctx

    # -- lifetime
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().pt_free(self._ctx)
            self._ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- dynamics
    def sweep(self, n: int = 1):
        _check(lib().pt_sweep(self._ctx, int(n)))

    def exchange(self):
        _check(lib().pt_exchange(self._ctx))

    def run(self, n_cycles: int):
        _check(lib().pt_run(self._ctx, int(n_cycles)))

    def sync(self):
        _check(lib().pt_sync(self._ctx))

    # -- state
    def observables(self, n: int = 0) -> Dict[str, np.ndarray]:
        inst = self.instances[n]
        R = inst.R
        o = dict(E_cl=np.zeros(R, np.int64), C=np.zeros(R, np.int64),
                 rung_of=np.zeros(R, np.int32), replica_of=np.zeros(R, np.int32),
                 acc=np.zeros(R - 1, np.uint64), att=np.zeros(R - 1, np.uint64),
                 roundtrips=np.zeros(R, np.uint64), label=np.zeros(R, np.int8),
                 sumE=np.zeros(R, np.int64), sumC=np.zeros(R, np.int64),
                 sumE2=np.zeros(R, np.int64), sumC2=np.zeros(R, np.int64),
                 nup=np.zeros(R, np.uint64), ndown=np.zeros(R, np.uint64),
                 sumCt=np.zeros((R, TAU_LAGS), np.int64))
        rec = _Obs(*[o[k].ctypes.data for k in ("E_cl", "C", "rung_of", "replica_of", "acc",
                                                 "att", "roundtrips", "label", "sumE", "sumC",
                                                 "sumE2", "sumC2", "nup", "ndown")], 0, 0, 0,
                   o["sumCt"].ctypes.data)
        _check(lib().pt_observables(self._ctx, int(n), C.byref(rec)))
        o["t"], o["e"], o["n_acc"] = int(rec.t), int(rec.e), int(rec.n_acc)
        return o

    def spins(self, n: int = 0) -> np.ndarray:
        inst = self.instances[n]
        out = np.zeros((inst.R, inst.M, inst.N), dtype=np.int8)
        _check(lib().pt_get_spins(self._ctx, int(n), out.ctypes.data))
        return out

    def set_spins(self, n: int, s: np.ndarray):
        s = _arr(s, np.int8)
        _check(lib().pt_set_spins(self._ctx, int(n), s.ctypes.data))

    def save(self) -> bytes:
        L = lib()
        ln = C.c_size_t(0)
        _check(L.pt_save(self._ctx, None, C.byref(ln)))
        buf = (C.c_char * ln.value)()
        _check(L.pt_save(self._ctx, C.cast(buf, C.c_void_p), C.byref(ln)))
        return bytes(buf)

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().pt_load(self._ctx, C.cast(buf, C.c_void_p), len(blob)))

    def info(self) -> Dict[str, float]:
        rec = _Info()
        _check(lib().pt_get_info(self._ctx, C.byref(rec)))
        return {name: getattr(rec, name) for name, _ in _Info._fields_}

    def timing_reset(self):
        _check(lib().pt_timing_reset(self._ctx))

    def timing_enable(self, on: bool):
        _check(lib().pt_timing_enable(self._ctx, 1 if on else 0))


class LadderNet:
    """Device-side parameters and Adam state of the ladder network, driven through the
    library's FP32 kernels (forward, cross-entropy gradients, Adam)."""

    N_IN, N_OUT = 32, 64

    def __init__(self, params: Optional[np.ndarray] = None, seed: int = 0):
        self.n = int(lib().pt_mlp_param_count())
        if params is None:
            params = init_ladder_params(seed)
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n:
            raise ValueError(f"expected {self.n} parameters, got {p.size}")
        self.params = torch.from_numpy(p.copy()).cuda()
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}

    def _workspace(self, batch: int):
        if batch not in self._ws:
            nb = int(lib().pt_mlp_workspace_bytes(batch))
            self._ws[batch] = torch.empty(nb, dtype=torch.uint8, device="cuda")
        return self._ws[batch]

    def forward(self, x) -> torch.Tensor:
        x = torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
        B = x.shape[0]
        out = torch.empty((B, self.N_OUT), dtype=torch.float32, device="cuda")
        rc = lib().pt_mlp_forward(self.params.data_ptr(), x.data_ptr(), out.data_ptr(), B,
                                  self._workspace(B).data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
        _check(rc)
        return out

    def loss_grad(self, x, q, kind: int = MLP_LOSS_SIGMOID) -> float:
        x = torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
        q = torch.as_tensor(q, dtype=torch.float32).cuda().contiguous()
        B = x.shape[0]
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        rc = lib().pt_mlp_loss_grad(self.params.data_ptr(), x.data_ptr(), q.data_ptr(), B,
                                    int(kind), self.grads.data_ptr(), loss.data_ptr(),
                                    self._workspace(B).data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
        _check(rc)
        return float(loss.item()) / B

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        rc = lib().pt_mlp_adam(self.params.data_ptr(), self.grads.data_ptr(), self.m.data_ptr(),
                               self.v.data_ptr(), self.n, lr, beta1, beta2, eps, self.step,
                               torch.cuda.current_stream().cuda_stream)
        _check(rc)

    def numpy_params(self) -> np.ndarray:
        return self.params.cpu().numpy().copy()


def init_ladder_params(seed: int = 0, out_bias: float = 0.0) -> np.ndarray:
    """He-uniform hidden weights, zero hidden biases, a zero output layer and output
    biases out_bias."""
    rng = np.random.default_rng(seed)
    sizes = [(128, 32), (128,), (128, 128), (128,), (64, 128), (64,)]
    out = []
    for k, shp in enumerate(sizes):
        if len(shp) == 2 and k < 4:
            lim = np.sqrt(6.0 / shp[1])
            out.append(rng.uniform(-lim, lim, size=shp).astype(np.float32).ravel())
        else:
            fill = out_bias if k == 5 else 0.0
            out.append(np.full(int(np.prod(shp)), fill, np.float32))
    return np.concatenate(out)
