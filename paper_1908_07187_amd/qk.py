"""ctypes binding of libqk.so (the C ABI declared in include/qk.h).

Argument marshalling only: every step of the state update runs in the HIP
kernels of libqk.so.  PyTorch provides device memory (its caching allocator,
through the allocator callbacks) and the HIP stream.  If the library is not
built this module raises ImportError-like errors loudly; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libqk.so")

QK_OK = 0
STATUS = {0: "QK_OK", -1: "QK_E_ARG", -2: "QK_E_NOT_UNITARY", -3: "QK_E_NOT_PERMUTATION", -4: "QK_E_OOM",
          -5: "QK_E_HIP", -6: "QK_E_STATE", -7: "QK_E_UNSUPPORTED"}
QK_C64, QK_C128 = 1, 2
DTYPES = {"c64": QK_C64, "complex64": QK_C64, "c128": QK_C128, "complex128": QK_C128}
BUILTINS = {"H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "T": 6, "SDG": 7, "TDG": 8, "RX": 9, "RY": 10, "RZ": 11,
            "PHASE": 12, "CPHASE": 13, "SWAP": 14, "RZZ": 15}

# Every exported symbol and its signature (restype, argtypes).
_P, _I32, _I64, _D, _SZ, _U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t, C.c_uint64
_I32P, _DP, _U8P, _U64P, _I64P = (C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_uint8),
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_int64))


class QkCond(C.Structure):
    _fields_ = [("cbit", C.c_int32), ("value", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
INDEX_FN = C.CFUNCTYPE(C.c_uint64, C.c_uint64, C.c_void_p)


class QkAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


QK_OP_GATE, QK_OP_MEASURE = 1, 2


class QkOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("gate", C.c_int32), ("targets", C.c_int32 * 2), ("n_targets", C.c_int32),
                ("controls", C.c_int32 * 4), ("n_controls", C.c_int32), ("conds", QkCond * 2),
                ("n_conds", C.c_int32), ("param", C.c_double), ("qubit", C.c_int32), ("cbit", C.c_int32),
                ("u", C.c_double)]


SIGNATURES = {
    "qk_create": (_I32, [_I32, C.POINTER(QkAllocator), _P, C.POINTER(_P)]),
    "qk_create_sparse": (_I32, [_I32, C.POINTER(QkAllocator), _P, _I64, C.POINTER(_P)]),
    "qk_sparse_nnz": (_I32, [_P, _I64P]),
    "qk_sparse_entries": (_I32, [_P, _U64P, _P, _I64, _I64P]),
    "qk_destroy": (_I32, [_P]),
    "qk_add_qubits": (_I32, [_P, _I32, _I32P]),
    "qk_add_cbits": (_I32, [_P, _I32, _I32P]),
    "qk_gate_builtin": (_I32, [C.c_char_p, _I32P]),
    "qk_define_gate_matrix": (_I32, [_P, C.c_char_p, _I32, _DP, _D, _I32P]),
    "qk_define_gate_index": (_I32, [_P, C.c_char_p, _I32, INDEX_FN, _P, _I32P]),
    "qk_define_gate_table": (_I32, [_P, C.c_char_p, _I32, _U64P, _I32P]),
    "qk_define_gate_affine": (_I32, [_P, C.c_char_p, _I32, _U64, _U64, _I32P]),
    "qk_define_gate_modmul": (_I32, [_P, C.c_char_p, _I32, _U64, _U64, _I32P]),
    "qk_apply_gate": (_I32, [_P, _I32, _I32P, _I32, _I32P, _I32, C.POINTER(QkCond), _I32, _DP, _I32]),
    "qk_measure": (_I32, [_P, _I32, _I32, _D]),
    "qk_measure_dev": (_I32, [_P, _I32, _I32, _P]),
    "qk_postselect": (_I32, [_P, _I32, _I32, _I32]),
    "qk_read_cbits": (_I32, [_P, _U8P, _I32]),
    "qk_sample": (_I32, [_P, _I32P, _I32, _DP, _I64, _U64P]),
    "qk_sample_dev": (_I32, [_P, _I32P, _I32, _P, _I64, _P]),
    "qk_probabilities": (_I32, [_P, _I32P, _I32, _DP]),
    "qk_read_measure_log": (_I32, [_P, _DP, _I32, _I32P]),
    "qk_get_state": (_I32, [_P, _P, _SZ]),
    "qk_set_state": (_I32, [_P, _P, _SZ]),
    "qk_state_ptr": (_I32, [_P, C.POINTER(_P), C.POINTER(_SZ)]),
    "qk_inner_product": (_I32, [_P, _P, _DP, _DP]),
    "qk_norm2": (_I32, [_P, _DP]),
    "qk_norm2_async": (_I32, [_P, C.c_void_p, _I32, _I32P]),
    "qk_read_cbits_async": (_I32, [_P, C.c_void_p, _I32]),
    "qk_set_fusion": (_I32, [_P, _I32]),
    "qk_flush": (_I32, [_P]),
    "qk_sync": (_I32, [_P]),
    "qk_num_qubits": (_I32, [_P, _I32P]),
    "qk_set_tuning": (_I32, [_P, C.c_char_p, _I32]),
    "qk_get_tuning": (_I32, [_P, C.c_char_p, _I32P]),
    "qk_stats": (_I32, [_P, _I64P, _I64P, _I64P]),
    "qk_reset": (_I32, [_P]),
    "qk_capture_begin": (_I32, [_P]),
    "qk_capture_end": (_I32, [_P, C.POINTER(_P)]),
    "qk_graph_launch": (_I32, [_P]),
    "qk_graph_destroy": (_I32, [_P]),
    "qk_batch_create": (_I32, [_I32, C.POINTER(QkAllocator), _P, C.POINTER(_P)]),
    "qk_batch_destroy": (_I32, [_P]),
    "qk_batch_add": (_I32, [_P, _I32, _I32, C.POINTER(QkOp), _I32, _I32P]),
    "qk_batch_run": (_I32, [_P]),
    "qk_batch_sync": (_I32, [_P]),
    "qk_batch_get_state": (_I32, [_P, _I32, _P, _SZ]),
    "qk_batch_read_cbits": (_I32, [_P, _I32, _U8P, _I32]),
    "qk_batch_layout": (_I32, [_P, _I32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "qk_batch_read_async": (_I32, [_P, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t]),
    "qk_batch_state_ptr": (_I32, [_P, _I32, C.POINTER(_P), C.POINTER(_SZ)]),
    "qk_batch_clear": (_I32, [_P]),
    "qk_batch_num_jobs": (_I32, [_P, _I32P]),
    "qk_batch_last_error": (C.c_char_p, [_P]),
    "qk_plan_fusion": (_I32, [_I32, C.POINTER(QkOp), _I32, _I32, _I32P, _U64P, _I32P, _I32, _DP, _SZ]),
    "qk_measure_noalloc": (_I32, [_I32, _P, _I32, _I32, _P, _P, _P, _P]),
    "qk_apply_ops": (_I32, [_P, C.POINTER(QkOp), _I32, _I32P]),
    "qk_last_error": (C.c_char_p, [_P]),
    "qk_status_string": (C.c_char_p, [_I32]),
}

_lib = None


def load(build_if_missing: bool = True):
    """Load libqk.so; build it first if it does not exist (never a fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise ImportError(f"{LIB_PATH} is not built")
        from .build import build
        build()
    # torch first: the library must bind to the HIP runtime torch already
    # holds (its device memory and streams are passed in).  Loaded before
    # torch, the library pulled in a second runtime, which then found no
    # device once torch's had initialised the GPU.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class QKError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


def _i32arr(xs):
    xs = [int(x) for x in xs]
    return (C.c_int32 * max(1, len(xs)))(*xs), len(xs)


# ------------------------------------------------------------------ torch plumbing

class _TorchDevice:
    """Caching-allocator callbacks and the stream handle from PyTorch."""

    def __init__(self, stream=None, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch: the HIP path cannot run here")
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.allocator = QkAllocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, ctx):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0)))
        except Exception:
            return None

    def _do_free(self, ptr, nbytes, stream, ctx):
        try:
            self.torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    @property
    def stream_handle(self) -> int:
        return int(self.stream.cuda_stream)


class Sim:
    """One state on the GPU.  Thin wrapper over the qk_* calls.  With
    ``sparse=N`` the state is kept as at most N nonzero (index, amplitude)
    entries (qk_create_sparse) instead of a dense vector."""

    def __init__(self, dtype: str = "c128", stream=None, allocator: str = "torch", device: int = 0,
                 sparse: Optional[int] = None):
        self.lib = load()
        self.dtype = dtype
        self.sparse = sparse
        self.np_dtype = np.complex64 if DTYPES[dtype] == QK_C64 else np.complex128
        h = C.c_void_p()
        if allocator == "torch":
            self._dev = _TorchDevice(stream, device)
            alloc, stream_h = C.byref(self._dev.allocator), C.c_void_p(self._dev.stream_handle)
        elif allocator == "none":
            # hipMalloc inside the library, null stream (CPU-side argument checks work without a GPU)
            self._dev = None
            alloc, stream_h = None, None
        else:
            raise ValueError(allocator)
        if sparse is None:
            st = self.lib.qk_create(DTYPES[dtype], alloc, stream_h, C.byref(h))
        else:
            st = self.lib.qk_create_sparse(DTYPES[dtype], alloc, stream_h, int(sparse), C.byref(h))
        if st != QK_OK:
            raise QKError(st, self.lib.qk_last_error(None).decode())
        self.h = h
        self.n = 0
        self.ncbits = 0
        self._builtin_cache = {}

    # -- errors / lifetime
    def _chk(self, st):
        if st != QK_OK:
            raise QKError(st, self.lib.qk_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._chk(self.lib.qk_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- registers
    def add_qubits(self, m: int) -> int:
        first = C.c_int32()
        self._chk(self.lib.qk_add_qubits(self.h, m, C.byref(first)))
        self.n += m
        return first.value

    def add_cbits(self, m: int) -> int:
        first = C.c_int32()
        self._chk(self.lib.qk_add_cbits(self.h, m, C.byref(first)))
        self.ncbits += m
        return first.value

    # -- gates
    def builtin(self, name: str) -> int:
        gid = self._builtin_cache.get(name)
        if gid is None:
            out = C.c_int32()
            st = self.lib.qk_gate_builtin(name.encode(), C.byref(out))
            if st != QK_OK:
                raise QKError(st, self.lib.qk_last_error(None).decode())
            gid = self._builtin_cache[name] = out.value
        return gid

    def define_matrix(self, name: str, m: np.ndarray, tol: float = 1e-10) -> int:
        m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
        k = int(round(np.log2(m.shape[0])))
        f = m.view(np.float64).reshape(-1)
        out = C.c_int32()
        self._chk(self.lib.qk_define_gate_matrix(self.h, name.encode(), k, f.ctypes.data_as(_DP), tol,
                                                 C.byref(out)))
        return out.value

    def define_table(self, name: str, table: np.ndarray) -> int:
        t = np.ascontiguousarray(np.asarray(table, dtype=np.uint64))
        k = int(round(np.log2(len(t))))
        out = C.c_int32()
        self._chk(self.lib.qk_define_gate_table(self.h, name.encode(), k, t.ctypes.data_as(_U64P), C.byref(out)))
        return out.value

    def define_index(self, name: str, k: int, fn) -> int:
        cb = INDEX_FN(lambda x, ctx: int(fn(int(x))))
        out = C.c_int32()
        self._chk(self.lib.qk_define_gate_index(self.h, name.encode(), k, cb, None, C.byref(out)))
        return out.value

    def define_affine(self, name: str, k: int, a: int, b: int) -> int:
        out = C.c_int32()
        self._chk(self.lib.qk_define_gate_affine(self.h, name.encode(), k, a, b, C.byref(out)))
        return out.value

    def define_modmul(self, name: str, k: int, a: int, N: int) -> int:
        out = C.c_int32()
        self._chk(self.lib.qk_define_gate_modmul(self.h, name.encode(), k, a, N, C.byref(out)))
        return out.value

    def apply(self, gate, targets: Sequence[int], controls: Sequence[int] = (),
              conds: Sequence[Tuple[int, int]] = (), params: Sequence[float] = ()):
        gid = self.builtin(gate) if isinstance(gate, str) else int(gate)
        t, nt = _i32arr(targets)
        c, nc = _i32arr(controls)
        cd = (QkCond * max(1, len(conds)))(*[QkCond(int(a), int(b)) for a, b in conds])
        p = (C.c_double * max(1, len(params)))(*[float(x) for x in params])
        self._chk(self.lib.qk_apply_gate(self.h, gid, t, nt, c, nc, cd, len(conds), p, len(params)))

    def apply_ops(self, ops, count: Optional[int] = None) -> None:
        """A ctypes array of QkOp records (batch.op_array) in one call."""
        done = C.c_int32()
        self._chk(self.lib.qk_apply_ops(self.h, ops, len(ops) if count is None else count, C.byref(done)))

    # -- measurement
    def measure(self, qubit: int, cbit: int = -1, u: float = 0.0):
        self._chk(self.lib.qk_measure(self.h, qubit, cbit, u))

    def measure_dev(self, qubit: int, cbit: int, d_u_ptr: int):
        self._chk(self.lib.qk_measure_dev(self.h, qubit, cbit, C.c_void_p(d_u_ptr)))

    def postselect(self, qubit: int, cbit: int, outcome: int):
        self._chk(self.lib.qk_postselect(self.h, qubit, cbit, outcome))

    def sample(self, uniforms, qubits=()) -> np.ndarray:
        """Deferred measurement: one shot per uniform in [0, 1); bit j of each
        result is bit qubits[j] of the drawn index (the index itself when
        qubits is empty).  The state is left unchanged."""
        qs = (C.c_int32 * max(1, len(qubits)))(*[int(q) for q in qubits])
        u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64).reshape(-1))
        out = np.empty(max(1, len(u)), dtype=np.uint64)
        self._chk(self.lib.qk_sample(self.h, qs, len(qubits), u.ctypes.data_as(_DP), len(u),
                                     out.ctypes.data_as(_U64P)))
        return out[: len(u)]

    def sample_dev(self, d_uniforms_ptr: int, n_shots: int, d_out_ptr: int, qubits=()):
        """As sample() with device arrays (n_shots doubles in, n_shots uint64 out); asynchronous."""
        qs = (C.c_int32 * max(1, len(qubits)))(*[int(q) for q in qubits])
        self._chk(self.lib.qk_sample_dev(self.h, qs, len(qubits), C.c_void_p(d_uniforms_ptr), n_shots,
                                         C.c_void_p(d_out_ptr)))

    def probabilities(self, qubits) -> np.ndarray:
        """Normalised distribution of the listed qubits (entry m: bit j of m = qubits[j])."""
        qs = (C.c_int32 * max(1, len(qubits)))(*[int(q) for q in qubits])
        out = np.empty(1 << len(qubits), dtype=np.float64)
        self._chk(self.lib.qk_probabilities(self.h, qs, len(qubits), out.ctypes.data_as(_DP)))
        return out

    def nnz(self) -> int:
        """Entries of a sparse state."""
        out = C.c_int64()
        self._chk(self.lib.qk_sparse_nnz(self.h, C.byref(out)))
        return out.value

    def entries(self) -> Tuple[np.ndarray, np.ndarray]:
        """(ascending indices uint64, amplitudes) of a sparse state."""
        n = self.nnz()
        idx = np.empty(max(1, n), dtype=np.uint64)
        amp = np.empty(max(1, n), dtype=self.np_dtype)
        got = C.c_int64()
        self._chk(self.lib.qk_sparse_entries(self.h, idx.ctypes.data_as(_U64P), C.c_void_p(amp.ctypes.data), len(idx),
                                             C.byref(got)))
        return idx[: got.value], amp[: got.value]

    def read_cbits(self, n: Optional[int] = None) -> np.ndarray:
        n = self.ncbits if n is None else n
        out = np.zeros(max(1, n), dtype=np.uint8)
        self._chk(self.lib.qk_read_cbits(self.h, out.ctypes.data_as(_U8P), n))
        return out[:n]

    def measure_log(self, count: int = 4096) -> np.ndarray:
        buf = np.zeros(3 * max(1, count), dtype=np.float64)
        w = C.c_int32()
        self._chk(self.lib.qk_read_measure_log(self.h, buf.ctypes.data_as(_DP), count, C.byref(w)))
        return buf[: 3 * w.value].reshape(-1, 3)

    # -- readout
    def state(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=self.np_dtype)
        self._chk(self.lib.qk_get_state(self.h, C.c_void_p(out.ctypes.data), out.nbytes))
        return out

    def set_state(self, psi: np.ndarray):
        a = np.ascontiguousarray(np.asarray(psi, dtype=self.np_dtype))
        self._chk(self.lib.qk_set_state(self.h, C.c_void_p(a.ctypes.data), a.nbytes))

    def state_ptr(self) -> Tuple[int, int]:
        p = C.c_void_p()
        nb = C.c_size_t()
        self._chk(self.lib.qk_state_ptr(self.h, C.byref(p), C.byref(nb)))
        return int(p.value or 0), int(nb.value)

    def inner(self, other: "Sim") -> complex:
        re, im = C.c_double(), C.c_double()
        self._chk(self.lib.qk_inner_product(self.h, other.h, C.byref(re), C.byref(im)))
        return complex(re.value, im.value)

    def norm2(self) -> float:
        out = C.c_double()
        self._chk(self.lib.qk_norm2(self.h, C.byref(out)))
        return out.value

    def norm2_async(self, host_ptr: int, capacity: int) -> int:
        """Enqueue the norm's partial sums and their copy to host memory at
        host_ptr (capacity doubles); returns their number nb.  After the
        stream reaches this point, norm2 = sum of the nb real parts in order
        (``norm2_from_partials``)."""
        count = C.c_int32()
        self._chk(self.lib.qk_norm2_async(self.h, C.c_void_p(host_ptr), int(capacity), C.byref(count)))
        return count.value

    def read_cbits_async(self, host_ptr: int, n: Optional[int] = None):
        """Enqueue the copy of the first n cbits (all by default) to host_ptr."""
        n = self.ncbits if n is None else n
        self._chk(self.lib.qk_read_cbits_async(self.h, C.c_void_p(host_ptr), int(n)))

    # -- execution control
    def set_fusion(self, k: int):
        self._chk(self.lib.qk_set_fusion(self.h, k))

    def flush(self):
        self._chk(self.lib.qk_flush(self.h))

    def sync(self):
        self._chk(self.lib.qk_sync(self.h))

    def set_tuning(self, key: str, value: int):
        self._chk(self.lib.qk_set_tuning(self.h, key.encode(), int(value)))

    def get_tuning(self, key: str) -> int:
        out = C.c_int32()
        self._chk(self.lib.qk_get_tuning(self.h, key.encode(), C.byref(out)))
        return out.value

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._chk(self.lib.qk_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {"sweeps": a.value, "fused_blocks": b.value, "fused_gates": c.value}


def measure_noalloc(dtype: str, d_state: int, n_qubits: int, qubit: int, d_u: int, d_cbit: int = 0,
                    d_result: int = 0, stream: int = 0):
    """qk_measure_noalloc on device addresses (plain integers; 0 = NULL)."""
    lib = load()
    st = lib.qk_measure_noalloc(DTYPES[dtype], C.c_void_p(d_state), int(n_qubits), int(qubit), C.c_void_p(d_u),
                                C.c_void_p(d_cbit or None), C.c_void_p(d_result or None), C.c_void_p(stream or None))
    if st != QK_OK:
        raise QKError(st, lib.qk_last_error(None).decode())


# ------------------------------------------------------------------ graphs

class Graph:
    """A captured sequence of calls on one Sim, replayed with one launch."""

    def __init__(self, sim: "Sim", handle):
        self.sim = sim
        self.h = handle

    def launch(self):
        self.sim._chk(self.sim.lib.qk_graph_launch(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.sim._chk(self.sim.lib.qk_graph_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _sim_reset(self):
    self._chk(self.lib.qk_reset(self.h))


def _sim_capture_begin(self):
    self._chk(self.lib.qk_capture_begin(self.h))


def _sim_capture_end(self) -> Graph:
    g = C.c_void_p()
    self._chk(self.lib.qk_capture_end(self.h, C.byref(g)))
    return Graph(self, g)


Sim.reset = _sim_reset
Sim.capture_begin = _sim_capture_begin
Sim.capture_end = _sim_capture_end


# ------------------------------------------------------------------ batches

class Batch:
    """Many small circuits (builtin gates + measurements) in one persistent launch."""

    def __init__(self, dtype: str = "c128", stream=None, device: int = 0):
        self.lib = load()
        self.dtype = dtype
        self.np_dtype = np.complex64 if DTYPES[dtype] == QK_C64 else np.complex128
        self._dev = _TorchDevice(stream, device)
        h = C.c_void_p()
        st = self.lib.qk_batch_create(DTYPES[dtype], C.byref(self._dev.allocator),
                                      C.c_void_p(self._dev.stream_handle), C.byref(h))
        if st != QK_OK:
            raise QKError(st, self.lib.qk_batch_last_error(None).decode())
        self.h = h
        self.jobs = []          # (n, ncbits)

    def _chk(self, st):
        if st != QK_OK:
            raise QKError(st, self.lib.qk_batch_last_error(self.h).decode())

    def add(self, n: int, ncbits: int, ops, count: Optional[int] = None) -> int:
        """ops: a list of QkOp, or a ctypes QkOp array with its record count."""
        if count is None:
            arr, count = (QkOp * max(1, len(ops)))(*ops), len(ops)
        else:
            arr = ops
        job = C.c_int32()
        self._chk(self.lib.qk_batch_add(self.h, n, ncbits, arr, count, C.byref(job)))
        self.jobs.append((n, ncbits))
        return job.value

    def run(self):
        self._chk(self.lib.qk_batch_run(self.h))

    def sync(self):
        self._chk(self.lib.qk_batch_sync(self.h))

    def state(self, job: int) -> np.ndarray:
        n = self.jobs[job][0]
        out = np.empty(1 << n, dtype=self.np_dtype)
        self._chk(self.lib.qk_batch_get_state(self.h, job, C.c_void_p(out.ctypes.data), out.nbytes))
        return out

    def cbits(self, job: int) -> np.ndarray:
        nc = self.jobs[job][1]
        out = np.zeros(max(1, nc), dtype=np.uint8)
        self._chk(self.lib.qk_batch_read_cbits(self.h, job, out.ctypes.data_as(_U8P), nc))
        return out[:nc]

    def layout(self, job: int) -> Tuple[int, int, int]:
        """(state byte offset, state bytes, cbit offset) of a job in the batch's buffers."""
        so, sb, co = C.c_size_t(), C.c_size_t(), C.c_size_t()
        self._chk(self.lib.qk_batch_layout(self.h, job, C.byref(so), C.byref(sb), C.byref(co)))
        return so.value, sb.value, co.value

    def sizes(self) -> Tuple[int, int]:
        """Total bytes of the batch's states and cbits."""
        if not self.jobs:
            return 0, 0
        so, sb, co = self.layout(len(self.jobs) - 1)
        return so + sb, co + self.jobs[-1][1]

    def read_async(self, host_states_ptr: int, state_bytes: int, host_cbits_ptr: int, cbit_bytes: int):
        """Enqueue the copy of every job's final state and cbits into host
        memory (see qk_batch_read_async); read it after the stream gets there."""
        self._chk(self.lib.qk_batch_read_async(self.h, C.c_void_p(host_states_ptr), int(state_bytes),
                                               C.c_void_p(host_cbits_ptr), int(cbit_bytes)))

    def clear(self):
        self._chk(self.lib.qk_batch_clear(self.h))
        self.jobs = []

    def close(self):
        if getattr(self, "h", None):
            self._chk(self.lib.qk_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_fusion(n: int, ops, max_k: int, with_matrices: bool = False):
    """Host-only fusion plan: [(qubit list, gates composed, matrix or None)]."""
    lib = load()
    arr = (QkOp * max(1, len(ops)))(*ops)
    nb = C.c_int32()
    st = lib.qk_plan_fusion(n, arr, len(ops), max_k, C.byref(nb), None, None, 0, None, 0)
    if st != QK_OK:
        raise QKError(st, lib.qk_last_error(None).decode())
    masks = (C.c_uint64 * max(1, nb.value))()
    gates = (C.c_int32 * max(1, nb.value))()
    cap = nb.value * (4 ** max_k) * 2 if with_matrices else 0
    mats = np.zeros(max(1, cap), dtype=np.float64)
    st = lib.qk_plan_fusion(n, arr, len(ops), max_k, C.byref(nb), masks, gates, nb.value,
                            mats.ctypes.data_as(_DP) if with_matrices else None, cap)
    if st != QK_OK:
        raise QKError(st, lib.qk_last_error(None).decode())
    out, off = [], 0
    for b in range(nb.value):
        qs = [q for q in range(64) if (masks[b] >> q) & 1]
        m = None
        if with_matrices:
            d = 1 << len(qs)
            m = mats[off: off + 2 * d * d].view(np.complex128).reshape(d, d).copy()
            off += 2 * d * d
        out.append((qs, gates[b], m))
    return out


def norm2_from_partials(parts, nb: int) -> float:
    """The norm from qk_norm2_async's copy: the nb real parts added in order
    (the same order, so the same value, as qk_norm2)."""
    total = 0.0
    for i in range(nb):
        total += float(parts[2 * i])
    return total
