"""MI355X-native negacyclic NTT over RNS prime moduli.

A thin ctypes binding of ``libntt.so`` (the C ABI in ``include/ntt.h``).  Every
step of every transform runs in the library's HIP kernels; this module only
checks shapes and passes device pointers and the current HIP stream.  PyTorch
supplies device memory and streams.  There is no CPU fallback: if the library
is not built, every call raises.

Paper: Chameleon (arXiv 2410.05934), Sec. II-D, Eq. (1) (the transform pair
and the convolution theorem) and Sec. V (the GPU NTT design this replaces).
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = ["Plan", "NTTError", "lib", "check_modulus", "find_root", "library_path",
           "FLAG_FORCE_INT64", "FLAG_ROW_RADIX8", "FLAG_ROW_RADIX4", "FLAG_FUSED", "FLAG_VALIDATE", "AUTOMORPH_TRANSFORMED", "flag_split", "stats_enable", "stats_reset", "stats_collect",
           "RaggedBatch", "batch_ragged", "debug_wait_limit", "BasisConversion", "OP_FORWARD", "OP_INVERSE", "OP_POLYMUL", "RAGGED_NO_GRAPH", "RAGGED_IN_WORKGROUP",
           "ragged_row_log", "tune_split", "tune_ragged", "tune_save", "tune_load", "tune_clear",
           "Server", "REQ_POLYMUL", "REQ_FORWARD", "REQ_INVERSE", "REQ_DEVICE", "REQ_HOST",
           "SERVER_SERIAL", "SERVER_DRY_RUN", "SERVER_MERGE_MODULI"]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libntt.so")
_lock = threading.Lock()
_lib = None

FLAG_FORCE_INT64 = 1 << 16
FLAG_ROW_RADIX8 = 1 << 17
FLAG_FUSED = 1 << 18
FLAG_ROW_RADIX4 = 1 << 19
FLAG_VALIDATE = 1 << 20
AUTOMORPH_TRANSFORMED = 1
BCONV_NO_MFMA = 1
BCONV_MFMA = 2
BCONV_NO_WS = 4

STATUS = {0: "NTT_OK", 1: "NTT_EINVAL", 2: "NTT_ENOTPRIME", 3: "NTT_ENOROOT", 4: "NTT_ERANGE",
          5: "NTT_ENOMEM", 6: "NTT_EDEVICE", 7: "NTT_EBUSY", 8: "NTT_ETIMEOUT"}


def flag_split(n1: int) -> int:
    """NTT_FLAG_SPLIT(n1): force n1 column stages (0 = single pass)."""
    return ((n1 + 1) & 0x1F) << 8


class NTTError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        self.name = STATUS.get(status, f"status {status}")
        super().__init__(f"{where}: {self.name}: {message}")


def library_path() -> str:
    return _LIB_PATH


_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_SIGS = {
    "ntt_plan_create": [ctypes.POINTER(_vp), _u32, ctypes.POINTER(_u64), _u32, _u32, _u32],
    "ntt_plan_destroy": [_vp],
    "ntt_plan_root": [_vp, _u32, ctypes.POINTER(_u64)],
    "ntt_plan_split": [_vp, ctypes.POINTER(_u32)],
    "ntt_plan_limb_class": [_vp, _u32, ctypes.POINTER(_u32)],
    "ntt_forward": [_vp, _vp, _u32, _vp],
    "ntt_inverse": [_vp, _vp, _u32, _vp],
    "ntt_pointwise_mul": [_vp, _vp, _vp, _vp, _u32, _vp],
    "ntt_mac": [_vp, _vp, _vp, _vp, _u32, _u32, _u32, _vp],
    "ntt_pointwise_mac": [_vp, _vp, _vp, _vp, _u32, _u32, _u32, _u32, _vp],
    "ntt_external_product": [_vp, _vp, _vp, _vp, _u32, _u32, _u32, _vp],
    "ntt_polymul": [_vp, _vp, _vp, _vp, _u32, _vp],
    "ntt_polymul_noalloc": [_vp, _vp, _vp, _vp, _u32, _vp],
    "ntt_automorph": [_vp, _vp, _vp, _u32, _u32, _u32, _vp],
    "ntt_forward_mul": [_vp, _vp, _vp, _vp, _u32, _vp],
    "ntt_cmux": [_vp, _vp, _vp, _vp, _vp, _u32, _u32, _u32, _u32, _vp],
    "ntt_bconv_create": [ctypes.POINTER(_vp), _u32, ctypes.POINTER(_u64), _u32, ctypes.POINTER(_u64),
                         _u32, _u32, _u32],
    "ntt_bconv": [_vp, _vp, _vp, _u32, _vp],
    "ntt_bconv_destroy": [_vp],
    "ntt_basis_ext_create": [ctypes.POINTER(_vp), _u32, ctypes.POINTER(_u64), _u32,
                             ctypes.POINTER(_u64), _u32, _u32, _u32],
    "ntt_mod_up": [_vp, _vp, _vp, _u32, _vp],
    "ntt_mod_down": [_vp, _vp, _vp, _u32, _vp],
    "ntt_basis_ext_destroy": [_vp],
    "ntt_external_product_decomposed": [_vp, _vp, _vp, _vp, _u32, _u32, _u32, _u32, _u32, _vp],
    "ntt_check_modulus": [_u32, _u64, _u32],
    "ntt_find_root": [_u32, _u64, ctypes.POINTER(_u64)],
    "ntt_plan_split_for": [_vp, _u32, ctypes.POINTER(_u32)],
    "ntt_ragged_create": [ctypes.POINTER(_vp), _vp, _u32, _u32],
    "ntt_ragged_run": [_vp, _vp],
    "ntt_ragged_info": [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32)],
    "ntt_ragged_destroy": [_vp],
    "ntt_batch_ragged": [_vp, _u32, _vp],
    "ntt_tune_split": [_u32, ctypes.POINTER(_u64), _u32, _u32, _u32, ctypes.POINTER(_u32),
                       ctypes.POINTER(ctypes.c_float)],
    "ntt_tune_ragged": [_u32, ctypes.POINTER(_u64), _u32, _u32, ctypes.POINTER(_u32),
                        ctypes.POINTER(ctypes.c_float)],
    "ntt_tune_save": [ctypes.c_char_p],
    "ntt_tune_load": [ctypes.c_char_p],
    "ntt_tune_clear": [],
    "ntt_server_create": [ctypes.POINTER(_vp), _u64, _u32, _u32, _u32],
    "ntt_server_submit": [_vp, _vp, ctypes.POINTER(_u64)],
    "ntt_server_wait": [_vp, _u64, _vp, ctypes.c_int32],
    "ntt_server_replay": [_vp, _vp, ctypes.POINTER(ctypes.c_double), _u32, ctypes.POINTER(_u64)],
    "ntt_server_counters_get": [_vp, _vp],
    "ntt_server_destroy": [_vp],
    "ntt_debug_wait_limit": [_u32, _u32],
    "ntt_stats_enable": [ctypes.c_int],
    "ntt_stats_reset": [],
    "ntt_stats_collect": [_vp, _u32, ctypes.POINTER(_u32)],
}


OP_FORWARD = 0
OP_INVERSE = 1
OP_POLYMUL = 2
RAGGED_NO_GRAPH = 1
RAGGED_IN_WORKGROUP = 1 << 1


def ragged_row_log(n2: int) -> int:
    """NTT_RAGGED_ROW_LOG(n2) flag."""
    return (n2 & 0xF) << 8


class _Job(ctypes.Structure):
    _fields_ = [("plan", _vp), ("op", _u32), ("batch", _u32), ("out", _vp), ("a", _vp), ("b", _vp)]


def _jobs_array(jobs):
    """jobs: (plan, OP_FORWARD | OP_INVERSE, tensor) transformed in place, or
    (plan, OP_POLYMUL, out, a, b)."""
    arr = (_Job * len(jobs))()
    for i, j in enumerate(jobs):
        plan, op = j[0], int(j[1])
        if op == OP_POLYMUL:
            out, a, b = j[2], j[3], j[4]
            n = plan._batch_of(out, f"job {i} out")
            if plan._batch_of(a, f"job {i} a") != n or plan._batch_of(b, f"job {i} b") != n:
                raise ValueError(f"job {i}: batch mismatch")
            arr[i] = _Job(plan._h.value, op, n, out.data_ptr(), a.data_ptr(), b.data_ptr())
        else:
            t = j[2]
            arr[i] = _Job(plan._h.value, op, plan._batch_of(t, f"job {i}"), t.data_ptr(), None, None)
    return arr


class RaggedBatch:
    """A reusable ragged batch: jobs (plan, op, tensor) -- or (plan, OP_POLYMUL,
    out, a, b) -- run as one persistent launch per word width plus grouped
    launches, replayed from a hipGraph unless no_graph is set.  The plans and
    tensors must outlive the batch."""

    def __init__(self, jobs, flags: int = 0):
        self._keep = list(jobs)
        arr = _jobs_array(jobs)
        h = _vp()
        _check(lib().ntt_ragged_create(ctypes.byref(h), ctypes.cast(arr, _vp), len(jobs), flags),
               "ntt_ragged_create")
        self._h = h

    def run(self, stream=None):
        _check(lib().ntt_ragged_run(self._h, _stream_handle(stream)), "ntt_ragged_run")

    def info(self):
        items, wgs = _u32(), _u32()
        _check(lib().ntt_ragged_info(self._h, ctypes.byref(items), ctypes.byref(wgs)), "ntt_ragged_info")
        return int(items.value), int(wgs.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ntt_ragged_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BasisConversion:
    """RNS basis conversion from src_moduli (L) to dst_moduli (M) for length N:
    out[b][j] = sum_i [x_i (Q/q_i)^-1]_(q_i) (Q/q_i) mod p_j (X + alpha Q, 0 <= alpha < L)."""

    def __init__(self, N: int, src_moduli, dst_moduli, word_bits: int = 64, mfma=None,
                 stationary: bool = True):
        """mfma: None lets the library choose, True asks for the int8 matrix cores
        wherever they apply, False keeps the vector units.  stationary=False keeps
        the matrix-core form that reloads its constant operands per tile."""
        self.N, self.word_bits = int(N), int(word_bits)
        self.L, self.M = len(src_moduli), len(dst_moduli)
        src = (_u64 * self.L)(*[int(q) for q in src_moduli])
        dst = (_u64 * self.M)(*[int(p) for p in dst_moduli])
        self._h = _vp()
        flags = (0 if mfma is None else (BCONV_MFMA if mfma else BCONV_NO_MFMA)) | \
            (0 if stationary else BCONV_NO_WS)
        _check(lib().ntt_bconv_create(ctypes.byref(self._h), self.N, src, self.L, dst, self.M,
                                      self.word_bits, flags), "ntt_bconv_create")

    def _batch(self, t, rows: int, name: str) -> int:
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
        if t.element_size() * 8 != self.word_bits:
            raise ValueError(f"{name} element size does not match word_bits")
        per = rows * self.N
        if t.numel() == 0 or t.numel() % per:
            raise ValueError(f"{name} has {t.numel()} elements, not a multiple of {per}")
        return t.numel() // per

    def __call__(self, out, x, stream=None):
        b = self._batch(x, self.L, "x")
        if self._batch(out, self.M, "out") != b:
            raise ValueError("batch mismatch")
        _check(lib().ntt_bconv(self._h, out.data_ptr(), x.data_ptr(), b, _stream_handle(stream)),
               "ntt_bconv")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ntt_bconv_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BasisExtension:
    """The key-switching basis Q = prod q_moduli (L limbs), P = prod p_moduli (K
    limbs) for length N.  mod_up: x[b][L][N] -> out[b][L + K][N] (x, then
    BConv_{Q->P}(x)); mod_down: x[b][L + K][N] -> out[b][L][N] with
    out_i = (x_i - BConv_{P->Q}(x_P)_i) P^-1 mod q_i."""

    def __init__(self, N: int, q_moduli, p_moduli, word_bits: int = 64, mfma=None,
                 stationary: bool = True):
        self.N, self.word_bits = int(N), int(word_bits)
        self.L, self.K = len(q_moduli), len(p_moduli)
        qs = (_u64 * self.L)(*[int(q) for q in q_moduli])
        ps = (_u64 * self.K)(*[int(p) for p in p_moduli])
        self._h = _vp()
        flags = (0 if mfma is None else (BCONV_MFMA if mfma else BCONV_NO_MFMA)) | \
            (0 if stationary else BCONV_NO_WS)
        _check(lib().ntt_basis_ext_create(ctypes.byref(self._h), self.N, qs, self.L, ps, self.K,
                                          self.word_bits, flags), "ntt_basis_ext_create")

    def _batch(self, t, rows: int, name: str) -> int:
        return BasisConversion._batch(self, t, rows, name)

    def mod_up(self, out, x, stream=None):
        b = self._batch(x, self.L, "x")
        if self._batch(out, self.L + self.K, "out") != b:
            raise ValueError("batch mismatch")
        _check(lib().ntt_mod_up(self._h, out.data_ptr(), x.data_ptr(), b, _stream_handle(stream)),
               "ntt_mod_up")
        return out

    def mod_down(self, out, x, stream=None):
        b = self._batch(x, self.L + self.K, "x")
        if self._batch(out, self.L, "out") != b:
            raise ValueError("batch mismatch")
        _check(lib().ntt_mod_down(self._h, out.data_ptr(), x.data_ptr(), b, _stream_handle(stream)),
               "ntt_mod_down")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ntt_basis_ext_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_ragged(jobs, stream=None) -> None:
    """One-shot ragged batch (no graph); returns after the stream has finished it."""
    arr = _jobs_array(jobs)
    _check(lib().ntt_batch_ragged(ctypes.cast(arr, _vp), len(jobs), _stream_handle(stream)),
           "ntt_batch_ragged")


def tune_split(N: int, moduli, word_bits: int, batch: int):
    """Autotune the pass split for this shape; returns (best n1, microseconds per fwd+inv)."""
    arr = (_u64 * len(moduli))(*[int(q) for q in moduli])
    best, us = _u32(), ctypes.c_float()
    _check(lib().ntt_tune_split(N, arr, len(moduli), word_bits, batch, ctypes.byref(best),
                                ctypes.byref(us)), "ntt_tune_split")
    return int(best.value), float(us.value)


def tune_ragged(N: int, moduli, batch: int):
    arr = (_u64 * len(moduli))(*[int(q) for q in moduli])
    best, us = _u32(), ctypes.c_float()
    _check(lib().ntt_tune_ragged(N, arr, len(moduli), batch, ctypes.byref(best), ctypes.byref(us)),
           "ntt_tune_ragged")
    return int(best.value), float(us.value)


def tune_save(path: str) -> None:
    _check(lib().ntt_tune_save(path.encode()), "ntt_tune_save")


def tune_load(path: str) -> None:
    _check(lib().ntt_tune_load(path.encode()), "ntt_tune_load")


def tune_clear() -> None:
    _check(lib().ntt_tune_clear(), "ntt_tune_clear")


REQ_POLYMUL, REQ_FORWARD, REQ_INVERSE = 0, 1, 2
REQ_DEVICE, REQ_HOST = 0, 1
SERVER_SERIAL, SERVER_DRY_RUN, SERVER_MERGE_MODULI = 1, 2, 4


class _Request(ctypes.Structure):
    _fields_ = [("op", _u32), ("N", _u32), ("word_bits", _u32), ("num_moduli", _u32),
                ("moduli", ctypes.POINTER(_u64)), ("batch", _u32), ("memory", _u32),
                ("a", _vp), ("b", _vp), ("out", _vp)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("id", _u64), ("status", ctypes.c_int32), ("batched_with", _u32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double), ("bytes", _u64),
                ("launch_id", _u64)]


class _ServerCounters(ctypes.Structure):
    _fields_ = [(n, _u64) for n in ("submitted", "completed", "rejected", "launches",
                                    "max_inflight_bytes", "max_inflight_requests",
                                    "budget_bytes", "plans_cached", "arena_bytes",
                                    "max_arena_bytes", "merged_launches", "direct_launches")]


class Server:
    """Continuous-batching request server (C++ thread inside libntt.so)."""

    def __init__(self, budget_bytes: int, n_streams: int = 4, max_batch: int = 0, flags: int = 0):
        h = _vp()
        _check(lib().ntt_server_create(ctypes.byref(h), int(budget_bytes), n_streams, max_batch, flags),
               "ntt_server_create")
        self._h = h

    def submit(self, op: int, N: int, moduli, word_bits: int, batch: int, a=0, b=0, out=0,
               memory: int = REQ_DEVICE) -> int:
        """a, b, out: device (or host) addresses as ints; returns the request id."""
        mods = (_u64 * len(moduli))(*[int(q) for q in moduli])
        r = _Request(op, N, word_bits, len(moduli), ctypes.cast(mods, ctypes.POINTER(_u64)), batch,
                     memory, a or None, b or None, out or None)
        rid = _u64()
        _check(lib().ntt_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "ntt_server_submit")
        return int(rid.value)

    def replay(self, requests, arrivals) -> list:
        """requests: list of (op, N, moduli, word_bits, batch, a, b, out[, memory]);
        arrivals: seconds after the call starts.  Submits at native speed."""
        n = len(requests)
        arr = (_Request * n)()
        keep = []
        for i, r in enumerate(requests):
            op, N, moduli, wb, batch, a, b, out = r[:8]
            memory = r[8] if len(r) > 8 else REQ_DEVICE
            mods = (_u64 * len(moduli))(*[int(q) for q in moduli])
            keep.append(mods)
            arr[i] = _Request(op, N, wb, len(moduli), ctypes.cast(mods, ctypes.POINTER(_u64)), batch,
                              memory, a or None, b or None, out or None)
        times = (ctypes.c_double * n)(*[float(t) for t in arrivals])
        ids = (_u64 * n)()
        _check(lib().ntt_server_replay(self._h, ctypes.cast(arr, _vp), times, n, ids), "ntt_server_replay")
        return [int(x) for x in ids]

    def wait(self, rid: int, timeout_ms: int = -1) -> dict:
        info = _RequestInfo()
        _check(lib().ntt_server_wait(self._h, rid, ctypes.byref(info), timeout_ms), "ntt_server_wait")
        return {"id": int(info.id), "status": int(info.status), "batched_with": int(info.batched_with),
                "t_submit": info.t_submit, "t_admit": info.t_admit, "t_launch": info.t_launch,
                "t_done": info.t_done, "bytes": int(info.bytes), "launch_id": int(info.launch_id)}

    def counters(self) -> dict:
        c = _ServerCounters()
        _check(lib().ntt_server_counters_get(self._h, ctypes.byref(c)), "ntt_server_counters_get")
        return {n: int(getattr(c, n)) for n, _ in _ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ntt_server_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_uint64),
                ("words", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


def debug_wait_limit(polls: int = 0, force_expire: bool = False) -> None:
    """Testing aid: poll bound of the single-launch form's waits (0 = default)
    and whether every such wait is made to give up (reported as NTT_ETIMEOUT)."""
    _check(lib().ntt_debug_wait_limit(int(polls), 1 if force_expire else 0), "ntt_debug_wait_limit")


def stats_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events on its own stream."""
    _check(lib().ntt_stats_enable(1 if on else 0), "ntt_stats_enable")


def stats_reset() -> None:
    _check(lib().ntt_stats_reset(), "ntt_stats_reset")


def stats_collect() -> dict:
    """{kernel name: {"launches", "words", "total_ms", "avg_ms"}} since the last reset."""
    n = _u32()
    _check(lib().ntt_stats_collect(None, 0, ctypes.byref(n)), "ntt_stats_collect")
    arr = (KernelStat * max(1, n.value))()
    _check(lib().ntt_stats_collect(ctypes.cast(arr, _vp), n.value, ctypes.byref(n)), "ntt_stats_collect")
    out = {}
    for i in range(n.value):
        s = arr[i]
        out[s.name.decode()] = {"launches": int(s.launches), "words": int(s.words),
                                "total_ms": float(s.total_ms),
                                "avg_ms": float(s.total_ms) / max(1, int(s.launches))}
    return out


def lib():
    """Load libntt.so once; raise loudly when it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                                   "`python -c 'import __graft_entry__ as g; g.build()'`")
            L = ctypes.CDLL(_LIB_PATH)
            for name, args in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = ctypes.c_int
            L.ntt_last_error.restype = ctypes.c_char_p
            L.ntt_last_error.argtypes = []
            L.ntt_version.restype = ctypes.c_char_p
            L.ntt_version.argtypes = []
            _lib = L
    return _lib


def _check(st: int, where: str) -> None:
    if st != 0:
        msg = lib().ntt_last_error().decode(errors="replace")
        raise NTTError(st, where, msg)


def check_modulus(N: int, q: int, word_bits: int) -> int:
    """Status code a plan would report for (N, q, word_bits); 0 = admissible."""
    return int(lib().ntt_check_modulus(N, q, word_bits))


def find_root(N: int, q: int) -> int:
    out = _u64()
    _check(lib().ntt_find_root(N, q, ctypes.byref(out)), "ntt_find_root")
    return int(out.value)


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """An NTT plan: length N, RNS moduli, word width; owns device twiddle tables.

    Tensors passed to the methods are contiguous CUDA (HIP) tensors of shape
    [batch, L, N] (or anything with batch*L*N elements) whose element size
    equals word_bits/8; torch.int64 / torch.int32 tensors hold the uint64 /
    uint32 words bit for bit.
    """

    def __init__(self, N: int, moduli, word_bits: int = 64, flags: int = 0):
        self.N = int(N)
        self.moduli = [int(q) for q in moduli]
        self.L = len(self.moduli)
        self.word_bits = int(word_bits)
        arr = (_u64 * self.L)(*self.moduli)
        h = _vp()
        _check(lib().ntt_plan_create(ctypes.byref(h), self.N, arr, self.L, self.word_bits, flags),
               "ntt_plan_create")
        self._h = h

    # -- queries -------------------------------------------------------------
    def root(self, limb: int) -> int:
        out = _u64()
        _check(lib().ntt_plan_root(self._h, limb, ctypes.byref(out)), "ntt_plan_root")
        return int(out.value)

    @property
    def split(self) -> int:
        out = _u32()
        _check(lib().ntt_plan_split(self._h, ctypes.byref(out)), "ntt_plan_split")
        return int(out.value)

    def limb_class(self, limb: int) -> int:
        out = _u32()
        _check(lib().ntt_plan_limb_class(self._h, limb, ctypes.byref(out)), "ntt_plan_limb_class")
        return int(out.value)

    def split_for(self, batch: int) -> int:
        out = _u32()
        _check(lib().ntt_plan_split_for(self._h, batch, ctypes.byref(out)), "ntt_plan_split_for")
        return int(out.value)

    @property
    def handle(self) -> int:
        return int(self._h.value)

    # -- helpers -------------------------------------------------------------
    def _batch_of(self, t, name: str) -> int:
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.element_size() * 8 != self.word_bits:
            raise ValueError(f"{name} element size {t.element_size()} does not match word_bits {self.word_bits}")
        per = self.L * self.N
        if t.numel() == 0 or t.numel() % per:
            raise ValueError(f"{name} has {t.numel()} elements, not a multiple of L*N={per}")
        return t.numel() // per

    # -- operations ----------------------------------------------------------
    def forward(self, x, stream=None):
        """In-place forward NTT of x[batch][L][N]; returns x."""
        b = self._batch_of(x, "x")
        _check(lib().ntt_forward(self._h, x.data_ptr(), b, _stream_handle(stream)), "ntt_forward")
        return x

    def inverse(self, x, stream=None):
        b = self._batch_of(x, "x")
        _check(lib().ntt_inverse(self._h, x.data_ptr(), b, _stream_handle(stream)), "ntt_inverse")
        return x

    def pointwise_mul(self, out, a, b, stream=None):
        n = self._batch_of(out, "out")
        if self._batch_of(a, "a") != n or self._batch_of(b, "b") != n:
            raise ValueError("batch mismatch")
        _check(lib().ntt_pointwise_mul(self._h, out.data_ptr(), a.data_ptr(), b.data_ptr(), n,
                                       _stream_handle(stream)), "ntt_pointwise_mul")
        return out

    def mac(self, out, a, key, rows: int, cols: int, stream=None):
        P = self._batch_of(a, "a")
        groups = (P + rows - 1) // rows
        if self._batch_of(key, "key") != rows * cols:
            raise ValueError("key must hold rows*cols polynomials")
        if self._batch_of(out, "out") != groups * cols:
            raise ValueError("out must hold ceil(P/rows)*cols polynomials")
        _check(lib().ntt_mac(self._h, out.data_ptr(), a.data_ptr(), key.data_ptr(), rows, cols, P,
                             _stream_handle(stream)), "ntt_mac")
        return out

    def pointwise_mac(self, acc, a, key, rows: int, cols: int, groups: int, batch_tail: int = 0,
                      stream=None):
        """acc[g][c] = sum_r a[g*rows + r] (.) key[r][c] for g < groups; the last group
        holds batch_tail operands (0 = rows)."""
        P = self._batch_of(a, "a")
        want = (groups - 1) * rows + (batch_tail or rows)
        if P != want:
            raise ValueError(f"a holds {P} operands, groups/rows/batch_tail say {want}")
        if self._batch_of(key, "key") != rows * cols:
            raise ValueError("key must hold rows*cols polynomials")
        if self._batch_of(acc, "acc") != groups * cols:
            raise ValueError("acc must hold groups*cols polynomials")
        _check(lib().ntt_pointwise_mac(self._h, acc.data_ptr(), a.data_ptr(), key.data_ptr(), rows,
                                       cols, groups, batch_tail, _stream_handle(stream)),
               "ntt_pointwise_mac")
        return acc

    def external_product(self, out, a, key, rows: int, cols: int, stream=None):
        """out[g][c] = INTT(sum_r NTT(a[g*rows + r]) (.) key[r][c]); a is not modified."""
        P = self._batch_of(a, "a")
        groups = (P + rows - 1) // rows
        if self._batch_of(key, "key") != rows * cols:
            raise ValueError("key must hold rows*cols polynomials")
        if self._batch_of(out, "out") != groups * cols:
            raise ValueError("out must hold ceil(P/rows)*cols polynomials")
        _check(lib().ntt_external_product(self._h, out.data_ptr(), a.data_ptr(), key.data_ptr(),
                                          rows, cols, P, _stream_handle(stream)),
               "ntt_external_product")
        return out

    def external_product_decomposed(self, out, ct, key, levels: int, log_base: int, stream=None):
        """out[g][col] = INTT(sum_r NTT(digit row r of ct[g]) (.) key[r][col]) with
        ct [num_ct][comps][L][N], key [comps*levels][cols][L][N], out [num_ct][cols][L][N]."""
        if ct.dim() != 4 or key.dim() != 4 or out.dim() != 4:
            raise ValueError("ct, key and out are [count][rows][L][N]")
        num_ct, comps = int(ct.shape[0]), int(ct.shape[1])
        cols = int(key.shape[1])
        if int(key.shape[0]) != comps * levels:
            raise ValueError("key must have comps*levels rows")
        if tuple(out.shape[:2]) != (num_ct, cols):
            raise ValueError("out must be [num_ct][cols][L][N]")
        for t, name in ((ct, "ct"), (key, "key"), (out, "out")):
            self._batch_of(t, name)
        _check(lib().ntt_external_product_decomposed(self._h, out.data_ptr(), ct.data_ptr(),
                                                     key.data_ptr(), num_ct, comps, levels,
                                                     log_base, cols, _stream_handle(stream)),
               "ntt_external_product_decomposed")
        return out

    def cmux(self, out, acc, rot, key, levels: int, log_base: int, stream=None):
        """out[g] = acc[g] + ExtProd(key, X^rot[g] acc[g] - acc[g]); acc/out
        [num_ct][comps][L][N], rot a device uint32 (int32) tensor of num_ct amounts,
        key [comps*levels][comps][L][N] in the transform domain."""
        if acc.dim() != 4 or key.dim() != 4 or out.shape != acc.shape:
            raise ValueError("acc/out are [num_ct][comps][L][N], key [comps*levels][comps][L][N]")
        num_ct, comps = int(acc.shape[0]), int(acc.shape[1])
        if tuple(key.shape[:2]) != (comps * levels, comps):
            raise ValueError("key must be [comps*levels][comps][L][N]")
        if not rot.is_cuda or rot.element_size() != 4 or rot.numel() != num_ct or not rot.is_contiguous():
            raise ValueError("rot must be a contiguous device tensor of num_ct 32-bit amounts")
        for t, name in ((acc, "acc"), (key, "key"), (out, "out")):
            self._batch_of(t, name)
        _check(lib().ntt_cmux(self._h, out.data_ptr(), acc.data_ptr(), rot.data_ptr(),
                              key.data_ptr(), num_ct, comps, levels, log_base,
                              _stream_handle(stream)), "ntt_cmux")
        return out

    def automorph(self, out, a, k: int, transformed: bool = False, stream=None):
        """out = sigma_k(a): a(x) -> a(x^k) per limb, k odd < 2N; coefficient domain,
        or the forward transform's slot order with transformed=True (out must not
        overlap a)."""
        n = self._batch_of(a, "a")
        if self._batch_of(out, "out") != n:
            raise ValueError("batch mismatch")
        _check(lib().ntt_automorph(self._h, out.data_ptr(), a.data_ptr(), n, int(k),
                                   AUTOMORPH_TRANSFORMED if transformed else 0,
                                   _stream_handle(stream)), "ntt_automorph")
        return out

    def forward_mul(self, out, a, b, stream=None):
        """Forward NTT of a and b in place and out = a (.) b, in one pass over the rows."""
        n = self._batch_of(out, "out")
        if self._batch_of(a, "a") != n or self._batch_of(b, "b") != n:
            raise ValueError("batch mismatch")
        _check(lib().ntt_forward_mul(self._h, out.data_ptr(), a.data_ptr(), b.data_ptr(), n,
                                     _stream_handle(stream)), "ntt_forward_mul")
        return out

    def polymul(self, out, a, b, stream=None):
        n = self._batch_of(out, "out")
        if self._batch_of(a, "a") != n or self._batch_of(b, "b") != n:
            raise ValueError("batch mismatch")
        _check(lib().ntt_polymul(self._h, out.data_ptr(), a.data_ptr(), b.data_ptr(), n,
                                 _stream_handle(stream)), "ntt_polymul")
        return out

    def polymul_noalloc(self, out, a, b, stream=None):
        """polymul with the library's fixed per-GPU scratch instead of a pool allocation."""
        n = self._batch_of(out, "out")
        if self._batch_of(a, "a") != n or self._batch_of(b, "b") != n:
            raise ValueError("batch mismatch")
        _check(lib().ntt_polymul_noalloc(self._h, out.data_ptr(), a.data_ptr(), b.data_ptr(), n,
                                         _stream_handle(stream)), "ntt_polymul_noalloc")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ntt_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
