"""Thin ctypes binding of libsnp (include/snp.h) with the same entry-point names.

Only argument marshalling happens here: host arrays of a system description
are passed as-is, device buffers are torch CUDA tensors whose ``data_ptr()``
is handed to the library, and the handle launches on the torch stream given at
load.  Every step of the computation runs in the library's HIP kernels; when
the library is not built, loading fails with an error instead of falling back.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import library_path

SNP_OK, SNP_ERR_INVALID, SNP_ERR_OVERFLOW, SNP_ERR_CAPACITY, SNP_ERR_BUDGET, SNP_ERR_DEVICE = range(6)
SNP_COUNT_I32, SNP_COUNT_U16 = 0, 1
SNP_PATH_AUTO, SNP_PATH_SPARSE, SNP_PATH_INT8 = 0, 1, 2
STOP_NAMES = {0: "EMPTY_FRONTIER", 1: "ALL_HALTING", 2: "DEPTH", 3: "CAP", 4: "BUDGET"}
SNP_STOP_EMPTY_FRONTIER, SNP_STOP_ALL_HALTING, SNP_STOP_DEPTH, SNP_STOP_CAP, SNP_STOP_BUDGET = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "OVERFLOW", 3: "CAPACITY", 4: "BUDGET", 5: "DEVICE"}

EXPORTED = ("snp_load", "snp_free", "snp_last_error", "snp_row_bytes", "snp_reset", "snp_expand", "snp_run",
            "snp_batch_load", "snp_batch_free", "snp_batch_offsets", "snp_batch_shape", "snp_batch_run",
            "snp_batch_run_static", "snp_get_tuning", "snp_set_tuning", "snp_autotune", "snp_load_tuning",
            "snp_run_batch")


class SnpError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class snp_desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("r", ctypes.c_int32),
        ("rule_neuron", ctypes.c_void_p), ("rule_i", ctypes.c_void_p), ("rule_j", ctypes.c_void_p),
        ("rule_c", ctypes.c_void_p), ("rule_p", ctypes.c_void_p),
        ("n_syn", ctypes.c_int32), ("syn_src", ctypes.c_void_p), ("syn_dst", ctypes.c_void_p),
        ("M", ctypes.c_void_p), ("count_type", ctypes.c_int32), ("rule_d", ctypes.c_void_p),
    ]


class snp_options(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int32), ("stop_at_cap", ctypes.c_int32),
        ("frontier_cap", ctypes.c_int64), ("child_budget", ctypes.c_int64),
        ("expand_max_count", ctypes.c_int64), ("max_rows", ctypes.c_int64),
        ("max_frontier", ctypes.c_int64), ("chunk", ctypes.c_int64),
        ("hash_mask", ctypes.c_uint64), ("profile", ctypes.c_int32), ("int8_max_k", ctypes.c_int32),
        ("deterministic", ctypes.c_int32), ("out_neuron", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("stage_rows", ctypes.c_int32),
    ]


class snp_tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int64), ("int8_tiles", ctypes.c_int32), ("sparse_run", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class snp_expand_stats(ctypes.Structure):
    _fields_ = [
        ("parents", ctypes.c_int64), ("halting_parents", ctypes.c_int64),
        ("children_total", ctypes.c_int64), ("enumerated", ctypes.c_int64),
        ("new_configs", ctypes.c_int64), ("duplicates", ctypes.c_int64), ("expanded", ctypes.c_int64),
        ("twins", ctypes.c_int64), ("collisions", ctypes.c_int64), ("chunks", ctypes.c_int64),
        ("int8_chunks", ctypes.c_int64),
        ("mfma_ops", ctypes.c_int64),
        ("truncated", ctypes.c_int32), ("budget_hit", ctypes.c_int32),
        ("path_used", ctypes.c_int32), ("int8_fallback", ctypes.c_int32),
        ("ns_psi", ctypes.c_int64), ("ns_expand", ctypes.c_int64), ("ns_insert", ctypes.c_int64),
        ("ns_flags", ctypes.c_int64), ("ns_commit", ctypes.c_int64), ("redone", ctypes.c_int64),
        ("keys_first", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


# the same layout as a numpy record, to read many entries at once
_STATS_NAMES = tuple(name for name, _ in snp_expand_stats._fields_)
_STATS_DTYPE = np.dtype([(name, np.int64 if ct is ctypes.c_int64 else np.int32)
                         for name, ct in snp_expand_stats._fields_], align=True)
assert _STATS_DTYPE.itemsize == ctypes.sizeof(snp_expand_stats)


def _stats_list(stats, n: int) -> list:
    return [dict(zip(_STATS_NAMES, row)) for row in np.frombuffer(stats, dtype=_STATS_DTYPE, count=n).tolist()]


_lib = None


def lib():
    """Load libsnp.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise FileNotFoundError(
                f"{path} is missing: build it with __graft_entry__.build() or "
                "python -m paper_1104_1824_amd.build")
        L = ctypes.CDLL(path)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.snp_load.argtypes = [ctypes.POINTER(snp_desc), ctypes.POINTER(snp_options), ctypes.POINTER(P)]
        L.snp_load.restype = I32
        L.snp_free.argtypes = [P]
        L.snp_free.restype = None
        L.snp_last_error.argtypes = []
        L.snp_last_error.restype = ctypes.c_char_p
        L.snp_row_bytes.argtypes = [P]
        L.snp_row_bytes.restype = I64
        L.snp_reset.argtypes = [P, P]
        L.snp_reset.restype = I32
        L.snp_expand.argtypes = [P, P, I64, P, I64, ctypes.POINTER(I64), P, P, ctypes.POINTER(snp_expand_stats)]
        L.snp_expand.restype = I32
        L.snp_run.argtypes = [P, P, I32, P, I64, ctypes.POINTER(I64), P, I32, ctypes.POINTER(I32),
                              ctypes.POINTER(I32), P, P, P]
        L.snp_run.restype = I32
        L.snp_batch_load.argtypes = [ctypes.POINTER(snp_desc), I32, ctypes.POINTER(snp_options), ctypes.POINTER(P)]
        L.snp_batch_load.restype = I32
        L.snp_batch_free.argtypes = [P]
        L.snp_batch_free.restype = None
        L.snp_batch_offsets.argtypes = [P, P]
        L.snp_batch_offsets.restype = I32
        L.snp_batch_shape.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.snp_batch_shape.restype = I32
        L.snp_batch_run.argtypes = [P, P, I32, I32, P, P, P, P, P]
        L.snp_batch_run.restype = I32
        L.snp_batch_run_static.argtypes = [P, P, I32, I32, P, P, P, P, P]
        L.snp_batch_run_static.restype = I32
        TP = ctypes.POINTER(snp_tuning)
        L.snp_get_tuning.argtypes = [P, TP]
        L.snp_get_tuning.restype = I32
        L.snp_set_tuning.argtypes = [P, TP]
        L.snp_set_tuning.restype = I32
        L.snp_autotune.argtypes = [P, P, I32, P, I64, ctypes.c_char_p, TP, ctypes.POINTER(ctypes.c_double)]
        L.snp_autotune.restype = I32
        L.snp_load_tuning.argtypes = [P, ctypes.c_char_p, I32, ctypes.POINTER(I32)]
        L.snp_load_tuning.restype = I32
        L.snp_run_batch.argtypes = [P, I32, P, I32, P, P, P, P]
        L.snp_run_batch.restype = I32
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != SNP_OK:
        raise SnpError(status, where, lib().snp_last_error().decode())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def check_buffer(t, name: str, elem_bytes: int, min_elems: int):
    """Host-side check of a buffer handed to the library: contiguous, elements of
    the size the library reads or writes, and at least min_elems of them (the
    kernels would otherwise run past the allocation)."""
    if not t.is_contiguous():
        raise ValueError(f"{name}: device buffers must be contiguous")
    if t.element_size() != elem_bytes:
        raise ValueError(f"{name}: elements of {t.element_size()} bytes, the library uses {elem_bytes}")
    if t.numel() < min_elems:
        raise ValueError(f"{name}: {t.numel()} elements, at least {min_elems} needed")


def _ptr(t, name: str = "buffer", elem_bytes: Optional[int] = None, min_elems: int = 0) -> Optional[int]:
    """Device pointer of a torch tensor (None stays None), after checking that it
    lives on the GPU and (when elem_bytes is given) its element size and length."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name}: the library takes GPU (HIP) tensors, got one on {getattr(t, 'device', '?')}")
    if elem_bytes is None:
        if not t.is_contiguous():
            raise ValueError(f"{name}: device buffers must be contiguous")
    else:
        check_buffer(t, name, elem_bytes, min_elems)
    return t.data_ptr()


def _eb(count_type: int) -> int:
    return 2 if count_type == SNP_COUNT_U16 else 4


class _RunBuffers:
    """Host outputs of snp_run with their addresses taken once."""

    def __init__(self, max_levels: int):
        self.max_levels = max_levels
        self.sizes = np.zeros(max_levels, dtype=np.int64)
        self.stats = (snp_expand_stats * max_levels)()
        self.n_configs, self.n_levels, self.stop = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int32(0)
        self.p_sizes = self.sizes.ctypes.data
        self.p_stats = ctypes.addressof(self.stats)
        self.r_configs = ctypes.byref(self.n_configs)
        self.r_levels = ctypes.byref(self.n_levels)
        self.r_stop = ctypes.byref(self.stop)


class Handle:
    """A loaded system (snp_system*); freed by close() or garbage collection."""

    def __init__(self, ptr: int, keep, m: int, count_type: int):
        self.ptr = ctypes.c_void_p(ptr)
        self._keep = keep
        self.m = m
        self.count_type = count_type
        self._run = None  # output buffers of snp_run, reused while max_levels stays

    def run_buffers(self, max_levels: int) -> "_RunBuffers":
        if self._run is None or self._run.max_levels != max_levels:
            self._run = _RunBuffers(max_levels)
        return self._run

    def close(self):
        if self.ptr:
            lib().snp_free(self.ptr)
            self.ptr = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _desc(system, keep, M=None) -> snp_desc:
    arrs = [_i32(system.rule_neuron), _i32(system.rule_i), _i32(system.rule_j), _i32(system.rule_c),
            _i32(system.rule_p), _i32(system.syn_src), _i32(system.syn_dst)]
    Mp = _i32(M) if M is not None else None
    keep.extend(arrs)
    if Mp is not None:
        keep.append(Mp)
    ct = SNP_COUNT_U16 if getattr(system, "count_type", "i32") == "u16" else SNP_COUNT_I32
    rd = getattr(system, "rule_d", None)
    rd = _i32(rd) if rd is not None else None
    if rd is not None:
        keep.append(rd)
    return snp_desc(int(system.m), int(arrs[0].shape[0]), arrs[0].ctypes.data, arrs[1].ctypes.data,
                    arrs[2].ctypes.data, arrs[3].ctypes.data, arrs[4].ctypes.data, int(arrs[5].shape[0]),
                    arrs[5].ctypes.data, arrs[6].ctypes.data, Mp.ctypes.data if Mp is not None else None, ct,
                    rd.ctypes.data if rd is not None else None)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream() if torch.cuda.is_available() else 0
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)


def snp_load(system, *, path: int = SNP_PATH_AUTO, stop_at_cap: bool = False, frontier_cap: int = 0,
             child_budget: int = 0, expand_max_count: int = -1, max_rows: int = 1 << 20,
             max_frontier: int = 0, chunk: int = 0, hash_mask: int = 0, profile: int = 0,
             int8_max_k: int = 0, deterministic: bool = False, out_neuron: int = 0, stream=None,
             M: Optional[np.ndarray] = None, stage_rows: int = 0) -> Handle:
    """snp_load.  ``system`` has m, rule_neuron/i/j/c/p, syn_src/dst and
    count_type ("i32" or "u16") attributes; ``stream`` is a torch.cuda.Stream
    (None: torch's current stream).  With ``out_neuron`` > 0 (1-based) rows
    hold m + 2 entries (the output neuron's spike train after the counts);
    a system with ``rule_d`` (delays) adds (wait, pend) per neuron owning a
    rule with a delay.  ``Handle.m`` is the row width the library reports."""
    arrs = []
    d = _desc(system, arrs, M)
    ct = d.count_type
    sp = _stream_ptr(stream)
    o = snp_options(int(path), int(bool(stop_at_cap)), int(frontier_cap), int(child_budget),
                    int(expand_max_count), int(max_rows), int(max_frontier), int(chunk),
                    int(hash_mask) & ((1 << 64) - 1), int(profile), int(int8_max_k), int(bool(deterministic)),
                    int(out_neuron), sp or None, int(stage_rows))
    out = ctypes.c_void_p()
    _check(lib().snp_load(ctypes.byref(d), ctypes.byref(o), ctypes.byref(out)), "snp_load")
    h = Handle(out.value, arrs, 0, ct)
    h.m = int(lib().snp_row_bytes(h.ptr)) // _eb(ct)
    return h


def snp_free(h: Handle):
    h.close()


def snp_row_bytes(h: Handle) -> int:
    return int(lib().snp_row_bytes(h.ptr))


def snp_reset(h: Handle, c0_dev):
    _check(lib().snp_reset(h.ptr, _ptr(c0_dev, "c0", _eb(h.count_type), h.m)), "snp_reset")


def snp_expand(h: Handle, frontier_dev, n: int, next_dev, next_capacity: int, parent_of_next=None,
               child_of_next=None):
    """Returns (n_next, stats dict)."""
    n_next = ctypes.c_int64(0)
    st = snp_expand_stats()
    eb, n, cap = _eb(h.count_type), int(n), int(next_capacity)
    status = lib().snp_expand(h.ptr, _ptr(frontier_dev, "frontier", eb, n * h.m), n,
                              _ptr(next_dev, "next", eb, cap * h.m), cap, ctypes.byref(n_next),
                              _ptr(parent_of_next, "parent_of_next", 8, cap),
                              _ptr(child_of_next, "child_of_next", 8, cap), ctypes.byref(st))
    if status != SNP_OK:
        err = SnpError(status, "snp_expand", lib().snp_last_error().decode())
        err.n_next = int(n_next.value)
        raise err
    return int(n_next.value), st.as_dict()


def snp_run(h: Handle, c0_dev, max_depth: int, out_dev, out_capacity: int, max_levels: int = 4096,
            parent_of=None, child_of=None, with_stats: bool = True) -> dict:
    """Returns dict(n_configs, level_sizes, stop_reason, level_stats)."""
    rb = h.run_buffers(max_levels)
    eb, cap = _eb(h.count_type), int(out_capacity)
    status = lib().snp_run(h.ptr, _ptr(c0_dev, "c0", eb, h.m), int(max_depth), _ptr(out_dev, "out", eb, cap * h.m),
                           cap, rb.r_configs, rb.p_sizes, int(max_levels), rb.r_levels, rb.r_stop,
                           rb.p_stats if with_stats else None, _ptr(parent_of, "parent_of", 8, cap),
                           _ptr(child_of, "child_of", 8, cap))
    if status != SNP_OK:
        err = SnpError(status, "snp_run", lib().snp_last_error().decode())
        err.n_configs = int(rb.n_configs.value)
        raise err
    L = int(rb.n_levels.value)
    return dict(
        n_configs=int(rb.n_configs.value),
        level_sizes=rb.sizes[:L].copy(),
        stop_reason=int(rb.stop.value),
        level_stats=_stats_list(rb.stats, L) if with_stats else None,
    )


def snp_get_tuning(h: Handle) -> dict:
    tu = snp_tuning()
    _check(lib().snp_get_tuning(h.ptr, ctypes.byref(tu)), "snp_get_tuning")
    return tu.as_dict()


def snp_set_tuning(h: Handle, chunk: int = 0, int8_tiles: int = 0, sparse_run: int = 0):
    tu = snp_tuning(int(chunk), int(int8_tiles), int(sparse_run))
    _check(lib().snp_set_tuning(h.ptr, ctypes.byref(tu)), "snp_set_tuning")


def snp_autotune(h: Handle, c0_dev, max_depth: int, out_dev, out_capacity: int,
                 cache_path: Optional[str] = None) -> dict:
    """snp_autotune; returns the settings applied plus their walk time "ms"."""
    eb = _eb(h.count_type)
    tu = snp_tuning()
    ms = ctypes.c_double()
    _check(lib().snp_autotune(h.ptr, _ptr(c0_dev, "c0", eb, h.m), int(max_depth),
                              _ptr(out_dev, "out", eb, int(out_capacity) * h.m), int(out_capacity),
                              cache_path.encode() if cache_path else None, ctypes.byref(tu), ctypes.byref(ms)),
           "snp_autotune")
    return dict(tu.as_dict(), ms=float(ms.value))


def snp_load_tuning(h: Handle, cache_path: str, max_depth: int) -> bool:
    found = ctypes.c_int32()
    _check(lib().snp_load_tuning(h.ptr, cache_path.encode(), int(max_depth), ctypes.byref(found)),
           "snp_load_tuning")
    return bool(found.value)


def torch_dtype(count_type: int):
    import torch
    return torch.uint16 if count_type == SNP_COUNT_U16 else torch.int32


class BatchHandle:
    """A loaded batch of systems (snp_batch*)."""

    def __init__(self, ptr: int, keep, n: int, count_type: int):
        self.ptr = ctypes.c_void_p(ptr)
        self._keep = keep
        self.n = n
        self.count_type = count_type
        self.total = None  # elements of the packed rows, read on first use

    def close(self):
        if self.ptr:
            lib().snp_batch_free(self.ptr)
            self.ptr = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def snp_batch_load(systems, stream=None, threads: int = 0) -> BatchHandle:
    """snp_batch_load; ``threads`` (256, 512 or 1024) fixes the threads per
    system, 0 lets the first run pick the fastest shape."""
    keep = []
    descs = (snp_desc * len(systems))(*[_desc(s, keep) for s in systems])
    o = snp_options()
    o.max_rows = 1
    o.chunk = int(threads)
    o.stream = _stream_ptr(stream) or None
    out = ctypes.c_void_p()
    _check(lib().snp_batch_load(descs, len(systems), ctypes.byref(o), ctypes.byref(out)), "snp_batch_load")
    return BatchHandle(out.value, (keep, descs), len(systems), int(descs[0].count_type))


def snp_batch_free(b: BatchHandle):
    b.close()


def snp_batch_offsets(b: BatchHandle) -> np.ndarray:
    off = np.zeros(b.n + 1, dtype=np.int64)
    _check(lib().snp_batch_offsets(b.ptr, off.ctypes.data), "snp_batch_offsets")
    return off


def snp_batch_shape(b: BatchHandle):
    """(threads per system, neurons per thread) in use; (0, 0) before the first run."""
    th, npt = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().snp_batch_shape(b.ptr, ctypes.byref(th), ctypes.byref(npt)), "snp_batch_shape")
    return th.value, npt.value


def snp_batch_run(b: BatchHandle, c0_dev, steps: int, final_dev, detect_repeats: bool = True) -> dict:
    """Returns dict of numpy arrays: halt_step, first_repeat, steps_done, digest."""
    n = b.n
    if b.total is None:
        b.total = int(snp_batch_offsets(b)[-1])
    eb = _eb(b.count_type)
    halt = np.zeros(n, dtype=np.int32)
    rep = np.zeros(n, dtype=np.int32)
    done = np.zeros(n, dtype=np.int32)
    dig = np.zeros(n, dtype=np.uint64)
    _check(lib().snp_batch_run(b.ptr, _ptr(c0_dev, "c0", eb, b.total), int(steps), int(bool(detect_repeats)),
                               _ptr(final_dev, "final", eb, b.total), halt.ctypes.data, rep.ctypes.data,
                               done.ctypes.data, dig.ctypes.data),
           "snp_batch_run")
    return dict(halt_step=halt, first_repeat=rep, steps_done=done, digest=dig)


def snp_batch_run_static(b: BatchHandle, c0_dev, steps: int, final_dev, detect_repeats: bool = True) -> dict:
    """snp_batch_run with the library's static scratch (no device allocation).
    Returns dict of numpy arrays: halt_step, first_repeat, steps_done, digest."""
    n = b.n
    if b.total is None:
        b.total = int(snp_batch_offsets(b)[-1])
    eb = _eb(b.count_type)
    halt = np.zeros(n, dtype=np.int32)
    rep = np.zeros(n, dtype=np.int32)
    done = np.zeros(n, dtype=np.int32)
    dig = np.zeros(n, dtype=np.uint64)
    _check(lib().snp_batch_run_static(b.ptr, _ptr(c0_dev, "c0", eb, b.total), int(steps), int(bool(detect_repeats)),
                                      _ptr(final_dev, "final", eb, b.total), halt.ctypes.data, rep.ctypes.data,
                                      done.ctypes.data, dig.ctypes.data),
           "snp_batch_run_static")
    return dict(halt_step=halt, first_repeat=rep, steps_done=done, digest=dig)


def snp_run_batch(handles, c0_list, steps: int, final_list) -> dict:
    """snp_run_batch over handles from snp_load: one row per system in c0_list
    and final_list (torch GPU tensors).  Returns dict of numpy arrays:
    halt_step, first_repeat, digest."""
    n = len(handles)
    if len(c0_list) != n or len(final_list) != n:
        raise ValueError("snp_run_batch: one c0 and one final buffer per handle")
    hp = (ctypes.c_void_p * n)(*[h.ptr.value for h in handles])
    cp = (ctypes.c_void_p * n)(*[_ptr(c, f"c0[{k}]", _eb(h.count_type), h.m)
                                 for k, (h, c) in enumerate(zip(handles, c0_list))])
    fp = (ctypes.c_void_p * n)(*[_ptr(f, f"final[{k}]", _eb(h.count_type), h.m)
                                 for k, (h, f) in enumerate(zip(handles, final_list))])
    halt = np.zeros(n, dtype=np.int32)
    rep = np.zeros(n, dtype=np.int32)
    dig = np.zeros(n, dtype=np.uint64)
    _check(lib().snp_run_batch(hp, n, cp, int(steps), fp, halt.ctypes.data, rep.ctypes.data, dig.ctypes.data),
           "snp_run_batch")
    return dict(halt_step=halt, first_repeat=rep, digest=dig)
