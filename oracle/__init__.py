"""Plain CPU oracle for the BFS expansion of an SN P system's computation tree.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg use it.  The simulator package never imports
it, and it imports nothing of the simulator.

``snp_oracle.c`` holds the arithmetic (Definition 2, rule applicability,
Algorithm 2 enumeration, Equation next-config, Algorithm 1 walk, the
deterministic single-branch run); this module only marshals arguments.
``alg2`` restates Algorithm 2 with the paper's own string lists for the
worked-example pins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libsnp_oracle.so")

OK, ERR_INVALID, ERR_OVERFLOW, ERR_CAPACITY, ERR_NOMEM = 0, 1, 2, 3, 5
STOP_EMPTY_FRONTIER, STOP_ALL_HALTING, STOP_DEPTH, STOP_CAP, STOP_BUDGET = 0, 1, 2, 3, 4
STOP_NAMES = {0: "EMPTY_FRONTIER", 1: "ALL_HALTING", 2: "DEPTH", 3: "CAP", 4: "BUDGET"}


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (single-threaded, -O2)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _System(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("r", ctypes.c_int32), ("n_syn", ctypes.c_int32),
        ("rule_neuron", ctypes.c_void_p), ("rule_i", ctypes.c_void_p), ("rule_j", ctypes.c_void_p),
        ("rule_c", ctypes.c_void_p), ("rule_p", ctypes.c_void_p),
        ("syn_src", ctypes.c_void_p), ("syn_dst", ctypes.c_void_p),
        ("count_max", ctypes.c_int64), ("rule_d", ctypes.c_void_p),
    ]


class _BfsOpts(ctypes.Structure):
    _fields_ = [
        ("max_depth", ctypes.c_int32), ("stop_at_cap", ctypes.c_int32),
        ("frontier_cap", ctypes.c_int64), ("child_budget", ctypes.c_int64),
        ("expand_max_count", ctypes.c_int64), ("first_only", ctypes.c_int32), ("out_neuron", ctypes.c_int32),
    ]


class _BfsResult(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_void_p), ("rows_cap", ctypes.c_int64),
        ("parent", ctypes.c_void_p), ("tindex", ctypes.c_void_p),
        ("level_sizes", ctypes.c_void_p), ("enumerated", ctypes.c_void_p),
        ("halting", ctypes.c_void_p), ("max_levels", ctypes.c_int32),
        ("n_levels", ctypes.c_int32), ("stop_reason", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("n_configs", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.or_matrix_dense.argtypes = [ctypes.POINTER(_System), P]
        lib.or_applicable.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.or_children.argtypes = [ctypes.POINTER(_System), P, ctypes.c_int64, P, P, P]
        lib.or_bfs.argtypes = [ctypes.POINTER(_System), P, ctypes.POINTER(_BfsOpts), ctypes.POINTER(_BfsResult)]
        lib.or_deterministic.argtypes = [ctypes.POINTER(_System), P, ctypes.c_int32, P, P, P, P, P]
        lib.or_child_at.argtypes = [ctypes.POINTER(_System), P, ctypes.c_int64, P]
        lib.or_mix64.argtypes = [ctypes.c_uint64]
        lib.or_mix64.restype = ctypes.c_uint64
        lib.or_config_hash.argtypes = [P, ctypes.c_int32]
        lib.or_config_hash.restype = ctypes.c_uint64
        lib.or_row_width.argtypes = [ctypes.POINTER(_System), ctypes.c_int32]
        lib.or_row_width.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


class _Sys:
    """Keeps the int32 arrays alive while the C struct points at them."""

    def __init__(self, sys):
        self.arrs = [_i32(sys.rule_neuron), _i32(sys.rule_i), _i32(sys.rule_j), _i32(sys.rule_c),
                     _i32(sys.rule_p), _i32(sys.syn_src), _i32(sys.syn_dst)]
        rd = getattr(sys, "rule_d", None)
        self.rule_d = None if rd is None else _i32(rd)
        a = self.arrs
        self.s = _System(int(sys.m), int(a[0].shape[0]), int(a[5].shape[0]),
                         a[0].ctypes.data, a[1].ctypes.data, a[2].ctypes.data, a[3].ctypes.data,
                         a[4].ctypes.data, a[5].ctypes.data, a[6].ctypes.data, int(sys.count_max),
                         None if self.rule_d is None else self.rule_d.ctypes.data)
        self.m, self.r = int(sys.m), int(a[0].shape[0])


def matrix_dense(sys) -> np.ndarray:
    """M_Pi of Definition 2 as an r x m int64 array."""
    S = _Sys(sys)
    M = np.zeros((S.r, S.m), dtype=np.int64)
    st = _load().or_matrix_dense(ctypes.byref(S.s), M.ctypes.data)
    if st:
        raise OracleError(st, "matrix_dense")
    return M


def applicable(n: int, i: int, j: int, c: int) -> bool:
    """a^n in L(a^i (a^j)*) and n >= c."""
    return bool(_load().or_applicable(int(n), int(i), int(j), int(c)))


def children(sys, C, max_out: int = 1 << 16):
    """Children of configuration C in Algorithm 2 order.

    Returns (rows [k, m] int64, spiking vectors [k, r] uint8, psi) where psi is
    the number of valid spiking vectors (0 for a halting configuration) and
    k = min(psi, max_out).
    """
    S = _Sys(sys)
    C = _i64(C)
    rows = np.zeros((max_out, S.m), dtype=np.int64)
    Sv = np.zeros((max_out, max(S.r, 1)), dtype=np.uint8)
    psi = ctypes.c_int64(0)
    st = _load().or_children(ctypes.byref(S.s), C.ctypes.data, max_out, rows.ctypes.data,
                             Sv.ctypes.data, ctypes.byref(psi))
    if st:
        raise OracleError(st, "children")
    k = min(psi.value, max_out)
    return rows[:k].copy(), Sv[:k, : S.r].copy(), psi.value


def child_at(sys, C, t: int) -> np.ndarray:
    """The child of C with index t in Algorithm 2 order."""
    S = _Sys(sys)
    C = _i64(C)
    out = np.zeros(S.m, dtype=np.int64)
    st = _load().or_child_at(ctypes.byref(S.s), C.ctypes.data, int(t), out.ctypes.data)
    if st:
        raise OracleError(st, "child_at")
    return out


def mix64(z: int) -> int:
    """The SplitMix64 output finaliser used by the trajectory digest."""
    return int(_load().or_mix64(int(z) & ((1 << 64) - 1)))


def config_hash(C) -> int:
    """H(C) = sum_n (uint32)C[n] * mix64((n + 1) * gamma) mod 2^64."""
    C = _i64(C)
    return int(_load().or_config_hash(C.ctypes.data, int(C.shape[0])))


@dataclass
class BfsResult:
    rows: np.ndarray          # [n_configs, m] int64, level by level
    level_sizes: np.ndarray   # [n_levels]
    parent: np.ndarray        # [n_configs] global index of the parent, -1 for C0
    tindex: np.ndarray        # [n_configs] index of the spiking vector among the parent's
    enumerated: np.ndarray    # [n_levels] children considered when expanding level k (0: not expanded)
    halting: np.ndarray       # [n_levels] parents of level k with no applicable rule, counted up to the
                              # parent of the last child enumerated (all of them unless cut by cap/budget)
    stop_reason: int

    @property
    def n_levels(self) -> int:
        return int(self.level_sizes.shape[0])

    def level(self, k: int) -> np.ndarray:
        off = int(self.level_sizes[:k].sum())
        return self.rows[off: off + int(self.level_sizes[k])]


def bfs(sys, c0=None, max_depth: int = -1, frontier_cap: int = 0, child_budget: int = 0,
        expand_max_count: int = -1, stop_at_cap: bool = False, rows_cap: int = 1 << 12,
        max_levels: int = 1 << 12, deterministic: bool = False, out_neuron: int = 0) -> BfsResult:
    """Algorithm 1 from C0: levels of new configurations in first-occurrence order.

    ``frontier_cap`` truncates every level to its first new configurations in
    enumeration order (truncated ones are not recorded); with ``stop_at_cap`` a
    level that reaches the cap also ends the walk.  ``deterministic`` keeps only
    the first spiking vector of every configuration (a single branch).
    ``out_neuron`` > 0 (1-based) follows that neuron's spikes to the
    environment: rows carry two more entries (spikes sent, at most 2 counted;
    steps from the first to the second), C0's being 0, 0 unless given.  A
    system with ``rule_d`` (delays) adds (wait, pend) per neuron owning a rule
    with a delay (``row_width``); a C0 of m entries starts them all open."""
    S = _Sys(sys)
    c0 = _i64(sys.c0 if c0 is None else c0)
    width = row_width(sys, out_neuron)
    if c0.shape[0] == S.m and width > S.m:
        c0 = np.concatenate([c0, np.zeros(width - S.m, dtype=np.int64)])
    if c0.shape[0] != width:
        raise ValueError(f"C0 has {c0.shape[0]} entries, rows have {width}")
    opts = _BfsOpts(int(max_depth), int(bool(stop_at_cap)), int(frontier_cap), int(child_budget),
                    int(expand_max_count), int(bool(deterministic)), int(out_neuron))
    cap = int(rows_cap)
    while True:
        rows = np.zeros((cap, width), dtype=np.int64)
        parent = np.zeros(cap, dtype=np.int64)
        tindex = np.zeros(cap, dtype=np.int64)
        lv = np.zeros(max_levels, dtype=np.int64)
        en = np.zeros(max_levels, dtype=np.int64)
        ha = np.zeros(max_levels, dtype=np.int64)
        res = _BfsResult(rows.ctypes.data, cap, parent.ctypes.data, tindex.ctypes.data,
                         lv.ctypes.data, en.ctypes.data, ha.ctypes.data, int(max_levels), 0, 0, 0, 0)
        st = _load().or_bfs(ctypes.byref(S.s), c0.ctypes.data, ctypes.byref(opts), ctypes.byref(res))
        if st == ERR_CAPACITY and cap < (1 << 31) and max_levels < (1 << 24):
            if res.n_configs >= cap or int(res.n_levels) < max_levels:
                cap *= 4
            else:
                max_levels *= 4
            continue
        if st:
            raise OracleError(st, "bfs")
        n, L = int(res.n_configs), int(res.n_levels)
        return BfsResult(rows[:n].copy(), lv[:L].copy(), parent[:n].copy(), tindex[:n].copy(),
                         en[:L].copy(), ha[:L].copy(), int(res.stop_reason))


def row_width(sys, out_neuron: int = 0) -> int:
    """Entries per row of a walk: the m counts, 2 for an output neuron's spike
    train, 2 (wait, pend) per neuron that owns a rule with a delay."""
    S = _Sys(sys)
    w = int(_load().or_row_width(ctypes.byref(S.s), int(out_neuron)))
    if w < 0:
        raise OracleError(ERR_NOMEM, "row_width")
    return w


def generated_numbers(res: BfsResult, m: int) -> list:
    """The numbers a walk with an output neuron generated: the steps between the
    output neuron's first two spikes, over every row whose train has both."""
    rows = res.rows
    return sorted({int(x) for x in rows[rows[:, m] >= 2, m + 1]})


@dataclass
class DetResult:
    final: np.ndarray
    halt_step: int
    first_repeat: int
    steps_done: int
    digest: int


def deterministic(sys, steps: int, c0=None) -> DetResult:
    """Single branch: every neuron fires its first applicable rule at every step."""
    S = _Sys(sys)
    c0 = _i64(sys.c0 if c0 is None else c0)
    final = np.zeros(S.m, dtype=np.int64)
    hs, fr, sd = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    dg = ctypes.c_uint64(0)
    st = _load().or_deterministic(ctypes.byref(S.s), c0.ctypes.data, int(steps), final.ctypes.data,
                                  ctypes.byref(hs), ctypes.byref(fr), ctypes.byref(sd), ctypes.byref(dg))
    if st:
        raise OracleError(st, "deterministic")
    return DetResult(final, hs.value, fr.value, sd.value, dg.value)
