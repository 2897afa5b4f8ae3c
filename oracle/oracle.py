"""Python face of the CPU oracle (``fsp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle proves the HIP path right and is timed as
the CPU baseline.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the product package and the product never imports it.

What each function computes is documented, with the paper's section, in
``fsp_oracle.c``.  Everything here is argument marshalling.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no intrinsics, plain C)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


class Stats(ctypes.Structure):
    _fields_ = [
        ("nodes_bounded", ctypes.c_int64),
        ("nodes_branched", ctypes.c_int64),
        ("nodes_pruned", ctypes.c_int64),
        ("leaves", ctypes.c_int64),
        ("found", ctypes.c_int32),
        ("root_lb", ctypes.c_int32),
        ("complete", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


def use_library(path: str | None):
    """Point this module at another build of the oracle (used by the test that
    plants mistakes in a copy of the source); ``None`` restores the default."""
    global _lib
    _lib = None
    if path is not None:
        _load(path)


def _load(path: str | None = None):
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = _LIB
        if not os.path.exists(_LIB):
            build(force=False)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.orc_front.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P]
    lib.orc_front.restype = None
    lib.orc_makespan.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
    lib.orc_makespan.restype = i64
    lib.orc_johnson_order.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, P, ctypes.c_int, P]
    lib.orc_johnson_order.restype = None
    lib.orc_lower_bound_pairs.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
    lib.orc_lower_bound_pairs.restype = i64
    lib.orc_lower_bound.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    lib.orc_lower_bound.restype = i64
    lib.orc_bound_pool.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, i64,
                                   P, ctypes.c_int]
    lib.orc_bound_pool.restype = None
    lib.orc_lower_bound_one_machine.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    lib.orc_lower_bound_one_machine.restype = i64
    lib.orc_bound_pool_one_machine.argtypes = [P, ctypes.c_int, ctypes.c_int, P,
                                               ctypes.c_int, i64, P, ctypes.c_int]
    lib.orc_bound_pool_one_machine.restype = None
    lib.orc_neh.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    lib.orc_neh.restype = i64
    lib.orc_brute_force.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    lib.orc_brute_force.restype = i64
    lib.orc_best_completion.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    lib.orc_best_completion.restype = i64
    lib.orc_bnb.argtypes = [P, ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, i64, P,
                            ctypes.POINTER(Stats)]
    lib.orc_bnb.restype = i64
    lib.orc_bnb_choice.argtypes = [P, ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, i64, P, P,
                                   ctypes.POINTER(Stats)]
    lib.orc_bnb_choice.restype = i64
    del i32
    _lib = lib
    return lib


def _p(p):
    p = np.ascontiguousarray(p, dtype=np.int32)
    assert p.ndim == 2
    return p, p.shape[0], p.shape[1]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _node(prefix, n):
    rec = np.zeros(max(n, len(prefix)) + 1, dtype=np.uint8)
    rec[0] = len(prefix)
    rec[1:1 + len(prefix)] = np.asarray(prefix, dtype=np.uint8)
    return rec


def front(p, seq):
    """Completion time of ``seq`` on every machine (int64[m])."""
    p, n, m = _p(p)
    s = np.ascontiguousarray(seq, dtype=np.uint8)
    out = np.zeros(m, dtype=np.int64)
    _load().orc_front(_ptr(p), n, m, _ptr(s), len(s), _ptr(out))
    return out


def makespan(p, seq):
    p, n, m = _p(p)
    s = np.ascontiguousarray(seq, dtype=np.uint8)
    return int(_load().orc_makespan(_ptr(p), n, m, _ptr(s), len(s)))


def johnson_order(p, k, l, jobs):
    p, n, m = _p(p)
    j = np.ascontiguousarray(jobs, dtype=np.uint8)
    out = np.zeros(len(j), dtype=np.uint8)
    _load().orc_johnson_order(_ptr(p), n, m, k, l, _ptr(j), len(j), _ptr(out))
    return out


def lower_bound(p, prefix):
    """Bound of the node whose scheduled prefix is ``prefix``."""
    p, n, m = _p(p)
    rec = _node(prefix, n)
    return int(_load().orc_lower_bound(_ptr(p), n, m, _ptr(rec)))


def lower_bound_pairs(p, prefix):
    """(bound, per-pair bounds in lexicographic (k,l) order)."""
    p, n, m = _p(p)
    rec = _node(prefix, n)
    out = np.zeros(m * (m - 1) // 2, dtype=np.int64)
    lb = _load().orc_lower_bound_pairs(_ptr(p), n, m, _ptr(rec), _ptr(out))
    return int(lb), out


def lower_bound_record(p, record):
    """Bound of one raw node record ``[d, s_1..s_d, ...]``."""
    p, n, m = _p(p)
    rec = np.ascontiguousarray(record, dtype=np.uint8)
    if len(rec) < n + 1:
        rec = np.concatenate([rec, np.zeros(n + 1 - len(rec), np.uint8)])
    return int(_load().orc_lower_bound(_ptr(p), n, m, _ptr(rec)))


def bound_pool(p, nodes, nthreads: int = 1):
    """Bounds of every record of a ``uint8[count, stride]`` pool (int32[count])."""
    p, n, m = _p(p)
    nodes = np.ascontiguousarray(nodes, dtype=np.uint8)
    count, stride = nodes.shape
    out = np.zeros(count, dtype=np.int32)
    _load().orc_bound_pool(_ptr(p), n, m, _ptr(nodes), stride, count, _ptr(out),
                           int(nthreads))
    return out


def lower_bound_one_machine(p, prefix):
    """One-machine bound of the node whose scheduled prefix is ``prefix``:
    max over machines of head + remaining work + smallest tail."""
    p, n, m = _p(p)
    rec = _node(prefix, n)
    return int(_load().orc_lower_bound_one_machine(_ptr(p), n, m, _ptr(rec)))


def bound_pool_one_machine(p, nodes, nthreads: int = 1):
    """One-machine bounds of every record of a ``uint8[count, stride]`` pool."""
    p, n, m = _p(p)
    nodes = np.ascontiguousarray(nodes, dtype=np.uint8)
    count, stride = nodes.shape
    out = np.zeros(count, dtype=np.int32)
    _load().orc_bound_pool_one_machine(_ptr(p), n, m, _ptr(nodes), stride, count,
                                       _ptr(out), int(nthreads))
    return out


def neh(p):
    p, n, m = _p(p)
    perm = np.zeros(n, dtype=np.uint8)
    c = _load().orc_neh(_ptr(p), n, m, _ptr(perm))
    return int(c), perm


def brute_force(p):
    p, n, m = _p(p)
    perm = np.zeros(n, dtype=np.uint8)
    c = _load().orc_brute_force(_ptr(p), n, m, _ptr(perm))
    return int(c), perm


def best_completion(p, prefix):
    p, n, m = _p(p)
    rec = _node(prefix, n)
    return int(_load().orc_best_completion(_ptr(p), n, m, _ptr(rec)))


def bnb(p, ub_in: int = 0, rule: int = 0, max_bounded: int = 0):
    """Sequential DFS branch-and-bound.  Returns (makespan, perm, Stats)."""
    p, n, m = _p(p)
    perm = np.zeros(n, dtype=np.uint8)
    st = Stats()
    c = _load().orc_bnb(_ptr(p), n, m, int(ub_in), int(rule), int(max_bounded),
                        _ptr(perm), ctypes.byref(st))
    return int(c), perm, st


def bnb_choice(p, lb1_depths, ub_in: int = 0, rule: int = 0, max_bounded: int = 0):
    """The same search with the one-machine bound at the depths in
    `lb1_depths` (0 < d < n) and the two-machine bound elsewhere (the
    per-depth choice of bound; Sec. VI).  Returns (makespan, perm, Stats)."""
    p, n, m = _p(p)
    mask = np.zeros(8, dtype=np.uint32)
    for d in lb1_depths:
        mask[int(d) >> 5] |= np.uint32(1 << (int(d) & 31))
    perm = np.zeros(n, dtype=np.uint8)
    st = Stats()
    c = _load().orc_bnb_choice(_ptr(p), n, m, int(ub_in), int(rule), int(max_bounded),
                               _ptr(mask), _ptr(perm), ctypes.byref(st))
    return int(c), perm, st
