"""CPU oracle for h-hop degrees and (k,h)-core numbers.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or
calls this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It is written from the definitions of Section II and
the peeling algorithms of Sections III-IV of the paper and shares no code
with the GPU path.

Two implementations:
  reference.py   literal Python (brute force over vertex sets, Algorithm 1
                 one vertex at a time, the linear k-core bin sort, a
                 level-synchronous peel) for small graphs;
  khc_oracle.c   plain C (bounded BFS h-degrees, the level-synchronous
                 peel with from-scratch recomputation and per-round trace,
                 the peeling-order certificate), loaded here through
                 ctypes; the peel is single-threaded, the per-vertex
                 loops of hdeg_list and certificate can use OpenMP threads.
The MLP of the learned approximate mode has its own reference in mlp.py
(pinned to finite differences).  The approximate decomposition itself has
no oracle: its output is an estimate whose error the tests measure against
the exact core numbers computed here (parity unpinned by design).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import reference  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "khc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile khc_oracle.c into liboracle.so with gcc (single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-fopenmp",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        lib.oracle_check_csr.argtypes = [u32, P, P]
        lib.oracle_hdeg.argtypes = [u32, P, P, P, u32, P]
        lib.oracle_hdeg_list.argtypes = [u32, P, P, P, u32, P, u64, P, P, ctypes.c_int]
        lib.oracle_peel.argtypes = [u32, P, P, u32, P, P, P, P, P, u64, P]
        lib.oracle_certificate.argtypes = [u32, P, P, u32, P, P, P, u64, P, ctypes.c_int]
        lib.oracle_peel_sampled.argtypes = [u32, P, P, u32, P, P, P]
        for f in (lib.oracle_check_csr, lib.oracle_hdeg, lib.oracle_hdeg_list,
                  lib.oracle_peel, lib.oracle_certificate, lib.oracle_peel_sampled):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    return int(g.n), rp, col


def _alive(alive, n):
    if alive is None:
        return None
    a = np.ascontiguousarray(alive, dtype=np.uint8)
    if a.shape != (n,):
        raise ValueError("alive mask must have n entries")
    return a


def check_csr(g) -> int:
    """0 if g is a simple undirected CSR graph, else a negative code."""
    n, rp, col = _graph(g)
    return _load().oracle_check_csr(n, _ptr(rp), _ptr(col))


def hdeg(g, h: int, alive=None) -> np.ndarray:
    """h-degree of every vertex of G(alive) (dead vertices: 0), uint32."""
    n, rp, col = _graph(g)
    a = _alive(alive, n)
    out = np.zeros(max(n, 1), dtype=np.uint32)
    rc = _load().oracle_hdeg(n, _ptr(rp), _ptr(col), _ptr(a), h, _ptr(out))
    if rc:
        raise MemoryError("oracle_hdeg failed")
    return out[:n]


def hdeg_list(g, h: int, verts, alive=None, threads: int = 1):
    """(h-degrees, scanned-arc counts) of the listed vertices only; the
    vertices may be split over `threads` OpenMP threads."""
    n, rp, col = _graph(g)
    a = _alive(alive, n)
    v = np.ascontiguousarray(verts, dtype=np.uint32)
    deg = np.zeros(max(v.size, 1), dtype=np.uint32)
    te = np.zeros(max(v.size, 1), dtype=np.uint64)
    rc = _load().oracle_hdeg_list(n, _ptr(rp), _ptr(col), _ptr(a), h, _ptr(v),
                                  v.size, _ptr(deg), _ptr(te), int(threads))
    if rc:
        raise MemoryError("oracle_hdeg_list failed")
    return deg[:v.size], te[:v.size]


def peel(g, h: int, trace: bool = False):
    """Level-synchronous peel.  Returns (core, round) or (core, round, trace)

    where trace is a (rounds, 3) uint32 array of (k, |P|, |A|).
    """
    n, rp, col = _graph(g)
    core = np.zeros(max(n, 1), dtype=np.uint32)
    rnd = np.zeros(max(n, 1), dtype=np.uint32)
    rounds = np.zeros(1, dtype=np.uint64)
    cap = n if trace else 0
    tk = np.zeros(max(cap, 1), dtype=np.uint32) if trace else None
    tp = np.zeros(max(cap, 1), dtype=np.uint32) if trace else None
    ta = np.zeros(max(cap, 1), dtype=np.uint32) if trace else None
    rc = _load().oracle_peel(n, _ptr(rp), _ptr(col), h, _ptr(core), _ptr(rnd),
                             _ptr(tk), _ptr(tp), _ptr(ta), cap, _ptr(rounds))
    if rc:
        raise RuntimeError(f"oracle_peel failed ({rc})")
    if not trace:
        return core[:n], rnd[:n]
    r = int(rounds[0])
    return core[:n], rnd[:n], np.stack([tk[:r], tp[:r], ta[:r]], axis=1)


def peel_sampled(g, h: int, sampled):
    """Sampling-based peeling on the vertex sample `sampled` (uint8 mask):
    (core, estimate at removal), both uint32."""
    n, rp, col = _graph(g)
    s = np.ascontiguousarray(sampled, dtype=np.uint8)
    if s.shape != (n,):
        raise ValueError("sample mask must have n entries")
    core = np.zeros(max(n, 1), dtype=np.uint32)
    est = np.zeros(max(n, 1), dtype=np.uint32)
    rc = _load().oracle_peel_sampled(n, _ptr(rp), _ptr(col), h, _ptr(s), _ptr(core), _ptr(est))
    if rc:
        raise MemoryError("oracle_peel_sampled failed")
    return core[:n], est[:n]


def certificate(g, h: int, core, rnd, verts=None, threads: int = 1):
    """Violation counts of the three peeling-order certificate conditions
    ((i) and (ii) on the listed vertices, all when verts is None; (iii) on
    all), with the vertices split over `threads` OpenMP threads."""
    n, rp, col = _graph(g)
    c = np.ascontiguousarray(core, dtype=np.uint32)
    r = np.ascontiguousarray(rnd, dtype=np.uint32)
    v = None if verts is None else np.ascontiguousarray(verts, dtype=np.uint32)
    fail = np.zeros(3, dtype=np.uint64)
    rc = _load().oracle_certificate(n, _ptr(rp), _ptr(col), h, _ptr(c), _ptr(r),
                                    _ptr(v), 0 if v is None else v.size, _ptr(fail), int(threads))
    if rc:
        raise MemoryError("oracle_certificate failed")
    return fail


def host_threads() -> int:
    """Threads this process may run on (its CPU affinity)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1
