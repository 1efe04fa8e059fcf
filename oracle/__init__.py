"""CPU oracle for the joins of "GPU-based Efficient Join Algorithms on Hadoop".

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and bench.py's cpu_baseline leg
are the only callers.  Nothing here is imported by the GPU library, and this package imports
nothing from it.  The arithmetic lives in ``oracle.c`` (plain C + OpenMP); this module builds and
loads it and converts numpy arrays.

Functions (each returns ``(count, pairs)``; ``pairs`` is an int32 array of shape [count, 2] in
canonical order -- ascending by (rid_R, rid_S) -- or None when ``want_pairs`` is False):

* ``theta_nlj``      brute-force nested loop over all |R|*|S| pairs (Section 2.3, the
                     definition of the equi and theta join, evaluated by nested loops).
* ``equi_nlj``       ``theta_nlj`` with the equality operator.
* ``equi_sortmerge`` sort-merge equi join (Section 2.3, "Sort merge join").
* ``band_window``    sorted-window evaluation of |R.a - S.a| <= w [and op_c].
* ``count_equi``     sum over keys of multiplicity products.
* ``count_lt``       number of pairs with R.a < S.a by binary search.

Operators are named: 'none', 'eq', 'ne', 'lt', 'le', 'gt', 'ge', 'band' (``R.x op S.x``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Private operator codes of oracle.c (ORC_*).
_OPS = {"none": 0, "eq": 1, "ne": 2, "lt": 3, "le": 4, "gt": 5, "ge": 6, "band": 7}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no hand-written SIMD) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        p32 = ctypes.POINTER(ctypes.c_int32)
        i64, u64 = ctypes.c_int64, ctypes.c_uint64
        lib.oracle_theta_nlj.restype = u64
        lib.oracle_theta_nlj.argtypes = [i64, p32, p32, p32, i64, p32, p32, p32,
                                         ctypes.c_int, i64, ctypes.c_int, p32, u64]
        lib.oracle_equi_sortmerge.restype = u64
        lib.oracle_equi_sortmerge.argtypes = [i64, p32, p32, i64, p32, p32, p32, u64]
        lib.oracle_band_window.restype = u64
        lib.oracle_band_window.argtypes = [i64, p32, p32, p32, i64, p32, p32, p32,
                                           i64, ctypes.c_int, p32, u64]
        lib.oracle_count_equi.restype = u64
        lib.oracle_count_equi.argtypes = [i64, p32, i64, p32]
        lib.oracle_count_lt.restype = u64
        lib.oracle_count_lt.argtypes = [i64, p32, i64, p32]
        lib.oracle_sort_pairs.restype = None
        lib.oracle_sort_pairs.argtypes = [p32, u64]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all cores)."""
    return int(_load().oracle_max_threads())


def _col(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _run(fn, head_args, _unused, want_pairs):
    """Call fn once to count; if pairs are wanted, call again with an exactly-sized buffer."""
    n = int(fn(*head_args, None, 0))
    if not want_pairs:
        return n, None
    out = np.empty((max(n, 1), 2), dtype=np.int32)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    n2 = int(fn(*head_args, ptr, n))
    assert n2 == n
    return n, out[:n]


def theta_nlj(Ra, Sa, op_a, w=0, Rc=None, Sc=None, op_c="none", Rrid=None, Srid=None,
              want_pairs=True):
    """Brute-force nested-loop theta join: all (i, j) with op_a(Ra[i], Sa[j]) and
    op_c(Rc[i], Sc[j])."""
    lib = _load()
    ra, pra = _col(Ra)
    sa, psa = _col(Sa)
    rc, prc = _col(Rc)
    sc, psc = _col(Sc)
    rr, prr = _col(Rrid)
    sr, psr = _col(Srid)
    if op_c != "none" and (rc is None or sc is None):
        raise ValueError("op_c needs both c columns")
    head = (len(ra), pra, prc, prr, len(sa), psa, psc, psr, _OPS[op_a], int(w), _OPS[op_c])
    return _run(lib.oracle_theta_nlj, head, None, want_pairs)


def equi_nlj(Rk, Sk, Rrid=None, Srid=None, want_pairs=True):
    """Brute-force nested-loop equi join."""
    return theta_nlj(Rk, Sk, "eq", Rrid=Rrid, Srid=Srid, want_pairs=want_pairs)


def equi_sortmerge(Rk, Sk, Rrid=None, Srid=None, want_pairs=True):
    """Sort-merge equi join."""
    lib = _load()
    rk, prk = _col(Rk)
    sk, psk = _col(Sk)
    rr, prr = _col(Rrid)
    sr, psr = _col(Srid)
    head = (len(rk), prk, prr, len(sk), psk, psr)
    return _run(lib.oracle_equi_sortmerge, head, None, want_pairs)


def band_window(Ra, Sa, w, Rc=None, Sc=None, op_c="none", Rrid=None, Srid=None, want_pairs=True):
    """Sorted-window band join |Ra - Sa| <= w [and op_c(Rc, Sc)]."""
    lib = _load()
    ra, pra = _col(Ra)
    sa, psa = _col(Sa)
    rc, prc = _col(Rc)
    sc, psc = _col(Sc)
    rr, prr = _col(Rrid)
    sr, psr = _col(Srid)
    if op_c != "none" and (rc is None or sc is None):
        raise ValueError("op_c needs both c columns")
    head = (len(ra), pra, prc, prr, len(sa), psa, psc, psr, int(w), _OPS[op_c])
    return _run(lib.oracle_band_window, head, None, want_pairs)


def count_equi(Rk, Sk) -> int:
    """Equi-join count: sum over keys of cntR[k] * cntS[k]."""
    lib = _load()
    rk, prk = _col(Rk)
    sk, psk = _col(Sk)
    return int(lib.oracle_count_equi(len(rk), prk, len(sk), psk))


def count_lt(Ra, Sa) -> int:
    """Number of pairs with Ra[i] < Sa[j]."""
    lib = _load()
    ra, pra = _col(Ra)
    sa, psa = _col(Sa)
    return int(lib.oracle_count_lt(len(ra), pra, len(sa), psa))


def sort_pairs(pairs):
    """Canonical order (ascending by rid_R, then rid_S) of an int32 [n, 2] array, in place."""
    lib = _load()
    p = np.ascontiguousarray(pairs, dtype=np.int32)
    lib.oracle_sort_pairs(p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(p))
    return p
