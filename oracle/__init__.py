"""CPU oracle for OpSparse's row-wise SpGEMM hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's ``cpu_baseline`` leg, never by the library.  It shares no
code with the GPU path (the library never imports this package and this
package never imports the library).

Contents
* ``row_stats``  - setup step (Section 5, setup): n_prod, a_len, b_max per row.
* ``symbolic``   - symbolic step (Section 2.2): distinct output columns per row.
* ``spgemm``     - the full product C = A*B (Eq. 1 / Eq. 2) with sorted
                   columns plus the scale S_ij = sum_k |A_ik B_kj|.
* ``bin_of``     - bin membership of the binning method (Section 5.1,
                   Alg. 1-2): the first bin whose inclusive upper range bound
                   holds the row's value; the last bin is unbounded.
* ``row_pointer``- exclusive prefix sum of row sizes (Section 5.3).
* ``threads``    - ``symbolic`` and ``spgemm`` take ``threads=T``: the same
                   per-row code on T threads over blocks of rows (rows are
                   independent, Section 2.1), bit-identical to T = 1.
* ``bin_ranges`` - binning ranges from table sizes and the ratio rule of
                   Section 5.7 (symbolic: t/ratio, numeric: (t+1)/ratio).

Matrices are duck-typed: any object with ``rows, cols, rpt(int64), col(int32),
val(float64)`` works.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.oracle_row_stats.restype = ctypes.c_int64
        lib.oracle_row_stats.argtypes = [I, P, P, P, P, P, P]
        lib.oracle_symbolic.restype = ctypes.c_int
        lib.oracle_symbolic.argtypes = [I, P, I, P, P, P, P, P]
        lib.oracle_numeric.restype = ctypes.c_int
        lib.oracle_numeric.argtypes = [I, P, I, P, P, P, P, P, P, P, P, P, P]
        lib.oracle_symbolic_mt.restype = ctypes.c_int
        lib.oracle_symbolic_mt.argtypes = [ctypes.c_int, I, P, I, P, P, P, P, P]
        lib.oracle_numeric_mt.restype = ctypes.c_int
        lib.oracle_numeric_mt.argtypes = [ctypes.c_int, I, P, I, P, P, P, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def host_threads(cap: int = 16) -> int:
    """Threads for the row-parallel oracle: the CPUs this process may use,
    at most ``cap``."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def row_stats(A, B) -> Tuple[np.ndarray, np.ndarray, np.ndarray, int]:
    """(n_prod, a_len, b_max, total n_prod) for every row of A*B."""
    assert A.cols == B.rows
    lib = _load()
    arpt, acol, brpt = _c(A.rpt, np.int64), _c(A.col, np.int32), _c(B.rpt, np.int64)
    nprod = np.empty(A.rows, np.int64)
    alen = np.empty(A.rows, np.int64)
    bmax = np.empty(A.rows, np.int64)
    tot = lib.oracle_row_stats(A.rows, _p(arpt), _p(acol), _p(brpt), _p(nprod), _p(alen), _p(bmax))
    return nprod, alen, bmax, int(tot)


def symbolic(A, B, rows: Optional[np.ndarray] = None, threads: int = 1) -> np.ndarray:
    """Distinct output columns per row (all rows, or the listed ones)."""
    assert A.cols == B.rows
    lib = _load()
    r = None if rows is None else _c(rows, np.int64)
    nr = A.rows if r is None else r.size
    nnz = np.empty(nr, np.int64)
    arpt, acol = _c(A.rpt, np.int64), _c(A.col, np.int32)
    brpt, bcol = _c(B.rpt, np.int64), _c(B.col, np.int32)
    rc = lib.oracle_symbolic_mt(int(threads), nr, _p(r), B.cols, _p(arpt), _p(acol), _p(brpt),
                                _p(bcol), _p(nnz))
    if rc != 0:
        raise MemoryError("oracle_symbolic failed")
    return nnz


def row_pointer(sizes: np.ndarray) -> np.ndarray:
    """Exclusive prefix sum with the total appended (Section 5.3)."""
    out = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(np.asarray(sizes, dtype=np.int64), out=out[1:])
    return out


def spgemm(A, B, rows: Optional[np.ndarray] = None, with_scale: bool = True, threads: int = 1):
    """C = A*B.  Returns (rpt, col, val, S) for all rows, or for the listed
    rows packed one after another (rpt then indexes that packing)."""
    assert A.cols == B.rows
    lib = _load()
    r = None if rows is None else _c(rows, np.int64)
    nr = A.rows if r is None else r.size
    nnz = symbolic(A, B, r, threads=threads)
    off = row_pointer(nnz)
    total = int(off[-1])
    ccol = np.empty(total, np.int32)
    cval = np.empty(total, np.float64)
    cabs = np.empty(total, np.float64) if with_scale else None
    arpt, acol, aval = _c(A.rpt, np.int64), _c(A.col, np.int32), _c(A.val, np.float64)
    brpt, bcol, bval = _c(B.rpt, np.int64), _c(B.col, np.int32), _c(B.val, np.float64)
    rc = lib.oracle_numeric_mt(int(threads), nr, _p(r), B.cols, _p(arpt), _p(acol), _p(aval),
                               _p(brpt), _p(bcol), _p(bval), _p(off), _p(ccol), _p(cval), _p(cabs))
    if rc != 0:
        raise RuntimeError("oracle_numeric failed (%d)" % rc)
    return off, ccol, cval, cabs


def bin_of(values: np.ndarray, upper: Sequence[int]) -> np.ndarray:
    """Bin of each value: first j with value <= upper[j]; values above every
    bound go to the last bin (index len(upper))."""
    v = np.asarray(values, dtype=np.int64)
    out = np.full(v.shape, len(upper), dtype=np.int64)
    for j in reversed(range(len(upper))):
        out[v <= upper[j]] = j
    return out


def bin_ranges(table_sizes: Sequence[int], ratio: float, numeric: bool) -> list:
    """Inclusive upper bounds that keep each table at least ``ratio`` times the
    largest value routed to it (Section 5.7): floor(t/ratio) in the symbolic
    step, min(t, floor((t+1)/ratio)) in the numeric step, whose printed
    ranges divide the table budget t+1 (table plus the condensing counter)
    yet never exceed the table itself."""
    from fractions import Fraction
    r = Fraction(str(ratio))          # exact: "1.2" -> 6/5
    out = []
    for t in table_sizes:
        x = (t + 1) if numeric else t
        out.append(min(t, int((x * r.denominator) // r.numerator)))
    return out


def compare(crpt, ccol, cval, ref, tol: float = 1e-12):
    """Compare a GPU result against ``ref = spgemm(...)``: rpt and col must be
    identical, and |c - c_ref| <= tol * S per entry.  Returns a dict of
    diagnostics; raises AssertionError on mismatch."""
    rrpt, rcol, rval, rabs = ref
    crpt = np.asarray(crpt, np.int64)
    assert crpt.shape == rrpt.shape, "rpt length"
    assert np.array_equal(crpt - crpt[0], rrpt - rrpt[0]), "rpt mismatch"
    assert np.array_equal(np.asarray(ccol, np.int32), rcol), "col mismatch"
    err = np.abs(np.asarray(cval, np.float64) - rval)
    bound = tol * rabs
    bad = err > bound
    nz = np.abs(rval) > 0
    rel = np.max(err[nz] / np.abs(rval[nz])) if np.any(nz) else 0.0
    sre = np.max(err[rabs > 0] / rabs[rabs > 0]) if np.any(rabs > 0) else 0.0
    assert not np.any(bad), "value mismatch at %d entries (max |d|/S=%g)" % (int(bad.sum()), sre)
    return {"max_err_over_S": float(sre), "max_rel_err": float(rel),
            "bit_exact_values": bool(np.array_equal(np.asarray(cval).view(np.int64), rval.view(np.int64)))}
