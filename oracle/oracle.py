"""NumPy front end of the plain CPU oracle (``ffp_oracle.c``).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and the GPU library never calls it.

Every function takes and returns NumPy ``int32`` arrays holding canonical
residues in ``[0, p)``; matrices are row-major.  The arithmetic itself lives in
``ffp_oracle.c`` (int64 / int128, reduced at every step); this file only
marshals arguments.  Paper: Dumas, Gautier, Pernet, Sultan, "Parallel
computation of echelon forms", Section 2.1 (routine semantics) and Section 4.1
(rank-profile-revealing pivoting, tile recursion).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffp_oracle.c")
_LIB = os.path.join(_HERE, "libffp_oracle.so")

ORC_OK = 0
ORC_E_ARG = -1
ORC_E_NOTPRIME = -2
ORC_E_RANGE = -3
ORC_E_SINGULAR = -4
ORC_E_CONVENTION = -5
ORC_E_SELFCHECK = -6
ORC_E_NOMEM = -7


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over rows).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, i32p, u32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint32
        lib.orc_is_prime.argtypes = [ctypes.c_uint64]
        lib.orc_is_prime.restype = ctypes.c_int
        lib.orc_inv.argtypes = [i64, i64]
        lib.orc_inv.restype = i64
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_fgemm.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, i64, u32, u32,
                                  i32p, i64, i32p, i64, u32, i32p, i64]
        lib.orc_ftrsm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  i64, i64, u32, u32, i32p, i64, i32p, i64]
        lib.orc_pivots.argtypes = [i64, i64, u32, i32p, i64, i32p, i32p,
                                   ctypes.POINTER(i64), ctypes.c_void_p]
        lib.orc_order.argtypes = [i64, i64, i64, i32p, i32p, i32p, i32p]
        lib.orc_order.restype = i64
        lib.orc_pluq.argtypes = [i64, i64, u32, i32p, i64, i32p, i32p,
                                 ctypes.POINTER(i64), i32p, i32p, ctypes.c_int]
        lib.orc_pluq_rowmajor.argtypes = [i64, i64, u32, i32p, i64, i32p, i32p, ctypes.POINTER(i64), i32p, i32p]
        lib.orc_rref.argtypes = [i64, i64, u32, i32p, i64, i32p, i32p, ctypes.POINTER(i64)]
        lib.orc_nullspace.argtypes = [i64, i64, u32, i32p, i64, i32p, ctypes.POINTER(i64)]
        lib.orc_solve.argtypes = [i64, i64, u32, i32p, i64, i64, i32p, i64, i32p, i64, i32p,
                                  ctypes.POINTER(i64)]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _mat(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    if a.ndim != 2:
        raise ValueError("expected a 2-D matrix")
    return a


def is_prime(n: int) -> bool:
    return bool(_load().orc_is_prime(int(n)))


def inv(a: int, p: int) -> int:
    return int(_load().orc_inv(int(a), int(p)))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def fgemm(A, B, C, p: int, alpha: int = 1, beta: int = 0, transA=False, transB=False) -> np.ndarray:
    """alpha*op(A)*op(B) + beta*C mod p (new array)."""
    A, B = _mat(A), _mat(B)
    C = _mat(C).copy()
    m, n = C.shape
    k = A.shape[0] if transA else A.shape[1]
    e = _load().orc_fgemm(int(bool(transA)), int(bool(transB)), m, n, k, p, alpha,
                          _ptr(A), A.shape[1], _ptr(B), B.shape[1], beta, _ptr(C), max(n, 1))
    if e:
        raise OracleError(e, "fgemm")
    return C


def ftrsm(side: int, uplo: int, trans: int, diag: int, T, B, p: int, alpha: int = 1) -> np.ndarray:
    """Triangular solve (see ffp_oracle.c: orc_ftrsm); returns the solution X."""
    T = _mat(T)
    X = _mat(B).copy()
    m, n = X.shape
    e = _load().orc_ftrsm(side, uplo, trans, diag, m, n, p, alpha, _ptr(T), max(T.shape[1], 1),
                          _ptr(X), max(n, 1))
    if e:
        raise OracleError(e, "ftrsm")
    return X


def pivots(A, p: int):
    """Pass 1: the pivot pairs of the row-major search, in row order.

    Returns (rank, rows, cols) with rows/cols int32 arrays of length rank."""
    A = _mat(A)
    m, n = A.shape
    k = max(min(m, n), 1)
    pr = np.zeros(k, np.int32)
    pc = np.zeros(k, np.int32)
    r = ctypes.c_int64(0)
    e = _load().orc_pivots(m, n, p, _ptr(A), max(n, 1), _ptr(pr), _ptr(pc), ctypes.byref(r), None)
    if e:
        raise OracleError(e, "pivots")
    return int(r.value), pr[: r.value].copy(), pc[: r.value].copy()


def order(m: int, n: int, rows, cols):
    """Pivot order of the four-quadrant recursion for the given pivot set."""
    rows = np.ascontiguousarray(rows, np.int32)
    cols = np.ascontiguousarray(cols, np.int32)
    r = len(rows)
    orow = np.zeros(max(r, 1), np.int32)
    ocol = np.zeros(max(r, 1), np.int32)
    cnt = _load().orc_order(m, n, r, _ptr(rows), _ptr(cols), _ptr(orow), _ptr(ocol))
    return orow[:cnt].copy(), ocol[:cnt].copy()


@dataclass
class PLUQ:
    LU: np.ndarray   # m x n, L (strictly lower, unit diagonal implied) and U in place
    P: np.ndarray    # m: original row placed at position i
    Q: np.ndarray    # n: original column placed at position j
    rank: int
    rrp: np.ndarray  # sorted row rank profile (length rank)
    crp: np.ndarray  # sorted column rank profile (length rank)

    def L(self) -> np.ndarray:
        m = self.LU.shape[0]
        r = self.rank
        L = np.tril(self.LU[:, :r].astype(np.int64), -1)
        L[np.arange(r), np.arange(r)] = 1
        return L[:m]

    def U(self) -> np.ndarray:
        r = self.rank
        return np.triu(self.LU[:r, :].astype(np.int64))


def pluq(A, p: int, selfcheck: bool = True) -> PLUQ:
    """Canonical rank-profile-revealing PLUQ of A over Z/pZ (see orc_pluq)."""
    W = _mat(A).copy()
    m, n = W.shape
    P = np.zeros(max(m, 1), np.int32)
    Q = np.zeros(max(n, 1), np.int32)
    k = max(min(m, n), 1)
    rrp = np.zeros(k, np.int32)
    crp = np.zeros(k, np.int32)
    r = ctypes.c_int64(0)
    e = _load().orc_pluq(m, n, p, _ptr(W), max(n, 1), _ptr(P), _ptr(Q), ctypes.byref(r),
                         _ptr(rrp), _ptr(crp), int(bool(selfcheck)))
    if e:
        raise OracleError(e, "pluq")
    r = int(r.value)
    return PLUQ(W, P[:m].copy(), Q[:n].copy(), r, rrp[:r].copy(), crp[:r].copy())


def pluq_rowmajor(A, p: int) -> PLUQ:
    """PLUQ in the order of the row-major search (see orc_pluq_rowmajor):
    pivots in increasing row order, the output of the slab algorithms."""
    W = _mat(A).copy()
    m, n = W.shape
    P = np.zeros(max(m, 1), np.int32)
    Q = np.zeros(max(n, 1), np.int32)
    k = max(min(m, n), 1)
    rrp = np.zeros(k, np.int32)
    crp = np.zeros(k, np.int32)
    r = ctypes.c_int64(0)
    e = _load().orc_pluq_rowmajor(m, n, p, _ptr(W), max(n, 1), _ptr(P), _ptr(Q), ctypes.byref(r),
                                  _ptr(rrp), _ptr(crp))
    if e:
        raise OracleError(e, "pluq_rowmajor")
    r = int(r.value)
    return PLUQ(W, P[:m].copy(), Q[:n].copy(), r, rrp[:r].copy(), crp[:r].copy())


def rref(A, p: int):
    """Reduced row echelon form by Gauss-Jordan (see orc_rref).

    Returns (rank, R, pivcols): R is r x n, pivcols the r pivot columns."""
    A = _mat(A)
    m, n = A.shape
    R = np.zeros((max(m, 1), max(n, 1)), np.int32)
    pc = np.zeros(max(n, 1), np.int32)
    r = ctypes.c_int64(0)
    e = _load().orc_rref(m, n, p, _ptr(A), max(n, 1), _ptr(R), _ptr(pc), ctypes.byref(r))
    if e:
        raise OracleError(e, "rref")
    r = int(r.value)
    return r, R.reshape(-1)[: m * n].reshape(m, n)[:r].copy(), pc[:r].copy()


def nullspace(A, p: int):
    """Right nullspace basis N (n x (n - r)), identity on the non-pivot rows."""
    A = _mat(A)
    m, n = A.shape
    N = np.zeros(max(n * n, 1), np.int32)
    r = ctypes.c_int64(0)
    e = _load().orc_nullspace(m, n, p, _ptr(A), max(n, 1), _ptr(N), ctypes.byref(r))
    if e:
        raise OracleError(e, "nullspace")
    r = int(r.value)
    return N[: n * (n - r)].reshape(n, n - r).copy()


def solve(A, B, p: int):
    """Solutions of A X = B zero on the non-pivot columns; returns (X, consistent, rank)."""
    A, B = _mat(A), _mat(B)
    m, n = A.shape
    nrhs = B.shape[1]
    X = np.zeros((max(n, 1), max(nrhs, 1)), np.int32)
    ok = np.zeros(max(nrhs, 1), np.int32)
    r = ctypes.c_int64(0)
    e = _load().orc_solve(m, n, p, _ptr(A), max(n, 1), nrhs, _ptr(B), max(nrhs, 1), _ptr(X), max(nrhs, 1),
                          _ptr(ok), ctypes.byref(r))
    if e:
        raise OracleError(e, "solve")
    return X[:n, :nrhs].copy(), ok[:nrhs].astype(bool), int(r.value)
