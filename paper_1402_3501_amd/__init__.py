"""ffpluq: exact rank-profile-revealing PLUQ over Z/pZ on AMD MI355X (gfx950).

Thin Python binding of ``libffpluq.so`` (C ABI in ``include/ffpluq.h``).  It
only marshals arguments: torch tensors provide device memory and the current
HIP stream; every step of every routine runs in the library's HIP kernels.
There is no fallback: if the library is missing or no GPU is present, calls
raise.

Paper: Dumas, Gautier, Pernet, Sultan, "Parallel computation of echelon
forms" (arXiv:1402.3501), Section 2.1 (fgemm, ftrsm, flaswp, PLUQ).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

PATH_AUTO, PATH_FP64, PATH_INT8 = 0, 1, 2
P_MAX_FP64 = 94906249
P_MAX_INT8 = 16711421
BATCH_MAX_DIM = 1024
BATCH_SHAPES = 4  # launch shapes the batched autotuner chooses from

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffpluq.so")
_lib = None


class FFPError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib.ffp_error_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})")
        self.code = code


def load():
    """Load libffpluq.so (built by __graft_entry__.build() / paper_1402_3501_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, vp, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "ffp_error_string": ([i32], ctypes.c_char_p),
        "ffp_version": ([], ctypes.c_char_p),
        "ffp_is_prime": ([u32], i32),
        "ffp_int8_limbs": ([u32], i32),
        "ffp_auto_path": ([u32, i64, i64, i64], i32),
        "ffp_fgemm_workspace": ([i32, i32, i64, i64, i64, u32, i32], sz),
        "ffp_fgemm": ([i32, i32, i64, i64, i64, u32, u32, vp, i64, vp, i64, u32, vp, i64, i32, vp, sz, vp], i32),
        "ffp_fgemm_noalloc": ([i32, i32, i64, i64, i64, u32, u32, vp, i64, vp, i64, u32, vp, i64, i32, vp], i32),
        "ffp_noalloc_scratch_bytes": ([], sz),
        "ffp_fgemm_wino_workspace": ([i32, i32, i64, i64, i64, u32, i32, i32], sz),
        "ffp_fgemm_wino": ([i32, i32, i64, i64, i64, u32, u32, vp, i64, vp, i64, u32, vp, i64, i32, i32, vp, sz, vp],
                           i32),
        "ffp_ftrsm_workspace": ([i32, i32, i32, i32, i64, i64, u32, i32], sz),
        "ffp_ftrsm": ([i32, i32, i32, i32, i64, i64, u32, u32, vp, i64, vp, i64, i32, vp, sz, vp], i32),
        "ffp_flaswp_workspace": ([i32, i64, i64], sz),
        "ffp_flaswp": ([i32, i64, i64, vp, i64, vp, i32, vp, sz, vp], i32),
        "ffp_pluq_workspace": ([i64, i64, u32, i32], sz),
        "ffp_pluq": ([i64, i64, u32, vp, i64, vp, vp, vp, ctypes.POINTER(i64), vp, vp, i32, vp, sz, vp], i32),
        "ffp_pluq_slab_workspace": ([i64, i64, u32, i32], sz),
        "ffp_pluq_slab": ([i64, i64, u32, vp, i64, vp, vp, vp, ctypes.POINTER(i64), vp, vp, i32, vp, sz, vp], i32),
        "ffp_lu_nopiv_workspace": ([i64, i64, u32, i32], sz),
        "ffp_lu_nopiv": ([i64, i64, u32, vp, i64, vp, i32, vp, sz, vp], i32),
        "ffp_check_range": ([i64, i64, u32, vp, i64, vp], i32),
        "ffp_lu_tiled_workspace": ([i32, i64, i64, i64, u32, i32], sz),
        "ffp_lu_tiled": ([i32, i64, i64, u32, vp, i64, i64, vp, i32, vp, sz, vp], i32),
        "ffp_reduction_count": ([i32, i64, i64, ctypes.POINTER(ctypes.c_double)], i32),
        "ffp_echelon_workspace": ([i32, i64, i64, i64, u32, i32], sz),
        "ffp_echelon": ([i32, i64, i64, u32, vp, i64, vp, vp, i64, vp, i64, i32, vp, sz, vp], i32),
        "ffp_nullspace_workspace": ([i32, i64, i64, i64, u32, i32], sz),
        "ffp_nullspace": ([i32, i64, i64, u32, vp, i64, vp, vp, i64, vp, i64, i32, vp, sz, vp], i32),
        "ffp_solve_workspace": ([i64, i64, i64, i64, u32, i32], sz),
        "ffp_solve": ([i64, i64, u32, vp, i64, vp, vp, i64, i64, vp, i64, vp, i64, vp, i32, vp, sz, vp], i32),
        "ffp_pluq_batched_workspace": ([i32, i32, i32, u32, i32], sz),
        "ffp_pluq_batched": ([i32, vp, vp, i32, i32, u32, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, sz, vp], i32),
        "ffp_pluq_batched_tune_workspace": ([i32, i32, i32, i64], sz),
        "ffp_pluq_batched_set_shape": ([i32, i32, i32, i32], i32),
        "ffp_pluq_batched_tune": ([i32, vp, vp, i32, i32, u32, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, i32,
                                   ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), vp, sz, vp], i32),
        "ffp_perm_to_swaps": ([i64, vp, vp], i32),
        "ffp_swaps_to_perm": ([i64, vp, vp], i32),
        "ffp_profile_enable": ([i32], i32),
        "ffp_profile_reset": ([], i32),
        "ffp_profile_read": ([i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)], i32),
        "ffp_profile_read_bytes": ([i32, ctypes.POINTER(ctypes.c_double)], i32),
        "ffp_profile_kind_name": ([i32], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _check(code: int, what: str):
    if code != 0:
        raise FFPError(code, what)


def _mat(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or t.dim() != 2 or not t.is_cuda:
        raise TypeError(f"{name} must be a 2-D int32 CUDA tensor")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must be row-major (unit column stride)")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)
    return ctypes.c_void_p(t.data_ptr()), max(int(ld), 1)


def _vec(t, name: str, dtype=None):
    torch = _torch()
    dtype = dtype or torch.int32
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    if nbytes == 0:
        return None, ctypes.c_void_p(0)
    w = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    return w, ctypes.c_void_p(w.data_ptr())


def version() -> str:
    return load().ffp_version().decode()


def is_prime(p: int) -> bool:
    return bool(load().ffp_is_prime(p))


def int8_limbs(p: int) -> int:
    return int(load().ffp_int8_limbs(p))


def auto_path(p: int, m: int, n: int, k: int) -> int:
    return int(load().ffp_auto_path(p, m, n, k))


def fgemm(A, B, C, p: int, alpha: int = 1, beta: int = 0, transA: bool = False, transB: bool = False,
          path: int = PATH_AUTO):
    """C <- alpha op(A) op(B) + beta C mod p, in place on C (returns C)."""
    lib = load()
    a, lda = _mat(A, "A")
    b, ldb = _mat(B, "B")
    c, ldc = _mat(C, "C")
    m, n = C.shape
    k = A.shape[0] if transA else A.shape[1]
    if (A.shape[1] if transA else A.shape[0]) != m or (B.shape[1] if transB else B.shape[0]) != k or \
            (B.shape[0] if transB else B.shape[1]) != n:
        raise ValueError("fgemm: shape mismatch")
    need = lib.ffp_fgemm_workspace(int(transA), int(transB), m, n, k, p, path)
    keep, ws = _workspace(need, C.device)
    _check(lib.ffp_fgemm(int(transA), int(transB), m, n, k, p, alpha, a, lda, b, ldb, beta, c, ldc, path,
                         ws, need, _stream(C)), "ffp_fgemm")
    return C


WINO_AUTO = -1


def fgemm_wino(A, B, C, p: int, alpha: int = 1, beta: int = 0, transA: bool = False, transB: bool = False,
               path: int = PATH_AUTO, levels: int = WINO_AUTO):
    """fgemm through Strassen-Winograd steps (levels; WINO_AUTO = the library's
    measured choice), in place on C (returns C)."""
    lib = load()
    a, lda = _mat(A, "A")
    b, ldb = _mat(B, "B")
    c, ldc = _mat(C, "C")
    m, n = C.shape
    k = A.shape[0] if transA else A.shape[1]
    if (A.shape[1] if transA else A.shape[0]) != m or (B.shape[1] if transB else B.shape[0]) != k or \
            (B.shape[0] if transB else B.shape[1]) != n:
        raise ValueError("fgemm_wino: shape mismatch")
    need = lib.ffp_fgemm_wino_workspace(int(transA), int(transB), m, n, k, p, path, levels)
    keep, ws = _workspace(need, C.device)
    _check(lib.ffp_fgemm_wino(int(transA), int(transB), m, n, k, p, alpha, a, lda, b, ldb, beta, c, ldc, path,
                              levels, ws, need, _stream(C)), "ffp_fgemm_wino")
    return C


def ftrsm(side: int, uplo: int, trans: int, diag: int, T, B, p: int, alpha: int = 1, path: int = PATH_AUTO):
    """Triangular solve in place on B (see include/ffpluq.h); returns B."""
    lib = load()
    t, ldt = _mat(T, "T")
    b, ldb = _mat(B, "B")
    m, n = B.shape
    d = m if side == 0 else n
    if T.shape[0] < d or T.shape[1] < d:
        raise ValueError("ftrsm: T too small")
    need = lib.ffp_ftrsm_workspace(side, uplo, trans, diag, m, n, p, path)
    keep, ws = _workspace(need, B.device)
    _check(lib.ffp_ftrsm(side, uplo, trans, diag, m, n, p, alpha, t, ldt, b, ldb, path, ws, need,
                         _stream(B)), "ffp_ftrsm")
    return B


def flaswp(dim: int, A, perm, inverse: bool = False):
    """Permute rows (dim 0) or columns (dim 1) of A in place; returns A."""
    lib = load()
    a, lda = _mat(A, "A")
    m, n = A.shape
    pv = _vec(perm, "perm")
    if perm.numel() != (m if dim == 0 else n):
        raise ValueError("flaswp: permutation length")
    need = lib.ffp_flaswp_workspace(dim, m, n)
    keep, ws = _workspace(need, A.device)
    _check(lib.ffp_flaswp(dim, m, n, a, lda, pv, int(inverse), ws, need, _stream(A)), "ffp_flaswp")
    return A


@dataclass
class PLUQResult:
    LU: object   # the input tensor, now holding L\U
    P: object    # int32[m] device
    Q: object    # int32[n] device
    rank: int
    rrp: object  # int32[rank] device (sorted row rank profile)
    crp: object  # int32[rank] device (sorted column rank profile)


def pluq(A, p: int, path: int = PATH_AUTO) -> PLUQResult:
    """Rank-profile-revealing PLUQ of A (in place).  Synchronises the stream."""
    torch = _torch()
    lib = load()
    a, lda = _mat(A, "A")
    m, n = A.shape
    dev = A.device
    P = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    k = max(min(m, n), 1)
    rrp = torch.empty(k, dtype=torch.int32, device=dev)
    crp = torch.empty(k, dtype=torch.int32, device=dev)
    rdev = torch.empty(1, dtype=torch.int64, device=dev)
    need = lib.ffp_pluq_workspace(m, n, p, path)
    keep, ws = _workspace(need, dev)
    r = ctypes.c_int64(-1)
    _check(lib.ffp_pluq(m, n, p, a, lda, _vec(P, "P"), _vec(Q, "Q"), _vec(rdev, "rank", torch.int64),
                        ctypes.byref(r), _vec(rrp, "rrp"), _vec(crp, "crp"), path, ws, need, _stream(A)),
           "ffp_pluq")
    r = int(r.value)
    return PLUQResult(A, P[:m], Q[:n], r, rrp[:r], crp[:r])


def pluq_slab(A, p: int, path: int = PATH_AUTO) -> PLUQResult:
    """Slab-recursive PLUQ of A in place (pivots in row order).  Synchronises."""
    torch = _torch()
    lib = load()
    a, lda = _mat(A, "A")
    m, n = A.shape
    dev = A.device
    P = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    k = max(min(m, n), 1)
    rrp = torch.empty(k, dtype=torch.int32, device=dev)
    crp = torch.empty(k, dtype=torch.int32, device=dev)
    need = lib.ffp_pluq_slab_workspace(m, n, p, path)
    keep, ws = _workspace(need, dev)
    r = ctypes.c_int64(-1)
    _check(lib.ffp_pluq_slab(m, n, p, a, lda, _vec(P, "P"), _vec(Q, "Q"), None, ctypes.byref(r), _vec(rrp, "rrp"),
                             _vec(crp, "crp"), path, ws, need, _stream(A)), "ffp_pluq_slab")
    r = int(r.value)
    return PLUQResult(A, P[:m], Q[:n], r, rrp[:r], crp[:r])


def pluq_workspace(m: int, n: int, p: int, path: int = PATH_AUTO) -> int:
    return int(load().ffp_pluq_workspace(m, n, p, path))


def pluq_into(A, p: int, P, Q, rank_dev, rrp, crp, ws, path: int = PATH_AUTO) -> int:
    """PLUQ with caller-provided outputs and workspace (no allocation); returns the rank."""
    lib = load()
    a, lda = _mat(A, "A")
    m, n = A.shape
    r = ctypes.c_int64(-1)
    _check(lib.ffp_pluq(m, n, p, a, lda, _vec(P, "P"), _vec(Q, "Q"),
                        _vec(rank_dev, "rank", rank_dev.dtype) if rank_dev is not None else None,
                        ctypes.byref(r), _vec(rrp, "rrp") if rrp is not None else None,
                        _vec(crp, "crp") if crp is not None else None, path,
                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(A)), "ffp_pluq")
    return int(r.value)


def lu_nopiv(A, p: int, info=None, ws=None, path: int = PATH_AUTO):
    """Plain LU in place for an input of generic rank profile (no host
    synchronisation).  Returns the device int32 ``info``: 0 when every pivot
    was nonzero, else 1 + the diagonal index of the first zero pivot."""
    torch = _torch()
    lib = load()
    a, lda = _mat(A, "A")
    m, n = A.shape
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    need = lib.ffp_lu_nopiv_workspace(m, n, p, path)
    if ws is None:
        keep, wsp = _workspace(need, A.device)
        wsz = need
    else:
        keep, wsp, wsz = ws, ctypes.c_void_p(ws.data_ptr()), ws.numel()
    _check(lib.ffp_lu_nopiv(m, n, p, a, lda, _vec(info, "info"), path, wsp, wsz, _stream(A)), "ffp_lu_nopiv")
    return info


def lu_nopiv_workspace(m: int, n: int, p: int, path: int = PATH_AUTO) -> int:
    return int(load().ffp_lu_nopiv_workspace(m, n, p, path))


LU_RIGHT, LU_CROUT, LU_LEFT, LU_TILE_RECURSIVE, LU_SLAB_RECURSIVE = 0, 1, 2, 3, 4


def lu_tiled(A, p: int, variant: int, k: int, info=None, ws=None, path: int = PATH_AUTO):
    """Tile-iterative LU in place (right-looking, Crout or left-looking, tile
    k) for an input of generic rank profile; returns the device int32 info
    (0, or 1 + the index of the first zero pivot).  No host synchronisation."""
    torch = _torch()
    lib = load()
    a, lda = _mat(A, "A")
    m, n = A.shape
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    need = lib.ffp_lu_tiled_workspace(variant, m, n, k, p, path)
    if ws is None:
        keep, wsp = _workspace(need, A.device)
        wsz = need
    else:
        keep, wsp, wsz = ws, ctypes.c_void_p(ws.data_ptr()), ws.numel()
    _check(lib.ffp_lu_tiled(variant, m, n, p, a, lda, k, _vec(info, "info"), path, wsp, wsz, _stream(A)),
           "ffp_lu_tiled")
    return info


def lu_tiled_workspace(variant: int, m: int, n: int, k: int, p: int, path: int = PATH_AUTO) -> int:
    return int(load().ffp_lu_tiled_workspace(variant, m, n, k, p, path))


def reduction_count(algorithm: int, n: int, k: int = 1) -> float:
    """Modular reductions the model of Section 3.1 charges an n x n LU (host only)."""
    c = ctypes.c_double(0.0)
    _check(load().ffp_reduction_count(algorithm, n, k, ctypes.byref(c)), "ffp_reduction_count")
    return c.value


def echelon(res: "PLUQResult", p: int, form: int = 0, path: int = PATH_AUTO):
    """Reduced row (form 0: r x n) or column (form 1: m x r) echelon form of
    the matrix factored in ``res`` (output of ``pluq``), as a new tensor."""
    torch = _torch()
    lib = load()
    a, lda = _mat(res.LU, "LU")
    m, n = res.LU.shape
    r = res.rank
    E = torch.empty((r, n) if form == 0 else (m, r), dtype=torch.int32, device=res.LU.device)
    if r == 0:
        return E
    e, lde = _mat(E, "E")
    need = lib.ffp_echelon_workspace(form, m, n, r, p, path)
    keep, ws = _workspace(need, E.device)
    _check(lib.ffp_echelon(form, m, n, p, a, lda, _vec(res.P, "P"), _vec(res.Q, "Q"), r, e, lde, path, ws, need,
                           _stream(E)), "ffp_echelon")
    return E


def nullspace(res: "PLUQResult", p: int, side: int = 0, path: int = PATH_AUTO):
    """Right (side 0: A N = 0, n x (n - r)) or left (side 1: N A = 0,
    (m - r) x m) nullspace basis, identity on the non-pivot columns / rows."""
    torch = _torch()
    lib = load()
    a, lda = _mat(res.LU, "LU")
    m, n = res.LU.shape
    r = res.rank
    shape = (n, n - r) if side == 0 else (m - r, m)
    N = torch.zeros(shape, dtype=torch.int32, device=res.LU.device)
    if N.numel() == 0:
        return N
    nn, ldn = _mat(N, "N")
    need = lib.ffp_nullspace_workspace(side, m, n, r, p, path)
    keep, ws = _workspace(need, N.device)
    _check(lib.ffp_nullspace(side, m, n, p, a, lda, _vec(res.P, "P"), _vec(res.Q, "Q"), r, nn, ldn, path, ws,
                             need, _stream(N)), "ffp_nullspace")
    return N


def solve(res: "PLUQResult", B, p: int, path: int = PATH_AUTO):
    """A X = B from the factorisation in ``res``: returns (X, consistent) with
    X (n x nrhs) zero off the pivot columns and consistent an int32 flag per
    column of B."""
    torch = _torch()
    lib = load()
    a, lda = _mat(res.LU, "LU")
    m, n = res.LU.shape
    b, ldb = _mat(B, "B")
    nrhs = B.shape[1]
    X = torch.zeros((n, nrhs), dtype=torch.int32, device=B.device)
    ok = torch.zeros(max(nrhs, 1), dtype=torch.int32, device=B.device)
    if nrhs == 0:
        return X, ok[:0]
    x, ldx = _mat(X, "X")
    need = lib.ffp_solve_workspace(m, n, res.rank, nrhs, p, path)
    keep, ws = _workspace(need, B.device)
    _check(lib.ffp_solve(m, n, p, a, lda, _vec(res.P, "P"), _vec(res.Q, "Q"), res.rank, nrhs, b, ldb, x, ldx,
                         _vec(ok, "consistent"), path, ws, need, _stream(B)), "ffp_solve")
    return X, ok[:nrhs]


def check_range(A, p: int) -> bool:
    """True when every entry of A lies in [0, p) (synchronises)."""
    a, lda = _mat(A, "A")
    m, n = A.shape
    rc = load().ffp_check_range(m, n, p, a, lda, _stream(A))
    if rc == -105:
        return False
    _check(rc, "ffp_check_range")
    return True


@dataclass
class BatchedResult:
    P: object
    Q: object
    rank: object
    rrp: object
    crp: object


def pluq_batched(ms, ns, A_packed, A_off, p: int, path: int = PATH_AUTO, max_m: int | None = None,
                 max_n: int | None = None) -> BatchedResult:
    """Factor many packed row-major matrices in one persistent launch (in place on A_packed).

    ms, ns, A_off: device tensors (int32, int32, int64).  Returns device outputs;
    P/Q/rrp/crp are packed at the exclusive prefix sums of ms / ns."""
    torch = _torch()
    lib = load()
    dev = A_packed.device
    batch = int(ms.numel())
    ms_h = ms.cpu().to(torch.int64)
    ns_h = ns.cpu().to(torch.int64)
    max_m = int(ms_h.max()) if max_m is None and batch else (max_m or 0)
    max_n = int(ns_h.max()) if max_n is None and batch else (max_n or 0)
    P_off = torch.zeros(batch, dtype=torch.int64)
    Q_off = torch.zeros(batch, dtype=torch.int64)
    if batch > 1:
        P_off[1:] = torch.cumsum(ms_h, 0)[:-1]
        Q_off[1:] = torch.cumsum(ns_h, 0)[:-1]
    tm, tn = int(ms_h.sum()), int(ns_h.sum())
    P_off, Q_off = P_off.to(dev), Q_off.to(dev)
    P = torch.empty(max(tm, 1), dtype=torch.int32, device=dev)
    Q = torch.empty(max(tn, 1), dtype=torch.int32, device=dev)
    rrp = torch.empty(max(tm, 1), dtype=torch.int32, device=dev)
    crp = torch.empty(max(tn, 1), dtype=torch.int32, device=dev)
    rank = torch.empty(max(batch, 1), dtype=torch.int32, device=dev)
    need = lib.ffp_pluq_batched_workspace(batch, max_m, max_n, p, path)
    keep, ws = _workspace(need, dev)
    _check(lib.ffp_pluq_batched(batch, _vec(ms, "ms"), _vec(ns, "ns"), max_m, max_n, p,
                                _vec(A_packed, "A_packed"), _vec(A_off, "A_off", torch.int64),
                                _vec(P, "P"), _vec(P_off, "P_off", torch.int64), _vec(Q, "Q"),
                                _vec(Q_off, "Q_off", torch.int64), _vec(rank, "rank"), _vec(rrp, "rrp"),
                                _vec(crp, "crp"), path, ws, need, _stream(A_packed)), "ffp_pluq_batched")
    return BatchedResult(P, Q, rank[:batch], rrp, crp)


def pluq_batched_tune(ms, ns, A_packed, A_off, p: int, path: int = PATH_AUTO):
    """Time each batched launch shape on this batch (restoring it in between),
    keep the fastest for later calls on batches of the same description, and
    leave the batch factored.  Returns (BatchedResult, chosen shape, list of
    per-shape milliseconds).  Synchronises."""
    torch = _torch()
    lib = load()
    dev = A_packed.device
    batch = int(ms.numel())
    ms_h = ms.cpu().to(torch.int64)
    ns_h = ns.cpu().to(torch.int64)
    max_m = int(ms_h.max()) if batch else 0
    max_n = int(ns_h.max()) if batch else 0
    P_off = torch.zeros(batch, dtype=torch.int64)
    Q_off = torch.zeros(batch, dtype=torch.int64)
    if batch > 1:
        P_off[1:] = torch.cumsum(ms_h, 0)[:-1]
        Q_off[1:] = torch.cumsum(ns_h, 0)[:-1]
    tm, tn = int(ms_h.sum()), int(ns_h.sum())
    P_off, Q_off = P_off.to(dev), Q_off.to(dev)
    P = torch.empty(max(tm, 1), dtype=torch.int32, device=dev)
    Q = torch.empty(max(tn, 1), dtype=torch.int32, device=dev)
    rrp = torch.empty(max(tm, 1), dtype=torch.int32, device=dev)
    crp = torch.empty(max(tn, 1), dtype=torch.int32, device=dev)
    rank = torch.empty(max(batch, 1), dtype=torch.int32, device=dev)
    a_elems = int(A_packed.numel())
    need = lib.ffp_pluq_batched_tune_workspace(batch, max_m, max_n, a_elems)
    keep, ws = _workspace(need, dev)
    shape = ctypes.c_int(-1)
    times = (ctypes.c_float * 8)()
    _check(lib.ffp_pluq_batched_tune(batch, _vec(ms, "ms"), _vec(ns, "ns"), max_m, max_n, p,
                                     _vec(A_packed, "A_packed"), a_elems, _vec(A_off, "A_off", torch.int64),
                                     _vec(P, "P"), _vec(P_off, "P_off", torch.int64), _vec(Q, "Q"),
                                     _vec(Q_off, "Q_off", torch.int64), _vec(rank, "rank"), _vec(rrp, "rrp"),
                                     _vec(crp, "crp"), path, ctypes.byref(shape), times, ws, need,
                                     _stream(A_packed)), "ffp_pluq_batched_tune")
    return BatchedResult(P, Q, rank[:batch], rrp, crp), shape.value, [times[i] for i in range(BATCH_SHAPES)]


def pluq_batched_set_shape(batch: int, max_m: int, max_n: int, shape: int) -> None:
    """Use launch shape ``shape`` for later batched calls of this description."""
    _check(load().ffp_pluq_batched_set_shape(batch, max_m, max_n, shape), "ffp_pluq_batched_set_shape")


def pluq_batched_into(ms, ns, max_m: int, max_n: int, A_packed, A_off, P, P_off, Q, Q_off, rank, rrp, crp,
                      ws, p: int, path: int = PATH_AUTO) -> None:
    """The batched factorisation into caller-provided outputs and workspace:
    no allocation and no host synchronisation (two kernel launches on the
    current stream), so the call can be captured in a graph."""
    torch = _torch()
    lib = load()
    batch = int(ms.numel())
    _check(lib.ffp_pluq_batched(batch, _vec(ms, "ms"), _vec(ns, "ns"), max_m, max_n, p,
                                _vec(A_packed, "A_packed"), _vec(A_off, "A_off", torch.int64),
                                _vec(P, "P"), _vec(P_off, "P_off", torch.int64), _vec(Q, "Q"),
                                _vec(Q_off, "Q_off", torch.int64), _vec(rank, "rank"),
                                _vec(rrp, "rrp") if rrp is not None else None,
                                _vec(crp, "crp") if crp is not None else None, path,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(A_packed)),
           "ffp_pluq_batched")


def perm_to_swaps(perm) -> np.ndarray:
    perm = np.ascontiguousarray(perm, np.int32)
    ipiv = np.zeros(max(len(perm), 1), np.int32)
    _check(load().ffp_perm_to_swaps(len(perm), perm.ctypes.data_as(ctypes.c_void_p),
                                    ipiv.ctypes.data_as(ctypes.c_void_p)), "ffp_perm_to_swaps")
    return ipiv[:len(perm)]


def swaps_to_perm(ipiv) -> np.ndarray:
    ipiv = np.ascontiguousarray(ipiv, np.int32)
    perm = np.zeros(max(len(ipiv), 1), np.int32)
    _check(load().ffp_swaps_to_perm(len(ipiv), ipiv.ctypes.data_as(ctypes.c_void_p),
                                    perm.ctypes.data_as(ctypes.c_void_p)), "ffp_swaps_to_perm")
    return perm[:len(ipiv)]


def profile_enable(on: bool = True):
    _check(load().ffp_profile_enable(int(on)), "ffp_profile_enable")


def profile_reset():
    _check(load().ffp_profile_reset(), "ffp_profile_reset")


def profile_read(path: int):
    """(launches, milliseconds, field_ops) accumulated for the dense product kernels of a path."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0)
    ops = ctypes.c_double(0)
    _check(load().ffp_profile_read(path, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(ops)),
           "ffp_profile_read")
    return int(n.value), float(ms.value), float(ops.value)


PROFILE_KINDS = 11


def profile_kind_name(kind: int) -> str:
    name = load().ffp_profile_kind_name(kind)
    return name.decode() if name else ""


def profile_read_all() -> dict:
    """{kind name: (launches, milliseconds, field_ops, bytes)} of every kernel
    family with at least one timed launch."""
    out = {}
    for kind in range(1, PROFILE_KINDS):
        n, ms, ops = profile_read(kind)
        if n:
            out[profile_kind_name(kind)] = (n, ms, ops, profile_read_bytes(kind))
    return out


def profile_read_bytes(path: int) -> float:
    """Algorithmic bytes (operands read once, result written once) of the same launches."""
    b = ctypes.c_double(0)
    _check(load().ffp_profile_read_bytes(path, ctypes.byref(b)), "ffp_profile_read_bytes")
    return float(b.value)
