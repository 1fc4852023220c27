"""ORACLE (test infrastructure only): Y = A X in FP64, its renormalised
iteration and the GNN-style step ReLU((A X) W).

Parity status: pinned.  The CSR product is checked against a pure-Python
triple loop on tiny inputs, against a dense product on small inputs, and
against closed forms at full size (Laplacian null vector, row-stochastic
matrices, identity).  The iteration is checked against closed-form power
iterations (diagonal matrices, path-graph eigenvectors).  The GNN step is
checked against pure-Python loops and against permutation and diagonal
weight matrices, whose products are known column by column.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_f64.c")
_LIB = os.path.join(_HERE, "_csr_f64.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_csr_spmm_f64.argtypes = [i64, p, p, p, p, i64, p]
        lib.oracle_csr_spmm_rows_f64.argtypes = [p, p, p, p, i64, p, i64, p]
        lib.oracle_col_sumsq_f64.argtypes = [i64, i64, p, p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the oracle's row loops (for timing it on fewer cores)."""
    _load().oracle_set_num_threads(int(t))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check_csr(csr):
    row_ptr = np.ascontiguousarray(csr.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(csr.col, dtype=np.int32)
    val = np.ascontiguousarray(csr.val, dtype=np.float32)
    return row_ptr, col, val


def csr_spmm(csr, X) -> np.ndarray:
    """FP64 Y = A X. X is converted exactly to float64 (it may be f32/f64)."""
    row_ptr, col, val = _check_csr(csr)
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = csr.n
    k = X.shape[1] if X.ndim == 2 else 1
    X = X.reshape(n, k)
    Y = np.empty((n, k), dtype=np.float64)
    if n:
        _load().oracle_csr_spmm_f64(n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(X), k, _ptr(Y))
    return Y


def csr_spmm_rows(csr, X, rows) -> np.ndarray:
    """FP64 rows of A X: out[r] = (A X)[rows[r]]."""
    row_ptr, col, val = _check_csr(csr)
    X = np.ascontiguousarray(X, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    k = X.shape[1]
    Y = np.empty((rows.shape[0], k), dtype=np.float64)
    if rows.shape[0]:
        _load().oracle_csr_spmm_rows_f64(_ptr(row_ptr), _ptr(col), _ptr(val), _ptr(X), k,
                                         _ptr(rows), rows.shape[0], _ptr(Y))
    return Y


def col_sumsq(Y) -> np.ndarray:
    """Per-column sum of squares, sequential over rows, FP64."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    n, k = Y.shape
    out = np.empty(k, dtype=np.float64)
    _load().oracle_col_sumsq_f64(n, k, _ptr(Y), _ptr(out))
    return out


def brute_force(csr, X) -> list:
    """Pure-Python triple loop over the CSR definition (tiny inputs only)."""
    n = csr.n
    k = len(X[0]) if n else 0
    Y = [[0.0] * k for _ in range(n)]
    rp = [int(v) for v in csr.row_ptr]
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            a = float(csr.val[p])
            c = int(csr.col[p])
            for j in range(k):
                Y[i][j] += a * float(X[c][j])
    return Y


def dense(csr) -> np.ndarray:
    """The matrix as a dense FP64 array (small inputs)."""
    A = np.zeros((csr.n, csr.n), dtype=np.float64)
    A[csr.rows(), csr.col.astype(np.int64)] = csr.val.astype(np.float64)
    return A


def renormalize(Y) -> tuple[np.ndarray, np.ndarray]:
    """sigma of the iteration: per-column 2-norm nu and X_next = Y / nu (0 if nu == 0)."""
    nu = np.sqrt(col_sumsq(Y))
    inv = np.zeros_like(nu)
    nz = nu > 0
    inv[nz] = 1.0 / nu[nz]
    return nu, Y * inv[None, :]


def iterate(csr, X0, T: int):
    """Free-running FP64 iteration X_{t+1} = Y_t / ||Y_t||_col with Y_t = A X_t.

    Returns (Ys, nus): the un-normalised products Y_t and their column norms.
    """
    X = np.asarray(X0, dtype=np.float64)
    Ys, nus = [], []
    for _ in range(T):
        Y = csr_spmm(csr, X)
        nu, X = renormalize(Y)
        Ys.append(Y)
        nus.append(nu)
    return Ys, nus


def gnn_layer(csr, X, W) -> np.ndarray:
    """One step of the GNN-style iteration (Section 2: sigma an element-wise
    function, here with a k x k weight matrix): Z = ReLU((A X) W) in FP64.
    A X is the CSR product above; the k x k product is a library matmul."""
    Y = csr_spmm(csr, X)
    return np.maximum(Y @ np.asarray(W, dtype=np.float64), 0.0)


def gnn_brute_force(csr, X, W) -> list:
    """Pure-Python loops of ReLU((A X) W) (tiny inputs only)."""
    Y = brute_force(csr, X)
    k = len(W)
    out = []
    for row in Y:
        z = []
        for j in range(k):
            acc = 0.0
            for i in range(k):
                acc += row[i] * float(W[i][j])
            z.append(acc if acc > 0.0 else 0.0)
        out.append(z)
    return out


def rel_fro(a, ref) -> float:
    """Relative Frobenius error ||a - ref||_F / ||ref||_F (0/0 -> 0)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(ref * ref)))
    num = float(np.sqrt(np.sum((a - ref) ** 2)))
    if den == 0.0:
        return num
    return num / den
