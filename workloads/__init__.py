"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module only *generates* inputs: sparsity patterns, matrix values and dense
feature matrices.  It holds none of the method's arithmetic (no products, no
decomposition, no norms), so that the oracle and the HIP path can both consume
its output without sharing any computation.

The paper evaluates on large SuiteSparse graphs (Section 7, Table 2).  Those
are not available here; seeded generators with the same structure stand in:

* 2D 5-point and 3D 7-point grids (low degree, small bandwidth in natural
  order) for the road-network / k-mer style matrices,
* R-MAT graphs with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) for the skewed
  web / social / traffic graphs.

All matrices are square CSR with int64 row pointers, int32 sorted unique
column indices and float32 values.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz], sorted and unique within each row
    val: np.ndarray      # float32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64[nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))


# ---------------------------------------------------------------------------
# sparsity patterns
# ---------------------------------------------------------------------------

def _pattern_from_keys(n: int, keys: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Sorted unique int64 keys row*n+col -> (row_ptr int64, col int32)."""
    keys = np.unique(keys)
    rows = keys // n
    col = (keys - rows * n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr, col


def _stencil_pattern(n: int, offsets, valid) -> tuple[np.ndarray, np.ndarray]:
    """CSR of a stencil: row v holds v + off for every offset whose mask is set.
    Offsets are ascending, so columns come out sorted without a sort."""
    v = np.arange(n, dtype=np.int64)
    cols = np.stack([v + off for off in offsets], axis=1)
    mask = np.stack(valid, axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    return row_ptr, cols[mask].astype(np.int32)


def grid2d_pattern(side: int, diagonal: bool = True) -> tuple[int, np.ndarray, np.ndarray]:
    """5-point stencil on a side x side grid, vertex id = y*side + x (natural order)."""
    n = side * side
    v = np.arange(n, dtype=np.int64)
    x = v % side
    offs = [-side, -1, 0, 1, side]
    valid = [v >= side, x > 0, np.full(n, diagonal), x < side - 1, v < n - side]
    row_ptr, col = _stencil_pattern(n, offs, valid)
    return n, row_ptr, col


def grid3d_pattern(side: int, diagonal: bool = True) -> tuple[int, np.ndarray, np.ndarray]:
    """7-point stencil on a side^3 grid, vertex id = (z*side + y)*side + x."""
    n = side ** 3
    s2 = side * side
    v = np.arange(n, dtype=np.int64)
    x = v % side
    y = (v // side) % side
    z = v // s2
    offs = [-s2, -side, -1, 0, 1, side, s2]
    valid = [z > 0, y > 0, x > 0, np.full(n, diagonal), x < side - 1, y < side - 1,
             z < side - 1]
    row_ptr, col = _stencil_pattern(n, offs, valid)
    return n, row_ptr, col


def rmat_pattern(scale: int, avg_degree: float, seed: int,
                 probs=(0.57, 0.19, 0.19, 0.05), relabel: bool = True,
                 chunk: int = 1 << 23) -> tuple[int, np.ndarray, np.ndarray]:
    """R-MAT graph with n = 2**scale vertices.

    Draws avg_degree/2 * n directed edges by recursive quadrant choice (no
    per-level noise), relabels vertices by a seeded random permutation,
    symmetrises, drops self loops and duplicates.  The resulting number of
    stored entries is below avg_degree * n because of duplicates.
    """
    n = 1 << scale
    m = int(round(avg_degree / 2 * n))
    rng = np.random.default_rng(seed)
    a, b, c, _ = probs
    t1, t2, t3 = a, a + b, a + b + c
    keys = []
    perm = rng.permutation(n).astype(np.int64) if relabel else None
    for start in range(0, m, chunk):
        cnt = min(chunk, m - start)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(cnt, dtype=np.float32)
            ub = r >= t2                      # quadrants c, d -> lower half
            vb = ((r >= t1) & (r < t2)) | (r >= t3)  # quadrants b, d -> right half
            u = (u << 1) | ub
            v = (v << 1) | vb
        if perm is not None:
            u = perm[u]
            v = perm[v]
        keep = u != v
        u = u[keep]
        v = v[keep]
        keys.append(u * n + v)
        keys.append(v * n + u)
    row_ptr, col = _pattern_from_keys(n, np.concatenate(keys))
    return n, row_ptr, col


# ---------------------------------------------------------------------------
# values
# ---------------------------------------------------------------------------

def values_uniform(row_ptr: np.ndarray, seed: int) -> np.ndarray:
    """Each stored entry independently U[-1, 1] (float32)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, int(row_ptr[-1])).astype(np.float32)


def values_sym_laplacian(n: int, row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """Symmetric normalised Laplacian I - D^{-1/2} A D^{-1/2} on the pattern.

    Degrees count off-diagonal entries.  The diagonal entry is 1 for a vertex
    with at least one neighbour and 0 otherwise; the off-diagonal entry (u, v)
    is -1/sqrt(d_u d_v).  Computed in float64, stored rounded to float32.
    """
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    off = rows != col
    deg = np.bincount(rows[off], minlength=n).astype(np.float64)
    val = np.zeros(rows.shape[0], dtype=np.float64)
    d_r = deg[rows[off]]
    d_c = deg[col[off]]
    val[off] = -1.0 / np.sqrt(d_r * d_c)
    diag = ~off
    val[diag] = (deg[rows[diag]] > 0).astype(np.float64)
    return val.astype(np.float32)


def values_row_normalized(n: int, row_ptr: np.ndarray) -> np.ndarray:
    """Every entry of row u equals 1/deg(u) (float32); empty rows stay empty."""
    deg = np.diff(row_ptr).astype(np.float64)
    w = np.zeros(n, dtype=np.float64)
    nz = deg > 0
    w[nz] = 1.0 / deg[nz]
    return np.repeat(w, np.diff(row_ptr)).astype(np.float32)


def features(n: int, k: int, seed: int) -> np.ndarray:
    """Dense row-major n x k feature matrix, entries N(0, 1), float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, k), dtype=np.float32)


# ---------------------------------------------------------------------------
# workload presets (the five evaluated configurations)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    graph: str          # "grid2d" | "grid3d" | "rmat"
    size: int           # side for grids, scale for R-MAT
    values: str         # "uniform" | "sym_laplacian" | "row_normalized"
    k: int
    b: int
    iters: int
    tag: int            # seed offset of the configuration
    avg_degree: float = 16.0
    dtypes: tuple = ("f32",)

    @property
    def seeds(self) -> dict:
        return dict(graph=1000 + self.tag, values=2000 + self.tag,
                    x=3000 + self.tag, decompose=4000 + self.tag)

    def describe(self) -> str:
        if self.graph == "grid2d":
            g = f"2D 5-point grid {self.size}x{self.size}"
        elif self.graph == "grid3d":
            g = f"3D 7-point grid {self.size}^3"
        else:
            g = f"R-MAT 2^{self.size} avg degree {self.avg_degree:g}"
        return f"{g}, {self.values} values, k={self.k}, b={self.b}, {self.iters} iterations"


WORKLOADS = {
    "grid64": Workload("grid64", "grid2d", 64, "uniform", 16, 64, 10, 1),
    "grid2048": Workload("grid2048", "grid2d", 2048, "sym_laplacian", 32, 2048, 20, 2),
    "rmat22": Workload("rmat22", "rmat", 22, "row_normalized", 64, 4096, 10, 3),
    "grid3d160": Workload("grid3d160", "grid3d", 160, "sym_laplacian", 128, 4096, 50, 4,
                          dtypes=("bf16", "f8e4m3")),
    "rmat22_k128": Workload("rmat22_k128", "rmat", 22, "row_normalized", 128, 4096, 50, 4,
                            dtypes=("bf16", "f8e4m3")),
}


def make_matrix(graph: str, size: int, values: str, seed_graph: int, seed_values: int,
                avg_degree: float = 16.0) -> CSR:
    if graph == "grid2d":
        n, row_ptr, col = grid2d_pattern(size)
    elif graph == "grid3d":
        n, row_ptr, col = grid3d_pattern(size)
    elif graph == "rmat":
        n, row_ptr, col = rmat_pattern(size, avg_degree, seed_graph)
    else:
        raise ValueError(f"unknown graph kind {graph!r}")
    if values == "uniform":
        val = values_uniform(row_ptr, seed_values)
    elif values == "sym_laplacian":
        val = values_sym_laplacian(n, row_ptr, col)
    elif values == "row_normalized":
        val = values_row_normalized(n, row_ptr)
    else:
        raise ValueError(f"unknown value kind {values!r}")
    return CSR(n, row_ptr, col, val)


def workload_matrix(w: Workload) -> CSR:
    s = w.seeds
    return make_matrix(w.graph, w.size, w.values, s["graph"], s["values"], w.avg_degree)


def workload_features(w: Workload, n: int, k: Optional[int] = None) -> np.ndarray:
    return features(n, k or w.k, w.seeds["x"])


def random_graph(n: int, p: float, seed: int, values: str = "uniform",
                 diagonal: bool = False) -> CSR:
    """Symmetric Erdos-Renyi pattern (for small tests), optional diagonal."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    u = iu[keep].astype(np.int64)
    v = ju[keep].astype(np.int64)
    parts = [u * n + v, v * n + u]
    if diagonal:
        d = np.arange(n, dtype=np.int64)
        parts.append(d * n + d)
    row_ptr, col = _pattern_from_keys(n, np.concatenate(parts)) if n else (
        np.zeros(1, np.int64), np.zeros(0, np.int32))
    if values == "uniform":
        val = values_uniform(row_ptr, seed + 1)
    elif values == "ones":
        val = np.ones(int(row_ptr[-1]), np.float32)
    else:
        raise ValueError(values)
    return CSR(n, row_ptr, col, val)


def from_edges(n: int, edges, values: str = "ones", seed: int = 0,
               diagonal: bool = False, symmetric: bool = True) -> CSR:
    """CSR from an explicit undirected (or directed) edge list."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    parts = [e[:, 0] * n + e[:, 1]]
    if symmetric:
        parts.append(e[:, 1] * n + e[:, 0])
    if diagonal:
        d = np.arange(n, dtype=np.int64)
        parts.append(d * n + d)
    keys = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    row_ptr, col = _pattern_from_keys(n, keys)
    if values == "ones":
        val = np.ones(int(row_ptr[-1]), np.float32)
    else:
        val = values_uniform(row_ptr, seed)
    return CSR(n, row_ptr, col, val)
