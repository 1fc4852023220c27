"""Python binding of libarrow: the arrow-decomposition SpMM for MI355X (gfx950).

Argument marshalling only: every step runs in the C++ host code or the HIP
kernels of ``libarrow.so``.  PyTorch supplies device memory and streams.

Paper: Gianinazzi et al., "Arrow Matrix Decomposition: A Novel Approach for
Communication-Efficient Sparse Matrix Multiplication", PPoPP 2024.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarrow.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_UNSUPPORTED, ERR_IO, ERR_INTERNAL = range(7)
F32, F16, BF16, F8E4M3 = 0, 1, 2, 3
LA_RANDOM_FOREST, LA_IDENTITY, LA_SEPARATOR = 0, 1, 2
KERNEL_CHUNKS, KERNEL_UPPER, KERNEL_LEVEL0, KERNEL_NORM, KERNEL_PERMUTE, KERNEL_COMBINE = range(6)
KERNEL_NAMES = {KERNEL_CHUNKS: "chunks", KERNEL_UPPER: "upper", KERNEL_COMBINE: "combine",
                KERNEL_LEVEL0: "level0", KERNEL_NORM: "norm", KERNEL_PERMUTE: "permute"}
ITER_RENORM = 1
STATIC_WORKSPACE_BYTES = 64 << 20

DTYPES = {"f32": F32, "f16": F16, "bf16": BF16, "f8e4m3": F8E4M3}
ELEM_SIZE = {F32: 4, F16: 2, BF16: 2, F8E4M3: 1}


class ArrowError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libarrow.so is not built ({LIB_PATH}); run "
                          "`python -m paper_2402_19364_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, U64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t)
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "arrow_decompose": [I64, P, P, P, P, pp],
        "arrow_decomp_info": [P, P],
        "arrow_decomp_level": [P, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), pp, pp, pp, pp],
        "arrow_decomp_save": [P, ctypes.c_char_p],
        "arrow_decomp_load": [ctypes.c_char_p, pp],
        "arrow_plan_create": [P, I32, P, pp],
        "arrow_set_allocator": [P, P, P],
        "arrow_plan_info": [P, P],
        "arrow_plan_footprint": [P, ctypes.POINTER(SZ)],
        "arrow_decomp_level_stats": [P, I32, P],
        "arrow_decomp_block_stats": [P, I32, I32, I32, P],
        "arrow_plan_kernel_bytes": [P, I32, I64, I32, ctypes.POINTER(I64)],
        "arrow_workspace_size": [P, I64, I32, ctypes.POINTER(SZ)],
        "arrow_iterate_workspace_size": [P, I64, I32, ctypes.POINTER(SZ)],
        "arrow_permute_in": [P, P, I64, P, I64, I32, I64, P, P, P],
        "arrow_permute_out": [P, P, I64, I32, I64, P, P, P, I64, P],
        "arrow_spmm": [P, P, I32, P, SZ, P],
        "arrow_spmm_static": [P, P, I32, P],
        "arrow_spmm_iterate": [P, P, P, I64, I64, I32, P, P, I32, U32, P, P, SZ, P],
        "arrow_csr_workspace_size": [I64, I64, ctypes.POINTER(SZ)],
        "arrow_csr_batch": [I64, P, ctypes.POINTER(I32)],
        "arrow_csr_spmm": [I64, P, P, P, P, P, I64, I64, I32, P, P, P],
        "arrow_plan_set_batch": [P, I32, I32],
        "arrow_copy": [P, P, I64, P],
        "arrow_profile_enable": [P, I32],
        "arrow_profile_query": [P, I32, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double)],
        "arrow_rocsparse_create": [I64, I64, P, P, P, P, P, I64, I64, I32, P, pp],
        "arrow_rocsparse_run": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I32
    lib.arrow_decomp_destroy.argtypes = [P]
    lib.arrow_decomp_destroy.restype = None
    lib.arrow_plan_destroy.argtypes = [P]
    lib.arrow_plan_destroy.restype = None
    lib.arrow_rocsparse_destroy.argtypes = [P]
    lib.arrow_rocsparse_destroy.restype = None
    for name in ("arrow_status_string",):
        getattr(lib, name).argtypes = [I32]
        getattr(lib, name).restype = ctypes.c_char_p
    lib.arrow_last_error.argtypes = []
    lib.arrow_last_error.restype = ctypes.c_char_p
    lib.arrow_version.argtypes = []
    lib.arrow_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def lib():
    return _load()


def _check(status: int):
    if status != OK:
        msg = _load().arrow_last_error().decode(errors="replace")
        raise ArrowError(status, msg)


class _DecompOpts(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("la", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("max_levels", ctypes.c_int32), ("threads", ctypes.c_int32)]


class _DecompInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("b", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("seconds", ctypes.c_double)]


class _LevelStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n_i", "nnz_i", "head_row_nnz", "head_col_nnz",
                                              "band_nnz", "active_rows")]


class _BlockStats(ctypes.Structure):
    _fields_ = [("nonzero_blocks", ctypes.c_int64), ("entries", ctypes.c_int64),
                ("max_density", ctypes.c_double), ("hist", ctypes.c_int64 * 10)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("b", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("footprint_bytes", ctypes.c_int64),
                ("chunked_rows", ctypes.c_int64), ("chunks", ctypes.c_int64),
                ("upper_rows", ctypes.c_int64), ("contributions", ctypes.c_int64),
                ("a_inf_norm", ctypes.c_double), ("upper_batch", ctypes.c_int32),
                ("level0_batch", ctypes.c_int32), ("fused_rows", ctypes.c_int64),
                ("level0_block_rows", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Operand(ctypes.Structure):
    """arrow_operand_t: one column block of one request (device pointers)."""
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("k", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("ldy", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("x_scale", ctypes.c_void_p),
                ("x_inv_norm", ctypes.c_void_p), ("x_maxabs", ctypes.c_void_p),
                ("y_scale", ctypes.c_void_p), ("y_maxabs", ctypes.c_void_p),
                ("y_norm", ctypes.c_void_p), ("y_inv_norm", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


def _np_ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _tptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _rows(t, name: str) -> int:
    """Row stride of a row-major 2-D tensor whose columns are contiguous."""
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be a 2-D tensor with contiguous columns")
    return t.stride(0)


def _stream_handle(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ---------------------------------------------------------------------------
# decomposition (host)
# ---------------------------------------------------------------------------

class Decomposition:
    """Host-side arrow decomposition (LA-Decompose, Section 5.1)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        self.from_cache = False

    @classmethod
    def from_csr(cls, n: int, row_ptr, col, val, b: int, seed: int = 0,
                 la: int = LA_RANDOM_FOREST, max_levels: int = 0,
                 threads: int = 0) -> "Decomposition":
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float32)
        if rp.shape[0] != n + 1:
            raise ValueError("row_ptr must have n + 1 entries")
        opts = _DecompOpts(b, la, seed & ((1 << 64) - 1), max_levels, threads)
        h = ctypes.c_void_p()
        _check(_load().arrow_decompose(n, _np_ptr(rp), _np_ptr(c) if c.size else None,
                                       _np_ptr(v) if v.size else None, ctypes.byref(opts),
                                       ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_matrix(cls, A, b: int, seed: int = 0, la: int = LA_RANDOM_FOREST,
                    max_levels: int = 0, threads: int = 0) -> "Decomposition":
        return cls.from_csr(A.n, A.row_ptr, A.col, A.val, b, seed, la, max_levels, threads)

    @classmethod
    def load(cls, path: str) -> "Decomposition":
        h = ctypes.c_void_p()
        _check(_load().arrow_decomp_load(os.fsencode(path), ctypes.byref(h)))
        return cls(h.value)

    def save(self, path: str) -> None:
        _check(_load().arrow_decomp_save(self._h, os.fsencode(path)))

    def info(self) -> dict:
        i = _DecompInfo()
        _check(_load().arrow_decomp_info(self._h, ctypes.byref(i)))
        return dict(n=i.n, nnz=i.nnz, b=i.b, levels=i.levels, seconds=i.seconds)

    def level(self, i: int) -> dict:
        """Copy of level i: n_i, vop (vertex of each position), CSR of B_i."""
        n_i = ctypes.c_int64()
        nnz = ctypes.c_int64()
        vop, rp, col, val = (ctypes.c_void_p() for _ in range(4))
        _check(_load().arrow_decomp_level(self._h, i, ctypes.byref(n_i), ctypes.byref(nnz),
                                          ctypes.byref(vop), ctypes.byref(rp),
                                          ctypes.byref(col), ctypes.byref(val)))

        def arr(ptr, count, ctype, dtype):
            if count == 0:
                return np.zeros(0, dtype=dtype)
            buf = (ctype * count).from_address(ptr.value)
            return np.frombuffer(buf, dtype=dtype).copy()

        return dict(n_i=n_i.value,
                    vop=arr(vop, n_i.value, ctypes.c_int32, np.int32),
                    row_ptr=arr(rp, n_i.value + 1, ctypes.c_int64, np.int64),
                    col=arr(col, nnz.value, ctypes.c_int32, np.int32),
                    val=arr(val, nnz.value, ctypes.c_float, np.float32))

    def level_stats(self, i: int) -> dict:
        """Counts of level i: n_i, nnz_i, head-row, head-column and band entries, active rows."""
        st = _LevelStats()
        _check(_load().arrow_decomp_level_stats(self._h, i, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _LevelStats._fields_}

    def block_stats(self, i: int, s: int, head_only: bool = False) -> dict:
        """Nonzero s x s blocks of level i and the histogram of their densities
        (tenths); head_only restricts to the head rows and columns."""
        st = _BlockStats()
        _check(_load().arrow_decomp_block_stats(self._h, i, s, 1 if head_only else 0,
                                                ctypes.byref(st)))
        return {"nonzero_blocks": st.nonzero_blocks, "entries": st.entries,
                "max_density": st.max_density, "hist": list(st.hist)}

    def levels(self) -> list:
        return [self.level(i) for i in range(self.info()["levels"])]

    def close(self):
        if self._h and self._h.value:
            _load().arrow_decomp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decompose_cached(n: int, row_ptr, col, val, b: int, cache_dir: str, seed: int = 0,
                     la: int = LA_RANDOM_FOREST, max_levels: int = 0,
                     threads: int = 0) -> "Decomposition":
    """Decomposition of a CSR matrix through an on-disk cache (serving cold
    starts): the file is named by a SHA-256 of the matrix and the options, is
    written with arrow_decomp_save on a miss and read with arrow_decomp_load on
    a hit (a file that fails to load is recomputed and replaced).  The thread
    count is not part of the key: the decomposition does not depend on it.
    The returned object's `from_cache` tells which happened."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float32)
    h = hashlib.sha256()
    h.update(np.array([1, n, b, seed & ((1 << 64) - 1), la, max_levels],
                      dtype=np.uint64).tobytes())
    for a in (rp, c, v):
        h.update(a.tobytes())
    os.makedirs(cache_dir, exist_ok=True)
    path = os.path.join(cache_dir, h.hexdigest()[:40] + ".arrowdec")
    if os.path.exists(path):
        try:
            d = Decomposition.load(path)
            d.from_cache = True
            return d
        except ArrowError:
            pass
    d = Decomposition.from_csr(n, rp, c, v, b, seed, la, max_levels, threads)
    tmp = f"{path}.tmp{os.getpid()}"
    d.save(tmp)
    os.replace(tmp, path)
    d.from_cache = False
    return d


# ---------------------------------------------------------------------------
# device allocator of plan buffers
# ---------------------------------------------------------------------------

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocator_keep = None  # the installed callbacks (ctypes needs them alive)


def set_allocator(alloc=None, free=None) -> None:
    """Install Python callables as the plan allocator: alloc(bytes, stream) ->
    device pointer (int, 0 on failure), free(ptr).  Both None restores
    hipMalloc / hipFree."""
    global _allocator_keep
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check(_load().arrow_set_allocator(None, None, None))
        _allocator_keep = None
        return

    def _a(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), stream or 0)) or None
        except Exception:  # a failed allocation is reported as NULL
            return None

    def _f(ptr, stream, ctx):
        try:
            free(int(ptr))
        except Exception:
            pass

    cb = (ALLOC_FN(_a), FREE_FN(_f))
    _check(_load().arrow_set_allocator(ctypes.cast(cb[0], ctypes.c_void_p),
                                       ctypes.cast(cb[1], ctypes.c_void_p), None))
    _allocator_keep = cb


def use_torch_allocator() -> None:
    """Plan buffers come from PyTorch's caching allocator (on the stream given
    to the plan), so plans share the pool with tensors and destroying a plan
    returns its memory to that pool without a device synchronisation."""
    import torch

    def alloc(nbytes, stream):
        s = stream if stream else torch.cuda.current_stream().cuda_stream
        return torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), s)

    set_allocator(alloc, torch.cuda.caching_allocator_delete)


# ---------------------------------------------------------------------------
# device plan
# ---------------------------------------------------------------------------

def _dtype_code(dtype) -> int:
    if isinstance(dtype, int):
        return dtype
    return DTYPES[dtype]


def torch_dtype(dtype):
    import torch
    return {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16,
            F8E4M3: torch.float8_e4m3fn}[_dtype_code(dtype)]


class Plan:
    """A decomposition uploaded to one GPU (device-resident, immutable)."""

    def __init__(self, decomp: Decomposition, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required for a plan")
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            _check(_load().arrow_plan_create(decomp._h, device, _stream_handle(stream),
                                             ctypes.byref(h)))
        self._h = h
        self.device = device
        inf = self.info()
        self.n = inf["n"]

    def info(self) -> dict:
        i = _PlanInfo()
        _check(_load().arrow_plan_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _PlanInfo._fields_}

    def set_batch(self, kernel: int, batch: int) -> None:
        """Gather batch of KERNEL_UPPER / KERNEL_LEVEL0: -1 automatic, 0 wide, 4..8 short."""
        _check(_load().arrow_plan_set_batch(self._h, kernel, batch))

    def footprint(self) -> int:
        """Device bytes owned by the plan."""
        out = ctypes.c_size_t()
        _check(_load().arrow_plan_footprint(self._h, ctypes.byref(out)))
        return out.value

    def kernel_bytes(self, kernel: int, k: int, dtype="f32") -> int:
        out = ctypes.c_int64()
        _check(_load().arrow_plan_kernel_bytes(self._h, kernel, k, _dtype_code(dtype),
                                               ctypes.byref(out)))
        return out.value

    def workspace_size(self, k: int, dtype="f32") -> int:
        out = ctypes.c_size_t()
        _check(_load().arrow_workspace_size(self._h, k, _dtype_code(dtype), ctypes.byref(out)))
        return out.value

    def iterate_workspace_size(self, k: int, dtype="f32") -> int:
        out = ctypes.c_size_t()
        _check(_load().arrow_iterate_workspace_size(self._h, k, _dtype_code(dtype),
                                                    ctypes.byref(out)))
        return out.value

    def workspace(self, nbytes: int):
        import torch
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")

    def empty(self, k: int, dtype="f32"):
        """An n x k plan-order buffer of the storage type."""
        import torch
        return torch.empty((self.n, k), dtype=torch_dtype(dtype), device=f"cuda:{self.device}")

    def permute_in(self, x, out, dtype="f32", x_scale=None, x_maxabs=None, stream=None):
        """out = P_{pi_0}^T x converted to `dtype` (x: FP32 original order)."""
        k = x.shape[1]
        if out.shape[1] != k:
            raise ValueError("x and out must have the same number of columns")
        _check(_load().arrow_permute_in(self._h, _tptr(x), _rows(x, "x"), _tptr(out),
                                        _rows(out, "out"), _dtype_code(dtype), k, _tptr(x_scale),
                                        _tptr(x_maxabs), _stream_handle(stream)))
        return out

    def permute_out(self, y_plan, out, dtype="f32", x_scale=None, col_factor=None, stream=None):
        """out (FP32, original order) = P_{pi_0} y_plan * scale * factor."""
        k = y_plan.shape[1]
        if out.shape[1] != k:
            raise ValueError("y_plan and out must have the same number of columns")
        _check(_load().arrow_permute_out(self._h, _tptr(y_plan), _rows(y_plan, "y_plan"),
                                         _dtype_code(dtype), k, _tptr(x_scale),
                                         _tptr(col_factor), _tptr(out), _rows(out, "out"),
                                         _stream_handle(stream)))
        return out

    def spmm(self, ops: Sequence[Operand], workspace, stream=None):
        arr = (Operand * len(ops))(*ops)
        _check(_load().arrow_spmm(self._h, ctypes.cast(arr, ctypes.c_void_p), len(ops),
                                  _tptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream_handle(stream)))

    def spmm_static(self, ops: Sequence[Operand], stream=None):
        """arrow_spmm with the library's fixed per-GPU workspace (allocates
        nothing; calls that overlap on one GPU race)."""
        arr = (Operand * len(ops))(*ops)
        _check(_load().arrow_spmm_static(self._h, ctypes.cast(arr, ctypes.c_void_p), len(ops),
                                         _stream_handle(stream)))

    def iterate(self, x, y, iters: int, dtype="f32", renorm: bool = True, norms=None,
                x_scale=None, y_scale=None, workspace=None, stream=None):
        k = x.shape[1]
        ld = _rows(x, "x")
        if tuple(y.shape) != tuple(x.shape) or _rows(y, "y") != ld:
            raise ValueError("x and y must have the same shape and row stride")
        if workspace is None:
            workspace = self.workspace(self.iterate_workspace_size(k, dtype))
        _check(_load().arrow_spmm_iterate(self._h, _tptr(x), _tptr(y), k, ld,
                                          _dtype_code(dtype), _tptr(x_scale), _tptr(y_scale),
                                          iters, ITER_RENORM if renorm else 0, _tptr(norms),
                                          _tptr(workspace),
                                          workspace.numel() * workspace.element_size(),
                                          _stream_handle(stream)))
        return y

    def profile(self, enable: bool):
        _check(_load().arrow_profile_enable(self._h, 1 if enable else 0))

    def profile_query(self, kernel: int):
        launches = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_load().arrow_profile_query(self._h, kernel, ctypes.byref(launches),
                                           ctypes.byref(ms)))
        return launches.value, ms.value

    def close(self):
        if self._h and self._h.value:
            _load().arrow_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def operand(x, y, dtype="f32", x_scale=None, x_inv_norm=None, x_maxabs=None, y_scale=None,
            y_maxabs=None, y_norm=None, y_inv_norm=None, w=None) -> Operand:
    """One operand of Plan.spmm.  With `w` (a contiguous k x k FP32 device
    tensor) the product is the GNN-style step y = ReLU((A x) w)."""
    if tuple(x.shape) != tuple(y.shape):
        raise ValueError("x and y must have the same shape")
    if w is not None and (tuple(w.shape) != (x.shape[1], x.shape[1]) or not w.is_contiguous()):
        raise ValueError("w must be a contiguous k x k tensor")
    return Operand(_tptr(x), _tptr(y), x.shape[1], _rows(x, "x"), _rows(y, "y"),
                   _dtype_code(dtype), 0, _tptr(x_scale), _tptr(x_inv_norm), _tptr(x_maxabs),
                   _tptr(y_scale), _tptr(y_maxabs), _tptr(y_norm), _tptr(y_inv_norm), _tptr(w))


def csr_workspace_size(n: int, k: int) -> int:
    out = ctypes.c_size_t()
    _check(_load().arrow_csr_workspace_size(n, k, ctypes.byref(out)))
    return out.value


def csr_batch(row_ptr) -> int:
    """Gather batch for csr_spmm from a host row_ptr (the plan's rule)."""
    import numpy as np
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    out = ctypes.c_int32()
    _check(_load().arrow_csr_batch(len(rp) - 1, rp.ctypes.data, ctypes.byref(out)))
    return out.value


def csr_spmm(n: int, row_ptr, col, val, x, y, sumsq_ws=None, norms=None, stream=None, batch=0):
    """Plain CSR baseline on the device (int32 row_ptr / col, FP32 values)."""
    ld = _rows(x, "x")
    if tuple(y.shape) != tuple(x.shape) or _rows(y, "y") != ld:
        raise ValueError("x and y must have the same shape and row stride")
    _check(_load().arrow_csr_spmm(n, _tptr(row_ptr), _tptr(col), _tptr(val), _tptr(x), _tptr(y),
                                  x.shape[1], ld, batch, _tptr(sumsq_ws), _tptr(norms),
                                  _stream_handle(stream)))
    return y


class RocsparseSpmm:
    """The vendor CSR SpMM as a comparison baseline (y = A x on one stream)."""

    def __init__(self, n, row_ptr, col, val, x, y, alg: int = 0, stream=None):
        ld = _rows(x, "x")
        if tuple(y.shape) != tuple(x.shape) or _rows(y, "y") != ld:
            raise ValueError("x and y must have the same shape and row stride")
        h = ctypes.c_void_p()
        _check(_load().arrow_rocsparse_create(n, col.numel(), _tptr(row_ptr), _tptr(col),
                                              _tptr(val), _tptr(x), _tptr(y), x.shape[1], ld,
                                              alg, _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._keep = (row_ptr, col, val, x, y)

    def run(self):
        _check(_load().arrow_rocsparse_run(self._h))

    def close(self):
        if self._h and self._h.value:
            _load().arrow_rocsparse_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy(src, dst, nbytes: int, stream=None):
    _check(_load().arrow_copy(_tptr(src), _tptr(dst), nbytes, _stream_handle(stream)))


def version() -> str:
    return _load().arrow_version().decode()
