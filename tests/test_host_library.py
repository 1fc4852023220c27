"""Host side of libarrow on the CPU: decomposition parity with the oracle's
LA-Decompose (bit-exact: integer / index work), validity at larger sizes,
save/load, error paths and the exported C-ABI symbols."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import decomp as D
from oracle import spmm as S

A_ = pytest.importorskip("paper_2402_19364_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_decompose(A, b, seed=0, la=A_.LA_RANDOM_FOREST, max_levels=0):
    return A_.Decomposition.from_matrix(A, b, seed=seed, la=la, max_levels=max_levels)


def _assert_same(levels_lib, levels_ref):
    assert len(levels_lib) == len(levels_ref)
    for L, R in zip(levels_lib, levels_ref):
        assert L["n_i"] == R["n_i"]
        assert np.array_equal(L["vop"], R["vop"])
        assert np.array_equal(L["row_ptr"], R["row_ptr"])
        assert np.array_equal(L["col"], R["col"])
        assert np.array_equal(L["val"].view(np.uint32), np.asarray(R["val"], np.float32).view(np.uint32))


def _small_graphs():
    gs = []
    for seed in range(5):
        gs.append(W.random_graph(60, 0.08, seed, diagonal=seed % 2 == 0))
    gs.append(W.make_matrix("grid2d", 12, "uniform", 0, 1))
    gs.append(W.make_matrix("grid3d", 5, "sym_laplacian", 0, 1))
    gs.append(W.make_matrix("rmat", 9, "row_normalized", 3, 4, 8))
    gs.append(W.from_edges(40, [(0, i) for i in range(1, 40)]))             # star
    gs.append(W.from_edges(50, [(i, i + 1) for i in range(49)]))            # path
    gs.append(W.from_edges(30, [], diagonal=True))                          # diagonal only
    gs.append(W.from_edges(17, []))                                         # empty
    gs.append(W.from_edges(20, [(0, 5), (5, 0), (3, 9)], symmetric=False))  # non-symmetric
    return gs


_LA_NAMES = {A_.LA_RANDOM_FOREST: "random_forest", A_.LA_IDENTITY: "identity",
             A_.LA_SEPARATOR: "separator"}


@pytest.mark.parametrize("la", [A_.LA_RANDOM_FOREST, A_.LA_IDENTITY, A_.LA_SEPARATOR])
@pytest.mark.parametrize("b", [2, 3, 8])
def test_decomposition_matches_oracle_bitwise(la, b):
    for i, A in enumerate(_small_graphs()):
        ref = D.la_decompose(A, b, seed=17 + i, la=_LA_NAMES[la])
        got = _lib_decompose(A, b, seed=17 + i, la=la).levels()
        _assert_same(got, ref)


def test_decomposition_matches_oracle_medium_rmat():
    A = W.make_matrix("rmat", 12, "row_normalized", 21, 22, 16)
    ref = D.la_decompose(A, 64, seed=5)
    got = _lib_decompose(A, 64, seed=5).levels()
    _assert_same(got, ref)
    assert len(got) >= 2


def test_nonsymmetric_medium_decomposition_matches_oracle_on_any_thread_count():
    # a directed R-MAT pattern (each stored entry kept with probability 0.7,
    # so most edges appear in one direction only) takes the listed-edge path
    # on several threads; the symmetric path is covered above
    A = W.make_matrix("rmat", 11, "row_normalized", 31, 32, 16)
    keep = np.random.default_rng(33).random(A.nnz) < 0.7
    rows = A.rows()[keep]
    B = W.from_edges(A.n, np.stack([rows, A.col[keep]], 1), values="uniform", seed=34,
                     diagonal=True, symmetric=False)
    assert B.nnz > 8192  # several threads' ranges
    ref = D.la_decompose(B, 32, seed=6)
    assert len(ref) >= 2
    for t in (1, 3, 8):
        _assert_same(A_.Decomposition.from_matrix(B, 32, seed=6, threads=t).levels(), ref)


def test_concurrent_decompositions_match_sequential_ones():
    # two host threads decompose at once (ctypes releases the GIL), sharing
    # the library's cache of large working blocks
    import threading
    mats = [W.make_matrix("rmat", 14, "row_normalized", 41, 42, 16),
            W.make_matrix("grid3d", 24, "sym_laplacian", 0, 1)]
    ref = [A_.Decomposition.from_matrix(M, 64, seed=9, threads=2).levels() for M in mats]
    got = [None, None]

    def work(i):
        got[i] = A_.Decomposition.from_matrix(mats[i], 64, seed=9, threads=2).levels()

    ts = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for i in range(2):
        _assert_same(got[i], ref[i])


def test_separator_decomposition_same_on_any_thread_count():
    # components of 2^16 vertices and more are laid out on threads of their
    # own: a 400 x 400 grid splits into such components at its first levels
    A = W.make_matrix("grid2d", 400, "sym_laplacian", 0, 1)
    ref = A_.Decomposition.from_matrix(A, 400, seed=3, la=A_.LA_SEPARATOR, threads=1).levels()
    D.validate(A, ref, 400)
    for t in (3, 8):
        got = A_.Decomposition.from_matrix(A, 400, seed=3, la=A_.LA_SEPARATOR, threads=t).levels()
        _assert_same(got, ref)


@pytest.mark.parametrize("cfg", ["grid64"])
def test_config_small_decomposition(cfg):
    w = W.WORKLOADS[cfg]
    A = W.workload_matrix(w)
    d = _lib_decompose(A, w.b, seed=w.seeds["decompose"])
    ref = D.la_decompose(A, w.b, seed=w.seeds["decompose"])
    _assert_same(d.levels(), ref)
    D.validate(A, d.levels(), w.b)


def test_large_decompositions_are_valid():
    A = W.make_matrix("grid2d", 256, "sym_laplacian", 0, 0)
    for la in (A_.LA_RANDOM_FOREST, A_.LA_IDENTITY):
        lv = _lib_decompose(A, 256, seed=4, la=la).levels()
        D.validate(A, lv, 256)
    lv = _lib_decompose(A, 256, la=A_.LA_IDENTITY).levels()
    assert len(lv) == 1  # natural-order grid, bandwidth = side = b
    R = W.make_matrix("rmat", 15, "row_normalized", 9, 10, 16)
    lv = _lib_decompose(R, 256, seed=1).levels()
    D.validate(R, lv, 256)
    X = np.random.default_rng(0).standard_normal((R.n, 4))
    # Eq. (1) on the library's levels equals A X (only at small n: dense per level)
    small = W.make_matrix("rmat", 8, "row_normalized", 1, 2, 8)
    lv = _lib_decompose(small, 4, seed=3).levels()
    Xs = np.random.default_rng(1).standard_normal((small.n, 3))
    assert np.allclose(D.product_via_levels(lv, small.n, Xs), S.csr_spmm(small, Xs),
                       rtol=1e-12, atol=1e-12)
    del X


def test_determinism_and_save_load(tmp_path):
    A = W.make_matrix("rmat", 11, "row_normalized", 1, 2, 16)
    d1 = _lib_decompose(A, 32, seed=9)
    d2 = _lib_decompose(A, 32, seed=9)
    _assert_same(d1.levels(), d2.levels())
    p = str(tmp_path / "d.arrow")
    d1.save(p)
    d3 = A_.Decomposition.load(p)
    _assert_same(d3.levels(), d1.levels())
    assert d3.info()["nnz"] == A.nnz
    raw = bytearray(open(p, "rb").read())
    raw[100] ^= 0xFF
    open(p, "wb").write(bytes(raw))
    with pytest.raises(A_.ArrowError) as e:
        A_.Decomposition.load(p)
    assert e.value.status == A_.ERR_IO
    with pytest.raises(A_.ArrowError):
        A_.Decomposition.load(str(tmp_path / "missing"))


def test_error_paths():
    A = W.random_graph(20, 0.2, 1)
    with pytest.raises(A_.ArrowError) as e:
        _lib_decompose(A, 1)
    assert e.value.status == A_.ERR_INVALID_ARG
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.col[bad.row_ptr[3]] = 99  # out of range
    with pytest.raises(A_.ArrowError):
        _lib_decompose(bad, 4)
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    r = int(np.argmax(np.diff(bad.row_ptr)))
    s = bad.row_ptr[r]
    bad.col[s], bad.col[s + 1] = bad.col[s + 1], bad.col[s]  # unsorted row
    with pytest.raises(A_.ArrowError):
        _lib_decompose(bad, 4)
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.row_ptr[5] = bad.row_ptr[6] + 1  # decreasing
    with pytest.raises(A_.ArrowError):
        _lib_decompose(bad, 4)
    R = W.make_matrix("rmat", 10, "row_normalized", 1, 2, 16)
    with pytest.raises(A_.ArrowError) as e:
        _lib_decompose(R, 2, max_levels=1)
    assert e.value.status == A_.ERR_UNSUPPORTED
    msg = A_.lib().arrow_last_error().decode()
    assert "max_levels" in msg


def test_level_stats_match_the_exported_levels():
    M = W.make_matrix("rmat", 12, "row_normalized", 1, 2, 16)
    b = 48
    d = _lib_decompose(M, b, seed=3)
    total = 0
    for i, L in enumerate(d.levels()):
        st = d.level_stats(i)
        rp, col = L["row_ptr"], L["col"].astype(np.int64)
        rows = np.repeat(np.arange(L["n_i"]), np.diff(rp))
        head_row = int(np.sum(rows < b))
        head_col = int(np.sum((rows >= b) & (col < b)))
        band = int(np.sum((rows >= b) & (col >= b)))
        assert st == {"n_i": L["n_i"], "nnz_i": len(col), "head_row_nnz": head_row,
                      "head_col_nnz": head_col, "band_nnz": band,
                      "active_rows": int(np.count_nonzero(np.diff(rp)))}, i
        assert np.all(np.abs(col[(rows >= b) & (col >= b)] - rows[(rows >= b) & (col >= b)]) <= b)
        total += st["nnz_i"]
    assert total == M.nnz
    with pytest.raises(A_.ArrowError):
        d.level_stats(len(d.levels()))


def test_gather_batch_rule():
    # smallest short batch (4..8) holding all entries of >= 99% of the rows
    assert A_.csr_batch(W.make_matrix("grid2d", 30, "uniform", 0, 1).row_ptr) == 5
    assert A_.csr_batch(W.make_matrix("grid3d", 8, "uniform", 0, 1).row_ptr) == 7
    assert A_.csr_batch(W.make_matrix("rmat", 12, "row_normalized", 1, 2, 16).row_ptr) == 0
    assert A_.csr_batch(np.arange(101, dtype=np.int64)) == 4          # one entry per row
    assert A_.csr_batch(np.zeros(1, dtype=np.int64)) == 0             # no rows
    lens = np.array([3] * 1000 + [20] * 10)                           # 10 long rows of 1010
    assert A_.csr_batch(np.concatenate([[0], np.cumsum(lens)])) == 4
    lens = np.array([3] * 1000 + [20] * 11)                           # 11 of 1011: too many
    assert A_.csr_batch(np.concatenate([[0], np.cumsum(lens)])) == 0
    lens = np.array([6] * 990 + [9] * 10)
    assert A_.csr_batch(np.concatenate([[0], np.cumsum(lens)])) == 6
    with pytest.raises(A_.ArrowError):
        A_.csr_batch(np.array([0, 3, 2], dtype=np.int64))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "arrow.h")).read()
    declared = set(re.findall(r"\b(arrow_[a-z0-9_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", A_.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = declared - exported
    assert not missing, missing
    for name in declared:
        getattr(A_.lib(), name)
    assert A_.version() == "1.0.0"


def _fnv1a(data: bytes) -> int:
    h = 1469598103934665603
    for c in data:
        h = ((h ^ c) * 1099511628211) & ((1 << 64) - 1)
    return h


def _rewrite(path, mutate):
    """Apply mutate(bytearray, layout) to a saved decomposition and restore a
    valid checksum, so only the structural checks can reject the file."""
    raw = bytearray(open(path, "rb").read())
    n = int(np.frombuffer(bytes(raw[16:24]), np.int64)[0])
    off = 56
    n_i = int(np.frombuffer(bytes(raw[off:off + 8]), np.int64)[0])
    nnz_i = int(np.frombuffer(bytes(raw[off + 8:off + 16]), np.int64)[0])
    vop_off = off + 16
    rp_off = vop_off + 4 * n_i
    col_off = rp_off + 8 * (n_i + 1)
    rp = np.frombuffer(bytes(raw[rp_off:col_off]), np.int64)
    mutate(raw, dict(n=n, n_i=n_i, nnz_i=nnz_i, vop=vop_off, rp=rp, col=col_off))
    body = bytes(raw[:-8])
    raw[-8:] = np.array([_fnv1a(body)], dtype=np.uint64).tobytes()
    open(path, "wb").write(bytes(raw))


def test_load_rejects_structurally_invalid_files(tmp_path):
    # a path in natural order: level 0 is the path itself (bandwidth 1)
    A = W.from_edges(10, [(i, i + 1) for i in range(9)])
    d = _lib_decompose(A, 2, la=A_.LA_IDENTITY)
    assert d.info()["levels"] == 1
    p = str(tmp_path / "ok.arrow")
    d.save(p)
    _rewrite(p, lambda raw, lay: None)          # checksum recomputed, nothing changed
    _assert_same(A_.Decomposition.load(p).levels(), d.levels())

    def outside_arrow(raw, lay):                # row 9: column 8 -> 5 (|9 - 5| > b, 5 >= b)
        e = int(lay["rp"][9])
        raw[lay["col"] + 4 * e:lay["col"] + 4 * e + 4] = np.int32(5).tobytes()

    def not_injective(raw, lay):                # position 1 holds the vertex of position 0
        raw[lay["vop"] + 4:lay["vop"] + 8] = raw[lay["vop"]:lay["vop"] + 4]

    def unsorted(raw, lay):                     # row 5 holds columns 4, 6: swap them
        e = int(lay["rp"][5])
        a = bytes(raw[lay["col"] + 4 * e:lay["col"] + 4 * e + 4])
        raw[lay["col"] + 4 * e:lay["col"] + 4 * e + 4] = raw[lay["col"] + 4 * e + 4:
                                                              lay["col"] + 4 * e + 8]
        raw[lay["col"] + 4 * e + 4:lay["col"] + 4 * e + 8] = a

    for name, fn, why in (("arrow", outside_arrow, "outside the arrow"),
                          ("inj", not_injective, "not injective"),
                          ("sort", unsorted, "not increasing")):
        q = str(tmp_path / f"{name}.arrow")
        d.save(q)
        _rewrite(q, fn)
        with pytest.raises(A_.ArrowError) as e:
            A_.Decomposition.load(q)
        assert e.value.status == A_.ERR_IO, name
        assert why in A_.lib().arrow_last_error().decode(), name


def test_allocator_and_threads_arguments():
    lib = A_.lib()
    # both functions or neither
    assert lib.arrow_set_allocator(None, None, None) == A_.OK
    cb = A_.ALLOC_FN(lambda n, s, c: None)
    assert lib.arrow_set_allocator(ctypes.cast(cb, ctypes.c_void_p), None, None) == \
        A_.ERR_INVALID_ARG
    with pytest.raises(ValueError):
        A_.set_allocator(lambda n, s: 0, None)
    A_.set_allocator(None, None)
    A = W.make_matrix("rmat", 10, "row_normalized", 5, 6, 16)
    with pytest.raises(A_.ArrowError) as e:
        A_.Decomposition.from_matrix(A, 16, threads=-1)
    assert e.value.status == A_.ERR_INVALID_ARG
    ref = _lib_decompose(A, 16, seed=4).levels()
    for t in (1, 2, 3, 8):
        _assert_same(A_.Decomposition.from_matrix(A, 16, seed=4, threads=t).levels(), ref)


def test_block_stats_match_a_brute_force_count():
    A = W.make_matrix("rmat", 11, "row_normalized", 7, 8, 16)
    b = 32
    d = _lib_decompose(A, b, seed=2)
    for i, L in enumerate(d.levels()[:3]):
        rows = np.repeat(np.arange(L["n_i"]), np.diff(L["row_ptr"]))
        col = L["col"].astype(np.int64)
        for s in (1, 4, 16, b):
            for head in (False, True):
                keep = (rows < b) | (col < b) if head else np.ones(col.size, bool)
                keys = (rows[keep] // s) * (L["n_i"] // s + 1) + col[keep] // s
                _, counts = np.unique(keys, return_counts=True)
                dens = counts / float(s * s)
                hist = np.bincount(np.minimum((dens * 10).astype(int), 9), minlength=10)
                st = d.block_stats(i, s, head_only=head)
                assert st["nonzero_blocks"] == counts.size and st["entries"] == int(keep.sum())
                assert st["hist"] == hist.tolist(), (i, s, head)
                assert st["max_density"] == (dens.max() if dens.size else 0.0)
    # one-entry blocks: every nonzero 1 x 1 block has density 1
    st = d.block_stats(0, 1)
    assert st["nonzero_blocks"] == st["entries"] == st["hist"][9]
    with pytest.raises(A_.ArrowError):
        d.block_stats(0, 0)


def test_decompose_cached_roundtrip(tmp_path):
    """The serving cache: a miss decomposes and writes the file, a hit loads
    the same levels bit for bit, other options or values miss, and a damaged
    file is recomputed."""
    A = W.make_matrix("rmat", 10, "row_normalized", 31, 32, 8)
    cache = str(tmp_path / "dec")
    d1 = A_.decompose_cached(A.n, A.row_ptr, A.col, A.val, 32, cache, seed=3)
    assert not d1.from_cache
    files = os.listdir(cache)
    assert len(files) == 1 and files[0].endswith(".arrowdec")
    d2 = A_.decompose_cached(A.n, A.row_ptr, A.col, A.val, 32, cache, seed=3, threads=4)
    assert d2.from_cache
    _assert_same(d2.levels(), d1.levels())
    d3 = A_.decompose_cached(A.n, A.row_ptr, A.col, A.val, 32, cache, seed=4)
    assert not d3.from_cache
    v = A.val.copy()
    v[0] = np.nextafter(v[0], np.float32(2.0))
    d4 = A_.decompose_cached(A.n, A.row_ptr, A.col, v, 32, cache, seed=3)
    assert not d4.from_cache and len(os.listdir(cache)) == 3
    path = os.path.join(cache, files[0])
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    open(path, "wb").write(bytes(raw))
    d5 = A_.decompose_cached(A.n, A.row_ptr, A.col, A.val, 32, cache, seed=3)
    assert not d5.from_cache
    _assert_same(d5.levels(), d1.levels())
    assert A_.decompose_cached(A.n, A.row_ptr, A.col, A.val, 32, cache, seed=3).from_cache


@pytest.mark.parametrize("graph", [("grid2d", 20, 8), ("grid3d", 8, 8), ("rmat", 11, 32)])
def test_separator_decomposition_matches_oracle_bitwise(graph):
    kind, size, b = graph
    A = W.make_matrix(kind, size, "uniform", 41, 42, 8)
    ref = D.la_decompose(A, b, seed=9, la="separator")
    got = _lib_decompose(A, b, seed=9, la=A_.LA_SEPARATOR).levels()
    _assert_same(got, ref)
    D.validate(A, got, b)
