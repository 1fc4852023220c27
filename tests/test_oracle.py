"""Pins of the oracle against what the paper and the mathematics fix (CPU only)."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import minimum_spanning_tree

import workloads as W
from oracle import decomp as D
from oracle import quant as Q
from oracle import spmm as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# CSR product
# ---------------------------------------------------------------------------

def _nonsym(n, p, seed):
    """Random non-symmetric matrix with a diagonal (transposes would show)."""
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < p)
    np.fill_diagonal(M, True)
    r, c = np.nonzero(M)
    key = r.astype(np.int64) * n + c
    rp, col = W._pattern_from_keys(n, key)
    val = rng.uniform(-1, 1, col.shape[0]).astype(np.float32)
    return W.CSR(n, rp, col, val)


@pytest.mark.parametrize("seed", range(4))
def test_csr_matches_python_brute_force_bitwise(seed):
    A = _nonsym(23, 0.2, seed)
    X = np.random.default_rng(seed).standard_normal((23, 5))
    got = S.csr_spmm(A, X)
    ref = np.array(S.brute_force(A, X.tolist()))
    assert np.array_equal(got, ref)


def test_csr_matches_dense_and_scipy():
    A = _nonsym(300, 0.03, 7)
    X = np.random.default_rng(1).standard_normal((300, 17))
    ref = S.dense(A) @ X
    assert np.allclose(S.csr_spmm(A, X), ref, rtol=1e-13, atol=1e-13)
    G = W.make_matrix("rmat", 12, "row_normalized", 5, 6, 8)
    Xg = np.random.default_rng(2).standard_normal((G.n, 8))
    ref2 = sp.csr_matrix((G.val.astype(np.float64), G.col, G.row_ptr), shape=(G.n, G.n)) @ Xg
    assert np.allclose(S.csr_spmm(G, Xg), ref2, rtol=1e-12, atol=1e-14)
    rows = np.array([0, 5, G.n - 1, 77], dtype=np.int64)
    assert np.array_equal(S.csr_spmm_rows(G, Xg, rows), S.csr_spmm(G, Xg)[rows])


def test_column_direction_shift_matrix():
    # A[i, (i+1) % n] = 1  =>  (A X)[i] = X[(i+1) % n]; catches a transposed operand.
    n = 11
    A = W.from_edges(n, [(i, (i + 1) % n) for i in range(n)], symmetric=False)
    X = np.arange(n * 3, dtype=np.float64).reshape(n, 3)
    assert np.array_equal(S.csr_spmm(A, X), np.roll(X, -1, axis=0))


def test_closed_forms_full_size_grid_laplacian():
    # L D^{1/2} 1 = 0 for L = I - D^{-1/2} A D^{-1/2} (exact up to fp32 rounding of L)
    A = W.make_matrix("grid2d", 512, "sym_laplacian", 0, 0)
    deg = np.diff(A.row_ptr).astype(np.float64) - 1.0
    y = S.csr_spmm(A, np.sqrt(deg)[:, None])
    assert np.max(np.abs(y)) < 2e-6
    A3 = W.make_matrix("grid3d", 24, "sym_laplacian", 0, 0)
    deg3 = np.diff(A3.row_ptr).astype(np.float64) - 1.0
    assert np.max(np.abs(S.csr_spmm(A3, np.sqrt(deg3)[:, None]))) < 2e-6


def test_closed_forms_row_stochastic_and_identity():
    G = W.make_matrix("rmat", 14, "row_normalized", 11, 12, 16)
    y = S.csr_spmm(G, np.ones((G.n, 2)))
    deg = np.diff(G.row_ptr)
    assert np.allclose(y[deg > 0], 1.0, atol=1e-5)
    assert np.all(y[deg == 0] == 0.0)
    n = 1000
    I = W.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
              np.ones(n, np.float32))
    X = np.random.default_rng(3).standard_normal((n, 4))
    assert np.array_equal(S.csr_spmm(I, X), X)


def test_generator_nnz_closed_forms():
    for s in (3, 17, 64):
        assert W.grid2d_pattern(s)[2].shape[0] == s * s + 4 * s * (s - 1)
    for s in (3, 9):
        assert W.grid3d_pattern(s)[2].shape[0] == s ** 3 + 6 * s * s * (s - 1)
    n, rp, col = W.rmat_pattern(10, 16, 99)
    n2, rp2, col2 = W.rmat_pattern(10, 16, 99)
    assert np.array_equal(col, col2) and np.array_equal(rp, rp2)
    A = sp.csr_matrix((np.ones(col.shape[0]), col, rp), shape=(n, n))
    assert (A - A.T).nnz == 0 and A.diagonal().sum() == 0


# ---------------------------------------------------------------------------
# iteration with per-column renormalisation
# ---------------------------------------------------------------------------

def test_iteration_diagonal_closed_form():
    n, T = 50, 12
    d = np.linspace(-1.3, 0.9, n).astype(np.float32)
    A = W.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d)
    X0 = np.random.default_rng(0).standard_normal((n, 3))
    Ys, nus = S.iterate(A, X0, T)
    dd = d.astype(np.float64)
    for t in range(T):
        Pt = (dd ** (t + 1))[:, None] * X0          # A^{t+1} X0
        Pprev = (dd ** t)[:, None] * X0
        # A X_t with X_0 as given and X_t = A^t X0 / ||A^t X0|| for t >= 1
        ref_Y = Pt if t == 0 else Pt / np.linalg.norm(Pprev, axis=0)
        assert S.rel_fro(Ys[t], ref_Y) < 1e-12
        assert np.allclose(nus[t], np.linalg.norm(ref_Y, axis=0), rtol=1e-12)


def test_iteration_path_eigenvector():
    # tridiag(-1, 2, -1): eigenvector sin(j k pi/(n+1)), eigenvalue 2 - 2 cos(k pi/(n+1));
    # k = n is the dominant one, so rounding along other eigenvectors decays.
    n = 64
    kk = n
    A = W.from_edges(n, [(i, i + 1) for i in range(n - 1)], diagonal=True)
    A.val[:] = np.where(A.rows() == A.col, 2.0, -1.0).astype(np.float32)
    j = np.arange(1, n + 1)
    x = np.sin(j * kk * math.pi / (n + 1))
    x /= np.linalg.norm(x)
    lam = 2 - 2 * math.cos(kk * math.pi / (n + 1))
    Ys, nus = S.iterate(A, x[:, None], 3)
    for t in range(3):
        assert np.allclose(Ys[t][:, 0], lam * x, atol=1e-13)
        assert abs(nus[t][0] - lam) < 1e-13


def test_zero_column_stays_zero():
    A = _nonsym(20, 0.2, 3)
    X = np.random.default_rng(0).standard_normal((20, 3))
    X[:, 1] = 0
    Ys, nus = S.iterate(A, X, 3)
    assert nus[0][1] == 0 and np.all(Ys[2][:, 1] == 0)


# ---------------------------------------------------------------------------
# decomposition: worked example, validator, reference LA-Decompose
# ---------------------------------------------------------------------------

def _read_fig3():
    b = n = None
    edges = []
    with open(os.path.join(GOLDEN, "fig3_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "b":
                b = int(line[1])
            elif line[0] == "n":
                n = int(line[1])
            else:
                edges.append((int(line[0]), int(line[1]), line[2]))
    return b, n, edges


def test_fig3_classification():
    b, n, edges = _read_fig3()
    for p, q, cls in edges:
        head = p < b or q < b
        band = abs(p - q) <= b
        got = "head" if head else ("band" if band else "remainder")
        assert got == cls, (p, q)
        assert bool(D.in_arrow(p, q, b)) == (cls != "remainder")
        assert bool(D.in_arrow(q, p, b)) == (cls != "remainder")
    # the remainder {2, 5} decomposes into one level whose only edge is a head
    # edge at positions 0 and 1 (B_1 of the figure)
    rem = [(p, q) for p, q, c in edges if c == "remainder"]
    R = W.from_edges(n, rem)
    levels = D.la_decompose(R, b)
    assert len(levels) == 1
    L = levels[0]
    pos = {int(v): i for i, v in enumerate(L["vop"])}
    ent = {(int(p), int(q)) for p, q in zip(np.repeat(np.arange(L["n_i"]), np.diff(L["row_ptr"])),
                                              L["col"])}
    assert {tuple(sorted((pos[2], pos[5])))} == {(0, 1)}
    assert ent == {(0, 1), (1, 0)}


def test_fig3_full_decomposition_given_pi0():
    """With the figure's pi_0 forced (identity), one classification step leaves
    exactly the remainder edge; the two levels rebuild A."""
    b, n, edges = _read_fig3()
    A = W.from_edges(n, [(p, q) for p, q, _ in edges], values="uniform", seed=3)
    r = A.rows()
    c = A.col.astype(np.int64)
    keep = D.in_arrow(r, c, b)
    assert {(int(x), int(y)) for x, y in zip(r[~keep], c[~keep])} == {(2, 5), (5, 2)}
    L0 = dict(n_i=n, vop=np.arange(n, dtype=np.int32),
              row_ptr=np.concatenate([[0], np.cumsum(np.bincount(r[keep], minlength=n))]),
              col=c[keep].astype(np.int32), val=A.val[keep])
    L1 = dict(n_i=2, vop=np.array([2, 5], np.int32), row_ptr=np.array([0, 1, 2]),
              col=np.array([1, 0], np.int32), val=A.val[~keep])
    D.validate(A, [L0, L1], b)
    assert np.array_equal(D.dense_sum([L0, L1], n), S.dense(A))


def _graphs():
    out = []
    for seed in range(6):
        out.append(W.random_graph(40, 0.12, seed, diagonal=seed % 2 == 0))
    out.append(W.make_matrix("grid2d", 9, "uniform", 0, 1))
    out.append(W.make_matrix("rmat", 7, "row_normalized", 3, 4, 8))
    out.append(W.from_edges(30, [(0, i) for i in range(1, 30)]))  # star
    out.append(W.from_edges(25, []))                              # empty
    out.append(W.from_edges(12, [], diagonal=True))               # diagonal only
    return out


@pytest.mark.parametrize("la", ["random_forest", "identity"])
@pytest.mark.parametrize("b", [2, 3, 5])
def test_reference_decomposition_is_valid(la, b):
    for A in _graphs():
        levels = D.la_decompose(A, b, seed=11, la=la)
        D.validate(A, levels, b)
        assert np.array_equal(D.dense_sum(levels, A.n), S.dense(A))
        X = np.random.default_rng(0).standard_normal((A.n, 3))
        assert np.allclose(D.product_via_levels(levels, A.n, X), S.csr_spmm(A, X),
                           rtol=1e-12, atol=1e-12)


def test_validator_catches_planted_mistakes():
    A = W.random_graph(40, 0.15, 5, diagonal=True)
    b = 3
    good = D.la_decompose(A, b, seed=1)
    D.validate(A, good, b)

    def clone():
        return [{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in L.items()}
                for L in good]

    bad = clone()                      # a dropped entry
    L = bad[0]
    L["col"] = L["col"][1:]
    L["val"] = L["val"][1:]
    L["row_ptr"] = np.maximum(L["row_ptr"] - 1, 0)
    with pytest.raises(D.InvalidDecomposition):
        D.validate(A, bad, b)
    bad = clone()                      # a changed value bit
    bad[0]["val"][3] = np.nextafter(bad[0]["val"][3], np.float32(2))
    with pytest.raises(D.InvalidDecomposition):
        D.validate(A, bad, b)
    bad = clone()                      # a non-injective map
    bad[0]["vop"][1] = bad[0]["vop"][0]
    with pytest.raises(D.InvalidDecomposition):
        D.validate(A, bad, b)
    # an entry outside the arrow: lay the star out with its centre last
    S_ = W.from_edges(12, [(0, i) for i in range(1, 12)])
    rp = np.zeros(13, np.int64)
    cols, rows = [], []
    for i in range(1, 12):
        rows += [11, i - 1]
        cols += [i - 1, 11]
    order = np.lexsort((cols, rows))
    rows = np.array(rows)[order]
    cols = np.array(cols)[order]
    rp[1:] = np.cumsum(np.bincount(rows, minlength=12))
    vop = np.array(list(range(1, 12)) + [0], np.int32)
    with pytest.raises(D.InvalidDecomposition):
        D.validate(S_, [dict(n_i=12, vop=vop, row_ptr=rp, col=cols.astype(np.int32),
                             val=np.ones(22, np.float32))], 2)


def test_special_cases():
    # star: everything in the head of one level
    A = W.from_edges(50, [(0, i) for i in range(1, 50)])
    lv = D.la_decompose(A, 2)
    assert len(lv) == 1 and lv[0]["vop"][0] == 0
    # path labelled in order: MSF = the path, root = end, identity layout
    P = W.from_edges(40, [(i, i + 1) for i in range(39)])
    lv = D.la_decompose(P, 2, seed=3)
    assert len(lv) == 1
    # n <= b and diagonal-only: one level
    assert len(D.la_decompose(W.random_graph(6, 0.5, 1, diagonal=True), 8)) == 1
    assert len(D.la_decompose(W.from_edges(9, [], diagonal=True), 2)) == 1
    # natural-order grid, identity arrangement, b >= side: one level
    G = W.make_matrix("grid2d", 16, "uniform", 0, 1)
    assert len(D.la_decompose(G, 16, la="identity")) == 1


def test_levels_shrink_and_are_compact():
    A = W.make_matrix("rmat", 10, "row_normalized", 8, 9, 16)
    lv = D.la_decompose(A, 16, seed=2)
    D.validate(A, lv, 16)
    nnz = [int(L["row_ptr"][-1]) for L in lv]
    assert nnz[0] > nnz[-1]
    for L in lv[1:]:
        rp = L["row_ptr"]
        n_i = L["n_i"]
        p = np.repeat(np.arange(n_i), np.diff(rp))
        assert n_i == 0 or max(p.max(), L["col"].max()) == n_i - 1


def _random_tree(n, rng, kind):
    if kind == "random":
        return [(i, int(rng.integers(0, i))) for i in range(1, n)]
    if kind == "caterpillar":
        spine = n // 3
        e = [(i, i + 1) for i in range(spine - 1)]
        e += [(i, int(rng.integers(0, spine))) for i in range(spine, n)]
        return e
    if kind == "broom":
        h = n // 2
        return [(i, i + 1) for i in range(h - 1)] + [(h - 1, i) for i in range(h, n)]
    if kind == "dary":
        return [(i, (i - 1) // 3) for i in range(1, n)]
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["random", "caterpillar", "broom", "dary"])
def test_smallest_first_lemma(kind):
    """Smallest-first order keeps at least min(n-1, ceil((x-1)(n-1)/x)+1) tree
    edges within an x*Delta band (Section 5.4 lemma)."""
    rng = np.random.default_rng(4)
    for n in (30, 200, 700):
        e = _random_tree(n, rng, kind)
        layout = D.smallest_first_order(list(range(n)), e)
        assert sorted(layout) == list(range(n))
        pos = np.empty(n, np.int64)
        pos[layout] = np.arange(n)
        deg = np.bincount(np.array(e).ravel(), minlength=n)
        Delta = int(deg.max())
        dist = np.array([abs(pos[a] - pos[c]) for a, c in e])
        for x in (2, 4, 8):
            need = min(n - 1, math.ceil((x - 1) * (n - 1) / x) + 1)
            assert int(np.sum(dist <= x * Delta)) >= need


def test_smallest_first_is_preorder_with_small_children_first():
    #      0
    #    / | \
    #   1  2  3        subtree sizes: 1 -> 3, 2 -> 1, 3 -> 2
    #  / \     \
    # 4   5     6
    e = [(0, 1), (0, 2), (0, 3), (1, 4), (1, 5), (3, 6)]
    assert D.smallest_first_order(list(range(7)), e) == [0, 2, 3, 6, 1, 4, 5]


def test_kruskal_matches_scipy_msf():
    rng = np.random.default_rng(0)
    for seed in range(5):
        A = W.random_graph(60, 0.08, seed)
        eu, ev = D._undirected_edges(A.rows(), A.col.astype(np.int64), A.n)
        keys = D.edge_keys(seed, 0, A.n, eu, ev)
        forest = D.kruskal_forest(A.n, eu, ev, keys)
        rank = np.empty(keys.shape[0], np.float64)
        rank[np.argsort(keys, kind="stable")] = np.arange(1, keys.shape[0] + 1)
        M = sp.coo_matrix((rank, (eu, ev)), shape=(A.n, A.n)).tocsr()
        T = minimum_spanning_tree(M).tocoo()
        ref = {tuple(sorted((int(a), int(c)))) for a, c in zip(T.row, T.col)}
        assert {tuple(sorted(x)) for x in forest} == ref
    del rng


def test_splitmix64_published_sequence():
    # Output of the SplitMix64 reference generator seeded with 1234567.
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [D.splitmix64_output(1234567, c) for c in range(5)] == ref
    u = np.array([0, 3, 7], np.int64)
    v = np.array([1, 9, 8], np.int64)
    k = D.edge_keys(5, 2, 10, u, v)
    s = D.level_seed(5, 2)
    assert [int(x) for x in k] == [D.splitmix64_output(s, int(a) * 10 + int(c))
                                   for a, c in zip(u, v)]


# ---------------------------------------------------------------------------
# storage formats
# ---------------------------------------------------------------------------

torch = pytest.importorskip("torch")


def test_decode_all_codes_match_torch():
    codes8 = np.arange(256, dtype=np.uint8)
    ref8 = torch.from_numpy(codes8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got8 = Q.decode(codes8, "f8e4m3")
    assert np.array_equal(np.isnan(got8), np.isnan(ref8))
    assert np.array_equal(got8[~np.isnan(ref8)], ref8[~np.isnan(ref8)])
    codes16 = np.arange(65536, dtype=np.uint16)
    for fmt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        ref = torch.from_numpy(codes16.view(np.int16)).view(tdt).to(torch.float64).numpy()
        got = Q.decode(codes16, fmt)
        fin = np.isfinite(ref)
        assert np.array_equal(got[fin], ref[fin])
        assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(200000) * np.exp(rng.uniform(-25, 8, 200000)),
        rng.uniform(-460, 460, 50000),
        Q.decode(np.arange(256, dtype=np.uint8), "f8e4m3")[:-1] * 1.0000001,
    ]).astype(np.float32)
    x = x[np.isfinite(x)]
    for fmt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16),
                     ("f8e4m3", torch.float8_e4m3fn)):
        vmax = Q.FORMATS[fmt][2]
        xs = x[np.abs(x) <= vmax]
        ref = torch.from_numpy(xs).to(tdt).to(torch.float64).numpy()
        got = Q.quantize(xs.astype(np.float64), fmt)
        assert np.array_equal(got, ref), fmt
        codes = Q.encode(xs.astype(np.float64), fmt)
        assert np.array_equal(Q.decode(codes, fmt), got)
        assert np.all(np.abs(got - xs) <= 0.5 * Q.spacing(xs, fmt))
