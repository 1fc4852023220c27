"""More pins of the oracle (CPU only): the error metric behind every parity
gate, the storage spacing behind the element-wise precision bound, and the
counting step of the LA-Decompose lemma (Section 5.1)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import decomp as D
from oracle import quant as Q
from oracle import spmm as S


# ---------------------------------------------------------------------------
# relative Frobenius error: values fixed by hand
# ---------------------------------------------------------------------------

def test_rel_fro_hand_values():
    # ||a - ref||_F = 3, ||ref||_F = 4 (a missing square root would give 9/16)
    assert S.rel_fro([[3.0, 0.0], [0.0, 4.0]], [[0.0, 0.0], [0.0, 4.0]]) == 0.75
    # 3-4-5 triangle across two entries: ||(3, 4)|| / ||(0, 12) + (5, 0)|| = 5 / 13
    assert math.isclose(S.rel_fro([[8.0], [16.0]], [[5.0], [12.0]]), 5.0 / 13.0,
                        rel_tol=0, abs_tol=1e-16)
    # every entry counts: an error in the second column alone
    assert math.isclose(S.rel_fro([[1.0, 2.0], [0.0, 0.0]], [[1.0, 0.0], [0.0, 0.0]]), 2.0,
                        rel_tol=0, abs_tol=1e-16)


def test_rel_fro_scaled_copy_and_zero_reference():
    rng = np.random.default_rng(3)
    ref = rng.standard_normal((50, 7))
    for c in (0.0, 0.5, 1.0, 1.25, -1.0):
        assert math.isclose(S.rel_fro(c * ref, ref), abs(c - 1.0), rel_tol=1e-14, abs_tol=1e-15)
    # zero reference: the absolute error (0 / 0 -> 0)
    z = np.zeros((4, 3))
    assert S.rel_fro(z, z) == 0.0
    a = np.zeros((4, 3))
    a[1, 2] = -2.0
    assert S.rel_fro(a, z) == 2.0
    # symmetric in the sign of the difference, not in its arguments
    assert S.rel_fro(ref + 1.0, ref) == S.rel_fro(ref - 1.0, ref)


# ---------------------------------------------------------------------------
# storage spacing: exact powers of two from the format definitions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fmt,x,expect", [
    ("f16", 1.0, 2.0 ** -10),          # 10 fraction bits
    ("f16", 1.5, 2.0 ** -10),
    ("f16", 2.0, 2.0 ** -9),           # the binade above a power of two
    ("f16", 65504.0, 32.0),            # largest finite, binade [2^15, 2^16)
    ("f16", 6.1e-5, 2.0 ** -24),       # below 2^-14: subnormal spacing
    ("f16", 2.0 ** -14, 2.0 ** -24),   # smallest normal
    ("bf16", 3.0, 2.0 ** -6),          # 7 fraction bits, binade [2, 4)
    ("bf16", 1.0, 2.0 ** -7),
    ("bf16", -0.75, 2.0 ** -8),        # sign does not matter
    ("f8e4m3", 448.0, 32.0),           # 3 fraction bits, binade [256, 512)
    ("f8e4m3", 1.0, 2.0 ** -3),
    ("f8e4m3", 0.001, 2.0 ** -9),      # below 2^-6: subnormal spacing
    ("f8e4m3", 2.0 ** -6, 2.0 ** -9),
    ("f8e4m3", 0.0, 2.0 ** -9),
])
def test_spacing_hand_values(fmt, x, expect):
    assert float(Q.spacing(np.array([x]), fmt)[0]) == expect


def test_spacing_f16_matches_numpy():
    # numpy's spacing of IEEE binary16 (a library routine), on positive values
    rng = np.random.default_rng(1)
    x = np.concatenate([np.exp(rng.uniform(np.log(1e-7), np.log(6.0e4), 20000)),
                        2.0 ** np.arange(-24, 16, dtype=np.float64)]).astype(np.float16)
    x = x[(x > 0) & np.isfinite(x)]
    ref = np.spacing(x).astype(np.float64)
    got = Q.spacing(x.astype(np.float64), "f16")
    assert np.array_equal(got, ref)


def test_spacing_is_the_gap_between_codes():
    # consecutive positive finite codes differ by exactly the spacing of the lower one
    for fmt, codes in (("f8e4m3", np.arange(0, 0x7E, dtype=np.uint8)),
                       ("f16", np.arange(0, 0x7BFF, dtype=np.uint16)),
                       ("bf16", np.arange(0, 0x7F7F, 7, dtype=np.uint16))):
        lo = Q.decode(codes, fmt)
        hi = Q.decode(codes + 1, fmt)
        assert np.array_equal(hi - lo, Q.spacing(lo, fmt)), fmt


# ---------------------------------------------------------------------------
# Section 5.1, LA-Decompose lemma: the counting (Markov) step.  In level i the
# edges of G'_i farther than b from the diagonal number at most
# lambda_{pi'_i}(G'_i) / (b + 1), and they are exactly the edges left to the
# next levels (every edge at a head vertex, and every band edge, lands in B_i).
# ---------------------------------------------------------------------------

def _remaining_edges(levels, start, n):
    """Undirected off-diagonal vertex pairs stored in levels >= start."""
    keys = []
    for L in levels[start:]:
        vop = np.asarray(L["vop"], dtype=np.int64)
        rp = np.asarray(L["row_ptr"], dtype=np.int64)
        p = np.repeat(np.arange(L["n_i"], dtype=np.int64), np.diff(rp))
        u, v = vop[p], vop[np.asarray(L["col"], dtype=np.int64)]
        off = u != v
        a, c = np.minimum(u[off], v[off]), np.maximum(u[off], v[off])
        keys.append(a * n + c)
    return np.unique(np.concatenate(keys)) if keys else np.zeros(0, dtype=np.int64)


def _lemma_graphs():
    out = [("rmat10", W.make_matrix("rmat", 10, "row_normalized", 21, 22, 16), 8),
           ("rmat10_b32", W.make_matrix("rmat", 10, "row_normalized", 23, 24, 16), 32),
           ("grid2d_24", W.make_matrix("grid2d", 24, "uniform", 25, 26), 4),
           ("grid3d_8", W.make_matrix("grid3d", 8, "uniform", 27, 28), 6),
           ("random_300", W.random_graph(300, 0.03, 29, diagonal=True), 5)]
    return out


@pytest.mark.parametrize("la", ["random_forest", "identity"])
@pytest.mark.parametrize("case", range(5))
def test_la_decompose_lemma_counting_step(case, la):
    name, A, b = _lemma_graphs()[case]
    trace = []
    levels = D.la_decompose(A, b, seed=7, la=la, trace=trace)
    D.validate(A, levels, b)
    assert len(trace) == len(levels)
    n = A.n
    checked = 0
    for i, tr in enumerate(trace):
        if tr["final"]:
            continue
        pos = tr["pos"]
        head = set(int(h) for h in tr["head"])
        gu, gv = tr["gu"], tr["gv"]
        assert not any(int(u) in head or int(v) in head for u, v in zip(gu, gv))
        dist = np.abs(pos[gu] - pos[gv])
        lam = int(dist.sum())                     # lambda_{pi'_i}(G'_i)
        far = dist > b
        # Markov: (b + 1) * #far <= sum of distances
        assert int(far.sum()) * (b + 1) <= lam, (name, i)
        # the far edges are exactly what the later levels hold
        want = np.unique(np.minimum(gu[far], gv[far]) * n + np.maximum(gu[far], gv[far]))
        assert np.array_equal(_remaining_edges(levels, i + 1, n), want), (name, i)
        checked += 1
    assert checked >= 1


# ---------------------------------------------------------------------------
# separator arrangement (Section 5.2): properties fixed by the definition and
# the bound of Table 1, checked with scipy's connected components
# ---------------------------------------------------------------------------

def _arrangement(A):
    eu, ev = D._undirected_edges(A.rows(), np.asarray(A.col, np.int64), A.n)
    order, singles = D.separator_arrangement(A.n, np.ones(A.n, dtype=bool), eu, ev)
    pos = np.full(A.n, -1, dtype=np.int64)
    pos[np.asarray(order, dtype=np.int64)] = np.arange(len(order))
    return eu, ev, order, singles, pos


def _scipy_components(n, eu, ev, keep):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    m = keep[eu] & keep[ev]
    G = sp.coo_matrix((np.ones(int(m.sum())), (eu[m], ev[m])), shape=(n, n))
    _, lab = connected_components(G, directed=False)
    return lab


@pytest.mark.parametrize("side", [6, 9, 16, 25])
def test_separator_top_level_is_a_two_thirds_separator_placed_first(side):
    """On a connected grid the first vertices placed form a separator S whose
    removal leaves components of at most 2n/3 vertices; after S every
    component occupies one contiguous range of positions, in increasing size."""
    A = W.make_matrix("grid2d", side, "uniform", 0, 1)
    eu, ev, order, singles, pos = _arrangement(A)
    n = A.n
    assert len(order) == n and singles.size == 0 and np.all(pos >= 0)
    # S = the longest prefix whose removal disconnects what follows, found by
    # growing the prefix until the rest is disconnected (or empty)
    for s_len in range(1, n + 1):
        keep = np.ones(n, dtype=bool)
        keep[np.asarray(order[:s_len])] = False
        lab = _scipy_components(n, eu, ev, keep)
        comps = np.unique(lab[keep])
        if comps.size >= 2:
            break
    sizes = np.array([np.count_nonzero(lab[keep] == c) for c in comps])
    assert sizes.max() * 3 <= 2 * n
    # each component contiguous after S, components in increasing size
    starts = []
    for c in comps:
        p = np.sort(pos[np.flatnonzero(keep & (lab == c))])
        assert p[-1] - p[0] + 1 == p.size
        starts.append((p[0], p.size))
    starts.sort()
    assert starts[0][0] == s_len
    assert [sz for _, sz in starts] == sorted(sz for _, sz in starts)


def test_separator_cost_bounds():
    """Table 1: planar graphs (2D grids, max degree 4) get an arrangement of
    cost O(n Delta sqrt(n)) -- the ratio stays below a constant while a random
    order grows like sqrt(n); a path gets at most n log2 n."""
    ratios = []
    for side in (8, 16, 32, 48):
        A = W.make_matrix("grid2d", side, "uniform", 0, 1)
        eu, ev, _, _, pos = _arrangement(A)
        n = A.n
        lam = np.abs(pos[eu] - pos[ev]).sum()
        rnd = np.random.default_rng(side).permutation(n)
        lam_rnd = np.abs(rnd[eu] - rnd[ev]).sum()
        ratios.append(lam / (n * 4 * math.sqrt(n)))
        assert lam < lam_rnd
    assert max(ratios) <= 1.5
    for n in (64, 256, 1024):
        lab = np.random.default_rng(n).permutation(n)
        eu = np.minimum(lab[:-1], lab[1:])
        ev = np.maximum(lab[:-1], lab[1:])
        order, singles = D.separator_arrangement(n, np.ones(n, dtype=bool), eu, ev)
        pos = np.empty(n, dtype=np.int64)
        pos[np.asarray(order)] = np.arange(n)
        assert np.abs(pos[eu] - pos[ev]).sum() <= n * math.log2(n)


def test_separator_decompositions_are_valid():
    for A, b in ((W.make_matrix("grid2d", 24, "sym_laplacian", 0, 1), 8),
                 (W.make_matrix("grid3d", 7, "sym_laplacian", 0, 1), 16),
                 (W.make_matrix("rmat", 10, "row_normalized", 5, 6, 8), 16),
                 (W.random_graph(200, 0.02, 4), 4)):
        D.validate(A, D.la_decompose(A, b, seed=2, la="separator"), b)


# ---------------------------------------------------------------------------
# GNN-style step ReLU((A X) W)
# ---------------------------------------------------------------------------

def test_gnn_layer_brute_force_and_special_weights():
    A = W.random_graph(30, 0.15, 7, values="uniform", diagonal=True)
    rng = np.random.default_rng(8)
    k = 5
    X = rng.standard_normal((A.n, k))
    Wm = rng.standard_normal((k, k))
    Z = S.gnn_layer(A, X, Wm)
    ref = np.array(S.gnn_brute_force(A, X.tolist(), Wm.tolist()))
    assert np.allclose(Z, ref, rtol=1e-12, atol=1e-12)
    assert np.all(Z >= 0) and np.any(Z > 0) and np.any(Z == 0)
    Y = S.csr_spmm(A, X)
    # a permutation matrix moves column j of A X to column perm[j] (a transposed
    # weight would move it to inv[j] instead)
    perm = np.array([2, 0, 4, 1, 3])
    P = np.zeros((k, k))
    P[np.arange(k), perm] = 1.0
    Zp = S.gnn_layer(A, X, P)
    for j in range(k):
        assert np.array_equal(Zp[:, perm[j]], np.maximum(Y[:, j], 0.0))
    # a diagonal weight scales each column, ReLU keeps the positive part
    d = np.array([2.0, -1.0, 0.5, -3.0, 0.0])
    Zd = S.gnn_layer(A, X, np.diag(d))
    for j in range(k):
        assert np.array_equal(Zd[:, j], np.maximum(d[j] * Y[:, j], 0.0))
