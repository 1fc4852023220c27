"""ORACLE (test infrastructure only): arrow decomposition reference and validator.

Paper: Gianinazzi et al., "Arrow Matrix Decomposition" (PPoPP'24).

Representation of a decomposition (shared *format* with the library's export,
no shared code): a list of levels, each a dict with

* ``n_i``   -- number of positions of the level (level 0: n),
* ``vop``   -- int32[n_i], the vertex at each position (pi_i^{-1} restricted to
               [0, n_i)),
* ``row_ptr``/``col``/``val`` -- CSR of B_i over positions, columns sorted.

Validator (pinned: exact invariants, brute-force dense check, worked example
of Fig. 3):

1. every map is injective into [0, n); level 0 is a bijection on [0, n)
   (the decomposition of Section 4 uses full permutations P_{pi_i}),
2. every stored (p, q) of B_i satisfies the arrow-width predicate of
   Section 1 (0-based: p < b or q < b or |p - q| <= b),
3. the multiset {(vop_i[p], vop_i[q], bits(v))} over all levels equals the
   multiset of A's stored entries (every entry in exactly one B_i, Section 4
   Eq. (1) and the storage lemma of Section 6.2).

Reference LA-Decompose (Section 5.1) with random spanning forest linear
arrangements (Section 5.3) and smallest-first tree order (Section 5.4), or
the separator arrangement (Section 5.2), with the readings of the points the
paper leaves open:

* degrees are taken in the undirected graph G_i of the symmetrised remaining
  pattern, self loops excluded;
* head = the b vertices of positive degree with the largest degree, ties to
  the smaller vertex id (fewer than b if fewer have positive degree);
* the standard-uniform edge weights are 64-bit SplitMix64 outputs
  (counter-based, see :func:`edge_keys`); the minimum spanning forest is
  unique under distinct keys, ties broken by (u, v);
* every tree is rooted at its smallest vertex id and laid out in
  smallest-first preorder, children by (subtree size, id) ascending;
* trees follow the head in decreasing size, ties by root id; trees of one
  vertex that still hold entries (to the head) come next, then vertices
  without entries, each group by id;
* separator arrangement: components in increasing size (ties by smallest
  id); the separator of a connected set is the first BFS level (from a
  pseudo-peripheral vertex: the last vertex reached by a BFS from the
  smallest id) at which the BFS has reached half of the set; BFS visits
  neighbours by id; vertices without edges in G'_i follow as for the
  forest;
* an entry (u, v) goes to B_i when its positions satisfy the arrow predicate,
  otherwise to A_{i+1};
* the loop runs while nnz(A_i) > 2b counted on the symmetrised pattern; the
  leftover (at most b undirected edges) forms a last level whose head is a
  greedy vertex cover (largest remaining degree first, ties by id), so it has
  at most b vertices and holds every leftover edge;
* level 0 always spans all n positions; later levels are compacted to
  n_i = 1 + the largest position holding an entry (the non-zeros are
  collected at the top, Section 4).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


# ---------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood: "Fast splittable pseudorandom number
# generators", OOPSLA 2014), used counter-based: output c of the generator
# with initial state s is mix(s + (c + 1) * GAMMA) mod 2^64.
# ---------------------------------------------------------------------------

def splitmix64_mix(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_output(state: int, c: int) -> int:
    return splitmix64_mix((state + (c + 1) * GAMMA) & MASK64)


def level_seed(seed: int, level: int) -> int:
    """Per-level stream seed: output `level` of the generator seeded with `seed`."""
    return splitmix64_output(seed & MASK64, level)


def edge_keys(seed: int, level: int, n: int, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Random weight of each undirected edge {u, v} (u < v) at a level: output
    u*n + v of the generator seeded with the level seed, as uint64."""
    s = np.uint64(level_seed(seed, level))
    c = u.astype(np.uint64) * np.uint64(n) + v.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = s + (c + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


# ---------------------------------------------------------------------------
# predicate and validator
# ---------------------------------------------------------------------------

def in_arrow(p, q, b):
    """Arrow-width-b predicate (Section 1), 0-based positions."""
    p = np.asarray(p, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    return (p < b) | (q < b) | (np.abs(p - q) <= b)


class InvalidDecomposition(AssertionError):
    pass


def validate(csr, levels, b: int) -> None:
    """Raise InvalidDecomposition unless `levels` is an exact b-arrow
    decomposition of `csr` (checks 1-3 of the module docstring)."""
    n = csr.n
    if len(levels) == 0:
        raise InvalidDecomposition("no levels")
    triples = []
    for i, L in enumerate(levels):
        n_i = int(L["n_i"])
        vop = np.asarray(L["vop"], dtype=np.int64)
        rp = np.asarray(L["row_ptr"], dtype=np.int64)
        col = np.asarray(L["col"], dtype=np.int64)
        val = np.asarray(L["val"], dtype=np.float32)
        if vop.shape != (n_i,) or rp.shape != (n_i + 1,):
            raise InvalidDecomposition(f"level {i}: shape mismatch")
        if n_i and (vop.min() < 0 or vop.max() >= n):
            raise InvalidDecomposition(f"level {i}: vertex out of range")
        if np.unique(vop).shape[0] != n_i:
            raise InvalidDecomposition(f"level {i}: map not injective")
        if i == 0 and n_i != n:
            raise InvalidDecomposition("level 0 is not a bijection on [0, n)")
        if rp[0] != 0 or np.any(np.diff(rp) < 0) or rp[-1] != col.shape[0]:
            raise InvalidDecomposition(f"level {i}: bad row pointers")
        if col.shape[0] and (col.min() < 0 or col.max() >= n_i):
            raise InvalidDecomposition(f"level {i}: column out of range")
        p = np.repeat(np.arange(n_i, dtype=np.int64), np.diff(rp))
        if not np.all(in_arrow(p, col, b)):
            bad = np.flatnonzero(~in_arrow(p, col, b))[0]
            raise InvalidDecomposition(
                f"level {i}: entry ({p[bad]}, {col[bad]}) outside arrow width {b}")
        triples.append((vop[p], vop[col], val.view(np.uint32)))
    u = np.concatenate([t[0] for t in triples])
    v = np.concatenate([t[1] for t in triples])
    bits = np.concatenate([t[2] for t in triples])
    order = np.lexsort((bits, v, u))
    ref_u = csr.rows()
    ref_v = np.asarray(csr.col, dtype=np.int64)
    ref_bits = np.asarray(csr.val, dtype=np.float32).view(np.uint32)
    ref_order = np.lexsort((ref_bits, ref_v, ref_u))
    if u.shape[0] != ref_u.shape[0]:
        raise InvalidDecomposition(
            f"entry count {u.shape[0]} != nnz(A) {ref_u.shape[0]}")
    if not (np.array_equal(u[order], ref_u[ref_order]) and
            np.array_equal(v[order], ref_v[ref_order]) and
            np.array_equal(bits[order], ref_bits[ref_order])):
        raise InvalidDecomposition("entries do not rebuild A exactly")


def dense_sum(levels, n: int) -> np.ndarray:
    """sum_i P_{pi_i} B_i P_{pi_i}^T as a dense FP64 matrix (tiny inputs)."""
    A = np.zeros((n, n), dtype=np.float64)
    for L in levels:
        vop = np.asarray(L["vop"], dtype=np.int64)
        rp = np.asarray(L["row_ptr"], dtype=np.int64)
        p = np.repeat(np.arange(int(L["n_i"]), dtype=np.int64), np.diff(rp))
        q = np.asarray(L["col"], dtype=np.int64)
        np.add.at(A, (vop[p], vop[q]), np.asarray(L["val"], np.float64))
    return A


def product_via_levels(levels, n: int, X) -> np.ndarray:
    """Eq. (1): sum_i P_i (B_i (P_i^T X)) evaluated level by level in FP64."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.zeros_like(X)
    for L in levels:
        n_i = int(L["n_i"])
        vop = np.asarray(L["vop"], dtype=np.int64)
        B = np.zeros((n_i, n_i), dtype=np.float64)
        rp = np.asarray(L["row_ptr"], dtype=np.int64)
        p = np.repeat(np.arange(n_i, dtype=np.int64), np.diff(rp))
        B[p, np.asarray(L["col"], dtype=np.int64)] = np.asarray(L["val"], np.float64)
        Xi = X[vop]            # P_i^T X restricted to the level's positions
        Y[vop] += B @ Xi       # scatter back through P_i
    return Y


# ---------------------------------------------------------------------------
# reference LA-Decompose
# ---------------------------------------------------------------------------

def _undirected_edges(r: np.ndarray, c: np.ndarray, n: int):
    off = r != c
    u = np.minimum(r[off], c[off])
    v = np.maximum(r[off], c[off])
    key = np.unique(u * max(n, 1) + v)
    return key // max(n, 1), key % max(n, 1)


def _degrees(eu, ev, n):
    return np.bincount(np.concatenate([eu, ev]), minlength=n).astype(np.int64)


def _head_by_degree(deg, b):
    cand = np.flatnonzero(deg > 0)
    order = np.lexsort((cand, -deg[cand]))  # degree desc, id asc
    return cand[order][:b]


def _greedy_cover(eu, ev, n):
    """Greedy vertex cover: repeatedly take the vertex with the most uncovered
    edges (ties: smaller id)."""
    eu = [int(x) for x in eu]
    ev = [int(x) for x in ev]
    alive = [True] * len(eu)
    cover = []
    while True:
        deg = {}
        for e in range(len(eu)):
            if alive[e]:
                deg[eu[e]] = deg.get(eu[e], 0) + 1
                deg[ev[e]] = deg.get(ev[e], 0) + 1
        if not deg:
            return np.asarray(cover, dtype=np.int64)
        best = min(deg, key=lambda x: (-deg[x], x))
        cover.append(best)
        for e in range(len(eu)):
            if alive[e] and (eu[e] == best or ev[e] == best):
                alive[e] = False


def kruskal_forest(n, eu, ev, keys):
    """Minimum spanning forest by Kruskal: edges by (key, u, v) ascending,
    union-find.  Returns the list of forest edges."""
    order = np.lexsort((ev, eu, keys))
    parent = list(range(n))

    def find(x):
        root = x
        while parent[root] != root:
            root = parent[root]
        while parent[x] != root:
            parent[x], x = root, parent[x]
        return root

    out = []
    for e in order:
        a, c = int(eu[e]), int(ev[e])
        ra, rc = find(a), find(c)
        if ra != rc:
            parent[max(ra, rc)] = min(ra, rc)
            out.append((a, c))
    return out


def smallest_first_order(vertices, tree_edges):
    """Smallest-first layout of one tree (Section 5.4): the root first, then
    the child subtrees one after the other in increasing size (ties by child
    id), each laid out recursively.  Root = smallest vertex id."""
    adj = {v: [] for v in vertices}
    for a, c in tree_edges:
        adj[a].append(c)
        adj[c].append(a)
    root = min(vertices)
    parent = {root: None}
    order = [root]
    for v in order:  # BFS to orient the tree
        for w in adj[v]:
            if w != parent[v]:
                parent[w] = v
                order.append(w)
    size = {v: 1 for v in vertices}
    for v in reversed(order):
        if parent[v] is not None:
            size[parent[v]] += size[v]
    children = {v: sorted((w for w in adj[v] if w != parent[v]), key=lambda w: (size[w], w))
                for v in vertices}
    layout = []
    stack = [root]
    while stack:
        v = stack.pop()
        layout.append(v)
        stack.extend(reversed(children[v]))
    return layout


def random_forest_arrangement(n, verts_mask, eu, ev, seed, level):
    """Random spanning forest linear arrangement (Section 5.3) of the graph on
    the vertices where verts_mask is true.  Returns (tree vertex order,
    singleton vertices) -- trees of >= 2 vertices in decreasing size (ties by
    root id), each in smallest-first order."""
    keys = edge_keys(seed, level, n, eu, ev)
    forest = kruskal_forest(n, eu, ev, keys)
    comp = {}
    adj_edges = {}
    # components of the forest
    parent = {}

    def find(x):
        while parent.get(x, x) != x:
            x = parent[x]
        return x

    for a, c in forest:
        ra, rc = find(a), find(c)
        parent.setdefault(ra, ra)
        parent.setdefault(rc, rc)
        if ra != rc:
            parent[max(ra, rc)] = min(ra, rc)
    for a, c in forest:
        r = find(a)
        comp.setdefault(r, set()).update((a, c))
        adj_edges.setdefault(r, []).append((a, c))
    trees = []
    for r, vs in comp.items():
        vs = sorted(vs)
        trees.append((len(vs), vs[0], vs, adj_edges[r]))
    trees.sort(key=lambda t: (-t[0], t[1]))
    tree_order = []
    in_tree = np.zeros(n, dtype=bool)
    for _, _, vs, es in trees:
        tree_order.extend(smallest_first_order(vs, es))
        in_tree[vs] = True
    singles = np.flatnonzero(verts_mask & ~in_tree)
    return tree_order, singles


def _components(vertices, adj, alive):
    """Connected components of the subgraph induced on `vertices` (alive),
    each a list in BFS order from its smallest vertex (neighbours by id)."""
    seen = set()
    comps = []
    for v0 in sorted(vertices):
        if v0 in seen:
            continue
        seen.add(v0)
        comp = [v0]
        for v in comp:
            for w in adj[v]:
                if alive[w] and w not in seen:
                    seen.add(w)
                    comp.append(w)
        comps.append(comp)
    return comps


def _bfs_levels(start, adj, alive):
    """BFS levels from `start` inside the alive vertices (neighbours by id)."""
    levels = [[start]]
    seen = {start}
    while True:
        nxt = []
        for v in levels[-1]:
            for w in adj[v]:
                if alive[w] and w not in seen:
                    seen.add(w)
                    nxt.append(w)
        if not nxt:
            return levels
        levels.append(nxt)


def separator_arrangement(n, verts_mask, eu, ev):
    """Separator-LA (Section 5.2) of the graph on the vertices where verts_mask
    is true.  A vertex set is arranged as: its connected components in
    increasing size (ties by smallest id), each arranged recursively; a
    connected set places a separator S first and then arranges the rest.  S
    is a level of a BFS level structure: start at the smallest vertex, restart
    from the last vertex that BFS reaches (a pseudo-peripheral vertex), and
    take the first level at which the BFS from there has reached at least
    half of the set.  Returns (order of the vertices in components of >= 2
    vertices, singleton vertices), like the random-forest arrangement."""
    adj = {}
    for a, c in zip(eu.tolist(), ev.tolist()):
        adj.setdefault(a, []).append(c)
        adj.setdefault(c, []).append(a)
    for v in adj:
        adj[v].sort()
    if not adj:
        return [], np.flatnonzero(verts_mask)
    alive = np.zeros(n, dtype=bool)
    alive[list(adj)] = True
    order = []
    # work items: ("set", vertices) arranges a set, ("place", vertices) emits
    stack = [("set", sorted(adj))]
    while stack:
        kind, vs = stack.pop()
        if kind == "place":
            order.extend(vs)
            continue
        comps = _components(vs, adj, alive)
        if len(comps) > 1:
            comps.sort(key=lambda cc: (len(cc), min(cc)))
            for cc in reversed(comps):
                stack.append(("set", cc))
            continue
        comp = comps[0]
        if len(comp) == 1:
            order.append(comp[0])
            alive[comp[0]] = False
            continue
        last = _bfs_levels(min(comp), adj, alive)[-1][-1]
        levels = _bfs_levels(last, adj, alive)
        reached = 0
        for lev in levels:
            reached += len(lev)
            if 2 * reached >= len(comp):
                sep = lev
                break
        for v in sep:
            alive[v] = False
        rest = [v for v in comp if alive[v]]
        if rest:
            stack.append(("set", rest))
        stack.append(("place", sep))
    singles = np.flatnonzero(verts_mask & ~np.isin(np.arange(n), np.asarray(order, dtype=np.int64)))
    return order, singles


def la_decompose(csr, b: int, seed: int = 0, la: str = "random_forest", trace=None):
    """Reference LA-Decompose.  Returns the list of levels (see module doc).

    If `trace` is a list, one dict per level is appended to it: the head
    vertices, the full position map `pos` (vertex -> position in pi_i, all n
    vertices) and the undirected edges (u < v) of G'_i, the graph on the
    non-head vertices (empty for the final vertex-cover level).  Tests use it
    to check the counting step of the LA-Decompose lemma."""
    if b < 2:
        raise ValueError("arrow width b must be >= 2")
    n = csr.n
    r = csr.rows()
    c = np.asarray(csr.col, dtype=np.int64)
    val = np.asarray(csr.val, dtype=np.float32)
    levels = []
    level = 0
    while True:
        eu, ev = _undirected_edges(r, c, n)
        n_diag = int(np.count_nonzero(r == c))
        if r.shape[0] == 0 and level > 0:
            break
        has_entry = np.zeros(n, dtype=bool)
        has_entry[r] = True
        has_entry[c] = True
        final = 2 * eu.shape[0] + n_diag <= 2 * b
        if final:
            head = _greedy_cover(eu, ev, n)
            is_head = np.zeros(n, dtype=bool)
            is_head[head] = True
            tree_order = []
            singles = np.flatnonzero(~is_head & has_entry)
        else:
            deg = _degrees(eu, ev, n)
            head = _head_by_degree(deg, b)
            is_head = np.zeros(n, dtype=bool)
            is_head[head] = True
            keep_e = ~is_head[eu] & ~is_head[ev]
            if la == "random_forest":
                tree_order, singles = random_forest_arrangement(
                    n, ~is_head & has_entry, eu[keep_e], ev[keep_e], seed, level)
            elif la == "separator":
                tree_order, singles = separator_arrangement(
                    n, ~is_head & has_entry, eu[keep_e], ev[keep_e])
            elif la == "identity":
                tree_order, singles = [], np.flatnonzero(~is_head & has_entry)
            else:
                raise ValueError(la)
        placed = np.zeros(n, dtype=bool)
        order = list(int(x) for x in head)
        placed[head] = True
        order.extend(tree_order)
        placed[np.asarray(tree_order, dtype=np.int64)] = True
        order.extend(int(x) for x in singles)
        placed[singles] = True
        order.extend(int(x) for x in np.flatnonzero(~placed))
        order = np.asarray(order, dtype=np.int64)
        assert order.shape[0] == n
        pos = np.empty(n, dtype=np.int64)
        pos[order] = np.arange(n, dtype=np.int64)
        p, q = pos[r], pos[c]
        keep = in_arrow(p, q, b)
        if final:
            assert np.all(keep)
        if trace is not None:
            if final:
                gu = gv = np.zeros(0, dtype=np.int64)
            else:
                gu, gv = eu[keep_e], ev[keep_e]
            trace.append(dict(head=np.asarray(head, dtype=np.int64), pos=pos.copy(),
                              gu=gu.astype(np.int64), gv=gv.astype(np.int64), final=final))
        kp, kq, kv = p[keep], q[keep], val[keep]
        if level == 0:
            n_i = n
        else:
            n_i = int(max(kp.max(), kq.max()) + 1) if kp.shape[0] else 0
        srt = np.lexsort((kq, kp))
        kp, kq, kv = kp[srt], kq[srt], kv[srt]
        rp = np.zeros(n_i + 1, dtype=np.int64)
        np.cumsum(np.bincount(kp, minlength=n_i), out=rp[1:])
        levels.append(dict(n_i=n_i, vop=order[:n_i].astype(np.int32), row_ptr=rp,
                           col=kq.astype(np.int32), val=kv))
        r, c, val = r[~keep], c[~keep], val[~keep]
        level += 1
        if r.shape[0] == 0:
            break
    return levels
