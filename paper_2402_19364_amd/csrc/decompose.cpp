// Host LA-Decompose (Section 4.1) with the random spanning forest linear
// arrangement (Section 4.3) and smallest-first tree order (Section 4.4).
//
// Per level i, on the undirected graph G_i of the symmetrised remaining
// pattern (self loops excluded):
//   1. head H_i: the b vertices of positive degree with the largest degree
//      (ties to the smaller id); they take positions 0 .. |H_i|-1,
//   2. every edge of G_i - H_i gets a 64-bit random weight (counter-based
//      SplitMix64 keyed by level and edge); Kruskal builds the unique minimum
//      spanning forest, ties by (u, v),
//   3. each tree is rooted at its smallest id and laid out in smallest-first
//      preorder (children by subtree size, then id); trees follow the head in
//      decreasing size (ties: root id); then single vertices that still hold
//      entries, then the rest, both by id,
//   4. a stored entry (u, v) goes to B_i when its positions (p, q) satisfy
//      p < b or q < b or |p - q| <= b, otherwise to A_{i+1}.
// The loop runs while nnz(A_i) > 2b (Section 4.1), counted on the symmetrised
// pattern; the leftover (at most b edges) becomes a last level whose head is a
// greedy vertex cover (most uncovered edges first, ties by id).  Level 0 spans
// all n positions; later levels keep positions [0, 1 + largest used).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <set>
#include <string>

#include "internal.h"

namespace arrow {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// Output c of the SplitMix64 generator started at state s.
inline uint64_t sm_output(uint64_t s, uint64_t c) { return sm_mix(s + (c + 1) * kGamma); }

int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

// Stable LSD radix sort of (key, payload) pairs by key, using only the low
// `bits` bits of the key.
void radix_sort(std::vector<uint64_t> &key, std::vector<uint32_t> &pay, int bits) {
    const size_t m = key.size();
    std::vector<uint64_t> k2(m);
    std::vector<uint32_t> p2(m);
    for (int shift = 0; shift < bits; shift += 8) {
        size_t cnt[257] = {0};
        for (size_t i = 0; i < m; ++i) ++cnt[((key[i] >> shift) & 0xFF) + 1];
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < m; ++i) {
            size_t dst = cnt[(key[i] >> shift) & 0xFF]++;
            k2[dst] = key[i];
            p2[dst] = pay[i];
        }
        key.swap(k2);
        pay.swap(p2);
    }
}

void radix_sort_keys(std::vector<uint64_t> &key, int bits) {
    const size_t m = key.size();
    std::vector<uint64_t> k2(m);
    for (int shift = 0; shift < bits; shift += 8) {
        size_t cnt[257] = {0};
        for (size_t i = 0; i < m; ++i) ++cnt[((key[i] >> shift) & 0xFF) + 1];
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < m; ++i) k2[cnt[(key[i] >> shift) & 0xFF]++] = key[i];
        key.swap(k2);
    }
}

struct Entries {  // remaining stored entries, in CSR order of A
    std::vector<int32_t> r, c;
    std::vector<float> v;
    size_t size() const { return r.size(); }
};

struct UnionFind {
    std::vector<int32_t> parent;
    explicit UnionFind(int64_t n) : parent(n) { std::iota(parent.begin(), parent.end(), 0); }
    int32_t find(int32_t x) {
        int32_t root = x;
        while (parent[root] != root) root = parent[root];
        while (parent[x] != root) {
            int32_t nx = parent[x];
            parent[x] = root;
            x = nx;
        }
        return root;
    }
};

// Smallest-first layouts of the trees of a forest over n vertices, trees in
// decreasing size (ties: smaller root).  Appends to `order`, marks `placed`.
void layout_forest(int64_t n, const std::vector<int32_t> &fu, const std::vector<int32_t> &fv,
                   std::vector<int32_t> &order, std::vector<uint8_t> &placed) {
    const size_t m = fu.size();
    if (m == 0) return;
    std::vector<int64_t> aptr(n + 1, 0);
    for (size_t e = 0; e < m; ++e) {
        ++aptr[fu[e] + 1];
        ++aptr[fv[e] + 1];
    }
    for (int64_t i = 0; i < n; ++i) aptr[i + 1] += aptr[i];
    std::vector<int32_t> adj(2 * m);
    {
        std::vector<int64_t> fill(aptr.begin(), aptr.end() - 1);
        for (size_t e = 0; e < m; ++e) {
            adj[fill[fu[e]]++] = fv[e];
            adj[fill[fv[e]]++] = fu[e];
        }
    }
    std::vector<int32_t> parent(n, -1), size(n, 0);
    std::vector<uint8_t> seen(n, 0);
    struct Tree { int64_t size; int32_t root; int64_t off; };
    std::vector<Tree> trees;
    std::vector<int32_t> layouts;  // concatenated per-tree layouts
    std::vector<int32_t> bfs, stack, kids;
    for (int64_t v0 = 0; v0 < n; ++v0) {
        if (seen[v0] || aptr[v0 + 1] == aptr[v0]) continue;
        // v0 is the smallest id of its tree: every smaller vertex was visited.
        bfs.clear();
        bfs.push_back((int32_t)v0);
        seen[v0] = 1;
        parent[v0] = -1;
        for (size_t h = 0; h < bfs.size(); ++h) {
            int32_t v = bfs[h];
            for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a) {
                int32_t w = adj[a];
                if (!seen[w]) {
                    seen[w] = 1;
                    parent[w] = v;
                    bfs.push_back(w);
                }
            }
        }
        for (size_t h = bfs.size(); h-- > 0;) {
            int32_t v = bfs[h];
            size[v] = 1;
            for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a)
                if (adj[a] != parent[v]) size[v] += size[adj[a]];
        }
        Tree t{(int64_t)bfs.size(), (int32_t)v0, (int64_t)layouts.size()};
        // preorder, children in increasing (subtree size, id)
        stack.clear();
        stack.push_back((int32_t)v0);
        while (!stack.empty()) {
            int32_t v = stack.back();
            stack.pop_back();
            layouts.push_back(v);
            kids.clear();
            for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a)
                if (adj[a] != parent[v]) kids.push_back(adj[a]);
            std::sort(kids.begin(), kids.end(), [&](int32_t x, int32_t y) {
                return size[x] != size[y] ? size[x] < size[y] : x < y;
            });
            for (size_t j = kids.size(); j-- > 0;) stack.push_back(kids[j]);
        }
        trees.push_back(t);
    }
    std::stable_sort(trees.begin(), trees.end(),
                     [](const Tree &a, const Tree &b) { return a.size > b.size; });
    for (const Tree &t : trees)
        for (int64_t j = 0; j < t.size; ++j) {
            int32_t v = layouts[t.off + j];
            order.push_back(v);
            placed[v] = 1;
        }
}

// Greedy vertex cover of a small edge set: repeatedly the vertex with the
// most uncovered edges, ties to the smaller id.
std::vector<int32_t> greedy_cover(int64_t n, const std::vector<int32_t> &eu,
                                  const std::vector<int32_t> &ev) {
    std::vector<int32_t> cover;
    const size_t m = eu.size();
    if (m == 0) return cover;
    std::vector<int32_t> verts;
    verts.reserve(2 * m);
    for (size_t e = 0; e < m; ++e) {
        verts.push_back(eu[e]);
        verts.push_back(ev[e]);
    }
    std::sort(verts.begin(), verts.end());
    verts.erase(std::unique(verts.begin(), verts.end()), verts.end());
    auto idx = [&](int32_t v) {
        return (size_t)(std::lower_bound(verts.begin(), verts.end(), v) - verts.begin());
    };
    const size_t nv = verts.size();
    std::vector<std::vector<size_t>> inc(nv);
    std::vector<int64_t> deg(nv, 0);
    for (size_t e = 0; e < m; ++e) {
        inc[idx(eu[e])].push_back(e);
        inc[idx(ev[e])].push_back(e);
        ++deg[idx(eu[e])];
        ++deg[idx(ev[e])];
    }
    std::set<std::pair<int64_t, int32_t>> pq;  // (-deg, vertex)
    for (size_t i = 0; i < nv; ++i) pq.insert({-deg[i], verts[i]});
    std::vector<uint8_t> covered(m, 0);
    while (!pq.empty() && pq.begin()->first < 0) {
        int32_t v = pq.begin()->second;
        size_t iv = idx(v);
        pq.erase(pq.begin());
        cover.push_back(v);
        for (size_t e : inc[iv]) {
            if (covered[e]) continue;
            covered[e] = 1;
            int32_t w = eu[e] == v ? ev[e] : eu[e];
            size_t iw = idx(w);
            pq.erase({-deg[iw], w});
            --deg[iw];
            pq.insert({-deg[iw], w});
        }
        deg[iv] = 0;
    }
    (void)n;
    return cover;
}

}  // namespace

arrow_status_t decompose(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const float *val, const arrow_decompose_opts_t &opts, Decomp &out) {
    auto t0 = std::chrono::steady_clock::now();
    if (n < 0 || n >= (int64_t(1) << 31)) {
        set_error("n must be in [0, 2^31)");
        return ARROW_ERR_INVALID_ARG;
    }
    if (opts.b < 2) {
        set_error("arrow width b must be >= 2");
        return ARROW_ERR_INVALID_ARG;
    }
    if (opts.la != ARROW_LA_RANDOM_FOREST && opts.la != ARROW_LA_IDENTITY) {
        set_error("unknown linear arrangement kind");
        return ARROW_ERR_INVALID_ARG;
    }
    if (!row_ptr || (n > 0 && row_ptr[n] > 0 && (!col || !val))) {
        set_error("null CSR array");
        return ARROW_ERR_INVALID_ARG;
    }
    if (row_ptr[0] != 0) {
        set_error("row_ptr[0] must be 0");
        return ARROW_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) {
            set_error("row_ptr must be non-decreasing (row " + std::to_string(i) + ")");
            return ARROW_ERR_INVALID_ARG;
        }
    }
    const int64_t nnz = row_ptr[n];
    if (nnz >= (int64_t(1) << 31)) {
        set_error("nnz must be < 2^31");
        return ARROW_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n) {
                set_error("column index out of range in row " + std::to_string(i));
                return ARROW_ERR_INVALID_ARG;
            }
            if (p > row_ptr[i] && col[p] <= col[p - 1]) {
                set_error("columns must be strictly increasing within row " + std::to_string(i));
                return ARROW_ERR_INVALID_ARG;
            }
        }
    }
    const int64_t b = opts.b;
    out = Decomp();
    out.n = n;
    out.nnz = nnz;
    out.b = opts.b;
    out.la = opts.la;
    out.seed = opts.seed;

    Entries rem;
    rem.r.resize(nnz);
    rem.c.assign(col, col + nnz);
    rem.v.assign(val, val + nnz);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) rem.r[p] = (int32_t)i;

    const uint64_t un = (uint64_t)std::max<int64_t>(n, 1);
    const int key_bits = bits_for(un * un - 1);
    std::vector<uint8_t> is_head(n), has_entry(n), placed(n);
    std::vector<int32_t> pos(n);
    for (int32_t level = 0;; ++level) {
        if (opts.max_levels > 0 && level >= opts.max_levels) {
            set_error("decomposition needs more than max_levels = " +
                      std::to_string(opts.max_levels) + " levels");
            out = Decomp();
            return ARROW_ERR_UNSUPPORTED;
        }
        const size_t m = rem.size();
        // undirected edges of the remaining pattern, sorted by (u, v)
        std::vector<uint64_t> ekey;
        ekey.reserve(m);
        int64_t n_diag = 0;
        for (size_t e = 0; e < m; ++e) {
            int32_t r = rem.r[e], c = rem.c[e];
            if (r == c) {
                ++n_diag;
                continue;
            }
            uint64_t u = (uint64_t)std::min(r, c), v = (uint64_t)std::max(r, c);
            ekey.push_back(u * un + v);
        }
        radix_sort_keys(ekey, key_bits);
        ekey.erase(std::unique(ekey.begin(), ekey.end()), ekey.end());
        const size_t ne = ekey.size();
        std::vector<int32_t> eu(ne), ev(ne);
        for (size_t e = 0; e < ne; ++e) {
            eu[e] = (int32_t)(ekey[e] / un);
            ev[e] = (int32_t)(ekey[e] % un);
        }
        std::vector<uint64_t>().swap(ekey);
        std::fill(has_entry.begin(), has_entry.end(), 0);
        for (size_t e = 0; e < m; ++e) {
            has_entry[rem.r[e]] = 1;
            has_entry[rem.c[e]] = 1;
        }
        std::fill(is_head.begin(), is_head.end(), 0);
        std::fill(placed.begin(), placed.end(), 0);
        std::vector<int32_t> order;
        order.reserve(n);
        const bool final_level = 2 * (int64_t)ne + n_diag <= 2 * b;
        if (final_level) {
            for (int32_t v : greedy_cover(n, eu, ev)) {
                order.push_back(v);
                is_head[v] = placed[v] = 1;
            }
        } else {
            std::vector<int64_t> deg(n, 0);
            for (size_t e = 0; e < ne; ++e) {
                ++deg[eu[e]];
                ++deg[ev[e]];
            }
            std::vector<int32_t> cand;
            for (int64_t v = 0; v < n; ++v)
                if (deg[v] > 0) cand.push_back((int32_t)v);
            auto better = [&](int32_t x, int32_t y) {
                return deg[x] != deg[y] ? deg[x] > deg[y] : x < y;
            };
            if ((int64_t)cand.size() > b) {
                std::nth_element(cand.begin(), cand.begin() + b, cand.end(), better);
                cand.resize(b);
            }
            std::sort(cand.begin(), cand.end(), better);
            for (int32_t v : cand) {
                order.push_back(v);
                is_head[v] = placed[v] = 1;
            }
            if (opts.la == ARROW_LA_RANDOM_FOREST) {
                // weights of the edges of G_i - H_i, Kruskal in (key, u, v) order
                std::vector<uint64_t> wkey;
                std::vector<uint32_t> widx;
                const uint64_t ls = sm_output(opts.seed, (uint64_t)level);
                for (size_t e = 0; e < ne; ++e) {
                    if (is_head[eu[e]] || is_head[ev[e]]) continue;
                    wkey.push_back(sm_output(ls, (uint64_t)eu[e] * (uint64_t)n + (uint64_t)ev[e]));
                    widx.push_back((uint32_t)e);
                }
                radix_sort(wkey, widx, 64);  // stable: equal keys keep (u, v) order
                UnionFind uf(n);
                std::vector<int32_t> fu, fv;
                for (size_t j = 0; j < widx.size(); ++j) {
                    int32_t a = eu[widx[j]], c = ev[widx[j]];
                    int32_t ra = uf.find(a), rc = uf.find(c);
                    if (ra != rc) {
                        uf.parent[std::max(ra, rc)] = std::min(ra, rc);
                        fu.push_back(a);
                        fv.push_back(c);
                    }
                }
                layout_forest(n, fu, fv, order, placed);
            }
        }
        for (int64_t v = 0; v < n; ++v)
            if (!placed[v] && has_entry[v]) {
                order.push_back((int32_t)v);
                placed[v] = 1;
            }
        for (int64_t v = 0; v < n; ++v)
            if (!placed[v]) order.push_back((int32_t)v);
        if ((int64_t)order.size() != n) {
            set_error("internal: arrangement is not a permutation");
            return ARROW_ERR_INTERNAL;
        }
        for (int64_t p = 0; p < n; ++p) pos[order[p]] = (int32_t)p;

        // classify the remaining entries
        Level L;
        std::vector<int32_t> kp, kq;
        std::vector<float> kv;
        Entries next;
        int64_t maxpos = -1;
        for (size_t e = 0; e < m; ++e) {
            int64_t p = pos[rem.r[e]], q = pos[rem.c[e]];
            bool keep = p < b || q < b || (p > q ? p - q : q - p) <= b;
            if (keep) {
                kp.push_back((int32_t)p);
                kq.push_back((int32_t)q);
                kv.push_back(rem.v[e]);
                maxpos = std::max(maxpos, std::max(p, q));
            } else {
                next.r.push_back(rem.r[e]);
                next.c.push_back(rem.c[e]);
                next.v.push_back(rem.v[e]);
            }
        }
        if (final_level && !next.r.empty()) {
            set_error("internal: last level left entries");
            return ARROW_ERR_INTERNAL;
        }
        L.n_i = level == 0 ? n : maxpos + 1;
        L.vop.assign(order.begin(), order.begin() + L.n_i);
        L.row_ptr.assign(L.n_i + 1, 0);
        for (int32_t p : kp) ++L.row_ptr[p + 1];
        for (int64_t i = 0; i < L.n_i; ++i) L.row_ptr[i + 1] += L.row_ptr[i];
        const size_t nk = kp.size();
        L.col.resize(nk);
        L.val.resize(nk);
        {
            std::vector<int64_t> fill(L.row_ptr.begin(), L.row_ptr.end() - 1);
            for (size_t e = 0; e < nk; ++e) {
                int64_t d = fill[kp[e]]++;
                L.col[d] = kq[e];
                L.val[d] = kv[e];
            }
        }
        std::vector<std::pair<int32_t, float>> tmp;
        for (int64_t i = 0; i < L.n_i; ++i) {
            int64_t s = L.row_ptr[i], t = L.row_ptr[i + 1];
            bool sorted = true;
            for (int64_t j = s + 1; j < t; ++j)
                if (L.col[j] < L.col[j - 1]) { sorted = false; break; }
            if (sorted) continue;
            tmp.clear();
            for (int64_t j = s; j < t; ++j) tmp.push_back({L.col[j], L.val[j]});
            std::sort(tmp.begin(), tmp.end(),
                      [](const std::pair<int32_t, float> &a, const std::pair<int32_t, float> &b) {
                          return a.first < b.first;
                      });
            for (int64_t j = s; j < t; ++j) {
                L.col[j] = tmp[j - s].first;
                L.val[j] = tmp[j - s].second;
            }
        }
        out.levels.push_back(std::move(L));
        rem = std::move(next);
        if (rem.size() == 0) break;
    }
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return ARROW_OK;
}

}  // namespace arrow
