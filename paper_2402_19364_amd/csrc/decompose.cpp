// Host LA-Decompose (Section 5.1) with the random spanning forest linear
// arrangement (Section 5.3) and smallest-first tree order (Section 5.4), or
// the separator arrangement (Section 5.2, layout_separator).
//
// Per level i, on the undirected graph G_i of the symmetrised remaining
// pattern (self loops excluded):
//   1. head H_i: the b vertices of positive degree with the largest degree
//      (ties to the smaller id); they take positions 0 .. |H_i|-1,
//   2. every edge of G_i - H_i gets a 64-bit random weight (counter-based
//      SplitMix64 keyed by level and edge: a bijection of the edge id, so the
//      weights are distinct and the minimum spanning forest is unique);
//      Boruvka rounds build it in parallel,
//   3. each tree is rooted at its smallest id and laid out in smallest-first
//      preorder (children by subtree size, then id); trees follow the head in
//      decreasing size (ties: root id); then single vertices that still hold
//      entries, then the rest, both by id,
//   4. a stored entry (u, v) goes to B_i when its positions (p, q) satisfy
//      p < b or q < b or |p - q| <= b, otherwise to A_{i+1}.
// The loop runs while nnz(A_i) > 2b (Section 5.1), counted on the symmetrised
// pattern; the leftover (at most b edges) becomes a last level whose head is a
// greedy vertex cover (most uncovered edges first, ties by id).  Level 0 spans
// all n positions; later levels keep positions [0, 1 + largest used).
//
// Every step runs on `threads` host threads (opts.threads, 0 = all) and gives
// the same result for any thread count: parallel loops write disjoint ranges
// at offsets from prefix sums, integer counts use atomic adds (order
// independent), and whatever atomic scatter leaves unordered is sorted by a
// unique key afterwards.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <numeric>
#include <set>
#include <string>
#include <thread>

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

// Runs fn(lo, hi, t) for t = 0 .. nt-1 over [0, count) split into contiguous
// ranges of equal size (thread t takes the t-th range), on nt threads; small
// counts run the same ranges one after the other on the calling thread.
// Every t is called (possibly with an empty range), so per-thread results
// are always written.
template <class F>
void par_for(int nt, int64_t count, F &&fn) {
    if (nt <= 1 || count < 4096) {
        for (int t = 0; t < std::max(nt, 1); ++t)
            fn(count * t / std::max(nt, 1), count * (t + 1) / std::max(nt, 1), t);
        return;
    }
    std::vector<std::thread> ts;
    ts.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        const int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
        ts.emplace_back([&fn, lo, hi, t] { fn(lo, hi, t); });
    }
    for (auto &th : ts) th.join();
}

// Runs fn(t) for t = 0 .. nt-1, one thread each (tasks of uneven size).
template <class F>
void par_each(int nt, F &&fn) {
    if (nt <= 1) {
        fn(0);
        return;
    }
    std::vector<std::thread> ts;
    ts.reserve(nt);
    for (int t = 0; t < nt; ++t) ts.emplace_back([&fn, t] { fn(t); });
    for (auto &th : ts) th.join();
}

// Exclusive prefix sum of per-thread counts; returns the total.
int64_t exclusive_scan(std::vector<int64_t> &c) {
    int64_t s = 0;
    for (auto &v : c) {
        const int64_t x = v;
        v = s;
        s += x;
    }
    return s;
}

inline void atomic_min_u64(uint64_t *p, uint64_t v) {
    uint64_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED)) {
    }
}

struct Entries {  // remaining stored entries, in CSR order of A
    std::vector<int32_t> r, c;
    std::vector<float> v;
    size_t size() const { return r.size(); }
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

// Separator arrangement (Section 5.2) of the graph with edges (fu, fv):
// a vertex set is laid out as its connected components in increasing size
// (ties: smaller smallest id), each recursively; a connected set places a
// separator S first and then lays out the rest.  S is the first level of a
// BFS level structure rooted at a pseudo-peripheral vertex (the last vertex
// reached by a BFS from the set's smallest id) at which the BFS has reached
// at least half of the set.  BFS visits neighbours in increasing id.  Appends
// to `order`, marks `placed`.
void layout_separator(int64_t n, const std::vector<int32_t> &fu, const std::vector<int32_t> &fv,
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
    std::vector<uint8_t> alive(n, 0);
    std::vector<int32_t> top;
    for (int64_t v = 0; v < n; ++v)
        if (aptr[v + 1] > aptr[v]) {
            std::sort(adj.begin() + aptr[v], adj.begin() + aptr[v + 1]);
            alive[v] = 1;
            top.push_back((int32_t)v);
        }
    std::vector<int32_t> stamp(n, 0);  // visit marks: stamp[v] == cur
    int32_t cur = 0;
    // BFS inside the alive vertices from `start`; `out` gets the visit order,
    // `lev` the offsets of the levels in it
    std::vector<int32_t> bfs;
    std::vector<int64_t> lev;
    auto bfs_levels = [&](int32_t start) {
        ++cur;
        bfs.clear();
        lev.clear();
        bfs.push_back(start);
        stamp[start] = cur;
        lev.push_back(0);
        size_t h = 0;
        while (h < bfs.size()) {
            const size_t end = bfs.size();
            lev.push_back((int64_t)end);
            for (; h < end; ++h) {
                const int32_t v = bfs[h];
                for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a) {
                    const int32_t w = adj[a];
                    if (alive[w] && stamp[w] != cur) {
                        stamp[w] = cur;
                        bfs.push_back(w);
                    }
                }
            }
        }
        // lev[i] .. lev[i+1]: level i (the last entry equals bfs.size())
    };
    struct Item {
        bool place;
        std::vector<int32_t> vs;
    };
    std::vector<Item> stack;
    stack.push_back({false, std::move(top)});
    std::vector<std::vector<int32_t>> comps;
    while (!stack.empty()) {
        Item it = std::move(stack.back());
        stack.pop_back();
        if (it.place) {
            for (int32_t v : it.vs) {
                order.push_back(v);
                placed[v] = 1;
            }
            continue;
        }
        // connected components of the set, seeds in increasing id
        std::sort(it.vs.begin(), it.vs.end());
        ++cur;
        comps.clear();
        for (int32_t v0 : it.vs) {
            if (stamp[v0] == cur) continue;
            stamp[v0] = cur;
            std::vector<int32_t> comp(1, v0);
            for (size_t h = 0; h < comp.size(); ++h) {
                const int32_t v = comp[h];
                for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a) {
                    const int32_t w = adj[a];
                    if (alive[w] && stamp[w] != cur) {
                        stamp[w] = cur;
                        comp.push_back(w);
                    }
                }
            }
            comps.push_back(std::move(comp));
        }
        if (comps.size() > 1) {
            // comp[0] is each component's smallest id
            std::stable_sort(comps.begin(), comps.end(),
                             [](const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
                                 return a.size() != b.size() ? a.size() < b.size() : a[0] < b[0];
                             });
            for (size_t j = comps.size(); j-- > 0;) stack.push_back({false, std::move(comps[j])});
            continue;
        }
        std::vector<int32_t> comp = std::move(comps[0]);
        if (comp.size() == 1) {
            order.push_back(comp[0]);
            placed[comp[0]] = 1;
            alive[comp[0]] = 0;
            continue;
        }
        bfs_levels(comp[0]);
        bfs_levels(bfs.back());
        size_t li = 0;
        while (2 * (size_t)lev[li + 1] < comp.size()) ++li;
        std::vector<int32_t> sep(bfs.begin() + lev[li], bfs.begin() + lev[li + 1]);
        for (int32_t v : sep) alive[v] = 0;
        std::vector<int32_t> rest;
        for (int32_t v : comp)
            if (alive[v]) rest.push_back(v);
        if (!rest.empty()) stack.push_back({false, std::move(rest)});
        stack.push_back({true, std::move(sep)});
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


// Undirected edges {u, v} (u < v) of the pattern of the remaining entries
// (sorted by (row, column)), sorted by (u, v) without duplicates; self loops
// are counted in n_diag.  Entries with r < c already come in (u, v) order;
// the others, keyed (c, r), are bucketed by ranges of c (per-thread counts,
// stable scatter) and each bucket is sorted; the two sorted key lists are
// then merged per range of u.
// Undirected edges of a symmetric remaining pattern: the entries above the
// diagonal, already sorted by (u, v) in CSR order (no duplicates: columns are
// strictly increasing within a row).
void upper_edges(int nt, const std::vector<int32_t> &R, const std::vector<int32_t> &C,
                 std::vector<int32_t> &eu, std::vector<int32_t> &ev, int64_t &n_diag) {
    const int64_t m = (int64_t)R.size();
    std::vector<int64_t> c1(nt, 0), cd(nt, 0);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t a = 0, d = 0;
        for (int64_t e = lo; e < hi; ++e) {
            a += R[e] < C[e];
            d += R[e] == C[e];
        }
        c1[t] = a, cd[t] = d;
    });
    n_diag = 0;
    for (int t = 0; t < nt; ++t) n_diag += cd[t];
    const int64_t ne = exclusive_scan(c1);
    eu.resize(ne);
    ev.resize(ne);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t o = c1[t];
        for (int64_t e = lo; e < hi; ++e)
            if (R[e] < C[e]) {
                eu[o] = R[e];
                ev[o] = C[e];
                ++o;
            }
    });
}

// Undirected edges {u, v} (u < v) of the remaining pattern, sorted and
// without duplicates, and the number of diagonal entries; `symmetric` (if
// not null) tells whether the pattern equals its transpose.
void undirected_edges(int nt, int64_t n, const std::vector<int32_t> &R,
                      const std::vector<int32_t> &C, std::vector<int32_t> &eu,
                      std::vector<int32_t> &ev, int64_t &n_diag, bool *symmetric = nullptr) {
    const int64_t m = (int64_t)R.size();
    const uint64_t un = (uint64_t)std::max<int64_t>(n, 1);
    const int P = 64 * nt;  // buckets of list 2 by ranges of c
    auto bucket_of = [&](int64_t c) { return (int)(c * P / std::max<int64_t>(n, 1)); };
    std::vector<int64_t> c1(nt, 0), cd(nt, 0), h2((size_t)nt * P, 0);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t a = 0, d = 0;
        int64_t *h = &h2[(size_t)t * P];
        for (int64_t e = lo; e < hi; ++e) {
            if (R[e] < C[e])
                ++a;
            else if (R[e] > C[e])
                ++h[bucket_of(C[e])];
            else
                ++d;
        }
        c1[t] = a, cd[t] = d;
    });
    n_diag = 0;
    for (int t = 0; t < nt; ++t) n_diag += cd[t];
    const int64_t m1 = exclusive_scan(c1);
    // bucket-major, thread-minor offsets: a stable scatter
    std::vector<int64_t> boff((size_t)nt * P), bstart(P + 1, 0);
    {
        int64_t s2 = 0;
        for (int q = 0; q < P; ++q) {
            bstart[q] = s2;
            for (int t = 0; t < nt; ++t) {
                boff[(size_t)t * P + q] = s2;
                s2 += h2[(size_t)t * P + q];
            }
        }
        bstart[P] = s2;
    }
    const int64_t m2 = bstart[P];
    std::vector<uint64_t> k1(m1), k2(m2);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t o = c1[t];
        int64_t *bo = &boff[(size_t)t * P];
        for (int64_t e = lo; e < hi; ++e) {
            if (R[e] < C[e])
                k1[o++] = (uint64_t)R[e] * un + (uint64_t)C[e];
            else if (R[e] > C[e])
                k2[bo[bucket_of(C[e])]++] = (uint64_t)C[e] * un + (uint64_t)R[e];
        }
    });
    par_for(nt, P, [&](int64_t lo, int64_t hi, int) {
        for (int64_t q = lo; q < hi; ++q) std::sort(k2.begin() + bstart[q], k2.begin() + bstart[q + 1]);
    });
    if (symmetric) {
        // the entries below the diagonal, transposed and sorted, equal the
        // ones above it exactly when the pattern is symmetric
        std::vector<uint8_t> same(nt, 1);
        if (m1 == m2)
            par_for(nt, m1, [&](int64_t lo, int64_t hi, int t) {
                for (int64_t i = lo; i < hi && same[t]; ++i) same[t] = k1[i] == k2[i];
            });
        *symmetric = m1 == m2;
        for (int t = 0; t < nt; ++t) *symmetric = *symmetric && same[t];
    }
    // merge the two sorted lists per range of u, dropping duplicates
    std::vector<int64_t> s1(nt + 1), s2(nt + 1), cnt(nt, 0);
    for (int t = 0; t <= nt; ++t) {
        const uint64_t key0 = (uint64_t)(n * t / nt) * un;
        s1[t] = std::lower_bound(k1.begin(), k1.end(), key0) - k1.begin();
        s2[t] = std::lower_bound(k2.begin(), k2.end(), key0) - k2.begin();
    }
    s1[nt] = m1;
    s2[nt] = m2;
    auto merge = [&](int t, bool write, int64_t o) {
        int64_t i = s1[t], j = s2[t], k = 0;
        uint64_t last = UINT64_MAX;
        while (i < s1[t + 1] || j < s2[t + 1]) {
            uint64_t x;
            if (j >= s2[t + 1] || (i < s1[t + 1] && k1[i] <= k2[j]))
                x = k1[i++];
            else
                x = k2[j++];
            if (x == last) continue;
            last = x;
            if (write) {
                eu[o + k] = (int32_t)(x / un);
                ev[o + k] = (int32_t)(x % un);
            }
            ++k;
        }
        return k;
    };
    par_each(nt, [&](int t) { cnt[t] = merge(t, false, 0); });
    const int64_t ne = exclusive_scan(cnt);
    eu.resize(ne);
    ev.resize(ne);
    par_each(nt, [&](int t) { merge(t, true, cnt[t]); });
}

// Minimum spanning forest of the edges listed in `live` under the distinct
// weights key[e], by Boruvka rounds: every component picks its lightest
// outgoing edge (atomic minimum of the weight), the picked edges join the
// forest and merge the components.  The forest is unique, so the result does
// not depend on the thread count.  Returns the forest's edges in edge order.
void boruvka_msf(int nt, int64_t n, const std::vector<int32_t> &eu,
                 const std::vector<int32_t> &ev, const std::vector<uint64_t> &key,
                 std::vector<int64_t> live, std::vector<int32_t> &fu,
                 std::vector<int32_t> &fv) {
    // per live edge: its index and the component labels of its endpoints
    // (labels are vertex ids of the component roots)
    int64_t m = (int64_t)live.size();
    std::vector<int32_t> cu(m), cv(m);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i) {
            cu[i] = eu[live[i]];
            cv[i] = ev[live[i]];
        }
    });
    std::vector<int32_t> parent(n);
    std::vector<uint64_t> best(n, UINT64_MAX);
    std::vector<int64_t> bedge(n, -1);
    std::vector<uint8_t> in_forest(eu.size(), 0);
    std::vector<int32_t> roots;  // labels touched this round
    std::vector<int64_t> cnt(nt);
    // compaction buffers, swapped with the live arrays every round (the live
    // count only shrinks, so they never grow)
    std::vector<int64_t> nlive(m);
    std::vector<int32_t> ncu(m), ncv(m);
    par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t v = lo; v < hi; ++v) parent[v] = (int32_t)v;
    });
    while (m > 0) {
        par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i) {
                const uint64_t k = key[live[i]];
                atomic_min_u64(&best[cu[i]], k);
                atomic_min_u64(&best[cv[i]], k);
            }
        });
        // the edge of each component's minimum (one writer: weights are distinct)
        par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i) {
                const uint64_t k = key[live[i]];
                if (best[cu[i]] == k) bedge[cu[i]] = i;
                if (best[cv[i]] == k) bedge[cv[i]] = i;
            }
        });
        // link: a component points at the other end of its edge
        par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i) {
                if (bedge[cu[i]] == i) {
                    parent[cu[i]] = cv[i];
                    __atomic_store_n(&in_forest[live[i]], (uint8_t)1, __ATOMIC_RELAXED);
                }
                if (bedge[cv[i]] == i) {
                    parent[cv[i]] = cu[i];
                    __atomic_store_n(&in_forest[live[i]], (uint8_t)1, __ATOMIC_RELAXED);
                }
            }
        });
        // the labels linked this round, in increasing order
        roots.clear();
        {
            std::vector<std::vector<int32_t>> part(nt);
            par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
                for (int64_t i = lo; i < hi; ++i) {
                    if (bedge[cu[i]] == i) part[t].push_back(cu[i]);
                    if (bedge[cv[i]] == i) part[t].push_back(cv[i]);
                }
            });
            for (auto &q : part) roots.insert(roots.end(), q.begin(), q.end());
            std::sort(roots.begin(), roots.end());
            roots.erase(std::unique(roots.begin(), roots.end()), roots.end());
        }
        const int64_t nr = (int64_t)roots.size();
        // two components that picked the same edge point at each other: the
        // smaller becomes the root
        par_for(nt, nr, [&](int64_t lo, int64_t hi, int) {
            for (int64_t j = lo; j < hi; ++j) {
                const int32_t v = roots[j], p = parent[v];
                if (parent[p] == v && v < p) parent[v] = v;
            }
        });
        // pointer jumping to the roots (only labels linked this round move)
        for (bool changed = true; changed;) {
            std::atomic<bool> ch{false};
            par_for(nt, nr, [&](int64_t lo, int64_t hi, int) {
                bool c = false;
                for (int64_t j = lo; j < hi; ++j) {
                    const int32_t v = roots[j], p = parent[v], g = parent[p];
                    if (g != p) {
                        parent[v] = g;
                        c = true;
                    }
                }
                if (c) ch = true;
            });
            changed = ch;
        }
        par_for(nt, nr, [&](int64_t lo, int64_t hi, int) {
            for (int64_t j = lo; j < hi; ++j) {
                best[roots[j]] = UINT64_MAX;
                bedge[roots[j]] = -1;
            }
        });
        // relabel the edges, keep those between different components (in order)
        par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
            int64_t c = 0;
            for (int64_t i = lo; i < hi; ++i) {
                cu[i] = parent[cu[i]];
                cv[i] = parent[cv[i]];
                c += cu[i] != cv[i];
            }
            cnt[t] = c;
        });
        std::vector<int64_t> off(cnt);
        const int64_t m2 = exclusive_scan(off);
        par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
            int64_t o = off[t];
            for (int64_t i = lo; i < hi; ++i)
                if (cu[i] != cv[i]) {
                    nlive[o] = live[i];
                    ncu[o] = cu[i];
                    ncv[o] = cv[i];
                    ++o;
                }
        });
        live.swap(nlive);
        cu.swap(ncu);
        cv.swap(ncv);
        m = m2;
    }
    fu.clear();
    fv.clear();
    for (size_t e = 0; e < eu.size(); ++e)
        if (in_forest[e]) {
            fu.push_back(eu[e]);
            fv.push_back(ev[e]);
        }
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
    if (opts.threads < 0) {
        set_error("threads must be >= 0 (0 = every hardware thread)");
        return ARROW_ERR_INVALID_ARG;
    }
    if (opts.la != ARROW_LA_RANDOM_FOREST && opts.la != ARROW_LA_IDENTITY &&
        opts.la != ARROW_LA_SEPARATOR) {
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
    const int nt = opts.threads > 0
                       ? opts.threads
                       : (int)std::max(1u, std::min(256u, std::thread::hardware_concurrency()));
    {
        // the first bad row (the same message for every thread count)
        std::vector<int64_t> bad_col(nt, INT64_MAX), bad_ord(nt, INT64_MAX);
        par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
            for (int64_t i = lo; i < hi; ++i)
                for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                    if (col[p] < 0 || col[p] >= n) {
                        if (bad_col[t] == INT64_MAX) bad_col[t] = i;
                    } else if (p > row_ptr[i] && col[p] <= col[p - 1]) {
                        if (bad_ord[t] == INT64_MAX) bad_ord[t] = i;
                    }
                }
        });
        const int64_t bc = *std::min_element(bad_col.begin(), bad_col.end());
        const int64_t bo = *std::min_element(bad_ord.begin(), bad_ord.end());
        if (bc != INT64_MAX && bc <= bo) {
            set_error("column index out of range in row " + std::to_string(bc));
            return ARROW_ERR_INVALID_ARG;
        }
        if (bo != INT64_MAX) {
            set_error("columns must be strictly increasing within row " + std::to_string(bo));
            return ARROW_ERR_INVALID_ARG;
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
    par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) rem.r[p] = (int32_t)i;
    });

    std::vector<uint8_t> is_head(n), has_entry(n), placed(n);
    std::vector<int32_t> pos(n);
    std::vector<int64_t> tcnt(nt), tcnt2(nt), tmax(nt);
    bool pattern_symmetric = false;
    for (int32_t level = 0;; ++level) {
        if (opts.max_levels > 0 && level >= opts.max_levels) {
            set_error("decomposition needs more than max_levels = " +
                      std::to_string(opts.max_levels) + " levels");
            out = Decomp();
            return ARROW_ERR_UNSUPPORTED;
        }
        const int64_t m = (int64_t)rem.size();
        // undirected edges of the remaining pattern, sorted by (u, v)
        std::vector<int32_t> eu, ev;
        int64_t n_diag = 0;
        // a symmetric pattern stays symmetric at every level ((u, v) and
        // (v, u) always land in the same level): its edges are then the
        // entries above the diagonal, in order
        if (level > 0 && pattern_symmetric)
            upper_edges(nt, rem.r, rem.c, eu, ev, n_diag);
        else
            undirected_edges(nt, n, rem.r, rem.c, eu, ev, n_diag,
                             level == 0 ? &pattern_symmetric : nullptr);
        const int64_t ne = (int64_t)eu.size();
        std::fill(has_entry.begin(), has_entry.end(), 0);
        par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
            for (int64_t e = lo; e < hi; ++e) {
                __atomic_store_n(&has_entry[rem.r[e]], (uint8_t)1, __ATOMIC_RELAXED);
                __atomic_store_n(&has_entry[rem.c[e]], (uint8_t)1, __ATOMIC_RELAXED);
            }
        });
        std::fill(is_head.begin(), is_head.end(), 0);
        std::fill(placed.begin(), placed.end(), 0);
        std::vector<int32_t> order;
        order.reserve(n);
        const bool final_level = 2 * ne + n_diag <= 2 * b;
        if (final_level) {
            for (int32_t v : greedy_cover(n, eu, ev)) {
                order.push_back(v);
                is_head[v] = placed[v] = 1;
            }
        } else {
            std::vector<int64_t> deg(n, 0);
            par_for(nt, ne, [&](int64_t lo, int64_t hi, int) {
                for (int64_t e = lo; e < hi; ++e) {
                    __atomic_fetch_add(&deg[eu[e]], (int64_t)1, __ATOMIC_RELAXED);
                    __atomic_fetch_add(&deg[ev[e]], (int64_t)1, __ATOMIC_RELAXED);
                }
            });
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
                // weights of the edges of G_i - H_i (a bijection of the edge id,
                // so all distinct), then the unique minimum spanning forest
                const uint64_t ls = sm_output(opts.seed, (uint64_t)level);
                std::vector<uint64_t> key(ne);
                par_for(nt, ne, [&](int64_t lo, int64_t hi, int t) {
                    int64_t c = 0;
                    for (int64_t e = lo; e < hi; ++e) {
                        key[e] = sm_output(ls, (uint64_t)eu[e] * (uint64_t)n + (uint64_t)ev[e]);
                        c += !is_head[eu[e]] && !is_head[ev[e]];
                    }
                    tcnt[t] = c;
                });
                std::vector<int64_t> off(tcnt.begin(), tcnt.end());
                const int64_t nl = exclusive_scan(off);
                std::vector<int64_t> live(nl);
                par_for(nt, ne, [&](int64_t lo, int64_t hi, int t) {
                    int64_t o = off[t];
                    for (int64_t e = lo; e < hi; ++e)
                        if (!is_head[eu[e]] && !is_head[ev[e]]) live[o++] = e;
                });
                std::vector<int32_t> fu, fv;
                boruvka_msf(nt, n, eu, ev, key, std::move(live), fu, fv);
                layout_forest(n, fu, fv, order, placed);
            } else if (opts.la == ARROW_LA_SEPARATOR) {
                // the edges of G_i - H_i
                std::vector<int32_t> gu, gv;
                for (int64_t e = 0; e < ne; ++e)
                    if (!is_head[eu[e]] && !is_head[ev[e]]) {
                        gu.push_back(eu[e]);
                        gv.push_back(ev[e]);
                    }
                layout_separator(n, gu, gv, order, placed);
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
        par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
            for (int64_t p = lo; p < hi; ++p) pos[order[p]] = (int32_t)p;
        });

        auto keep_of = [&](int64_t e, int64_t &p, int64_t &q) {
            p = pos[rem.r[e]];
            q = pos[rem.c[e]];
            return p < b || q < b || (p > q ? p - q : q - p) <= b;
        };
        par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
            int64_t c = 0, mx = -1;
            for (int64_t e = lo; e < hi; ++e) {
                int64_t p, q;
                if (keep_of(e, p, q)) {
                    ++c;
                    mx = std::max(mx, std::max(p, q));
                }
            }
            tcnt[t] = c;
            tmax[t] = mx;
        });
        for (int t = 0; t < nt; ++t) tcnt2[t] = 0;
        int64_t maxpos = -1;
        for (int t = 0; t < nt; ++t) maxpos = std::max(maxpos, tmax[t]);
        std::vector<int64_t> koff(tcnt.begin(), tcnt.end());
        const int64_t nk = exclusive_scan(koff);
        Entries next;
        next.r.resize(m - nk);
        next.c.resize(m - nk);
        next.v.resize(m - nk);
        std::vector<int32_t> kp(nk), kq(nk);
        std::vector<float> kv(nk);
        par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
            int64_t o = koff[t], o2 = lo - koff[t];
            for (int64_t e = lo; e < hi; ++e) {
                int64_t p, q;
                if (keep_of(e, p, q)) {
                    kp[o] = (int32_t)p;
                    kq[o] = (int32_t)q;
                    kv[o] = rem.v[e];
                    ++o;
                } else {
                    next.r[o2] = rem.r[e];
                    next.c[o2] = rem.c[e];
                    next.v[o2] = rem.v[e];
                    ++o2;
                }
            }
        });
        if (final_level && !next.r.empty()) {
            set_error("internal: last level left entries");
            return ARROW_ERR_INTERNAL;
        }
        Level L;
        L.n_i = level == 0 ? n : maxpos + 1;
        L.vop.assign(order.begin(), order.begin() + L.n_i);
        L.row_ptr.assign(L.n_i + 1, 0);
        par_for(nt, nk, [&](int64_t lo, int64_t hi, int) {
            for (int64_t e = lo; e < hi; ++e)
                __atomic_fetch_add(&L.row_ptr[kp[e] + 1], (int64_t)1, __ATOMIC_RELAXED);
        });
        for (int64_t i = 0; i < L.n_i; ++i) L.row_ptr[i + 1] += L.row_ptr[i];
        L.col.resize(nk);
        L.val.resize(nk);
        {
            // scatter by row (any order within a row), then sort each row by
            // column: positions within a row are distinct, so the order is unique
            std::vector<int64_t> fill(L.row_ptr.begin(), L.row_ptr.end() - 1);
            par_for(nt, nk, [&](int64_t lo, int64_t hi, int) {
                for (int64_t e = lo; e < hi; ++e) {
                    const int64_t d = __atomic_fetch_add(&fill[kp[e]], (int64_t)1, __ATOMIC_RELAXED);
                    L.col[d] = kq[e];
                    L.val[d] = kv[e];
                }
            });
        }
        // rows split into ranges of equal entry counts (head rows are long)
        std::vector<int64_t> rcut(nt + 1, 0);
        for (int t = 1; t < nt; ++t)
            rcut[t] = std::max<int64_t>(
                rcut[t - 1], std::lower_bound(L.row_ptr.begin(), L.row_ptr.end() - 1,
                                              nk * t / nt) - L.row_ptr.begin());
        rcut[nt] = L.n_i;
        par_each(nt, [&](int tt) {
          {
            const int64_t lo = rcut[tt], hi = rcut[tt + 1];
            std::vector<std::pair<int32_t, float>> tmp;
            for (int64_t i = lo; i < hi; ++i) {
                const int64_t s = L.row_ptr[i], t = L.row_ptr[i + 1];
                bool sorted = true;
                for (int64_t j = s + 1; j < t; ++j)
                    if (L.col[j] < L.col[j - 1]) {
                        sorted = false;
                        break;
                    }
                if (sorted) continue;
                tmp.clear();
                for (int64_t j = s; j < t; ++j) tmp.push_back({L.col[j], L.val[j]});
                std::sort(tmp.begin(), tmp.end(),
                          [](const std::pair<int32_t, float> &a,
                             const std::pair<int32_t, float> &c) { return a.first < c.first; });
                for (int64_t j = s; j < t; ++j) {
                    L.col[j] = tmp[j - s].first;
                    L.val[j] = tmp[j - s].second;
                }
            }
          }
        });
        out.levels.push_back(std::move(L));
        rem = std::move(next);
        if (rem.size() == 0) break;
    }
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return ARROW_OK;
}

}  // namespace arrow
