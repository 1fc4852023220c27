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
// unique key afterwards or does not affect the result (the forest is unique,
// and its layout does not depend on the order of its edges).
//
// A symmetric pattern stays symmetric at every level (an entry and its
// transpose always land in the same level).  Once level 0 has found A's
// pattern symmetric, each level reads its graph from the rows of the
// remaining entries (degrees, the first Boruvka round, the edges above the
// diagonal) instead of a sorted, merged edge list.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <thread>

#include <sys/mman.h>

#include "host_threads.h"
#include "internal.h"

namespace arrow {
namespace {

// Working arrays of a decomposition.  Every level allocates and releases
// large arrays whose sizes only shrink from level to level, and the pages of
// fresh memory from the OS are faulted in and zeroed on first touch, a cost
// comparable to the work on them.  Blocks of kBigBlock bytes or more are
// therefore kept when released (up to kCachedBlocks of them) and handed out
// again (the smallest one that holds the request, if it is at most twice its
// size) while a decomposition runs; when the last running decomposition ends
// they go back to the OS.
constexpr size_t kBigBlock = size_t(1) << 20;
constexpr size_t kBlockHeader = 64;  // block size, keeps the data 64-byte aligned
constexpr size_t kCachedBlocks = 8;  // released blocks kept (R-MAT 2^22 peaks at 2.5 GB, not 3.9)

struct BlockCache {
    std::mutex mu;
    std::multimap<size_t, char *> free_blocks;  // by size
    int users = 0;
};
BlockCache &block_cache() {
    static BlockCache c;
    return c;
}

size_t block_len(size_t bytes) { return (kBlockHeader + bytes + 4095) & ~size_t(4095); }
void block_free(char *b) { munmap(b, block_len(*reinterpret_cast<size_t *>(b))); }

void *cache_get(size_t bytes) {
    if (bytes < kBigBlock) return ::operator new(bytes);
    BlockCache &c = block_cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.free_blocks.lower_bound(bytes);
        if (it != c.free_blocks.end() && it->first <= 2 * bytes) {
            char *b = it->second;
            c.free_blocks.erase(it);
            return b + kBlockHeader;
        }
    }
    // fresh blocks come straight from the OS, with transparent huge pages
    // asked for (fewer page faults on first touch, fewer TLB misses in the
    // random accesses of the steps), at a 2 MiB boundary
    const size_t len = block_len(bytes), huge = size_t(2) << 20;
    char *raw = static_cast<char *>(
        mmap(nullptr, len + huge, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0));
    if (raw == MAP_FAILED) throw std::bad_alloc();
    const size_t head = (huge - reinterpret_cast<uintptr_t>(raw) % huge) % huge;
    if (head) munmap(raw, head);
    if (huge - head) munmap(raw + head + len, huge - head);
    char *b = raw + head;
    madvise(b, len, MADV_HUGEPAGE);
    *reinterpret_cast<size_t *>(b) = bytes;
    return b + kBlockHeader;
}

void cache_put(void *p, size_t bytes) {
    if (!p) return;
    if (bytes < kBigBlock) {
        ::operator delete(p);
        return;
    }
    char *b = static_cast<char *>(p) - kBlockHeader;
    BlockCache &c = block_cache();
    std::lock_guard<std::mutex> g(c.mu);
    if (c.users > 0) {
        c.free_blocks.emplace(*reinterpret_cast<size_t *>(b), b);
        // at most kCachedBlocks wait for reuse; the largest go back first
        while (c.free_blocks.size() > kCachedBlocks) {
            auto last = std::prev(c.free_blocks.end());
            block_free(last->second);
            c.free_blocks.erase(last);
        }
    } else {
        block_free(b);
    }
}

// Marks a running decomposition; the last one to end empties the cache.
struct CacheUser {
    CacheUser() {
        std::lock_guard<std::mutex> g(block_cache().mu);
        ++block_cache().users;
    }
    ~CacheUser() {
        BlockCache &c = block_cache();
        std::lock_guard<std::mutex> g(c.mu);
        if (--c.users == 0) {
            for (auto &kv : c.free_blocks) block_free(kv.second);
            c.free_blocks.clear();
        }
    }
};

template <class T>
struct CacheAlloc {
    using value_type = T;
    CacheAlloc() = default;
    template <class U>
    CacheAlloc(const CacheAlloc<U> &) {}
    T *allocate(size_t n) { return static_cast<T *>(cache_get(n * sizeof(T))); }
    void deallocate(T *p, size_t n) { cache_put(p, n * sizeof(T)); }
    template <class U>
    bool operator==(const CacheAlloc<U> &) const { return true; }
    template <class U>
    bool operator!=(const CacheAlloc<U> &) const { return false; }
};
template <class T>
using Vec = std::vector<T, CacheAlloc<T>>;

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

inline void atomic_min_u64(uint64_t *p, uint64_t v) {
    uint64_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED)) {
    }
}

struct Entries {  // remaining stored entries, in CSR order of A
    Vec<int32_t> r, c;
    Vec<float> v;
    size_t size() const { return r.size(); }
};

// Smallest-first layouts of the trees of a forest over n vertices, trees in
// decreasing size (ties: smaller root).  Appends to `order`, marks `placed`.
// A tree is rooted at its smallest id by a BFS, which fills slots h = 0, 1,
// ... with the vertices in visit order and records each slot's parent slot
// up[h]; a vertex's children are pushed together, so they take consecutive
// slots and up is nondecreasing within a tree.  Subtree sizes follow in
// reverse slot order.  In the preorder with children by increasing (subtree
// size, id), a child sits 1 + (sizes of its earlier siblings) after its
// parent: those offsets are computed per parent in parallel, and the
// positions in one pass in slot order (a parent before its children).
void layout_forest(int nt, int64_t n, const Vec<int32_t> &fu, const Vec<int32_t> &fv,
                   Vec<int32_t> &order, Vec<uint8_t> &placed) {
    const int64_t m = (int64_t)fu.size();
    if (m == 0) return;
    // adjacency of the forest (any order within a vertex)
    Vec<int64_t> aptr(n + 1, 0);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
        for (int64_t e = lo; e < hi; ++e) {
            __atomic_fetch_add(&aptr[fu[e] + 1], (int64_t)1, __ATOMIC_RELAXED);
            __atomic_fetch_add(&aptr[fv[e] + 1], (int64_t)1, __ATOMIC_RELAXED);
        }
    });
    for (int64_t i = 0; i < n; ++i) aptr[i + 1] += aptr[i];
    Vec<int32_t> adj(2 * m);
    {
        Vec<int64_t> fill(aptr.begin(), aptr.end() - 1);
        par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
            for (int64_t e = lo; e < hi; ++e) {
                adj[__atomic_fetch_add(&fill[fu[e]], (int64_t)1, __ATOMIC_RELAXED)] = fv[e];
                adj[__atomic_fetch_add(&fill[fv[e]], (int64_t)1, __ATOMIC_RELAXED)] = fu[e];
            }
        });
    }
    // BFS of every tree from its smallest id (trees found in increasing root)
    struct Tree { int64_t size; int64_t slot; };
    Vec<Tree> trees;
    Vec<int32_t> bfs, up;
    bfs.reserve(m + (m >> 2) + 16);
    up.reserve(m + (m >> 2) + 16);
    {
        Vec<uint8_t> seen(n, 0);
        for (int64_t v0 = 0; v0 < n; ++v0) {
            if (seen[v0] || aptr[v0 + 1] == aptr[v0]) continue;
            const int64_t start = (int64_t)bfs.size();
            bfs.push_back((int32_t)v0);
            up.push_back(-1);
            seen[v0] = 1;
            for (int64_t h = start; h < (int64_t)bfs.size(); ++h) {
                const int32_t v = bfs[h];
                for (int64_t a = aptr[v]; a < aptr[v + 1]; ++a) {
                    const int32_t w = adj[a];
                    if (!seen[w]) {
                        seen[w] = 1;
                        bfs.push_back(w);
                        up.push_back((int32_t)h);
                    }
                }
            }
            trees.push_back({(int64_t)bfs.size() - start, start});
        }
    }
    const int64_t N = (int64_t)bfs.size();
    Vec<int32_t> size(N, 0), rel(N, 0), cbeg(N, 0), cend(N, 0);
    for (int64_t h = N; h-- > 0;) {
        size[h] += 1;
        if (up[h] >= 0) size[up[h]] += size[h];
    }
    // the children of slot j are the slots [cbeg[j], cend[j])
    par_for(nt, N, [&](int64_t lo, int64_t hi, int) {
        for (int64_t h = lo; h < hi; ++h) {
            const int32_t j = up[h];
            if (j < 0) continue;
            if (h == 0 || up[h - 1] != j) cbeg[j] = (int32_t)h;
            if (h == N - 1 || up[h + 1] != j) cend[j] = (int32_t)h + 1;
        }
    });
    // offsets of the children behind their parent
    par_for(nt, N, [&](int64_t lo, int64_t hi, int) {
        Vec<int32_t> kids;
        for (int64_t j = lo; j < hi; ++j) {
            if (cend[j] == cbeg[j]) continue;
            kids.clear();
            for (int32_t h = cbeg[j]; h < cend[j]; ++h) kids.push_back(h);
            std::sort(kids.begin(), kids.end(), [&](int32_t x, int32_t y) {
                return size[x] != size[y] ? size[x] < size[y] : bfs[x] < bfs[y];
            });
            int32_t o = 1;
            for (int32_t h : kids) {
                rel[h] = o;
                o += size[h];
            }
        }
    });
    // positions: roots at their tree's offset, then parents before children
    std::stable_sort(trees.begin(), trees.end(),
                     [](const Tree &x, const Tree &y) { return x.size > y.size; });
    {
        int64_t off = 0;
        for (const Tree &t : trees) {
            rel[t.slot] = (int32_t)off;
            off += t.size;
        }
    }
    Vec<int32_t> &pos = size;  // sizes are no longer needed
    for (int64_t h = 0; h < N; ++h) pos[h] = up[h] >= 0 ? pos[up[h]] + rel[h] : rel[h];
    const size_t base = order.size();
    order.resize(base + N);
    par_for(nt, N, [&](int64_t lo, int64_t hi, int) {
        for (int64_t h = lo; h < hi; ++h) {
            order[base + pos[h]] = bfs[h];
            placed[bfs[h]] = 1;
        }
    });
}

// Sorts distinct vertex ids in [0, n) increasingly: least-significant-digit
// radix sort with 11-bit digits for long lists, std::sort for short ones.
void sort_ids(Vec<int32_t> &v, int64_t n, Vec<int32_t> &tmp) {
    if (v.size() < 1024) {
        std::sort(v.begin(), v.end());
        return;
    }
    constexpr int kBits = 11, kR = 1 << kBits;
    tmp.resize(v.size());
    int64_t cnt[kR];
    for (int shift = 0; shift == 0 || (n - 1) >> shift; shift += kBits) {
        std::fill(cnt, cnt + kR, 0);
        for (int32_t x : v) ++cnt[(x >> shift) & (kR - 1)];
        int64_t s = 0;
        for (int d = 0; d < kR; ++d) {
            const int64_t c = cnt[d];
            cnt[d] = s;
            s += c;
        }
        for (int32_t x : v) tmp[cnt[(x >> shift) & (kR - 1)]++] = x;
        v.swap(tmp);
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
//
// The components of a set are disjoint and not adjacent through live
// vertices, so large ones are laid out on threads of their own (at most nt
// at a time), each into its own list; the lists are joined in component
// order, so the result does not depend on the thread count.  Visit marks
// take globally increasing stamps.
void layout_separator(int nt, int64_t n, const Vec<int32_t> &fu, const Vec<int32_t> &fv,
                      Vec<int32_t> &order, Vec<uint8_t> &placed) {
    const int64_t m = (int64_t)fu.size();
    if (m == 0) return;
    Vec<int64_t> aptr(n + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
        ++aptr[fu[e] + 1];
        ++aptr[fv[e] + 1];
    }
    for (int64_t i = 0; i < n; ++i) aptr[i + 1] += aptr[i];
    Vec<int32_t> adj(2 * m);
    {
        Vec<int64_t> fill(aptr.begin(), aptr.end() - 1);
        for (int64_t e = 0; e < m; ++e) {
            adj[fill[fu[e]]++] = fv[e];
            adj[fill[fv[e]]++] = fu[e];
        }
    }
    Vec<uint8_t> alive(n, 0);
    par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t v = lo; v < hi; ++v)
            if (aptr[v + 1] > aptr[v]) {
                std::sort(adj.begin() + aptr[v], adj.begin() + aptr[v + 1]);
                alive[v] = 1;
            }
    });
    Vec<int32_t> top;
    for (int64_t v = 0; v < n; ++v)
        if (alive[v]) top.push_back((int32_t)v);
    Vec<int32_t> stamp(n, 0);  // visit marks: stamp[v] == the visit's stamp
    std::atomic<int32_t> next_stamp{0};
    std::atomic<int> spare{nt - 1};  // threads that may still be started
    constexpr size_t kParallelSet = size_t(1) << 16;
    auto take_thread = [&] {
        int s = spare.load();
        while (s > 0 && !spare.compare_exchange_weak(s, s - 1)) {
        }
        return s > 0;
    };
    // lays out the set vs (a union of components of the live graph) into out
    std::function<void(Vec<int32_t> &&, Vec<int32_t> &)> solve = [&](Vec<int32_t> &&vs,
                                                                       Vec<int32_t> &out) {
        Vec<int32_t> sort_tmp, bfs;
        Vec<int64_t> lev;
        // BFS inside the live vertices from `start`: the visit order in bfs,
        // level i in bfs[lev[i] .. lev[i+1]) (the last entry equals bfs.size())
        auto bfs_levels = [&](int32_t start) {
            const int32_t cur = ++next_stamp;
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
        };
        for (;;) {
            // connected components of the set, seeds in increasing id
            sort_ids(vs, n, sort_tmp);
            const int32_t cur = ++next_stamp;
            Vec<Vec<int32_t>> comps;
            for (int32_t v0 : vs) {
                if (stamp[v0] == cur) continue;
                stamp[v0] = cur;
                Vec<int32_t> comp(1, v0);
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
            Vec<int32_t>().swap(vs);
            if (comps.size() > 1) {
                // comp[0] is each component's smallest id
                std::stable_sort(comps.begin(), comps.end(),
                                 [](const Vec<int32_t> &x, const Vec<int32_t> &y) {
                                     return x.size() != y.size() ? x.size() < y.size()
                                                                 : x[0] < y[0];
                                 });
                Vec<Vec<int32_t>> outs(comps.size());
                std::vector<std::thread> ts;
                for (size_t j = 0; j < comps.size(); ++j) {
                    if (comps[j].size() >= kParallelSet && take_thread()) {
                        ts.emplace_back([&, j] {
                            solve(std::move(comps[j]), outs[j]);
                            spare.fetch_add(1);
                        });
                    } else {
                        solve(std::move(comps[j]), outs[j]);
                    }
                }
                for (auto &th : ts) th.join();
                for (auto &o : outs) out.insert(out.end(), o.begin(), o.end());
                return;
            }
            Vec<int32_t> comp = std::move(comps[0]);
            if (comp.size() == 1) {
                out.push_back(comp[0]);
                alive[comp[0]] = 0;
                return;
            }
            bfs_levels(comp[0]);
            bfs_levels(bfs.back());
            size_t li = 0;
            while (2 * (size_t)lev[li + 1] < comp.size()) ++li;
            for (int64_t i = lev[li]; i < lev[li + 1]; ++i) {
                out.push_back(bfs[i]);
                alive[bfs[i]] = 0;
            }
            // then the rest of the set
            for (int32_t v : comp)
                if (alive[v]) vs.push_back(v);
            if (vs.empty()) return;
        }
    };
    Vec<int32_t> out;
    solve(std::move(top), out);
    for (int32_t v : out) {
        order.push_back(v);
        placed[v] = 1;
    }
}

// Greedy vertex cover of a small edge set: repeatedly the vertex with the
// most uncovered edges, ties to the smaller id.
Vec<int32_t> greedy_cover(int64_t n, const Vec<int32_t> &eu,
                                  const Vec<int32_t> &ev) {
    Vec<int32_t> cover;
    const size_t m = eu.size();
    if (m == 0) return cover;
    Vec<int32_t> verts;
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
    Vec<Vec<size_t>> inc(nv);
    Vec<int64_t> deg(nv, 0);
    for (size_t e = 0; e < m; ++e) {
        inc[idx(eu[e])].push_back(e);
        inc[idx(ev[e])].push_back(e);
        ++deg[idx(eu[e])];
        ++deg[idx(ev[e])];
    }
    std::set<std::pair<int64_t, int32_t>> pq;  // (-deg, vertex)
    for (size_t i = 0; i < nv; ++i) pq.insert({-deg[i], verts[i]});
    Vec<uint8_t> covered(m, 0);
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


// Undirected edges of a symmetric remaining pattern: the entries above the
// diagonal, already sorted by (u, v) in CSR order (no duplicates: columns are
// strictly increasing within a row).
void upper_edges(int nt, const Vec<int32_t> &R, const Vec<int32_t> &C,
                 Vec<int32_t> &eu, Vec<int32_t> &ev, int64_t &n_diag) {
    const int64_t m = (int64_t)R.size();
    Vec<int64_t> c1(nt, 0), cd(nt, 0);
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

// Undirected edges {u, v} (u < v) of the pattern of the remaining entries
// (in CSR order), sorted by (u, v) without duplicates, and the number of
// diagonal entries.  Entries with r < c already come in (u, v) order; the
// others, keyed (c, r), are bucketed by ranges of c (per-thread counts,
// stable scatter) and counting-sorted by c within a bucket; the two sorted
// key lists are then merged per range of u.  With `symmetric` (not null) it
// tells whether the pattern equals its transpose, and a symmetric pattern
// returns no list (its graph is read from the rows).
void undirected_edges(int nt, int64_t n, const Vec<int32_t> &R,
                      const Vec<int32_t> &C, Vec<int32_t> &eu,
                      Vec<int32_t> &ev, int64_t &n_diag, bool *symmetric = nullptr) {
    const int64_t m = (int64_t)R.size();
    const uint64_t un = (uint64_t)std::max<int64_t>(n, 1);
    const int P = 64 * nt;  // buckets of list 2 by ranges of c
    auto bucket_of = [&](int64_t c) { return (int)(c * P / std::max<int64_t>(n, 1)); };
    Vec<int64_t> c1(nt, 0), cd(nt, 0), h2((size_t)nt * P, 0);
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
    Vec<int64_t> boff((size_t)nt * P), bstart(P + 1, 0);
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
    Vec<uint64_t> k2(m2);
    Vec<int32_t> r2(m2), c2(m2);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t *bo = &boff[(size_t)t * P];
        for (int64_t e = lo; e < hi; ++e)
            if (R[e] > C[e]) {
                const int64_t d = bo[bucket_of(C[e])]++;
                r2[d] = R[e];
                c2[d] = C[e];
            }
    });
    // within a bucket the entries are in CSR order (increasing r): a stable
    // counting sort by c leaves them sorted by (c, r)
    par_for(nt, P, [&](int64_t lo, int64_t hi, int) {
        Vec<int64_t> h;
        for (int64_t q = lo; q < hi; ++q) {
            const int64_t s0 = bstart[q], s1 = bstart[q + 1];
            if (s0 == s1) continue;
            const int64_t clo = (q * std::max<int64_t>(n, 1) + P - 1) / P;
            const int64_t chi = ((q + 1) * std::max<int64_t>(n, 1) + P - 1) / P;
            h.assign(chi - clo + 1, 0);
            for (int64_t i = s0; i < s1; ++i) ++h[c2[i] - clo + 1];
            for (int64_t j = 0; j < chi - clo; ++j) h[j + 1] += h[j];
            for (int64_t i = s0; i < s1; ++i)
                k2[s0 + h[c2[i] - clo]++] = (uint64_t)c2[i] * un + (uint64_t)r2[i];
        }
    });
    Vec<int32_t>().swap(r2);
    Vec<int32_t>().swap(c2);
    if (symmetric) {
        // the entries below the diagonal, transposed and sorted, equal the
        // ones above it (in CSR order) exactly when the pattern is symmetric
        Vec<uint8_t> same(nt, 1);
        if (m1 == m2)
            par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
                int64_t o = c1[t];
                for (int64_t e = lo; e < hi && same[t]; ++e)
                    if (R[e] < C[e]) same[t] = k2[o++] == (uint64_t)R[e] * un + (uint64_t)C[e];
            });
        *symmetric = m1 == m2;
        for (int t = 0; t < nt; ++t) *symmetric = *symmetric && same[t];
        if (*symmetric) {
            // the caller reads the graph from the rows
            eu.clear();
            ev.clear();
            return;
        }
    }
    Vec<uint64_t> k1(m1);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t o = c1[t];
        for (int64_t e = lo; e < hi; ++e)
            if (R[e] < C[e]) k1[o++] = (uint64_t)R[e] * un + (uint64_t)C[e];
    });
    // merge the two sorted lists per range of u, dropping duplicates
    Vec<int64_t> s1(nt + 1), s2(nt + 1), cnt(nt, 0);
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

// Pointer jumping: every vertex of `list` (non-roots of a forest of parent
// pointers) ends pointing at its root.  A vertex leaves the list once its
// parent is a root; the list is consumed.
void jump_to_roots(int nt, Vec<int32_t> &parent, Vec<int32_t> &list) {
    std::vector<Vec<int32_t>> keep(nt);
    while (!list.empty()) {
        par_for(nt, (int64_t)list.size(), [&](int64_t lo, int64_t hi, int t) {
            keep[t].clear();
            for (int64_t j = lo; j < hi; ++j) {
                const int32_t v = list[j], p = parent[v], g = parent[p];
                if (g != p) {
                    parent[v] = g;
                    keep[t].push_back(v);
                }
            }
        });
        list.clear();
        for (auto &q : keep) list.insert(list.end(), q.begin(), q.end());
    }
}

// Boruvka rounds of a minimum spanning forest under distinct weights: every
// component picks its lightest outgoing edge (atomic minimum of the weight),
// the picked edges join the forest and merge the components.  The forest is
// unique, so the result does not depend on the thread count.
//
// `parent` holds every vertex's component label (the vertex id of the
// component's root; parent[r] == r for a root).  Each live edge carries its
// weight kk, its id and the labels cu, cv of its endpoints' components.
// Thread t owns the edges [seg_lo[t], seg_lo[t] + seg_n[t]).  A round makes
// two passes over them: the first relabels both ends through the previous
// round's merges, drops edges inside one component and takes the minima; the
// second links every component to the far end of its picked edge and
// compacts the edges kept by the first pass within the thread's range.
// Appends the ids of the forest's edges to `chosen` (in no particular order).
void boruvka_rounds(int nt, Vec<int32_t> &parent, Vec<int32_t> &cu,
                    Vec<int32_t> &cv, Vec<uint64_t> &kk,
                    Vec<int32_t> &id, const Vec<int64_t> &seg_lo,
                    Vec<int64_t> &seg_n, Vec<int32_t> &chosen) {
    const int64_t n = (int64_t)parent.size();
    Vec<uint64_t> best(n, UINT64_MAX);
    Vec<Vec<int32_t>> linked(nt), ids(nt);
    Vec<int32_t> roots;
    Vec<int64_t> alive(nt);
    // ranges of a few thousand edges run on the calling thread
    auto each = [&](auto &&fn) {
        int64_t total = 0;
        for (int t = 0; t < nt; ++t) total += seg_n[t];
        if (total < 4096) {
            for (int t = 0; t < nt; ++t) fn(t);
        } else {
            par_each(nt, fn);
        }
    };
    for (;;) {
        // relabel, drop edges inside a component, take the minima
        each([&](int t) {
            int64_t a = 0;
            const int64_t lo = seg_lo[t], hi = lo + seg_n[t];
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t pu = parent[cu[i]], pv = parent[cv[i]];
                cu[i] = pu;
                cv[i] = pv;
                if (pu == pv) continue;
                ++a;
                atomic_min_u64(&best[pu], kk[i]);
                atomic_min_u64(&best[pv], kk[i]);
            }
            alive[t] = a;
        });
        int64_t total = 0;
        for (int t = 0; t < nt; ++t) total += alive[t];
        if (total == 0) break;
        // link each component along its minimum edge (one writer per
        // component: weights are distinct); keep the edges that joined two
        // components, in order, at the front of the thread's range
        each([&](int t) {
            linked[t].clear();
            const int64_t lo = seg_lo[t], hi = lo + seg_n[t];
            int64_t o = lo;
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t u = cu[i], v = cv[i];
                if (u == v) continue;
                const uint64_t k = kk[i];
                const bool pu = best[u] == k, pv = best[v] == k;
                if (pu) {
                    parent[u] = v;
                    linked[t].push_back(u);
                }
                if (pv) {
                    parent[v] = u;
                    linked[t].push_back(v);
                }
                if (pu || pv) ids[t].push_back(id[i]);
                cu[o] = u;
                cv[o] = v;
                kk[o] = k;
                id[o] = id[i];
                ++o;
            }
            seg_n[t] = o - lo;
        });
        roots.clear();
        for (auto &q : linked) roots.insert(roots.end(), q.begin(), q.end());
        const int64_t nr = (int64_t)roots.size();
        // two components that picked the same edge point at each other: the
        // smaller becomes the root
        par_for(nt, nr, [&](int64_t lo, int64_t hi, int) {
            for (int64_t j = lo; j < hi; ++j) {
                const int32_t v = roots[j], p = parent[v];
                if (parent[p] == v && v < p) parent[v] = v;
            }
        });
        par_for(nt, nr, [&](int64_t lo, int64_t hi, int) {
            for (int64_t j = lo; j < hi; ++j) best[roots[j]] = UINT64_MAX;
        });
        // only the labels linked in this Boruvka round move
        jump_to_roots(nt, parent, roots);
    }
    for (auto &q : ids) chosen.insert(chosen.end(), q.begin(), q.end());
}

// Minimum spanning forest of the edges listed in `live` (indices into the
// edge list eu, ev) under the distinct weights key[e].
void boruvka_msf(int nt, int64_t n, const Vec<int32_t> &eu,
                 const Vec<int32_t> &ev, const Vec<uint64_t> &key,
                 const Vec<int64_t> &live, Vec<int32_t> &fu,
                 Vec<int32_t> &fv) {
    const int64_t m = (int64_t)live.size();
    Vec<int32_t> cu(m), cv(m), id(m);
    Vec<uint64_t> kk(m);
    Vec<int64_t> seg_lo(nt), seg_n(nt);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        seg_lo[t] = lo;
        seg_n[t] = hi - lo;
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t e = live[i];
            cu[i] = eu[e];
            cv[i] = ev[e];
            id[i] = (int32_t)e;
            kk[i] = key[e];
        }
    });
    Vec<int32_t> parent(n);
    par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t v = lo; v < hi; ++v) parent[v] = (int32_t)v;
    });
    Vec<int32_t> chosen;
    boruvka_rounds(nt, parent, cu, cv, kk, id, seg_lo, seg_n, chosen);
    fu.resize(chosen.size());
    fv.resize(chosen.size());
    for (size_t j = 0; j < chosen.size(); ++j) {
        fu[j] = eu[chosen[j]];
        fv[j] = ev[chosen[j]];
    }
}

// Row pointers of the remaining entries (in CSR order), the rows that hold a
// diagonal entry, and their number.
void rows_of(int nt, int64_t n, const Vec<int32_t> &R, const Vec<int32_t> &C,
             Vec<int64_t> &ptr, Vec<uint8_t> &diag, int64_t &n_diag) {
    const int64_t m = (int64_t)R.size();
    ptr.assign(n + 1, 0);
    diag.assign(n, 0);
    Vec<int64_t> cd(nt, 0);
    par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
        int64_t d = 0;
        for (int64_t e = lo; e < hi;) {
            const int32_t r = R[e];
            int64_t f = e;
            for (; f < hi && R[f] == r; ++f)
                if (C[f] == r) {
                    diag[r] = 1;
                    ++d;
                }
            __atomic_fetch_add(&ptr[r + 1], f - e, __ATOMIC_RELAXED);
            e = f;
        }
        cd[t] = d;
    });
    n_diag = 0;
    for (int t = 0; t < nt; ++t) n_diag += cd[t];
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
}

// The minimum spanning forest of the graph G - H of a symmetric remaining
// pattern (edges: the entries off the diagonal, the vertices of H removed)
// under the weights w(u, v) = SplitMix64 output u * n + v of state ls
// (u < v), the same edge weights as the listed form above.  The first
// Boruvka round takes each vertex's lightest edge straight from its row;
// the later rounds run over the entries above the diagonal that still join
// two components.
void forest_from_rows(int nt, int64_t n, const Vec<int64_t> &ptr,
                      const Vec<int32_t> &R, const Vec<int32_t> &C,
                      const Vec<uint8_t> &is_head, uint64_t ls,
                      Vec<int32_t> &fu, Vec<int32_t> &fv) {
    const uint64_t un = (uint64_t)n;
    auto weight = [&](int32_t a, int32_t b) {
        return a < b ? sm_output(ls, (uint64_t)a * un + (uint64_t)b)
                     : sm_output(ls, (uint64_t)b * un + (uint64_t)a);
    };
    // first Boruvka round: every vertex of G - H with an edge picks its lightest one
    Vec<int32_t> pick(n, -1), parent(n);
    par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t v = lo; v < hi; ++v) {
            parent[v] = (int32_t)v;
            if (is_head[v]) continue;
            uint64_t bk = UINT64_MAX;
            int32_t bw = -1;
            for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
                const int32_t w = C[e];
                if (w == v || is_head[w]) continue;
                const uint64_t k = weight((int32_t)v, w);
                if (k < bk) {
                    bk = k;
                    bw = w;
                }
            }
            pick[v] = bw;
        }
    });
    // link along the picks; a pair that picked each other keeps the smaller
    // as its root and contributes its edge once
    Vec<Vec<int32_t>> fu_t(nt), fv_t(nt), linked_t(nt);
    par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
        for (int64_t v = lo; v < hi; ++v) {
            const int32_t w = pick[v];
            if (w < 0) continue;
            const bool mutual = pick[w] == v;
            if (mutual && v < w) continue;  // v stays a root
            parent[v] = w;
            linked_t[t].push_back((int32_t)v);
            fu_t[t].push_back((int32_t)std::min<int64_t>(v, w));
            fv_t[t].push_back((int32_t)std::max<int64_t>(v, w));
        }
    });
    Vec<int32_t> linked;
    fu.clear();
    fv.clear();
    for (int t = 0; t < nt; ++t) {
        linked.insert(linked.end(), linked_t[t].begin(), linked_t[t].end());
        fu.insert(fu.end(), fu_t[t].begin(), fu_t[t].end());
        fv.insert(fv.end(), fv_t[t].begin(), fv_t[t].end());
    }
    jump_to_roots(nt, parent, linked);
    // the components that have an edge (their roots picked one), numbered
    // 0 .. nc-1 in root order: the later rounds work on these compact
    // labels (smaller arrays for their random accesses)
    Vec<int32_t> cid(n);
    int64_t nc = 0;
    {
        Vec<int64_t> c(nt);
        par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
            int64_t k = 0;
            for (int64_t v = lo; v < hi; ++v) k += pick[v] >= 0 && parent[v] == v;
            c[t] = k;
        });
        nc = exclusive_scan(c);
        par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
            int32_t k = (int32_t)c[t];
            for (int64_t v = lo; v < hi; ++v)
                if (pick[v] >= 0 && parent[v] == v) cid[v] = k++;
        });
    }
    Vec<int32_t>().swap(pick);
    // the edges above the diagonal that join two components after the first round,
    // by rows (columns are sorted within a row: the entries above the
    // diagonal are a row's tail); thread t writes them from the offset of
    // its rows' entries above the diagonal
    auto upper_begin = [&](int64_t v) {
        return std::upper_bound(C.begin() + ptr[v], C.begin() + ptr[v + 1], (int32_t)v) -
               C.begin();
    };
    Vec<int64_t> rcut(nt + 1), cnt(nt), seg_lo(nt), seg_n(nt);
    {
        const int64_t m = ptr[n];
        for (int t = 0; t <= nt; ++t)
            rcut[t] = std::lower_bound(ptr.begin(), ptr.end() - 1, m * t / nt) - ptr.begin();
        rcut[nt] = n;
        for (int t = 1; t <= nt; ++t) rcut[t] = std::max(rcut[t], rcut[t - 1]);
    }
    par_each(nt, [&](int t) {
        int64_t c = 0;
        for (int64_t v = rcut[t]; v < rcut[t + 1]; ++v)
            if (!is_head[v]) c += ptr[v + 1] - upper_begin(v);
        cnt[t] = c;
    });
    const int64_t nup = exclusive_scan(cnt);
    Vec<int32_t> cu(nup), cv(nup), id(nup);
    Vec<uint64_t> kk(nup);
    par_each(nt, [&](int t) {
        int64_t o = cnt[t];
        seg_lo[t] = o;
        for (int64_t v = rcut[t]; v < rcut[t + 1]; ++v) {
            if (is_head[v]) continue;
            const int32_t pv = parent[v];
            for (int64_t e = upper_begin(v); e < ptr[v + 1]; ++e) {
                const int32_t w = C[e];
                if (is_head[w] || parent[w] == pv) continue;
                cu[o] = cid[pv];
                cv[o] = cid[parent[w]];
                kk[o] = weight((int32_t)v, w);
                id[o] = (int32_t)e;
                ++o;
            }
        }
        seg_n[t] = o - seg_lo[t];
    });
    Vec<int32_t>().swap(parent);
    Vec<int32_t>().swap(cid);
    Vec<int32_t> label(nc), chosen;
    par_for(nt, nc, [&](int64_t lo, int64_t hi, int) {
        for (int64_t j = lo; j < hi; ++j) label[j] = (int32_t)j;
    });
    boruvka_rounds(nt, label, cu, cv, kk, id, seg_lo, seg_n, chosen);
    for (const int32_t e : chosen) {
        fu.push_back(R[e]);
        fv.push_back(C[e]);
    }
}

}  // namespace


arrow_status_t decompose(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const float *val, const arrow_decompose_opts_t &opts, Decomp &out) {
    auto t0 = std::chrono::steady_clock::now();
    CacheUser cache_user;
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
    const int nt = host_threads(opts.threads);
    {
        // the first bad row (the same message for every thread count)
        Vec<int64_t> bad_col(nt, INT64_MAX), bad_ord(nt, INT64_MAX);
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

    Vec<uint8_t> is_head(n), has_entry(n), placed(n);
    Vec<int32_t> pos(n);
    Vec<int64_t> tcnt(nt), tmax(nt);
    bool pattern_symmetric = false;
    for (int32_t level = 0;; ++level) {
        if (opts.max_levels > 0 && level >= opts.max_levels) {
            set_error("decomposition needs more than max_levels = " +
                      std::to_string(opts.max_levels) + " levels");
            out = Decomp();
            return ARROW_ERR_UNSUPPORTED;
        }
        const int64_t m = (int64_t)rem.size();
        // undirected edges of the remaining pattern, sorted by (u, v).  A
        // symmetric pattern stays symmetric at every level ((u, v) and (v, u)
        // always land in the same level): its graph is then read from the
        // rows of the remaining entries, and the edge list (the entries above
        // the diagonal, in order) is formed only where a step needs it.
        Vec<int32_t> eu, ev;
        int64_t n_diag = 0, ne = 0;
        Vec<int64_t> rptr;
        Vec<uint8_t> rdiag;
        if (level == 0 || !pattern_symmetric)
            undirected_edges(nt, n, rem.r, rem.c, eu, ev, n_diag,
                             level == 0 ? &pattern_symmetric : nullptr);
        if (pattern_symmetric) {
            rows_of(nt, n, rem.r, rem.c, rptr, rdiag, n_diag);
            ne = (m - n_diag) / 2;
            par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
                for (int64_t v = lo; v < hi; ++v) has_entry[v] = rptr[v + 1] > rptr[v];
            });
        } else {
            ne = (int64_t)eu.size();
            std::fill(has_entry.begin(), has_entry.end(), 0);
            par_for(nt, m, [&](int64_t lo, int64_t hi, int) {
                for (int64_t e = lo; e < hi; ++e) {
                    __atomic_store_n(&has_entry[rem.r[e]], (uint8_t)1, __ATOMIC_RELAXED);
                    __atomic_store_n(&has_entry[rem.c[e]], (uint8_t)1, __ATOMIC_RELAXED);
                }
            });
        }
        auto edge_list = [&] {
            if (pattern_symmetric && eu.empty() && ne > 0) {
                int64_t nd = 0;
                upper_edges(nt, rem.r, rem.c, eu, ev, nd);
            }
        };
        std::fill(is_head.begin(), is_head.end(), 0);
        std::fill(placed.begin(), placed.end(), 0);
        Vec<int32_t> order;
        order.reserve(n);
        const bool final_level = 2 * ne + n_diag <= 2 * b;
        if (final_level) {
            edge_list();
            for (int32_t v : greedy_cover(n, eu, ev)) {
                order.push_back(v);
                is_head[v] = placed[v] = 1;
            }
        } else {
            Vec<int64_t> deg(n, 0);
            if (pattern_symmetric) {
                par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
                    for (int64_t v = lo; v < hi; ++v) deg[v] = rptr[v + 1] - rptr[v] - rdiag[v];
                });
            } else {
                par_for(nt, ne, [&](int64_t lo, int64_t hi, int) {
                    for (int64_t e = lo; e < hi; ++e) {
                        __atomic_fetch_add(&deg[eu[e]], (int64_t)1, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&deg[ev[e]], (int64_t)1, __ATOMIC_RELAXED);
                    }
                });
            }
            Vec<int32_t> cand;
            {
                Vec<Vec<int32_t>> part(nt);
                par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
                    for (int64_t v = lo; v < hi; ++v)
                        if (deg[v] > 0) part[t].push_back((int32_t)v);
                });
                for (auto &q : part) cand.insert(cand.end(), q.begin(), q.end());
            }
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
                Vec<int32_t> fu, fv;
                if (pattern_symmetric) {
                    forest_from_rows(nt, n, rptr, rem.r, rem.c, is_head, ls, fu, fv);
                } else {
                    Vec<uint64_t> key(ne);
                    par_for(nt, ne, [&](int64_t lo, int64_t hi, int t) {
                        int64_t c = 0;
                        for (int64_t e = lo; e < hi; ++e) {
                            key[e] = sm_output(ls, (uint64_t)eu[e] * (uint64_t)n + (uint64_t)ev[e]);
                            c += !is_head[eu[e]] && !is_head[ev[e]];
                        }
                        tcnt[t] = c;
                    });
                    Vec<int64_t> off(tcnt.begin(), tcnt.end());
                    const int64_t nl = exclusive_scan(off);
                    Vec<int64_t> live(nl);
                    par_for(nt, ne, [&](int64_t lo, int64_t hi, int t) {
                        int64_t o = off[t];
                        for (int64_t e = lo; e < hi; ++e)
                            if (!is_head[eu[e]] && !is_head[ev[e]]) live[o++] = e;
                    });
                    boruvka_msf(nt, n, eu, ev, key, live, fu, fv);
                }
                layout_forest(nt, n, fu, fv, order, placed);
            } else if (opts.la == ARROW_LA_SEPARATOR) {
                // the edges of G_i - H_i
                edge_list();
                Vec<int32_t> gu, gv;
                for (int64_t e = 0; e < ne; ++e)
                    if (!is_head[eu[e]] && !is_head[ev[e]]) {
                        gu.push_back(eu[e]);
                        gv.push_back(ev[e]);
                    }
                layout_separator(nt, n, gu, gv, order, placed);
            }
        }
        // then the unplaced vertices that hold entries, then the rest, by id
        {
            Vec<int64_t> c_ent(nt), c_rest(nt);
            par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
                int64_t a = 0, r = 0;
                for (int64_t v = lo; v < hi; ++v)
                    if (!placed[v]) (has_entry[v] ? a : r) += 1;
                c_ent[t] = a;
                c_rest[t] = r;
            });
            const int64_t base = (int64_t)order.size();
            const int64_t n_ent = exclusive_scan(c_ent);
            const int64_t n_rest = exclusive_scan(c_rest);
            order.resize(base + n_ent + n_rest);
            par_for(nt, n, [&](int64_t lo, int64_t hi, int t) {
                int64_t a = base + c_ent[t], r = base + n_ent + c_rest[t];
                for (int64_t v = lo; v < hi; ++v)
                    if (!placed[v]) order[has_entry[v] ? a++ : r++] = (int32_t)v;
            });
        }
        if ((int64_t)order.size() != n) {
            set_error("internal: arrangement is not a permutation");
            return ARROW_ERR_INTERNAL;
        }
        par_for(nt, n, [&](int64_t lo, int64_t hi, int) {
            for (int64_t p = lo; p < hi; ++p) pos[order[p]] = (int32_t)p;
        });

        // classify: an entry whose positions (p, q) satisfy p < b or q < b or
        // |p - q| <= b goes to B_i (its q is kept in Q), the others to A_{i+1}
        if (rptr.empty()) {
            int64_t nd = 0;
            rows_of(nt, n, rem.r, rem.c, rptr, rdiag, nd);
        }
        Vec<int32_t> Q(m);
        Vec<int32_t> row_keep(n, 0);  // entries of a vertex's row kept in B_i
        par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
            int64_t c = 0, mx = -1;
            for (int64_t e = lo; e < hi;) {
                const int32_t r = rem.r[e];
                const int64_t p = pos[r];
                int64_t f = e, k = 0;
                for (; f < hi && rem.r[f] == r; ++f) {
                    const int64_t q = pos[rem.c[f]];
                    if (p < b || q < b || (p > q ? p - q : q - p) <= b) {
                        Q[f] = (int32_t)q;
                        ++k;
                        mx = std::max(mx, std::max(p, q));
                    } else {
                        Q[f] = -1;
                    }
                }
                __atomic_fetch_add(&row_keep[r], (int32_t)k, __ATOMIC_RELAXED);
                c += k;
                e = f;
            }
            tcnt[t] = c;
            tmax[t] = mx;
        });
        int64_t maxpos = -1;
        for (int t = 0; t < nt; ++t) maxpos = std::max(maxpos, tmax[t]);
        Vec<int64_t> moff(nt);
        int64_t nk = 0;
        {
            int64_t o = 0;
            for (int t = 0; t < nt; ++t) {
                moff[t] = o;
                o += (m * (t + 1) / nt - m * t / nt) - tcnt[t];
                nk += tcnt[t];
            }
        }
        // A_{i+1}: the entries that move on, still in CSR order
        Entries next;
        next.r.resize(m - nk);
        next.c.resize(m - nk);
        next.v.resize(m - nk);
        par_for(nt, m, [&](int64_t lo, int64_t hi, int t) {
            int64_t o = moff[t];
            for (int64_t e = lo; e < hi; ++e)
                if (Q[e] < 0) {
                    next.r[o] = rem.r[e];
                    next.c[o] = rem.c[e];
                    next.v[o] = rem.v[e];
                    ++o;
                }
        });
        if (final_level && !next.r.empty()) {
            set_error("internal: last level left entries");
            return ARROW_ERR_INTERNAL;
        }
        // B_i in position order: row p holds the kept entries of vertex
        // order[p]'s row, sorted by q (positions within a row are distinct)
        Level L;
        L.n_i = level == 0 ? n : maxpos + 1;
        L.vop.assign(order.begin(), order.begin() + L.n_i);
        L.row_ptr.assign(L.n_i + 1, 0);
        par_for(nt, L.n_i, [&](int64_t lo, int64_t hi, int) {
            for (int64_t q = lo; q < hi; ++q) L.row_ptr[q + 1] = row_keep[order[q]];
        });
        for (int64_t i = 0; i < L.n_i; ++i) L.row_ptr[i + 1] += L.row_ptr[i];
        L.col.resize(nk);
        L.val.resize(nk);
        // rows split into ranges of equal entry counts (head rows are long)
        Vec<int64_t> rcut(nt + 1, 0);
        for (int t = 1; t < nt; ++t)
            rcut[t] = std::max<int64_t>(
                rcut[t - 1], std::lower_bound(L.row_ptr.begin(), L.row_ptr.end() - 1,
                                              nk * t / nt) - L.row_ptr.begin());
        rcut[nt] = L.n_i;
        par_each(nt, [&](int tt) {
            Vec<std::pair<int32_t, float>> tmp;
            for (int64_t i = rcut[tt]; i < rcut[tt + 1]; ++i) {
                const int32_t v = order[i];
                const int64_t s0 = L.row_ptr[i], s1 = L.row_ptr[i + 1];
                if (s0 == s1) continue;
                int64_t d = s0;
                bool sorted = true;
                for (int64_t e = rptr[v]; e < rptr[v + 1]; ++e)
                    if (Q[e] >= 0) {
                        if (d > s0 && Q[e] < L.col[d - 1]) sorted = false;
                        L.col[d] = Q[e];
                        L.val[d] = rem.v[e];
                        ++d;
                    }
                if (sorted) continue;
                tmp.clear();
                for (int64_t j = s0; j < s1; ++j) tmp.push_back({L.col[j], L.val[j]});
                std::sort(tmp.begin(), tmp.end(),
                          [](const std::pair<int32_t, float> &a,
                             const std::pair<int32_t, float> &c) { return a.first < c.first; });
                for (int64_t j = s0; j < s1; ++j) {
                    L.col[j] = tmp[j - s0].first;
                    L.val[j] = tmp[j - s0].second;
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
