// Plan construction (host) and launch orchestration.
//
// The decomposition's levels become three row passes in level-0 order:
//  * chunk pass: every row longer than kLongRow, cut into chunks of kChunk
//    entries (the hub rows behind the load imbalance discussed in Section
//    7.3; most of them are head rows of B_0, the row tiles of Section 4.1);
//  * upper pass: the rows of B_i (i >= 1) not folded into level 0, with
//    columns mapped to level-0 positions through sigma_i = pi_0 o pi_i^{-1};
//  * level-0 pass: per row, the entries of B_0 and of the short rows of
//    levels >= 1 of the same vertex (folded in), as 16-bit codes: relative to
//    the row inside the band, the head column, or an index into the block's
//    far-column table (folded entries and a short head row's columns beyond
//    the band); plus a list per row of the partial rows to add: its own
//    chunks, then the upper-pass rows of the same vertex by level (the
//    accumulation of Alg. 2, in a fixed order).
#include "plan.h"

#include <atomic>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "host_threads.h"

namespace arrow {
namespace {

#define HIP_OK(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));          \
            return ARROW_ERR_HIP;                                                  \
        }                                                                          \
    } while (0)

Allocator g_allocator;

template <class T>
arrow_status_t upload(Plan &p, T *&dst, const std::vector<T> &src, hipStream_t s) {
    dst = nullptr;
    if (src.empty()) return ARROW_OK;
    void *d = nullptr;
    const size_t bytes = src.size() * sizeof(T);
    if (p.allocator.alloc) {
        d = p.allocator.alloc(bytes, s, p.allocator.ctx);
        if (!d) {
            set_error("the plan allocator returned NULL for " + std::to_string(bytes) + " bytes");
            return ARROW_ERR_OUT_OF_MEMORY;
        }
        if (reinterpret_cast<uintptr_t>(d) % 256 != 0) {
            p.allocator.free(d, nullptr, p.allocator.ctx);
            set_error("the plan allocator returned a pointer that is not 256-byte aligned");
            return ARROW_ERR_INVALID_ARG;
        }
    } else {
        hipError_t e = hipMalloc(&d, bytes);
        if (e != hipSuccess) {
            set_error(std::string("hipMalloc of plan array: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? ARROW_ERR_OUT_OF_MEMORY : ARROW_ERR_HIP;
        }
    }
    p.allocs.push_back(d);
    p.footprint += (int64_t)(src.size() * sizeof(T));
    HIP_OK(hipMemcpyAsync(d, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    dst = static_cast<T *>(d);
    return ARROW_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t count_true(const std::vector<uint8_t> &m) {
    int64_t c = 0;
    for (uint8_t v : m) c += v;
    return c;
}

}  // namespace

Allocator current_allocator() { return g_allocator; }
void set_allocator(const Allocator &a) { g_allocator = a; }

int64_t elem_size(int dtype) { return dtype == kF32 ? 4 : (dtype == kF8E4M3 ? 1 : 2); }

int tile_width(int64_t k) {
    for (int kt : {128, 64, 32, 16})
        if (k % kt == 0) return kt;
    return 0;
}

static int64_t nblocks_of(int64_t rows, int64_t rpb) { return (rows + rpb - 1) / rpb; }

// Workgroups of a pass over `rows` rows (blocks of rpb rows, bpw blocks each).
static int64_t nwg_of(int64_t rows, int64_t rpb, int64_t bpw) {
    return nblocks_of(nblocks_of(rows, rpb), bpw);
}

static void set_geometry(RowPass &rp, int64_t rows, int rpb, int bpw) {
    rp.nrows = rows;
    rp.rows_per_block = rpb;
    rp.blocks_per_wg = bpw;
    rp.nwg = (int32_t)nwg_of(rows, rpb, bpw);
}

template <class I>
int32_t choose_batch(int64_t nrows, const I *ptr, const int32_t *cptr) {
    if (nrows <= 0) return kBatchWide;
    const int64_t allowed = nrows / 100;  // rows that may need more than one batch
    if (cptr) {
        int64_t many = 0;
        for (int64_t r = 0; r < nrows; ++r) many += (cptr[r + 1] - cptr[r]) > 2;
        if (many > allowed) return kBatchWide;
    }
    int64_t longer[kBatchMax + 1] = {};  // rows with more than u entries
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t len = (int64_t)(ptr[r + 1] - ptr[r]);
        for (int u = kBatchMin; u <= kBatchMax; ++u) longer[u] += len > u;
    }
    for (int u = kBatchMin; u <= kBatchMax; ++u)
        if (longer[u] <= allowed) return u;
    return kBatchWide;
}
template int32_t choose_batch<int32_t>(int64_t, const int32_t *, const int32_t *);
template int32_t choose_batch<int64_t>(int64_t, const int64_t *, const int32_t *);

// Partial slots of the final pass (one per workgroup of the level-0 pass).
static int l0_blocks_per_wg(int dtype) {
    return dtype == kF16 || dtype == kF8E4M3 ? kBlocksPerWgScaled : kBlocksPerWg;
}
static int64_t final_parts(int64_t n, int64_t rpb) { return nwg_of(n, rpb, kBlocksPerWg); }
static int64_t final_parts(const Plan &p, int dtype) {
    return nwg_of(p.n, p.l0_rpb, l0_blocks_per_wg(dtype));
}

void plan_build(const Decomp &d, Plan &p, PlanArrays &h) {
    const int nt = host_threads(0);
    p.n = d.n;
    p.nnz = d.nnz;
    p.b = d.b;
    p.levels = (int32_t)d.levels.size();
    p.code16 = 3LL * d.b <= 65535;
    const int64_t n = d.n, b = d.b;
    const Level &L0 = d.levels[0];

    std::vector<int32_t> pos0(n);
    for (int64_t q = 0; q < n; ++q) pos0[L0.vop[q]] = (int32_t)q;

    // |A| row sums for the FP8/FP16 scale bound
    {
        // (a level's rows belong to distinct vertices: its rows run in
        // parallel, each vertex's sum in the same order as one thread)
        std::vector<double> rs(n, 0.0);
        for (const Level &L : d.levels)
            par_for(nt, L.n_i, [&](int64_t lo, int64_t hi, int) {
                for (int64_t q = lo; q < hi; ++q)
                    for (int64_t e = L.row_ptr[q]; e < L.row_ptr[q + 1]; ++e)
                        rs[L.vop[q]] += std::fabs((double)L.val[e]);
            });
        for (double v : rs) p.a_inf = std::max(p.a_inf, v);
    }

    // rows of levels >= 1 that hold entries, grouped by the level-0 row of
    // their vertex (level order within a vertex); `order` keeps (level, pos)
    struct UpRow { int32_t level; int32_t pos; };
    auto up_len = [&](const UpRow &u) -> int64_t {
        const Level &L = d.levels[u.level];
        return L.row_ptr[u.pos + 1] - L.row_ptr[u.pos];
    };
    std::vector<int64_t> vrow_ptr(n + 1, 0);
    for (int32_t i = 1; i < p.levels; ++i) {
        const Level &L = d.levels[i];
        for (int64_t q = 0; q < L.n_i; ++q)
            if (L.row_ptr[q + 1] > L.row_ptr[q]) ++vrow_ptr[pos0[L.vop[q]] + 1];
    }
    for (int64_t r = 0; r < n; ++r) vrow_ptr[r + 1] += vrow_ptr[r];
    std::vector<UpRow> vrows(vrow_ptr[n]);
    std::vector<int64_t> order;  // indices into vrows, in (level, position) order
    order.reserve(vrows.size());
    {
        std::vector<int64_t> fill(vrow_ptr.begin(), vrow_ptr.end() - 1);
        for (int32_t i = 1; i < p.levels; ++i) {
            const Level &L = d.levels[i];
            for (int64_t q = 0; q < L.n_i; ++q)
                if (L.row_ptr[q + 1] > L.row_ptr[q]) {
                    const int64_t si = fill[pos0[L.vop[q]]]++;
                    vrows[si] = {i, (int32_t)q};
                    order.push_back(si);
                }
        }
    }

    // level-0 rows of the chunk pass: long rows (the hub rows among the head
    // rows of B_0 in particular).  A short head row stays in the level-0
    // pass: its columns beyond the band (q > r + b) go through the block's
    // far-column table like folded entries.
    std::vector<uint8_t> chunked0(n, 0);
    auto head_far = [&](int64_t r) -> int64_t {  // entries of row r beyond the band
        int64_t c = 0;
        if (r < b)
            for (int64_t e = L0.row_ptr[r]; e < L0.row_ptr[r + 1]; ++e) c += L0.col[e] > r + b;
        return c;
    };
    for (int64_t r = 0; r < n; ++r) chunked0[r] = L0.row_ptr[r + 1] - L0.row_ptr[r] > kLongRow;

    // Level-0 block size: the largest of 256, 128, 64 rows for which 95% of
    // the blocks' entries (level 0 plus the short rows that may fold in) fit
    // the LDS staging area.
    p.l0_rpb = kMaxBlockRows;
    for (int rpb = kMaxBlockRows; rpb >= 64; rpb /= 2) {
        p.l0_rpb = rpb;
        const int64_t nblk = nblocks_of(n, rpb);
        int64_t over = 0;
        for (int64_t blk = 0; blk < nblk; ++blk) {
            int64_t ne = 0;
            for (int64_t r = blk * rpb; r < std::min<int64_t>(n, (blk + 1) * rpb); ++r) {
                if (chunked0[r]) continue;
                ne += L0.row_ptr[r + 1] - L0.row_ptr[r];
                for (int64_t si = vrow_ptr[r]; si < vrow_ptr[r + 1]; ++si) {
                    const int64_t ul = up_len(vrows[si]);
                    if (ul <= kLongRow) ne += ul;
                }
            }
            over += ne > kStageEntries;
        }
        if (over * 20 <= nblk) break;
    }
    const int64_t rpb0 = p.l0_rpb;

    // Cross-level accumulation at entry level: a short row of a level >= 1
    // joins the entry list of its vertex's level-0 row (columns mapped through
    // sigma_i), as long as the row stays within kFuseRow entries and the
    // 16-bit codes 3b+1+j of the block's far-column table have room.  The
    // rest keep the upper pass and reach the level-0 row as partial rows.
    // (and the block's table fits the kernel's LDS staging)
    const int64_t far_cap =
        p.code16 ? std::min<int64_t>(65535 - 3 * (int64_t)b, kStageFarWide) : INT64_MAX;
    std::vector<uint8_t> fused(vrows.size(), 0);
    for (int64_t blk = 0; blk < nblocks_of(n, rpb0); ++blk) {
        int64_t far = 0;
        // the head rows' own far entries first (a head row that does not fit
        // the code space goes to the chunk pass)
        for (int64_t r = blk * rpb0; r < std::min<int64_t>({n, (blk + 1) * rpb0, (int64_t)b});
             ++r) {
            if (chunked0[r] || !p.code16) continue;
            const int64_t hf = head_far(r);
            if (far + hf > far_cap)
                chunked0[r] = 1;
            else
                far += hf;
        }
        for (int64_t r = blk * rpb0; r < std::min<int64_t>(n, (blk + 1) * rpb0); ++r) {
            if (chunked0[r]) continue;
            int64_t len = L0.row_ptr[r + 1] - L0.row_ptr[r];
            for (int64_t si = vrow_ptr[r]; si < vrow_ptr[r + 1]; ++si) {
                const int64_t ul = up_len(vrows[si]);
                if (ul > kLongRow || len + ul > kFuseRow || far + ul > far_cap) continue;
                fused[si] = 1;
                len += ul;
                far += ul;
                ++p.fused_rows;
            }
        }
    }

    // upper rows: the rows of levels >= 1 not folded in, in (level, position) order
    std::vector<UpRow> up;
    std::vector<int64_t> up_of(vrows.size(), -1);  // vrows index -> upper row
    for (int64_t si : order)
        if (!fused[si]) {
            up_of[si] = (int64_t)up.size();
            up.push_back(vrows[si]);
        }
    p.n_up = (int64_t)up.size();

    // chunks: level-0 chunked rows, then chunked upper rows.  A row with at
    // least kWindowRow far entries (beyond the head columns and the band
    // around the row's own level-0 position) splits into a local group and
    // one group per column window of its far entries; any other long row is
    // one group.  Each group is cut into chunks of at most kChunk entries,
    // ascending column within a group.  The windows split the far entries of
    // the split rows into kChunkWindows ranges of level-0 columns with equal
    // entry counts.
    auto is_far = [&](int64_t c, int64_t r0) { return c >= b && std::llabs(c - r0) > b; };
    auto far_count = [&](const Level &L, int64_t q, bool map, int64_t r0) {
        int64_t nf = 0;
        for (int64_t e = L.row_ptr[q]; e < L.row_ptr[q + 1]; ++e)
            nf += is_far(map ? pos0[L.vop[L.col[e]]] : L.col[e], r0);
        return nf;
    };
    std::vector<int64_t> win_lo(kChunkWindows + 1, n);  // window w: [win_lo[w], win_lo[w+1])
    {
        // far entries per level-0 column over the rows that split (counted
        // in parallel over the long rows)
        std::vector<int64_t> cnt(n + 1, 0);
        struct LongRow { const Level *L; int64_t q, r0; bool map; };
        std::vector<LongRow> long_rows;
        for (int64_t r = 0; r < n; ++r)
            if (chunked0[r]) long_rows.push_back({&L0, r, r, false});
        for (int64_t si = 0; si < (int64_t)vrows.size(); ++si)
            if (!fused[si] && up_len(vrows[si]) > kLongRow) {
                const Level &L = d.levels[vrows[si].level];
                long_rows.push_back({&L, vrows[si].pos, (int64_t)pos0[L.vop[vrows[si].pos]], true});
            }
        std::vector<int64_t> tot_t(nt, 0);
        par_for(nt, (int64_t)long_rows.size(), [&](int64_t lo, int64_t hi, int t) {
            for (int64_t j = lo; j < hi; ++j) {
                const LongRow &lr = long_rows[j];
                const Level &L = *lr.L;
                const int64_t nf = far_count(L, lr.q, lr.map, lr.r0);
                if (nf < kWindowRow) continue;
                for (int64_t e = L.row_ptr[lr.q]; e < L.row_ptr[lr.q + 1]; ++e) {
                    const int64_t c = lr.map ? pos0[L.vop[L.col[e]]] : L.col[e];
                    if (is_far(c, lr.r0)) __atomic_fetch_add(&cnt[c + 1], (int64_t)1, __ATOMIC_RELAXED);
                }
                tot_t[t] += nf;
            }
        });
        int64_t tot = 0;
        for (int64_t x : tot_t) tot += x;
        for (int64_t c = 0; c < n; ++c) cnt[c + 1] += cnt[c];
        win_lo[0] = 0;
        int64_t c = 0;
        for (int w = 1; w < kChunkWindows; ++w) {
            const int64_t target = (tot * w + kChunkWindows - 1) / kChunkWindows;
            while (c < n && cnt[c] < target) ++c;
            win_lo[w] = c;
        }
    }
    auto window_of = [&](int64_t c) -> int {
        return (int)(std::upper_bound(win_lo.begin() + 1, win_lo.end() - 1, c) -
                     (win_lo.begin() + 1));
    };
    auto &ch_ptr = h.ch_ptr, &ch_col = h.ch_col;
    auto &ch_val = h.ch_val;
    ch_ptr.assign(1, 0);
    std::vector<int16_t> ch_group;  // window of a chunk, kChunkWindows = not windowed
    std::vector<int32_t> l0_chunk_first(n, -1), l0_chunk_count(n, 0);
    std::vector<std::pair<int32_t, int32_t>> up_chunks(p.n_up, {-1, 0});
    // The chunked rows (level-0 rows by position, then upper rows in order),
    // each cut into chunks on its own (threads take rows in turn), then
    // appended in that order.
    struct ChunkRow {
        const Level *L;
        int64_t q, r0;
        bool map;
        int64_t up_row;  // upper row, or -1 for a level-0 row
        std::vector<int32_t> col, len;  // columns in chunk order, chunk lengths
        std::vector<float> val;
        std::vector<int16_t> group;
    };
    std::vector<ChunkRow> crows;
    for (int64_t r = 0; r < n; ++r)
        if (chunked0[r]) crows.push_back({&L0, r, r, false, -1, {}, {}, {}, {}});
    for (int64_t s = 0; s < p.n_up; ++s) {
        const Level &L = d.levels[up[s].level];
        const int64_t q = up[s].pos;
        if (L.row_ptr[q + 1] - L.row_ptr[q] > kLongRow)
            crows.push_back({&L, q, (int64_t)pos0[L.vop[q]], true, s, {}, {}, {}, {}});
    }
    {
        // a row's entries by (group, column), cut into chunks of at most
        // kChunk entries within a group, ascending column
        std::atomic<size_t> next{0};
        par_each(nt, [&](int) {
            std::vector<std::pair<int64_t, int64_t>> ents;  // (group * n + column, entry)
            for (size_t j; (j = next.fetch_add(1)) < crows.size();) {
                ChunkRow &cr = crows[j];
                const Level &L = *cr.L;
                const int64_t e0 = L.row_ptr[cr.q], e1 = L.row_ptr[cr.q + 1];
                const bool split = far_count(L, cr.q, cr.map, cr.r0) >= kWindowRow;
                ents.clear();
                for (int64_t e = e0; e < e1; ++e) {
                    const int64_t c = cr.map ? pos0[L.vop[L.col[e]]] : L.col[e];
                    const int64_t g = split && is_far(c, cr.r0) ? window_of(c) : kChunkWindows;
                    ents.push_back({g * n + c, e});
                }
                std::stable_sort(ents.begin(), ents.end(),
                                 [](const std::pair<int64_t, int64_t> &x,
                                    const std::pair<int64_t, int64_t> &y) { return x.first < y.first; });
                for (size_t i = 0; i < ents.size();) {
                    const int64_t g = ents[i].first / n;
                    size_t k = i;
                    while (k < ents.size() && k - i < (size_t)kChunk && ents[k].first / n == g) ++k;
                    for (size_t u = i; u < k; ++u) {
                        cr.col.push_back((int32_t)(ents[u].first % n));
                        cr.val.push_back(L.val[ents[u].second]);
                    }
                    cr.len.push_back((int32_t)(k - i));
                    cr.group.push_back((int16_t)g);
                    i = k;
                }
            }
        });
        for (size_t j = 0; j < crows.size(); ++j) {
            ChunkRow &cr = crows[j];
            const int32_t first = (int32_t)(ch_ptr.size() - 1);
            ch_col.insert(ch_col.end(), cr.col.begin(), cr.col.end());
            ch_val.insert(ch_val.end(), cr.val.begin(), cr.val.end());
            for (size_t c = 0; c < cr.len.size(); ++c) {
                ch_ptr.push_back(ch_ptr.back() + cr.len[c]);
                ch_group.push_back(cr.group[c]);
            }
            const int32_t count = (int32_t)cr.len.size();
            if (cr.up_row < 0) {
                l0_chunk_first[cr.q] = first;
                l0_chunk_count[cr.q] = count;
            } else {
                up_chunks[cr.up_row] = {first, count};
            }
            ++p.chunked_rows;
            std::vector<int32_t>().swap(cr.col);
            std::vector<float>().swap(cr.val);
        }
    }
    auto &l0_ptr = h.l0_ptr;
    auto &l0_code = h.l0_code;
    auto &l0_col = h.l0_col;
    auto &l0_val = h.l0_val;
    auto &far_ptr = h.far_ptr, &far_col = h.far_col;
    std::vector<uint8_t> seen_l0(n, 0), seen_up(n, 0), seen_ch(n, 0);
    auto mark = [](std::vector<uint8_t> &seen, int64_t c) {
        __atomic_store_n(&seen[c], (uint8_t)1, __ATOMIC_RELAXED);
    };
    // level-0 rows: entry counts per row and far-table counts per block,
    // then every block's codes (or columns), values and far table in parallel
    const int64_t nblk0 = nblocks_of(n, rpb0);
    l0_ptr.assign(n + 1, 0);
    far_ptr.assign(nblk0 + 1, 0);
    par_for(nt, nblk0, [&](int64_t lo, int64_t hi, int) {
        for (int64_t blk = lo; blk < hi; ++blk) {
            int64_t nf = 0;
            for (int64_t r = blk * rpb0; r < std::min<int64_t>(n, (blk + 1) * rpb0); ++r) {
                if (chunked0[r]) continue;
                int64_t len = L0.row_ptr[r + 1] - L0.row_ptr[r];
                if (p.code16) nf += head_far(r);
                for (int64_t si = vrow_ptr[r]; si < vrow_ptr[r + 1]; ++si)
                    if (fused[si]) {
                        len += up_len(vrows[si]);
                        if (p.code16) nf += up_len(vrows[si]);
                    }
                l0_ptr[r + 1] = (int32_t)len;
            }
            far_ptr[blk + 1] = (int32_t)nf;
        }
    });
    for (int64_t r = 0; r < n; ++r) l0_ptr[r + 1] += l0_ptr[r];
    for (int64_t blk = 0; blk < nblk0; ++blk) far_ptr[blk + 1] += far_ptr[blk];
    if (p.code16)
        l0_code.resize(l0_ptr[n]);
    else
        l0_col.resize(l0_ptr[n]);
    l0_val.resize(l0_ptr[n]);
    far_col.resize(far_ptr[nblk0]);
    par_for(nt, nblk0, [&](int64_t lo, int64_t hi, int) {
        for (int64_t blk = lo; blk < hi; ++blk) {
            int64_t f = far_ptr[blk];
            for (int64_t r = blk * rpb0; r < std::min<int64_t>(n, (blk + 1) * rpb0); ++r) {
                if (chunked0[r]) continue;
                int64_t o = l0_ptr[r];
                for (int64_t e = L0.row_ptr[r]; e < L0.row_ptr[r + 1]; ++e, ++o) {
                    const int64_t q = L0.col[e];
                    if (p.code16 && q > r + b) {  // a head row's column beyond the band
                        l0_code[o] = (uint16_t)(3 * (int64_t)b + 1 + (f - far_ptr[blk]));
                        far_col[f++] = (int32_t)q;
                    } else if (p.code16) {
                        const int64_t code = q >= r - b ? q - r + b : 2 * b + 1 + q;
                        l0_code[o] = (uint16_t)code;
                    } else {
                        l0_col[o] = (int32_t)q;
                    }
                    l0_val[o] = L0.val[e];
                    mark(seen_l0, q);
                }
                for (int64_t si = vrow_ptr[r]; si < vrow_ptr[r + 1]; ++si) {
                    if (!fused[si]) continue;
                    const Level &L = d.levels[vrows[si].level];
                    const int64_t q = vrows[si].pos;
                    for (int64_t e = L.row_ptr[q]; e < L.row_ptr[q + 1]; ++e, ++o) {
                        const int32_t c = pos0[L.vop[L.col[e]]];
                        if (p.code16) {
                            l0_code[o] = (uint16_t)(3 * (int64_t)b + 1 + (f - far_ptr[blk]));
                            far_col[f++] = c;
                        } else {
                            l0_col[o] = c;
                        }
                        l0_val[o] = L.val[e];
                        mark(seen_l0, c);
                    }
                }
            }
        }
    });
    p.l0_nfar = (int64_t)far_col.size();
    // upper rows that are not chunked: columns mapped to level-0 positions
    auto &up_ptr = h.up_ptr, &up_col = h.up_col, &up_cptr = h.up_cptr, &up_cidx = h.up_cidx;
    auto &up_val = h.up_val;
    up_ptr.assign(p.n_up + 1, 0);
    up_cptr.assign(p.n_up + 1, 0);
    for (int64_t s = 0; s < p.n_up; ++s) {
        const int64_t len = up_len(up[s]);
        up_ptr[s + 1] = up_ptr[s] + (int32_t)(len > kLongRow ? 0 : len);
    }
    up_col.resize(up_ptr[p.n_up]);
    up_val.resize(up_ptr[p.n_up]);
    par_for(nt, p.n_up, [&](int64_t lo, int64_t hi, int) {
        for (int64_t s = lo; s < hi; ++s) {
            if (up_ptr[s + 1] == up_ptr[s]) continue;
            const Level &L = d.levels[up[s].level];
            const int64_t q = up[s].pos;
            int64_t o = up_ptr[s];
            for (int64_t e = L.row_ptr[q]; e < L.row_ptr[q + 1]; ++e, ++o) {
                const int32_t c = pos0[L.vop[L.col[e]]];
                up_col[o] = c;
                up_val[o] = L.val[e];
                mark(seen_up, c);
            }
        }
    });
    p.n_chunks = (int64_t)ch_ptr.size() - 1;
    // Chunk placement.  Workgroup w of the chunk pass runs on XCD w % kXcds
    // (dispatch is round-robin over the XCDs) and takes kChunksPerBlock
    // consecutive chunk slots (a unit).  XCD x gets the units of the windows
    // w = x, x + kXcds, ... (in that order), then every kXcds-th unit of the
    // other chunks, so each XCD's L2 holds the hot X rows of its own windows.
    // Within a group the chunks run in order of their first column.  Slots an
    // XCD does not fill stay empty (no entries, no partial row).  Only the
    // storage moves: chunk c's partial row sits at n_up + chunk_slot[c] and
    // every list keeps its order, so the sums do not depend on the placement.
    std::vector<int32_t> chunk_slot(p.n_chunks);
    {
        std::vector<std::vector<int32_t>> grp(kChunkWindows + 1);
        for (int64_t c = 0; c < p.n_chunks; ++c) grp[ch_group[c]].push_back((int32_t)c);
        // (groups sorted in parallel, on (first column, chunk) keys)
        std::atomic<int> next_g{0};
        par_each(std::min(nt, kChunkWindows + 1), [&](int) {
            std::vector<std::pair<int32_t, int32_t>> key;
            for (int w; (w = next_g.fetch_add(1)) <= kChunkWindows;) {
                std::vector<int32_t> &g = grp[w];
                key.resize(g.size());
                for (size_t i = 0; i < g.size(); ++i) key[i] = {ch_col[ch_ptr[g[i]]], g[i]};
                std::stable_sort(key.begin(), key.end(),
                                 [](const std::pair<int32_t, int32_t> &x,
                                    const std::pair<int32_t, int32_t> &y) { return x.first < y.first; });
                for (size_t i = 0; i < g.size(); ++i) g[i] = key[i].second;
            }
        });
        constexpr int U = kChunksPerBlock;
        std::vector<std::vector<std::pair<size_t, int>>> xcd_units(kXcds);  // (group, first)
        for (int w = 0; w <= kChunkWindows; ++w)
            for (size_t i = 0; i < grp[w].size(); i += U) {
                const int x = w < kChunkWindows ? w % kXcds : (int)((i / U) % kXcds);
                xcd_units[x].push_back({(size_t)w, (int)i});
            }
        size_t per_xcd = 0;
        for (auto &v : xcd_units) per_xcd = std::max(per_xcd, v.size());
        p.ch_slots = (int64_t)per_xcd * kXcds * U;
        std::vector<int32_t> slot_chunk(p.ch_slots, -1);
        for (int x = 0; x < kXcds; ++x)
            for (size_t j = 0; j < xcd_units[x].size(); ++j) {
                const std::vector<int32_t> &g = grp[xcd_units[x][j].first];
                const size_t i0 = (size_t)xcd_units[x][j].second;
                for (size_t i = i0; i < std::min(g.size(), i0 + U); ++i)
                    slot_chunk[(j * kXcds + x) * U + (i - i0)] = g[i];
            }
        std::vector<int32_t> nptr(p.ch_slots + 1, 0), ncol(ch_col.size());
        std::vector<float> nval(ch_val.size());
        for (int64_t slot = 0; slot < p.ch_slots; ++slot) {
            const int32_t c = slot_chunk[slot];
            nptr[slot + 1] = nptr[slot] + (c >= 0 ? ch_ptr[c + 1] - ch_ptr[c] : 0);
            if (c >= 0) chunk_slot[c] = (int32_t)slot;
        }
        par_for(nt, p.ch_slots, [&](int64_t lo, int64_t hi, int) {
            for (int64_t slot = lo; slot < hi; ++slot) {
                const int32_t c = slot_chunk[slot];
                if (c < 0) continue;
                std::copy(ch_col.begin() + ch_ptr[c], ch_col.begin() + ch_ptr[c + 1],
                          ncol.begin() + nptr[slot]);
                std::copy(ch_val.begin() + ch_ptr[c], ch_val.begin() + ch_ptr[c + 1],
                          nval.begin() + nptr[slot]);
            }
        });
        ch_ptr.swap(nptr);
        ch_col.swap(ncol);
        ch_val.swap(nval);
    }
    p.s_rows = p.n_up + p.ch_slots;
    for (int32_t c : ch_col) seen_ch[c] = 1;
    // partial rows listed by the upper rows: their own chunks
    for (int64_t s = 0; s < p.n_up; ++s) {
        for (int32_t c = 0; c < up_chunks[s].second; ++c)
            up_cidx.push_back((int32_t)(p.n_up + chunk_slot[up_chunks[s].first + c]));
        up_cptr[s + 1] = (int32_t)up_cidx.size();
    }
    // partial rows listed by the level-0 rows: own chunks, then the upper rows
    // of the same vertex by level
    auto &l0_cptr = h.l0_cptr, &l0_cidx = h.l0_cidx;
    l0_cptr.assign(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t c = 0; c < l0_chunk_count[r]; ++c)
            l0_cidx.push_back((int32_t)(p.n_up + chunk_slot[l0_chunk_first[r] + c]));
        for (int64_t si = vrow_ptr[r]; si < vrow_ptr[r + 1]; ++si)
            if (!fused[si]) l0_cidx.push_back((int32_t)up_of[si]);
        l0_cptr[r + 1] = (int32_t)l0_cidx.size();
    }
    // long lists go to the combine pass, in units of at most kCombineUnit
    // partial rows: such a row lists its units' sums
    {
        auto &hv_ptr = h.hv_ptr, &hv_idx = h.hv_idx;
        hv_ptr.assign(1, 0);
        std::vector<int32_t> cptr(n + 1, 0), cidx;
        cidx.reserve(l0_cidx.size());
        const int64_t row0 = p.n_up + p.ch_slots;
        for (int64_t r = 0; r < n; ++r) {
            const int32_t c0 = l0_cptr[r], c1 = l0_cptr[r + 1];
            const int64_t len = c1 - c0;
            if (len > kCombineList) {
                const int64_t nu = (len + kCombineUnit - 1) / kCombineUnit;
                for (int64_t u = 0; u < nu; ++u) {
                    cidx.push_back((int32_t)(row0 + (int64_t)hv_ptr.size() - 1));
                    hv_idx.insert(hv_idx.end(), l0_cidx.begin() + c0 + len * u / nu,
                                  l0_cidx.begin() + c0 + len * (u + 1) / nu);
                    hv_ptr.push_back((int32_t)hv_idx.size());
                }
            } else {
                cidx.insert(cidx.end(), l0_cidx.begin() + c0, l0_cidx.begin() + c1);
            }
            cptr[r + 1] = (int32_t)cidx.size();
        }
        p.n_heavy = (int64_t)hv_ptr.size() - 1;
        p.hv_nlist = (int64_t)hv_idx.size();
        p.s_rows += p.n_heavy;
        if (p.n_heavy == 0) {
            hv_ptr.clear();
        } else {
            l0_cptr.swap(cptr);
            l0_cidx.swap(cidx);
        }
    }
    p.l0_batch = p.l0_batch_auto = choose_batch<int32_t>(n, l0_ptr.data(), l0_cptr.data());
    p.up_batch = p.up_batch_auto =
        choose_batch<int32_t>(p.n_up, up_ptr.data(), up_cptr.data());
    // Passes of mixed row lengths (wide batch): process each block's rows
    // longest first, so the row groups of a wave get rows of similar length
    // (a wave waits for its longest row).  Only the schedule changes.
    auto block_order = [&](int64_t rows, int64_t rpb, const std::vector<int32_t> &ptr,
                           const std::vector<int32_t> &cptr) {
        std::vector<uint8_t> ord(rows);
        std::vector<int32_t> idx;
        for (int64_t r0 = 0; r0 < rows; r0 += rpb) {
            const int64_t nr = std::min<int64_t>(rpb, rows - r0);
            idx.resize(nr);
            for (int64_t i = 0; i < nr; ++i) idx[i] = (int32_t)i;
            auto work = [&](int32_t i) {
                const int64_t r = r0 + i;
                return (int64_t)(ptr[r + 1] - ptr[r]) + 2 * (int64_t)(cptr[r + 1] - cptr[r]);
            };
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int32_t x, int32_t y) { return work(x) > work(y); });
            for (int64_t i = 0; i < nr; ++i) ord[r0 + i] = (uint8_t)idx[i];
        }
        return ord;
    };
    // per-block entry / list offsets (the row offsets at the block starts)
    auto block_offsets = [&](int64_t rows, int64_t rpb, const std::vector<int32_t> &ptr) {
        std::vector<int32_t> o;
        for (int64_t r0 = 0; r0 < rows; r0 += rpb) o.push_back(ptr[r0]);
        o.push_back(ptr[rows]);
        return o;
    };
    h.l0_blk_e = block_offsets(n, rpb0, l0_ptr);
    h.l0_blk_c = block_offsets(n, rpb0, l0_cptr);
    auto &up_blk_e = h.up_blk_e, &up_blk_c = h.up_blk_c;
    if (p.n_up > 0) {
        up_blk_e = block_offsets(p.n_up, kRowsPerBlock, up_ptr);
        up_blk_c = block_offsets(p.n_up, kRowsPerBlock, up_cptr);
    }
    auto &l0_order = h.l0_order, &up_order = h.up_order;
    if (p.l0_batch_auto == kBatchWide) l0_order = block_order(n, rpb0, l0_ptr, l0_cptr);
    if (p.up_batch_auto == kBatchWide && p.n_up > 0)
        up_order = block_order(p.n_up, kRowsPerBlock, up_ptr, up_cptr);
    p.l0_nnz = (int64_t)l0_val.size();
    p.l0_ncontrib = (int64_t)l0_cidx.size();
    p.up_nnz = (int64_t)up_val.size();
    p.up_ncontrib = (int64_t)up_cidx.size();
    p.ch_nnz = (int64_t)ch_val.size();
    p.distinct_l0 = count_true(seen_l0);
    p.distinct_up = count_true(seen_up);
    p.distinct_ch = count_true(seen_ch);
}

arrow_status_t plan_create(const Decomp &d, int device, hipStream_t stream, Plan *&out) {
    out = nullptr;
    Plan *pp = new (std::nothrow) Plan();
    if (!pp) {
        set_error("host allocation of the plan failed");
        return ARROW_ERR_OUT_OF_MEMORY;
    }
    Plan &p = *pp;
    p.device = device;
    p.allocator = g_allocator;
    PlanArrays h;
    plan_build(d, p, h);
    const Level &L0 = d.levels[0];

    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        set_error(std::string("hipSetDevice: ") + hipGetErrorString(e));
        delete pp;
        return ARROW_ERR_HIP;
    }
    arrow_status_t st = ARROW_OK;
#define UP(dst, src)                                \
    if (st == ARROW_OK) st = upload(p, dst, src, stream);
    UP(p.l0_ptr, h.l0_ptr);
    if (p.code16) {
        uint16_t *codes = nullptr;
        UP(codes, h.l0_code);
        p.l0_idx = codes;
    } else {
        int32_t *cols = nullptr;
        UP(cols, h.l0_col);
        p.l0_idx = cols;
    }
    UP(p.l0_val, h.l0_val);
    UP(p.l0_cptr, h.l0_cptr);
    UP(p.l0_cidx, h.l0_cidx);
    UP(p.l0_order, h.l0_order);
    UP(p.up_order, h.up_order);
    UP(p.l0_blk_e, h.l0_blk_e);
    UP(p.l0_blk_c, h.l0_blk_c);
    UP(p.up_blk_e, h.up_blk_e);
    UP(p.up_blk_c, h.up_blk_c);
    if (p.l0_nfar > 0) {
        UP(p.l0_fptr, h.far_ptr);
        UP(p.l0_fcol, h.far_col);
    }
    UP(p.up_ptr, h.up_ptr);
    UP(p.up_col, h.up_col);
    UP(p.up_val, h.up_val);
    UP(p.up_cptr, h.up_cptr);
    UP(p.up_cidx, h.up_cidx);
    UP(p.ch_ptr, h.ch_ptr);
    UP(p.ch_col, h.ch_col);
    UP(p.ch_val, h.ch_val);
    UP(p.vop0, L0.vop);
    if (p.n_heavy > 0) {
        UP(p.hv_ptr, h.hv_ptr);
        UP(p.hv_idx, h.hv_idx);
    }
#undef UP
    if (st == ARROW_OK) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error(std::string("plan upload: ") + hipGetErrorString(e));
            st = ARROW_ERR_HIP;
        }
    }
    if (st != ARROW_OK) {
        plan_destroy(pp);
        return st;
    }
    out = pp;
    return ARROW_OK;
}

void plan_destroy(Plan *p) {
    if (!p) return;
    hipSetDevice(p->device);
    for (void *a : p->allocs) {
        if (p->allocator.free)
            p->allocator.free(a, nullptr, p->allocator.ctx);
        else
            hipFree(a);
    }
    for (const ProfRec &r : p->prof_recs) {
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    for (hipEvent_t ev : p->ev_pool) hipEventDestroy(ev);
    delete p;
}

size_t op_workspace(const Plan &p, int64_t k, int dtype) {
    const int64_t nb = final_parts(p, dtype);
    return align256((size_t)p.s_rows * k * 4) + align256((size_t)k * nb * 8) +
           align256((size_t)k * nb * 4);
}

namespace {

hipEvent_t pool_event(Plan &p) {
    if (!p.ev_pool.empty()) {
        hipEvent_t ev = p.ev_pool.back();
        p.ev_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
}

struct ProfScope {
    Plan &p;
    int kernel;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(Plan &pl, int k, hipStream_t st) : p(pl), kernel(k), s(st) {
        if (!p.prof || p.prof_recs.size() >= 200000) return;
        a = pool_event(p);
        b = pool_event(p);
        if (a && b) hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (a && b) {
            hipEventRecord(b, s);
            p.prof_recs.push_back({kernel, a, b, s});
        }
    }
};

#define LAUNCH_OK(expr)                                                            \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error(std::string("kernel launch: ") + hipGetErrorString(e_));     \
            return ARROW_ERR_HIP;                                                  \
        }                                                                          \
    } while (0)

}  // namespace

arrow_status_t spmm_group(Plan &p, const OpState *ops, int nops, void *const *wss,
                          hipStream_t s) {
    const int64_t n = p.n;
    if (n == 0 || nops == 0) return ARROW_OK;
    const int dtype = ops[0].dtype;
    const int kt = tile_width(ops[0].k);
    const int64_t es = elem_size(dtype);
    const int64_t nb = final_parts(p, dtype);

    RowPass ch{};
    set_geometry(ch, p.ch_slots, kChunksPerBlock, 1);
    ch.ptr = p.ch_ptr;
    ch.idx = p.ch_col;
    ch.val = p.ch_val;
    ch.b = p.b;
    ch.out_row0 = (int32_t)p.n_up;
    ch.batch = kBatchWide;

    RowPass upp{};
    set_geometry(upp, p.n_up, kRowsPerBlock, kBlocksPerWg);
    upp.ptr = p.up_ptr;
    upp.idx = p.up_col;
    upp.val = p.up_val;
    upp.cptr = p.up_cptr;
    upp.cidx = p.up_cidx;
    upp.lists = p.up_ncontrib > 0;
    upp.order = p.up_order;
    upp.blk_e = p.up_batch != kBatchWide ? p.up_blk_e : nullptr;
    upp.blk_c = p.up_batch != kBatchWide ? p.up_blk_c : nullptr;
    upp.b = p.b;
    upp.out_row0 = 0;
    upp.batch = p.up_batch;

    RowPass l0{};
    set_geometry(l0, n, p.l0_rpb, l0_blocks_per_wg(dtype));
    l0.ptr = p.l0_ptr;
    l0.idx = p.l0_idx;
    l0.val = p.l0_val;
    l0.cptr = p.l0_cptr;
    l0.cidx = p.l0_cidx;
    l0.lists = p.l0_ncontrib > 0;
    l0.order = p.l0_order;
    // one-round-trip staging for the short batches (measured: a little faster
    // on the grids, a little slower on the wide R-MAT pass)
    l0.blk_e = p.l0_batch != kBatchWide ? p.l0_blk_e : nullptr;
    l0.blk_c = p.l0_batch != kBatchWide ? p.l0_blk_c : nullptr;
    l0.fptr = p.l0_fptr;
    l0.fcol = p.l0_fcol;
    l0.b = p.b;
    l0.batch = p.l0_batch;

    // every column tile of every operand; launches take up to kMaxTiles each
    std::vector<Tile> tiles;
    for (int o = 0; o < nops; ++o) {
        const OpState &op = ops[o];
        const int64_t k = op.k;
        char *w = static_cast<char *>(wss[o]);
        float *sbuf = reinterpret_cast<float *>(w);
        w += align256((size_t)p.s_rows * k * 4);
        double *psum = reinterpret_cast<double *>(w);
        w += align256((size_t)k * nb * 8);
        float *pmax = reinterpret_cast<float *>(w);
        for (int64_t c0 = 0; c0 < k; c0 += kt) {
            Tile t{};
            t.x = static_cast<const char *>(op.x) + c0 * es;
            t.ldx = op.ldx;
            t.x_span = ((n - 1) * op.ldx + kt) * es;
            t.s = sbuf + c0;
            t.s_out = sbuf + c0;
            t.lds = k;
            t.s_span = (p.s_rows * k - c0) * 4;
            t.y = static_cast<char *>(op.y) + c0 * es;
            t.ldy = op.ldy;
            t.x_scale = op.x_scale ? op.x_scale + c0 : nullptr;
            t.x_inv_norm = op.x_inv_norm ? op.x_inv_norm + c0 : nullptr;
            t.x_maxabs = op.x_maxabs ? op.x_maxabs + c0 : nullptr;
            t.y_scale = op.y_scale ? op.y_scale + c0 : nullptr;
            t.part_sumsq = psum + c0 * nb;
            t.part_max = pmax + c0 * nb;
            t.part_ld = nb;
            t.a_inf = (float)p.a_inf;
            t.w = op.w;  // only with one tile per operand (k = tile width)
            tiles.push_back(t);
        }
    }
    for (size_t t0 = 0; t0 < tiles.size(); t0 += kMaxTiles) {
        TileSet ts{};
        ts.n = (int32_t)std::min<size_t>(kMaxTiles, tiles.size() - t0);
        for (int i = 0; i < ts.n; ++i) ts.t[i] = tiles[t0 + i];
        if (p.n_chunks > 0) {
            ProfScope ps(p, ARROW_KERNEL_CHUNKS, s);
            LAUNCH_OK(launch_row_pass(kt, dtype, kPassChunk, false, ch, ts, s));
        }
        if (p.n_up > 0) {
            ProfScope ps(p, ARROW_KERNEL_UPPER, s);
            LAUNCH_OK(launch_row_pass(kt, dtype, kPassUpper, false, upp, ts, s));
        }
        if (p.n_heavy > 0) {
            ProfScope ps(p, ARROW_KERNEL_COMBINE, s);
            CombineArgs ca{p.hv_ptr, p.hv_idx, p.n_heavy, p.n_up + p.ch_slots};
            LAUNCH_OK(launch_combine(kt, ca, ts, s));
        }
        {
            ProfScope ps(p, ARROW_KERNEL_LEVEL0, s);
            LAUNCH_OK(launch_row_pass(kt, dtype, kPassLevel0, p.code16, l0, ts, s));
        }
    }
    for (int o = 0; o < nops; ++o) {
        const OpState &op = ops[o];
        if (!(op.y_norm || op.y_inv_norm || op.y_maxabs)) continue;
        char *w = static_cast<char *>(wss[o]) + align256((size_t)p.s_rows * op.k * 4);
        NormArgs na{};
        na.part_sumsq = reinterpret_cast<double *>(w);
        na.part_max = op.y_maxabs ? reinterpret_cast<float *>(w + align256((size_t)op.k * nb * 8))
                                  : nullptr;
        na.part_ld = nb;
        na.nparts = (int32_t)nb;
        na.norm = op.y_norm;
        na.inv_norm = op.y_inv_norm;
        na.maxabs = op.y_maxabs;
        ProfScope ps(p, ARROW_KERNEL_NORM, s);
        LAUNCH_OK(launch_norm(na, (int)op.k, s));
    }
    return ARROW_OK;
}

arrow_status_t spmm_one(Plan &p, const OpState &op, void *ws, hipStream_t s) {
    return spmm_group(p, &op, 1, &ws, s);
}

int64_t kernel_bytes(const Plan &p, int kernel, int64_t k, int dtype) {
    const int64_t sx = elem_size(dtype);
    const int64_t nb = final_parts(p, dtype);
    const bool scaled = dtype == kF16 || dtype == kF8E4M3;
    switch (kernel) {
    case ARROW_KERNEL_CHUNKS:
        if (p.n_chunks == 0) return 0;
        return p.ch_nnz * 8 + (p.ch_slots + 1) * 4 + p.distinct_ch * k * sx + p.n_chunks * k * 4;
    case ARROW_KERNEL_UPPER:
        if (p.n_up == 0) return 0;
        return p.up_nnz * 8 + (p.n_up + 1) * 8 + (p.up_order ? p.n_up : 0) +
               (p.up_batch != kBatchWide ? (nblocks_of(p.n_up, kRowsPerBlock) + 1) * 8 : 0) +
               p.up_ncontrib * (4 + k * 4) +
               p.distinct_up * k * sx + p.n_up * k * 4;
    case ARROW_KERNEL_LEVEL0:
        // row offsets, plus list offsets unless no row lists a partial row
        // (a short-batch pass then skips them)
        return p.l0_nnz * ((p.code16 ? 2 : 4) + 4) +
               (p.n + 1) * (p.l0_ncontrib > 0 || p.l0_batch == kBatchWide ? 8 : 4) +
               (p.l0_order ? p.n : 0) +
               (p.l0_batch != kBatchWide ? (nblocks_of(p.n, p.l0_rpb) + 1) * 8 : 0) +
               (p.l0_nfar > 0 ? p.l0_nfar * 4 + (nblocks_of(p.n, p.l0_rpb) + 1) * 4 : 0) +
               p.l0_ncontrib * (4 + k * 4) + p.distinct_l0 * k * sx + p.n * k * sx +
               nb * k * (8 + (scaled ? 4 : 0)) + k * (scaled ? 16 : 8);
    case ARROW_KERNEL_NORM:
        return nb * k * (8 + (scaled ? 4 : 0)) + k * 16;
    case ARROW_KERNEL_PERMUTE:
        return p.n * 4 + p.n * k * (4 + sx);
    case ARROW_KERNEL_COMBINE:
        if (p.n_heavy == 0) return 0;
        return (p.n_heavy + 1) * 4 + p.hv_nlist * (4 + k * 4) + p.n_heavy * k * 4;
    default:
        return -1;
    }
}

size_t plain_csr_workspace(int64_t n, int64_t k) {
    const int64_t nb = final_parts(n, kRowsPerBlock);
    return align256((size_t)k * nb * 8);
}

arrow_status_t plain_csr(int64_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                         const float *x, float *y, int64_t k, int64_t ld, int32_t batch,
                         double *ws, double *norms, hipStream_t s) {
    if (n == 0) return ARROW_OK;
    const int kt = tile_width(k);
    const int64_t nb = final_parts(n, kRowsPerBlock);
    RowPass rp{};
    set_geometry(rp, n, kRowsPerBlock, kBlocksPerWg);
    rp.ptr = row_ptr;
    rp.idx = col;
    rp.val = val;
    rp.b = 0;
    rp.batch = batch;
    for (int64_t c0 = 0; c0 < k; c0 += kt) {
        Tile t{};
        t.x = x + c0;
        t.ldx = ld;
        t.x_span = ((n - 1) * ld + kt) * 4;
        t.y = y + c0;
        t.ldy = ld;
        t.part_sumsq = ws ? ws + c0 * nb : nullptr;
        t.part_ld = nb;
        TileSet ts{};
        ts.t[0] = t;
        ts.n = 1;
        LAUNCH_OK(launch_row_pass(kt, kF32, kPassPlain, false, rp, ts, s));
    }
    if (ws && norms) {
        NormArgs na{};
        na.part_sumsq = ws;
        na.part_ld = nb;
        na.nparts = (int32_t)nb;
        na.norm = norms;
        LAUNCH_OK(launch_norm(na, (int)k, s));
    }
    return ARROW_OK;
}

}  // namespace arrow
