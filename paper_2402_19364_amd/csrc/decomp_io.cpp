// Save / load of a decomposition: versioned little-endian binary with an
// FNV-1a 64-bit checksum of everything before the trailer.
//
// Layout: "ARWDEC01" | u32 version | u32 0 | i64 n | i64 nnz | i32 b | i32 la |
//         u64 seed | i32 levels | i32 0 | per level: i64 n_i | i64 nnz_i |
//         i32 vop[n_i] | i64 row_ptr[n_i+1] | i32 col[nnz_i] | f32 val[nnz_i] |
//         u64 checksum
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace arrow {
namespace {

constexpr char kMagic[8] = {'A', 'R', 'W', 'D', 'E', 'C', '0', '1'};
constexpr uint32_t kVersion = 1;

struct Writer {
    FILE *f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void put(const void *p, size_t bytes) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < bytes; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
        if (bytes && fwrite(p, 1, bytes, f) != bytes) ok = false;
    }
    template <class T> void pod(const T &v) { put(&v, sizeof(T)); }
};

struct Reader {
    FILE *f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void get(void *p, size_t bytes) {
        if (!ok) return;
        if (bytes && fread(p, 1, bytes, f) != bytes) {
            ok = false;
            return;
        }
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < bytes; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    }
    template <class T> void pod(T &v) { get(&v, sizeof(T)); }
};

}  // namespace

arrow_status_t save_decomp(const Decomp &d, const char *path) {
    FILE *f = fopen(path, "wb");
    if (!f) {
        set_error(std::string("cannot open for writing: ") + path);
        return ARROW_ERR_IO;
    }
    Writer w{f};
    w.put(kMagic, 8);
    w.pod(kVersion);
    w.pod(uint32_t(0));
    w.pod(d.n);
    w.pod(d.nnz);
    w.pod(d.b);
    w.pod(d.la);
    w.pod(d.seed);
    w.pod(int32_t(d.levels.size()));
    w.pod(int32_t(0));
    for (const Level &L : d.levels) {
        w.pod(L.n_i);
        w.pod(int64_t(L.col.size()));
        w.put(L.vop.data(), L.vop.size() * sizeof(int32_t));
        w.put(L.row_ptr.data(), L.row_ptr.size() * sizeof(int64_t));
        w.put(L.col.data(), L.col.size() * sizeof(int32_t));
        w.put(L.val.data(), L.val.size() * sizeof(float));
    }
    uint64_t h = w.h;
    bool ok = w.ok && fwrite(&h, sizeof(h), 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok) {
        set_error(std::string("write failed: ") + path);
        return ARROW_ERR_IO;
    }
    return ARROW_OK;
}

arrow_status_t load_decomp(const char *path, Decomp &out) {
    FILE *f = fopen(path, "rb");
    if (!f) {
        set_error(std::string("cannot open: ") + path);
        return ARROW_ERR_IO;
    }
    Reader r{f};
    Decomp d;
    char magic[8];
    uint32_t version = 0, pad = 0;
    int32_t nlev = 0, pad2 = 0;
    r.get(magic, 8);
    r.pod(version);
    r.pod(pad);
    r.pod(d.n);
    r.pod(d.nnz);
    r.pod(d.b);
    r.pod(d.la);
    r.pod(d.seed);
    r.pod(nlev);
    r.pod(pad2);
    auto fail = [&](const char *why) {
        fclose(f);
        set_error(std::string("corrupt decomposition file (") + why + "): " + path);
        return ARROW_ERR_IO;
    };
    if (!r.ok || memcmp(magic, kMagic, 8) != 0) return fail("magic");
    if (version != kVersion) return fail("version");
    if (d.n < 0 || d.nnz < 0 || nlev < 1 || nlev > 4096 || d.b < 2) return fail("header");
    int64_t total = 0;
    for (int32_t i = 0; i < nlev && r.ok; ++i) {
        Level L;
        int64_t nnz_i = 0;
        r.pod(L.n_i);
        r.pod(nnz_i);
        if (!r.ok || L.n_i < 0 || L.n_i > d.n || nnz_i < 0 || nnz_i > d.nnz - total)
            return fail("level header");
        total += nnz_i;
        L.vop.resize(L.n_i);
        L.row_ptr.resize(L.n_i + 1);
        L.col.resize(nnz_i);
        L.val.resize(nnz_i);
        r.get(L.vop.data(), L.vop.size() * sizeof(int32_t));
        r.get(L.row_ptr.data(), L.row_ptr.size() * sizeof(int64_t));
        r.get(L.col.data(), L.col.size() * sizeof(int32_t));
        r.get(L.val.data(), L.val.size() * sizeof(float));
        if (!r.ok) return fail("truncated");
        if (L.row_ptr[0] != 0 || L.row_ptr[L.n_i] != nnz_i) return fail("row pointers");
        for (int64_t p = 0; p < L.n_i; ++p)
            if (L.row_ptr[p + 1] < L.row_ptr[p]) return fail("row pointers");
        for (int64_t p = 0; p < L.n_i; ++p)
            if (L.vop[p] < 0 || L.vop[p] >= d.n) return fail("vertex map");
        {
            // the map of a level is injective (level 0: a permutation of [0, n))
            std::vector<uint8_t> used(d.n, 0);
            for (int64_t p = 0; p < L.n_i; ++p) {
                if (used[L.vop[p]]) return fail("vertex map is not injective");
                used[L.vop[p]] = 1;
            }
        }
        const int64_t b = d.b;
        for (int64_t p = 0; p < L.n_i; ++p)
            for (int64_t e = L.row_ptr[p]; e < L.row_ptr[p + 1]; ++e) {
                const int64_t q = L.col[e];
                if (q < 0 || q >= L.n_i) return fail("column");
                if (e > L.row_ptr[p] && q <= L.col[e - 1]) return fail("columns not increasing");
                // arrow width b (Section 1): head row, head column or the band
                if (!(p < b || q < b || (p > q ? p - q : q - p) <= b))
                    return fail("entry outside the arrow shape");
            }
        d.levels.push_back(std::move(L));
    }
    uint64_t expect = r.h, stored = 0;
    if (fread(&stored, sizeof(stored), 1, f) != 1) return fail("truncated");
    if (stored != expect) return fail("checksum");
    if (total != d.nnz) return fail("entry count");
    if (d.levels[0].n_i != d.n) return fail("level 0 size");
    fclose(f);
    out = std::move(d);
    return ARROW_OK;
}

}  // namespace arrow
