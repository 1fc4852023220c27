// extern "C" boundary of libarrow: argument checks, error reporting, handles.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "arrow.h"
#include "internal.h"
#include "plan.h"

struct arrow_decomp_s {
    arrow::Decomp d;
};
struct arrow_plan_s {
    arrow::Plan *p;
};

namespace arrow {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace arrow

using arrow::set_error;

int arrow::plan_device(arrow_plan_t p) { return p ? p->p->device : -1; }

namespace {

bool valid_dtype(arrow_dtype_t t) { return t >= ARROW_F32 && t <= ARROW_F8E4M3; }
bool scaled(arrow_dtype_t t) { return t == ARROW_F16 || t == ARROW_F8E4M3; }

arrow_status_t check_dense(const void *p, int64_t ld, int64_t k, arrow_dtype_t dt, int64_t rows,
                           const char *what) {
    if (rows > 0 && !p) {
        set_error(std::string(what) + " is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    if (ld < k) {
        set_error(std::string(what) + ": ld must be >= k");
        return ARROW_ERR_INVALID_ARG;
    }
    const int64_t es = arrow::elem_size(dt);
    if ((reinterpret_cast<uintptr_t>(p) % 16) != 0 || (ld * es) % 16 != 0) {
        set_error(std::string(what) + ": base pointer and row stride must be 16-byte aligned");
        return ARROW_ERR_INVALID_ARG;
    }
    return ARROW_OK;
}

arrow_status_t check_k(int64_t k) {
    if (k <= 0 || k % 16 != 0 || k > (1 << 20)) {
        set_error("k must be a positive multiple of 16");
        return ARROW_ERR_INVALID_ARG;
    }
    return ARROW_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

bool overlaps(const void *a, int64_t abytes, const void *b, int64_t bbytes) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

}  // namespace

extern "C" {

const char *arrow_version(void) { return "1.0.0"; }

const char *arrow_last_error(void) { return arrow::g_last_error.c_str(); }

const char *arrow_status_string(arrow_status_t s) {
    switch (s) {
    case ARROW_OK: return "ok";
    case ARROW_ERR_INVALID_ARG: return "invalid argument";
    case ARROW_ERR_OUT_OF_MEMORY: return "out of memory";
    case ARROW_ERR_HIP: return "HIP runtime error";
    case ARROW_ERR_UNSUPPORTED: return "unsupported";
    case ARROW_ERR_IO: return "I/O error";
    case ARROW_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
    }
}

arrow_status_t arrow_decompose(int64_t n, const int64_t *row_ptr, const int32_t *col,
                               const float *val, const arrow_decompose_opts_t *opts,
                               arrow_decomp_t *out) {
    if (!out) {
        set_error("out is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!opts) {
        set_error("opts is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow_decomp_s *h = new (std::nothrow) arrow_decomp_s();
    if (!h) {
        set_error("host allocation failed");
        return ARROW_ERR_OUT_OF_MEMORY;
    }
    arrow_status_t st;
    try {
        st = arrow::decompose(n, row_ptr, col, val, *opts, h->d);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed during decomposition");
        st = ARROW_ERR_OUT_OF_MEMORY;
    }
    if (st != ARROW_OK) {
        delete h;
        return st;
    }
    *out = h;
    return ARROW_OK;
}

arrow_status_t arrow_decomp_info(arrow_decomp_t d, arrow_decomp_info_t *out) {
    if (!d || !out) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    out->n = d->d.n;
    out->nnz = d->d.nnz;
    out->b = d->d.b;
    out->levels = (int32_t)d->d.levels.size();
    out->seconds = d->d.seconds;
    return ARROW_OK;
}

arrow_status_t arrow_decomp_level_stats(arrow_decomp_t d, int32_t level,
                                        arrow_level_stats_t *out) {
    if (!d || !out) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    if (level < 0 || level >= (int32_t)d->d.levels.size()) {
        set_error("level out of range");
        return ARROW_ERR_INVALID_ARG;
    }
    const arrow::Level &L = d->d.levels[level];
    const int64_t b = d->d.b;
    arrow_level_stats_t st{};
    st.n_i = L.n_i;
    st.nnz_i = (int64_t)L.col.size();
    for (int64_t q = 0; q < L.n_i; ++q) {
        const int64_t e0 = L.row_ptr[q], e1 = L.row_ptr[q + 1];
        st.active_rows += e1 > e0;
        for (int64_t e = e0; e < e1; ++e) {
            if (q < b)
                ++st.head_row_nnz;
            else if (L.col[e] < b)
                ++st.head_col_nnz;
            else
                ++st.band_nnz;
        }
    }
    *out = st;
    return ARROW_OK;
}

arrow_status_t arrow_decomp_block_stats(arrow_decomp_t d, int32_t level, int32_t s,
                                        int32_t region, arrow_block_stats_t *out) {
    if (!d || !out) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    if (level < 0 || level >= (int32_t)d->d.levels.size()) {
        set_error("level out of range");
        return ARROW_ERR_INVALID_ARG;
    }
    if (s < 1 || (region != 0 && region != 1)) {
        set_error("block size must be >= 1 and region 0 or 1");
        return ARROW_ERR_INVALID_ARG;
    }
    const arrow::Level &L = d->d.levels[level];
    const int64_t b = d->d.b;
    arrow_block_stats_t st{};
    std::vector<int64_t> cols;
    const double area = (double)s * (double)s;
    for (int64_t r0 = 0; r0 < L.n_i; r0 += s) {
        // block columns of the entries of block row r0 / s, counted by sorting
        cols.clear();
        for (int64_t p = r0; p < std::min<int64_t>(L.n_i, r0 + s); ++p)
            for (int64_t e = L.row_ptr[p]; e < L.row_ptr[p + 1]; ++e) {
                const int64_t q = L.col[e];
                if (region == 1 && !(p < b || q < b)) continue;
                cols.push_back(q / s);
            }
        std::sort(cols.begin(), cols.end());
        st.entries += (int64_t)cols.size();
        for (size_t i = 0; i < cols.size();) {
            size_t j = i;
            while (j < cols.size() && cols[j] == cols[i]) ++j;
            const double dens = (double)(j - i) / area;
            st.max_density = std::max(st.max_density, dens);
            ++st.hist[std::min(9, (int)(dens * 10.0))];
            ++st.nonzero_blocks;
            i = j;
        }
    }
    *out = st;
    return ARROW_OK;
}

arrow_status_t arrow_decomp_level(arrow_decomp_t d, int32_t level, int64_t *n_i, int64_t *nnz_i,
                                  const int32_t **vertex_of_pos, const int64_t **row_ptr,
                                  const int32_t **col, const float **val) {
    if (!d || !n_i || !nnz_i || !vertex_of_pos || !row_ptr || !col || !val) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    if (level < 0 || level >= (int32_t)d->d.levels.size()) {
        set_error("level out of range");
        return ARROW_ERR_INVALID_ARG;
    }
    const arrow::Level &L = d->d.levels[level];
    *n_i = L.n_i;
    *nnz_i = (int64_t)L.col.size();
    *vertex_of_pos = L.vop.data();
    *row_ptr = L.row_ptr.data();
    *col = L.col.data();
    *val = L.val.data();
    return ARROW_OK;
}

arrow_status_t arrow_decomp_save(arrow_decomp_t d, const char *path) {
    if (!d || !path) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    return arrow::save_decomp(d->d, path);
}

arrow_status_t arrow_decomp_load(const char *path, arrow_decomp_t *out) {
    if (!out || !path) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    *out = nullptr;
    arrow_decomp_s *h = new (std::nothrow) arrow_decomp_s();
    if (!h) {
        set_error("host allocation failed");
        return ARROW_ERR_OUT_OF_MEMORY;
    }
    arrow_status_t st;
    try {
        st = arrow::load_decomp(path, h->d);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while loading");
        st = ARROW_ERR_OUT_OF_MEMORY;
    }
    if (st != ARROW_OK) {
        delete h;
        return st;
    }
    *out = h;
    return ARROW_OK;
}

void arrow_decomp_destroy(arrow_decomp_t d) { delete d; }

arrow_status_t arrow_set_allocator(arrow_alloc_fn alloc, arrow_free_fn free_fn, void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) {
        set_error("give both the alloc and the free function, or neither");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow::Allocator a;
    a.alloc = alloc;
    a.free = free_fn;
    a.ctx = alloc ? ctx : nullptr;
    arrow::set_allocator(a);
    return ARROW_OK;
}

arrow_status_t arrow_plan_create(arrow_decomp_t d, int32_t device, void *stream,
                                 arrow_plan_t *out) {
    if (!out) {
        set_error("out is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!d) {
        set_error("decomposition is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        set_error("device index out of range (or no HIP device)");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow_plan_s *h = new (std::nothrow) arrow_plan_s();
    if (!h) {
        set_error("host allocation failed");
        return ARROW_ERR_OUT_OF_MEMORY;
    }
    DeviceGuard g(device);
    arrow_status_t st;
    try {
        st = arrow::plan_create(d->d, device, static_cast<hipStream_t>(stream), h->p);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while building the plan");
        st = ARROW_ERR_OUT_OF_MEMORY;
    }
    if (st != ARROW_OK) {
        delete h;
        return st;
    }
    *out = h;
    return ARROW_OK;
}

void arrow_plan_destroy(arrow_plan_t p) {
    if (!p) return;
    arrow::plan_destroy(p->p);
    delete p;
}

arrow_status_t arrow_plan_info(arrow_plan_t p, arrow_plan_info_t *out) {
    if (!p || !out) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    const arrow::Plan &P = *p->p;
    out->n = P.n;
    out->nnz = P.nnz;
    out->b = P.b;
    out->levels = P.levels;
    out->footprint_bytes = P.footprint;
    out->chunked_rows = P.chunked_rows;
    out->chunks = P.n_chunks;
    out->upper_rows = P.n_up;
    out->contributions = P.l0_ncontrib;
    out->a_inf_norm = P.a_inf;
    out->upper_batch = P.up_batch;
    out->level0_batch = P.l0_batch;
    out->fused_rows = P.fused_rows;
    out->level0_block_rows = P.l0_rpb;
    out->reserved = 0;
    return ARROW_OK;
}

arrow_status_t arrow_plan_footprint(arrow_plan_t p, size_t *bytes) {
    if (!p || !bytes) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    *bytes = (size_t)p->p->footprint;
    return ARROW_OK;
}

static bool valid_batch(int32_t batch) {
    return batch == arrow::kBatchWide || (batch >= arrow::kBatchMin && batch <= arrow::kBatchMax);
}

arrow_status_t arrow_plan_set_batch(arrow_plan_t p, int32_t kernel, int32_t batch) {
    if (!p) {
        set_error("NULL plan");
        return ARROW_ERR_INVALID_ARG;
    }
    if (kernel != ARROW_KERNEL_UPPER && kernel != ARROW_KERNEL_LEVEL0) {
        set_error("the gather batch applies to ARROW_KERNEL_UPPER and ARROW_KERNEL_LEVEL0 only");
        return ARROW_ERR_INVALID_ARG;
    }
    if (batch != -1 && !valid_batch(batch)) {
        set_error("batch must be -1 (automatic), 0 (wide) or in [4, 8]");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow::Plan &P = *p->p;
    if (kernel == ARROW_KERNEL_UPPER)
        P.up_batch = batch == -1 ? P.up_batch_auto : batch;
    else
        P.l0_batch = batch == -1 ? P.l0_batch_auto : batch;
    return ARROW_OK;
}

arrow_status_t arrow_plan_kernel_bytes(arrow_plan_t p, int32_t kernel, int64_t k,
                                       arrow_dtype_t dtype, int64_t *bytes) {
    if (!p || !bytes) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    if (kernel < 0 || kernel >= ARROW_KERNEL_COUNT || !valid_dtype(dtype) || k <= 0) {
        set_error("bad kernel id, dtype or k");
        return ARROW_ERR_INVALID_ARG;
    }
    *bytes = arrow::kernel_bytes(*p->p, kernel, k, dtype);
    return ARROW_OK;
}

arrow_status_t arrow_workspace_size(arrow_plan_t p, int64_t k, arrow_dtype_t dtype,
                                    size_t *bytes) {
    if (!p || !bytes) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    if (arrow_status_t st = check_k(k)) return st;
    if (!valid_dtype(dtype)) {
        set_error("bad dtype");
        return ARROW_ERR_INVALID_ARG;
    }
    *bytes = arrow::op_workspace(*p->p, k, dtype);
    return ARROW_OK;
}

arrow_status_t arrow_iterate_workspace_size(arrow_plan_t p, int64_t k, arrow_dtype_t dtype,
                                            size_t *bytes) {
    size_t base = 0;
    if (arrow_status_t st = arrow_workspace_size(p, k, dtype, &base)) return st;
    const size_t zb = ((size_t)p->p->n * k * arrow::elem_size(dtype) + 255) & ~size_t(255);
    const size_t state = ((size_t)k * (2 * 8 + 2 * 4 + 2 * 4) + 255) & ~size_t(255);
    *bytes = base + zb + state;
    return ARROW_OK;
}

arrow_status_t arrow_permute_in(arrow_plan_t p, const float *x, int64_t ldx, void *x_plan,
                                int64_t ld, arrow_dtype_t dtype, int64_t k, float *x_scale,
                                float *x_maxabs, void *stream) {
    if (!p) {
        set_error("plan is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    const arrow::Plan &P = *p->p;
    if (arrow_status_t st = check_k(k)) return st;
    if (!valid_dtype(dtype)) {
        set_error("bad dtype");
        return ARROW_ERR_INVALID_ARG;
    }
    if (arrow_status_t st = check_dense(x, ldx, k, ARROW_F32, P.n, "x")) return st;
    if (arrow_status_t st = check_dense(x_plan, ld, k, dtype, P.n, "x_plan")) return st;
    if (scaled(dtype) && !x_scale) {
        set_error("x_scale is required for F16 / F8E4M3");
        return ARROW_ERR_INVALID_ARG;
    }
    if (P.n == 0) return ARROW_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard g(P.device);
    const int kt = arrow::tile_width(k);
    const int64_t es = arrow::elem_size(dtype);
    unsigned *bits = reinterpret_cast<unsigned *>(x_maxabs);
    hipError_t e = hipSuccess;
    if (scaled(dtype)) {
        // per-column max |x| -> power-of-two scale; then max |code| into x_maxabs
        unsigned *tmp = reinterpret_cast<unsigned *>(x_scale);
        e = arrow::launch_fill_u32(tmp, 0u, k, s);
        if (e == hipSuccess) e = arrow::launch_colmax(x, ldx, P.n, (int)k, tmp, s);
        if (e == hipSuccess) e = arrow::launch_scale_from_max(dtype, tmp, x_scale, (int)k, s);
    }
    if (e == hipSuccess && bits) e = arrow::launch_fill_u32(bits, 0u, k, s);
    for (int64_t c0 = 0; e == hipSuccess && c0 < k; c0 += kt)
        e = arrow::launch_permute_in(kt, dtype, x + c0, ldx, P.vop0, P.n,
                                     static_cast<char *>(x_plan) + c0 * es, ld,
                                     scaled(dtype) ? x_scale + c0 : nullptr,
                                     bits ? bits + c0 : nullptr, s);
    if (e != hipSuccess) {
        set_error(std::string("permute_in launch: ") + hipGetErrorString(e));
        return ARROW_ERR_HIP;
    }
    return ARROW_OK;
}

arrow_status_t arrow_permute_out(arrow_plan_t p, const void *y_plan, int64_t ld,
                                 arrow_dtype_t dtype, int64_t k, const float *x_scale,
                                 const double *col_factor, float *y, int64_t ldy, void *stream) {
    if (!p) {
        set_error("plan is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    const arrow::Plan &P = *p->p;
    if (arrow_status_t st = check_k(k)) return st;
    if (!valid_dtype(dtype)) {
        set_error("bad dtype");
        return ARROW_ERR_INVALID_ARG;
    }
    if (arrow_status_t st = check_dense(y_plan, ld, k, dtype, P.n, "y_plan")) return st;
    if (arrow_status_t st = check_dense(y, ldy, k, ARROW_F32, P.n, "y")) return st;
    if (P.n == 0) return ARROW_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard g(P.device);
    const int kt = arrow::tile_width(k);
    const int64_t es = arrow::elem_size(dtype);
    for (int64_t c0 = 0; c0 < k; c0 += kt) {
        hipError_t e = arrow::launch_permute_out(
            kt, dtype, static_cast<const char *>(y_plan) + c0 * es, ld, P.vop0, P.n,
            x_scale ? x_scale + c0 : nullptr, col_factor ? col_factor + c0 : nullptr, y + c0, ldy,
            s);
        if (e != hipSuccess) {
            set_error(std::string("permute_out launch: ") + hipGetErrorString(e));
            return ARROW_ERR_HIP;
        }
    }
    return ARROW_OK;
}

static arrow_status_t check_op(const arrow::Plan &P, const arrow_operand_t &o) {
    if (arrow_status_t st = check_k(o.k)) return st;
    if (!valid_dtype(o.dtype)) {
        set_error("bad dtype");
        return ARROW_ERR_INVALID_ARG;
    }
    if (arrow_status_t st = check_dense(o.x, o.ldx, o.k, o.dtype, P.n, "x")) return st;
    if (arrow_status_t st = check_dense(o.y, o.ldy, o.k, o.dtype, P.n, "y")) return st;
    const int64_t es = arrow::elem_size(o.dtype);
    if (P.n > 0 && overlaps(o.x, ((P.n - 1) * o.ldx + o.k) * es, o.y, ((P.n - 1) * o.ldy + o.k) * es)) {
        set_error("x and y must not overlap");
        return ARROW_ERR_INVALID_ARG;
    }
    if (scaled(o.dtype) && !o.y_scale) {
        set_error("y_scale is required for F16 / F8E4M3");
        return ARROW_ERR_INVALID_ARG;
    }
    if (o.w && (o.dtype != ARROW_F32 || arrow::tile_width(o.k) != o.k)) {
        set_error("the GNN-style epilogue (w) needs F32 and k in {16, 32, 64, 128}");
        return ARROW_ERR_UNSUPPORTED;
    }
    return ARROW_OK;
}

arrow_status_t arrow_spmm(arrow_plan_t p, const arrow_operand_t *ops, int32_t num_ops,
                          void *workspace, size_t ws_bytes, void *stream) {
    if (!p || (num_ops > 0 && !ops) || num_ops < 0) {
        set_error("NULL plan or operands");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow::Plan &P = *p->p;
    size_t need = 0;
    for (int32_t i = 0; i < num_ops; ++i) {
        if (arrow_status_t st = check_op(P, ops[i])) return st;
        need += arrow::op_workspace(P, ops[i].k, ops[i].dtype);
    }
    if (need > 0 && (!workspace || ws_bytes < need)) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return ARROW_ERR_INVALID_ARG;
    }
    // the products of one call run together: no operand's output may overlap
    // another operand's input or output
    for (int32_t i = 0; i < num_ops && P.n > 0; ++i) {
        const int64_t esi = arrow::elem_size(ops[i].dtype);
        const int64_t yb = ((P.n - 1) * ops[i].ldy + ops[i].k) * esi;
        for (int32_t j = 0; j < num_ops; ++j) {
            if (j == i) continue;
            const int64_t esj = arrow::elem_size(ops[j].dtype);
            if (overlaps(ops[i].y, yb, ops[j].x, ((P.n - 1) * ops[j].ldx + ops[j].k) * esj) ||
                overlaps(ops[i].y, yb, ops[j].y, ((P.n - 1) * ops[j].ldy + ops[j].k) * esj)) {
                set_error("operand " + std::to_string(i) + " writes memory that operand " +
                          std::to_string(j) + " reads or writes");
                return ARROW_ERR_INVALID_ARG;
            }
        }
    }
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return ARROW_ERR_INVALID_ARG;
    }
    DeviceGuard g(P.device);
    // operands of one storage type and tile width share one launch sequence
    // (the matrix is read once for all of them); each operand's result is the
    // one it gets alone
    std::vector<arrow::OpState> st(num_ops);
    std::vector<void *> ws(num_ops);
    char *w = static_cast<char *>(workspace);
    for (int32_t i = 0; i < num_ops; ++i) {
        const arrow_operand_t &o = ops[i];
        st[i] = arrow::OpState{o.x, o.y, o.k, o.ldx, o.ldy, o.dtype, o.x_scale, o.x_inv_norm,
                               o.x_maxabs, o.y_scale, o.y_maxabs, o.y_norm, o.y_inv_norm, o.w};
        ws[i] = w;
        w += arrow::op_workspace(P, o.k, o.dtype);
    }
    std::vector<uint8_t> done(num_ops, 0);
    std::vector<arrow::OpState> gops;
    std::vector<void *> gws;
    for (int32_t i = 0; i < num_ops; ++i) {
        if (done[i]) continue;
        gops.clear();
        gws.clear();
        for (int32_t j = i; j < num_ops; ++j)
            if (!done[j] && st[j].dtype == st[i].dtype &&
                arrow::tile_width(st[j].k) == arrow::tile_width(st[i].k) &&
                (st[j].w != nullptr) == (st[i].w != nullptr)) {
                gops.push_back(st[j]);
                gws.push_back(ws[j]);
                done[j] = 1;
            }
        if (arrow_status_t r = arrow::spmm_group(P, gops.data(), (int)gops.size(), gws.data(),
                                                 static_cast<hipStream_t>(stream)))
            return r;
    }
    return ARROW_OK;
}

arrow_status_t arrow_spmm_iterate(arrow_plan_t p, const void *x, void *y, int64_t k, int64_t ld,
                                  arrow_dtype_t dtype, const float *x_scale, float *y_scale,
                                  int32_t iters, uint32_t flags, double *norms, void *workspace,
                                  size_t ws_bytes, void *stream) {
    if (!p) {
        set_error("plan is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow::Plan &P = *p->p;
    if (iters < 0) {
        set_error("iters must be >= 0");
        return ARROW_ERR_INVALID_ARG;
    }
    if (flags & ~uint32_t(ARROW_ITER_RENORM)) {
        set_error("unknown flags");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow_operand_t probe{};
    probe.x = x;
    probe.y = y;
    probe.k = k;
    probe.ldx = probe.ldy = ld;
    probe.dtype = dtype;
    probe.y_scale = y_scale;
    if (arrow_status_t st = check_op(P, probe)) return st;
    size_t need = 0;
    arrow_iterate_workspace_size(p, k, dtype, &need);
    if (!workspace || ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return ARROW_ERR_INVALID_ARG;
    }
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return ARROW_ERR_INVALID_ARG;
    }
    if (iters == 0 || P.n == 0) return ARROW_OK;
    DeviceGuard g(P.device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t base = arrow::op_workspace(P, k, dtype);
    char *w = static_cast<char *>(workspace);
    void *z = w + base;
    const size_t zb = ((size_t)P.n * k * arrow::elem_size(dtype) + 255) & ~size_t(255);
    char *stp = w + base + zb;
    double *inv[2] = {reinterpret_cast<double *>(stp), reinterpret_cast<double *>(stp) + k};
    float *scl[2] = {reinterpret_cast<float *>(stp + 16 * k),
                     reinterpret_cast<float *>(stp + 16 * k) + k};
    float *mx[2] = {reinterpret_cast<float *>(stp + 24 * k),
                    reinterpret_cast<float *>(stp + 24 * k) + k};
    const bool renorm = flags & ARROW_ITER_RENORM;
    const bool sc = scaled(dtype);
    for (int32_t t = 0; t < iters; ++t) {
        arrow::OpState op{};
        // outputs alternate so that the last one lands in y; the scratch
        // buffer z is compact (row stride k)
        const bool x_is_z = t > 0 && (iters - t) % 2 != 0;
        const bool y_is_z = (iters - 1 - t) % 2 != 0;
        op.x = t == 0 ? x : (x_is_z ? z : y);
        op.y = y_is_z ? z : y;
        op.k = k;
        op.ldx = x_is_z ? k : ld;
        op.ldy = y_is_z ? k : ld;
        op.dtype = dtype;
        op.x_scale = t == 0 ? x_scale : (sc ? scl[(t - 1) % 2] : nullptr);
        op.x_inv_norm = (t == 0 || !renorm) ? nullptr : inv[(t - 1) % 2];
        op.x_maxabs = (t == 0 || !sc) ? nullptr : mx[(t - 1) % 2];
        op.y_scale = sc ? (t == iters - 1 ? y_scale : scl[t % 2]) : nullptr;
        op.y_maxabs = sc ? mx[t % 2] : nullptr;
        op.y_norm = norms ? norms + (int64_t)t * k : nullptr;
        op.y_inv_norm = inv[t % 2];
        if (arrow_status_t r = arrow::spmm_one(P, op, w, s)) return r;
    }
    return ARROW_OK;
}

arrow_status_t arrow_csr_workspace_size(int64_t n, int64_t k, size_t *bytes) {
    if (!bytes || n < 0) {
        set_error("bad argument");
        return ARROW_ERR_INVALID_ARG;
    }
    if (arrow_status_t st = check_k(k)) return st;
    *bytes = arrow::plain_csr_workspace(n, k);
    return ARROW_OK;
}

arrow_status_t arrow_csr_batch(int64_t n, const int64_t *row_ptr, int32_t *batch) {
    if (n < 0 || !batch || (n > 0 && !row_ptr)) {
        set_error("bad argument");
        return ARROW_ERR_INVALID_ARG;
    }
    for (int64_t r = 0; r < n; ++r)
        if (row_ptr[r + 1] < row_ptr[r]) {
            set_error("row_ptr must be non-decreasing");
            return ARROW_ERR_INVALID_ARG;
        }
    *batch = arrow::choose_batch<int64_t>(n, row_ptr, nullptr);
    return ARROW_OK;
}

arrow_status_t arrow_csr_spmm(int64_t n, const int32_t *row_ptr, const int32_t *col,
                              const float *val, const float *x, float *y, int64_t k, int64_t ld,
                              int32_t batch, double *sumsq_ws, double *norms, void *stream) {
    if (n < 0 || (n > 0 && !row_ptr)) {
        set_error("bad CSR");
        return ARROW_ERR_INVALID_ARG;
    }
    if (!valid_batch(batch)) {
        set_error("batch must be 0 (wide) or in [4, 8]");
        return ARROW_ERR_INVALID_ARG;
    }
    if (arrow_status_t st = check_k(k)) return st;
    if (arrow_status_t st = check_dense(x, ld, k, ARROW_F32, n, "x")) return st;
    if (arrow_status_t st = check_dense(y, ld, k, ARROW_F32, n, "y")) return st;
    if (n > 0 && overlaps(x, ((n - 1) * ld + k) * 4, y, ((n - 1) * ld + k) * 4)) {
        set_error("x and y must not overlap");
        return ARROW_ERR_INVALID_ARG;
    }
    return arrow::plain_csr(n, row_ptr, col, val, x, y, k, ld, batch, sumsq_ws, norms,
                            static_cast<hipStream_t>(stream));
}

arrow_status_t arrow_copy(const void *src, void *dst, int64_t bytes, void *stream) {
    if (bytes < 0 || bytes % 16 != 0 || (bytes > 0 && (!src || !dst)) ||
        reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16) {
        set_error("copy: bytes must be a multiple of 16 and pointers 16-byte aligned");
        return ARROW_ERR_INVALID_ARG;
    }
    hipError_t e = arrow::launch_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        set_error(std::string("copy launch: ") + hipGetErrorString(e));
        return ARROW_ERR_HIP;
    }
    return ARROW_OK;
}

arrow_status_t arrow_profile_enable(arrow_plan_t p, int32_t enable) {
    if (!p) {
        set_error("plan is NULL");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow::Plan &P = *p->p;
    DeviceGuard g(P.device);
    if (enable) {
        for (const arrow::ProfRec &r : P.prof_recs) {
            P.ev_pool.push_back(r.start);
            P.ev_pool.push_back(r.stop);
        }
        P.prof_recs.clear();
    }
    P.prof = enable != 0;
    return ARROW_OK;
}

arrow_status_t arrow_profile_query(arrow_plan_t p, int32_t kernel, int64_t *launches,
                                   double *total_ms) {
    if (!p || !launches || !total_ms) {
        set_error("NULL argument");
        return ARROW_ERR_INVALID_ARG;
    }
    arrow::Plan &P = *p->p;
    DeviceGuard g(P.device);
    int64_t cnt = 0;
    double tot = 0.0;
    for (const arrow::ProfRec &r : P.prof_recs) {
        if (r.kernel != kernel) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) {
            set_error("hipEventSynchronize failed");
            return ARROW_ERR_HIP;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            set_error("hipEventElapsedTime failed");
            return ARROW_ERR_HIP;
        }
        ++cnt;
        tot += ms;
    }
    *launches = cnt;
    *total_ms = tot;
    return ARROW_OK;
}

}  // extern "C"
