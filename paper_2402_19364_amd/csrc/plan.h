// Device plan: the decomposition laid out as row passes in level-0 order.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace arrow {

constexpr int kLongRow = 32;      // rows with more entries go through the chunk pass
constexpr int kFuseRow = 64;      // longest level-0 row after folding in rows of levels >= 1
constexpr int kRowsPerBlock = kMaxBlockRows;       // rows per staged block
constexpr int kBlocksPerWg = 1;                    // blocks walked by one workgroup
// Blocks walked by one workgroup of the level-0 pass of the scaled formats
// (FP16, FP8), whose prologue also derives the per-column output scales.
constexpr int kBlocksPerWgScaled = 1;
constexpr int kChunksPerBlock = kChunksPerWave * 4;  // chunks per workgroup of the chunk pass
// Column windows of the chunk pass's far entries (a multiple of kXcds).
#ifndef ARROW_CHUNK_WINDOWS
#define ARROW_CHUNK_WINDOWS 8
#endif
constexpr int kChunkWindows = ARROW_CHUNK_WINDOWS;
static_assert(kChunkWindows % kXcds == 0, "chunk windows");
// Rows with at least this many far entries are split by column window.
#ifndef ARROW_WINDOW_ROW
#define ARROW_WINDOW_ROW 256
#endif
constexpr int kWindowRow = ARROW_WINDOW_ROW;
// Level-0 rows listing more partial rows than this have them summed by the
// combine pass first (a hub row's chunks, added in parallel instead of one
// batch after another by one lane group).
#ifndef ARROW_COMBINE_LIST
#define ARROW_COMBINE_LIST 32
#endif
constexpr int kCombineList = ARROW_COMBINE_LIST;
// A long list is cut into units of at most this many partial rows (equal
// shares), each summed by its own workgroup into one partial row; the row
// then lists its units' sums in order.
#ifndef ARROW_COMBINE_UNIT
#define ARROW_COMBINE_UNIT 64
#endif
constexpr int kCombineUnit = ARROW_COMBINE_UNIT;

struct ProfRec {
    int kernel;
    hipEvent_t start, stop;
    hipStream_t stream;
};

// Device allocator of plan buffers (arrow_set_allocator); null functions =
// hipMalloc / hipFree.
struct Allocator {
    arrow_alloc_fn alloc = nullptr;
    arrow_free_fn free = nullptr;
    void *ctx = nullptr;
};
Allocator current_allocator();
void set_allocator(const Allocator &a);

struct Plan {
    int device = 0;
    Allocator allocator;  // the allocator the plan's buffers came from
    int64_t n = 0, nnz = 0;
    int32_t b = 0, levels = 0;
    double a_inf = 0.0;
    bool code16 = true;

    // level-0 pass (n rows)
    int32_t *l0_ptr = nullptr;
    void *l0_idx = nullptr;
    float *l0_val = nullptr;
    int32_t *l0_cptr = nullptr;
    uint8_t *l0_order = nullptr;        // per-block processing order (wide batch), or null
    int32_t *l0_blk_e = nullptr, *l0_blk_c = nullptr;  // per-block entry / list offsets
    int32_t *l0_cidx = nullptr;
    int64_t l0_nnz = 0, l0_ncontrib = 0;
    int32_t l0_rpb = kMaxBlockRows;     // rows per staged block of the level-0 pass
    int32_t *l0_fptr = nullptr;         // [blocks + 1] far-column table of each block
    int32_t *l0_fcol = nullptr;         // pi_0 columns of entries folded in from levels >= 1
    int64_t l0_nfar = 0;                // entries in the far-column tables
    int64_t fused_rows = 0;             // rows of levels >= 1 folded into level-0 rows
    // upper pass (rows of levels >= 1 with entries)
    int64_t n_up = 0;
    int32_t *up_ptr = nullptr, *up_col = nullptr;
    float *up_val = nullptr;
    int32_t *up_cptr = nullptr, *up_cidx = nullptr;
    uint8_t *up_order = nullptr;
    int32_t *up_blk_e = nullptr, *up_blk_c = nullptr;
    int64_t up_nnz = 0, up_ncontrib = 0;
    // chunk pass
    int64_t n_chunks = 0, chunked_rows = 0;
    int64_t ch_slots = 0;  // chunk slots (a multiple of kXcds * kChunksPerBlock; some empty)
    int32_t *ch_ptr = nullptr, *ch_col = nullptr;
    float *ch_val = nullptr;
    int64_t ch_nnz = 0;
    // permutation pi_0^{-1}
    int32_t *vop0 = nullptr;

    // gather batch of the upper and level-0 passes (kBatchWide or a short batch)
    int32_t up_batch = kBatchWide, l0_batch = kBatchWide;
    int32_t up_batch_auto = kBatchWide, l0_batch_auto = kBatchWide;

    // level-0 rows with more than kCombineList listed partial rows: their
    // lists cut into units, unit j summed by the combine pass into partial
    // row n_up + ch_slots + j
    int64_t n_heavy = 0, hv_nlist = 0;  // units, partial rows they sum
    int32_t *hv_ptr = nullptr, *hv_idx = nullptr;

    int64_t s_rows = 0;  // partial-row buffer rows = n_up + ch_slots + n_heavy
    // distinct X rows each pass reads (algorithmic byte model)
    int64_t distinct_l0 = 0, distinct_up = 0, distinct_ch = 0;

    std::vector<void *> allocs;
    int64_t footprint = 0;

    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> ev_pool;
};

// Host arrays of a plan, before upload (the device arrays of the same names).
struct PlanArrays {
    std::vector<int32_t> l0_ptr, l0_col, l0_cptr, l0_cidx, l0_blk_e, l0_blk_c, far_ptr, far_col;
    std::vector<uint16_t> l0_code;
    std::vector<float> l0_val;
    std::vector<uint8_t> l0_order, up_order;
    std::vector<int32_t> up_ptr, up_col, up_cptr, up_cidx, up_blk_e, up_blk_c;
    std::vector<float> up_val;
    std::vector<int32_t> ch_ptr, ch_col;
    std::vector<float> ch_val;
    std::vector<int32_t> hv_ptr, hv_idx;
};
// Builds the plan's host arrays and fills the scalar fields of `p` (no
// device work).
void plan_build(const Decomp &d, Plan &p, PlanArrays &h);
arrow_status_t plan_create(const Decomp &d, int device, hipStream_t stream, Plan *&out);
void plan_destroy(Plan *p);

struct OpState {
    const void *x;
    void *y;
    int64_t k, ldx, ldy;
    int dtype;
    const float *x_scale;
    const double *x_inv_norm;
    const float *x_maxabs;
    float *y_scale;
    float *y_maxabs;
    double *y_norm;
    double *y_inv_norm;
    const float *w;  // GNN-style epilogue weights (k x k), or null
};

int64_t elem_size(int dtype);
int tile_width(int64_t k);
size_t op_workspace(const Plan &p, int64_t k, int dtype);
// Enqueue one product for one operand; `ws` holds op_workspace bytes.
arrow_status_t spmm_one(Plan &p, const OpState &op, void *ws, hipStream_t s);
// One product for each of `nops` operands of one storage type and one tile
// width, as one launch sequence over all their column tiles (the matrix is
// read once per launch); wss[o] holds op_workspace bytes for operand o.  Every
// operand's result is bitwise the one spmm_one gives it alone.
arrow_status_t spmm_group(Plan &p, const OpState *ops, int nops, void *const *wss,
                          hipStream_t s);
int64_t kernel_bytes(const Plan &p, int kernel, int64_t k, int dtype);

// Gather batch for a row pass from its rows' entry counts (ptr, host) and
// listed partial-row counts (cptr, host, or null): the smallest short batch
// that holds all entries of at least 99% of the rows, provided at least 99%
// of the rows list at most 2 partial rows; kBatchWide otherwise.
template <class I>
int32_t choose_batch(int64_t nrows, const I *ptr, const int32_t *cptr);

arrow_status_t plain_csr(int64_t n, const int32_t *row_ptr, const int32_t *col, const float *val,
                         const float *x, float *y, int64_t k, int64_t ld, int32_t batch,
                         double *ws, double *norms, hipStream_t s);
size_t plain_csr_workspace(int64_t n, int64_t k);

}  // namespace arrow
