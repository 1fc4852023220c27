// Launch interface of the HIP kernels (host and device compile units).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace arrow {

enum : int { kF32 = 0, kF16 = 1, kBF16 = 2, kF8E4M3 = 3 };
enum : int { kPassChunk = 0, kPassUpper = 1, kPassLevel0 = 2, kPassPlain = 3 };
constexpr int kMaxBlockRows = 256;   // rows per staged block (at most)
constexpr int kStageEntries = 2048;  // matrix entries staged in LDS per block
constexpr int kStageLists = 512;     // listed partial rows staged in LDS per block
// far-column table entries staged in LDS per block: short-batch passes,
// wide-batch passes (the plan keeps every block's table within the larger)
constexpr int kStageFar = 1024, kStageFarWide = 2048;
constexpr int kChunk = 64;           // entries per chunk of a head row or long row
constexpr int kXcds = 8;             // XCDs of an MI355X; dispatch sends workgroup i to XCD i % 8
#ifndef ARROW_CHUNKS_PER_WAVE
#define ARROW_CHUNKS_PER_WAVE 2
#endif
constexpr int kChunksPerWave = ARROW_CHUNKS_PER_WAVE;  // consecutive chunks reduced by one wave
// Gather batch of a row pass.  kBatchWide gathers 8 entries of a row per batch
// and up to 8 listed partial rows at a time; a short batch u in
// [kBatchMin, kBatchMax] gathers u entries per batch and partial rows 2 at a
// time, holding fewer registers (more waves per SIMD) for passes whose rows
// are short.  The batch changes the schedule, not the summation order of a
// product (results agree up to the sign of a zero); the column sums of
// squares are reduced in a batch-dependent fixed order.
constexpr int kBatchWide = 0;
constexpr int kBatchMin = 4, kBatchMax = 8;

// One row pass over a CSR-like set of rows.
struct RowPass {
    int64_t nrows;
    int32_t rows_per_block;  // <= kMaxBlockRows
    int32_t blocks_per_wg;   // consecutive blocks walked by one workgroup
    int32_t nwg;             // workgroups = ceil(blocks / blocks_per_wg)
    const int32_t *ptr;   // [nrows + 1] direct entry offsets
    const void *idx;      // uint16 codes (level-0 band/head) or int32 pi_0 columns
    const float *val;
    const int32_t *cptr;  // [nrows + 1] listed partial rows (or null when unused)
    const int32_t *cidx;  // rows of the partial buffer
    int32_t lists;        // 0: no row lists a partial row (cptr is all zero)
    const uint8_t *order; // per row: the row within its block processed at this
                          // slot (rows of a block ordered by length), or null;
                          // followed by wide batches only
    const int32_t *blk_e; // [blocks + 1] entry offset of each block (ptr at the
                          // block starts), or null
    const int32_t *blk_c; // [blocks + 1] list offset of each block (with blk_e)
    // level-0 pass with 16-bit codes: code 3b+1+j names entry j of the
    // block's far-column table fcol[fptr[block] ...] (null: no far entries)
    const int32_t *fptr;
    const int32_t *fcol;
    int32_t b;
    int32_t out_row0;     // first partial-buffer row written by this pass
    int32_t batch;        // kBatchWide or a short batch in [kBatchMin, kBatchMax]
};

// One column tile of one operand (all pointers offset to the tile's first column).
struct Tile {
    const void *x;
    int64_t ldx;
    int64_t x_span;       // bytes from x to the end of the last row's tile
    const float *s;       // partial-row buffer (FP32), read by the upper / level-0 passes
    float *s_out;         // partial-row buffer written by the chunk / upper passes
    int64_t lds;
    int64_t s_span;       // bytes from s to the end of the partial-row buffer
    void *y;
    int64_t ldy;
    const float *x_scale;
    const double *x_inv_norm;
    const float *x_maxabs;
    float *y_scale;
    double *part_sumsq;   // [KT][part_ld]
    float *part_max;
    int64_t part_ld;
    float a_inf;
    const float *w;       // k x k weights of the GNN-style epilogue (row-major), or null
};

// Column tiles of the operands of one launch (same storage type and tile
// width), run one after the other by every workgroup.
constexpr int kMaxTiles = 8;
struct TileSet {
    Tile t[kMaxTiles];
    int32_t n;
};

struct NormArgs {
    const double *part_sumsq;
    const float *part_max;
    int64_t part_ld;
    int32_t nparts;
    double *norm, *inv_norm, *norms_hist;
    float *maxabs;
};

hipError_t launch_row_pass(int kt, int dtype, int mode, bool code16, const RowPass &rp,
                           const TileSet &t, hipStream_t s);

// Rows of the level-0 pass with long lists of partial rows: their lists cut
// into units; unit j (partial rows idx[ptr[j]] .. idx[ptr[j+1]-1], in order)
// is summed into partial row out_row0 + j, and the row lists its units' sums.
struct CombineArgs {
    const int32_t *ptr;  // [nrows + 1]
    const int32_t *idx;
    int64_t nrows;
    int64_t out_row0;
};
hipError_t launch_combine(int kt, const CombineArgs &a, const TileSet &t, hipStream_t s);
hipError_t launch_norm(const NormArgs &a, int k, hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, unsigned v, int64_t count, hipStream_t s);
hipError_t launch_colmax(const float *x, int64_t ldx, int64_t n, int k, unsigned *out,
                         hipStream_t s);
hipError_t launch_scale_from_max(int dtype, unsigned *bits, float *scale, int k, hipStream_t s);
hipError_t launch_permute_in(int kt, int dtype, const float *x, int64_t ldx, const int32_t *vop,
                             int64_t n, void *xp, int64_t ld, const float *scale,
                             unsigned *codemax, hipStream_t s);
hipError_t launch_permute_out(int kt, int dtype, const void *yp, int64_t ld, const int32_t *vop,
                              int64_t n, const float *scale, const double *factor, float *y,
                              int64_t ldy, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);

}  // namespace arrow
