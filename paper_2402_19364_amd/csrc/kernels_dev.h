// Device code of the arrow-decomposition SpMM for gfx950 (CDNA4, wave64),
// included by the per-storage-type translation units (kernels_<type>.hip)
// and by kernels.hip, which dispatches on the storage type.
#pragma once
//
// HIP kernels of the arrow-decomposition SpMM for gfx950 (CDNA4, wave64).
//
// Y = A X over A = sum_i P_{pi_i} B_i P_{pi_i}^T (Section 4, Eq. (1)) runs as
// three row passes and a norm pass, all in level-0 (pi_0) order:
//
//   chunk pass   the long rows (mostly the hub rows among the head rows,
//                the row tiles B^(0,j) of Section 4.1), split into nnz chunks
//                of bounded length; each chunk writes one FP32 partial row.
//   upper pass   the rows of levels i >= 1 not folded into level 0; their
//                columns were mapped through pi_0 o pi_i^{-1} at plan time, so
//                X is gathered directly in level-0 order (the forward
//                permutation of Alg. 2 as a fused gather); FP32 output.
//   level-0 pass the entries of B_0 and the folded entries of levels >= 1 of
//                the same vertex (16-bit codes: band, head column, or far
//                table), plus the listed partial rows of the other passes (the
//                reverse accumulation of Alg. 2 and the Reduce of Alg. 1),
//                scaled by the per-column factor, stored once in the storage
//                type, with FP64 per-block column sums of squares (and max
//                |code| for scaled formats).
//   norm pass    fixed-order FP64 reduction of the block partials per column.
//
// Lane layout: every lane owns 16 bytes of an X row (8 bytes for FP8 in the row
// passes, 16 in the chunk pass), VEC
// elements; LPR = KT / VEC lanes cover a row's column tile, a wave handles
// 64 / LPR rows at a time.  Matrix entries and X rows are read with plain loads (X rows are
// reused through L2 by neighbouring rows of the band); Y is written with
// non-temporal stores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.h"

namespace arrow {
namespace dev {

constexpr int kWave = 64;
constexpr int kBlockThreads = 256;
constexpr int kGnnRows = 16;  // rows of one matrix-core tile of the GNN-style epilogue
constexpr int kWaves = kBlockThreads / kWave;

// Native clang vectors (the non-temporal builtins need them).
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned vu4 __attribute__((ext_vector_type(4)));
typedef unsigned vu2 __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void store_nt(void *p, vf4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<vf4 *>(p));
}
__device__ __forceinline__ void store_nt(void *p, vu4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<vu4 *>(p));
}
__device__ __forceinline__ void store_nt(void *p, vu2 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<vu2 *>(p));
}

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_to_f32(uint32_t code) {
    return __uint_as_float(code << 16);
}
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float f16_to_f32(uint32_t code) {
    _Float16 h = __builtin_bit_cast(_Float16, (uint16_t)code);
    return (float)h;
}
__device__ __forceinline__ uint32_t f32_to_f16(float f) {  // round to nearest even
    _Float16 h = (_Float16)f;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
// One lane word at base + off: a wave-uniform base (SGPRs) plus a 32-bit
// per-lane byte offset, so a gather costs one VGPR of address and no 64-bit math.
template <class W, class O>
__device__ __forceinline__ W loadw(const char *base, O off) {
    return *reinterpret_cast<const W *>(base + off);
}
template <class O>
__device__ __forceinline__ vu4 load16(const char *base, O off) {
    return loadw<vu4>(base, off);
}

template <int DT> struct Fmt;
template <> struct Fmt<kF32> {
    using Raw = vu4;  // one lane's 16 bytes
    static constexpr int kVec = 4;
    static constexpr int kBytes = 16;
    static constexpr float kMax = 3.402823466e38f;
    static constexpr bool kScaled = false;
    __device__ static void decode(vu4 a, float (&v)[kVec]) {
        v[0] = __uint_as_float(a.x); v[1] = __uint_as_float(a.y);
        v[2] = __uint_as_float(a.z); v[3] = __uint_as_float(a.w);
    }
    // Rounds v in place to the stored value and writes it.
    __device__ static void store(void *p, float (&v)[kVec]) {
        vf4 a = {v[0], v[1], v[2], v[3]};
        store_nt(p, a);
    }
};
template <> struct Fmt<kBF16> {
    using Raw = vu4;
    static constexpr int kVec = 8;
    static constexpr int kBytes = 16;
    static constexpr float kMax = 3.38953139e38f;
    static constexpr bool kScaled = false;
    __device__ static void decode(vu4 a, float (&v)[kVec]) {
        uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = bf16_to_f32(w[i] & 0xFFFFu);
            v[2 * i + 1] = bf16_to_f32(w[i] >> 16);
        }
    }
    __device__ static void store(void *p, float (&v)[kVec]) {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t lo = f32_to_bf16(v[2 * i]), hi = f32_to_bf16(v[2 * i + 1]);
            v[2 * i] = bf16_to_f32(lo);
            v[2 * i + 1] = bf16_to_f32(hi);
            w[i] = lo | (hi << 16);
        }
        vu4 a = {w[0], w[1], w[2], w[3]};
        store_nt(p, a);
    }
};
template <> struct Fmt<kF16> {
    using Raw = vu4;
    static constexpr int kVec = 8;
    static constexpr int kBytes = 16;
    static constexpr float kMax = 65504.0f;
    static constexpr bool kScaled = true;
    __device__ static void decode(vu4 a, float (&v)[kVec]) {
        uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = f16_to_f32(w[i] & 0xFFFFu);
            v[2 * i + 1] = f16_to_f32(w[i] >> 16);
        }
    }
    __device__ static void store(void *p, float (&v)[kVec]) {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t lo = f32_to_f16(v[2 * i]), hi = f32_to_f16(v[2 * i + 1]);
            v[2 * i] = f16_to_f32(lo);
            v[2 * i + 1] = f16_to_f32(hi);
            w[i] = lo | (hi << 16);
        }
        vu4 a = {w[0], w[1], w[2], w[3]};
        store_nt(p, a);
    }
};
template <> struct Fmt<kF8E4M3> {
    using Raw = vu2;  // 8 values per lane keep the per-column state small
    static constexpr int kVec = 8;
    static constexpr int kBytes = 8;
    static constexpr float kMax = 448.0f;
    static constexpr bool kScaled = true;
    // gfx950 converts OCP E4M3FN in hardware, two values per instruction
    __device__ static void decode(vu2 a, float (&v)[kVec]) {
        uint32_t w[2] = {a.x, a.y};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
            const v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
            v[4 * i] = lo.x;
            v[4 * i + 1] = lo.y;
            v[4 * i + 2] = hi.x;
            v[4 * i + 3] = hi.y;
        }
    }
    // round to nearest even; inputs are clamped to +-448 first (the scale
    // guarantees |v| <= 448 up to rounding, and the format has no infinity)
    __device__ static void store(void *p, float (&v)[kVec]) {
        uint32_t w[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = fminf(fmaxf(v[4 * i + j], -448.0f), 448.0f);
            int pk = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
            pk = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], pk, true);
            w[i] = (uint32_t)pk;
        }
        vu2 a = {w[0], w[1]};
        store_nt(p, a);
        decode(a, v);
    }
};

// FP8 with 16 values per lane, for the chunk pass: its gathers then move
// 16 bytes like those of the other formats (it keeps no per-column state, so
// the wider lanes cost few registers there; the row passes keep 8 values).
struct FmtF8Wide {
    using Raw = vu4;  // 16 values per lane: a gather moves 16 bytes like the other formats
    static constexpr int kVec = 16;
    static constexpr int kBytes = 16;
    static constexpr float kMax = 448.0f;
    static constexpr bool kScaled = true;
    // gfx950 converts OCP E4M3FN in hardware, two values per instruction
    __device__ static void decode(vu4 a, float (&v)[kVec]) {
        uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
            const v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
            v[4 * i] = lo.x;
            v[4 * i + 1] = lo.y;
            v[4 * i + 2] = hi.x;
            v[4 * i + 3] = hi.y;
        }
    }
    // round to nearest even; inputs are clamped to +-448 first (the scale
    // guarantees |v| <= 448 up to rounding, and the format has no infinity)
    __device__ static void store(void *p, float (&v)[kVec]) {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = fminf(fmaxf(v[4 * i + j], -448.0f), 448.0f);
            int pk = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
            pk = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], pk, true);
            w[i] = (uint32_t)pk;
        }
        vu4 a = {w[0], w[1], w[2], w[3]};
        store_nt(p, a);
        decode(a, v);
    }
};

// Format of the chunk pass's gathers.
template <int DT> struct GatherFmt { using type = Fmt<DT>; };
template <> struct GatherFmt<kF8E4M3> { using type = FmtF8Wide; };

// Smallest power of two >= x (x > 0, finite); 1 for x <= 0.
__device__ __forceinline__ float pow2_ceil(double x) {
    if (!(x > 0.0)) return 1.0f;
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
    if (m == 0.5) e -= 1;
    return (float)ldexp(1.0, e);
}

// Workgroup -> slot (block group) of the row passes.  Dispatch sends
// workgroup i to XCD i % kXcds; the j-th workgroup of XCD x takes slot
// row_slot(x, j), so each XCD walks stretches of kXcdSpan consecutive slots
// (its L2 keeps the band rows the stretch's blocks share) while the eight
// XCDs stay within one window of 8 * kXcdSpan slots (they share the band
// window through the Infinity Cache).  The grid is padded to a multiple of
// 8 * kXcdSpan workgroups per tile; slots past the pass's end exit at once.
#ifndef ARROW_XCD_SPAN
#define ARROW_XCD_SPAN 16
#endif
constexpr int kXcdSpan = ARROW_XCD_SPAN;
__device__ __forceinline__ int row_slot(int x, int j) {
    return (j / kXcdSpan) * (kXcds * kXcdSpan) + x * kXcdSpan + j % kXcdSpan;
}

// ---------------------------------------------------------------------------
// row kernel
// ---------------------------------------------------------------------------

// Each workgroup walks `blocks_per_wg` consecutive blocks of rows_per_block
// rows.  Per block it first stages the row pointers, the list pointers and up
// to kStageEntries matrix entries into LDS with coalesced loads, so that the
// per-row work only waits on the X-row gathers: a lane group reads up to 8
// entries of its row from LDS and issues their 8 independent X-row loads
// before accumulating.  Entries beyond the staged range (a block with more
// entries than fit) are read from global memory.
// Register target: the FP32 final pass without partial-row lists and with a
// batch of at most 5 entries fits 72 VGPRs (7 waves per SIMD) without spills
// when the allocator is asked to; other variants keep the default.
template <int DT, bool CONTRIB, bool FINAL, int BATCH, bool GNN>
constexpr int row_waves_hint() {
    return DT == kF32 && FINAL && !CONTRIB && BATCH != kBatchWide && BATCH <= 5 && !GNN ? 7 : 1;
}
// A launch covers the column tiles of several operands (same storage type
// and tile width): the n workgroups of one slot (one per tile) run on the
// same XCD, so the block's matrix entries come from HBM once for all
// operands (requests on one graph batched into a wider k).  Each tile sees
// the workgroup partition and the sums of a launch with that tile alone.
template <int KT, int DT, bool CODE16, bool CONTRIB, bool FINAL, bool OFF32, int BATCH, bool FAR,
          bool GNN = false>
__global__ __launch_bounds__(kBlockThreads) __attribute__((
    amdgpu_waves_per_eu(row_waves_hint<DT, CONTRIB, FINAL, BATCH, GNN>()))) void row_kernel(RowPass rp,
                                                                                         TileSet ts) {
    // the n tiles of a slot run on the slot's XCD (see row_slot)
    const int xcd = blockIdx.x % kXcds;
    const int rest = blockIdx.x / kXcds;
    const Tile &t = ts.t[rest % ts.n];
    const int wg = row_slot(xcd, rest / ts.n);
    if (wg >= rp.nwg) return;  // grid padding
    using F = Fmt<DT>;
    constexpr int VEC = F::kVec;
    constexpr int LPR = KT / VEC;             // lanes per row
    constexpr int RPW = kWave / LPR;          // rows per wave and round
    constexpr int RPR = RPW * kWaves;         // rows per workgroup and round
    constexpr int UNR = BATCH == kBatchWide ? 8 : BATCH;  // entries gathered per row and batch
    static_assert(LPR >= 1 && kWave % LPR == 0, "tile width");
    constexpr int kElem = DT == kF32 ? 4 : (DT == kF8E4M3 ? 1 : 2);
    using IdxT = typename std::conditional<CODE16, uint16_t, int32_t>::type;

    __shared__ int32_t s_ptr[kMaxBlockRows + 1];
    // processing order of the block's rows (wide batches only: short batches
    // serve passes of uniform rows and keep their LDS for occupancy)
    constexpr bool ORDER = BATCH == kBatchWide;
    __shared__ uint8_t s_ord[ORDER ? kMaxBlockRows : 1];
    const bool ordered = ORDER && rp.order != nullptr;
    __shared__ int32_t s_cptr[CONTRIB ? kMaxBlockRows + 1 : 1];
    __shared__ int32_t s_cidx[CONTRIB ? kStageLists : 1];
    __shared__ IdxT s_idx[kStageEntries];
    __shared__ float s_val[kStageEntries];
    // the block's far-column table (code 3b+1+j names entry j); short
    // batches (uniform short rows, few folded entries) keep a smaller table
    // so that more workgroups share the LDS
    constexpr int STAGE_FAR = BATCH == kBatchWide ? kStageFarWide : kStageFar;
    __shared__ int32_t s_ftab[FAR ? STAGE_FAR : 1];
    __shared__ int32_t s_fb[2];

    const int tid = threadIdx.x;
    const int lane = tid % kWave;
    const int wave = tid / kWave;
    const int g = lane / LPR;
    const int sub = lane % LPR;
    const IdxT *gidx = reinterpret_cast<const IdxT *>(rp.idx);

    // X and partial-row byte offsets fit 32 bits when both buffers span less
    // than 4 GiB
    using Off = typename std::conditional<OFF32, uint32_t, uint64_t>::type;
    const char *xbase = reinterpret_cast<const char *>(t.x);
    const Off xstride = (Off)(t.ldx * kElem);
    const Off xlane = (Off)(sub * F::kBytes);

    // Per-column state of the final pass, in LDS (registers stay free for the
    // gathers): mul_j = x_scale_j * (1/nu_j) / c_j, the output scale c_j (a
    // power of two; 1 for unscaled formats) and, per wave, running FP64 sums
    // of squares and max |code| of the stored values in code units (scaled by
    // c_j^2 once at the end, exactly).  For the scaled formats c_j is the
    // power of two with |Y[:, j]| <= ||A||_inf x_scale_j max|code_j| / nu_j
    // <= c_j * max.
    // Short batches keep the lane's own columns' factors and sums in registers
    // (a butterfly once at the end); the wide batch, short of registers, keeps
    // them in LDS and reduces the row groups every round.
    constexpr bool LDS_SUMS = BATCH == kBatchWide;
    __shared__ float s_mul[FINAL ? KT : 1];
    __shared__ float s_c[FINAL ? KT : 1];
    __shared__ double s_ssq[FINAL ? kWaves : 1][FINAL ? KT : 1];
    __shared__ float s_max[FINAL ? kWaves : 1][FINAL ? KT : 1];
    // GNN-style epilogue: each wave stages kGnnRows finished rows (padded
    // rows: fewer LDS bank conflicts) and their row numbers (-1: none)
    static_assert(!GNN || (DT == kF32 && FINAL), "GNN epilogue");
    __shared__ float s_gt[GNN ? kWaves : 1][GNN ? kGnnRows : 1][GNN ? KT + 4 : 1];
    __shared__ int32_t s_gr[GNN ? kWaves : 1][GNN ? kGnnRows : 1];
    // the k x k weights in matrix-core fragment order (k <= 32, where it
    // beats reading them through the caches even at one workgroup less per
    // CU; larger k reads them through the caches, keeping the LDS for
    // occupancy): the four
    // k-steps 4 kq .. 4 kq + 3 of column
    // block jb that lane l feeds in are the 16 bytes at ((jb (k/16) + kq) 64
    // + l) 4, so a lane reads them with one conflict-free 16-byte load
    constexpr bool WLDS = GNN && KT <= 32;
    __shared__ float s_w[WLDS ? KT * KT : 1];
    float mul[LDS_SUMS ? 1 : VEC];
    double ssq[LDS_SUMS ? 1 : VEC];
    float cmax[LDS_SUMS ? 1 : VEC];
    if constexpr (WLDS) {
        for (int e = tid; e < KT * KT; e += kBlockThreads) {
            const int j4 = e % 4, l = (e / 4) % kWave, fq = e / (4 * kWave);
            const int kq = fq % (KT / 16), jb = fq / (KT / 16);
            s_w[e] = t.w[(int64_t)(16 * kq + 4 * j4 + l / 16) * KT + 16 * jb + l % 16];
        }
    }
    if constexpr (FINAL) {
        for (int j = tid; j < KT; j += kBlockThreads) {
            const float xs = t.x_scale ? t.x_scale[j] : 1.0f;
            const double inv = t.x_inv_norm ? t.x_inv_norm[j] : 1.0;
            const float fac = (float)((double)xs * inv);
            float c = 1.0f;
            if constexpr (F::kScaled) {
                const float xm = t.x_maxabs ? t.x_maxabs[j] : F::kMax;
                c = pow2_ceil((double)t.a_inf * (double)xs * (double)xm * inv /
                              (double)F::kMax);
                if (wg == 0 && t.y_scale) t.y_scale[j] = c;
            }
            s_mul[j] = fac * (1.0f / c);
            s_c[j] = c;
        }
        for (int i = tid; i < kWaves * KT; i += kBlockThreads) {
            s_ssq[i / KT][i % KT] = 0.0;
            s_max[i / KT][i % KT] = 0.0f;
        }
        __syncthreads();
        if constexpr (!LDS_SUMS) {
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                mul[i] = s_mul[sub * VEC + i];
                ssq[i] = 0.0;
                cmax[i] = 0.0f;
            }
        }
    }

    // GNN-style epilogue of the wave's staged rows: Z = ReLU(Y W) for a
    // 16-row tile on matrix cores (16x16x4 FP32 products: lane l holds
    // A[l % 16][l / 16] and B[l / 16][l % 16], result register q of lane l is
    // D[4 (l / 16) + q][l % 16]), written back over the tile, then every row
    // group stores its rows and adds their squares to the wave's column sums.
    // The first `cnt` slots hold rows (cnt is a multiple of RPW).
    auto gnn_flush = [&](int cnt) {
        if constexpr (GNN) {
            constexpr int NK = KT / 4, NJ = KT / 16;
            const int li = lane % 16, lk = lane / 16;
            __builtin_amdgcn_wave_barrier();
            // all NJ column blocks accumulate together over groups of four
            // k-steps, so every register array is indexed by constants
            vf4 d[NJ];
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb) d[jb] = vf4{0.0f, 0.0f, 0.0f, 0.0f};
            for (int kq = 0; kq < NK / 4; ++kq) {
                float a4[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) a4[j] = s_gt[wave][li][16 * kq + 4 * j + lk];
#pragma unroll
                for (int jb = 0; jb < NJ; ++jb) {
                    float b4[4];
                    if constexpr (WLDS) {
                        const float4 q4 = *reinterpret_cast<const float4 *>(
                            &s_w[((jb * (NK / 4) + kq) * kWave + lane) * 4]);
                        b4[0] = q4.x;
                        b4[1] = q4.y;
                        b4[2] = q4.z;
                        b4[3] = q4.w;
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            b4[j] = t.w[(int64_t)(16 * kq + 4 * j + lk) * KT + 16 * jb + li];
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        d[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[j], b4[j], d[jb], 0, 0, 0);
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    s_gt[wave][4 * lk + q][16 * jb + li] = fmaxf(d[jb][q], 0.0f);
            __builtin_amdgcn_wave_barrier();
            for (int sl = g; sl < cnt; sl += RPW) {
                const int row = s_gr[wave][sl];
                float v[VEC];
#pragma unroll
                for (int i = 0; i < VEC; ++i) v[i] = row >= 0 ? s_gt[wave][sl][sub * VEC + i] : 0.0f;
                if (row >= 0) {
                    char *yp = reinterpret_cast<char *>(t.y) + (int64_t)row * t.ldy * kElem +
                               (int64_t)sub * F::kBytes;
                    F::store(yp, v);
                }
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    double sq = (double)v[i] * (double)v[i];
                    if constexpr (LDS_SUMS) {
#pragma unroll
                        for (int off = LPR; off < kWave; off <<= 1) sq += __shfl_xor(sq, off);
                        if (g == 0) s_ssq[wave][sub * VEC + i] += sq;
                    } else {
                        ssq[i] += sq;  // the lane's own sums (butterfly at the end)
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    };

    for (int bi = 0; bi < rp.blocks_per_wg; ++bi) {
        const int64_t row0 = ((int64_t)wg * rp.blocks_per_wg + bi) * rp.rows_per_block;
        if (row0 >= rp.nrows) break;
        const int nr = (int)(row0 + rp.rows_per_block < rp.nrows ? rp.rows_per_block
                                                                  : rp.nrows - row0);
        const int blk = (int)(row0 / rp.rows_per_block);
        // The block's entry, list and far-table ranges: from the plan's
        // per-block offset tables when present (small, L2-resident), so the
        // entries are staged together with the row offsets in one round trip;
        // otherwise from the staged row offsets, one round trip later.
        const bool one_phase = rp.blk_e != nullptr;
        int e0 = 0, ne = 0, cb = 0, nc = 0, fb = 0, nf = 0;
        if (one_phase) {
            e0 = rp.blk_e[blk];
            ne = rp.blk_e[blk + 1] - e0;
            if constexpr (CONTRIB) {
                cb = rp.blk_c[blk];
                nc = rp.blk_c[blk + 1] - cb;
            }
            if constexpr (FAR) {
                fb = rp.fptr[blk];
                nf = rp.fptr[blk + 1] - fb;
            }
        }
        __syncthreads();  // the previous block is done with the staged data
        for (int i = tid; i <= nr; i += kBlockThreads) {
            s_ptr[i] = rp.ptr[row0 + i];
            if constexpr (CONTRIB) s_cptr[i] = rp.cptr[row0 + i];
            if (ordered && i < nr) s_ord[i] = rp.order[row0 + i];
        }
        if (!one_phase) {
            if constexpr (FAR) {
                if (tid < 2) s_fb[tid] = rp.fptr[blk + tid];
            }
            __syncthreads();
            // block-uniform values: kept in scalar registers
            e0 = __builtin_amdgcn_readfirstlane(s_ptr[0]);
            ne = __builtin_amdgcn_readfirstlane(s_ptr[nr]) - e0;
            if constexpr (CONTRIB) {
                cb = __builtin_amdgcn_readfirstlane(s_cptr[0]);
                nc = __builtin_amdgcn_readfirstlane(s_cptr[nr]) - cb;
            }
            if constexpr (FAR) {
                fb = __builtin_amdgcn_readfirstlane(s_fb[0]);
                nf = __builtin_amdgcn_readfirstlane(s_fb[1]) - fb;
            }
        }
        // Block-uniform choice: the block's entries and its far-column table
        // come from LDS when they fit, otherwise every one is read from global
        // memory.
        const bool staged = ne <= kStageEntries && (!FAR || nf <= STAGE_FAR);
        if (staged) {
            for (int i = tid; i < ne; i += kBlockThreads) {
                s_idx[i] = gidx[e0 + i];
                s_val[i] = rp.val[e0 + i];
            }
            if constexpr (FAR) {
                for (int i = tid; i < nf; i += kBlockThreads) s_ftab[i] = rp.fcol[fb + i];
            }
        }
        // the block's list of partial rows, staged the same way
        bool cstaged = true;
        if constexpr (CONTRIB) {
            cstaged = nc <= kStageLists;
            if (cstaged)
                for (int i = tid; i < nc; i += kBlockThreads) s_cidx[i] = rp.cidx[cb + i];
        }
        __syncthreads();

        // Block-uniform sources (LDS or global) are compile-time in the row loop,
        // so no load has to pick its address space at run time.
        auto rows = [&](auto staged_tag, auto cstaged_tag) {
            constexpr bool STAGED = decltype(staged_tag)::value;
            constexpr bool CSTAGED = decltype(cstaged_tag)::value;
            // wave-uniform trip count: the final pass reduces across the
            // wave's row groups every round (rows past the block end are idle)
            int gcnt = 0;  // rows staged in the wave's GNN tile
            for (int rbase = wave * RPW; rbase < nr; rbase += RPR) {
                const int rq = rbase + g;  // slot in the block's processing order
                const bool live = rq < nr;
                // the row of this slot (the plan may order a block's rows by
                // length, so a wave's row groups get rows of similar length)
                const int rl = live ? (ordered ? (int)s_ord[rq] : rq) : nr - 1;
                const int rs = rl;  // an idle group reads a valid row...
                const int64_t r = row0 + rl;
                const int a = s_ptr[rs] - e0;
                const int len = live ? s_ptr[rs + 1] - e0 - a : 0;  // ...and gathers nothing
                const int rb = (int)r - rp.b;  // band start (16-bit codes)
                float acc[VEC];
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc[i] = 0.0f;
                for (int e = 0; e < len; e += UNR) {
                    // padding slots of the last batch re-read the batch's first
                    // entry (a valid address) and contribute an exact zero
                    float av[UNR];
                    int col[UNR];
                    bool ok[UNR];
                    bool anyfar = false;
#pragma unroll
                    for (int u = 0; u < UNR; ++u) {
                        ok[u] = e + u < len;
                        const int ee = a + (ok[u] ? e + u : e);
                        IdxT code;
                        float v;
                        if constexpr (STAGED) {
                            code = s_idx[ee];
                            v = s_val[ee];
                        } else {
                            code = gidx[e0 + ee];
                            v = rp.val[e0 + ee];
                        }
                        av[u] = ok[u] ? v : 0.0f;
                        if constexpr (CODE16) {
                            // band (<= 2b), head column (<= 3b), or entry j of the
                            // block's far-column table (3b+1+j)
                            const int cc = code;
                            col[u] = cc <= 2 * rp.b ? rb + cc : cc - 2 * rp.b - 1;
                            if constexpr (FAR) anyfar |= cc > 3 * rp.b;
                        } else {
                            col[u] = code;
                        }
                    }
                    if constexpr (FAR) {
                        // the batch's folded entries (waves whose batch has none
                        // skip this): their columns from the block's far-column
                        // table, staged in LDS or read directly (index clamped to
                        // the table's first entry, which exists since the wave's
                        // batch holds a far code)
                        if (__builtin_amdgcn_ballot_w64(anyfar)) {
#pragma unroll
                            for (int u = 0; u < UNR; ++u) {
                                const int ee = a + (ok[u] ? e + u : e);
                                int cc, far;
                                if constexpr (STAGED) {
                                    cc = s_idx[ee];
                                    const int fi = cc - 3 * rp.b - 1;
                                    far = s_ftab[fi > 0 ? fi : 0];
                                } else {
                                    cc = gidx[e0 + ee];
                                    const int fi = cc - 3 * rp.b - 1;
                                    far = rp.fcol[fb + (fi > 0 ? fi : 0)];
                                }
                                col[u] = cc > 3 * rp.b ? far : col[u];
                            }
                        }
                    }
                    Off off[UNR];
#pragma unroll
                    for (int u = 0; u < UNR; ++u) off[u] = (Off)col[u] * xstride + xlane;
                    typename F::Raw xr[UNR];
#pragma unroll
                    for (int u = 0; u < UNR; ++u) xr[u] = loadw<typename F::Raw>(xbase, off[u]);
#pragma unroll
                    for (int u = 0; u < UNR; ++u) {
                        const typename F::Raw w = ok[u] ? xr[u] : typename F::Raw{};
                        float xv[VEC];
                        F::decode(w, xv);
#pragma unroll
                        for (int i = 0; i < VEC; ++i) acc[i] = fmaf(av[u], xv[i], acc[i]);
                    }
                }
                if constexpr (CONTRIB) {
                    // listed partial rows (FP32), gathered in batches like the
                    // entries: (wide batch) up to 8 at a time while more than 2
                    // remain, then 2; (short batch) 2 at a time
                    const int c0 = s_cptr[rs] - cb, c1 = live ? s_cptr[rs + 1] - cb : c0;
                    const char *sbase = reinterpret_cast<const char *>(t.s);
                    auto batch = [&](int c, auto width_tag) {
                        constexpr int W = decltype(width_tag)::value;
                        Off soff[W];
                        bool ok[W];
#pragma unroll
                        for (int u = 0; u < W; ++u) {
                            ok[u] = c + u < c1;
                            const int cc = ok[u] ? c + u : c;
                            int row;
                            if constexpr (CSTAGED)
                                row = s_cidx[cc];
                            else
                                row = rp.cidx[cb + cc];
                            soff[u] = ((Off)row * (Off)t.lds + (Off)(sub * VEC)) * 4;
                        }
                        vu4 sv[W][VEC / 4];
#pragma unroll
                        for (int u = 0; u < W; ++u)
#pragma unroll
                            for (int q = 0; q < VEC / 4; ++q)
                                sv[u][q] = load16(sbase, soff[u] + (Off)(16 * q));
#pragma unroll
                        for (int u = 0; u < W; ++u)
#pragma unroll
                            for (int q = 0; q < VEC / 4; ++q) {
                                const vu4 w = ok[u] ? sv[u][q] : vu4{0u, 0u, 0u, 0u};
                                acc[4 * q] += __uint_as_float(w.x);
                                acc[4 * q + 1] += __uint_as_float(w.y);
                                acc[4 * q + 2] += __uint_as_float(w.z);
                                acc[4 * q + 3] += __uint_as_float(w.w);
                            }
                    };
                    constexpr int WIDE =
                        BATCH != kBatchWide ? 2 : (VEC >= 16 ? 2 : (VEC >= 8 ? 4 : 8));
                    int c = c0;
                    for (; c1 - c > 2; c += WIDE) batch(c, std::integral_constant<int, WIDE>{});
                    if (c < c1) batch(c, std::integral_constant<int, 2>{});
                }
                if constexpr (FINAL && GNN) {
                    // stage the scaled row in the wave's tile; a full tile
                    // (or the wave's last round of the block) goes through
                    // the k x k product
#pragma unroll
                    for (int i = 0; i < VEC; ++i)
                        s_gt[wave][gcnt + g][sub * VEC + i] = acc[i] * s_mul[sub * VEC + i];
                    if (sub == 0) s_gr[wave][gcnt + g] = live ? (int)r : -1;
                    gcnt += RPW;
                    if (gcnt == kGnnRows || rbase + RPR >= nr) {
                        gnn_flush(gcnt);
                        gcnt = 0;
                    }
                } else if constexpr (FINAL && !LDS_SUMS) {
                    if (live) {
#pragma unroll
                        for (int i = 0; i < VEC; ++i) acc[i] = acc[i] * mul[i];
                        char *yp = reinterpret_cast<char *>(t.y) + r * t.ldy * kElem +
                                   (int64_t)sub * F::kBytes;
                        F::store(yp, acc);  // acc now holds the stored codes as floats
#pragma unroll
                        for (int i = 0; i < VEC; ++i) {
                            ssq[i] += (double)acc[i] * (double)acc[i];
                            if constexpr (F::kScaled) cmax[i] = fmaxf(cmax[i], fabsf(acc[i]));
                        }
                    }
                } else if constexpr (FINAL) {
#pragma unroll
                    for (int i = 0; i < VEC; ++i) acc[i] = acc[i] * s_mul[sub * VEC + i];
                    if (live) {
                        char *yp = reinterpret_cast<char *>(t.y) + r * t.ldy * kElem +
                                   (int64_t)sub * F::kBytes;
                        F::store(yp, acc);  // acc now holds the stored codes as floats
                    }
                    // the round's squares (and max |code|): fixed butterfly over
                    // the row groups, then group 0 adds them to the wave's sums
#pragma unroll
                    for (int i = 0; i < VEC; ++i) {
                        double v = (double)acc[i] * (double)acc[i];
                        float m = fabsf(acc[i]);
#pragma unroll
                        for (int off = LPR; off < kWave; off <<= 1) {
                            v += __shfl_xor(v, off);
                            if constexpr (F::kScaled) m = fmaxf(m, __shfl_xor(m, off));
                        }
                        if (g == 0) {
                            s_ssq[wave][sub * VEC + i] += v;
                            if constexpr (F::kScaled)
                                s_max[wave][sub * VEC + i] = fmaxf(s_max[wave][sub * VEC + i], m);
                        }
                    }
                } else {
                    if (!live) continue;
                    float *sp = t.s_out + (int64_t)(rp.out_row0 + r) * t.lds + sub * VEC;
#pragma unroll
                    for (int i = 0; i < VEC; i += 4)
                        *reinterpret_cast<float4 *>(sp + i) =
                            make_float4(acc[i], acc[i + 1], acc[i + 2], acc[i + 3]);
                }
            }
        };
        if constexpr (CONTRIB) {
            if (staged) {
                if (cstaged)
                    rows(std::true_type{}, std::true_type{});
                else
                    rows(std::true_type{}, std::false_type{});
            } else {
                if (cstaged)
                    rows(std::false_type{}, std::true_type{});
                else
                    rows(std::false_type{}, std::false_type{});
            }
        } else {
            if (staged)
                rows(std::true_type{}, std::true_type{});
            else
                rows(std::false_type{}, std::true_type{});
        }
    }

    if constexpr (FINAL && !LDS_SUMS) {
        // the lane sums: fixed butterfly across the row groups of the wave
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            double v = ssq[i];
            float m = cmax[i];
#pragma unroll
            for (int off = LPR; off < kWave; off <<= 1) {
                v += __shfl_xor(v, off);
                m = fmaxf(m, __shfl_xor(m, off));
            }
            if (g == 0) {
                s_ssq[wave][sub * VEC + i] = v;
                s_max[wave][sub * VEC + i] = m;
            }
        }
    }
    if constexpr (FINAL) {
        // the waves' sums in index order, scaled to values by c^2 (exact)
        __syncthreads();
        for (int j = tid; j < KT; j += kBlockThreads) {
            double v = s_ssq[0][j];
            float m = s_max[0][j];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                v += s_ssq[w][j];
                m = fmaxf(m, s_max[w][j]);
            }
            const double c = s_c[j];
            if (t.part_sumsq) t.part_sumsq[(int64_t)j * t.part_ld + wg] = v * (c * c);
            if (t.part_max) t.part_max[(int64_t)j * t.part_ld + wg] = m;
        }
    }
}

// Chunk pass: each wave reduces kChunksPerWave consecutive chunks (at most
// kChunk entries each, of a head row or long row) one after the other.  A
// chunk's entries arrive with one coalesced load (lane j holds entry j), and
// the next chunk's entries are loaded while the current chunk's X rows are
// gathered, so a chunk costs one memory round trip.  The lane groups take
// interleaved entries (group g: entries g, g + RPW, ...; handed over by
// cross-lane reads), so all of a chunk's gathers are in flight together; the
// group sums are combined by a fixed butterfly over the group bits and group
// 0 writes the FP32 partial row.  A workgroup handles rows_per_block =
// kWaves * kChunksPerWave consecutive chunks.
#ifndef ARROW_CHUNK_WAVES
#define ARROW_CHUNK_WAVES 1
#endif
template <int KT, int DT, bool OFF32>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(
    ARROW_CHUNK_WAVES))) void chunk_kernel(RowPass rp, TileSet ts) {
    // workgroup i runs on XCD i % kXcds and takes unit (i / kXcds / n) * kXcds
    // + i % kXcds of tile (i / kXcds) % n, so every tile of a unit runs on the
    // XCD the plan placed the unit on (the grid is a multiple of kXcds
    // workgroups per tile)
    const int xcd = blockIdx.x % kXcds;
    const int rest = blockIdx.x / kXcds;
    const Tile &t = ts.t[rest % ts.n];
    using F = typename GatherFmt<DT>::type;
    constexpr int VEC = F::kVec;
    constexpr int LPR = KT / VEC;
    constexpr int RPW = kWave / LPR;                 // lane groups per wave
    constexpr int PER = (kChunk + RPW - 1) / RPW;    // entries per group and chunk
    constexpr int UNR = PER < 8 ? PER : 8;
    static_assert(kChunk == kWave && PER % UNR == 0, "chunk layout");
    constexpr int kElem = DT == kF32 ? 4 : (DT == kF8E4M3 ? 1 : 2);
    using Off = typename std::conditional<OFF32, uint32_t, uint64_t>::type;
    const int wg = (rest / ts.n) * kXcds + xcd;
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int g = lane / LPR;
    const int sub = lane % LPR;
    const int32_t *gidx = reinterpret_cast<const int32_t *>(rp.idx);
    const char *xbase = reinterpret_cast<const char *>(t.x);
    const Off xstride = (Off)(t.ldx * kElem);
    const Off xlane = (Off)(sub * F::kBytes);
    const int64_t c0 = ((int64_t)wg * kWaves + wave) * kChunksPerWave;
    if (c0 >= rp.nrows) return;
    // chunk bounds: lane i <= kChunksPerWave holds ptr[min(c0 + i, nrows)]
    int bnd = 0;
    if (lane <= kChunksPerWave) bnd = rp.ptr[c0 + lane < rp.nrows ? c0 + lane : rp.nrows];
    // entries of chunk i: lane j holds entry j (column 0, value 0 past its end)
    auto fetch = [&](int i, int &col, float &val) {
        const int e0 = __builtin_amdgcn_readlane(bnd, i);
        const int e1 = __builtin_amdgcn_readlane(bnd, i + 1);
        col = 0;
        val = 0.0f;
        if (e0 + lane < e1) {
            col = gidx[e0 + lane];
            val = rp.val[e0 + lane];
        }
    };
    int col, ncol = 0;
    float val, nval = 0.0f;
    fetch(0, col, val);
    for (int i = 0; i < kChunksPerWave; ++i) {
        // an empty slot (or one past the end of the pass) holds no entries
        const int len = __builtin_amdgcn_readlane(bnd, i + 1) - __builtin_amdgcn_readlane(bnd, i);
        if (i + 1 < kChunksPerWave) fetch(i + 1, ncol, nval);
        if (len <= 0) {
            col = ncol;
            val = nval;
            continue;
        }
        float acc[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc[k] = 0.0f;
        for (int u0 = 0; u0 < PER && RPW * u0 < len; u0 += UNR) {
            float av[UNR];
            Off off[UNR];
            bool ok[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int j = g + RPW * (u0 + u);  // < kWave
                ok[u] = j < len;
                const int cj = __shfl(col, j);
                const float vj = __shfl(val, j);
                av[u] = ok[u] ? vj : 0.0f;
                off[u] = (Off)cj * xstride + xlane;
            }
            typename F::Raw xr[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) xr[u] = loadw<typename F::Raw>(xbase, off[u]);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const typename F::Raw w = ok[u] ? xr[u] : typename F::Raw{};
                float xv[VEC];
                F::decode(w, xv);
#pragma unroll
                for (int k = 0; k < VEC; ++k) acc[k] = fmaf(av[u], xv[k], acc[k]);
            }
        }
#pragma unroll
        for (int off = LPR; off < kWave; off <<= 1)
#pragma unroll
            for (int k = 0; k < VEC; ++k) acc[k] += __shfl_xor(acc[k], off);
        if (g == 0) {
            float *sp = t.s_out + (int64_t)(rp.out_row0 + c0 + i) * t.lds + sub * VEC;
#pragma unroll
            for (int k = 0; k < VEC; k += 4)
                *reinterpret_cast<float4 *>(sp + k) =
                    make_float4(acc[k], acc[k + 1], acc[k + 2], acc[k + 3]);
        }
        col = ncol;
        val = nval;
    }
}



// ---------------------------------------------------------------------------
// permutation kernels (Section 6.1: work in pi_0 order, permute at the ends)
// ---------------------------------------------------------------------------



// colmax (float bits of max |x|) -> power-of-two scale s_j with max/s_j <= kMax.
// `bits` and `scale` may be the same buffer.
template <int DT>
__global__ void scale_from_max_kernel(const unsigned *bits, float *scale, int k) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < k) {
        const float m = __uint_as_float(bits[j]);
        scale[j] = pow2_ceil((double)m / (double)Fmt<DT>::kMax);
    }
}

// x_plan[p] = convert(x[vop[p]] / scale): one lane group per row.
template <int KT, int DT>
__global__ __launch_bounds__(kBlockThreads) void permute_in_kernel(
    const float *x, int64_t ldx, const int32_t *vop, int64_t n, void *xp, int64_t ld,
    const float *scale, unsigned *codemax) {
    using F = Fmt<DT>;
    constexpr int VEC = F::kVec;
    constexpr int LPR = KT / VEC;
    constexpr int RPB = kBlockThreads / LPR;
    constexpr int kElem = DT == kF32 ? 4 : (DT == kF8E4M3 ? 1 : 2);
    const int sub = threadIdx.x % LPR;
    float m[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) m[i] = 0.0f;
    // rows in a grid-stride loop: the running max |code| per column stays in
    // registers and each workgroup issues one atomic per column at the end
    for (int64_t p = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR; p < n;
         p += (int64_t)gridDim.x * RPB) {
        const float *src = x + (int64_t)vop[p] * ldx + sub * VEC;
        float v[VEC];
#pragma unroll
        for (int i = 0; i < VEC; i += 4) {
            float4 a = *reinterpret_cast<const float4 *>(src + i);
            v[i] = a.x; v[i + 1] = a.y; v[i + 2] = a.z; v[i + 3] = a.w;
        }
        if (scale) {
#pragma unroll
            for (int i = 0; i < VEC; ++i) v[i] = v[i] / scale[sub * VEC + i];
        }
        F::store(reinterpret_cast<char *>(xp) + (p * ld * kElem) + sub * F::kBytes, v);
#pragma unroll
        for (int i = 0; i < VEC; ++i) m[i] = fmaxf(m[i], fabsf(v[i]));
    }
    if (codemax) {
        __shared__ float s_m[kWaves][KT];
        const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            float mm = m[i];
#pragma unroll
            for (int off = LPR; off < kWave; off <<= 1) mm = fmaxf(mm, __shfl_xor(mm, off));
            if (lane < LPR) s_m[wave][sub * VEC + i] = mm;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < KT; j += kBlockThreads) {
            float mm = s_m[0][j];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) mm = fmaxf(mm, s_m[w][j]);
            atomicMax(codemax + j, __float_as_uint(mm));
        }
    }
}

// y[vop[p]] = yp[p] * scale * factor (FP32 out).
template <int KT, int DT>
__global__ __launch_bounds__(kBlockThreads) void permute_out_kernel(
    const void *yp, int64_t ld, const int32_t *vop, int64_t n, const float *scale,
    const double *factor, float *y, int64_t ldy) {
    using F = Fmt<DT>;
    constexpr int VEC = F::kVec;
    constexpr int LPR = KT / VEC;
    constexpr int RPB = kBlockThreads / LPR;
    constexpr int kElem = DT == kF32 ? 4 : (DT == kF8E4M3 ? 1 : 2);
    const int sub = threadIdx.x % LPR;
    const int64_t p = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR;
    if (p >= n) return;
    float v[VEC];
    F::decode(*reinterpret_cast<const typename F::Raw *>(reinterpret_cast<const char *>(yp) +
                                                          p * ld * kElem + sub * F::kBytes),
              v);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        const int j = sub * VEC + i;
        double f = 1.0;
        if (scale) f *= (double)scale[j];
        if (factor) f *= factor[j];
        v[i] = (float)((double)v[i] * f);
    }
    float *dst = y + (int64_t)vop[p] * ldy + sub * VEC;
#pragma unroll
    for (int i = 0; i < VEC; i += 4)
        *reinterpret_cast<float4 *>(dst + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
}


}  // namespace dev

// ---------------------------------------------------------------------------
// launch templates (instantiated once per storage type)
// ---------------------------------------------------------------------------

// The level-0 pass with the GNN-style epilogue (FP32; kernels_gnn.hip).
hipError_t gnn_level0(int kt, bool off32, bool code16, const RowPass &rp, const TileSet &t,
                      hipStream_t s);

namespace detail {

template <int KT, int DT, bool OFF32, int BATCH>
hipError_t launch_row_b(int mode, bool code16, const RowPass &rp, const TileSet &t,
                        hipStream_t s) {
    // row passes: whole stretches of 8 * kXcdSpan slots (see row_slot); the
    // chunk pass's slot count is already a multiple of kXcds
    const int64_t span = (int64_t)kXcds * (mode == kPassChunk ? 1 : dev::kXcdSpan);
    const int64_t slots = (rp.nwg + span - 1) / span * span;
    dim3 grid((unsigned)(slots * t.n)), block(dev::kBlockThreads);
    switch (mode) {
    case kPassChunk:
        hipLaunchKernelGGL((dev::chunk_kernel<KT, DT, OFF32>), grid, block, 0, s, rp, t);
        break;
    case kPassUpper:
        hipLaunchKernelGGL((dev::row_kernel<KT, DT, false, true, false, OFF32, BATCH, false>),
                           grid, block, 0, s, rp, t);
        break;
    case kPassLevel0:
        if (code16 && rp.fptr && !rp.lists && BATCH != kBatchWide) {
            // folded entries, no partial rows to add (every row of levels >= 1
            // folded, no long rows): no list staging at all
            hipLaunchKernelGGL(
                (dev::row_kernel<KT, DT, true, false, true, OFF32, BATCH, true>), grid, block,
                0, s, rp, t);
        } else if (code16 && rp.fptr) {  // with folded entries of levels >= 1
            hipLaunchKernelGGL((dev::row_kernel<KT, DT, true, true, true, OFF32, BATCH, true>),
                               grid, block, 0, s, rp, t);
        } else if (code16 && !rp.lists && BATCH != kBatchWide) {  // one level, no long rows
            hipLaunchKernelGGL(
                (dev::row_kernel<KT, DT, true, false, true, OFF32, BATCH, false>), grid, block,
                0, s, rp, t);
        } else if (code16) {
            hipLaunchKernelGGL((dev::row_kernel<KT, DT, true, true, true, OFF32, BATCH, false>),
                               grid, block, 0, s, rp, t);
        } else {  // int32 columns (b > 21845): wide batches only
            hipLaunchKernelGGL(
                (dev::row_kernel<KT, DT, false, true, true, OFF32, kBatchWide, false>), grid,
                block, 0, s, rp, t);
        }
        break;
    case kPassPlain:  // plain CSR (FP32 only): int32 columns, no contributions, final store
        if constexpr (DT == kF32)
            hipLaunchKernelGGL(
                (dev::row_kernel<KT, DT, false, false, true, OFF32, BATCH, false>), grid, block,
                0, s, rp, t);
        else
            return hipErrorInvalidValue;
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Short batches are built for 32-bit offsets only (X and the partial-row
// buffer below 4 GiB); larger operands take the wide batch.
template <int KT, int DT, bool OFF32>
hipError_t launch_row_o(int mode, bool code16, const RowPass &rp, const TileSet &t,
                        hipStream_t s) {
    if (rp.nwg <= 0) return hipSuccess;
    if (mode == kPassLevel0 && t.t[0].w)
        return DT == kF32 ? gnn_level0(KT, OFF32, code16, rp, t, s) : hipErrorInvalidValue;
    if constexpr (OFF32) {
        if (mode != kPassChunk) {
            switch (rp.batch) {
            case 4: return launch_row_b<KT, DT, true, 4>(mode, code16, rp, t, s);
            case 5: return launch_row_b<KT, DT, true, 5>(mode, code16, rp, t, s);
            case 6: return launch_row_b<KT, DT, true, 6>(mode, code16, rp, t, s);
            case 7: return launch_row_b<KT, DT, true, 7>(mode, code16, rp, t, s);
            case 8: return launch_row_b<KT, DT, true, 8>(mode, code16, rp, t, s);
            default: break;
            }
        }
    }
    return launch_row_b<KT, DT, OFF32, kBatchWide>(mode, code16, rp, t, s);
}

template <int KT, int DT>
hipError_t launch_row_t(int mode, bool code16, const RowPass &rp, const TileSet &t, hipStream_t s) {
    bool off32 = true;
    for (int i = 0; i < t.n; ++i)
        off32 = off32 && t.t[i].x_span < (int64_t(1) << 32) && t.t[i].s_span < (int64_t(1) << 32);
    if (off32) return launch_row_o<KT, DT, true>(mode, code16, rp, t, s);
    return launch_row_o<KT, DT, false>(mode, code16, rp, t, s);
}

template <int DT>
hipError_t launch_row_dt(int kt, int mode, bool code16, const RowPass &rp, const TileSet &t,
                         hipStream_t s) {
    switch (kt) {
    case 16: return launch_row_t<16, DT>(mode, code16, rp, t, s);
    case 32: return launch_row_t<32, DT>(mode, code16, rp, t, s);
    case 64: return launch_row_t<64, DT>(mode, code16, rp, t, s);
    case 128: return launch_row_t<128, DT>(mode, code16, rp, t, s);
    default: return hipErrorInvalidValue;
    }
}

template <int KT, int DT>
hipError_t launch_perm_in_t(const float *x, int64_t ldx, const int32_t *vop, int64_t n, void *xp,
                            int64_t ld, const float *scale, unsigned *codemax, hipStream_t s) {
    constexpr int LPR = KT / dev::Fmt<DT>::kVec;
    constexpr int RPB = dev::kBlockThreads / LPR;
    int64_t blocks = (n + RPB - 1) / RPB;
    if (codemax && blocks > 4096) blocks = 4096;  // grid-stride: few atomics per column
    dim3 grid((unsigned)blocks);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((dev::permute_in_kernel<KT, DT>), grid, dim3(dev::kBlockThreads), 0, s, x,
                       ldx, vop, n, xp, ld, scale, codemax);
    return hipGetLastError();
}

template <int KT, int DT>
hipError_t launch_perm_out_t(const void *yp, int64_t ld, const int32_t *vop, int64_t n,
                             const float *scale, const double *factor, float *y, int64_t ldy,
                             hipStream_t s) {
    constexpr int LPR = KT / dev::Fmt<DT>::kVec;
    constexpr int RPB = dev::kBlockThreads / LPR;
    dim3 grid((unsigned)((n + RPB - 1) / RPB));
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((dev::permute_out_kernel<KT, DT>), grid, dim3(dev::kBlockThreads), 0, s,
                       yp, ld, vop, n, scale, factor, y, ldy);
    return hipGetLastError();
}

}  // namespace detail

// Per-storage-type entry points, explicitly instantiated in kernels_<type>.hip.
template <int DT>
hipError_t row_pass_dt(int kt, int mode, bool code16, const RowPass &rp, const TileSet &t,
                       hipStream_t s) {
    switch (kt) {
    case 16: return detail::launch_row_t<16, DT>(mode, code16, rp, t, s);
    case 32: return detail::launch_row_t<32, DT>(mode, code16, rp, t, s);
    case 64: return detail::launch_row_t<64, DT>(mode, code16, rp, t, s);
    case 128: return detail::launch_row_t<128, DT>(mode, code16, rp, t, s);
    default: return hipErrorInvalidValue;
    }
}

template <int DT>
hipError_t permute_in_dt(int kt, const float *x, int64_t ldx, const int32_t *vop, int64_t n,
                         void *xp, int64_t ld, const float *scale, unsigned *codemax,
                         hipStream_t s) {
    switch (kt) {
    case 16: return detail::launch_perm_in_t<16, DT>(x, ldx, vop, n, xp, ld, scale, codemax, s);
    case 32: return detail::launch_perm_in_t<32, DT>(x, ldx, vop, n, xp, ld, scale, codemax, s);
    case 64: return detail::launch_perm_in_t<64, DT>(x, ldx, vop, n, xp, ld, scale, codemax, s);
    case 128: return detail::launch_perm_in_t<128, DT>(x, ldx, vop, n, xp, ld, scale, codemax, s);
    default: return hipErrorInvalidValue;
    }
}

template <int DT>
hipError_t permute_out_dt(int kt, const void *yp, int64_t ld, const int32_t *vop, int64_t n,
                          const float *scale, const double *factor, float *y, int64_t ldy,
                          hipStream_t s) {
    switch (kt) {
    case 16: return detail::launch_perm_out_t<16, DT>(yp, ld, vop, n, scale, factor, y, ldy, s);
    case 32: return detail::launch_perm_out_t<32, DT>(yp, ld, vop, n, scale, factor, y, ldy, s);
    case 64: return detail::launch_perm_out_t<64, DT>(yp, ld, vop, n, scale, factor, y, ldy, s);
    case 128: return detail::launch_perm_out_t<128, DT>(yp, ld, vop, n, scale, factor, y, ldy, s);
    default: return hipErrorInvalidValue;
    }
}

#define ARROW_DECLARE_DT(DT_)                                                                  \
    extern template hipError_t row_pass_dt<DT_>(int, int, bool, const RowPass &, const TileSet &, \
                                                hipStream_t);                                  \
    extern template hipError_t permute_in_dt<DT_>(int, const float *, int64_t, const int32_t *, \
                                                  int64_t, void *, int64_t, const float *,     \
                                                  unsigned *, hipStream_t);                     \
    extern template hipError_t permute_out_dt<DT_>(int, const void *, int64_t, const int32_t *, \
                                                   int64_t, const float *, const double *,      \
                                                   float *, int64_t, hipStream_t);
#define ARROW_INSTANTIATE_DT(DT_)                                                              \
    template hipError_t row_pass_dt<DT_>(int, int, bool, const RowPass &, const TileSet &,        \
                                         hipStream_t);                                         \
    template hipError_t permute_in_dt<DT_>(int, const float *, int64_t, const int32_t *,       \
                                           int64_t, void *, int64_t, const float *, unsigned *, \
                                           hipStream_t);                                        \
    template hipError_t permute_out_dt<DT_>(int, const void *, int64_t, const int32_t *,       \
                                            int64_t, const float *, const double *, float *,    \
                                            int64_t, hipStream_t);

}  // namespace arrow
