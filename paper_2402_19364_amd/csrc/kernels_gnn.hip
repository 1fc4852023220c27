// Level-0 pass with the GNN-style epilogue ReLU((A X) W) (FP32), in a
// translation unit of its own so that the library builds in parallel.  The
// list-free level-0 passes (every row of levels >= 1 folded in, no long rows:
// the grids) keep the plan's short gather batch; the others take the wide one.
#include "kernels_dev.h"

namespace arrow {
namespace {

template <int KT, bool OFF32, int BATCH, bool CODE16, bool CONTRIB, bool FAR>
hipError_t go(const RowPass &rp, const TileSet &t, hipStream_t s) {
    const int64_t span = (int64_t)kXcds * dev::kXcdSpan;
    const int64_t slots = (rp.nwg + span - 1) / span * span;
    dim3 grid((unsigned)(slots * t.n)), block(dev::kBlockThreads);
    hipLaunchKernelGGL(
        (dev::row_kernel<KT, kF32, CODE16, CONTRIB, true, OFF32, BATCH, FAR, true>), grid, block,
        0, s, rp, t);
    return hipGetLastError();
}

template <int KT, bool OFF32, int BATCH>
hipError_t short_batch(bool far, const RowPass &rp, const TileSet &t, hipStream_t s) {
    return far ? go<KT, OFF32, BATCH, true, false, true>(rp, t, s)
               : go<KT, OFF32, BATCH, true, false, false>(rp, t, s);
}

template <int KT, bool OFF32>
hipError_t pass(bool code16, const RowPass &rp, const TileSet &t, hipStream_t s) {
    if (rp.nwg <= 0) return hipSuccess;
    if constexpr (OFF32) {
        if (code16 && !rp.lists && rp.batch != kBatchWide) {
            const bool far = rp.fptr != nullptr;
            switch (rp.batch) {
            case 4: return short_batch<KT, OFF32, 4>(far, rp, t, s);
            case 5: return short_batch<KT, OFF32, 5>(far, rp, t, s);
            case 6: return short_batch<KT, OFF32, 6>(far, rp, t, s);
            case 7: return short_batch<KT, OFF32, 7>(far, rp, t, s);
            case 8: return short_batch<KT, OFF32, 8>(far, rp, t, s);
            default: break;
            }
        }
    }
    if (code16 && rp.fptr) return go<KT, OFF32, kBatchWide, true, true, true>(rp, t, s);
    if (code16) return go<KT, OFF32, kBatchWide, true, true, false>(rp, t, s);
    return go<KT, OFF32, kBatchWide, false, true, false>(rp, t, s);
}

template <int KT>
hipError_t pass_kt(bool off32, bool code16, const RowPass &rp, const TileSet &t, hipStream_t s) {
    return off32 ? pass<KT, true>(code16, rp, t, s) : pass<KT, false>(code16, rp, t, s);
}

}  // namespace

hipError_t gnn_level0(int kt, bool off32, bool code16, const RowPass &rp, const TileSet &t,
                      hipStream_t s) {
    switch (kt) {
    case 16: return pass_kt<16>(off32, code16, rp, t, s);
    case 32: return pass_kt<32>(off32, code16, rp, t, s);
    case 64: return pass_kt<64>(off32, code16, rp, t, s);
    case 128: return pass_kt<128>(off32, code16, rp, t, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace arrow
