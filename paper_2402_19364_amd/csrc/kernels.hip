// Dispatch of the HIP kernels by storage type, and the kernels that do not
// depend on it (norms, column maxima, scales, streaming copy).  The row and
// permutation kernels of each storage type are compiled in kernels_<type>.hip.
#include "kernels_dev.h"

namespace arrow {
namespace dev {

// One workgroup per column: fixed-order FP64 sum of the block partials.
constexpr int kNormThreads = 1024;  // one wide workgroup per column: few, long reductions
__global__ __launch_bounds__(kNormThreads) void norm_kernel(NormArgs a) {
    const int j = blockIdx.x;
    const double *ps = a.part_sumsq + (int64_t)j * a.part_ld;
    double v = 0.0;
    float m = 0.0f;
    // thread t adds partials t, t + 1024, t + 2048, ... in that order; the
    // loads of a group of kPer are issued before the adds
    constexpr int kPer = 16;
    for (int base = threadIdx.x; base < a.nparts; base += kNormThreads * kPer) {
        double vals[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = base + u * kNormThreads;
            vals[u] = i < a.nparts ? ps[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) v += vals[u];
    }
    if (a.part_max) {
        const float *pm = a.part_max + (int64_t)j * a.part_ld;
        for (int base = threadIdx.x; base < a.nparts; base += kNormThreads * kPer) {
            float vals[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int i = base + u * kNormThreads;
                vals[u] = i < a.nparts ? pm[i] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u) m = fmaxf(m, vals[u]);
        }
    }
    __shared__ double sv[kNormThreads];
    __shared__ float sm[kNormThreads];
    sv[threadIdx.x] = v;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = kNormThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sv[threadIdx.x] += sv[threadIdx.x + s];
            sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ss = sv[0];
        const double nu = sqrt(ss);
        if (a.norm) a.norm[j] = nu;
        if (a.inv_norm) a.inv_norm[j] = nu > 0.0 ? 1.0 / nu : 0.0;
        if (a.norms_hist) a.norms_hist[j] = nu;
        if (a.maxabs) a.maxabs[j] = sm[0];
    }
}

// Per-column max |x| of an FP32 matrix: float bits of non-negative values
// order like unsigned integers, so an atomic max is order independent.
// Each workgroup reduces its rows in registers and LDS first and issues one
// atomic per column, so the atomics stay few (one per workgroup and column).
__global__ __launch_bounds__(kBlockThreads) void colmax_kernel(const float *x, int64_t ldx,
                                                                int64_t n, int k,
                                                                unsigned *out) {
    __shared__ float s_m[kWaves][64];
    const int j = threadIdx.x % 64;
    const int rsub = threadIdx.x / 64;
    for (int jb = 0; jb < k; jb += 64) {
        const int jj = jb + j;
        float m = 0.0f;
        if (jj < k) {
            const int64_t stride = (int64_t)gridDim.x * 4;
            int64_t r = (int64_t)blockIdx.x * 4 + rsub;
            for (; r + 3 * stride < n; r += 4 * stride) {  // four independent loads in flight
                const float a = x[r * ldx + jj], b = x[(r + stride) * ldx + jj];
                const float c = x[(r + 2 * stride) * ldx + jj], d = x[(r + 3 * stride) * ldx + jj];
                m = fmaxf(m, fmaxf(fmaxf(fabsf(a), fabsf(b)), fmaxf(fabsf(c), fabsf(d))));
            }
            for (; r < n; r += stride) m = fmaxf(m, fabsf(x[r * ldx + jj]));
        }
        s_m[rsub][j] = m;
        __syncthreads();
        if (rsub == 0 && jj < k) {
            const float mm = fmaxf(fmaxf(s_m[0][j], s_m[1][j]), fmaxf(s_m[2][j], s_m[3][j]));
            atomicMax(out + jj, __float_as_uint(mm));
        }
        __syncthreads();
    }
}

__global__ void fill_u32_kernel(unsigned *p, unsigned v, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Streaming copy (HBM calibration): plain 16-byte loads and stores in a
// grid-stride loop over a fixed grid of 1024 workgroups (4 per CU), the
// configuration that streams fastest on MI355X among those measured
// (deeper unrolling, non-temporal hints and larger grids were all slower).
__global__ __launch_bounds__(kBlockThreads) void copy_kernel(const vu4 *src, vu4 *dst,
                                                             int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * kBlockThreads;
    for (int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; i < count; i += stride)
        dst[i] = src[i];
}

// Sum of one unit of a long list of FP32 partial rows (a hub row of the
// level-0 pass, which would otherwise add them one batch after another on a
// single lane group): workgroup (j, tile) splits unit j into G contiguous
// slices, lane group g adds slice g in list order, and the G slice sums are
// added in slice order.  The order depends on the unit and the tile width
// only.
template <int KT>
__global__ __launch_bounds__(kBlockThreads) void combine_kernel(CombineArgs a, TileSet ts) {
    constexpr int LPR = KT / 4;              // lanes per row, 4 columns (16 bytes) each
    constexpr int G = kBlockThreads / LPR;   // lane groups
    const Tile &t = ts.t[blockIdx.x % ts.n];
    const int64_t j = blockIdx.x / ts.n;
    if (j >= a.nrows) return;
    const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
    const int64_t c0 = a.ptr[j], len = a.ptr[j + 1] - c0;
    const int64_t lo = c0 + len * g / G, hi = c0 + len * (g + 1) / G;
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int64_t c = lo;
    // four rows in flight at a time, added in list order
    for (; c + 4 <= hi; c += 4) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            v[u] = *reinterpret_cast<const float4 *>(t.s + (int64_t)a.idx[c + u] * t.lds + sub * 4);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    for (; c < hi; ++c) {
        const float4 v = *reinterpret_cast<const float4 *>(t.s + (int64_t)a.idx[c] * t.lds + sub * 4);
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    __shared__ float4 s_part[G][LPR];
    s_part[g][sub] = acc;
    __syncthreads();
    if (threadIdx.x < LPR) {
        float4 sum = s_part[0][sub];
        for (int q = 1; q < G; ++q) {
            sum.x += s_part[q][sub].x;
            sum.y += s_part[q][sub].y;
            sum.z += s_part[q][sub].z;
            sum.w += s_part[q][sub].w;
        }
        *reinterpret_cast<float4 *>(t.s_out + (a.out_row0 + j) * t.lds + sub * 4) = sum;
    }
}

}  // namespace dev

ARROW_DECLARE_DT(kF32)
ARROW_DECLARE_DT(kF16)
ARROW_DECLARE_DT(kBF16)
ARROW_DECLARE_DT(kF8E4M3)


hipError_t launch_row_pass(int kt, int dtype, int mode, bool code16, const RowPass &rp,
                           const TileSet &t, hipStream_t s) {
    switch (dtype) {
    case kF32: return row_pass_dt<kF32>(kt, mode, code16, rp, t, s);
    case kF16: return row_pass_dt<kF16>(kt, mode, code16, rp, t, s);
    case kBF16: return row_pass_dt<kBF16>(kt, mode, code16, rp, t, s);
    case kF8E4M3: return row_pass_dt<kF8E4M3>(kt, mode, code16, rp, t, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_combine(int kt, const CombineArgs &a, const TileSet &t, hipStream_t s) {
    if (a.nrows <= 0) return hipSuccess;
    const dim3 grid((unsigned)(a.nrows * t.n)), block(dev::kBlockThreads);
    switch (kt) {
    case 16: hipLaunchKernelGGL(dev::combine_kernel<16>, grid, block, 0, s, a, t); break;
    case 32: hipLaunchKernelGGL(dev::combine_kernel<32>, grid, block, 0, s, a, t); break;
    case 64: hipLaunchKernelGGL(dev::combine_kernel<64>, grid, block, 0, s, a, t); break;
    case 128: hipLaunchKernelGGL(dev::combine_kernel<128>, grid, block, 0, s, a, t); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_norm(const NormArgs &a, int k, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::norm_kernel, dim3(k), dim3(dev::kNormThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, unsigned v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::fill_u32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       s, p, v, count);
    return hipGetLastError();
}

hipError_t launch_colmax(const float *x, int64_t ldx, int64_t n, int k, unsigned *out,
                         hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    int64_t blocks = (n + 4 * 64 - 1) / (4 * 64);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(dev::colmax_kernel, dim3((unsigned)blocks), dim3(dev::kBlockThreads), 0, s,
                       x, ldx, n, k, out);
    return hipGetLastError();
}

hipError_t launch_scale_from_max(int dtype, unsigned *bits, float *scale, int k, hipStream_t s) {
    dim3 grid((k + 255) / 256), block(256);
    if (dtype == kF16)
        hipLaunchKernelGGL(dev::scale_from_max_kernel<kF16>, grid, block, 0, s, bits, scale, k);
    else if (dtype == kF8E4M3)
        hipLaunchKernelGGL(dev::scale_from_max_kernel<kF8E4M3>, grid, block, 0, s, bits, scale, k);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_permute_in(int kt, int dtype, const float *x, int64_t ldx, const int32_t *vop,
                             int64_t n, void *xp, int64_t ld, const float *scale,
                             unsigned *codemax, hipStream_t s) {
    switch (dtype) {
    case kF32: return permute_in_dt<kF32>(kt, x, ldx, vop, n, xp, ld, scale, codemax, s);
    case kF16: return permute_in_dt<kF16>(kt, x, ldx, vop, n, xp, ld, scale, codemax, s);
    case kBF16: return permute_in_dt<kBF16>(kt, x, ldx, vop, n, xp, ld, scale, codemax, s);
    case kF8E4M3: return permute_in_dt<kF8E4M3>(kt, x, ldx, vop, n, xp, ld, scale, codemax, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_permute_out(int kt, int dtype, const void *yp, int64_t ld, const int32_t *vop,
                              int64_t n, const float *scale, const double *factor, float *y,
                              int64_t ldy, hipStream_t s) {
    switch (dtype) {
    case kF32: return permute_out_dt<kF32>(kt, yp, ld, vop, n, scale, factor, y, ldy, s);
    case kF16: return permute_out_dt<kF16>(kt, yp, ld, vop, n, scale, factor, y, ldy, s);
    case kBF16: return permute_out_dt<kBF16>(kt, yp, ld, vop, n, scale, factor, y, ldy, s);
    case kF8E4M3: return permute_out_dt<kF8E4M3>(kt, yp, ld, vop, n, scale, factor, y, ldy, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t s) {
    const int64_t count = bytes / 16;
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + dev::kBlockThreads - 1) / dev::kBlockThreads;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(dev::copy_kernel, dim3((unsigned)blocks), dim3(dev::kBlockThreads), 0, s,
                       reinterpret_cast<const dev::vu4 *>(src), reinterpret_cast<dev::vu4 *>(dst), count);
    return hipGetLastError();
}

}  // namespace arrow
