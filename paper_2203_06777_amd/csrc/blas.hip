// BLAS-1 and FP64 reductions over internal fields.
//
// Every internal layout is a permutation of the (complex) components with
// re/im adjacent, so norms, inner products and axpy work on the flat array of
// 16-byte vectors.  Reductions accumulate in FP64 per lane, combine the 64
// lanes of a wave with cross-lane shuffles in a fixed butterfly order, the
// waves of a block through LDS in index order, and the kRedBlocks block
// partials in a second single-block pass: the result is bitwise reproducible.
#include "dwf_device.h"

namespace dwf {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of (a, b) in fixed order; valid in thread 0.
__device__ inline void block_sum2(double &a, double &b) {
    __shared__ double sa[kRedThreads / 64], sb[kRedThreads / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0;
        b = 0;
        for (int k = 0; k < kRedThreads / 64; ++k) {
            a += sa[k];
            b += sb[k];
        }
    }
}

// dot = 0: partial[2*blk] = sum |x|^2.  dot = 1: partial = sum conj(x) y (re, im).
template <int P, int DOT>
__global__ void __launch_bounds__(kRedThreads) k_reduce(double *partials, const u32x4 *x, const u32x4 *y, long nv) {
    constexpr int R = 2 * PT<P>::G;
    using A = typename PT<P>::A;
    double re = 0, im = 0;
    for (long v = (long)blockIdx.x * kRedThreads + threadIdx.x; v < nv; v += (long)gridDim.x * kRedThreads) {
        A xv[R];
        unpack16<P>(x[v], xv);
        if (DOT) {
            A yv[R];
            unpack16<P>(y[v], yv);
#pragma unroll
            for (int k = 0; k < R; k += 2) {
                re += (double)xv[k] * yv[k] + (double)xv[k + 1] * yv[k + 1];
                im += (double)xv[k] * yv[k + 1] - (double)xv[k + 1] * yv[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) re += (double)xv[k] * xv[k];
        }
    }
    block_sum2(re, im);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = re;
        partials[2 * blockIdx.x + 1] = im;
    }
}

// r = b - ap (FP64) with the partials of |r|^2 in k_reduce's order: the true residual of
// the defect correction in one pass.
__global__ void __launch_bounds__(kRedThreads) k_residual64(double *partials, u32x4 *r, const u32x4 *b,
                                                            const u32x4 *ap, long nv) {
    double re = 0, im = 0;
    for (long v = (long)blockIdx.x * kRedThreads + threadIdx.x; v < nv; v += (long)gridDim.x * kRedThreads) {
        double bv[2], av[2];
        unpack16<DWF_F64>(b[v], bv);
        unpack16<DWF_F64>(ap[v], av);
        bv[0] -= av[0];
        bv[1] -= av[1];
        r[v] = pack16<DWF_F64>(bv);
        re += bv[0] * bv[0];
        re += bv[1] * bv[1];
    }
    block_sum2(re, im);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = re;
        partials[2 * blockIdx.x + 1] = im;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_finalize(double *dst, const double *partials, int nparts) {
    double re = 0, im = 0;
    for (int k = threadIdx.x; k < nparts; k += kRedThreads) {
        re += partials[2 * k];
        im += partials[2 * k + 1];
    }
    block_sum2(re, im);
    if (threadIdx.x == 0) {
        dst[0] = re;
        dst[1] = im;
    }
}

// y = a x + y with complex a, arithmetic in the storage's arithmetic type.
template <int P>
__global__ void __launch_bounds__(256) k_axpy(u32x4 *y, const u32x4 *x, double ar, double ai, long nv) {
    constexpr int R = 2 * PT<P>::G;
    using A = typename PT<P>::A;
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    A xv[R], yv[R];
    unpack16<P>(x[v], xv);
    unpack16<P>(y[v], yv);
    const A r = (A)ar, i = (A)ai;
#pragma unroll
    for (int k = 0; k < R; k += 2) {
        const A xr = xv[k], xi = xv[k + 1];
        yv[k] += r * xr - i * xi;
        yv[k + 1] += r * xi + i * xr;
    }
    y[v] = pack16<P>(yv);
}

// Deterministic finite pattern in [-1, 1] (used by the tuner to exercise every launch shape).
template <int P>
__global__ void __launch_bounds__(256) k_fill_pattern(u32x4 *f, long nv) {
    constexpr int R = 2 * PT<P>::G;
    using A = typename PT<P>::A;
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    A vals[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        unsigned h = (unsigned)(v * R + k) * 2654435761u;
        h ^= h >> 15;
        vals[k] = (A)((int)(h % 2001u) - 1000) * (A)1e-3;
    }
    f[v] = pack16<P>(vals);
}

// Count 16-byte vectors that differ bitwise.
__global__ void __launch_bounds__(256) k_count_diff(const u32x4 *a, const u32x4 *b, long nv, unsigned *count) {
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    const u32x4 x = a[v], y = b[v];
    const unsigned d = (x.x ^ y.x) | (x.y ^ y.y) | (x.z ^ y.z) | (x.w ^ y.w);
    if (d) atomicAdd(count, 1u);
}

int launch_fill_pattern(void *f, size_t bytes, int prec, hipStream_t st) {
    const long nv = (long)(bytes / 16);
    const unsigned nb = (unsigned)((nv + 255) / 256);
    u32x4 *fv = (u32x4 *)f;
    switch (prec) {
        case DWF_F64: hipLaunchKernelGGL(k_fill_pattern<DWF_F64>, nb, 256, 0, st, fv, nv); break;
        case DWF_F32: hipLaunchKernelGGL(k_fill_pattern<DWF_F32>, nb, 256, 0, st, fv, nv); break;
        case DWF_F16: hipLaunchKernelGGL(k_fill_pattern<DWF_F16>, nb, 256, 0, st, fv, nv); break;
        default: hipLaunchKernelGGL(k_fill_pattern<DWF_BF16>, nb, 256, 0, st, fv, nv); break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

int launch_count_diff(const void *a, const void *b, size_t bytes, unsigned *count, hipStream_t st) {
    const long nv = (long)(bytes / 16);
    hipLaunchKernelGGL(k_count_diff, (unsigned)((nv + 255) / 256), 256, 0, st, (const u32x4 *)a, (const u32x4 *)b, nv,
                       count);
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

static long nvec(long ncomplex, int prec) {
    const int g = prec == DWF_F64 ? 1 : prec == DWF_F32 ? 2 : 4;
    return ncomplex / g;
}

int launch_reduce(double *partials, double *dst, const void *x, const void *y, long n, int prec, int dot,
                  hipStream_t st) {
    const long nv = nvec(n, prec);
    const u32x4 *xv = (const u32x4 *)x, *yv = (const u32x4 *)y;
#define DWF_RED(P)                                                                                                 \
    if (dot) hipLaunchKernelGGL((k_reduce<P, 1>), kRedBlocks, kRedThreads, 0, st, partials, xv, yv, nv);          \
    else hipLaunchKernelGGL((k_reduce<P, 0>), kRedBlocks, kRedThreads, 0, st, partials, xv, yv, nv);
    switch (prec) {
        case DWF_F64: DWF_RED(DWF_F64) break;
        case DWF_F32: DWF_RED(DWF_F32) break;
        case DWF_F16: DWF_RED(DWF_F16) break;
        default: DWF_RED(DWF_BF16) break;
    }
#undef DWF_RED
    if (dst) hipLaunchKernelGGL(k_finalize, 1, kRedThreads, 0, st, dst, partials, kRedBlocks);
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

int launch_residual64(double *partials, double *dst, void *r, const void *b, const void *ap, long n, hipStream_t st) {
    const long nv = nvec(n, DWF_F64);
    hipLaunchKernelGGL(k_residual64, kRedBlocks, kRedThreads, 0, st, partials, (u32x4 *)r, (const u32x4 *)b,
                       (const u32x4 *)ap, nv);
    hipLaunchKernelGGL(k_finalize, 1, kRedThreads, 0, st, dst, partials, kRedBlocks);
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

int launch_axpy(void *y, double ar, double ai, const void *x, long n, int prec, hipStream_t st) {
    const long nv = nvec(n, prec);
    const unsigned nb = (unsigned)((nv + 255) / 256);
    u32x4 *yv = (u32x4 *)y;
    const u32x4 *xv = (const u32x4 *)x;
    switch (prec) {
        case DWF_F64: hipLaunchKernelGGL(k_axpy<DWF_F64>, nb, 256, 0, st, yv, xv, ar, ai, nv); break;
        case DWF_F32: hipLaunchKernelGGL(k_axpy<DWF_F32>, nb, 256, 0, st, yv, xv, ar, ai, nv); break;
        case DWF_F16: hipLaunchKernelGGL(k_axpy<DWF_F16>, nb, 256, 0, st, yv, xv, ar, ai, nv); break;
        default: hipLaunchKernelGGL(k_axpy<DWF_BF16>, nb, 256, 0, st, yv, xv, ar, ai, nv); break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

}  // namespace dwf
