// Device-side helpers shared by the HIP translation units: the SELL-64 row
// view, XCD-aware block numbering, deterministic wave/block reductions, the
// phase-stamped stop flags.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mmncg {
namespace dev {

template <class V>
struct SV {
    const int64_t *sptr;
    const int *col;
    const V *val;
    const int *row_out;
    int nrows, nslices;
};

template <class V>
SV<V> view(const Sell &A);
template <>
inline SV<double> view<double>(const Sell &A) {
    return SV<double>{A.sptr, A.col, A.val, A.row_out, A.nrows, A.nslices};
}
template <>
inline SV<float> view<float>(const Sell &A) {
    return SV<float>{A.sptr, A.col, A.val32, A.row_out, A.nrows, A.nslices};
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int logical_block() {
    int G = gridDim.x, b = blockIdx.x;
    if (G >= 8 && (G & 7) == 0) return (b & 7) * (G >> 3) + (b >> 3);
    return b;
}

// contiguous slice range of this block
__device__ __forceinline__ void slice_range(int nslices, int &s0, int &s1) {  // NOLINT
    int G = gridDim.x;
    int per = (nslices + G - 1) / G;
    s0 = logical_block() * per;
    s1 = min(nslices, s0 + per);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block reduction of NQ quantities (sum, or max where is_max bit set). Result
// valid in every thread. Uses `sh` (kWaves * NQ doubles of shared memory).
template <int NQ, int NW = kWaves>
__device__ __forceinline__ void block_reduce(double (&v)[NQ], unsigned is_max, double *sh) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = ((is_max >> q) & 1) ? wave_max(v[q]) : wave_sum(v[q]);
    if (lane_id() == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[wave_id() * NQ + q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double t = sh[q];
        for (int w = 1; w < NW; ++w) t = ((is_max >> q) & 1) ? fmax(t, sh[w * NQ + q]) : t + sh[w * NQ + q];
        v[q] = t;
    }
    __syncthreads();
}

template <int NQ, int NW = kWaves>
__device__ __forceinline__ void write_partials(double (&v)[NQ], unsigned is_max, double *part, double *sh) {
    block_reduce<NQ, NW>(v, is_max, sh);
    if (threadIdx.x == 0) {
        int lb = logical_block();
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[q * kMaxPartials + lb] = v[q];
    }
}

// every block re-reduces partial slots (fixed order): out[q] = sum/max over nblk
template <int NQ, int NW = kWaves>
__device__ __forceinline__ void read_partials(const double *part, int nblk, unsigned is_max, double (&out)[NQ],
                                              double *sh) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = 0.0;
    for (int i = threadIdx.x; i < nblk; i += NW * 64)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double x = part[q * kMaxPartials + i];
            out[q] = ((is_max >> q) & 1) ? fmax(out[q], x) : out[q] + x;
        }
    block_reduce<NQ, NW>(out, is_max, sh);
}

// Stop flags carry the phase of the kernel that raised them. Every launch of
// an iterative loop has a phase number increasing along the stream; a kernel
// of phase P skips its work only when a kernel of an earlier phase stopped the
// loop (0 < flag < P). A kernel never reacts to a flag raised by its own
// launch, so all blocks of one launch take the same branch.
__device__ __forceinline__ bool stopped_before(const int *flag, int phase) {
    int f = *flag;
    return f != 0 && f < phase;
}

// ---------------------------------------------------------------------------
// row kernels: symmetric 3x3 block row (xx yy zz xy xz yz), scalar row, vec3 rows
// ---------------------------------------------------------------------------
template <class V>
__device__ __forceinline__ void row_block6(const SV<V> &A, int s, int ln, const double *__restrict__ x,
                                           double &o0, double &o1, double &o2) {
    int64_t base = A.sptr[s];
    int w = (int)((A.sptr[s + 1] - base) >> 6);
    o0 = o1 = o2 = 0.0;
    for (int k = 0; k < w; ++k) {
        int64_t e = base + 64 * k;
        int c = A.col[e + ln];
        const V *v = A.val + e * 6 + ln;
        double vxx = (double)v[0], vyy = (double)v[64], vzz = (double)v[128];
        double vxy = (double)v[192], vxz = (double)v[256], vyz = (double)v[320];
        double x0 = x[3 * (int64_t)c], x1 = x[3 * (int64_t)c + 1], x2 = x[3 * (int64_t)c + 2];
        o0 += vxx * x0 + vxy * x1 + vxz * x2;
        o1 += vxy * x0 + vyy * x1 + vyz * x2;
        o2 += vxz * x0 + vyz * x1 + vzz * x2;
    }
}

template <class V, class X>
__device__ __forceinline__ double row_scalar(const SV<V> &A, int s, int ln, const X *__restrict__ x) {
    int64_t base = A.sptr[s];
    int w = (int)((A.sptr[s + 1] - base) >> 6);
    double acc = 0.0;
    for (int k = 0; k < w; ++k) {
        int64_t e = base + 64 * k + ln;
        acc += (double)A.val[e] * (double)x[A.col[e]];
    }
    return acc;
}

template <class V>
__device__ __forceinline__ float row_scalar_f32(const SV<V> &A, int s, int ln, const float *__restrict__ x) {
    int64_t base = A.sptr[s];
    int w = (int)((A.sptr[s + 1] - base) >> 6);
    float acc = 0.0f;
    for (int k = 0; k < w; ++k) {
        int64_t e = base + 64 * k + ln;
        acc = fmaf((float)A.val[e], x[A.col[e]], acc);
    }
    return acc;
}

// sum_k vec3_k . x[col_k] (x node-major 3-vectors)
template <class V>
__device__ __forceinline__ double row_vec3_dot(const SV<V> &A, int s, int ln, const double *__restrict__ x) {
    int64_t base = A.sptr[s];
    int w = (int)((A.sptr[s + 1] - base) >> 6);
    double acc = 0.0;
    for (int k = 0; k < w; ++k) {
        int64_t e = base + 64 * k;
        int c = A.col[e + ln];
        const V *v = A.val + e * 3 + ln;
        acc += (double)v[0] * x[3 * (int64_t)c] + (double)v[64] * x[3 * (int64_t)c + 1] +
               (double)v[128] * x[3 * (int64_t)c + 2];
    }
    return acc;
}

// sum_k vec3_k * u[col_k]
template <class V>
__device__ __forceinline__ void row_vec3_scale(const SV<V> &A, int s, int ln, const double *__restrict__ u,
                                               double &o0, double &o1, double &o2) {
    int64_t base = A.sptr[s];
    int w = (int)((A.sptr[s + 1] - base) >> 6);
    o0 = o1 = o2 = 0.0;
    for (int k = 0; k < w; ++k) {
        int64_t e = base + 64 * k;
        double uc = u[A.col[e + ln]];
        const V *v = A.val + e * 3 + ln;
        o0 += (double)v[0] * uc;
        o1 += (double)v[64] * uc;
        o2 += (double)v[128] * uc;
    }
}


}  // namespace dev
}  // namespace mmncg
