// Device-side helpers shared by the HIP translation units: the SELL-64 row
// view, instance tiles of a RowMap with XCD-aware block numbering,
// deterministic wave/block reductions and the phase-stamped stop flags.
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

// Hardware blocks are dealt round-robin to the 8 XCDs; renumber them so that
// each XCD runs one contiguous eighth of the logical blocks (the tables of a
// RowMap hold a multiple of 8 blocks).
__device__ __forceinline__ int logical_block() {
    int G = gridDim.x, b = blockIdx.x;
    if (G >= 8 && (G & 7) == 0) return (b & 7) * (G >> 3) + (b >> 3);
    return b;
}

struct Tile {
    int inst, s0, s1, b;
};
// the tile of this block; inst < 0 marks padding blocks (no work, no partials)
__device__ __forceinline__ Tile tile_of(const RowMap &M) {
    int b = logical_block();
    int4 t = M.tab[b];
    return Tile{t.x, t.y, t.z, b};
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

// Block reduction of NQ quantities (sum, or max where is_max bit set); result
// valid in every thread; `sh` holds NW * NQ doubles of shared memory.
template <int NQ, int NW>
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

// this block's partials -> part[q * stride + b]
template <int NQ, int NW>
__device__ __forceinline__ void write_part(double (&v)[NQ], unsigned is_max, double *part, int stride, int b,
                                           double *sh) {
    block_reduce<NQ, NW>(v, is_max, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[(size_t)q * stride + b] = v[q];
}

// fixed-order reduction of the partials of blocks [b0, b1); result in every thread
template <int NQ, int NW>
__device__ __forceinline__ void read_part(const double *part, int stride, int b0, int b1, unsigned is_max,
                                          double (&out)[NQ], double *sh) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = 0.0;
    for (int i = b0 + (int)threadIdx.x; i < b1; i += NW * 64)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double x = part[(size_t)q * stride + i];
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
// SELL-64 rows
// ---------------------------------------------------------------------------
// The row walks below take their entries in groups of G: the column indices
// and values of a group are loaded first, then its gathers, then the products
// are added in entry order (the same sums as one entry at a time), so that a
// wave has a group's loads in flight at once. A group's entries past the
// slice's width are skipped (the test is uniform over the wave). Values stay
// in their stored type until they are multiplied. A larger G holds more
// registers, so fewer waves fit a SIMD: each kernel takes the G measured
// fastest for it.
// symmetric 3x3 block row (xx yy zz xy xz yz) times node-major 3-vectors
template <int G, class V>
__device__ __forceinline__ void row_block6(const SV<V> &A, int s, int ln, const double *__restrict__ x, double &o0,
                                           double &o1, double &o2) {
    const int64_t base = A.sptr[s];
    const int w = (int)((A.sptr[s + 1] - base) >> 6);
    // difference form (see row_scalar3): the diagonal block holds the row sum
    const int64_t row = (int64_t)s * 64 + ln;
    const double xi0 = x[3 * row], xi1 = x[3 * row + 1], xi2 = x[3 * row + 2];
    o0 = o1 = o2 = 0.0;
#pragma unroll 1
    for (int k0 = 0; k0 < w; k0 += G) {
        int cc[G];
        V vv[G][6];
        double xx[G][3];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const int64_t e = base + 64 * (k0 + k);
                cc[k] = A.col[e + ln];
                const V *v = A.val + e * 6 + ln;
#pragma unroll
                for (int q = 0; q < 6; ++q) vv[k][q] = v[64 * q];
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const int64_t c = cc[k];
                const bool dg = c == row;
                xx[k][0] = dg ? xi0 : x[3 * c] - xi0;
                xx[k][1] = dg ? xi1 : x[3 * c + 1] - xi1;
                xx[k][2] = dg ? xi2 : x[3 * c + 2] - xi2;
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const double vxx = (double)vv[k][0], vyy = (double)vv[k][1], vzz = (double)vv[k][2];
                const double vxy = (double)vv[k][3], vxz = (double)vv[k][4], vyz = (double)vv[k][5];
                o0 += vxx * xx[k][0] + vxy * xx[k][1] + vxz * xx[k][2];
                o1 += vxy * xx[k][0] + vyy * xx[k][1] + vyz * xx[k][2];
                o2 += vxz * xx[k][0] + vyz * xx[k][1] + vzz * xx[k][2];
            }
        }
    }
}

// scalar row times a plain vector, entries in groups of G as above
template <int G, class V, class X>
__device__ __forceinline__ double row_scalar(const SV<V> &A, int s, int ln, const X *__restrict__ x) {
    const int64_t base = A.sptr[s];
    const int w = (int)((A.sptr[s + 1] - base) >> 6);
    double acc = 0.0;
#pragma unroll 1
    for (int k0 = 0; k0 < w; k0 += G) {
        int cc[G];
        V vv[G];
        double xx[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const int64_t e = base + 64 * (k0 + k) + ln;
                cc[k] = A.col[e];
                vv[k] = A.val[e];
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (k0 + k < w) xx[k] = (double)x[cc[k]];
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (k0 + k < w) acc += (double)vv[k] * xx[k];
    }
    return acc;
}

// scalar row applied to each component of node-major 3-vectors, for a
// matrix stored in difference form (the local operators C and S): the
// diagonal entry holds the row sum R_i and every other entry A_ij acts on
// x_j - x_i, so (A x)_i = R_i x_i + sum_{j != i} A_ij (x_j - x_i), which is A x
// in exact arithmetic. The exchange rows sum to zero, so a uniform x gives
// exactly no exchange field whatever the precision of the stored values; in
// the plain form FP32 rounding of the entries leaves row sums of about 6e-8
// of the diagonal, a spurious radial field and an energy offset.
template <class V>
__device__ __forceinline__ void row_scalar3(const SV<V> &A, int s, int ln, const double *__restrict__ x, double &o0,
                                            double &o1, double &o2) {
    int64_t base = A.sptr[s];
    int w = (int)((A.sptr[s + 1] - base) >> 6);
    const int64_t row = (int64_t)s * 64 + ln;
    const double xi0 = x[3 * row], xi1 = x[3 * row + 1], xi2 = x[3 * row + 2];
    o0 = o1 = o2 = 0.0;
    for (int k = 0; k < w; ++k) {
        int64_t e = base + 64 * k + ln;
        double a = (double)A.val[e];
        int64_t c = A.col[e];
        const bool dg = c == row;
        o0 += a * (dg ? xi0 : x[3 * c] - xi0);
        o1 += a * (dg ? xi1 : x[3 * c + 1] - xi1);
        o2 += a * (dg ? xi2 : x[3 * c + 2] - xi2);
    }
}

// sum_k vec3_k . x[col_k]
template <int G, class V>
__device__ __forceinline__ double row_vec3_dot(const SV<V> &A, int s, int ln, const double *__restrict__ x) {
    const int64_t base = A.sptr[s];
    const int w = (int)((A.sptr[s + 1] - base) >> 6);
    double acc = 0.0;
#pragma unroll 1
    for (int k0 = 0; k0 < w; k0 += G) {
        int cc[G];
        V vv[G][3];
        double xx[G][3];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const int64_t e = base + 64 * (k0 + k);
                cc[k] = A.col[e + ln];
                const V *v = A.val + e * 3 + ln;
                vv[k][0] = v[0];
                vv[k][1] = v[64];
                vv[k][2] = v[128];
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const int64_t c = cc[k];
                xx[k][0] = x[3 * c];
                xx[k][1] = x[3 * c + 1];
                xx[k][2] = x[3 * c + 2];
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (k0 + k < w)
                acc += (double)vv[k][0] * xx[k][0] + (double)vv[k][1] * xx[k][1] + (double)vv[k][2] * xx[k][2];
    }
    return acc;
}

// sum_k vec3_k * u[col_k]
template <int G, class V>
__device__ __forceinline__ void row_vec3_scale(const SV<V> &A, int s, int ln, const double *__restrict__ u,
                                               double &o0, double &o1, double &o2) {
    const int64_t base = A.sptr[s];
    const int w = (int)((A.sptr[s + 1] - base) >> 6);
    o0 = o1 = o2 = 0.0;
#pragma unroll 1
    for (int k0 = 0; k0 < w; k0 += G) {
        int cc[G];
        V vv[G][3];
        double uu[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                const int64_t e = base + 64 * (k0 + k);
                cc[k] = A.col[e + ln];
                const V *v = A.val + e * 3 + ln;
                vv[k][0] = v[0];
                vv[k][1] = v[64];
                vv[k][2] = v[128];
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (k0 + k < w) uu[k] = u[cc[k]];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k0 + k < w) {
                o0 += (double)vv[k][0] * uu[k];
                o1 += (double)vv[k][1] * uu[k];
                o2 += (double)vv[k][2] * uu[k];
            }
        }
    }
}

}  // namespace dev
}  // namespace mmncg
