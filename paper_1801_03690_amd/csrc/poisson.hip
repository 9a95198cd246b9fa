// Scalar-potential solve K u = b (the magnetostatic subproblem of every energy
// evaluation; the paper solves it with preconditioned CG, Sec. 3.1) by
// Jacobi-preconditioned CG on gfx950.
//
// Two kernels per CG iteration:
//   A: convergence test, beta, p_new = D^-1 r + beta p_old (own rows) and
//      q = K p_new, where the neighbour values of p_new are formed on the fly
//      from r, D^-1 and p_old (p is double-buffered, so no block reads a value
//      another block is overwriting); partial p.q.
//   B: alpha, x += alpha p_new, r -= alpha q; partials r.z, r.r.
// Each kernel re-reduces the partials of the previous one in a fixed order
// (every block gets the same scalars; no fences, no floating-point atomics),
// and the r.z / r.r partials alternate between two slots, so every launch of a
// chunk of iterations has fixed arguments: the chunk is captured once into a
// HIP graph and replayed until the device-side flag reports convergence. Stop
// flags carry the phase of the kernel that raised them (device_common.h).
//
// Vector type VT is double (FP64 mode) or float (inner solve of the FP32-bulk
// mode, wrapped in FP64 defect correction); reductions are always FP64.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace mmncg {

using namespace dev;

namespace {

// Poisson kernels run 1024-thread blocks (16 waves, one SELL slice each at a
// time) on at most 256 blocks: every CU holds a block of 16 waves, and the
// partials a kernel re-reduces fit one load per thread.
constexpr int kPB = 1024;
constexpr int kPW = kPB / 64;
constexpr int kPMaxBlocks = 256;

// partial regions (slot q of region R at part + (R + q) * kMaxPartials):
//   RZ0 = 0, RZ1 = 2 (r.z, r.r written by kernel B of even / odd iterations),
//   PQ = 4 (p.q of kernel A), INIT = 5 (b.b, r.z, r.r of the start)
constexpr int kRZ0 = 0, kRZ1 = 2, kPQ = 4, kINIT = 5;
__device__ __forceinline__ double *pslot(double *part, int r) { return part + (size_t)r * kMaxPartials; }
__device__ __forceinline__ const double *pslot(const double *part, int r) { return part + (size_t)r * kMaxPartials; }

// r = b - K u; partials (b.b, r.D^-1.r, r.r)
template <class MT>
__global__ __launch_bounds__(kPB) void k_pcg_init64(SV<MT> K, const double *__restrict__ b,
                                                       const double *__restrict__ u, double *__restrict__ r,
                                                       const double *__restrict__ invD, double *__restrict__ part,
                                                       int with_rz) {
    __shared__ double sh[kPW * 3];
    int s0, s1;
    slice_range(K.nslices, s0, s1);
    int ln = lane_id();
    double acc[3] = {0, 0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kPW) {
        double ku = row_scalar(K, s, ln, u);
        int row = s * 64 + ln;
        if (row < K.nrows) {
            double bi = b[row];
            double ri = bi - ku;
            r[row] = ri;
            acc[0] += bi * bi;
            if (with_rz) acc[1] += ri * (ri * invD[row]);
            acc[2] += ri * ri;
        }
    }
    write_partials<3, kPW>(acc, 0u, pslot(part, kINIT), sh);
}

// start of the FP32 inner solve K x = r64 * scale: x = 0, r32 = r64 * scale; partials (-, r.z, r.r)
__global__ __launch_bounds__(kPB) void k_pcg_init32(int n, int nslices, const double *__restrict__ r64,
                                                       double scale, float *__restrict__ x, float *__restrict__ r,
                                                       const float *__restrict__ invD, double *__restrict__ part) {
    __shared__ double sh[kPW * 3];
    int s0, s1;
    slice_range(nslices, s0, s1);
    double acc[3] = {0, 0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kPW) {
        int i = s * 64 + lane_id();
        if (i < n) {
            float ri = (float)(r64[i] * scale);
            x[i] = 0.0f;
            r[i] = ri;
            acc[1] += (double)ri * (double)(ri * invD[i]);
            acc[2] += (double)ri * (double)ri;
        }
    }
    write_partials<3, kPW>(acc, 0u, pslot(part, kINIT), sh);
}

// one block: reduce the start partials into the CG state and seed the ring so
// that the first kernel A sees r.z (new) and +inf (old), i.e. beta = 0.
// mode 0: tol2 = rtol2 * b.b (FP64 solve); mode 1: tol2 = rtol2 * r.r (FP32
// inner solve, relative to its own start); mode 2: residual only (no CG start).
__global__ __launch_bounds__(kPB) void k_pcg_init_fin(double *__restrict__ part, int nblk, double rtol2, int mode,
                                                         PcgState *__restrict__ st) {
    __shared__ double sh[kPW * 3];
    double t[3];
    read_partials<3, kPW>(pslot(part, kINIT), nblk, 0u, t, sh);
    const double bb = t[0], rz = t[1], rr = t[2];
    const double tol2 = (mode == 1) ? rtol2 * rr : rtol2 * bb;
    if (threadIdx.x == 0) {
        st->bb = bb;
        st->rz = rz;
        st->rr = rr;
        st->tol2 = tol2;
        st->iters = 0;
        st->zero_u = (mode != 1 && bb == 0.0) ? 1 : 0;
        st->done = (mode == 2 || (mode != 1 && bb == 0.0) || rr <= tol2) ? 1 : 0;
    }
    if (mode == 2) return;
    double *nw = pslot(part, kRZ1), *od = pslot(part, kRZ0);
    for (int i = threadIdx.x; i < nblk; i += kPB) {
        nw[i] = (i == 0) ? rz : 0.0;
        nw[kMaxPartials + i] = (i == 0) ? rr : 0.0;
        od[i] = (i == 0) ? __builtin_huge_val() : 0.0;
        od[kMaxPartials + i] = 0.0;
    }
}

__device__ __forceinline__ int row_or_zero(int s, int ln, int nrows) {
    int row = s * 64 + ln;
    return row < nrows ? row : 0;
}

template <class VT>
__device__ __forceinline__ VT pval(const VT *__restrict__ r, const VT *__restrict__ invD,
                                   const VT *__restrict__ p_old, VT beta, int64_t c) {
    VT z = r[c] * invD[c];
    return beta != (VT)0 ? z + beta * p_old[c] : z;
}

// kernel A of iteration j (odd = j & 1): convergence test on the residual of
// iteration j-1 (every block decides alike; block 0 raises the flag), then
// beta, p_new = D^-1 r + beta p_old, q = K p_new, partial p_new.q
template <class MT, class VT>
__global__ __launch_bounds__(kPB) void k_pcg_a(SV<MT> K, const VT *__restrict__ r, const VT *__restrict__ invD,
                                                  const VT *__restrict__ p_old, VT *__restrict__ p_new,
                                                  VT *__restrict__ q, PcgState *__restrict__ st, int phase, int odd,
                                                  double *__restrict__ part) {
    if (stopped_before(&st->done, phase)) return;
    __shared__ double sh[kPW * 2];
    const int nblk = gridDim.x;
    double nw[2], od[1];
    read_partials<2, kPW>(pslot(part, odd ? kRZ0 : kRZ1), nblk, 0u, nw, sh);
    if (nw[1] <= st->tol2) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->done = phase;
        return;
    }
    read_partials<1, kPW>(pslot(part, odd ? kRZ1 : kRZ0), nblk, 0u, od, sh);
    const VT beta = (VT)(nw[0] / od[0]);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->iters += 1;
    int s0, s1;
    slice_range(K.nslices, s0, s1);
    int ln = lane_id();
    double acc[1] = {0};
    for (int s = s0 + wave_id(); s < s1; s += kPW) {
        int64_t base = K.sptr[s];
        int w = (int)((K.sptr[s + 1] - base) >> 6);
        VT qv = 0;
        // entries in groups of 8 with every load of a group issued before use
        for (int k0 = 0; k0 < w; k0 += 8) {
            int cc[8];
            VT vv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                bool in = k0 + k < w;
                int64_t e = base + 64 * (k0 + k) + ln;
                cc[k] = in ? K.col[e] : row_or_zero(s, ln, K.nrows);
                vv[k] = in ? (VT)K.val[e] : (VT)0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) qv += vv[k] * pval(r, invD, p_old, beta, cc[k]);
        }
        int row = s * 64 + ln;
        if (row < K.nrows) {
            VT pn = pval(r, invD, p_old, beta, row);
            p_new[row] = pn;
            q[row] = qv;
            acc[0] += (double)pn * (double)qv;
        }
    }
    write_partials<1, kPW>(acc, 0u, pslot(part, kPQ), sh);
}

// kernel B of iteration j: alpha = r.z / p.q; x += alpha p, r -= alpha q;
// partials (r.z, r.r) into the ring slot of iteration j
template <class VT, class XT>
__global__ __launch_bounds__(kPB) void k_pcg_b(int n, int nslices, XT *__restrict__ x, VT *__restrict__ r,
                                                  const VT *__restrict__ p, const VT *__restrict__ q,
                                                  const VT *__restrict__ invD, PcgState *__restrict__ st, int phase,
                                                  int odd, double *__restrict__ part) {
    if (stopped_before(&st->done, phase)) return;
    __shared__ double sh[kPW * 2];
    const int nblk = gridDim.x;
    double pq[1], rz[1];
    read_partials<1, kPW>(pslot(part, kPQ), nblk, 0u, pq, sh);
    read_partials<1, kPW>(pslot(part, odd ? kRZ0 : kRZ1), nblk, 0u, rz, sh);
    const VT a = (VT)(rz[0] / pq[0]);
    int s0, s1;
    slice_range(nslices, s0, s1);
    double acc[2] = {0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kPW) {
        int i = s * 64 + lane_id();
        if (i < n) {
            x[i] += (XT)(a * p[i]);
            VT ri = r[i] - a * q[i];
            r[i] = ri;
            acc[0] += (double)ri * (double)(ri * invD[i]);
            acc[1] += (double)ri * (double)ri;
        }
    }
    write_partials<2, kPW>(acc, 0u, pslot(part, odd ? kRZ1 : kRZ0), sh);
}

__global__ __launch_bounds__(kPB) void k_add_correction(int n, double *__restrict__ u, const float *__restrict__ x,
                                                           double scale) {
    int i = blockIdx.x * kPB + threadIdx.x;
    if (i < n) u[i] += scale * (double)x[i];
}

inline int nslices_of(int n) { return (n + 63) / 64; }

inline int pgrid(int nrows) {
    int g = (nslices_of(nrows) + kPW - 1) / kPW;
    if (g < 1) g = 1;
    if (g > kPMaxBlocks) g = kPMaxBlocks;
    if (g >= 8) g = (g + 7) & ~7;
    return g;
}

}  // namespace

void launch_pcg_init64(const Sell &K, const double *b, const double *u, double *r, const double *invD, double rtol2,
                       PcgState *st, double *part, bool fp32, hipStream_t s) {
    int g = pgrid(K.nrows);
    if (fp32)
        hipLaunchKernelGGL(k_pcg_init64<float>, dim3(g), dim3(kPB), 0, s, view<float>(K), b, u, r, invD, part, 1);
    else
        hipLaunchKernelGGL(k_pcg_init64<double>, dim3(g), dim3(kPB), 0, s, view<double>(K), b, u, r, invD, part, 1);
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(1), dim3(kPB), 0, s, part, g, rtol2, 0, st);
}

void launch_residual64(const Sell &K, const double *b, const double *u, double *r, PcgState *st, double *part,
                       hipStream_t s) {
    int g = pgrid(K.nrows);
    hipLaunchKernelGGL(k_pcg_init64<float>, dim3(g), dim3(kPB), 0, s, view<float>(K), b, u, r, nullptr, part, 0);
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(1), dim3(kPB), 0, s, part, g, 0.0, 2, st);
}

void launch_pcg_init32(int n, const double *r64, double scale, float *x, float *r, const float *invD, double inner2,
                       PcgState *st, double *part, hipStream_t s) {
    int g = pgrid(n);
    hipLaunchKernelGGL(k_pcg_init32, dim3(g), dim3(kPB), 0, s, n, nslices_of(n), r64, scale, x, r, invD, part);
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(1), dim3(kPB), 0, s, part, g, inner2, 1, st);
}

void launch_pcg_iter64(const Sell &K, double *u, double *r, double *p_old, double *p_new, double *q,
                       const double *invD, PcgState *st, int phase_a, int odd, double *part, hipStream_t s) {
    int g = pgrid(K.nrows);
    hipLaunchKernelGGL((k_pcg_a<double, double>), dim3(g), dim3(kPB), 0, s, view<double>(K), r, invD, p_old,
                       p_new, q, st, phase_a, odd, part);
    hipLaunchKernelGGL((k_pcg_b<double, double>), dim3(g), dim3(kPB), 0, s, K.nrows, nslices_of(K.nrows), u, r,
                       p_new, q, invD, st, phase_a + 1, odd, part);
}

void launch_pcg_iter32(const Sell &K, float *x, float *r, float *p_old, float *p_new, float *q, const float *invD,
                       PcgState *st, int phase_a, int odd, double *part, hipStream_t s) {
    int g = pgrid(K.nrows);
    hipLaunchKernelGGL((k_pcg_a<float, float>), dim3(g), dim3(kPB), 0, s, view<float>(K), r, invD, p_old, p_new,
                       q, st, phase_a, odd, part);
    hipLaunchKernelGGL((k_pcg_b<float, float>), dim3(g), dim3(kPB), 0, s, K.nrows, nslices_of(K.nrows), x, r,
                       p_new, q, invD, st, phase_a + 1, odd, part);
}

void launch_add_correction(int n, double *u, const float *x, double scale, hipStream_t s) {
    int g = (n + kPB - 1) / kPB;
    hipLaunchKernelGGL(k_add_correction, dim3(g), dim3(kPB), 0, s, n, u, x, scale);
}

}  // namespace mmncg
