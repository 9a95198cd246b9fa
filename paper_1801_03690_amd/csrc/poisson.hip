// Scalar-potential solve K u = b (the magnetostatic subproblem of every energy
// evaluation; the paper solves it with preconditioned CG, Sec. 3.1) by
// Jacobi-preconditioned CG on gfx950, for every instance of a batch at once.
//
// Two kernels per CG iteration:
//   A: convergence test, beta, p_new = D^-1 r + beta p_old (own rows) and
//      q = K p_new, where the neighbour values of p_new are formed on the fly
//      from r, D^-1 and p_old (p is double-buffered, so no block reads a value
//      another block is overwriting); partial p.q.
//   B: alpha, x += alpha p_new, r -= alpha q; partials r.z, r.r.
// Each kernel re-reduces the previous kernel's partials of its own instance in
// a fixed order (every block of the instance gets the same scalars; no fences,
// no floating-point atomics). The r.z / r.r partials alternate between two
// slot pairs, so every launch of a chunk of iterations has fixed arguments:
// the chunk is captured once into a HIP graph and replayed until every
// instance's flag reports convergence. Once an instance's flag is up, every
// later kernel of it returns at once, in this replay and in any further one
// (replays are launched speculatively, ahead of the host seeing the flag).
// All blocks of a kernel A take the same convergence decision from the same
// partials, so a block that already sees the flag raised by its own launch
// behaves as if it had decided itself.
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
// time), at most kMaxBlocksPerInst blocks per instance.
constexpr int kPB = kPoissonBlock;
constexpr int kPW = kPB / 64;

// partial slots (slot q at part + q * stride):
//   RZ0 = 0-1, RZ1 = 2-3 (r.z, r.r written by kernel B of even / odd iterations),
//   PQ = 4 (p.q of kernel A), INIT = 5-7 (b.b, r.z, r.r of the start)
constexpr int kRZ0 = 0, kRZ1 = 2, kPQ = 4, kINIT = 5;

__device__ __forceinline__ double *slot(double *part, int stride, int q) { return part + (size_t)q * stride; }
__device__ __forceinline__ const double *slot(const double *part, int stride, int q) {
    return part + (size_t)q * stride;
}

// r = b - K u; partials (b.b, r.D^-1.r, r.r)
template <class MT>
__global__ __launch_bounds__(kPB) void k_pcg_init64(SV<MT> K, RowMap M, const int *__restrict__ act,
                                                    const double *__restrict__ b, const double *__restrict__ u,
                                                    double *__restrict__ r, const double *__restrict__ invD,
                                                    double *__restrict__ part, int with_rz) {
    Tile t = tile_of(M);
    if (t.inst < 0 || (act && !act[t.inst])) return;
    __shared__ double sh[kPW * 3];
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[3] = {0, 0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += kPW) {
        double ku = row_scalar(K, s, ln, u);
        int row = s * 64 + ln;
        if (row < rend) {
            double bi = b[row];
            double ri = bi - ku;
            r[row] = ri;
            acc[0] += bi * bi;
            if (with_rz) acc[1] += ri * (ri * invD[row]);
            acc[2] += ri * ri;
        }
    }
    write_part<3, kPW>(acc, 0u, slot(part, M.nblk, kINIT), M.nblk, t.b, sh);
}

// start of the FP32 inner solve K x = r64 * scale_i: x = 0, r32 = r64 * scale_i
__global__ __launch_bounds__(kPB) void k_pcg_init32(RowMap M, const double *__restrict__ pin,
                                                    const double *__restrict__ r64, float *__restrict__ x,
                                                    float *__restrict__ r, const float *__restrict__ invD,
                                                    double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !(pin[4 * t.inst + 1] > 0.0)) return;
    __shared__ double sh[kPW * 3];
    const double scale = pin[4 * t.inst];
    const int rend = M.rend[t.inst];
    double acc[3] = {0, 0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += kPW) {
        int i = s * 64 + lane_id();
        if (i < rend) {
            float ri = (float)(r64[i] * scale);
            x[i] = 0.0f;
            r[i] = ri;
            acc[1] += (double)ri * (double)(ri * invD[i]);
            acc[2] += (double)ri * (double)ri;
        }
    }
    write_part<3, kPW>(acc, 0u, slot(part, M.nblk, kINIT), M.nblk, t.b, sh);
}

// one block per instance: reduce the start partials into the instance's CG
// state and seed the ring so that the first kernel A sees r.z (new) and +inf
// (old), i.e. beta = 0.
// mode 0: CG start, tol2 = rtol2 * b.b; mode 1: FP32 inner start, tol2 =
// pin[1] * r.r (inactive when pin[1] <= 0); mode 2: residual only (no CG).
__global__ __launch_bounds__(kPB) void k_pcg_init_fin(RowMap M, double *__restrict__ part, double rtol2, int mode,
                                                      const int *__restrict__ act, const double *__restrict__ pin,
                                                      PcgState *__restrict__ st) {
    __shared__ double sh[kPW * 3];
    const int i = blockIdx.x;
    const bool on = (mode == 1) ? (pin[4 * i + 1] > 0.0) : (act ? act[i] != 0 : true);
    if (!on) {
        if (threadIdx.x == 0) {
            st[i].done = 1;
            st[i].active = 0;
        }
        return;
    }
    const int S = M.nblk, b0 = M.ipb[i], b1 = M.ipb[i + 1];
    double t[3];
    read_part<3, kPW>(slot(part, S, kINIT), S, b0, b1, 0u, t, sh);
    const double bb = t[0], rz = t[1], rr = t[2];
    const double tol2 = (mode == 1) ? pin[4 * i + 1] * rr : rtol2 * bb;
    if (threadIdx.x == 0) {
        st[i].bb = bb;
        st[i].rr = rr;
        st[i].tol2 = tol2;
        st[i].iters = 0;
        st[i].active = 1;
        st[i].zero_u = (mode != 1 && bb == 0.0) ? 1 : 0;
        st[i].done = (mode == 2 || (mode != 1 && bb == 0.0) || rr <= tol2) ? 1 : 0;
    }
    if (mode == 2) return;
    double *nw = slot(part, S, kRZ1), *od = slot(part, S, kRZ0);
    for (int k = b0 + (int)threadIdx.x; k < b1; k += kPB) {
        nw[k] = (k == b0) ? rz : 0.0;
        nw[(size_t)S + k] = (k == b0) ? rr : 0.0;
        od[k] = (k == b0) ? __builtin_huge_val() : 0.0;
        od[(size_t)S + k] = 0.0;
    }
}

__device__ __forceinline__ int row_or_zero(int s, int ln, int rend) {
    int row = s * 64 + ln;
    return row < rend ? row : 0;
}

template <class VT>
__device__ __forceinline__ VT pval(const VT *__restrict__ r, const VT *__restrict__ invD,
                                   const VT *__restrict__ p_old, VT beta, int64_t c) {
    VT z = r[c] * invD[c];
    return beta != (VT)0 ? z + beta * p_old[c] : z;
}

// kernel A of iteration j (odd = j & 1): convergence test on the residual of
// iteration j-1 (every block of the instance decides alike; its first block
// raises the flag), then beta, p_new = D^-1 r + beta p_old, q = K p_new,
// partial p_new.q
template <class MT, class VT>
__global__ __launch_bounds__(kPB) void k_pcg_a(SV<MT> K, RowMap M, const VT *__restrict__ r,
                                               const VT *__restrict__ invD, const VT *__restrict__ p_old,
                                               VT *__restrict__ p_new, VT *__restrict__ q, PcgState *__restrict__ st,
                                               int phase, int odd, double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    PcgState *si = st + t.inst;
    if (si->done) return;
    __shared__ double sh[kPW * 2];
    const int S = M.nblk, b0 = M.ipb[t.inst], b1 = M.ipb[t.inst + 1];
    double nw[2], od[1];
    read_part<2, kPW>(slot(part, S, odd ? kRZ0 : kRZ1), S, b0, b1, 0u, nw, sh);
    if (nw[1] <= si->tol2) {
        if (t.b == b0 && threadIdx.x == 0) si->done = phase;
        return;
    }
    read_part<1, kPW>(slot(part, S, odd ? kRZ1 : kRZ0), S, b0, b1, 0u, od, sh);
    const VT beta = (VT)(nw[0] / od[0]);
    if (t.b == b0 && threadIdx.x == 0) si->iters += 1;
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[1] = {0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += kPW) {
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
                cc[k] = in ? K.col[e] : row_or_zero(s, ln, rend);
                vv[k] = in ? (VT)K.val[e] : (VT)0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) qv += vv[k] * pval(r, invD, p_old, beta, cc[k]);
        }
        int row = s * 64 + ln;
        if (row < rend) {
            VT pn = pval(r, invD, p_old, beta, row);
            p_new[row] = pn;
            q[row] = qv;
            acc[0] += (double)pn * (double)qv;
        }
    }
    write_part<1, kPW>(acc, 0u, slot(part, S, kPQ), S, t.b, sh);
}

// kernel B of iteration j: alpha = r.z / p.q; x += alpha p, r -= alpha q;
// partials (r.z, r.r) into the ring slot of iteration j
template <class VT, class XT>
__global__ __launch_bounds__(kPB) void k_pcg_b(RowMap M, XT *__restrict__ x, VT *__restrict__ r,
                                               const VT *__restrict__ p, const VT *__restrict__ q,
                                               const VT *__restrict__ invD, PcgState *__restrict__ st, int phase,
                                               int odd, double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0 || st[t.inst].done) return;
    __shared__ double sh[kPW * 2];
    const int S = M.nblk, b0 = M.ipb[t.inst], b1 = M.ipb[t.inst + 1];
    double pq[1], rz[1];
    read_part<1, kPW>(slot(part, S, kPQ), S, b0, b1, 0u, pq, sh);
    read_part<1, kPW>(slot(part, S, odd ? kRZ0 : kRZ1), S, b0, b1, 0u, rz, sh);
    const VT a = (VT)(rz[0] / pq[0]);
    const int rend = M.rend[t.inst];
    double acc[2] = {0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += kPW) {
        int i = s * 64 + lane_id();
        if (i < rend) {
            x[i] += (XT)(a * p[i]);
            VT ri = r[i] - a * q[i];
            r[i] = ri;
            acc[0] += (double)ri * (double)(ri * invD[i]);
            acc[1] += (double)ri * (double)ri;
        }
    }
    write_part<2, kPW>(acc, 0u, slot(part, S, odd ? kRZ1 : kRZ0), S, t.b, sh);
}

// u += rn_i * x32 for the instances with an inner solve
__global__ __launch_bounds__(kPB) void k_add_correction(RowMap M, const double *__restrict__ pin, double *__restrict__ u,
                                                        const float *__restrict__ x) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !(pin[4 * t.inst + 1] > 0.0)) return;
    const double sc = pin[4 * t.inst + 2];
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += kPW) {
        int i = s * 64 + lane_id();
        if (i < rend) u[i] += sc * (double)x[i];
    }
}

}  // namespace

void launch_pcg_init64(const PcgLaunch &a, const int *act, double rtol2, bool fp32_matrix, hipStream_t s) {
    const RowMap &M = *a.M;
    if (fp32_matrix)
        hipLaunchKernelGGL(k_pcg_init64<float>, dim3(M.nblk), dim3(kPB), 0, s, view<float>(*a.K), M, act, a.b, a.u,
                           a.r, a.invD, a.part, 1);
    else
        hipLaunchKernelGGL(k_pcg_init64<double>, dim3(M.nblk), dim3(kPB), 0, s, view<double>(*a.K), M, act, a.b, a.u,
                           a.r, a.invD, a.part, 1);
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kPB), 0, s, M, a.part, rtol2, 0, act, a.pin, a.st);
}

void launch_residual64(const PcgLaunch &a, const int *act, hipStream_t s) {
    const RowMap &M = *a.M;
    hipLaunchKernelGGL(k_pcg_init64<float>, dim3(M.nblk), dim3(kPB), 0, s, view<float>(*a.K), M, act, a.b, a.u, a.r,
                       a.invD, a.part, 0);
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kPB), 0, s, M, a.part, 0.0, 2, act, a.pin, a.st);
}

void launch_pcg_init32(const PcgLaunch &a, hipStream_t s) {
    const RowMap &M = *a.M;
    hipLaunchKernelGGL(k_pcg_init32, dim3(M.nblk), dim3(kPB), 0, s, M, a.pin, a.r, a.x32, a.r32, a.invD32, a.part);
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kPB), 0, s, M, a.part, 0.0, 1, nullptr, a.pin, a.st);
}

void launch_pcg_iter64(const PcgLaunch &a, int phase_a, int odd, hipStream_t s) {
    const RowMap &M = *a.M;
    double *po = odd ? a.p1 : a.p0, *pn = odd ? a.p0 : a.p1;
    hipLaunchKernelGGL((k_pcg_a<double, double>), dim3(M.nblk), dim3(kPB), 0, s, view<double>(*a.K), M, a.r, a.invD,
                       po, pn, a.q, a.st, phase_a, odd, a.part);
    hipLaunchKernelGGL((k_pcg_b<double, double>), dim3(M.nblk), dim3(kPB), 0, s, M, a.u, a.r, pn, a.q, a.invD, a.st,
                       phase_a + 1, odd, a.part);
}

void launch_pcg_iter32(const PcgLaunch &a, int phase_a, int odd, hipStream_t s) {
    const RowMap &M = *a.M;
    float *po = odd ? a.p32b : a.p32a, *pn = odd ? a.p32a : a.p32b;
    hipLaunchKernelGGL((k_pcg_a<float, float>), dim3(M.nblk), dim3(kPB), 0, s, view<float>(*a.K), M, a.r32, a.invD32,
                       po, pn, a.q32, a.st, phase_a, odd, a.part);
    hipLaunchKernelGGL((k_pcg_b<float, float>), dim3(M.nblk), dim3(kPB), 0, s, M, a.x32, a.r32, pn, a.q32, a.invD32,
                       a.st, phase_a + 1, odd, a.part);
}

void launch_add_correction(const PcgLaunch &a, hipStream_t s) {
    const RowMap &M = *a.M;
    hipLaunchKernelGGL(k_add_correction, dim3(M.nblk), dim3(kPB), 0, s, M, a.pin, a.u, a.x32);
}

}  // namespace mmncg
