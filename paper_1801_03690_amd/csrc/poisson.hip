// Scalar-potential solve K u = b (the magnetostatic subproblem of every energy
// evaluation; the paper solves it with preconditioned CG, Sec. 3.1) by
// Jacobi-preconditioned CG on gfx950, for every instance of a batch at once.
//
// The CG runs in its single-reduction form (Chronopoulos and Gear), which
// produces the iterates of preconditioned CG in exact arithmetic but needs
// one global reduction per iteration. With u = D^-1 r and w = K u:
//   gamma = r.u, delta = w.u, beta = gamma / gamma_prev,
//   alpha = gamma / (delta - beta gamma / alpha_prev),
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//   w = K D^-1 r (new r), partials of the new gamma, delta and r.r.
// A kernel boundary is the only grid-wide synchronization used, so one kernel
// is one iteration: it re-reduces the previous kernel's partials of its own
// instance in a fixed order (every block of the instance gets the same
// scalars; no fences, no floating-point atomics), updates its own rows, and
// forms K u_new where the neighbour values u_new = D^-1 (r - alpha (w + beta
// s)) are computed on the fly from the previous iteration's r, w and s, kept
// per node in one record with D^-1 (one load per stored matrix entry). The
// records are double-buffered by iteration parity, so no block reads a value
// another block is overwriting. Every launch of a chunk of iterations
// has fixed arguments: the chunk is captured once into a HIP graph and
// replayed until every instance's flag reports convergence. Once an
// instance's flag is up, every later kernel of it returns at once, in this
// replay and in any further one (replays are launched ahead of the host
// seeing the flag). All blocks of an iteration take the same convergence
// decision from the same partials, so a block that already sees the flag
// raised by its own launch behaves as if it had decided itself.
//
// Vector type VT is double (FP64 mode) or float (inner solve of the FP32-bulk
// mode, wrapped in FP64 defect correction); reductions are always FP64.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace mmncg {

using namespace dev;

namespace {

// Poisson kernels run blocks of NW waves (4, 8 or 16; one SELL slice per wave
// at a time), at most kMaxBlocksPerInst blocks per instance; the block shape
// and the slices per block of each instance come from the row map and the
// launch (autotuned or defaults).
constexpr int kFinBlock = 256;  // one block per instance for the start reductions
constexpr int kFinW = kFinBlock / 64;

// partial slots (slot q at part + q * stride):
//   P0 = 0-2, P1 = 3-5 (gamma, delta, r.r for iterations of even / odd
//   parity to read), INIT = 6-7 (b.b, r.r of the start residual)
constexpr int kP0 = 0, kP1 = 3, kINIT = 6;

__device__ __forceinline__ double *slot(double *part, int stride, int q) { return part + (size_t)q * stride; }
__device__ __forceinline__ const double *slot(const double *part, int stride, int q) {
    return part + (size_t)q * stride;
}

// r = b - K u; partials (b.b, r.r)
// (r at r[row * rs]: rs = 1 for a plain array, 4 for the r field of PcgNode<double>)
template <class MT, int NW>
__global__ __launch_bounds__(NW * 64) void k_pcg_residual(SV<MT> K, RowMap M, const int *__restrict__ act,
                                                      const double *__restrict__ b, const double *__restrict__ u,
                                                      double *__restrict__ r, int rs, double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0 || (act && !act[t.inst])) return;
    __shared__ double sh[NW * 2];
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[2] = {0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double ku = row_scalar<sizeof(MT) == 4 ? 8 : 4>(K, s, ln, u);
        int row = s * 64 + ln;
        if (row < rend) {
            double bi = b[row];
            double ri = bi - ku;
            r[(int64_t)row * rs] = ri;
            acc[0] += bi * bi;
            acc[1] += ri * ri;
        }
    }
    write_part<2, NW>(acc, 0u, slot(part, M.nblk, kINIT), M.nblk, t.b, sh);
}

// start of the FP32 inner solve K x = r64 * scale_i: x = 0, r32 = r64 * scale_i
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_pcg_start32(RowMap M, const double *__restrict__ pin,
                                                     const double *__restrict__ r64, float *__restrict__ x,
                                                     PcgNode<float> *__restrict__ q) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !(pin[4 * t.inst + 1] > 0.0)) return;
    const double scale = pin[4 * t.inst];
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int i = s * 64 + lane_id();
        if (i < rend) {
            x[i] = 0.0f;
            q[i].r = (float)(r64[i] * scale);
        }
    }
}

// w = K D^-1 r for the start residual (r in the records of buffer 0); writes
// whole records {r, w, 0, D^-1} of buffer 0 (a store of single fields would
// write the whole record back anyway; the first iteration writes whole
// records of buffer 1). Neighbours read only the r field, which the store
// rewrites with the value it already holds. Partials (gamma, delta, r.r)
// into P0. Entries go in groups as in row_abc. Active instances: act[i] when
// act is given, else those with an inner solve.
template <class MT, class VT, int NW>
__global__ __launch_bounds__(NW * 64) void k_pcg_start_w(SV<MT> K, RowMap M, const int *__restrict__ act,
                                                     const double *__restrict__ pin, PcgNode<VT> *__restrict__ q0,
                                                     const VT *__restrict__ invD, double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    if (act ? !act[t.inst] : !(pin[4 * t.inst + 1] > 0.0)) return;
    __shared__ double sh[NW * 3];
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[3] = {0, 0, 0};
    constexpr int G = sizeof(VT) == 4 ? 8 : 4;
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        const int64_t base = K.sptr[s];
        const int wd = (int)((K.sptr[s + 1] - base) >> 6);
        VT wv = 0;
#pragma unroll 1
        for (int k0 = 0; k0 < wd; k0 += G) {
            int cc[G];
            VT vv[G], dd[G], rn[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (k0 + k < wd) {
                    const int64_t e = base + 64 * (k0 + k) + ln;
                    cc[k] = K.col[e];
                    vv[k] = (VT)K.val[e];
                }
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (k0 + k < wd) {
                    dd[k] = invD[cc[k]];
                    rn[k] = q0[cc[k]].r;
                }
            }
#pragma unroll
            for (int k = 0; k < G; ++k)
                if (k0 + k < wd) wv += vv[k] * (dd[k] * rn[k]);
        }
        int row = s * 64 + ln;
        if (row < rend) {
            const VT ri = q0[row].r, di = invD[row];
            const VT ui = di * ri;
            q0[row] = PcgNode<VT>{ri, wv, (VT)0, di};
            acc[0] += (double)ri * (double)ui;
            acc[1] += (double)wv * (double)ui;
            acc[2] += (double)ri * (double)ri;
        }
    }
    write_part<3, NW>(acc, 0u, slot(part, M.nblk, kP0), M.nblk, t.b, sh);
}

// one block per instance: reduce the start partials into the instance's CG
// state and seed the scalar ring so that the first iteration has beta = 0.
// mode 0: CG start, tol2 = rtol2 * b.b; mode 1: FP32 inner start, tol2 =
// pin[1] * r.r (inactive when pin[1] <= 0); mode 2: residual only (no CG).
__global__ __launch_bounds__(kFinBlock) void k_pcg_init_fin(RowMap M, const double *__restrict__ part, double rtol2,
                                                      int mode, const int *__restrict__ act,
                                                      const double *__restrict__ pin, PcgState *__restrict__ st) {
    __shared__ double sh[kFinW * 3];
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
    double ini[2] = {0, 0}, p0[3] = {0, 0, 0};
    if (mode != 1) read_part<2, kFinW>(slot(part, S, kINIT), S, b0, b1, 0u, ini, sh);
    if (mode != 2) read_part<3, kFinW>(slot(part, S, kP0), S, b0, b1, 0u, p0, sh);
    const double bb = ini[0], rr = (mode == 1) ? p0[2] : ini[1];
    const double tol2 = (mode == 1) ? pin[4 * i + 1] * rr : rtol2 * bb;
    if (threadIdx.x == 0) {
        st[i].bb = bb;
        st[i].rr = rr;
        st[i].tol2 = tol2;
        st[i].iters = 0;
        st[i].active = 1;
        st[i].zero_u = (mode != 1 && bb == 0.0) ? 1 : 0;
        st[i].done = (mode == 2 || (mode != 1 && bb == 0.0) || rr <= tol2) ? 1 : 0;
        // iteration 0 reads slot 1: gamma_prev = inf gives beta = 0
        st[i].gamma[1] = __builtin_huge_val();
        st[i].alpha[1] = 1.0;
    }
}

// A, B, C of one row: sums over the slice's entries of K_ac D_c^-1 times r_c,
// w_c and s_c, from the neighbour records. Entries go in groups (8 in FP32,
// 4 in FP64) whose column/value loads and record gathers are all issued
// before any is used, so a wave keeps several gathers in flight. Entries past
// the slice's width stand in as the slice's first row (a row of the same
// instance) with value 0; the width is uniform over the wave, so those lanes
// issue no loads of matrix storage. With NT the matrix loads are marked
// non-temporal: a matrix too large to stay in the Infinity Cache between
// iterations then does not evict the records the gathers reuse.
template <class MT, class VT, bool NT>
__device__ __forceinline__ void row_abc(const SV<MT> &K, int s, int ln, const PcgNode<VT> *__restrict__ q0, VT &pa,
                                        VT &pb, VT &pc) {
    constexpr int G = sizeof(VT) == 4 ? 8 : 4;
    const int64_t base = K.sptr[s];
    const int wd = (int)((K.sptr[s + 1] - base) >> 6);
    pa = pb = pc = (VT)0;
    for (int k0 = 0; k0 < wd; k0 += G) {
        int cc[G];
        VT vv[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const bool in = k0 + k < wd;
            const int64_t e = base + 64 * (k0 + k) + ln;
            if (NT) {
                cc[k] = in ? __builtin_nontemporal_load(K.col + e) : s * 64;
                vv[k] = in ? (VT)__builtin_nontemporal_load(K.val + e) : (VT)0;
            } else {
                cc[k] = in ? K.col[e] : s * 64;
                vv[k] = in ? (VT)K.val[e] : (VT)0;
            }
        }
        PcgNode<VT> nq[G];
#pragma unroll
        for (int k = 0; k < G; ++k) nq[k] = q0[cc[k]];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const VT kd = vv[k] * nq[k].d;
            pa += kd * nq[k].r;
            pb += kd * nq[k].w;
            pc += kd * nq[k].s;
        }
    }
}

// one CG iteration of parity `par`: reads r, w, s of buffer par and the
// partials P[par]; writes buffer par ^ 1 and P[par ^ 1].
// w_new = K D^-1 (r - alpha (w + beta s)) is formed as A - alpha (B + beta C)
// with A, B, C the products of K D^-1 with r, w and s: these do not depend on
// the iteration's scalars, so the matrix gathers of a wave's first slice are
// issued before the block has reduced the previous partials.
template <class MT, class VT, class XT, int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void k_pcg_iter(SV<MT> K, RowMap M, PcgVecs<VT> v, XT *__restrict__ x,
                                                      const VT *__restrict__ invD, PcgState *__restrict__ st, int par,
                                                      double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    PcgState *si = st + t.inst;
    __shared__ double sh[NW * 3];
    __shared__ int sdone;
    const int S = M.nblk, b0 = M.ipb[t.inst], b1 = M.ipb[t.inst + 1];
    const double *pp = slot((const double *)part, S, par ? kP1 : kP0);
    double g3[3] = {0, 0, 0};
    for (int i = b0 + (int)threadIdx.x; i < b1; i += NW * 64) {
        g3[0] += pp[i];
        g3[1] += pp[(size_t)S + i];
        g3[2] += pp[2 * (size_t)S + i];
    }
    // the flag is read once per block, so every wave of the block takes the
    // same branch even while another block raises it
    if (threadIdx.x == 0) sdone = si->done;
    __syncthreads();
    if (sdone) return;
    const PcgNode<VT> *__restrict__ q0 = v.q[par];
    PcgNode<VT> *__restrict__ q1 = v.q[par ^ 1];
    VT *__restrict__ p = v.p;
    const int rend = M.rend[t.inst], ln = lane_id();
    // everything of the wave's first slice that does not depend on this
    // iteration's scalars is loaded before the block reduces the partials:
    // the instance's CG scalars, the matrix products and the own-row values
    const double tol2 = si->tol2, gprev = si->gamma[par ^ 1], aprev = si->alpha[par ^ 1];
    const int sf = t.s0 + wave_id();
    const int rf = sf * 64 + ln;
    VT pa = 0, pb = 0, pc = 0;
    if (sf < t.s1) row_abc<MT, VT, NT>(K, sf, ln, q0, pa, pb, pc);
    PcgNode<VT> me_f{0, 0, 0, 0};
    VT p_f = 0;
    XT x_f = 0;
    if (sf < t.s1 && rf < rend) {
        me_f = q0[rf];
        p_f = p[rf];
        x_f = x[rf];
    }
    block_reduce<3, NW>(g3, 0u, sh);
    const double gam = g3[0], del = g3[1], rr = g3[2];
    if (rr <= tol2) {
        if (t.b == b0 && threadIdx.x == 0) si->done = 2 + par;
        return;
    }
    const double beta = gam / gprev;
    const double alpha = gam / (del - beta * gam / aprev);
    if (t.b == b0 && threadIdx.x == 0) {
        si->gamma[par] = gam;
        si->alpha[par] = alpha;
        si->iters += 1;
    }
    const VT a = (VT)alpha, bt = (VT)beta;
    double acc[3] = {0, 0, 0};
    for (int s = sf; s < t.s1; s += NW) {
        if (s != sf) row_abc<MT, VT, NT>(K, s, ln, q0, pa, pb, pc);
        int row = s * 64 + ln;
        if (row < rend) {
            const PcgNode<VT> me = (s == sf) ? me_f : q0[row];
            const VT pold = (s == sf) ? p_f : p[row];
            const XT xold = (s == sf) ? x_f : x[row];
            const VT dinv = me.d, ri = me.r;
            VT sn = bt != (VT)0 ? me.w + bt * me.s : me.w;
            VT pn = bt != (VT)0 ? dinv * ri + bt * pold : dinv * ri;
            VT rn = ri - a * sn;
            VT wn = bt != (VT)0 ? pa - a * (pb + bt * pc) : pa - a * pb;
            x[row] = xold + (XT)(a * pn);
            p[row] = pn;
            // whole record in one store (partial-record stores leave every
            // cache line partly written)
            q1[row] = PcgNode<VT>{rn, wn, sn, dinv};
            VT un = dinv * rn;
            acc[0] += (double)rn * (double)un;
            acc[1] += (double)wn * (double)un;
            acc[2] += (double)rn * (double)rn;
        }
    }
    write_part<3, NW>(acc, 0u, slot(part, S, par ? kP0 : kP1), S, t.b, sh);
}

// u += rn_i * x32 for the instances with an inner solve
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_add_correction(RowMap M, const double *__restrict__ pin, double *__restrict__ u,
                                                        const float *__restrict__ x) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !(pin[4 * t.inst + 1] > 0.0)) return;
    const double sc = pin[4 * t.inst + 2];
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int i = s * 64 + lane_id();
        if (i < rend) u[i] += sc * (double)x[i];
    }
}

}  // namespace

// instantiate the launch for the block shape of the row map
#define MMNCG_NW_SWITCH(nw, ...)            \
    switch (nw) {                           \
        case 4: {                           \
            constexpr int NW = 4;           \
            __VA_ARGS__;                    \
        } break;                            \
        case 8: {                           \
            constexpr int NW = 8;           \
            __VA_ARGS__;                    \
        } break;                            \
        default: {                          \
            constexpr int NW = 16;          \
            __VA_ARGS__;                    \
        } break;                            \
    }

void launch_pcg_init64(const PcgLaunch &a, const int *act, double rtol2, hipStream_t s) {
    const RowMap &M = *a.M;
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_residual<double, NW>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                             view<double>(*a.K), M, act, a.b, a.u, &a.v64.q[0]->r, 4, a.part);
                    hipLaunchKernelGGL((k_pcg_start_w<double, double, NW>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                       view<double>(*a.K), M, act, a.pin, a.v64.q[0], a.invD, a.part))
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kFinBlock), 0, s, M, (const double *)a.part, rtol2, 0, act,
                       a.pin, a.st);
}

void launch_residual64(const PcgLaunch &a, const int *act, hipStream_t s) {
    const RowMap &M = *a.M;
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_residual<float, NW>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                             view<float>(*a.K), M, act, a.b, a.u, a.r64, 1, a.part))
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kFinBlock), 0, s, M, (const double *)a.part, 0.0, 2, act,
                       a.pin, a.st);
}

void launch_pcg_init32(const PcgLaunch &a, hipStream_t s) {
    const RowMap &M = *a.M;
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_start32<NW>), dim3(M.nblk), dim3(NW * 64), 0, s, M, a.pin,
                                             (const double *)a.r64, a.x32, a.v32.q[0]);
                    hipLaunchKernelGGL((k_pcg_start_w<float, float, NW>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                       view<float>(*a.K), M, (const int *)nullptr, a.pin, a.v32.q[0], a.invD32,
                                       a.part))
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kFinBlock), 0, s, M, (const double *)a.part, 0.0, 1,
                       (const int *)nullptr, a.pin, a.st);
}

// matrices whose stored entries (value + column index) exceed this stay out
// of the Infinity Cache between iterations and are loaded non-temporally
constexpr int64_t kStreamMatrixBytes = int64_t(128) << 20;

void launch_pcg_iter64(const PcgLaunch &a, int parity, hipStream_t s) {
    const RowMap &M = *a.M;
    if (a.K->padded * int64_t(sizeof(double) + sizeof(int)) > kStreamMatrixBytes)
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_iter<double, double, double, NW, true>), dim3(M.nblk),
                                                 dim3(NW * 64), 0, s, view<double>(*a.K), M, a.v64, a.u, a.invD, a.st,
                                                 parity, a.part))
    else
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_iter<double, double, double, NW, false>), dim3(M.nblk),
                                                 dim3(NW * 64), 0, s, view<double>(*a.K), M, a.v64, a.u, a.invD, a.st,
                                                 parity, a.part))
}

void launch_pcg_iter32(const PcgLaunch &a, int parity, hipStream_t s) {
    const RowMap &M = *a.M;
    if (a.K->padded * int64_t(sizeof(float) + sizeof(int)) > kStreamMatrixBytes)
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_iter<float, float, float, NW, true>), dim3(M.nblk),
                                                 dim3(NW * 64), 0, s, view<float>(*a.K), M, a.v32, a.x32, a.invD32,
                                                 a.st, parity, a.part))
    else
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_iter<float, float, float, NW, false>), dim3(M.nblk),
                                                 dim3(NW * 64), 0, s, view<float>(*a.K), M, a.v32, a.x32, a.invD32,
                                                 a.st, parity, a.part))
}

void launch_pcg_residual_q(const PcgLaunch &a, const int *act, bool fp32_matrix, hipStream_t s) {
    const RowMap &M = *a.M;
    if (fp32_matrix)
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_residual<float, NW>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                                 view<float>(*a.K), M, act, a.b, a.u, &a.v64.q[0]->r, 4, a.part))
    else
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_residual<double, NW>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                                 view<double>(*a.K), M, act, a.b, a.u, &a.v64.q[0]->r, 4, a.part))
}

void launch_pcg_start32_only(const PcgLaunch &a, hipStream_t s) {
    const RowMap &M = *a.M;
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_pcg_start32<NW>), dim3(M.nblk), dim3(NW * 64), 0, s, M, a.pin,
                                             (const double *)a.r64, a.x32, a.v32.q[0]))
}

void launch_pcg_fin(const PcgLaunch &a, const int *act, double rtol2, int mode, hipStream_t s) {
    const RowMap &M = *a.M;
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(M.ninst), dim3(kFinBlock), 0, s, M, (const double *)a.part, rtol2, mode,
                       act, a.pin, a.st);
}

void launch_add_correction(const PcgLaunch &a, hipStream_t s) {
    const RowMap &M = *a.M;
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_add_correction<NW>), dim3(M.nblk), dim3(NW * 64), 0, s, M, a.pin,
                                             a.u, a.x32))
}

}  // namespace mmncg
