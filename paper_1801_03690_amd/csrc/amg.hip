// Algebraic-multigrid preconditioned CG for the scalar-potential system
// K u = b (the paper preconditions its CG with algebraic multigrid, Sec. 3.1;
// the hierarchy is smoothed aggregation, built on the host in amg.cpp).
//
// The CG keeps the single-reduction form of the Jacobi path: one global
// reduction per iteration, read by the first kernel of the next iteration.
// With u = M r (one V(1,1) cycle) and w = K u:
//   gamma = r.u, delta = w.u, beta = gamma / gamma_prev,
//   alpha = gamma / (delta - beta gamma / alpha_prev),
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s.
// One iteration is a chain of launches:
//   k_amg_iter     scalars, the updates of own rows, and the first half of
//                  the fine pre-smoothing t = r - omega K D^-1 r: K D^-1 r of
//                  the new r is formed from the previous r, w, s records of
//                  the neighbours as in the Jacobi path (no extra pass);
//   coarse levels  restriction b_1 = P_0^T t_0; on each coarse level one
//                  sparse product down (pre-smoothing and restriction
//                  multiplied out) and one up (both smoothing sweeps and the
//                  coarse correction); a dense solve on the coarsest level;
//                  the prolongation z = omega D^-1 r + P_0 y_1;
//   k_amg_post0    u = z + omega D^-1 (r - K z) on the fine level, partial
//                  gamma;
//   k_amg_w        w = K u into a plain vector, partials delta and r.r.
// Every kernel of an iteration skips the rows of an instance whose sticky
// flag is up (the flag only changes inside k_amg_iter, which every later
// launch follows in stream order): the row-map kernels by their blocks'
// instance, the cycle's CSR and dense kernels through a per-row (per-entry)
// instance table. The
// cycle runs in VT (double in the FP64 mode, float in the mixed form of the
// FP32-bulk mode) and the CG vectors in RT (double); reductions are FP64.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace mmncg {

using namespace dev;

namespace {

constexpr int kAB = 256;  // threads per block of the coarse-level kernels
constexpr int kP0 = 0, kP1 = 3;

// rows of an instance whose stop flag is up (and padding rows) are skipped
// when st is given; iof[row] is the instance of the row (-1: padding), or
// iof is null for a single instance (one flag, no table)
__device__ __forceinline__ bool skip_row(const int *iof, const PcgState *st, int row) {
    if (!st) return false;
    if (!iof) return st[0].done;
    const int i = iof[row];
    return i < 0 || st[i].done;
}

// sum over the GL lanes of a row group (GL divides 64)
template <int GL, class VT>
__device__ __forceinline__ VT group_sum(VT v) {
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GL);
    return v;
}

// one CSR row times x, GL lanes per row; the row's sum in every lane of the group
template <int GL, class VT>
__device__ __forceinline__ VT csr_row(const int *__restrict__ p, const int *__restrict__ j,
                                      const VT *__restrict__ v, const VT *__restrict__ x, int row, int gl) {
    VT acc = 0;
    const int e1 = p[row + 1];
#pragma unroll 2
    for (int e = p[row] + gl; e < e1; e += GL) acc += v[e] * x[j[e]];
    return group_sum<GL>(acc);
}

// y = A x for a CSR matrix (the fine restriction R, and the fused down and up
// operators of the coarse levels; GL lanes per row)
template <class VT, int GL>
__global__ __launch_bounds__(kAB) void k_amg_spmv(int n, const int *__restrict__ p, const int *__restrict__ j,
                                                      const VT *__restrict__ v, const VT *__restrict__ x,
                                                      VT *__restrict__ y, const int *__restrict__ iof,
                                                      const PcgState *st) {
    const int row = (int)((blockIdx.x * (unsigned)kAB + threadIdx.x) / GL), gl = threadIdx.x % GL;
    if (row >= n || skip_row(iof, st, row)) return;
    const VT s = csr_row<GL>(p, j, v, x, row, gl);
    // rows without entries (padding; instances solved densely on this level) are not written
    if (gl == 0 && p[row + 1] > p[row]) y[row] = s;
}

// z = omega D^-1 b + P y on the fine level, omega D^-1 per row in wd (b at
// b[row * bs]: bs = 4 for the r field of the CG records, whose type RT may be
// wider than the cycle's VT)
template <class VT, class RT, int GL>
__global__ __launch_bounds__(kAB) void k_amg_prolong(int n, const int *__restrict__ p, const int *__restrict__ j,
                                                     const VT *__restrict__ v, const VT *__restrict__ wd,
                                                     const RT *__restrict__ b, int bs, const VT *__restrict__ yc,
                                                     VT *__restrict__ z, const int *__restrict__ iof,
                                                     const PcgState *st) {
    const int row = (int)((blockIdx.x * (unsigned)kAB + threadIdx.x) / GL), gl = threadIdx.x % GL;
    if (row >= n || skip_row(iof, st, row)) return;
    const VT s = csr_row<GL>(p, j, v, yc, row, gl);
    if (gl == 0) z[row] = wd[row] * (VT)b[(int64_t)row * bs] + s;
}

// y = Ainv b for the instances whose coarsest level this is: one wave per
// dense row; row r is row r - drow0[k] of table entry k = dinst[r] (instance
// dwho[k], or 0 when dwho is null; skipped once its flag is up when st is
// given), whose
// inverse starts at daoff[k] (rows dld[k] apart, a multiple of 4 values,
// padding zero) and whose b and y rows start at row dboff[k] of the level.
// With a plain b (bs = 1; each instance's block padded to dld with zeros)
// every lane loads 16 bytes of the row and of b at a time; with b in the CG
// records (bs = 4), one value.
template <class VT, class BT>
__global__ __launch_bounds__(kAB) void k_amg_dense(int nrows, const int *__restrict__ dinst,
                                                   const int *__restrict__ drow0, const int *__restrict__ dn,
                                                   const int *__restrict__ dld, const int64_t *__restrict__ daoff,
                                                   const int *__restrict__ dboff, const int *__restrict__ dwho,
                                                   const VT *__restrict__ Ainv, const BT *__restrict__ b, int bs,
                                                   VT *__restrict__ y, const PcgState *st) {
    const int r = (int)(blockIdx.x * (kAB / 64) + wave_id()), ln = lane_id();
    if (r >= nrows || (st && !dwho && st[0].done)) return;
    const int k = dinst[r];
    if (st && dwho && st[dwho[k]].done) return;
    const int row = r - drow0[k], n = dn[k], ld = dld[k], bo = dboff[k];
    const VT *a = Ainv + daoff[k] + (int64_t)row * ld;
    const BT *bb = b + (int64_t)bo * bs;
    VT acc = 0;
    if (bs == 1) {
        constexpr int V = 16 / sizeof(VT);
        typedef VT vec __attribute__((ext_vector_type(V)));
        const vec *av = (const vec *)a;
        const vec *bv = (const vec *)bb;
        for (int q = ln; q < ld / V; q += 64) {
            const vec x = av[q], w = bv[q];
#pragma unroll
            for (int e = 0; e < V; ++e) acc += x[e] * w[e];
        }
    } else {
        for (int c = ln; c < n; c += 64) acc += a[c] * (VT)bb[(int64_t)c * bs];
    }
    acc = group_sum<64>(acc);
    if (ln == 0) y[bo + row] = acc;
}

// one SELL row of K times x (and optionally times y entrywise: sum K_ac y_c
// x_c) with G column/value loads and gathers in flight per lane; entries past
// the slice's width stand in as the slice's first row with value 0. With NT
// the matrix loads are non-temporal (a matrix larger than the Infinity Cache
// then does not evict the vectors the gathers reuse).
template <class MT, class VT, bool TWO, bool NT>
__device__ __forceinline__ VT row_gather(const SV<MT> &K, int s, int ln, const VT *__restrict__ x, int xs,
                                         const VT *__restrict__ y) {
    constexpr int G = sizeof(VT) == 4 ? 8 : 4;
    const int64_t base = K.sptr[s];
    const int wd = (int)((K.sptr[s + 1] - base) >> 6);
    VT acc = 0;
    for (int k0 = 0; k0 < wd; k0 += G) {
        int cc[G];
        VT vv[G], xv[G], yv[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const bool in = k0 + k < wd;
            const int64_t e = base + 64 * (k0 + k) + ln;
            cc[k] = in ? (NT ? __builtin_nontemporal_load(K.col + e) : K.col[e]) : s * 64;
            vv[k] = in ? (VT)(NT ? __builtin_nontemporal_load(K.val + e) : K.val[e]) : (VT)0;
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
            xv[k] = x[(int64_t)cc[k] * xs];
            if (TWO) yv[k] = y[cc[k]];
        }
#pragma unroll
        for (int k = 0; k < G; ++k) acc += TWO ? vv[k] * (yv[k] * xv[k]) : vv[k] * xv[k];
    }
    return acc;
}

// fine level, start of a cycle from a residual that is not produced by
// k_amg_iter (the CG start, or a plain vector): t = r - omega K D^-1 r with r
// at r[row * rs] and the instance's omega. With q given (the CG start), also sets w = s = 0 and d =
// D^-1 in the records q (the r fields are left alone: neighbours read them).
template <class MT, class VT, class CT, int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void k_amg_pre0(SV<MT> K, RowMap M, const VT *__restrict__ r, int rs,
                                                      const VT *__restrict__ invD, const VT *__restrict__ om,
                                                      CT *__restrict__ t, PcgNode<VT> *__restrict__ q) {
    Tile tl = tile_of(M);
    if (tl.inst < 0) return;
    const VT omega = om[tl.inst];
    const int rend = M.rend[tl.inst], ln = lane_id();
    for (int s = tl.s0 + wave_id(); s < tl.s1; s += NW) {
        const VT acc = row_gather<MT, VT, true, NT>(K, s, ln, r, rs, invD);
        const int row = s * 64 + ln;
        if (row < rend) {
            t[row] = (CT)(r[(int64_t)row * rs] - omega * acc);
            if (q) {
                q[row].w = (VT)0;
                q[row].s = (VT)0;
                q[row].d = invD[row];
            }
        }
    }
}

// fine level: u = z + omega D^-1 (r - K z) (omega D^-1 per row in wd; with wd
// null, u = z: a single dense level) in the cycle's type VT, stored as the
// CG's type RT; partial gamma = r.u of the stored values into slot gslot
// (skipped when part is null); instances whose flag is up are skipped when
// st is given
template <class MT, class VT, class RT, int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void k_amg_post0(SV<MT> K, RowMap M, const RT *__restrict__ r, int rs,
                                                       const VT *__restrict__ wd, const VT *__restrict__ z,
                                                       RT *__restrict__ u, double *__restrict__ part, int gslot,
                                                       const PcgState *st) {
    Tile tl = tile_of(M);
    if (tl.inst < 0 || (st && st[tl.inst].done)) return;
    __shared__ double sh[NW];
    const int rend = M.rend[tl.inst], ln = lane_id();
    double acc[1] = {0};
    for (int s = tl.s0 + wave_id(); s < tl.s1; s += NW) {
        const VT kz = row_gather<MT, VT, false, NT>(K, s, ln, z, 1, (const VT *)nullptr);
        const int row = s * 64 + ln;
        if (row < rend) {
            const RT ri = r[(int64_t)row * rs];
            const RT ui = wd ? (RT)(z[row] + wd[row] * ((VT)ri - kz)) : (RT)z[row];
            u[row] = ui;
            acc[0] += (double)ri * (double)ui;
        }
    }
    if (part) write_part<1, NW>(acc, 0u, part + (size_t)gslot * M.nblk, M.nblk, tl.b, sh);
}

// fine level: w = K u into the plain vector wf (the records' w field is not
// used by the multigrid CG: a store of one 8-byte field into 32-byte records
// writes whole records back); partials (delta = w.u, r.r, with r at
// r[row * rs]) into slots wslot, wslot + 1
template <class MT, class VT, int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void k_amg_w(SV<MT> K, RowMap M, VT *__restrict__ wf,
                                                   const VT *__restrict__ r, int rs, const VT *__restrict__ u,
                                                   double *__restrict__ part, int wslot, const PcgState *st) {
    Tile tl = tile_of(M);
    if (tl.inst < 0 || (st && st[tl.inst].done)) return;
    __shared__ double sh[NW * 2];
    const int rend = M.rend[tl.inst], ln = lane_id();
    double acc[2] = {0, 0};
    for (int s = tl.s0 + wave_id(); s < tl.s1; s += NW) {
        const VT ku = row_gather<MT, VT, false, NT>(K, s, ln, u, 1, (const VT *)nullptr);
        const int row = s * 64 + ln;
        if (row < rend) {
            const VT ri = r[(int64_t)row * rs];
            wf[row] = ku;
            acc[0] += (double)ku * (double)u[row];
            acc[1] += (double)ri * (double)ri;
        }
    }
    write_part<2, NW>(acc, 0u, part + (size_t)wslot * M.nblk, M.nblk, tl.b, sh);
}

// K D^-1 times r, w and s of the neighbours (r, s and D^-1 from the records,
// w from the plain vector wf; one row of the slice, this lane)
template <class MT, class VT, bool NT>
__device__ __forceinline__ void row_abc(const SV<MT> &K, int s, int ln, const PcgNode<VT> *__restrict__ q0,
                                        const VT *__restrict__ wf, VT &pa, VT &pb, VT &pc) {
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
            cc[k] = in ? (NT ? __builtin_nontemporal_load(K.col + e) : K.col[e]) : s * 64;
            vv[k] = in ? (VT)(NT ? __builtin_nontemporal_load(K.val + e) : K.val[e]) : (VT)0;
        }
        PcgNode<VT> nq[G];
        VT nw[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            nq[k] = q0[cc[k]];
            nw[k] = wf[cc[k]];
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const VT kd = vv[k] * nq[k].d;
            pa += kd * nq[k].r;
            pb += kd * nw[k];
            pc += kd * nq[k].s;
        }
    }
}

// the updates of one CG iteration of parity par (reads records q[par], w in
// wf and the partials P[par]; writes records q[par ^ 1] (their w field unused:
// k_amg_w writes the new w to wf), and r_new once more as the plain vector rf,
// which the rest of the iteration reads instead of the records) and
// t = r_new - omega K D^-1 r_new,
// where K D^-1 r_new = A - alpha (B + beta C) with A, B, C the products of
// K D^-1 with the old r, w, s
template <class MT, class VT, class XT, class CT, int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void k_amg_iter(SV<MT> K, RowMap M, PcgVecs<VT> v, XT *__restrict__ x,
                                                      const VT *__restrict__ uu, CT *__restrict__ tt,
                                                      VT *__restrict__ rf, const VT *__restrict__ wf,
                                                      const VT *__restrict__ om,
                                                      PcgState *__restrict__ st, int par,
                                                      const double *__restrict__ part) {
    Tile tl = tile_of(M);
    if (tl.inst < 0) return;
    PcgState *si = st + tl.inst;
    __shared__ double sh[NW * 3];
    __shared__ int sdone;
    const int S = M.nblk, b0 = M.ipb[tl.inst], b1 = M.ipb[tl.inst + 1];
    const double *pp = part + (size_t)(par ? kP1 : kP0) * S;
    double g3[3] = {0, 0, 0};
    for (int i = b0 + (int)threadIdx.x; i < b1; i += NW * 64) {
        g3[0] += pp[i];
        g3[1] += pp[(size_t)S + i];
        g3[2] += pp[2 * (size_t)S + i];
    }
    if (threadIdx.x == 0) sdone = si->done;
    __syncthreads();
    if (sdone) return;
    const PcgNode<VT> *__restrict__ q0 = v.q[par];
    PcgNode<VT> *__restrict__ q1 = v.q[par ^ 1];
    VT *__restrict__ p = v.p;
    const int rend = M.rend[tl.inst], ln = lane_id();
    const double tol2 = si->tol2, gprev = si->gamma[par ^ 1], aprev = si->alpha[par ^ 1];
    const int sf = tl.s0 + wave_id();
    VT pa = 0, pb = 0, pc = 0;
    if (sf < tl.s1) row_abc<MT, VT, NT>(K, sf, ln, q0, wf, pa, pb, pc);
    block_reduce<3, NW>(g3, 0u, sh);
    const double gam = g3[0], del = g3[1], rr = g3[2];
    if (rr <= tol2) {
        if (tl.b == b0 && threadIdx.x == 0) si->done = 2 + par;
        return;
    }
    const double beta = gam / gprev;
    const double alpha = gam / (del - beta * gam / aprev);
    if (tl.b == b0 && threadIdx.x == 0) {
        si->gamma[par] = gam;
        si->alpha[par] = alpha;
        si->iters += 1;
    }
    const VT a = (VT)alpha, bt = (VT)beta, omega = om[tl.inst];
    for (int s = sf; s < tl.s1; s += NW) {
        if (s != sf) row_abc<MT, VT, NT>(K, s, ln, q0, wf, pa, pb, pc);
        const int row = s * 64 + ln;
        if (row < rend) {
            const PcgNode<VT> me = q0[row];
            const VT ui = uu[row];
            const VT wi = wf[row];
            const VT sn = bt != (VT)0 ? wi + bt * me.s : wi;
            const VT pn = bt != (VT)0 ? ui + bt * p[row] : ui;
            const VT rn = me.r - a * sn;
            const VT kdr = bt != (VT)0 ? pa - a * (pb + bt * pc) : pa - a * pb;
            x[row] = x[row] + (XT)(a * pn);
            p[row] = pn;
            q1[row] = PcgNode<VT>{rn, (VT)0, sn, me.d};
            rf[row] = rn;
            tt[row] = (CT)(rn - omega * kdr);
        }
    }
}

}  // namespace

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

// lanes per row of a CSR kernel: chosen per matrix from its mean row length
#define MMNCG_GL_SWITCH(gl, ...)            \
    switch (gl) {                           \
        case 1: {                           \
            constexpr int GL = 1;           \
            __VA_ARGS__;                    \
        } break;                            \
        case 2: {                           \
            constexpr int GL = 2;           \
            __VA_ARGS__;                    \
        } break;                            \
        case 4: {                           \
            constexpr int GL = 4;           \
            __VA_ARGS__;                    \
        } break;                            \
        case 8: {                           \
            constexpr int GL = 8;           \
            __VA_ARGS__;                    \
        } break;                            \
        case 16: {                          \
            constexpr int GL = 16;          \
            __VA_ARGS__;                    \
        } break;                            \
        case 32: {                          \
            constexpr int GL = 32;          \
            __VA_ARGS__;                    \
        } break;                            \
        default: {                          \
            constexpr int GL = 64;          \
            __VA_ARGS__;                    \
        } break;                            \
    }

namespace {

template <int GL>
dim3 grid_rows(int n) {
    const int64_t th = (int64_t)n * GL;
    return dim3((unsigned)((th + kAB - 1) / kAB));
}

template <class VT>
const int *iof_of(const AmgLaunch<VT> &g, const AmgLevel<VT> &lv) {
    return g.single ? nullptr : lv.iof;
}

template <class VT, class BT>
void dense(const AmgLevel<VT> &lv, bool single, const BT *b, int bs, VT *y, const PcgState *st, hipStream_t s) {
    if (lv.ndense > 0)
        hipLaunchKernelGGL((k_amg_dense<VT, BT>), dim3((unsigned)((lv.ndense + kAB / 64 - 1) / (kAB / 64))),
                           dim3(kAB), 0, s, lv.ndense, lv.dinst, lv.drow0, lv.dn, lv.dld, lv.daoff, lv.dboff,
                           single ? (const int *)nullptr : lv.dwho, lv.Ainv, b, bs, y, st);
}

// everything between the fine pre-smoothing and the fine post-smoothing:
// z0 = omega D^-1 r + P V(P^T t0) with r at r[row * rs] (of the CG's type RT):
// the restriction, the fused operators of the coarse levels down, the dense
// solves of the instances that end on each level, the fused operators up,
// and the prolongation. With a single level (one instance, n_pot small),
// z0 = K^-1 r from the dense inverse.
template <class VT, class RT>
void lower_cycle(const AmgLaunch<VT> &g, const RT *r, int rs, const PcgState *st, hipStream_t s) {
    const AmgLevel<VT> &f = g.lv[0];
    if (g.nlev == 1) {
        dense(f, g.single, r, rs, f.z, st, s);
        return;
    }
    const int L = g.nlev - 1;
    const AmgLevel<VT> &c1 = g.lv[1];
    MMNCG_GL_SWITCH(f.gR, hipLaunchKernelGGL((k_amg_spmv<VT, GL>), grid_rows<GL>(c1.n), dim3(kAB), 0, s, c1.n, f.Rp,
                                             f.Rj, f.Rv, (const VT *)f.t, c1.b, iof_of(g, c1), st))
    for (int l = 1; l < L; ++l) {
        const AmgLevel<VT> &a = g.lv[l], &c = g.lv[l + 1];
        MMNCG_GL_SWITCH(a.gD, hipLaunchKernelGGL((k_amg_spmv<VT, GL>), grid_rows<GL>(c.n), dim3(kAB), 0, s, c.n,
                                                 a.Dp, a.Dj, a.Dv, (const VT *)a.b, c.b, iof_of(g, c), st))
    }
    for (int l = L; l >= 1; --l) {
        const AmgLevel<VT> &a = g.lv[l];
        dense(a, g.single, (const VT *)a.b, 1, a.y, st, s);
        // [b_l; y_{l+1}] is one array starting at b_l
        if (l < L)
            MMNCG_GL_SWITCH(a.gU, hipLaunchKernelGGL((k_amg_spmv<VT, GL>), grid_rows<GL>(a.n), dim3(kAB), 0, s, a.n,
                                                     a.Up, a.Uj, a.Uv, (const VT *)a.b, a.y, iof_of(g, a), st))
    }
    MMNCG_GL_SWITCH(f.gP, hipLaunchKernelGGL((k_amg_prolong<VT, RT, GL>), grid_rows<GL>(f.n), dim3(kAB), 0, s, f.n,
                                             f.Pp, f.Pj, f.Pv, (const VT *)f.wd, r, rs, (const VT *)c1.y, f.z, iof_of(g, f),
                                             st))
}

// The fine-level vectors of the CG (records, direction, u) are of type RT;
// the cycle and the stored fine matrix used inside it and by the CG are of
// type VT (VT = RT = double in the FP64 solve; VT = float, RT = double in
// the mixed solve: FP32-stored operators and cycle, FP64 Krylov vectors).
template <class VT, class RT>
struct FineArgs {
    const RT *invD;    // D^-1 of the records
    const RT *omega;   // per instance, the fine smoothing weight in RT
    RT *u;             // preconditioned residual
    RT *rf;            // the residual as a plain vector (written by k_amg_iter)
    RT *wf;            // w = K u as a plain vector (written by k_amg_w)
};

template <class VT>
const VT *post_wd(const AmgLaunch<VT> &g) {
    return g.nlev > 1 ? g.lv[0].wd : nullptr;
}

// one cycle on the fine level from the residual r (at r[row * rs]) into u;
// with a CG, also the records' start fields (q) and the partials of the
// start (gamma, then delta and r.r in P0)
// matrices whose stored entries (value + column index) exceed this stay out
// of the Infinity Cache between passes and are loaded non-temporally
constexpr int64_t kStreamMatrixBytes = int64_t(128) << 20;
template <class VT>
bool stream_matrix(const PcgLaunch &a) {
    return a.K->padded * int64_t(sizeof(VT) + sizeof(int)) > kStreamMatrixBytes;
}

template <class VT, class RT, bool NT>
void fine_cycle_nt(const PcgLaunch &a, const AmgLaunch<VT> &g, const FineArgs<VT, RT> &fa, const RT *r, int rs,
                   PcgNode<RT> *q, bool cg, hipStream_t s) {
    const RowMap &M = *a.M;
    const AmgLevel<VT> &f = g.lv[0];
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_amg_pre0<VT, RT, VT, NW, NT>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                             view<VT>(*a.K), M, r, rs, fa.invD, fa.omega, f.t, q))
    lower_cycle(g, r, rs, (const PcgState *)nullptr, s);
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_amg_post0<VT, VT, RT, NW, NT>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                             view<VT>(*a.K), M, r, rs, post_wd(g), (const VT *)f.z, fa.u,
                                             cg ? a.part : (double *)nullptr, kP0, (const PcgState *)nullptr))
    if (cg)
        MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_amg_w<VT, RT, NW, NT>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                                 view<VT>(*a.K), M, fa.wf, r, rs, (const RT *)fa.u, a.part, kP0 + 1,
                                                 (const PcgState *)nullptr))
}

template <class VT, class RT>
void fine_cycle(const PcgLaunch &a, const AmgLaunch<VT> &g, const FineArgs<VT, RT> &fa, const RT *r, int rs,
                PcgNode<RT> *q, bool cg, hipStream_t s) {
    // t (unused with a single level) and the records' start fields
    if (stream_matrix<VT>(a))
        fine_cycle_nt<VT, RT, true>(a, g, fa, r, rs, q, cg, s);
    else
        fine_cycle_nt<VT, RT, false>(a, g, fa, r, rs, q, cg, s);
}

template <class VT, class RT, class XT, bool NT>
void amg_iter_nt(const PcgLaunch &a, const AmgLaunch<VT> &g, const FineArgs<VT, RT> &fa, const PcgVecs<RT> &v, XT *x,
                 int par, hipStream_t s) {
    const RowMap &M = *a.M;
    const AmgLevel<VT> &f = g.lv[0];
    PcgNode<RT> *q1 = v.q[par ^ 1];
    const int ws = par ? kP0 : kP1;  // this iteration's new partials
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_amg_iter<VT, RT, XT, VT, NW, NT>), dim3(M.nblk), dim3(NW * 64), 0,
                                             s, view<VT>(*a.K), M, v, x, (const RT *)fa.u, f.t, fa.rf,
                                             (const RT *)fa.wf, fa.omega, a.st, par, (const double *)a.part))
    const RT *rf = fa.rf;
    // a single dense level takes b from the records (its plain-b path loads
    // VT vectors padded with zeros, which rf is not)
    if (g.nlev > 1) lower_cycle(g, rf, 1, (const PcgState *)a.st, s);
    else lower_cycle(g, (const RT *)&q1->r, 4, (const PcgState *)a.st, s);
    MMNCG_NW_SWITCH(a.nw, hipLaunchKernelGGL((k_amg_post0<VT, VT, RT, NW, NT>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                             view<VT>(*a.K), M, rf, 1, post_wd(g), (const VT *)f.z, fa.u, a.part,
                                             ws, (const PcgState *)a.st);
                    hipLaunchKernelGGL((k_amg_w<VT, RT, NW, NT>), dim3(M.nblk), dim3(NW * 64), 0, s,
                                       view<VT>(*a.K), M, fa.wf, rf, 1, (const RT *)fa.u, a.part, ws + 1,
                                       (const PcgState *)a.st))
}

template <class VT, class RT, class XT>
void amg_iter(const PcgLaunch &a, const AmgLaunch<VT> &g, const FineArgs<VT, RT> &fa, const PcgVecs<RT> &v, XT *x,
              int par, hipStream_t s) {
    if (stream_matrix<VT>(a)) amg_iter_nt<VT, RT, XT, true>(a, g, fa, v, x, par, s);
    else amg_iter_nt<VT, RT, XT, false>(a, g, fa, v, x, par, s);
}

FineArgs<double, double> fine64(const PcgLaunch &a, const AmgLaunch<double> &g) {
    return FineArgs<double, double>{a.invD, g.omega, g.u, g.rf, g.wf};
}
FineArgs<float, float> fine32(const PcgLaunch &a, const AmgLaunch<float> &g) {
    return FineArgs<float, float>{a.invD32, g.omega, g.u, (float *)nullptr, (float *)nullptr};
}
FineArgs<float, double> finemix(const PcgLaunch &a, const AmgLaunch<double> &g64) {
    return FineArgs<float, double>{a.invD, g64.omega, g64.u, g64.rf, g64.wf};
}

}  // namespace

void launch_amg_init64(const PcgLaunch &a, const AmgLaunch<double> &g, const int *act, double rtol2, hipStream_t s) {
    launch_pcg_residual_q(a, act, false, s);
    fine_cycle<double, double>(a, g, fine64(a, g), &a.v64.q[0]->r, 4, a.v64.q[0], true, s);
    launch_pcg_fin(a, act, rtol2, 0, s);
}

void launch_amg_initmix(const PcgLaunch &a, const AmgLaunch<float> &g, const AmgLaunch<double> &g64, const int *act,
                        double rtol2, hipStream_t s) {
    launch_pcg_residual_q(a, act, true, s);
    fine_cycle<float, double>(a, g, finemix(a, g64), &a.v64.q[0]->r, 4, a.v64.q[0], true, s);
    launch_pcg_fin(a, act, rtol2, 0, s);
}

void launch_amg_iter64(const PcgLaunch &a, const AmgLaunch<double> &g, int parity, hipStream_t s) {
    amg_iter<double, double, double>(a, g, fine64(a, g), a.v64, a.u, parity, s);
}

void launch_amg_itermix(const PcgLaunch &a, const AmgLaunch<float> &g, const AmgLaunch<double> &g64, int parity,
                        hipStream_t s) {
    amg_iter<float, double, double>(a, g, finemix(a, g64), a.v64, a.u, parity, s);
}

void launch_amg_apply64(const PcgLaunch &a, const AmgLaunch<double> &g, const double *r, hipStream_t s) {
    fine_cycle<double, double>(a, g, fine64(a, g), r, 1, (PcgNode<double> *)nullptr, false, s);
}

void launch_amg_apply32(const PcgLaunch &a, const AmgLaunch<float> &g, const float *r, hipStream_t s) {
    fine_cycle<float, float>(a, g, fine32(a, g), r, 1, (PcgNode<float> *)nullptr, false, s);
}

}  // namespace mmncg
