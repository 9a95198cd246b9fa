// HIP kernels (gfx950) of the micromagnetic PNCG hot path.
//
// Layout. Every sparse operator is stored SELL-64: a wavefront owns a slice of
// 64 consecutive rows, one row per lane, and walks the slice's entries
// column-major, so the k-th load of the wave reads 64 consecutive values and
// 64 consecutive column indices (one 512 B / 256 B coalesced transaction).
// Vectors on magnet nodes are node-major AoS doubles (x, y, z); vectors on
// potential nodes are plain arrays. A block of 256 threads (4 waves) owns a
// contiguous range of slices; blocks are renumbered so that each of the 8 XCDs
// (blocks are dealt round-robin to XCDs) gets one contiguous eighth of the
// rows, keeping the neighbour gathers of a row range inside one L2.
//
// Reductions are deterministic: each block writes one partial per quantity
// into a fixed slot, and the consumer (the next kernel, every block of it, or
// a one-block finalize kernel) re-reduces the partials in a fixed order. No
// floating-point atomics anywhere, so repeated runs are bitwise identical.
//
// Operator values may be stored in FP32 (template parameter V) for the
// FP32-bulk mode; products and sums are always formed in FP64 except in the
// FP32 inner Poisson CG, whose vectors are FP32 and whose dot products are
// accumulated in FP64.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace mmncg {

using namespace dev;

namespace {

// ---------------------------------------------------------------------------
// plain operator kernels (used by the checking ABI and as building blocks)
// ---------------------------------------------------------------------------
template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_block6(SV<V> A, const double *__restrict__ x, double *__restrict__ y) {
    int s0, s1;
    slice_range(A.nslices, s0, s1);
    int ln = lane_id();
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        double o0, o1, o2;
        row_block6(A, s, ln, x, o0, o1, o2);
        int row = s * 64 + ln;
        if (row < A.nrows) {
            y[3 * (int64_t)row] = o0;
            y[3 * (int64_t)row + 1] = o1;
            y[3 * (int64_t)row + 2] = o2;
        }
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_scalar(SV<V> A, const double *__restrict__ x, double *__restrict__ y) {
    int s0, s1;
    slice_range(A.nslices, s0, s1);
    int ln = lane_id();
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        double o = row_scalar(A, s, ln, x);
        int row = s * 64 + ln;
        if (row < A.nrows) y[row] = o;
    }
}

// scalar rows applied to node-major 3-vectors: y_i = sum_k a_k x_{c_k} (each component)
template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_scalar3(SV<V> A, const double *__restrict__ x, double *__restrict__ y) {
    int s0, s1;
    slice_range(A.nslices, s0, s1);
    int ln = lane_id();
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int64_t base = A.sptr[s];
        int w = (int)((A.sptr[s + 1] - base) >> 6);
        double o0 = 0, o1 = 0, o2 = 0;
        for (int k = 0; k < w; ++k) {
            int64_t e = base + 64 * k + ln;
            double a = (double)A.val[e];
            int64_t c = A.col[e];
            o0 += a * x[3 * c];
            o1 += a * x[3 * c + 1];
            o2 += a * x[3 * c + 2];
        }
        int row = s * 64 + ln;
        if (row < A.nrows) {
            y[3 * (int64_t)row] = o0;
            y[3 * (int64_t)row + 1] = o1;
            y[3 * (int64_t)row + 2] = o2;
        }
    }
}

// b[row_out[r]] = sum_k B_k . m[col_k]  (divergence right-hand side; rows are
// the free magnet nodes, every other entry of b stays zero)
template <class V>
__global__ __launch_bounds__(kBlock) void k_bmul(SV<V> B, const double *__restrict__ m, double *__restrict__ b) {
    int s0, s1;
    slice_range(B.nslices, s0, s1);
    int ln = lane_id();
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        double o = row_vec3_dot(B, s, ln, m);
        int row = s * 64 + ln;
        if (row < B.nrows) b[B.row_out[row]] = o;
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_btmul(SV<V> Bt, const double *__restrict__ u, double *__restrict__ g) {
    int s0, s1;
    slice_range(Bt.nslices, s0, s1);
    int ln = lane_id();
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        double o0, o1, o2;
        row_vec3_scale(Bt, s, ln, u, o0, o1, o2);
        int row = s * 64 + ln;
        if (row < Bt.nrows) {
            g[3 * (int64_t)row] = o0;
            g[3 * (int64_t)row + 1] = o1;
            g[3 * (int64_t)row + 2] = o2;
        }
    }
}

// ---------------------------------------------------------------------------
// eval epilogue: G = C m + B^T u - L h; lambda = m.G; g = G - lambda m;
// torque = |g| / L; reductions for energies and the line search
// partial slots: 0 Eloc, 1 Ezee, 2 Edemag, 3 dF, 4 dphi, 5 |g|^2, 6 max torque, 7 max |g|_inf,
// 8 max |m-x0|_inf, 9 max |m|_inf
// ---------------------------------------------------------------------------
constexpr unsigned kEvalMaxMask = (1u << 6) | (1u << 7) | (1u << 8) | (1u << 9);

template <class V>
__global__ __launch_bounds__(kBlock) void k_eval_epilogue(
    SV<V> C, SV<V> S, SV<V> Bt, int cmode, int use_demag, const double *__restrict__ m, const double *__restrict__ u,
    const double *__restrict__ L, double hx, double hy, double hz, double *__restrict__ G, double *__restrict__ g,
    double *__restrict__ lam, const double *__restrict__ x0, const double *__restrict__ g0v,
    const double *__restrict__ lam0, const double *__restrict__ d, double alpha, double *__restrict__ part) {
    __shared__ double sh[kWaves * 10];
    int s0, s1;
    slice_range(C.nslices, s0, s1);
    int ln = lane_id();
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        double c0 = 0, c1 = 0, c2 = 0;
        // cmode: 0 none, 1 exchange only (S), 2 anisotropy only (C - S), 3 both (C)
        if (cmode & 2) row_block6(C, s, ln, m, c0, c1, c2);
        if (cmode == 1 || cmode == 2) {
            int64_t base = S.sptr[s];
            int w = (int)((S.sptr[s + 1] - base) >> 6);
            double e0 = 0, e1 = 0, e2 = 0;
            for (int k = 0; k < w; ++k) {
                int64_t e = base + 64 * k + ln;
                double a = (double)S.val[e];
                int64_t c = S.col[e];
                e0 += a * m[3 * c];
                e1 += a * m[3 * c + 1];
                e2 += a * m[3 * c + 2];
            }
            if (cmode == 1) {
                c0 = e0; c1 = e1; c2 = e2;
            } else {
                c0 -= e0; c1 -= e1; c2 -= e2;
            }
        }
        double d0 = 0, d1 = 0, d2 = 0;
        if (use_demag) row_vec3_scale(Bt, s, ln, u, d0, d1, d2);
        int a = s * 64 + ln;
        if (a < C.nrows) {
            int64_t a3 = 3 * (int64_t)a;
            double m0 = m[a3], m1 = m[a3 + 1], m2 = m[a3 + 2];
            double La = L[a];
            double G0v = c0 + d0 - La * hx, G1v = c1 + d1 - La * hy, G2v = c2 + d2 - La * hz;
            double l = m0 * G0v + m1 * G1v + m2 * G2v;
            double g0 = G0v - l * m0, g1 = G1v - l * m1, g2 = G2v - l * m2;
            double gg = g0 * g0 + g1 * g1 + g2 * g2;
            G[a3] = G0v; G[a3 + 1] = G1v; G[a3 + 2] = G2v;
            g[a3] = g0; g[a3 + 1] = g1; g[a3 + 2] = g2;
            lam[a] = l;
            acc[0] += 0.5 * (m0 * c0 + m1 * c1 + m2 * c2);
            acc[1] += -La * (hx * m0 + hy * m1 + hz * m2);
            acc[2] += 0.5 * (m0 * d0 + m1 * d1 + m2 * d2);
            acc[5] += gg;
            acc[6] = fmax(acc[6], sqrt(gg) / La);
            acc[7] = fmax(acc[7], fmax(fabs(g0), fmax(fabs(g1), fabs(g2))));
            acc[9] = fmax(acc[9], fmax(fabs(m0), fmax(fabs(m1), fabs(m2))));
            if (x0) {
                double xa = x0[a3], xb = x0[a3 + 1], xc = x0[a3 + 2];
                double da = d[a3], db = d[a3 + 1], dc = d[a3 + 2];
                double wa = xa + alpha * da, wb = xb + alpha * db, wc = xc + alpha * dc;
                double wn = sqrt(wa * wa + wb * wb + wc * wc);
                // energy difference between unit vectors in tangential form:
                // 1/2 [dx.(g + g0) + 1/2 (lambda - lambda0) |dx|^2]  (= 1/2 dx.(G + G0))
                double e0 = m0 - xa, e1 = m1 - xb, e2 = m2 - xc;
                double dx2 = e0 * e0 + e1 * e1 + e2 * e2;
                acc[3] += 0.5 * (e0 * (g0 + g0v[a3]) + e1 * (g1 + g0v[a3 + 1]) + e2 * (g2 + g0v[a3 + 2]) +
                                 0.5 * (l - lam0[a]) * dx2);
                acc[4] += (g0 * da + g1 * db + g2 * dc) / wn;
                acc[8] = fmax(acc[8], fmax(fabs(m0 - xa), fmax(fabs(m1 - xb), fabs(m2 - xc))));
            }
        }
    }
    write_partials<10>(acc, kEvalMaxMask, part, sh);
}

// x_t = N(x0 + alpha d)
__global__ __launch_bounds__(kBlock) void k_trial(int n, const double *__restrict__ x0, const double *__restrict__ d,
                                                  double alpha, double *__restrict__ xt) {
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= n) return;
    int64_t a3 = 3 * (int64_t)a;
    double w0 = x0[a3] + alpha * d[a3], w1 = x0[a3 + 1] + alpha * d[a3 + 1], w2 = x0[a3 + 2] + alpha * d[a3 + 2];
    double nn = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    xt[a3] = w0 / nn;
    xt[a3 + 1] = w1 / nn;
    xt[a3 + 2] = w2 / nn;
}

// one block: out[q] = sum/max of partial slot q over nblk
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ part, int nblk, int nslot, unsigned is_max,
                                                     double *__restrict__ out) {
    __shared__ double sh[kWaves];
    for (int q = 0; q < nslot; ++q) {
        bool mx = (is_max >> q) & 1;
        double v = 0.0;
        for (int i = threadIdx.x; i < nblk; i += kBlock) {
            double x = part[q * kMaxPartials + i];
            v = mx ? fmax(v, x) : v + x;
        }
        v = mx ? wave_max(v) : wave_sum(v);
        if (lane_id() == 0) sh[wave_id()] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = sh[0];
            for (int w = 1; w < kWaves; ++w) t = mx ? fmax(t, sh[w]) : t + sh[w];
            out[q] = t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// inner PCG on the preconditioner: P v = C v - (m.(C v)) m - lambda v
// partial slots: INIT (rz, gg); PQ (1); RZ ring (rz, rr) x 2
// flags: [0] stop, [1] iterations, [2] exit reason (1 li1, 2 li2, 3 li3)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double jacobi_inv(const double *invDex, const double *dscale, int a) {
    return dscale ? invDex[a] / dscale[a] : invDex[a];
}

__global__ __launch_bounds__(kBlock) void k_prec_init(int n, int nslices, const double *__restrict__ gv,
                                                      const double *__restrict__ invDex,
                                                      const double *__restrict__ dscale, double *__restrict__ y,
                                                      double *__restrict__ r, double *__restrict__ p,
                                                      double *__restrict__ part, int *__restrict__ flags) {
    __shared__ double sh[kWaves * 2];
    int s0, s1;
    slice_range(nslices, s0, s1);
    double acc[2] = {0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int a = s * 64 + lane_id();
        if (a < n) {
            double iD = jacobi_inv(invDex, dscale, a);
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                double gi = gv[i];
                y[i] = 0.0;
                r[i] = gi;
                p[i] = gi * iD;
                acc[0] += gi * (gi * iD);
                acc[1] += gi * gi;
            }
        }
    }
    write_partials<2>(acc, 0u, part, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flags[0] = 0;
        flags[1] = 0;
        flags[2] = 1;
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_prec_apply(SV<V> C, const double *__restrict__ m,
                                                       const double *__restrict__ lam, const double *__restrict__ p,
                                                       double *__restrict__ q, double *__restrict__ part,
                                                       const int *__restrict__ flags, int phase) {
    if (stopped_before(flags, phase)) return;
    __shared__ double sh[kWaves];
    int s0, s1;
    slice_range(C.nslices, s0, s1);
    int ln = lane_id();
    double acc[1] = {0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        double c0, c1, c2;
        row_block6(C, s, ln, p, c0, c1, c2);
        int a = s * 64 + ln;
        if (a < C.nrows) {
            int64_t a3 = 3 * (int64_t)a;
            double m0 = m[a3], m1 = m[a3 + 1], m2 = m[a3 + 2];
            double mc = m0 * c0 + m1 * c1 + m2 * c2;
            double l = lam[a];
            double p0 = p[a3], p1 = p[a3 + 1], p2 = p[a3 + 2];
            double q0 = c0 - mc * m0 - l * p0, q1 = c1 - mc * m1 - l * p1, q2 = c2 - mc * m2 - l * p2;
            q[a3] = q0;
            q[a3 + 1] = q1;
            q[a3 + 2] = q2;
            acc[0] += p0 * q0 + p1 * q1 + p2 * q2;
        }
    }
    write_partials<1>(acc, 0u, part, sh);
}

// (li2) if p.Pp <= 0: stop (y = g when j == 0); else alpha step; partials (r.z, r.r)
__global__ __launch_bounds__(kBlock) void k_prec_update(int n, int nslices, int j, const double *__restrict__ gv,
                                                        const double *__restrict__ invDex,
                                                        const double *__restrict__ dscale, double *__restrict__ y,
                                                        double *__restrict__ r, const double *__restrict__ p,
                                                        const double *__restrict__ q,
                                                        const double *__restrict__ part_pq,
                                                        const double *__restrict__ part_rz_prev, int rz_slot,
                                                        double *__restrict__ part_out, int nblk,
                                                        int *__restrict__ flags, int phase) {
    if (stopped_before(flags, phase)) return;
    __shared__ double sh[kWaves * 2];
    double pq[1], rz[2];
    read_partials<1>(part_pq, nblk, 0u, pq, sh);
    int s0, s1;
    slice_range(nslices, s0, s1);
    if (!(pq[0] > 0.0)) {
        if (j == 0)
            for (int s = s0 + wave_id(); s < s1; s += kWaves) {
                int a = s * 64 + lane_id();
                if (a < n)
                    for (int c = 0; c < 3; ++c) y[3 * (int64_t)a + c] = gv[3 * (int64_t)a + c];
            }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            flags[0] = phase;
            flags[2] = 2;
        }
        return;
    }
    // rz of the previous step: slot rz_slot of part_rz_prev (the INIT layout has rz in slot 0 too)
    read_partials<2>(part_rz_prev, nblk, 0u, rz, sh);
    double alpha = rz[rz_slot] / pq[0];
    double acc[2] = {0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int a = s * 64 + lane_id();
        if (a < n) {
            double iD = jacobi_inv(invDex, dscale, a);
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                y[i] += alpha * p[i];
                double ri = r[i] - alpha * q[i];
                r[i] = ri;
                acc[0] += ri * (ri * iD);
                acc[1] += ri * ri;
            }
        }
    }
    write_partials<2>(acc, 0u, part_out, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) flags[1] = j + 1;
}

// (li3) |r| < min(0.5, sqrt(|g|)) |g|: stop; else p = D^-1 r + beta p
__global__ __launch_bounds__(kBlock) void k_prec_pupdate(int n, int nslices, const double *__restrict__ invDex,
                                                         const double *__restrict__ dscale, double *__restrict__ p,
                                                         const double *__restrict__ r,
                                                         const double *__restrict__ part_init,
                                                         const double *__restrict__ part_new,
                                                         const double *__restrict__ part_old, int old_slot, int nblk,
                                                         int *__restrict__ flags, int phase) {
    if (stopped_before(flags, phase)) return;
    __shared__ double sh[kWaves * 2];
    double ini[2], nw[2], od[2];
    read_partials<2>(part_init, nblk, 0u, ini, sh);
    read_partials<2>(part_new, nblk, 0u, nw, sh);
    double gn = sqrt(ini[1]);
    double eta = fmin(0.5, sqrt(gn));
    if (sqrt(nw[1]) < eta * gn) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            flags[0] = phase;
            flags[2] = 3;
        }
        return;
    }
    read_partials<2>(part_old, nblk, 0u, od, sh);
    double beta = nw[0] / od[old_slot];
    int s0, s1;
    slice_range(nslices, s0, s1);
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int a = s * 64 + lane_id();
        if (a < n) {
            double iD = jacobi_inv(invDex, dscale, a);
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                p[i] = r[i] * iD + beta * p[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// direction: dots then update with beta*ZA and the descent safeguard
// dot slots: 0 <g1-g0,y1>, 1 <g1-g0,d>, 2 <g1,y1>, 3 <g1,d>, 4 <g1-g0,g1>, 5 <g1,g1>
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_dir_dots(int n3, int nslices3, const double *__restrict__ g1,
                                                     const double *__restrict__ g0, const double *__restrict__ y1,
                                                     const double *__restrict__ d, double *__restrict__ part) {
    __shared__ double sh[kWaves * 6];
    int s0, s1;
    slice_range(nslices3, s0, s1);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int i = s * 64 + lane_id();
        if (i < n3) {
            double a = g1[i], b = g0 ? g0[i] : 0.0, y = y1[i], dd = d ? d[i] : 0.0;
            double dg = a - b;
            acc[0] += dg * y;
            acc[1] += dg * dd;
            acc[2] += a * y;
            acc[3] += a * dd;
            acc[4] += dg * a;
            acc[5] += a * a;
        }
    }
    write_partials<6>(acc, 0u, part, sh);
}

// mode written to info[0]: 0 -y+beta d, 1 fallback -g+beta2 d, 2 -g
// partial slots out: 0 <g1,dnew>, 1 max |dnew_a| (per node norm) -- per node needs the 3 components,
// so this kernel runs over nodes
__global__ __launch_bounds__(kBlock) void k_dir_update(int n, int nslices, const double *__restrict__ g1,
                                                       const double *__restrict__ y1, double *__restrict__ d,
                                                       const double *__restrict__ part_dots, int nblk_dots, int first,
                                                       double *__restrict__ part_out, int *__restrict__ info) {
    __shared__ double sh[kWaves * 6];
    double t[6];
    read_partials<6>(part_dots, nblk_dots, 0u, t, sh);
    double cy, cd, cg;  // d_new = cy * y1 + cd * d + cg * g1
    int mode;
    if (first) {
        // initial direction -y; if not descent, -g
        if (-t[2] < 0.0) { cy = -1; cd = 0; cg = 0; mode = 0; }
        else { cy = 0; cd = 0; cg = -1; mode = 2; }
    } else {
        double num = t[0], den = t[1];
        double beta = (num > 0.0 && den > 0.0) ? num / den : 0.0;
        double dpn = -t[2] + beta * t[3];
        if (dpn < 0.0) { cy = -1; cd = beta; cg = 0; mode = 0; }
        else {
            double num2 = t[4];
            double beta2 = (num2 > 0.0 && den > 0.0) ? num2 / den : 0.0;
            double dpn2 = -t[5] + beta2 * t[3];
            if (dpn2 < 0.0) { cy = 0; cd = beta2; cg = -1; mode = 1; }
            else { cy = 0; cd = 0; cg = -1; mode = 2; }
        }
    }
    int s0, s1;
    slice_range(nslices, s0, s1);
    double acc[2] = {0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int a = s * 64 + lane_id();
        if (a < n) {
            double nn = 0.0;
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                double dv = (cd != 0.0 ? cd * d[i] : 0.0) + cy * y1[i] + cg * g1[i];
                d[i] = dv;
                acc[0] += g1[i] * dv;
                nn += dv * dv;
            }
            acc[1] = fmax(acc[1], sqrt(nn));
        }
    }
    write_partials<2>(acc, 2u, part_out, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) info[0] = mode;
}

// energy split: 1/2 m.(S m)  (exchange part)
template <class V>
__global__ __launch_bounds__(kBlock) void k_energy_split(SV<V> S, const double *__restrict__ m, double *__restrict__ part) {
    __shared__ double sh[kWaves];
    int s0, s1;
    slice_range(S.nslices, s0, s1);
    int ln = lane_id();
    double acc[1] = {0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int64_t base = S.sptr[s];
        int w = (int)((S.sptr[s + 1] - base) >> 6);
        double e0 = 0, e1 = 0, e2 = 0;
        for (int k = 0; k < w; ++k) {
            int64_t e = base + 64 * k + ln;
            double a = (double)S.val[e];
            int64_t c = S.col[e];
            e0 += a * m[3 * c];
            e1 += a * m[3 * c + 1];
            e2 += a * m[3 * c + 2];
        }
        int a = s * 64 + ln;
        if (a < S.nrows) acc[0] += 0.5 * (m[3 * (int64_t)a] * e0 + m[3 * (int64_t)a + 1] * e1 + m[3 * (int64_t)a + 2] * e2);
    }
    write_partials<1>(acc, 0u, part, sh);
}

// mean magnetization sums (L m, L) and max | |m_a| - 1 |
__global__ __launch_bounds__(kBlock) void k_mavg(int n, int nslices, const double *__restrict__ m,
                                                 const double *__restrict__ L, double *__restrict__ part) {
    __shared__ double sh[kWaves * 5];
    int s0, s1;
    slice_range(nslices, s0, s1);
    double acc[5] = {0, 0, 0, 0, 0};
    for (int s = s0 + wave_id(); s < s1; s += kWaves) {
        int a = s * 64 + lane_id();
        if (a < n) {
            int64_t a3 = 3 * (int64_t)a;
            double La = L[a];
            double m0 = m[a3], m1 = m[a3 + 1], m2 = m[a3 + 2];
            acc[0] += La * m0;
            acc[1] += La * m1;
            acc[2] += La * m2;
            acc[3] += La;
            double nn = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
            acc[4] = fmax(acc[4], (nn == nn) ? fabs(nn - 1.0) : 1e300);
        }
    }
    write_partials<5>(acc, 1u << 4, part, sh);
}

// lambda_a = m_a . G_a
__global__ __launch_bounds__(kBlock) void k_lambda(int n, const double *__restrict__ m, const double *__restrict__ G,
                                                   double *__restrict__ lam) {
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= n) return;
    int64_t a3 = 3 * (int64_t)a;
    lam[a] = m[a3] * G[a3] + m[a3 + 1] * G[a3 + 1] + m[a3 + 2] * G[a3 + 2];
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

inline int nslices_of(int n) { return (n + 63) / 64; }

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
int grid_for_rows(int nrows) {
    int ns = nslices_of(nrows);
    int g = (ns + kWaves - 1) / kWaves;
    if (g < 1) g = 1;
    if (g > kMaxPartials) g = kMaxPartials;
    if (g >= 8) g = (g + 7) & ~7;
    if (g > kMaxPartials) g = kMaxPartials;
    return g;
}


void launch_spmv_block6(const Sell &C, const double *x, double *y, bool fp32, hipStream_t s) {
    int g = grid_for_rows(C.nrows);
    if (fp32) hipLaunchKernelGGL(k_spmv_block6<float>, dim3(g), dim3(kBlock), 0, s, view<float>(C), x, y);
    else hipLaunchKernelGGL(k_spmv_block6<double>, dim3(g), dim3(kBlock), 0, s, view<double>(C), x, y);
}
void launch_spmv_scalar(const Sell &A, const double *x, double *y, bool fp32, hipStream_t s) {
    int g = grid_for_rows(A.nrows);
    if (fp32) hipLaunchKernelGGL(k_spmv_scalar<float>, dim3(g), dim3(kBlock), 0, s, view<float>(A), x, y);
    else hipLaunchKernelGGL(k_spmv_scalar<double>, dim3(g), dim3(kBlock), 0, s, view<double>(A), x, y);
}
void launch_spmv_scalar3(const Sell &A, const double *x, double *y, bool fp32, hipStream_t s) {
    int g = grid_for_rows(A.nrows);
    if (fp32) hipLaunchKernelGGL(k_spmv_scalar3<float>, dim3(g), dim3(kBlock), 0, s, view<float>(A), x, y);
    else hipLaunchKernelGGL(k_spmv_scalar3<double>, dim3(g), dim3(kBlock), 0, s, view<double>(A), x, y);
}
void launch_bmul(const Sell &B, const double *m, double *b, bool fp32, hipStream_t s) {
    if (B.nrows == 0) return;
    int g = grid_for_rows(B.nrows);
    if (fp32) hipLaunchKernelGGL(k_bmul<float>, dim3(g), dim3(kBlock), 0, s, view<float>(B), m, b);
    else hipLaunchKernelGGL(k_bmul<double>, dim3(g), dim3(kBlock), 0, s, view<double>(B), m, b);
}
void launch_btmul(const Sell &Bt, const double *u, double *gout, bool fp32, hipStream_t s) {
    int g = grid_for_rows(Bt.nrows);
    if (fp32) hipLaunchKernelGGL(k_btmul<float>, dim3(g), dim3(kBlock), 0, s, view<float>(Bt), u, gout);
    else hipLaunchKernelGGL(k_btmul<double>, dim3(g), dim3(kBlock), 0, s, view<double>(Bt), u, gout);
}

void launch_eval_epilogue(const Sell &C, const Sell &S, const Sell &Bt, int cmode, int use_demag, const double *m,
                          const double *u, const double *L, const double h[3], double *G, double *g, double *lam,
                          const double *x0, const double *g0, const double *lam0, const double *d, double alpha,
                          double *part, bool fp32, hipStream_t s) {
    int gr = grid_for_rows(C.nrows);
    if (fp32)
        hipLaunchKernelGGL(k_eval_epilogue<float>, dim3(gr), dim3(kBlock), 0, s, view<float>(C), view<float>(S),
                           view<float>(Bt), cmode, use_demag, m, u, L, h[0], h[1], h[2], G, g, lam, x0, g0, lam0, d,
                           alpha, part);
    else
        hipLaunchKernelGGL(k_eval_epilogue<double>, dim3(gr), dim3(kBlock), 0, s, view<double>(C), view<double>(S),
                           view<double>(Bt), cmode, use_demag, m, u, L, h[0], h[1], h[2], G, g, lam, x0, g0, lam0, d,
                           alpha, part);
}
unsigned eval_max_mask() { return kEvalMaxMask; }

void launch_trial(int n, const double *x0, const double *d, double alpha, double *xt, hipStream_t s) {
    int g = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_trial, dim3(g), dim3(kBlock), 0, s, n, x0, d, alpha, xt);
}
void launch_finalize(const double *part, int nblk, int nslot, unsigned is_max, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, part, nblk, nslot, is_max, out);
}

void launch_prec_init(int n, const double *gv, const double *invDex, const double *dscale, double *y, double *r,
                      double *p, double *part, int *flags, hipStream_t s) {
    int g = grid_for_rows(n);
    hipLaunchKernelGGL(k_prec_init, dim3(g), dim3(kBlock), 0, s, n, nslices_of(n), gv, invDex, dscale, y, r, p, part,
                       flags);
}
void launch_prec_apply(const Sell &C, const double *m, const double *lam, const double *p, double *q, double *part,
                       const int *flags, int phase, bool fp32, hipStream_t s) {
    int g = grid_for_rows(C.nrows);
    if (fp32)
        hipLaunchKernelGGL(k_prec_apply<float>, dim3(g), dim3(kBlock), 0, s, view<float>(C), m, lam, p, q, part, flags,
                           phase);
    else
        hipLaunchKernelGGL(k_prec_apply<double>, dim3(g), dim3(kBlock), 0, s, view<double>(C), m, lam, p, q, part,
                           flags, phase);
}
void launch_prec_update(int n, int j, const double *gv, const double *invDex, const double *dscale, double *y,
                        double *r, const double *p, const double *q, const double *part_pq, const double *part_rz_prev,
                        int rz_slot, double *part_out, int *flags, int phase, hipStream_t s) {
    int g = grid_for_rows(n);
    hipLaunchKernelGGL(k_prec_update, dim3(g), dim3(kBlock), 0, s, n, nslices_of(n), j, gv, invDex, dscale, y, r, p, q,
                       part_pq, part_rz_prev, rz_slot, part_out, g, flags, phase);
}
void launch_prec_pupdate(int n, const double *invDex, const double *dscale, double *p, const double *r,
                         const double *part_init, const double *part_new, const double *part_old, int old_slot,
                         int *flags, int phase, hipStream_t s) {
    int g = grid_for_rows(n);
    hipLaunchKernelGGL(k_prec_pupdate, dim3(g), dim3(kBlock), 0, s, n, nslices_of(n), invDex, dscale, p, r, part_init,
                       part_new, part_old, old_slot, g, flags, phase);
}

void launch_dir_dots(int n, const double *g1, const double *g0, const double *y1, const double *d, double *part,
                     int *nblk_out, hipStream_t s) {
    int n3 = 3 * n;
    int g = grid_for_rows(n3);
    *nblk_out = g;
    hipLaunchKernelGGL(k_dir_dots, dim3(g), dim3(kBlock), 0, s, n3, nslices_of(n3), g1, g0, y1, d, part);
}
void launch_dir_update(int n, const double *g1, const double *y1, double *d, const double *part_dots, int nblk_dots,
                       int first, double *part_out, int *info, hipStream_t s) {
    int g = grid_for_rows(n);
    hipLaunchKernelGGL(k_dir_update, dim3(g), dim3(kBlock), 0, s, n, nslices_of(n), g1, y1, d, part_dots, nblk_dots,
                       first, part_out, info);
}

void launch_energy_split(const Sell &S, const double *m, double *part, bool fp32, hipStream_t s) {
    int g = grid_for_rows(S.nrows);
    if (fp32) hipLaunchKernelGGL(k_energy_split<float>, dim3(g), dim3(kBlock), 0, s, view<float>(S), m, part);
    else hipLaunchKernelGGL(k_energy_split<double>, dim3(g), dim3(kBlock), 0, s, view<double>(S), m, part);
}
void launch_mavg(int n, const double *m, const double *L, double *part, hipStream_t s) {
    int g = grid_for_rows(n);
    hipLaunchKernelGGL(k_mavg, dim3(g), dim3(kBlock), 0, s, n, nslices_of(n), m, L, part);
}
void launch_lambda(int n, const double *m, const double *G, double *lam, hipStream_t s) {
    int g = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_lambda, dim3(g), dim3(kBlock), 0, s, n, m, G, lam);
}
void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)g), dim3(kBlock), 0, s, n, x, y);
}

}  // namespace mmncg
