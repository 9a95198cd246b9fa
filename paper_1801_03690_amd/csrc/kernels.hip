// HIP kernels (gfx950) of the micromagnetic PNCG hot path, batched over
// independent problem instances.
//
// Layout. Every sparse operator is stored SELL-64: a wavefront owns a slice of
// 64 consecutive rows, one row per lane, and walks the slice's entries
// column-major, so the k-th load of the wave reads 64 consecutive values and
// 64 consecutive column indices. Vectors on magnet nodes are node-major AoS
// doubles (x, y, z); vectors on potential nodes are plain arrays. Instances
// are concatenated, each padded to whole slices; a RowMap gives every block
// one instance and a contiguous slice range of it (internal.h), so one launch
// serves every instance and each instance's reductions read only its blocks.
//
// Reductions are deterministic: each block writes one partial per quantity
// into a fixed slot and the consumer (a later kernel, every block of it, or a
// one-block-per-instance finalize kernel) re-reduces them in a fixed order.
// No floating-point atomics anywhere.
//
// Operator values may be stored in FP32 (template parameter V) for the
// FP32-bulk mode; products and sums are formed in FP64.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace mmncg {

using namespace dev;

namespace {

constexpr int NW = kBlock / 64;  // waves per block of the magnet-row kernels

__device__ __forceinline__ StateV pick(const StateV &a, const StateV &b, const StateV &c, int role) {
    return role == 1 ? b : (role == 2 ? c : a);
}

// ---------------------------------------------------------------------------
// plain operators (checking ABI and building blocks)
// ---------------------------------------------------------------------------
template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_block6(SV<V> A, RowMap M, const double *__restrict__ x,
                                                        double *__restrict__ y) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    const int rend = M.rend[t.inst], ln = lane_id();
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double o0, o1, o2;
        row_block6<2>(A, s, ln, x, o0, o1, o2);
        int row = s * 64 + ln;
        if (row < rend) {
            y[3 * (int64_t)row] = o0;
            y[3 * (int64_t)row + 1] = o1;
            y[3 * (int64_t)row + 2] = o2;
        }
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_scalar(SV<V> A, RowMap M, const double *__restrict__ x,
                                                        double *__restrict__ y) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    const int rend = M.rend[t.inst], ln = lane_id();
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double o = row_scalar<4>(A, s, ln, x);
        int row = s * 64 + ln;
        if (row < rend) y[row] = o;
    }
}

// b[row_out[r]] = sum_k B_k . m[col_k] over the free magnet nodes; every
// other entry of b stays zero. m is the state the instance evaluates.
template <class V>
__global__ __launch_bounds__(kBlock) void k_bmul(SV<V> B, RowMap MB, const int *__restrict__ act, StateV s0v,
                                                 StateV s1v, StateV s2v, const int *__restrict__ role,
                                                 double *__restrict__ b) {
    Tile t = tile_of(MB);
    if (t.inst < 0 || (act && !act[t.inst])) return;
    const double *m = pick(s0v, s1v, s2v, role ? role[t.inst] : 0).x;
    const int rend = MB.rend[t.inst], ln = lane_id();
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double o = row_vec3_dot<4>(B, s, ln, m);
        int row = s * 64 + ln;
        if (row < rend) b[B.row_out[row]] = o;
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_btmul(SV<V> Bt, RowMap M, const double *__restrict__ u,
                                                  double *__restrict__ g) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    const int rend = M.rend[t.inst], ln = lane_id();
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double o0, o1, o2;
        row_vec3_scale<2>(Bt, s, ln, u, o0, o1, o2);
        int row = s * 64 + ln;
        if (row < rend) {
            g[3 * (int64_t)row] = o0;
            g[3 * (int64_t)row + 1] = o1;
            g[3 * (int64_t)row + 2] = o2;
        }
    }
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------
// x_role = N(x_cur + alpha_i d) for the active instances
__global__ __launch_bounds__(kBlock) void k_trial(RowMap M, const int *__restrict__ act, const int *__restrict__ role,
                                                  StateV s0v, StateV s1v, StateV s2v, const double *__restrict__ d,
                                                  const double *__restrict__ alpha) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst]) return;
    const int rl = role[t.inst];
    if (rl == 0) return;
    double *xt = pick(s0v, s1v, s2v, rl).x;
    const double *x0 = s0v.x;
    const double a = alpha[t.inst];
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int r = s * 64 + lane_id();
        if (r < rend) {
            int64_t r3 = 3 * (int64_t)r;
            double w0 = x0[r3] + a * d[r3], w1 = x0[r3 + 1] + a * d[r3 + 1], w2 = x0[r3 + 2] + a * d[r3 + 2];
            double nn = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
            xt[r3] = w0 / nn;
            xt[r3 + 1] = w1 / nn;
            xt[r3 + 2] = w2 / nn;
        }
    }
}

// G = C m + B^T u - L h; lambda = m.G; g = G - lambda m; torque |g| / L;
// partials: 0 Eloc, 1 Ezee, 2 Edemag, 3 dF, 4 dphi, 5 |g|^2, 6 max torque,
// 7 max |g|_inf, 8 max |m-x0|_inf, 9 max |m|_inf. With role != 0 the point is
// a line-search trial relative to the current state (role 0) along d.
constexpr unsigned kEvalMaxMask = (1u << 6) | (1u << 7) | (1u << 8) | (1u << 9);

template <class V>
__global__ __launch_bounds__(kBlock) void k_eval_epilogue(SV<V> C, SV<V> S, SV<V> Bt, RowMap M, int cmode,
                                                          int use_demag, const int *__restrict__ act,
                                                          const int *__restrict__ role, StateV s0v, StateV s1v,
                                                          StateV s2v, const double *__restrict__ u,
                                                          const double *__restrict__ L, const double *__restrict__ h3,
                                                          const double *__restrict__ d,
                                                          const double *__restrict__ alpha, double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0 || (act && !act[t.inst])) return;
    __shared__ double sh[NW * kEvalParts];
    const int rl = role ? role[t.inst] : 0;
    const StateV sv = pick(s0v, s1v, s2v, rl);
    const double *__restrict__ m = sv.x;
    const double hx = h3[3 * t.inst], hy = h3[3 * t.inst + 1], hz = h3[3 * t.inst + 2];
    const double a = (rl != 0) ? alpha[t.inst] : 0.0;
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[kEvalParts] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double c0 = 0, c1 = 0, c2 = 0;
        // cmode: 0 none, 1 exchange only (S), 2 anisotropy only (C - S), 3 both (C)
        if (cmode & 2) row_block6<2>(C, s, ln, m, c0, c1, c2);
        if (cmode == 1 || cmode == 2) {
            double e0, e1, e2;
            row_scalar3(S, s, ln, m, e0, e1, e2);
            if (cmode == 1) {
                c0 = e0; c1 = e1; c2 = e2;
            } else {
                c0 -= e0; c1 -= e1; c2 -= e2;
            }
        }
        double d0 = 0, d1 = 0, d2 = 0;
        if (use_demag) row_vec3_scale<2>(Bt, s, ln, u, d0, d1, d2);
        int r = s * 64 + ln;
        if (r < rend) {
            int64_t r3 = 3 * (int64_t)r;
            double m0 = m[r3], m1 = m[r3 + 1], m2 = m[r3 + 2];
            double La = L[r];
            double Gx = c0 + d0 - La * hx, Gy = c1 + d1 - La * hy, Gz = c2 + d2 - La * hz;
            double l = m0 * Gx + m1 * Gy + m2 * Gz;
            double g0 = Gx - l * m0, g1 = Gy - l * m1, g2 = Gz - l * m2;
            double gg = g0 * g0 + g1 * g1 + g2 * g2;
            sv.G[r3] = Gx; sv.G[r3 + 1] = Gy; sv.G[r3 + 2] = Gz;
            sv.g[r3] = g0; sv.g[r3 + 1] = g1; sv.g[r3 + 2] = g2;
            sv.lam[r] = l;
            acc[0] += 0.5 * (m0 * c0 + m1 * c1 + m2 * c2);
            acc[1] += -La * (hx * m0 + hy * m1 + hz * m2);
            acc[2] += 0.5 * (m0 * d0 + m1 * d1 + m2 * d2);
            acc[5] += gg;
            acc[6] = fmax(acc[6], sqrt(gg) / La);
            acc[7] = fmax(acc[7], fmax(fabs(g0), fmax(fabs(g1), fabs(g2))));
            acc[9] = fmax(acc[9], fmax(fabs(m0), fmax(fabs(m1), fabs(m2))));
            if (rl != 0) {
                const double *x0 = s0v.x, *g0v = s0v.g, *lam0 = s0v.lam;
                double xa = x0[r3], xb = x0[r3 + 1], xc = x0[r3 + 2];
                double da = d[r3], db = d[r3 + 1], dc = d[r3 + 2];
                double wa = xa + a * da, wb = xb + a * db, wc = xc + a * dc;
                double wn = sqrt(wa * wa + wb * wb + wc * wc);
                // energy difference between unit vectors in tangential form:
                // 1/2 [dx.(g + g0) + 1/2 (lambda - lambda0) |dx|^2]  (= 1/2 dx.(G + G0))
                double e0 = m0 - xa, e1 = m1 - xb, e2 = m2 - xc;
                double dx2 = e0 * e0 + e1 * e1 + e2 * e2;
                acc[3] += 0.5 * (e0 * (g0 + g0v[r3]) + e1 * (g1 + g0v[r3 + 1]) + e2 * (g2 + g0v[r3 + 2]) +
                                 0.5 * (l - lam0[r]) * dx2);
                acc[4] += (g0 * da + g1 * db + g2 * dc) / wn;
                acc[8] = fmax(acc[8], fmax(fabs(e0), fmax(fabs(e1), fabs(e2))));
            }
        }
    }
    write_part<kEvalParts, NW>(acc, kEvalMaxMask, part, M.nblk, t.b, sh);
}

// one block per instance: out[i * nslot + q] = reduction of slot q over the instance's blocks
__global__ __launch_bounds__(kBlock) void k_finalize_inst(const double *__restrict__ part, int stride,
                                                          const int *__restrict__ ipb, int nslot, unsigned is_max,
                                                          double *__restrict__ out) {
    __shared__ double sh[NW];
    const int i = blockIdx.x;
    const int b0 = ipb[i], b1 = ipb[i + 1];
    for (int q = 0; q < nslot; ++q) {
        double v[1];
        read_part<1, NW>(part + (size_t)q * stride, stride, b0, b1, (is_max >> q) & 1, v, sh);
        if (threadIdx.x == 0) out[(size_t)i * nslot + q] = v[0];
    }
}

// state 0 <- state from[i] (1 or 2) for the instances that accepted a trial;
// the projected gradient of the replaced state is kept in gprev (beta*ZA needs
// g of both iterates)
__global__ __launch_bounds__(kBlock) void k_copy_state(RowMap M, const int *__restrict__ from, StateV s0v, StateV s1v,
                                                       StateV s2v, double *__restrict__ gprev) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    const int f = from[t.inst];
    if (f == 0) return;
    const StateV src = pick(s0v, s1v, s2v, f);
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int r = s * 64 + lane_id();
        if (r < rend) {
            int64_t r3 = 3 * (int64_t)r;
            for (int c = 0; c < 3; ++c) {
                gprev[r3 + c] = s0v.g[r3 + c];
                s0v.x[r3 + c] = src.x[r3 + c];
                s0v.G[r3 + c] = src.G[r3 + c];
                s0v.g[r3 + c] = src.g[r3 + c];
            }
            s0v.lam[r] = src.lam[r];
        }
    }
}

// ---------------------------------------------------------------------------
// inner PCG on the preconditioner: P v = C v - (m.(C v)) m - lambda v
// partial slots: INIT 0-1 (r.z, g.g), PQ 2, RZ0 3-4, RZ1 5-6 (r.z, r.r)
// flags per instance (4 ints): stop phase, iterations, exit reason (1 li1, 2 li2, 3 li3)
// ---------------------------------------------------------------------------
constexpr int kPrINIT = 0, kPrPQ = 2, kPrRZ0 = 3, kPrRZ1 = 5;

__device__ __forceinline__ double jacobi_inv(const double *invDex, const double *dscale, int a) {
    return dscale ? invDex[a] / dscale[a] : invDex[a];
}

__global__ __launch_bounds__(kBlock) void k_prec_init(RowMap M, const int *__restrict__ act,
                                                      const double *__restrict__ gv, const double *__restrict__ invDex,
                                                      const double *__restrict__ dscale, double *__restrict__ y,
                                                      double *__restrict__ r, double *__restrict__ p,
                                                      double *__restrict__ part, int *__restrict__ flags) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst]) return;
    __shared__ double sh[NW * 2];
    const int rend = M.rend[t.inst];
    double acc[2] = {0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend) {
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
    write_part<2, NW>(acc, 0u, part + (size_t)kPrINIT * M.nblk, M.nblk, t.b, sh);
    if (t.b == M.ipb[t.inst] && threadIdx.x == 0) {
        flags[4 * t.inst] = 0;
        flags[4 * t.inst + 1] = 0;
        flags[4 * t.inst + 2] = 1;
    }
}

// FORM selects the terms of eq. (precond): 0 all but the last, 1 all four
// (the last, -(v . grad F) m, with grad F = g + lambda m), 2 without the
// lambda v term as well
template <class V, int FORM>
__global__ __launch_bounds__(kBlock) void k_prec_apply(SV<V> C, RowMap M, const int *__restrict__ act,
                                                       const double *__restrict__ m, const double *__restrict__ lam,
                                                       const double *__restrict__ g, const double *__restrict__ p,
                                                       double *__restrict__ q, double *__restrict__ part,
                                                       const int *__restrict__ flags, int phase) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst] || stopped_before(flags + 4 * t.inst, phase)) return;
    __shared__ double sh[NW];
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[1] = {0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double c0, c1, c2;
        row_block6<1>(C, s, ln, p, c0, c1, c2);
        int a = s * 64 + ln;
        if (a < rend) {
            int64_t a3 = 3 * (int64_t)a;
            double m0 = m[a3], m1 = m[a3 + 1], m2 = m[a3 + 2];
            double mc = m0 * c0 + m1 * c1 + m2 * c2;
            double l = FORM == 2 ? 0.0 : lam[a];
            double p0 = p[a3], p1 = p[a3 + 1], p2 = p[a3 + 2];
            double q0 = c0 - mc * m0 - l * p0, q1 = c1 - mc * m1 - l * p1, q2 = c2 - mc * m2 - l * p2;
            if (FORM == 1) {
                const double la = lam[a];
                const double vG = p0 * (g[a3] + la * m0) + p1 * (g[a3 + 1] + la * m1) + p2 * (g[a3 + 2] + la * m2);
                q0 -= vG * m0;
                q1 -= vG * m1;
                q2 -= vG * m2;
            }
            q[a3] = q0;
            q[a3 + 1] = q1;
            q[a3 + 2] = q2;
            acc[0] += p0 * q0 + p1 * q1 + p2 * q2;
        }
    }
    write_part<1, NW>(acc, 0u, part + (size_t)kPrPQ * M.nblk, M.nblk, t.b, sh);
}

// (li2) if p.Pp <= 0: stop (y = g when j == 0); else alpha step; partials (r.z, r.r)
__global__ __launch_bounds__(kBlock) void k_prec_update(RowMap M, const int *__restrict__ act, int j,
                                                        const double *__restrict__ gv,
                                                        const double *__restrict__ invDex,
                                                        const double *__restrict__ dscale, double *__restrict__ y,
                                                        double *__restrict__ r, const double *__restrict__ p,
                                                        const double *__restrict__ q, double *__restrict__ part,
                                                        int *__restrict__ flags, int phase) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst] || stopped_before(flags + 4 * t.inst, phase)) return;
    __shared__ double sh[NW * 2];
    const int S = M.nblk, b0 = M.ipb[t.inst], b1 = M.ipb[t.inst + 1];
    double pq[1], rz[1];
    read_part<1, NW>(part + (size_t)kPrPQ * S, S, b0, b1, 0u, pq, sh);
    const int rend = M.rend[t.inst];
    if (!(pq[0] > 0.0)) {
        if (j == 0)
            for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
                int a = s * 64 + lane_id();
                if (a < rend)
                    for (int c = 0; c < 3; ++c) y[3 * (int64_t)a + c] = gv[3 * (int64_t)a + c];
            }
        if (t.b == b0 && threadIdx.x == 0) {
            flags[4 * t.inst] = phase;
            flags[4 * t.inst + 2] = 2;
        }
        return;
    }
    const int prev = (j == 0) ? kPrINIT : ((j & 1) ? kPrRZ1 : kPrRZ0);
    const int next = ((j + 1) & 1) ? kPrRZ1 : kPrRZ0;
    read_part<1, NW>(part + (size_t)prev * S, S, b0, b1, 0u, rz, sh);
    const double alpha = rz[0] / pq[0];
    double acc[2] = {0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend) {
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
    write_part<2, NW>(acc, 0u, part + (size_t)next * S, S, t.b, sh);
    if (t.b == b0 && threadIdx.x == 0) flags[4 * t.inst + 1] = j + 1;
}

// (li3) |r| < min(0.5, sqrt(|g|)) |g|: stop; else p = D^-1 r + beta p
__global__ __launch_bounds__(kBlock) void k_prec_pupdate(RowMap M, const int *__restrict__ act, int j,
                                                         const double *__restrict__ invDex,
                                                         const double *__restrict__ dscale, double *__restrict__ p,
                                                         const double *__restrict__ r, const double *__restrict__ part,
                                                         int *__restrict__ flags, int phase) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst] || stopped_before(flags + 4 * t.inst, phase)) return;
    __shared__ double sh[NW * 2];
    const int S = M.nblk, b0 = M.ipb[t.inst], b1 = M.ipb[t.inst + 1];
    const int prev = (j == 0) ? kPrINIT : ((j & 1) ? kPrRZ1 : kPrRZ0);
    const int next = ((j + 1) & 1) ? kPrRZ1 : kPrRZ0;
    double ini[2], nw[2], od[1];
    read_part<2, NW>(part + (size_t)kPrINIT * S, S, b0, b1, 0u, ini, sh);
    read_part<2, NW>(part + (size_t)next * S, S, b0, b1, 0u, nw, sh);
    const double gn = sqrt(ini[1]);
    const double eta = fmin(0.5, sqrt(gn));
    if (sqrt(nw[1]) < eta * gn) {
        if (t.b == b0 && threadIdx.x == 0) {
            flags[4 * t.inst] = phase;
            flags[4 * t.inst + 2] = 3;
        }
        return;
    }
    read_part<1, NW>(part + (size_t)prev * S, S, b0, b1, 0u, od, sh);
    const double beta = nw[0] / od[0];
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend) {
            double iD = jacobi_inv(invDex, dscale, a);
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                p[i] = r[i] * iD + beta * p[i];
            }
        }
    }
}

// beta* of the preconditioned NCG (Sec. 2.1, eqs. FR*, PRP*, HS*, and Alg. 4's
// ZA, the HS form restarted when y_{j+1}.g_{j+1} <= y_{j+1}.g_j) from num =
// <g1 - g0, y1>, den = <g1 - g0, d>, gy1 = <g1, y1> and gy0 = <g0, y0> of the
// previous direction; a non-positive denominator gives 0
__device__ __forceinline__ double beta_star(int kind, double num, double den, double gy1, double gy0) {
    switch (kind) {
        case 1: return gy0 > 0.0 ? gy1 / gy0 : 0.0;
        case 2: return gy0 > 0.0 ? num / gy0 : 0.0;
        case 3: return den > 0.0 ? num / den : 0.0;
        default: return (num > 0.0 && den > 0.0) ? num / den : 0.0;
    }
}

// ---------------------------------------------------------------------------
// direction: dots, then beta* (ZA unless another kind is asked for) with the
// descent safeguard; <g, y> of the direction taken is kept per instance in gy
// (<g, g> when g stands in for y), and the dots kernel snapshots it into
// gy_old for the update kernel, which overwrites gy. first[i] bits:
// 1 = first direction of a field or a restart (no beta term), 2 = take g in
// place of the preconditioned y (no preconditioner, or steepest descent)
// dot slots: 0 <g1-g0,y1>, 1 <g1-g0,d>, 2 <g1,y1>, 3 <g1,d>, 4 <g1-g0,g1>, 5 <g1,g1>
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_dir_dots(RowMap M, const int *__restrict__ act,
                                                     const int *__restrict__ first, const double *__restrict__ g1,
                                                     const double *__restrict__ g0, const double *__restrict__ y1,
                                                     const double *__restrict__ d, double *__restrict__ part,
                                                     const double *__restrict__ gy, double *__restrict__ gy_old) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst]) return;
    if (t.b == M.ipb[t.inst] && threadIdx.x == 0) gy_old[t.inst] = gy[t.inst];
    __shared__ double sh[NW * kDirParts];
    const int fm = first[t.inst];
    const bool fst = (fm & 1) != 0;
    const double *__restrict__ yv = (fm & 2) ? g1 : y1;
    const int rend = M.rend[t.inst];
    double acc[kDirParts] = {0, 0, 0, 0, 0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend)
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                double gn = g1[i], go = fst ? 0.0 : g0[i], yy = yv[i], dd = fst ? 0.0 : d[i];
                double dg = gn - go;
                acc[0] += dg * yy;
                acc[1] += dg * dd;
                acc[2] += gn * yy;
                acc[3] += gn * dd;
                acc[4] += dg * gn;
                acc[5] += gn * gn;
            }
    }
    write_part<kDirParts, NW>(acc, 0u, part, M.nblk, t.b, sh);
}

// info[i] = mode: 0 -y + beta d, 1 fallback -g + beta2 d, 2 -g; partials out: <g1,dnew>, max |dnew_a|
__global__ __launch_bounds__(kBlock) void k_dir_update(RowMap M, const int *__restrict__ act,
                                                       const int *__restrict__ first, const double *__restrict__ g1,
                                                       const double *__restrict__ y1, double *__restrict__ d,
                                                       const double *__restrict__ part_dots,
                                                       double *__restrict__ part_out, int *__restrict__ info,
                                                       int kind, const double *__restrict__ gy_old,
                                                       double *__restrict__ gy) {
    Tile t = tile_of(M);
    if (t.inst < 0 || !act[t.inst]) return;
    __shared__ double sh[NW * kDirParts];
    double tt[kDirParts];
    read_part<kDirParts, NW>(part_dots, M.nblk, M.ipb[t.inst], M.ipb[t.inst + 1], 0u, tt, sh);
    const int fm = first[t.inst];
    const double *__restrict__ yv = (fm & 2) ? g1 : y1;
    double cy, cd, cg;  // d_new = cy y + cd d + cg g1
    int mode;
    if (fm & 1) {
        if (-tt[2] < 0.0) { cy = -1; cd = 0; cg = 0; mode = 0; }
        else { cy = 0; cd = 0; cg = -1; mode = 2; }
    } else {
        const double gy0 = gy_old[t.inst];
        double beta = beta_star(kind, tt[0], tt[1], tt[2], gy0);
        double dpn = -tt[2] + beta * tt[3];
        if (dpn < 0.0) { cy = -1; cd = beta; cg = 0; mode = 0; }
        else {
            double beta2 = beta_star(kind, tt[4], tt[1], tt[5], gy0);
            double dpn2 = -tt[5] + beta2 * tt[3];
            if (dpn2 < 0.0) { cy = 0; cd = beta2; cg = -1; mode = 1; }
            else { cy = 0; cd = 0; cg = -1; mode = 2; }
        }
    }
    const int rend = M.rend[t.inst];
    double acc[2] = {0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend) {
            double nn = 0.0;
            for (int c = 0; c < 3; ++c) {
                int64_t i = 3 * (int64_t)a + c;
                double dv = (cd != 0.0 ? cd * d[i] : 0.0) + cy * yv[i] + cg * g1[i];
                d[i] = dv;
                acc[0] += g1[i] * dv;
                nn += dv * dv;
            }
            acc[1] = fmax(acc[1], sqrt(nn));
        }
    }
    write_part<2, NW>(acc, 2u, part_out, M.nblk, t.b, sh);
    if (t.b == M.ipb[t.inst] && threadIdx.x == 0) {
        info[t.inst] = mode;
        gy[t.inst] = mode == 0 ? tt[2] : tt[5];
    }
}

// exchange part of the energy: 1/2 m.(S m)
template <class V>
__global__ __launch_bounds__(kBlock) void k_energy_split(SV<V> S, RowMap M, const double *__restrict__ m,
                                                         double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    __shared__ double sh[NW];
    const int rend = M.rend[t.inst], ln = lane_id();
    double acc[1] = {0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        double e0, e1, e2;
        row_scalar3(S, s, ln, m, e0, e1, e2);
        int a = s * 64 + ln;
        if (a < rend)
            acc[0] += 0.5 * (m[3 * (int64_t)a] * e0 + m[3 * (int64_t)a + 1] * e1 + m[3 * (int64_t)a + 2] * e2);
    }
    write_part<1, NW>(acc, 0u, part, M.nblk, t.b, sh);
}

// sums (L m, L) and max | |m_a| - 1 | (NaN counts as a huge deviation)
__global__ __launch_bounds__(kBlock) void k_mavg(RowMap M, const double *__restrict__ m, const double *__restrict__ L,
                                                 double *__restrict__ part) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    __shared__ double sh[NW * 5];
    const int rend = M.rend[t.inst];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend) {
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
    write_part<5, NW>(acc, 1u << 4, part, M.nblk, t.b, sh);
}

// lambda_a = m_a . G_a
__global__ __launch_bounds__(kBlock) void k_lambda(RowMap M, const double *__restrict__ m,
                                                   const double *__restrict__ G, double *__restrict__ lam) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        int a = s * 64 + lane_id();
        if (a < rend) {
            int64_t a3 = 3 * (int64_t)a;
            lam[a] = m[a3] * G[a3] + m[a3 + 1] * G[a3 + 1] + m[a3 + 2] * G[a3 + 2];
        }
    }
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

// per-instance operations on the scalar potential (see launch_pot_op)
__global__ __launch_bounds__(kBlock) void k_pot_op(RowMap M, const int *__restrict__ op,
                                                   const double *__restrict__ rho, double *__restrict__ u,
                                                   double *__restrict__ ux, double *__restrict__ ut) {
    Tile t = tile_of(M);
    if (t.inst < 0) return;
    const int o = op[t.inst];
    if (o == POT_NONE) return;
    const double q = rho[t.inst];
    const int rend = M.rend[t.inst];
    for (int s = t.s0 + wave_id(); s < t.s1; s += NW) {
        const int i = s * 64 + lane_id();
        if (i >= rend) continue;
        switch (o) {
            case POT_UX_U: ux[i] = u[i]; break;
            case POT_UT_U: ut[i] = u[i]; break;
            case POT_UX_UT: ux[i] = ut[i]; break;
            case POT_INTERP: u[i] = ux[i] + q * (ut[i] - ux[i]); break;
            default: {
                const double v = u[i];
                ux[i] = v;
                ut[i] = v;
            } break;
        }
    }
}

__global__ void k_fill(int64_t n, double *__restrict__ x, double v) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}

// out[i] = in[idx[i]] (idx a permutation of [0, n))
__global__ void k_gather(int64_t n, const int *__restrict__ idx, const double *__restrict__ in,
                         double *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = in[idx[i]];
}

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
unsigned eval_max_mask() { return kEvalMaxMask; }

void launch_spmv_block6(const Sell &C, const RowMap &M, const double *x, double *y, bool fp32, hipStream_t s) {
    if (fp32) hipLaunchKernelGGL(k_spmv_block6<float>, dim3(M.nblk), dim3(kBlock), 0, s, view<float>(C), M, x, y);
    else hipLaunchKernelGGL(k_spmv_block6<double>, dim3(M.nblk), dim3(kBlock), 0, s, view<double>(C), M, x, y);
}
void launch_spmv_scalar(const Sell &A, const RowMap &M, const double *x, double *y, bool fp32, hipStream_t s) {
    if (fp32) hipLaunchKernelGGL(k_spmv_scalar<float>, dim3(M.nblk), dim3(kBlock), 0, s, view<float>(A), M, x, y);
    else hipLaunchKernelGGL(k_spmv_scalar<double>, dim3(M.nblk), dim3(kBlock), 0, s, view<double>(A), M, x, y);
}
void launch_bmul(const Sell &B, const RowMap &MB, const int *act, const StateV *sv, const int *role, double *b,
                 bool fp32, hipStream_t s) {
    if (B.nrows == 0) return;
    if (fp32)
        hipLaunchKernelGGL(k_bmul<float>, dim3(MB.nblk), dim3(kBlock), 0, s, view<float>(B), MB, act, sv[0], sv[1],
                           sv[2], role, b);
    else
        hipLaunchKernelGGL(k_bmul<double>, dim3(MB.nblk), dim3(kBlock), 0, s, view<double>(B), MB, act, sv[0], sv[1],
                           sv[2], role, b);
}
void launch_btmul(const Sell &Bt, const RowMap &M, const double *u, double *gout, bool fp32, hipStream_t s) {
    if (fp32) hipLaunchKernelGGL(k_btmul<float>, dim3(M.nblk), dim3(kBlock), 0, s, view<float>(Bt), M, u, gout);
    else hipLaunchKernelGGL(k_btmul<double>, dim3(M.nblk), dim3(kBlock), 0, s, view<double>(Bt), M, u, gout);
}

void launch_trial(const RowMap &M, const int *act, const int *role, const StateV st[3], const double *d,
                  const double *alpha, hipStream_t s) {
    hipLaunchKernelGGL(k_trial, dim3(M.nblk), dim3(kBlock), 0, s, M, act, role, st[0], st[1], st[2], d, alpha);
}
void launch_eval_epilogue(const EvalLaunch &e, hipStream_t s) {
    const RowMap &M = *e.M;
    if (e.fp32)
        hipLaunchKernelGGL(k_eval_epilogue<float>, dim3(M.nblk), dim3(kBlock), 0, s, view<float>(*e.C),
                           view<float>(*e.S), view<float>(*e.Bt), M, e.cmode, e.use_demag, e.act, e.role, e.st[0],
                           e.st[1], e.st[2], e.u, e.L, e.h3, e.d, e.alpha, e.part);
    else
        hipLaunchKernelGGL(k_eval_epilogue<double>, dim3(M.nblk), dim3(kBlock), 0, s, view<double>(*e.C),
                           view<double>(*e.S), view<double>(*e.Bt), M, e.cmode, e.use_demag, e.act, e.role, e.st[0],
                           e.st[1], e.st[2], e.u, e.L, e.h3, e.d, e.alpha, e.part);
}
void launch_finalize_inst(const RowMap &M, const double *part, int nslot, unsigned is_max, double *out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_inst, dim3(M.ninst), dim3(kBlock), 0, s, part, M.nblk, M.ipb, nslot, is_max, out);
}
void launch_copy_state(const RowMap &M, const int *from, const StateV st[3], double *gprev, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_state, dim3(M.nblk), dim3(kBlock), 0, s, M, from, st[0], st[1], st[2], gprev);
}

void launch_prec_init(const PrecLaunch &a, hipStream_t s) {
    const RowMap &M = *a.M;
    hipLaunchKernelGGL(k_prec_init, dim3(M.nblk), dim3(kBlock), 0, s, M, a.act, a.g, a.invDex, a.dscale, a.y, a.r,
                       a.p, a.part, a.flags);
}
void launch_prec_iter(const PrecLaunch &a, int j, bool last, hipStream_t s) {
    launch_prec_apply(a, j, s);
    launch_prec_tail(a, j, last, s);
}

void launch_prec_apply(const PrecLaunch &a, int j, hipStream_t s) {
    const RowMap &M = *a.M;
    const int ph = 3 * j;
#define MMNCG_PREC_APPLY(V, F)                                                                                     \
    hipLaunchKernelGGL((k_prec_apply<V, F>), dim3(M.nblk), dim3(kBlock), 0, s, view<V>(*a.C), M, a.act, a.m, a.lam, \
                       a.g, a.p, a.q, a.part, a.flags, ph + 1)
    if (a.fp32) {
        if (a.form == 1) MMNCG_PREC_APPLY(float, 1);
        else if (a.form == 2) MMNCG_PREC_APPLY(float, 2);
        else MMNCG_PREC_APPLY(float, 0);
    } else {
        if (a.form == 1) MMNCG_PREC_APPLY(double, 1);
        else if (a.form == 2) MMNCG_PREC_APPLY(double, 2);
        else MMNCG_PREC_APPLY(double, 0);
    }
#undef MMNCG_PREC_APPLY
}

void launch_prec_tail(const PrecLaunch &a, int j, bool last, hipStream_t s) {
    const RowMap &M = *a.M;
    const int ph = 3 * j;
    hipLaunchKernelGGL(k_prec_update, dim3(M.nblk), dim3(kBlock), 0, s, M, a.act, j, a.g, a.invDex, a.dscale, a.y,
                       a.r, a.p, a.q, a.part, a.flags, ph + 2);
    if (!last)
        hipLaunchKernelGGL(k_prec_pupdate, dim3(M.nblk), dim3(kBlock), 0, s, M, a.act, j, a.invDex, a.dscale, a.p, a.r,
                           a.part, a.flags, ph + 3);
}

void launch_dir(const RowMap &M, const int *act, const int *first, const double *g1, const double *g0,
                const double *y1, double *d, double *part_dots, double *part_out, int *info, int beta_kind,
                double *gy, hipStream_t s) {
    hipLaunchKernelGGL(k_dir_dots, dim3(M.nblk), dim3(kBlock), 0, s, M, act, first, g1, g0, y1, d, part_dots,
                       (const double *)gy, gy + M.ninst);
    hipLaunchKernelGGL(k_dir_update, dim3(M.nblk), dim3(kBlock), 0, s, M, act, first, g1, y1, d, part_dots, part_out,
                       info, beta_kind, (const double *)(gy + M.ninst), gy);
}

void launch_energy_split(const Sell &S, const RowMap &M, const double *m, double *part, bool fp32, hipStream_t s) {
    if (fp32) hipLaunchKernelGGL(k_energy_split<float>, dim3(M.nblk), dim3(kBlock), 0, s, view<float>(S), M, m, part);
    else hipLaunchKernelGGL(k_energy_split<double>, dim3(M.nblk), dim3(kBlock), 0, s, view<double>(S), M, m, part);
}
void launch_mavg(const RowMap &M, const double *m, const double *L, double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_mavg, dim3(M.nblk), dim3(kBlock), 0, s, M, m, L, part);
}
void launch_lambda(const RowMap &M, const double *m, const double *G, double *lam, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda, dim3(M.nblk), dim3(kBlock), 0, s, M, m, G, lam);
}
void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)g), dim3(kBlock), 0, s, n, x, y);
}
void launch_fill(int64_t n, double *x, double v, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(kBlock), 0, s, n, x, v);
}

void launch_pot_op(const RowMap &M, const int *op, const double *rho, double *u, double *ux, double *ut,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_pot_op, dim3(M.nblk), dim3(kBlock), 0, s, M, op, rho, u, ux, ut);
}
void launch_gather(int64_t n, const int *idx, const double *in, double *out, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)g), dim3(kBlock), 0, s, n, idx, in, out);
}

}  // namespace mmncg
