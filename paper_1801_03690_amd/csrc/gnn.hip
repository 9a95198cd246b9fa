// HIP kernels (gfx950) of the learned component: a per-node graph network on
// the magnet nodes that proposes the start of the next minimization and a
// scaling of the preconditioner's Jacobi diagonal (not part of the paper's
// method; the method's own minimizer always runs to the same tolerance).
//
// Dense layers run on the matrix cores: gfx950's v_mfma_f32_16x16x32_bf16
// with BF16 operands (FP32 activations and FP32 master weights rounded to
// nearest even when loaded) and FP32 accumulation; a debug mode runs the same
// products with FP32 operands on the vector units. Neighbour means, heads, losses and the
// optimizer run in FP32 on the vector units. Every reduction over nodes is a
// fixed-order two-stage sum (per-block partials, then one pass over the
// blocks): no floating-point atomics, so training is deterministic.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mmncg {

namespace {

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// D += A B on one 16 x 16 tile, k = 32: lane l supplies A(l % 16, 8 (l / 16) + j)
// and B(8 (l / 16) + j, l % 16), j = 0..7 (BF16 bit patterns), and holds
// D(4 (l / 16) + j, l % 16), j = 0..3
__device__ __forceinline__ f32x4 mfma32(const s16x8 &a, const s16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                    0, 0);
}

constexpr int kGB = 256;   // threads per block
constexpr int kRowsPerBlock = 64;   // rows of the row-GEMM per block (16 per wave)
constexpr int kTnRows = 256;        // rows reduced per block in the weight-gradient products

__device__ __forceinline__ short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float silu_f(float x) { return x * sigm(x); }
__device__ __forceinline__ float dsilu_f(float x) {
    float s = sigm(x);
    return s * (1.0f + x * (1.0f - s));
}

// epilogue of the row products: Y = v (0), Ypre = v and Y = silu(v) (1),
// Y = R + v (2), Y += v (3)
template <int EPI>
__device__ __forceinline__ void mm_store(int row, int col, float v, float *__restrict__ Y, int ldy,
                                         float *__restrict__ Ypre, int ldp, const float *__restrict__ R, int ldr) {
    if (EPI == 0) {
        Y[(size_t)row * ldy + col] = v;
    } else if (EPI == 1) {
        Ypre[(size_t)row * ldp + col] = v;
        Y[(size_t)row * ldy + col] = silu_f(v);
    } else if (EPI == 2) {
        Y[(size_t)row * ldy + col] = R[(size_t)row * ldr + col] + v;
    } else {
        Y[(size_t)row * ldy + col] += v;
    }
}

// ---------------------------------------------------------------------------
// Y[M x NC] = A[M x K] B[K x NC] (+ bias) with an epilogue.
// A(i, k) = A[i * lda + k]; B(k, j) = W[k * ldw + j], or W[j * ldw + k] when
// transposed. A block stages B in LDS as BF16 and computes 64 rows; wave w
// owns rows 16w..16w+15 and all NC columns (NC / 16 MFMA tiles of mfma32).
// K is a multiple of 32.
// ---------------------------------------------------------------------------
template <int NC, int EPI>
__global__ __launch_bounds__(kGB) void k_mm(int M, int K, const float *__restrict__ A, int lda,
                                            const float *__restrict__ W, int ldw, int transW,
                                            const float *__restrict__ bias, float *__restrict__ Y, int ldy,
                                            float *__restrict__ Ypre, int ldp, const float *__restrict__ R, int ldr) {
    __shared__ short Bs[128 * NC];
    for (int e = threadIdx.x; e < K * NC; e += kGB) {
        int k = e / NC, j = e % NC;
        Bs[e] = to_bf16(transW ? W[(size_t)j * ldw + k] : W[(size_t)k * ldw + j]);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blockIdx.x * kRowsPerBlock + 16 * w;
    const int li = lane & 15, lk = 8 * (lane >> 4), lo = 4 * (lane >> 4);
    f32x4 acc[NC / 16];
#pragma unroll
    for (int t = 0; t < NC / 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int arow = r0 + li;
    for (int k0 = 0; k0 < K; k0 += 32) {
        s16x8 a;
        if (arow < M) {
            const float *ap = A + (size_t)arow * lda + k0 + lk;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = to_bf16(ap[j]);
        } else {
            a = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
#pragma unroll
        for (int t = 0; t < NC / 16; ++t) {
            const short *bp = Bs + (size_t)(k0 + lk) * NC + 16 * t + li;
            s16x8 b;
#pragma unroll
            for (int j = 0; j < 8; ++j) b[j] = bp[j * NC];
            acc[t] = mfma32(a, b, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NC / 16; ++t) {
        const int col = 16 * t + li;
        const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = r0 + lo + j;
            if (row < M) mm_store<EPI>(row, col, acc[t][j] + bv, Y, ldy, Ypre, ldp, R, ldr);
        }
    }
}

// the same product with FP32 operands on the vector units (the debug mode):
// one thread per output, k summed in order
template <int NC, int EPI>
__global__ __launch_bounds__(kGB) void k_mm32(int M, int K, const float *__restrict__ A, int lda,
                                              const float *__restrict__ W, int ldw, int transW,
                                              const float *__restrict__ bias, float *__restrict__ Y, int ldy,
                                              float *__restrict__ Ypre, int ldp, const float *__restrict__ R,
                                              int ldr) {
    const int64_t e = (int64_t)blockIdx.x * kGB + threadIdx.x;
    if (e >= (int64_t)M * NC) return;
    const int row = (int)(e / NC), col = (int)(e % NC);
    float acc = 0.0f;
    for (int k = 0; k < K; ++k)
        acc = fmaf(A[(size_t)row * lda + k], transW ? W[(size_t)col * ldw + k] : W[(size_t)k * ldw + col], acc);
    mm_store<EPI>(row, col, acc + (bias ? bias[col] : 0.0f), Y, ldy, Ypre, ldp, R, ldr);
}

// ---------------------------------------------------------------------------
// weight gradients: part[blk][KI x NC] = sum over the block's rows r of
// A[r][i] B[r][j] (MFMA with the rows as the reduction dimension, 32 rows per
// step: lane l supplies rows r0 + 8 (l / 16) + j); the partials are summed
// over blocks by k_reduce_blocks
// ---------------------------------------------------------------------------
template <int KI, int NC>
__global__ __launch_bounds__(kGB) void k_mm_tn(int M, const float *__restrict__ A, int lda,
                                               const float *__restrict__ B, int ldb, float *__restrict__ part) {
    constexpr int TI = KI / 16, TJ = NC / 16, NT = TI * TJ, TPW = (NT + 3) / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = 8 * (lane >> 4), lo = 4 * (lane >> 4);
    const int rbeg = blockIdx.x * kTnRows;
    f32x4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int r0 = rbeg; r0 < rbeg + kTnRows && r0 < M; r0 += 32) {
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = w + 4 * q;
            if (tile >= NT) continue;
            const int it = tile / TJ, jt = tile % TJ;
            s16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int r = r0 + lk + j;
                a[j] = r < M ? to_bf16(A[(size_t)r * lda + 16 * it + li]) : (short)0;
                b[j] = r < M ? to_bf16(B[(size_t)r * ldb + 16 * jt + li]) : (short)0;
            }
            acc[q] = mfma32(a, b, acc[q]);
        }
    }
    float *out = part + (size_t)blockIdx.x * KI * NC;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = w + 4 * q;
        if (tile >= NT) continue;
        const int it = tile / TJ, jt = tile % TJ;
#pragma unroll
        for (int j = 0; j < 4; ++j) out[(16 * it + lo + j) * NC + 16 * jt + li] = acc[q][j];
    }
}

// FP32 version (small products, and every weight gradient in the debug
// mode): thread t of block row y owns output t + 256 y = (i, j), i = . / NC;
// A == null means a column of ones (column sums of B)
__global__ __launch_bounds__(kGB) void k_tn32(int M, int KI, int NC, const float *__restrict__ A, int lda,
                                              const float *__restrict__ B, int ldb, float *__restrict__ part) {
    const int t = threadIdx.x + kGB * blockIdx.y;
    if (t >= KI * NC) return;
    const int i = t / NC, j = t % NC;
    const int rbeg = blockIdx.x * kTnRows;
    const int rend = min(M, rbeg + kTnRows);
    float acc = 0.0f;
    for (int r = rbeg; r < rend; ++r) acc += (A ? A[(size_t)r * lda + i] : 1.0f) * B[(size_t)r * ldb + j];
    part[(size_t)blockIdx.x * KI * NC + t] = acc;
}

// out[e] (=, or += when accumulate) = sum over blocks b of part[b][e], in order
__global__ __launch_bounds__(kGB) void k_reduce_blocks(int nblk, int len, const float *__restrict__ part,
                                                       float *__restrict__ out, int accumulate) {
    const int e = blockIdx.x * kGB + threadIdx.x;
    if (e >= len) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * len + e];
    out[e] = accumulate ? out[e] + s : s;
}

// ---------------------------------------------------------------------------
// graph kernels (one wave per node, lane = channel of 64)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_agg(int n, const int *__restrict__ ptr, const int *__restrict__ idx,
                                             const float *__restrict__ invdeg, const float *__restrict__ H, int ldh,
                                             float *__restrict__ out, int ldo) {
    const int i = blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), c = threadIdx.x & 63;
    if (i >= n) return;
    float s = 0.0f;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) s += H[(size_t)idx[e] * ldh + c];
    out[(size_t)i * ldo + c] = s * invdeg[i];
}

// out[j] += sum over neighbours i of j of G[i] / deg_i (adjacency is symmetric)
__global__ __launch_bounds__(kGB) void k_agg_t_add(int n, const int *__restrict__ ptr, const int *__restrict__ idx,
                                                   const float *__restrict__ invdeg, const float *__restrict__ G,
                                                   int ldg, float *__restrict__ out, int ldo) {
    const int j = blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), c = threadIdx.x & 63;
    if (j >= n) return;
    float s = 0.0f;
    for (int e = ptr[j]; e < ptr[j + 1]; ++e) {
        const int i = idx[e];
        s += G[(size_t)i * ldg + c] * invdeg[i];
    }
    out[(size_t)j * ldo + c] += s;
}

// q[i][c] += sum_e ebar[i][e] We2[e][c]
__global__ __launch_bounds__(kGB) void k_edge_add(int n, const float *__restrict__ ebar,
                                                  const float *__restrict__ We2, float *__restrict__ q, int ldq) {
    const int i = blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), c = threadIdx.x & 63;
    if (i >= n) return;
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) s += ebar[4 * i + e] * We2[e * 64 + c];
    q[(size_t)i * ldq + c] += s;
}

// y[i][c] = x[i][c] * silu'(pre[i][c]) (contiguous n x 64)
__global__ __launch_bounds__(kGB) void k_silu_bwd(int64_t len, const float *__restrict__ x,
                                                  const float *__restrict__ pre, float *__restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * kGB + threadIdx.x;
    if (e < len) y[e] = x[e] * dsilu_f(pre[e]);
}

// out[i][c] += in[i * ldi + c] for c < 64
__global__ __launch_bounds__(kGB) void k_add64(int n, const float *__restrict__ in, int ldi, float *__restrict__ out,
                                               int ldo) {
    const int i = blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), c = threadIdx.x & 63;
    if (i < n) out[(size_t)i * ldo + c] += in[(size_t)i * ldi + c];
}

__global__ __launch_bounds__(kGB) void k_copy64(int n, const float *__restrict__ in, int ldi, float *__restrict__ out,
                                                int ldo) {
    const int i = blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), c = threadIdx.x & 63;
    if (i < n) out[(size_t)i * ldo + c] = in[(size_t)i * ldi + c];
}

// ---------------------------------------------------------------------------
// heads: zm = h Wm + bm, dm = zm - (zm.m) m; zs = h Ws + bs,
// s = clip(softplus(zs) + 1/4, 1/4, 4)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void k_heads(int n, const float *__restrict__ h, const float *__restrict__ Wm,
                                               const float *__restrict__ bm, const float *__restrict__ Ws,
                                               const float *__restrict__ bs, const double *__restrict__ m,
                                               float *__restrict__ zm, float *__restrict__ zs, double *__restrict__ dm,
                                               double *__restrict__ s) {
    const int i = blockIdx.x * kGB + threadIdx.x;
    if (i >= n) return;
    float a0 = bm[0], a1 = bm[1], a2 = bm[2], as = bs[0];
    const float *hi = h + (size_t)i * 64;
    for (int c = 0; c < 64; ++c) {
        const float v = hi[c];
        a0 += v * Wm[3 * c];
        a1 += v * Wm[3 * c + 1];
        a2 += v * Wm[3 * c + 2];
        as += v * Ws[c];
    }
    zm[3 * i] = a0;
    zm[3 * i + 1] = a1;
    zm[3 * i + 2] = a2;
    zs[i] = as;
    const double m0 = m[3 * i], m1 = m[3 * i + 1], m2 = m[3 * i + 2];
    const double p = a0 * m0 + a1 * m1 + a2 * m2;
    if (dm) {
        dm[3 * i] = a0 - p * m0;
        dm[3 * i + 1] = a1 - p * m1;
        dm[3 * i + 2] = a2 - p * m2;
    }
    const float sp = (as > 20.0f ? as : log1pf(__expf(as))) + 0.25f;
    if (s) s[i] = fminf(fmaxf(sp, 0.25f), 4.0f);
}

// loss terms and the gradients at the heads' inputs:
//   d_zm = P_m (inv_dm2 2 L (dm - dm*) / sum L), d_zs = w_s 2 (log s - log s*) / (n s) * sigma(zs) inside the clip;
// block partial of the loss
__global__ __launch_bounds__(kGB) void k_loss_heads(int n, const float *__restrict__ zm, const float *__restrict__ zs,
                                                    const double *__restrict__ m, const double *__restrict__ dm_t,
                                                    const double *__restrict__ s_t, const double *__restrict__ L,
                                                    double inv_sumL, double inv_dm2, double w_s, double inv_n,
                                                    float *__restrict__ d_zm, float *__restrict__ d_zs,
                                                    double *__restrict__ part) {
    __shared__ double sh[kGB / 64];
    const int i = blockIdx.x * kGB + threadIdx.x;
    double lv = 0.0;
    if (i < n) {
        const double m0 = m[3 * i], m1 = m[3 * i + 1], m2 = m[3 * i + 2];
        const double z0 = zm[3 * i], z1 = zm[3 * i + 1], z2 = zm[3 * i + 2];
        const double p = z0 * m0 + z1 * m1 + z2 * m2;
        const double e0 = z0 - p * m0 - dm_t[3 * i], e1 = z1 - p * m1 - dm_t[3 * i + 1],
                     e2 = z2 - p * m2 - dm_t[3 * i + 2];
        const double cw = inv_dm2 * L[i] * inv_sumL;
        lv += cw * (e0 * e0 + e1 * e1 + e2 * e2);
        const double g0 = 2.0 * cw * e0, g1 = 2.0 * cw * e1, g2 = 2.0 * cw * e2;
        const double gp = g0 * m0 + g1 * m1 + g2 * m2;
        d_zm[3 * i] = (float)(g0 - gp * m0);
        d_zm[3 * i + 1] = (float)(g1 - gp * m1);
        d_zm[3 * i + 2] = (float)(g2 - gp * m2);
        const double z = zs[i];
        const double sp = (z > 20.0 ? z : log1p(exp(z))) + 0.25;
        const double s = fmin(fmax(sp, 0.25), 4.0);
        const double dl = log(s) - log(s_t[i]);
        lv += w_s * inv_n * dl * dl;
        const double inside = (sp > 0.25 && sp < 4.0) ? 1.0 : 0.0;
        d_zs[i] = (float)(w_s * inv_n * 2.0 * dl / s * inside / (1.0 + exp(-z)));
    }
    // block sum in a fixed order
    for (int off = 32; off > 0; off >>= 1) lv += __shfl_xor(lv, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = lv;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(kGB) void k_sum_blocks(int nblk, const double *__restrict__ part, double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    out[0] = s;
}

// dh[i][c] = d_zm[i] . Wm[c] + d_zs[i] Ws[c]
__global__ __launch_bounds__(kGB) void k_heads_dh(int n, const float *__restrict__ d_zm, const float *__restrict__ d_zs,
                                                  const float *__restrict__ Wm, const float *__restrict__ Ws,
                                                  float *__restrict__ dh) {
    const int i = blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), c = threadIdx.x & 63;
    if (i >= n) return;
    dh[(size_t)i * 64 + c] = d_zm[3 * i] * Wm[3 * c] + d_zm[3 * i + 1] * Wm[3 * c + 1] +
                             d_zm[3 * i + 2] * Wm[3 * c + 2] + d_zs[i] * Ws[c];
}

// Adam with bias correction (bc1 = 1 - b1^t, bc2 = 1 - b2^t)
__global__ __launch_bounds__(kGB) void k_adam(int np, float *__restrict__ th, const float *__restrict__ g,
                                              float *__restrict__ m1, float *__restrict__ m2, float lr, float b1,
                                              float b2, float eps, float bc1, float bc2) {
    const int e = blockIdx.x * kGB + threadIdx.x;
    if (e >= np) return;
    const float gi = g[e];
    const float a = b1 * m1[e] + (1.0f - b1) * gi;
    const float v = b2 * m2[e] + (1.0f - b2) * gi * gi;
    m1[e] = a;
    m2[e] = v;
    th[e] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
}

// node features (columns as in the oracle): 0-2 m, 3-5 h_next, 6-8 h_next -
// h_prev, 9-11 -(C m)/L, 12-14 -(G - C m + L h_next)/L, 15-17 -g/L, 18-20
// static (D / mean D, L / mean L, deg / max deg), 21-31 zero
__global__ __launch_bounds__(kGB) void k_features(int n, const double *__restrict__ m, const double *__restrict__ G,
                                                  const double *__restrict__ g, const double *__restrict__ Cm,
                                                  const double *__restrict__ L, const float *__restrict__ stat,
                                                  double hn0, double hn1, double hn2, double hp0, double hp1,
                                                  double hp2, float *__restrict__ X) {
    const int i = blockIdx.x * kGB + threadIdx.x;
    if (i >= n) return;
    float *x = X + (size_t)i * 32;
    const double La = L[i];
    const double hn[3] = {hn0, hn1, hn2}, hp[3] = {hp0, hp1, hp2};
    for (int c = 0; c < 3; ++c) {
        const int64_t e = 3 * (int64_t)i + c;
        x[c] = (float)m[e];
        x[3 + c] = (float)hn[c];
        x[6 + c] = (float)(hn[c] - hp[c]);
        x[9 + c] = (float)(-Cm[e] / La);
        x[12 + c] = (float)(-(G[e] - Cm[e] + La * hn[c]) / La);
        x[15 + c] = (float)(-g[e] / La);
    }
    x[18] = stat[3 * i];
    x[19] = stat[3 * i + 1];
    x[20] = stat[3 * i + 2];
    for (int c = 21; c < 32; ++c) x[c] = 0.0f;
}

// Xn = (X - mu) / sd, column-wise over the 32 features (FP32, before any BF16 rounding)
__global__ __launch_bounds__(kGB) void k_norm_features(int64_t n32, const float *__restrict__ X,
                                                       const float *__restrict__ mu, const float *__restrict__ sd,
                                                       float *__restrict__ Xn) {
    const int64_t e = (int64_t)blockIdx.x * kGB + threadIdx.x;
    if (e < n32) {
        const int c = (int)(e & 31);
        Xn[e] = (X[e] - mu[c]) / sd[c];
    }
}

__global__ void k_f64_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * kGB + threadIdx.x;
    if (e < n) b[e] = (float)a[e];
}
__global__ void k_f32_to_f64(int64_t n, const float *__restrict__ a, double *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * kGB + threadIdx.x;
    if (e < n) b[e] = (double)a[e];
}

// training targets per node a: dm*_a = P_{m_a}(m1_a - m_a) (the step to the
// next minimizer in the tangent plane of m_a) and s*_a = 1 + t_a / D_a with
// t_a the mean over the two directions normal to m_a of the magnetostatic
// Hessian's diagonal (diag3, per component): t = (sum_c diag_c - sum_c
// m_c^2 diag_c) / 2; invD = 1 / D
__global__ __launch_bounds__(kGB) void k_targets(int n, const double *__restrict__ m, const double *__restrict__ m1,
                                                 const double *__restrict__ diag3, const double *__restrict__ invD,
                                                 double *__restrict__ dmt, double *__restrict__ st) {
    const int a = blockIdx.x * kGB + threadIdx.x;
    if (a >= n) return;
    const int64_t a3 = 3 * (int64_t)a;
    const double m0 = m[a3], mx = m[a3 + 1], mz = m[a3 + 2];
    const double d0 = m1[a3] - m0, d1 = m1[a3 + 1] - mx, d2 = m1[a3 + 2] - mz;
    const double dm = d0 * m0 + d1 * mx + d2 * mz;
    dmt[a3] = d0 - dm * m0;
    dmt[a3 + 1] = d1 - dm * mx;
    dmt[a3 + 2] = d2 - dm * mz;
    const double g0 = diag3[a3], g1 = diag3[a3 + 1], g2 = diag3[a3 + 2];
    const double t = 0.5 * ((g0 + g1 + g2) - (m0 * m0 * g0 + mx * mx * g1 + mz * mz * g2));
    st[a] = 1.0 + t * invD[a];
}

// column sums and sums of squares of X (n x 32) in FP64: block b writes the
// 64 partials of its rows (thread t: column t % 32, every 8th row), summed
// over blocks in order by k_sum_cols
constexpr int kMomRows = 2048;
__global__ __launch_bounds__(kGB) void k_moments(int n, const float *__restrict__ X, double *__restrict__ part) {
    __shared__ double sh[kGB][2];
    const int col = threadIdx.x % 32, rg = threadIdx.x / 32;
    const int r0 = blockIdx.x * kMomRows, r1 = min(n, r0 + kMomRows);
    double s1 = 0.0, s2 = 0.0;
    for (int r = r0 + rg; r < r1; r += kGB / 32) {
        const double x = (double)X[(int64_t)r * 32 + col];
        s1 += x;
        s2 += x * x;
    }
    sh[threadIdx.x][0] = s1;
    sh[threadIdx.x][1] = s2;
    __syncthreads();
    if (threadIdx.x < 32) {
        double a = 0.0, b = 0.0;
        for (int g = 0; g < kGB / 32; ++g) {
            a += sh[g * 32 + threadIdx.x][0];
            b += sh[g * 32 + threadIdx.x][1];
        }
        part[(int64_t)blockIdx.x * 64 + threadIdx.x] = a;
        part[(int64_t)blockIdx.x * 64 + 32 + threadIdx.x] = b;
    }
}
__global__ void k_sum_cols(int nblk, const double *__restrict__ part, double *__restrict__ out) {
    const int q = threadIdx.x;  // 64 threads
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(int64_t)b * 64 + q];
    out[q] = acc;
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void gnn_targets(int n, const double *m, const double *m1, const double *diag3, const double *invD, double *dmt,
                 double *st, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_targets, dim3(blocks_for(n, kGB)), dim3(kGB), 0, s, n, m, m1, diag3, invD, dmt, st);
}
int gnn_moment_blocks(int n) { return n > 0 ? (int)blocks_for(n, kMomRows) : 1; }
void gnn_moments(int n, const float *X, double *part, double *out, hipStream_t s) {
    const int nb = gnn_moment_blocks(n);
    hipLaunchKernelGGL(k_moments, dim3(nb), dim3(kGB), 0, s, n, X, part);
    hipLaunchKernelGGL(k_sum_cols, dim3(1), dim3(64), 0, s, nb, (const double *)part, out);
}

// ===========================================================================
// launchers
// ===========================================================================
void gnn_mm(int M, int K, int NC, int epi, const float *A, int lda, const float *W, int ldw, bool transW,
            const float *bias, float *Y, int ldy, float *Ypre, int ldp, const float *R, int ldr, bool f32,
            hipStream_t s) {
    if (M <= 0) return;
    const dim3 g(f32 ? blocks_for((int64_t)M * NC, kGB) : blocks_for(M, kRowsPerBlock)), b(kGB);
#define MMNCG_MM(NCV, E)                                                                                             \
    if (f32)                                                                                                         \
        hipLaunchKernelGGL((k_mm32<NCV, E>), g, b, 0, s, M, K, A, lda, W, ldw, transW ? 1 : 0, bias, Y, ldy, Ypre, ldp, \
                           R, ldr);                                                                                  \
    else                                                                                                             \
        hipLaunchKernelGGL((k_mm<NCV, E>), g, b, 0, s, M, K, A, lda, W, ldw, transW ? 1 : 0, bias, Y, ldy, Ypre, ldp, \
                           R, ldr)
#define MMNCG_MM_E(NCV)          \
    switch (epi) {               \
        case 0: MMNCG_MM(NCV, 0); break; \
        case 1: MMNCG_MM(NCV, 1); break; \
        case 2: MMNCG_MM(NCV, 2); break; \
        default: MMNCG_MM(NCV, 3); break; \
    }
    if (NC == 32) {
        MMNCG_MM_E(32)
    } else if (NC == 64) {
        MMNCG_MM_E(64)
    } else {
        MMNCG_MM_E(128)
    }
#undef MMNCG_MM_E
#undef MMNCG_MM
}

int gnn_tn_blocks(int M) { return (int)blocks_for(M, kTnRows); }

void gnn_mm_tn(int M, int KI, int NC, const float *A, int lda, const float *B, int ldb, float *part, float *out,
               bool accumulate, bool f32, hipStream_t s) {
    const int nb = gnn_tn_blocks(M);
    if (M <= 0) return;
    if (f32) hipLaunchKernelGGL(k_tn32, dim3(nb, blocks_for(KI * 64, kGB)), dim3(kGB), 0, s, M, KI, 64, A, lda, B, ldb, part);
    else if (KI == 32) hipLaunchKernelGGL((k_mm_tn<32, 64>), dim3(nb), dim3(kGB), 0, s, M, A, lda, B, ldb, part);
    else if (KI == 64) hipLaunchKernelGGL((k_mm_tn<64, 64>), dim3(nb), dim3(kGB), 0, s, M, A, lda, B, ldb, part);
    else hipLaunchKernelGGL((k_mm_tn<128, 64>), dim3(nb), dim3(kGB), 0, s, M, A, lda, B, ldb, part);
    (void)NC;
    const int len = KI * 64;
    hipLaunchKernelGGL(k_reduce_blocks, dim3(blocks_for(len, kGB)), dim3(kGB), 0, s, nb, len, (const float *)part, out,
                       accumulate ? 1 : 0);
}

void gnn_tn32(int M, int KI, int NC, const float *A, int lda, const float *B, int ldb, float *part, float *out,
              hipStream_t s) {
    const int nb = gnn_tn_blocks(M);
    if (M <= 0) return;
    hipLaunchKernelGGL(k_tn32, dim3(nb), dim3(kGB), 0, s, M, KI, NC, A, lda, B, ldb, part);
    const int len = KI * NC;
    hipLaunchKernelGGL(k_reduce_blocks, dim3(blocks_for(len, kGB)), dim3(kGB), 0, s, nb, len, (const float *)part, out,
                       0);
}

void gnn_agg(int n, const int *ptr, const int *idx, const float *invdeg, const float *H, int ldh, float *out, int ldo,
             hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_agg, dim3(blocks_for(n, kGB / 64)), dim3(kGB), 0, s, n, ptr, idx, invdeg, H, ldh, out, ldo);
}
void gnn_agg_t_add(int n, const int *ptr, const int *idx, const float *invdeg, const float *G, int ldg, float *out,
                   int ldo, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_agg_t_add, dim3(blocks_for(n, kGB / 64)), dim3(kGB), 0, s, n, ptr, idx, invdeg, G, ldg,
                           out, ldo);
}
void gnn_edge_add(int n, const float *ebar, const float *We2, float *q, int ldq, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_edge_add, dim3(blocks_for(n, kGB / 64)), dim3(kGB), 0, s, n, ebar, We2, q, ldq);
}
void gnn_silu_bwd(int64_t len, const float *x, const float *pre, float *y, hipStream_t s) {
    if (len > 0) hipLaunchKernelGGL(k_silu_bwd, dim3(blocks_for(len, kGB)), dim3(kGB), 0, s, len, x, pre, y);
}
void gnn_add64(int n, const float *in, int ldi, float *out, int ldo, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_add64, dim3(blocks_for(n, kGB / 64)), dim3(kGB), 0, s, n, in, ldi, out, ldo);
}
void gnn_copy64(int n, const float *in, int ldi, float *out, int ldo, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_copy64, dim3(blocks_for(n, kGB / 64)), dim3(kGB), 0, s, n, in, ldi, out, ldo);
}
void gnn_heads(int n, const float *h, const float *Wm, const float *bm, const float *Ws, const float *bs,
               const double *m, float *zm, float *zs, double *dm, double *sv, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_heads, dim3(blocks_for(n, kGB)), dim3(kGB), 0, s, n, h, Wm, bm, Ws, bs, m, zm, zs, dm, sv);
}
int gnn_loss_blocks(int n) { return (int)blocks_for(n, kGB); }
void gnn_loss_heads(int n, const float *zm, const float *zs, const double *m, const double *dm_t, const double *s_t,
                    const double *L, double inv_sumL, double inv_dm2, double w_s, float *d_zm, float *d_zs,
                    double *part, double *loss_out, hipStream_t s) {
    const int nb = gnn_loss_blocks(n);
    hipLaunchKernelGGL(k_loss_heads, dim3(nb), dim3(kGB), 0, s, n, zm, zs, m, dm_t, s_t, L, inv_sumL, inv_dm2, w_s,
                       1.0 / n, d_zm, d_zs, part);
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(64), 0, s, nb, (const double *)part, loss_out);
}
void gnn_heads_dh(int n, const float *d_zm, const float *d_zs, const float *Wm, const float *Ws, float *dh,
                  hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_heads_dh, dim3(blocks_for(n, kGB / 64)), dim3(kGB), 0, s, n, d_zm, d_zs, Wm, Ws, dh);
}
void gnn_adam(int np, float *th, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps,
              float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(np, kGB)), dim3(kGB), 0, s, np, th, g, m1, m2, lr, b1, b2, eps, bc1,
                       bc2);
}
void gnn_features(int n, const double *m, const double *G, const double *g, const double *Cm, const double *L,
                  const float *stat, const double hn[3], const double hp[3], float *X, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_features, dim3(blocks_for(n, kGB)), dim3(kGB), 0, s, n, m, G, g, Cm, L, stat, hn[0], hn[1],
                           hn[2], hp[0], hp[1], hp[2], X);
}
void gnn_norm_features(int n, const float *X, const float *mu, const float *sd, float *Xn, hipStream_t s) {
    const int64_t n32 = 32 * (int64_t)n;
    if (n32 > 0) hipLaunchKernelGGL(k_norm_features, dim3(blocks_for(n32, kGB)), dim3(kGB), 0, s, n32, X, mu, sd, Xn);
}
void gnn_f64_to_f32(int64_t n, const double *a, float *b, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks_for(n, kGB)), dim3(kGB), 0, s, n, a, b);
}
void gnn_f32_to_f64(int64_t n, const float *a, double *b, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks_for(n, kGB)), dim3(kGB), 0, s, n, a, b);
}

}  // namespace mmncg
