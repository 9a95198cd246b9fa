// Host side of the learned component (not part of the paper's method): the
// graph of a context's magnet nodes, the network's parameters and optimizer
// state, forward and backward passes built from the kernels of gnn.hip, the
// Hutchinson probe of the magnetostatic diagonal, and the proposal the curve
// driver asks for at each new field value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <set>
#include <vector>

#include "context.h"

struct mm_graph {
    mm_ctx *c = nullptr;
    int n = 0;
    long nnz = 0;
    int *ptr = nullptr, *idx = nullptr;
    float *invdeg = nullptr, *ebar = nullptr, *stat = nullptr, *X = nullptr;
    double sumL = 0.0;
    std::vector<void *> mem;
};

// The network is independent of any one context: it keeps the device, the
// stream and the allocator callbacks of the context it was created on (not
// that context's buffers), so graphs of other contexts on the same device can
// use it and it survives their uploads.
struct mm_gnn {
    int device = 0;
    hipStream_t stream = nullptr;
    mm_alloc_fn ualloc = nullptr;
    mm_free_fn ufree = nullptr;
    void *user = nullptr;
    std::string err;
    float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    float *mu = nullptr, *sd = nullptr;   // input standardization (32 each)
    long t = 0;
    bool f32 = false;  // debug mode: FP32 operands in the dense layers (mm_gnn_set_precision)
    int cap = 0;  // workspace rows
    std::vector<void *> ws;
    float *X = nullptr, *Xn = nullptr, *y0 = nullptr, *h3 = nullptr, *zm = nullptr, *zs = nullptr, *dh = nullptr, *dt = nullptr,
          *dy = nullptr, *dz = nullptr, *da = nullptr, *d_zm = nullptr, *d_zs = nullptr, *part = nullptr;
    float *z[3] = {}, *a[3] = {}, *y1[3] = {}, *tt[3] = {};
    double *m = nullptr, *dmt = nullptr, *st = nullptr, *lpart = nullptr, *loss = nullptr, *dm = nullptr,
           *s = nullptr;
    std::vector<void *> mem;
};

namespace mmncg {
namespace {

constexpr int kF = 32, kW = 64, kLayers = 3;
// flat parameter offsets (row-major [in][out]; see the C ABI)
constexpr int oWin = 0, oBin = kF * kW, oLayer0 = oBin + kW;
constexpr int kLayerSize = kW * kW + 4 * kW + 2 * kW * kW + kW + kW * kW + kW;
constexpr int oHeads = oLayer0 + kLayers * kLayerSize;
constexpr int kNParams = oHeads + kW * 3 + 3 + kW + 1;
int oWe1(int l) { return oLayer0 + l * kLayerSize; }
int oWe2(int l) { return oWe1(l) + kW * kW; }
int oW1(int l) { return oWe2(l) + 4 * kW; }
int ob1(int l) { return oW1(l) + 2 * kW * kW; }
int oW2(int l) { return ob1(l) + kW; }
int ob2(int l) { return oW2(l) + kW * kW; }
constexpr int oWm = oHeads, obm = oWm + kW * 3, oWs = obm + 3, obs = oWs + kW;

template <class T>
T *galloc(mm_ctx *c, std::vector<void *> &keep, size_t n) {
    T *p = dalloc_n<T>(c, n);
    keep.push_back(p);
    return p;
}
void release(mm_ctx *c, std::vector<void *> &keep) {
    for (void *p : keep) dfree(c, p);
    keep.clear();
}

// network memory: the creating context's allocator, not tracked by it
template <class T>
T *nalloc(mm_gnn *g, std::vector<void *> &keep, size_t n) {
    size_t bytes = std::max<size_t>(n * sizeof(T), 256);
    void *p = nullptr;
    if (g->ualloc) {
        p = g->ualloc(bytes, g->user);
        if (!p) throw ApiError{MM_ENOMEM, "device allocation callback failed"};
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw ApiError{MM_ENOMEM, "hipMalloc failed"};
    }
    keep.push_back(p);
    return (T *)p;
}
void nrelease(mm_gnn *g, std::vector<void *> &keep) {
    for (void *p : keep) {
        if (g->ufree) g->ufree(p, g->user);
        else (void)hipFree(p);
    }
    keep.clear();
}

template <class F>
int gguard(mm_gnn *g, F &&f) {
    if (!g) return MM_EINVAL;
    try {
        HIPCHK(hipSetDevice(g->device));
        int rc = f();
        if (rc >= 0) g->err.clear();
        return rc;
    } catch (const ApiError &e) {
        g->err = e.msg;
        return e.code;
    } catch (const HipError &e) {
        g->err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
        (void)hipGetLastError();
        return MM_EDEVICE;
    } catch (const std::bad_alloc &) {
        g->err = "host allocation failed";
        return MM_ENOMEM;
    } catch (const std::exception &e) {
        g->err = e.what();
        return MM_EDEVICE;
    }
}
void gsync(mm_gnn *g) { HIPCHK(hipStreamSynchronize(g->stream)); }

void copy_d_in(hipStream_t s, double *dst, const double *src, size_t n) {
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}
void copy_d_out(hipStream_t s, double *dst, const double *src, size_t n) {
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
}

void copy_f32_in(hipStream_t s, float *dst, const float *src, size_t n) {
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(float),
                          is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}
void copy_f32_out(mm_ctx *c, float *dst, const float *src, size_t n) {
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(float),
                          is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
}

void ensure_ws(mm_gnn *g, int n) {
    if (n <= g->cap) return;
    gsync(g);
    nrelease(g, g->ws);
    const size_t N = (size_t)std::max(n, 1);
    g->X = nalloc<float>(g, g->ws, N * kF);
    g->Xn = nalloc<float>(g, g->ws, N * kF);
    g->y0 = nalloc<float>(g, g->ws, N * kW);
    for (int l = 0; l < kLayers; ++l) {
        g->z[l] = nalloc<float>(g, g->ws, N * 2 * kW);
        g->a[l] = nalloc<float>(g, g->ws, N * kW);
        g->y1[l] = nalloc<float>(g, g->ws, N * kW);
        g->tt[l] = nalloc<float>(g, g->ws, N * kW);
    }
    g->h3 = nalloc<float>(g, g->ws, N * kW);
    g->zm = nalloc<float>(g, g->ws, N * 3);
    g->zs = nalloc<float>(g, g->ws, N);
    g->dh = nalloc<float>(g, g->ws, N * kW);
    g->dt = nalloc<float>(g, g->ws, N * kW);
    g->dy = nalloc<float>(g, g->ws, N * kW);
    g->dz = nalloc<float>(g, g->ws, N * 2 * kW);
    g->da = nalloc<float>(g, g->ws, N * kW);
    g->d_zm = nalloc<float>(g, g->ws, N * 3);
    g->d_zs = nalloc<float>(g, g->ws, N);
    g->part = nalloc<float>(g, g->ws, (size_t)gnn_tn_blocks(n) * 2 * kW * kW);
    g->m = nalloc<double>(g, g->ws, N * 3);
    g->dmt = nalloc<double>(g, g->ws, N * 3);
    g->st = nalloc<double>(g, g->ws, N);
    g->dm = nalloc<double>(g, g->ws, N * 3);
    g->s = nalloc<double>(g, g->ws, N);
    g->lpart = nalloc<double>(g, g->ws, (size_t)gnn_loss_blocks(n) + 1);
    g->loss = nalloc<double>(g, g->ws, 1);
    g->cap = n;
}

// forward pass on raw features X (device, n x 32) and m (device, n x 3);
// dm, s (device doubles, may be null) receive the heads' outputs. The
// features are standardized in FP32 first (g->Xn), before the first product
// rounds them to BF16.
void forward(mm_gnn *g, mm_graph *gr, const float *X, const double *m, double *dm, double *sv) {
    const int n = gr->n;
    hipStream_t s = g->stream;
    const float *th = g->theta;
    gnn_norm_features(n, X, g->mu, g->sd, g->Xn, s);
    gnn_mm(n, kF, kW, 1, g->Xn, kF, th + oWin, kW, false, th + oBin, g->z[0], 2 * kW, g->y0, kW, nullptr, 0, g->f32, s);
    for (int l = 0; l < kLayers; ++l) {
        float *z = g->z[l];
        gnn_agg(n, gr->ptr, gr->idx, gr->invdeg, z, 2 * kW, g->a[l], kW, s);
        gnn_mm(n, kW, kW, 0, g->a[l], kW, th + oWe1(l), kW, false, nullptr, z + kW, 2 * kW, nullptr, 0, nullptr, 0, g->f32, s);
        gnn_edge_add(n, gr->ebar, th + oWe2(l), z + kW, 2 * kW, s);
        gnn_mm(n, 2 * kW, kW, 1, z, 2 * kW, th + oW1(l), kW, false, th + ob1(l), g->tt[l], kW, g->y1[l], kW, nullptr,
               0, g->f32, s);
        float *hn = (l + 1 < kLayers) ? g->z[l + 1] : g->h3;
        const int ldh = (l + 1 < kLayers) ? 2 * kW : kW;
        gnn_mm(n, kW, kW, 2, g->tt[l], kW, th + oW2(l), kW, false, th + ob2(l), hn, ldh, nullptr, 0, z, 2 * kW, g->f32, s);
    }
    gnn_heads(n, g->h3, th + oWm, th + obm, th + oWs, th + obs, m, g->zm, g->zs, dm, sv, s);
}

// backward pass after forward(); d_zm, d_zs hold the loss gradient at the heads
void backward(mm_gnn *g, mm_graph *gr) {
    const int n = gr->n;
    hipStream_t s = g->stream;
    const float *th = g->theta;
    float *gr_ = g->grad;
    float *part = g->part;
    gnn_tn32(n, kW, 3, g->h3, kW, g->d_zm, 3, part, gr_ + oWm, s);
    gnn_tn32(n, 1, 3, nullptr, 0, g->d_zm, 3, part, gr_ + obm, s);
    gnn_tn32(n, kW, 1, g->h3, kW, g->d_zs, 1, part, gr_ + oWs, s);
    gnn_tn32(n, 1, 1, nullptr, 0, g->d_zs, 1, part, gr_ + obs, s);
    gnn_heads_dh(n, g->d_zm, g->d_zs, th + oWm, th + oWs, g->dh, s);
    for (int l = kLayers - 1; l >= 0; --l) {
        float *z = g->z[l];
        gnn_mm_tn(n, kW, kW, g->tt[l], kW, g->dh, kW, part, gr_ + oW2(l), false, g->f32, s);
        gnn_tn32(n, 1, kW, nullptr, 0, g->dh, kW, part, gr_ + ob2(l), s);
        gnn_mm(n, kW, kW, 0, g->dh, kW, th + oW2(l), kW, true, nullptr, g->dt, kW, nullptr, 0, nullptr, 0, g->f32, s);
        gnn_silu_bwd((int64_t)n * kW, g->dt, g->y1[l], g->dy, s);
        gnn_mm_tn(n, 2 * kW, kW, z, 2 * kW, g->dy, kW, part, gr_ + oW1(l), false, g->f32, s);
        gnn_tn32(n, 1, kW, nullptr, 0, g->dy, kW, part, gr_ + ob1(l), s);
        gnn_mm(n, kW, 2 * kW, 0, g->dy, kW, th + oW1(l), kW, true, nullptr, g->dz, 2 * kW, nullptr, 0, nullptr, 0, g->f32, s);
        gnn_add64(n, g->dz, 2 * kW, g->dh, kW, s);
        gnn_mm_tn(n, kW, kW, g->a[l], kW, g->dz + kW, 2 * kW, part, gr_ + oWe1(l), false, g->f32, s);
        gnn_tn32(n, 4, kW, gr->ebar, 4, g->dz + kW, 2 * kW, part, gr_ + oWe2(l), s);
        gnn_mm(n, kW, kW, 0, g->dz + kW, 2 * kW, th + oWe1(l), kW, true, nullptr, g->da, kW, nullptr, 0, nullptr, 0, g->f32, s);
        gnn_agg_t_add(n, gr->ptr, gr->idx, gr->invdeg, g->da, kW, g->dh, kW, s);
    }
    gnn_silu_bwd((int64_t)n * kW, g->dh, g->y0, g->dy, s);
    gnn_mm_tn(n, kF, kW, g->Xn, kF, g->dy, kW, part, gr_ + oWin, false, g->f32, s);
    gnn_tn32(n, 1, kW, nullptr, 0, g->dy, kW, part, gr_ + oBin, s);
}

// features of the current state of instance 0 (st[0] filled by an
// evaluation at h_next) into gr->X
void features_from_state(mm_ctx *c, mm_graph *gr, const double hp[3], const double hn[3]) {
    launch_spmv_block6(c->C, c->Mm.map, c->st[0].x, c->tmp3, false, c->stream);
    gnn_features(gr->n, c->st[0].x, c->st[0].G, c->st[0].g, c->tmp3, c->L, gr->stat, hn, hp, gr->X, c->stream);
}

// a graph of any context on the network's device; that context's queued
// work is finished first (its buffers are read on the network's stream)
void check_pair(mm_gnn *g, mm_graph *gr) {
    if (!g || !gr) throw ApiError{MM_EINVAL, "null network or graph"};
    if (gr->c->device != g->device) throw ApiError{MM_EINVAL, "network and graph are on different devices"};
    if (gr->c->stream != g->stream) sync(gr->c);
}

// one forward + backward pass on a sample (gradient left in g->grad); the loss
double loss_grad_step(mm_gnn *g, mm_graph *gr, const float *X, const double *m, const double *dm_target,
                      const double *s_target, double inv_dm2, double w_s) {
    check_pair(g, gr);
    if (!m || !dm_target || !s_target) throw ApiError{MM_EINVAL, "m and both targets are required"};
    if (!(inv_dm2 >= 0) || !(w_s >= 0)) throw ApiError{MM_EINVAL, "loss weights must be >= 0"};
    const int n = gr->n;
    ensure_ws(g, n);
    hipStream_t st = g->stream;
    const float *Xd = gr->X;
    if (X) {
        copy_f32_in(st, g->X, X, (size_t)kF * n);
        Xd = g->X;
    }
    copy_d_in(st, g->m, m, 3 * (size_t)n);
    copy_d_in(st, g->dmt, dm_target, 3 * (size_t)n);
    copy_d_in(st, g->st, s_target, n);
    forward(g, gr, Xd, g->m, nullptr, nullptr);
    gnn_loss_heads(n, g->zm, g->zs, g->m, g->dmt, g->st, gr->c->L, 1.0 / gr->sumL, inv_dm2, w_s, g->d_zm, g->d_zs,
                   g->lpart, g->loss, st);
    backward(g, gr);
    double lv = 0.0;
    HIPCHK(hipMemcpyAsync(&lv, g->loss, sizeof(double), hipMemcpyDeviceToHost, st));
    gsync(g);
    return lv;
}

// one bias-corrected Adam step with the last gradient (enqueued)
void adam_step(mm_gnn *g, double lr, double beta1, double beta2, double eps) {
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        throw ApiError{MM_EINVAL, "bad Adam constants"};
    g->t += 1;
    const double bc1 = 1.0 - std::pow(beta1, (double)g->t), bc2 = 1.0 - std::pow(beta2, (double)g->t);
    gnn_adam(kNParams, g->theta, g->grad, g->m1, g->m2, (float)lr, (float)beta1, (float)beta2, (float)eps,
             (float)bc1, (float)bc2, g->stream);
}

// SplitMix64 (Steele, Lea and Flood): the shuffles of mm_gnn_train
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// first word of a parameter file of mm_gnn_save ("MMGNN" + format 1)
constexpr int64_t kGnnFileMagic = 0x31004E4E474D4DLL;

}  // namespace

void gnn_propose(mm_ctx *c, mm_gnn *g, mm_graph *gr, const double h_prev[3], const double h_next[3]) {
    if (!g || !gr || gr->c != c) throw ApiError{MM_EINVAL, "network and graph of this context are required"};
    ensure_ws(g, gr->n);
    features_from_state(c, gr, h_prev, h_next);
    check_pair(g, gr);
    forward(g, gr, gr->X, c->st[0].x, c->d, c->dscale);
    if (g->stream != c->stream) gsync(g);
}

}  // namespace mmncg

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

long mm_gnn_param_count(void) { return mmncg::kNParams; }

int mm_gnn_create(mm_ctx *c, mm_gnn **out) {
    if (!out) return MM_EINVAL;
    *out = nullptr;
    return guarded(c, [&] {
        mm_gnn *g = new mm_gnn();
        g->device = c->device;
        g->stream = c->stream;
        g->ualloc = c->ualloc;
        g->ufree = c->ufree;
        g->user = c->user;
        try {
            g->theta = nalloc<float>(g, g->mem, kNParams);
            g->grad = nalloc<float>(g, g->mem, kNParams);
            g->m1 = nalloc<float>(g, g->mem, kNParams);
            g->m2 = nalloc<float>(g, g->mem, kNParams);
            g->mu = nalloc<float>(g, g->mem, kF);
            g->sd = nalloc<float>(g, g->mem, kF);
            for (float *p : {g->theta, g->grad, g->m1, g->m2})
                HIPCHK(hipMemsetAsync(p, 0, kNParams * sizeof(float), g->stream));
            std::vector<float> z(kF, 0.0f), o(kF, 1.0f);
            HIPCHK(hipMemcpyAsync(g->mu, z.data(), kF * sizeof(float), hipMemcpyHostToDevice, g->stream));
            HIPCHK(hipMemcpyAsync(g->sd, o.data(), kF * sizeof(float), hipMemcpyHostToDevice, g->stream));
            gsync(g);
        } catch (...) {
            nrelease(g, g->mem);
            delete g;
            throw;
        }
        *out = g;
        return MM_OK;
    });
}

int mm_gnn_destroy(mm_gnn *g) {
    if (!g) return MM_EINVAL;
    (void)hipSetDevice(g->device);
    (void)hipStreamSynchronize(g->stream);
    nrelease(g, g->ws);
    nrelease(g, g->mem);
    delete g;
    return MM_OK;
}

const char *mm_gnn_last_error(const mm_gnn *g) { return g ? g->err.c_str() : "null network"; }

int mm_gnn_set_precision(mm_gnn *g, int precision) {
    if (!g) return MM_EINVAL;
    if (precision != MM_GNN_BF16 && precision != MM_GNN_FP32) {
        g->err = "precision must be MM_GNN_BF16 or MM_GNN_FP32";
        return MM_EINVAL;
    }
    g->f32 = precision == MM_GNN_FP32;
    g->err.clear();
    return MM_OK;
}

int mm_gnn_set_params(mm_gnn *g, const double *theta) {
    return gguard(g, [&] {
        if (!theta) throw ApiError{MM_EINVAL, "null parameters"};
        std::vector<float> h(kNParams);
        std::vector<double> src(kNParams);
        if (is_device_ptr(theta)) HIPCHK(hipMemcpy(src.data(), theta, kNParams * sizeof(double), hipMemcpyDeviceToHost));
        else std::memcpy(src.data(), theta, kNParams * sizeof(double));
        for (int i = 0; i < kNParams; ++i) {
            if (!std::isfinite(src[i])) throw ApiError{MM_EINVAL, "non-finite parameter"};
            h[i] = (float)src[i];
        }
        HIPCHK(hipMemcpyAsync(g->theta, h.data(), kNParams * sizeof(float), hipMemcpyHostToDevice, g->stream));
        for (float *p : {g->m1, g->m2}) HIPCHK(hipMemsetAsync(p, 0, kNParams * sizeof(float), g->stream));
        g->t = 0;
        gsync(g);
        return MM_OK;
    });
}

int mm_gnn_set_input_norm(mm_gnn *g, const double *mu, const double *sd) {
    return gguard(g, [&] {
        if (!mu || !sd) throw ApiError{MM_EINVAL, "null mean or spread"};
        std::vector<float> a(kF), b(kF);
        for (int c = 0; c < kF; ++c) {
            if (!std::isfinite(mu[c]) || !(sd[c] > 0) || !std::isfinite(sd[c]))
                throw ApiError{MM_EINVAL, "spreads must be finite and positive"};
            a[c] = (float)mu[c];
            b[c] = (float)sd[c];
        }
        HIPCHK(hipMemcpyAsync(g->mu, a.data(), kF * sizeof(float), hipMemcpyHostToDevice, g->stream));
        HIPCHK(hipMemcpyAsync(g->sd, b.data(), kF * sizeof(float), hipMemcpyHostToDevice, g->stream));
        gsync(g);
        return MM_OK;
    });
}

int mm_gnn_get_params(mm_gnn *g, double *theta) {
    return gguard(g, [&] {
        if (!theta) throw ApiError{MM_EINVAL, "null parameters"};
        std::vector<float> h(kNParams);
        HIPCHK(hipMemcpyAsync(h.data(), g->theta, kNParams * sizeof(float), hipMemcpyDeviceToHost, g->stream));
        gsync(g);
        std::vector<double> d(h.begin(), h.end());
        if (is_device_ptr(theta)) HIPCHK(hipMemcpy(theta, d.data(), kNParams * sizeof(double), hipMemcpyHostToDevice));
        else std::memcpy(theta, d.data(), kNParams * sizeof(double));
        return MM_OK;
    });
}

int mm_graph_create(mm_ctx *c, mm_graph **out) {
    if (!out) return MM_EINVAL;
    *out = nullptr;
    return guarded(c, [&] {
        require_single(c);
        if (c->tets.empty()) throw ApiError{MM_ESTATE, "the graph needs a mesh set with mm_mesh_upload"};
        const InstInfo &I = c->inst[0];
        const int n = I.n_mag;
        std::vector<int> local(c->xyz.size() / 3, -1);
        for (int a = 0; a < n; ++a) local[I.node_of_mag[a]] = a;
        std::vector<std::set<int>> nb(n);
        const long nt = (long)c->region.size();
        for (long t = 0; t < nt; ++t) {
            if (c->region[t] <= 0) continue;
            int v[4];
            for (int k = 0; k < 4; ++k) v[k] = local[c->tets[4 * t + k]];
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q)
                    if (p != q) nb[v[p]].insert(v[q]);
        }
        std::vector<int> ptr(n + 1, 0), idx;
        for (int a = 0; a < n; ++a) {
            for (int b : nb[a]) idx.push_back(b);
            ptr[a + 1] = (int)idx.size();
        }
        auto X = [&](int a, int k) { return c->xyz[3 * (size_t)I.node_of_mag[a] + k]; };
        double lsum = 0.0;
        for (int a = 0; a < n; ++a)
            for (int e = ptr[a]; e < ptr[a + 1]; ++e) {
                const int b = idx[e];
                double d2 = 0.0;
                for (int k = 0; k < 3; ++k) d2 += (X(b, k) - X(a, k)) * (X(b, k) - X(a, k));
                lsum += std::sqrt(d2);
            }
        const double ell = idx.empty() ? 1.0 : lsum / (double)idx.size();
        std::vector<float> ebar(4 * (size_t)n, 0.0f), invdeg(n, 0.0f), stat(3 * (size_t)n);
        int maxdeg = 1;
        for (int a = 0; a < n; ++a) maxdeg = std::max(maxdeg, ptr[a + 1] - ptr[a]);
        // lumped volumes and exchange diagonal of the context
        std::vector<double> L(n), iD(n);
        HIPCHK(hipMemcpyAsync(L.data(), c->L, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(iD.data(), c->invDex, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        sync(c);
        double Lm = 0.0, Dm = 0.0;
        for (int a = 0; a < n; ++a) {
            Lm += L[a];
            Dm += 1.0 / iD[a];
        }
        const double sumL = Lm;
        Lm /= n;
        Dm /= n;
        for (int a = 0; a < n; ++a) {
            const int dg = ptr[a + 1] - ptr[a];
            double acc[4] = {0, 0, 0, 0};
            for (int e = ptr[a]; e < ptr[a + 1]; ++e) {
                const int b = idx[e];
                double d[3], d2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    d[k] = (X(b, k) - X(a, k)) / ell;
                    d2 += d[k] * d[k];
                }
                for (int k = 0; k < 3; ++k) acc[k] += d[k];
                acc[3] += std::sqrt(d2);
            }
            for (int k = 0; k < 4; ++k) ebar[4 * (size_t)a + k] = dg ? (float)(acc[k] / dg) : 0.0f;
            invdeg[a] = dg ? 1.0f / (float)dg : 0.0f;
            stat[3 * (size_t)a] = (float)((1.0 / iD[a]) / Dm);
            stat[3 * (size_t)a + 1] = (float)(L[a] / Lm);
            stat[3 * (size_t)a + 2] = (float)dg / (float)maxdeg;
        }
        mm_graph *gr = new mm_graph();
        gr->c = c;
        gr->n = n;
        gr->nnz = (long)idx.size();
        gr->sumL = sumL;
        try {
            gr->ptr = galloc<int>(c, gr->mem, n + 1);
            gr->idx = galloc<int>(c, gr->mem, std::max<size_t>(idx.size(), 1));
            gr->invdeg = galloc<float>(c, gr->mem, n);
            gr->ebar = galloc<float>(c, gr->mem, 4 * (size_t)n);
            gr->stat = galloc<float>(c, gr->mem, 3 * (size_t)n);
            gr->X = galloc<float>(c, gr->mem, (size_t)kF * n);
            HIPCHK(hipMemcpyAsync(gr->ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
            if (!idx.empty())
                HIPCHK(hipMemcpyAsync(gr->idx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(gr->invdeg, invdeg.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(gr->ebar, ebar.data(), ebar.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(gr->stat, stat.data(), stat.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemsetAsync(gr->X, 0, (size_t)kF * n * sizeof(float), c->stream));
            sync(c);
        } catch (...) {
            release(c, gr->mem);
            delete gr;
            throw;
        }
        *out = gr;
        return MM_OK;
    });
}

int mm_graph_destroy(mm_graph *gr) {
    if (!gr) return MM_EINVAL;
    mm_ctx *c = gr->c;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    release(c, gr->mem);
    delete gr;
    return MM_OK;
}

int mm_graph_size(const mm_graph *gr, long *n_nodes, long *n_edges) {
    if (!gr) return MM_EINVAL;
    if (n_nodes) *n_nodes = gr->n;
    if (n_edges) *n_edges = gr->nnz;
    return MM_OK;
}

int mm_gnn_features(mm_graph *gr, const double *m, const double h_prev[3], const double h_next[3], float *X) {
    if (!gr) return MM_EINVAL;
    mm_ctx *c = gr->c;
    return guarded(c, [&] {
        require_single(c);
        if (!m || !h_prev || !h_next) throw ApiError{MM_EINVAL, "m and both fields are required"};
        load_m(c, m);
        double hp[3], hn[3];
        reduce_field(c->inst[0], h_prev, hp);
        reduce_field(c->inst[0], h_next, hn);
        eval_all(c, c->opts, std::vector<double>(hn, hn + 3));
        features_from_state(c, gr, hp, hn);
        if (X) copy_f32_out(c, X, gr->X, (size_t)kF * gr->n);
        sync(c);
        return MM_OK;
    });
}

int mm_gnn_forward(mm_gnn *g, mm_graph *gr, const float *X, const double *m, double *dm, double *s) {
    return gguard(g, [&] {
        check_pair(g, gr);
        if (!m) throw ApiError{MM_EINVAL, "m is required"};
        const int n = gr->n;
        ensure_ws(g, n);
        const float *Xd = gr->X;
        if (X) {
            copy_f32_in(g->stream, g->X, X, (size_t)kF * n);
            Xd = g->X;
        }
        copy_d_in(g->stream, g->m, m, 3 * (size_t)n);
        forward(g, gr, Xd, g->m, g->dm, g->s);
        if (dm) copy_d_out(g->stream, dm, g->dm, 3 * (size_t)n);
        if (s) copy_d_out(g->stream, s, g->s, n);
        gsync(g);
        return MM_OK;
    });
}

int mm_gnn_loss_grad(mm_gnn *g, mm_graph *gr, const float *X, const double *m, const double *dm_target,
                     const double *s_target, double inv_dm2, double w_s, double *loss, double *grad) {
    return gguard(g, [&] {
        const double lv = loss_grad_step(g, gr, X, m, dm_target, s_target, inv_dm2, w_s);
        hipStream_t st = g->stream;
        if (grad) {
            std::vector<float> h(kNParams);
            HIPCHK(hipMemcpyAsync(h.data(), g->grad, kNParams * sizeof(float), hipMemcpyDeviceToHost, st));
            gsync(g);
            std::vector<double> d(h.begin(), h.end());
            if (is_device_ptr(grad)) HIPCHK(hipMemcpy(grad, d.data(), kNParams * sizeof(double), hipMemcpyHostToDevice));
            else std::memcpy(grad, d.data(), kNParams * sizeof(double));
        }
        gsync(g);
        if (loss) *loss = lv;
        return MM_OK;
    });
}

int mm_gnn_adam(mm_gnn *g, double lr, double beta1, double beta2, double eps) {
    return gguard(g, [&] {
        adam_step(g, lr, beta1, beta2, eps);
        gsync(g);
        return MM_OK;
    });
}

int mm_gnn_train(mm_gnn *g, long n_samples, mm_graph *const *graphs, const float *const *X, const double *const *m,
                 const double *const *dm_target, const double *const *s_target, const double *inv_dm2, double w_s,
                 int epochs, double lr, unsigned long long seed, double *epoch_loss) {
    return gguard(g, [&] {
        if (n_samples < 1 || !graphs || !X || !m || !dm_target || !s_target || !inv_dm2 || epochs < 0)
            throw ApiError{MM_EINVAL, "bad training arguments"};
        std::vector<long> order(n_samples);
        for (long k = 0; k < n_samples; ++k) order[k] = k;
        SplitMix64 rng{seed};
        for (int ep = 0; ep < epochs; ++ep) {
            // Fisher-Yates with the counter-based generator: the same seed gives the same order
            for (long k = n_samples - 1; k > 0; --k) std::swap(order[k], order[(long)(rng.next() % (uint64_t)(k + 1))]);
            double tot = 0.0;
            for (long k : order) {
                tot += loss_grad_step(g, graphs[k], X[k], m[k], dm_target[k], s_target[k], inv_dm2[k], w_s);
                adam_step(g, lr, 0.9, 0.999, 1e-8);
            }
            gsync(g);
            if (epoch_loss) epoch_loss[ep] = tot / (double)n_samples;
        }
        return MM_OK;
    });
}

int mm_gnn_save(mm_gnn *g, const char *path) {
    return gguard(g, [&] {
        if (!path) throw ApiError{MM_EINVAL, "null path"};
        std::vector<float> th(kNParams), mu(kF), sd(kF);
        HIPCHK(hipMemcpyAsync(th.data(), g->theta, kNParams * sizeof(float), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipMemcpyAsync(mu.data(), g->mu, kF * sizeof(float), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipMemcpyAsync(sd.data(), g->sd, kF * sizeof(float), hipMemcpyDeviceToHost, g->stream));
        gsync(g);
        const std::string tmp = std::string(path) + ".tmp";
        FILE *f = std::fopen(tmp.c_str(), "wb");
        if (!f) throw ApiError{MM_EINVAL, std::string("cannot write ") + path};
        const int64_t hdr[3] = {kGnnFileMagic, (int64_t)kNParams, (int64_t)kF};
        bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 && std::fwrite(th.data(), sizeof(float), th.size(), f) == th.size() &&
                  std::fwrite(mu.data(), sizeof(float), kF, f) == (size_t)kF &&
                  std::fwrite(sd.data(), sizeof(float), kF, f) == (size_t)kF;
        ok = (std::fclose(f) == 0) && ok;
        if (!ok || std::rename(tmp.c_str(), path) != 0) throw ApiError{MM_EINVAL, std::string("cannot write ") + path};
        return MM_OK;
    });
}

int mm_gnn_load(mm_gnn *g, const char *path) {
    return gguard(g, [&] {
        if (!path) throw ApiError{MM_EINVAL, "null path"};
        FILE *f = std::fopen(path, "rb");
        if (!f) throw ApiError{MM_EINVAL, std::string("cannot read ") + path};
        int64_t hdr[3] = {0, 0, 0};
        std::vector<float> th(kNParams), mu(kF), sd(kF);
        bool ok = std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == kGnnFileMagic && hdr[1] == kNParams && hdr[2] == kF &&
                  std::fread(th.data(), sizeof(float), th.size(), f) == th.size() &&
                  std::fread(mu.data(), sizeof(float), kF, f) == (size_t)kF &&
                  std::fread(sd.data(), sizeof(float), kF, f) == (size_t)kF;
        std::fclose(f);
        if (!ok) throw ApiError{MM_EINVAL, std::string("not a parameter file of this network: ") + path};
        for (float v : th)
            if (!std::isfinite(v)) throw ApiError{MM_EINVAL, "non-finite parameter"};
        for (int c = 0; c < kF; ++c)
            if (!std::isfinite(mu[c]) || !(sd[c] > 0) || !std::isfinite(sd[c])) throw ApiError{MM_EINVAL, "bad standardization"};
        HIPCHK(hipMemcpyAsync(g->theta, th.data(), kNParams * sizeof(float), hipMemcpyHostToDevice, g->stream));
        HIPCHK(hipMemcpyAsync(g->mu, mu.data(), kF * sizeof(float), hipMemcpyHostToDevice, g->stream));
        HIPCHK(hipMemcpyAsync(g->sd, sd.data(), kF * sizeof(float), hipMemcpyHostToDevice, g->stream));
        // a loaded network starts a fresh optimizer state
        HIPCHK(hipMemsetAsync(g->m1, 0, kNParams * sizeof(float), g->stream));
        HIPCHK(hipMemsetAsync(g->m2, 0, kNParams * sizeof(float), g->stream));
        g->t = 0;
        gsync(g);
        return MM_OK;
    });
}

int mm_gnn_targets(mm_graph *gr, const double *m, const double *m_next, const double *diag3, double *dm_target,
                   double *s_target) {
    if (!gr) return MM_EINVAL;
    mm_ctx *c = gr->c;
    return guarded(c, [&] {
        require_single(c);
        if (!m || !m_next || !diag3 || !dm_target || !s_target) throw ApiError{MM_EINVAL, "null vector"};
        const int n = gr->n;
        std::vector<void *> tmp;
        double *dm_ = galloc<double>(c, tmp, 3 * (size_t)n), *dm1 = galloc<double>(c, tmp, 3 * (size_t)n),
               *dd = galloc<double>(c, tmp, 3 * (size_t)n), *dt = galloc<double>(c, tmp, 3 * (size_t)n),
               *ds = galloc<double>(c, tmp, (size_t)n);
        try {
            copy_in(c, dm_, m, 3 * (size_t)n);
            copy_in(c, dm1, m_next, 3 * (size_t)n);
            copy_in(c, dd, diag3, 3 * (size_t)n);
            gnn_targets(n, dm_, dm1, dd, c->invDex, dt, ds, c->stream);
            copy_out(c, dm_target, dt, 3 * (size_t)n);
            copy_out(c, s_target, ds, (size_t)n);
            sync(c);
        } catch (...) {
            release(c, tmp);
            throw;
        }
        release(c, tmp);
        return MM_OK;
    });
}

int mm_gnn_moments(mm_graph *gr, const float *X, double *sum, double *sumsq) {
    if (!gr) return MM_EINVAL;
    mm_ctx *c = gr->c;
    return guarded(c, [&] {
        if (!X || !sum || !sumsq) throw ApiError{MM_EINVAL, "null argument"};
        const int n = gr->n;
        std::vector<void *> tmp;
        float *dX = galloc<float>(c, tmp, (size_t)kF * std::max(n, 1));
        double *part = galloc<double>(c, tmp, 64 * (size_t)gnn_moment_blocks(n)), *out = galloc<double>(c, tmp, 64);
        std::vector<double> h(64);
        try {
            copy_f32_in(c->stream, dX, X, (size_t)kF * n);
            gnn_moments(n, dX, part, out, c->stream);
            HIPCHK(hipMemcpyAsync(h.data(), out, 64 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            sync(c);
        } catch (...) {
            release(c, tmp);
            throw;
        }
        release(c, tmp);
        std::memcpy(sum, h.data(), 32 * sizeof(double));
        std::memcpy(sumsq, h.data() + 32, 32 * sizeof(double));
        return MM_OK;
    });
}

int mm_jacobi_diag(mm_ctx *c, double *D) {
    return guarded(c, [&] {
        require_single(c);
        if (!D) throw ApiError{MM_EINVAL, "null output"};
        const int nm = c->inst[0].n_mag;
        std::vector<double> iD(nm);
        HIPCHK(hipMemcpyAsync(iD.data(), c->invDex, nm * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        sync(c);
        for (double &v : iD) v = 1.0 / v;
        if (is_device_ptr(D)) HIPCHK(hipMemcpy(D, iD.data(), nm * sizeof(double), hipMemcpyHostToDevice));
        else std::memcpy(D, iD.data(), nm * sizeof(double));
        return MM_OK;
    });
}

int mm_demag_diag(mm_ctx *c, const double *probes, int n_probe, double rtol, double *diag) {
    return guarded(c, [&] {
        require_single(c);
        if (!probes || n_probe < 1 || !diag || !(rtol > 0)) throw ApiError{MM_EINVAL, "bad probe arguments"};
        const InstInfo &I = c->inst[0];
        const int nm = I.n_mag, np = I.n_pot;
        std::vector<double> acc(3 * (size_t)nm, 0.0), z(3 * (size_t)nm), v(3 * (size_t)nm);
        // keep the warm start aside; every probe solves from u = 0
        HIPCHK(hipMemcpyAsync(c->usave, c->u, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        for (int p = 0; p < n_probe; ++p) {
            const double *zp = probes + 3 * (size_t)nm * p;
            copy_in(c, c->tmp3, zp, 3 * (size_t)nm);
            HIPCHK(hipMemcpyAsync(z.data(), c->tmp3, z.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            launch_fill(np, c->b, 0.0, c->stream);
            launch_fill(np, c->u, 0.0, c->stream);
            StateV sv[3];
            sv[0].x = c->tmp3;
            if (c->B.nrows > 0) launch_bmul(c->B, c->Mb.map, nullptr, sv, nullptr, c->b, false, c->stream);
            c->act()[0] = 1;
            upload_ctl(c);
            poisson(c, rtol, c->opts.poisson_maxit, false, c->opts.poisson_prec == MM_PREC_AMG, {0});
            launch_btmul(c->Bt, c->Mm.map, c->u, c->pq, false, c->stream);
            HIPCHK(hipMemcpyAsync(v.data(), c->pq, v.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            sync(c);
            for (size_t e = 0; e < acc.size(); ++e) acc[e] += z[e] * v[e];
        }
        launch_fill(np, c->b, 0.0, c->stream);
        HIPCHK(hipMemcpyAsync(c->u, c->usave, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        sync(c);
        for (double &a : acc) a /= n_probe;
        if (is_device_ptr(diag)) HIPCHK(hipMemcpy(diag, acc.data(), acc.size() * sizeof(double), hipMemcpyHostToDevice));
        else std::memcpy(diag, acc.data(), acc.size() * sizeof(double));
        return MM_OK;
    });
}

}  // extern "C"
