// Context, device operators and the host control of the PNCG minimizer
// (Alg. 4 with beta*ZA, the local-field preconditioner solved by Alg. 1, and
// field stepping), behind the C ABI of include/mmncg.h.
//
// The host only makes scalar decisions (line-search steps, stopping); every
// vector operation runs in the HIP kernels of kernels.hip on the context's
// stream. Scalars come back through a small pinned buffer, once per
// evaluation, once per direction update and once per chunk of Poisson CG
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mmncg.h"
#include "internal.h"

using namespace mmncg;

namespace {

constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;

struct HipError {
    hipError_t e;
    const char *what;
};
#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t _e = (x);                        \
        if (_e != hipSuccess) throw HipError{_e, #x}; \
    } while (0)

struct ApiError {
    int code;
    std::string msg;
};

// partial-buffer arena layout (units of kMaxPartials doubles)
enum PartSlot {
    PS_EVAL = 0,                    // 10
    PS_CG_INIT = PS_EVAL + 10,      // 3
    PS_CG_PQ = PS_CG_INIT + 3,      // 1
    PS_CG_RZ0 = PS_CG_PQ + 1,       // 2
    PS_CG_RZ1 = PS_CG_RZ0 + 2,      // 2
    PS_PR_INIT = PS_CG_RZ1 + 2,     // 2
    PS_PR_PQ = PS_PR_INIT + 2,      // 1
    PS_PR_RZ0 = PS_PR_PQ + 1,       // 2
    PS_PR_RZ1 = PS_PR_RZ0 + 2,      // 2
    PS_DIR_DOTS = PS_PR_RZ1 + 2,    // 6
    PS_DIR_OUT = PS_DIR_DOTS + 6,   // 2
    PS_MISC = PS_DIR_OUT + 2,       // 5
    PS_TOTAL = PS_MISC + 5
};
// device scalar slots
enum ScSlot { SC_EVAL = 0, SC_CG = 16, SC_DIR = 24, SC_MISC = 32, SC_TOTAL = 48 };
// device int flags
enum FlagSlot { FL_CG_DONE = 0, FL_CG_ITERS = 1, FL_PREC = 4, FL_DIR = 8, FL_TOTAL = 16 };

struct State {
    double *x = nullptr, *G = nullptr, *g = nullptr, *lam = nullptr;
    double E = 0;       // total energy
    double Eloc = 0, Ez = 0, Ed = 0;
    double tmax = 0, ginf = 0, minf = 0;
};

}  // namespace

struct mm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mm_alloc_fn ualloc = nullptr;
    mm_free_fn ufree = nullptr;
    void *user = nullptr;
    std::string err;
    std::vector<void *> allocs;

    // mesh (host copy until materials arrive)
    std::vector<double> xyz;
    std::vector<int> tets, region;
    bool have_mesh = false, have_mat = false;

    Assembly as;
    Sell C, S, K, B, Bt;
    double *L = nullptr, *invDex = nullptr, *invDK = nullptr;
    float *invDK32 = nullptr;
    bool fp32_ready = false;

    // vectors on magnet nodes
    State st[3];
    double *d = nullptr, *y = nullptr, *pr = nullptr, *pp = nullptr, *pq = nullptr, *dscale = nullptr,
           *tmp3 = nullptr;
    // vectors on potential nodes
    double *u = nullptr, *b = nullptr, *cr = nullptr, *cp = nullptr, *cp2 = nullptr, *cq = nullptr, *usave = nullptr;
    float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *p32b = nullptr, *q32 = nullptr;
    PcgState *pst = nullptr;     // device
    PcgState *hpst = nullptr;    // pinned host mirror
    double *ppart = nullptr;     // partials of the Poisson kernels
    hipGraphExec_t graph64 = nullptr, graph32 = nullptr;
    double *part = nullptr;
    double *dsc = nullptr, *hsc = nullptr;
    int *dflags = nullptr, *hflags = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

    mm_opts opts;
    long last_poisson_iters = 16;
    // kernel timing (mm_profile)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
    double prof_launches = 0, prof_seconds = 0, prof_units = 0;
    // counters of the current minimization
    long c_evals = 0, c_mi = 0, c_li = 0;
    double t_mag = 0, t_lin = 0;

    int n_mag() const { return as.n_mag; }
    int n_pot() const { return as.n_pot; }
};

namespace {

double *partp(mm_ctx *c, int slot) { return c->part + (size_t)slot * kMaxPartials; }

void set_err(mm_ctx *c, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
}

void *dalloc(mm_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->ualloc) {
        p = c->ualloc(bytes, c->user);
        if (!p) throw ApiError{MM_ENOMEM, "device allocation callback failed"};
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw ApiError{MM_ENOMEM, "hipMalloc failed (" + std::to_string(bytes) + " bytes)"};
        }
    }
    c->allocs.push_back(p);
    return p;
}
template <class T>
T *dalloc_n(mm_ctx *c, size_t n) {
    return (T *)dalloc(c, n * sizeof(T));
}

void free_all(mm_ctx *c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipGraphExec_t *g : {&c->graph64, &c->graph32}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
    for (void *p : c->allocs) {
        if (c->ufree) c->ufree(p, c->user);
        else (void)hipFree(p);
    }
    c->allocs.clear();
}

size_t device_bytes_estimate(const mm_ctx *c);

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

void copy_in(mm_ctx *c, double *dst, const double *src, size_t n) {
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
}
void copy_out(mm_ctx *c, double *dst, const double *src, size_t n) {
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
}
void sync(mm_ctx *c) { HIPCHK(hipStreamSynchronize(c->stream)); }

// pull n scalars from the device scalar area (slot) and wait
void pull(mm_ctx *c, int slot, int n) {
    HIPCHK(hipMemcpyAsync(c->hsc + slot, c->dsc + slot, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// event pairs around the timed kernel; harvested at the next synchronization
void prof_mark(mm_ctx *c) {
    if (!c->prof_on) return;
    if (c->prof_used == c->prof_ev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->prof_ev.push_back(e);
    }
    HIPCHK(hipEventRecord(c->prof_ev[c->prof_used++], c->stream));
}
void prof_harvest(mm_ctx *c) {
    if (c->prof_used < 2) {
        c->prof_used = 0;
        return;
    }
    for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->prof_ev[i], c->prof_ev[i + 1]));
        c->prof_seconds += ms * 1e-3;
        c->prof_launches += 1;
    }
    c->prof_used = 0;
}

// ---------------------------------------------------------------------------
// SELL-64 upload
// ---------------------------------------------------------------------------
void upload_sell(mm_ctx *c, const HostCsr &h, Sell &d) {
    d.nrows = h.nrows;
    d.vw = h.vw;
    d.nslices = (h.nrows + kSlice - 1) / kSlice;
    std::vector<int64_t> sptr(d.nslices + 1, 0);
    for (int s = 0; s < d.nslices; ++s) {
        int64_t w = 0;
        for (int r = s * kSlice; r < std::min(h.nrows, (s + 1) * kSlice); ++r) w = std::max(w, h.ptr[r + 1] - h.ptr[r]);
        sptr[s + 1] = sptr[s] + w * kSlice;
    }
    d.padded = sptr[d.nslices];
    d.nnz = h.ptr.empty() ? 0 : h.ptr[h.nrows];
    std::vector<int> col(std::max<int64_t>(d.padded, 1), 0);
    std::vector<double> val(std::max<int64_t>(d.padded * h.vw, 1), 0.0);
    for (int s = 0; s < d.nslices; ++s) {
        for (int ln = 0; ln < kSlice; ++ln) {
            int r = s * kSlice + ln;
            if (r >= h.nrows) break;
            for (int64_t k = 0; k < h.ptr[r + 1] - h.ptr[r]; ++k) {
                int64_t e = sptr[s] + kSlice * k;
                col[e + ln] = h.col[h.ptr[r] + k];
                for (int q = 0; q < h.vw; ++q) val[e * h.vw + q * kSlice + ln] = h.val[(h.ptr[r] + k) * h.vw + q];
            }
        }
    }
    d.sptr = dalloc_n<int64_t>(c, sptr.size());
    d.col = dalloc_n<int>(c, col.size());
    d.val = dalloc_n<double>(c, val.size());
    d.val32 = dalloc_n<float>(c, val.size());
    HIPCHK(hipMemcpyAsync(d.sptr, sptr.data(), sptr.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(d.col, col.data(), col.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(d.val, val.data(), val.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_to_f32((int64_t)val.size(), d.val, d.val32, c->stream);
    if (!h.row_out.empty()) {
        d.row_out = dalloc_n<int>(c, h.row_out.size());
        HIPCHK(hipMemcpyAsync(d.row_out, h.row_out.data(), h.row_out.size() * sizeof(int), hipMemcpyHostToDevice,
                              c->stream));
    }
    sync(c);  // host vectors go out of scope
}

void upload_vec(mm_ctx *c, double *dst, const std::vector<double> &v) {
    HIPCHK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    sync(c);
}

void setup_device(mm_ctx *c) {
    free_all(c);
    const int nm = c->n_mag(), np = c->n_pot();
    upload_sell(c, c->as.C, c->C);
    upload_sell(c, c->as.S, c->S);
    upload_sell(c, c->as.K, c->K);
    upload_sell(c, c->as.B, c->B);
    upload_sell(c, c->as.Bt, c->Bt);
    c->L = dalloc_n<double>(c, nm);
    c->invDex = dalloc_n<double>(c, nm);
    c->invDK = dalloc_n<double>(c, np);
    c->invDK32 = dalloc_n<float>(c, np);
    upload_vec(c, c->L, c->as.L);
    std::vector<double> t(nm);
    for (int a = 0; a < nm; ++a) t[a] = 1.0 / c->as.Dex[a];
    upload_vec(c, c->invDex, t);
    std::vector<double> tk(np);
    for (int r = 0; r < np; ++r) tk[r] = 1.0 / c->as.DK[r];
    upload_vec(c, c->invDK, tk);
    launch_to_f32(np, c->invDK, c->invDK32, c->stream);
    for (auto &s : c->st) {
        s.x = dalloc_n<double>(c, 3 * (size_t)nm);
        s.G = dalloc_n<double>(c, 3 * (size_t)nm);
        s.g = dalloc_n<double>(c, 3 * (size_t)nm);
        s.lam = dalloc_n<double>(c, nm);
    }
    c->d = dalloc_n<double>(c, 3 * (size_t)nm);
    c->y = dalloc_n<double>(c, 3 * (size_t)nm);
    c->pr = dalloc_n<double>(c, 3 * (size_t)nm);
    c->pp = dalloc_n<double>(c, 3 * (size_t)nm);
    c->pq = dalloc_n<double>(c, 3 * (size_t)nm);
    c->tmp3 = dalloc_n<double>(c, 3 * (size_t)nm);
    c->dscale = dalloc_n<double>(c, nm);
    c->u = dalloc_n<double>(c, np);
    c->b = dalloc_n<double>(c, np);
    c->cr = dalloc_n<double>(c, np);
    c->cp = dalloc_n<double>(c, np);
    c->cp2 = dalloc_n<double>(c, np);
    c->cq = dalloc_n<double>(c, np);
    c->usave = dalloc_n<double>(c, np);
    c->p32b = dalloc_n<float>(c, np);
    c->pst = dalloc_n<PcgState>(c, 1);
    c->ppart = dalloc_n<double>(c, kPcgPartDoubles);
    c->x32 = dalloc_n<float>(c, np);
    c->r32 = dalloc_n<float>(c, np);
    c->p32 = dalloc_n<float>(c, np);
    c->q32 = dalloc_n<float>(c, np);
    c->part = dalloc_n<double>(c, (size_t)PS_TOTAL * kMaxPartials);
    c->dsc = dalloc_n<double>(c, SC_TOTAL);
    c->dflags = dalloc_n<int>(c, FL_TOTAL);
    HIPCHK(hipMemsetAsync(c->u, 0, np * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->b, 0, np * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->part, 0, (size_t)PS_TOTAL * kMaxPartials * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->dflags, 0, FL_TOTAL * sizeof(int), c->stream));
    HIPCHK(hipMemsetAsync(c->pst, 0, sizeof(PcgState), c->stream));
    HIPCHK(hipMemsetAsync(c->ppart, 0, kPcgPartDoubles * sizeof(double), c->stream));
    sync(c);
    c->last_poisson_iters = 16;
}

// ---------------------------------------------------------------------------
// Poisson: K u = b (warm start u), Jacobi-PCG; FP64 or FP32 defect correction
// ---------------------------------------------------------------------------
constexpr int kPcgChunk = 8;  // CG iterations per captured graph (even: the p double buffer returns)

// capture kPcgChunk iterations (2 kernels each) once per context and mode
hipGraphExec_t pcg_graph(mm_ctx *c, bool fp32) {
    hipGraphExec_t &ge = fp32 ? c->graph32 : c->graph64;
    if (ge) return ge;
    hipStream_t s = c->stream;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < kPcgChunk; ++j) {
        const int ph = 2 * j + 2;
        if (fp32) {
            float *po = (j & 1) ? c->p32b : c->p32, *pn = (j & 1) ? c->p32 : c->p32b;
            launch_pcg_iter32(c->K, c->x32, c->r32, po, pn, c->q32, c->invDK32, c->pst, ph, j & 1, c->ppart, s);
        } else {
            double *po = (j & 1) ? c->cp2 : c->cp, *pn = (j & 1) ? c->cp : c->cp2;
            launch_pcg_iter64(c->K, c->u, c->cr, po, pn, c->cq, c->invDK, c->pst, ph, j & 1, c->ppart, s);
        }
    }
    HIPCHK(hipStreamEndCapture(s, &g));
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    return ge;
}

void pull_pcg(mm_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->hpst, c->pst, sizeof(PcgState), hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// replay graph chunks until the device flag reports convergence; returns
// iterations. With timing on, HIP events bracket every batch of replays and
// the executed iterations of the batch are counted (speculative replays after
// convergence return at once; their time stays in the measurement).
bool use_graphs() {
    static bool on = [] {
        const char *e = std::getenv("MMNCG_NO_GRAPH");
        return !(e && std::atoi(e) != 0);
    }();
    return on;
}

void pcg_chunk_eager(mm_ctx *c, bool fp32) {
    hipStream_t s = c->stream;
    for (int j = 0; j < kPcgChunk; ++j) {
        const int ph = 2 * j + 2;
        if (fp32) {
            float *po = (j & 1) ? c->p32b : c->p32, *pn = (j & 1) ? c->p32 : c->p32b;
            launch_pcg_iter32(c->K, c->x32, c->r32, po, pn, c->q32, c->invDK32, c->pst, ph, j & 1, c->ppart, s);
        } else {
            double *po = (j & 1) ? c->cp2 : c->cp, *pn = (j & 1) ? c->cp : c->cp2;
            launch_pcg_iter64(c->K, c->u, c->cr, po, pn, c->cq, c->invDK, c->pst, ph, j & 1, c->ppart, s);
        }
    }
}

long pcg_replay(mm_ctx *c, bool fp32, long maxit) {
    hipGraphExec_t ge = use_graphs() ? pcg_graph(c, fp32) : nullptr;
    long expect = std::max<long>(kPcgChunk, c->last_poisson_iters);
    long nrep = (expect + kPcgChunk - 1) / kPcgChunk;
    long launched = 0, seen = 0;
    for (;;) {
        prof_mark(c);
        for (long k = 0; k < nrep; ++k) {
            if (ge) HIPCHK(hipGraphLaunch(ge, c->stream));
            else pcg_chunk_eager(c, fp32);
        }
        prof_mark(c);
        launched += nrep * kPcgChunk;
        pull_pcg(c);
        if (c->prof_on) {
            prof_harvest(c);
            c->prof_units += c->hpst->iters - seen;
            seen = c->hpst->iters;
        }
        if (c->hpst->done || c->hpst->zero_u) break;
        if (launched >= maxit) throw ApiError{MM_NOT_CONVERGED, "scalar-potential CG did not converge"};
        nrep = std::max<long>(1, (expect / 8 + kPcgChunk - 1) / kPcgChunk);
    }
    return c->hpst->iters;
}

long poisson_fp64(mm_ctx *c, double rtol, long maxit) {
    const int n = c->n_pot();
    if (n == 0) return 0;
    launch_pcg_init64(c->K, c->b, c->u, c->cr, c->invDK, rtol * rtol, c->pst, c->ppart, false, c->stream);
    long it = pcg_replay(c, false, maxit);
    if (c->hpst->zero_u) {
        HIPCHK(hipMemsetAsync(c->u, 0, n * sizeof(double), c->stream));
        return 0;
    }
    c->last_poisson_iters = std::max<long>(4, it);
    return it;
}

long poisson_fp32(mm_ctx *c, double rtol, long maxit) {
    const int n = c->n_pot();
    if (n == 0) return 0;
    hipStream_t s = c->stream;
    long total = 0;
    for (int outer = 0; outer < 50; ++outer) {
        launch_residual64(c->K, c->b, c->u, c->cr, c->pst, c->ppart, s);
        pull_pcg(c);
        double bb = c->hpst->bb, rr = c->hpst->rr;
        if (bb == 0.0) {
            HIPCHK(hipMemsetAsync(c->u, 0, n * sizeof(double), s));
            return total;
        }
        if (rr <= rtol * rtol * bb) return total;
        double rn = std::sqrt(rr);
        // relative target of the inner FP32 solve: not beyond what the last correction needs
        double inner = std::max(1e-5, 0.5 * rtol * std::sqrt(bb) / rn);
        inner = std::min(inner, 1e-1);
        launch_pcg_init32(n, c->cr, 1.0 / rn, c->x32, c->r32, c->invDK32, inner * inner, c->pst, c->ppart, s);
        long it = pcg_replay(c, true, maxit - total);
        total += it;
        c->last_poisson_iters = std::max<long>(4, it);
        launch_add_correction(n, c->u, c->x32, rn, s);
        if (total >= maxit) throw ApiError{MM_NOT_CONVERGED, "scalar-potential CG did not converge"};
    }
    throw ApiError{MM_NOT_CONVERGED, "scalar-potential defect correction did not converge"};
}

long poisson(mm_ctx *c, double rtol, long maxit, bool fp32) {
    HIPCHK(hipEventRecord(c->ev[0], c->stream));
    long it = fp32 ? poisson_fp32(c, rtol, maxit) : poisson_fp64(c, rtol, maxit);
    HIPCHK(hipEventRecord(c->ev[1], c->stream));
    HIPCHK(hipEventSynchronize(c->ev[1]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    c->t_mag += ms * 1e-3;
    c->c_mi += it;
    return it;
}

// ---------------------------------------------------------------------------
// evaluation at st.x (energy, gradient, projection), optionally with the
// line-search extras relative to the state x0 along d with step alpha
// ---------------------------------------------------------------------------
int cmode_of(int terms) { return ((terms & MM_T_EXCH) ? 1 : 0) | ((terms & MM_T_ANIS) ? 2 : 0); }

void eval(mm_ctx *c, State &st, const double h[3], const mm_opts &o, const State *x0 = nullptr,
          double alpha = 0.0, double *dF = nullptr, double *dphi = nullptr, double *dxinf = nullptr) {
    hipStream_t s = c->stream;
    const bool fp32 = o.precision == MM_FP32_BULK;
    const int nm = c->n_mag();
    const bool demag = (o.terms & MM_T_DEMAG) && c->n_pot() > 0 && c->B.nrows > 0;
    if (demag) {
        launch_bmul(c->B, st.x, c->b, fp32, s);
        poisson(c, o.poisson_rtol, o.poisson_maxit, fp32);
    }
    double hz[3] = {0, 0, 0};
    if (o.terms & MM_T_ZEE)
        for (int k = 0; k < 3; ++k) hz[k] = h[k];
    launch_eval_epilogue(c->C, c->S, c->Bt, cmode_of(o.terms), demag ? 1 : 0, st.x, c->u, c->L, hz, st.G, st.g,
                         st.lam, x0 ? x0->x : nullptr, x0 ? x0->g : nullptr, x0 ? x0->lam : nullptr,
                         x0 ? c->d : nullptr, alpha, partp(c, PS_EVAL), fp32, s);
    launch_finalize(partp(c, PS_EVAL), grid_for_rows(nm), kEvalParts, eval_max_mask(), c->dsc + SC_EVAL, s);
    pull(c, SC_EVAL, kEvalParts);
    const double *r = c->hsc + SC_EVAL;
    st.Eloc = r[0];
    st.Ez = r[1];
    st.Ed = r[2];
    st.E = r[0] + r[1] + r[2];
    st.tmax = r[6];
    st.ginf = r[7];
    st.minf = r[9];
    if (dF) *dF = r[3];
    if (dphi) *dphi = r[4];
    if (dxinf) *dxinf = r[8];
    c->c_evals++;
}

double exchange_energy(mm_ctx *c, const double *m, bool fp32) {
    launch_energy_split(c->S, m, partp(c, PS_MISC), fp32, c->stream);
    launch_finalize(partp(c, PS_MISC), grid_for_rows(c->n_mag()), 1, 0u, c->dsc + SC_MISC, c->stream);
    pull(c, SC_MISC, 1);
    return c->hsc[SC_MISC];
}

void energy_parts(mm_ctx *c, const State &st, const mm_opts &o, double E[5]) {
    const bool fp32 = o.precision == MM_FP32_BULK;
    double ex = 0.0, an = 0.0;
    int cm = cmode_of(o.terms);
    if (cm == 3) {
        ex = exchange_energy(c, st.x, fp32);
        an = st.Eloc - ex;
    } else if (cm == 1) {
        ex = st.Eloc;
    } else if (cm == 2) {
        an = st.Eloc;
    }
    E[0] = ex;
    E[1] = an;
    E[2] = st.Ez;
    E[3] = st.Ed;
    E[4] = st.E;
}

// ---------------------------------------------------------------------------
// preconditioner: at most jmax steps of Alg. 1 on P y = g (exits li1-li3);
// the iteration count is fetched at the next synchronization
// ---------------------------------------------------------------------------
void precondition(mm_ctx *c, const State &st, int jmax, const double *dscale, const mm_opts &o) {
    hipStream_t s = c->stream;
    const int nm = c->n_mag();
    const bool fp32 = o.precision == MM_FP32_BULK;
    HIPCHK(hipEventRecord(c->ev[2], s));
    if (jmax <= 0) {
        HIPCHK(hipMemcpyAsync(c->y, st.g, 3 * (size_t)nm * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemsetAsync(c->dflags + FL_PREC, 0, 4 * sizeof(int), s));
    } else {
        int *fl = c->dflags + FL_PREC;
        launch_prec_init(nm, st.g, c->invDex, dscale, c->y, c->pr, c->pp, partp(c, PS_PR_INIT), fl, s);
        for (int j = 0; j < jmax; ++j) {
            const double *prev = (j == 0) ? partp(c, PS_PR_INIT) : partp(c, (j & 1) ? PS_PR_RZ1 : PS_PR_RZ0);
            double *nw = partp(c, ((j + 1) & 1) ? PS_PR_RZ1 : PS_PR_RZ0);
            const int ph = 3 * j;
            launch_prec_apply(c->C, st.x, st.lam, c->pp, c->pq, partp(c, PS_PR_PQ), fl, ph + 1, fp32, s);
            launch_prec_update(nm, j, st.g, c->invDex, dscale, c->y, c->pr, c->pp, c->pq, partp(c, PS_PR_PQ), prev, 0,
                               nw, fl, ph + 2, s);
            if (j + 1 < jmax)
                launch_prec_pupdate(nm, c->invDex, dscale, c->pp, c->pr, partp(c, PS_PR_INIT), nw, prev, 0, fl,
                                    ph + 3, s);
        }
    }
    HIPCHK(hipEventRecord(c->ev[3], s));
    HIPCHK(hipMemcpyAsync(c->hflags + FL_PREC, c->dflags + FL_PREC, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
}
void account_precondition(mm_ctx *c) {
    // call after a synchronization that follows precondition()
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    c->t_lin += ms * 1e-3;
    c->c_li += c->hflags[FL_PREC + 1];
}

// direction: first -> d = -y (or -g); else beta*ZA with the descent safeguard.
// returns phi'(0) = <g1, d>, dmax and the safeguard mode (0, 1, 2)
void direction(mm_ctx *c, const State &s1, const State *s0, bool first, double *dp0, double *dmax, int *mode) {
    hipStream_t s = c->stream;
    const int nm = c->n_mag();
    int nb = 0;
    launch_dir_dots(nm, s1.g, first ? nullptr : s0->g, c->y, first ? nullptr : c->d, partp(c, PS_DIR_DOTS), &nb, s);
    launch_dir_update(nm, s1.g, c->y, c->d, partp(c, PS_DIR_DOTS), nb, first ? 1 : 0, partp(c, PS_DIR_OUT),
                      c->dflags + FL_DIR, s);
    launch_finalize(partp(c, PS_DIR_OUT), grid_for_rows(nm), 2, 2u, c->dsc + SC_DIR, s);
    HIPCHK(hipMemcpyAsync(c->hflags + FL_DIR, c->dflags + FL_DIR, sizeof(int), hipMemcpyDeviceToHost, s));
    pull(c, SC_DIR, 2);
    *dp0 = c->hsc[SC_DIR];
    *dmax = c->hsc[SC_DIR + 1];
    *mode = c->hflags[FL_DIR];
}

// ---------------------------------------------------------------------------
// line search on phi(alpha) = F(N(x + alpha d)): capped rotation, sufficient
// decrease on the exact quadratic energy difference, one cubic interpolation,
// then halving (the paper asks only for an approximate search that avoids too
// long steps)
// ---------------------------------------------------------------------------
bool cubic_step(double at, double dFt, double dp0, double dpt, double *ac) {
    double d1 = dp0 + dpt - 3.0 * dFt / at;
    double disc = d1 * d1 - dp0 * dpt;
    if (!(disc >= 0.0) || !std::isfinite(disc)) return false;
    double d2 = std::sqrt(disc);
    double den = dpt - dp0 + 2.0 * d2;
    if (!(den != 0.0) || !std::isfinite(den)) return false;
    double a = at - at * (dpt + d2 - d1) / den;
    if (!std::isfinite(a)) return false;
    *ac = a;
    return true;
}

struct LsResult {
    bool ok;
    int idx;        // state index holding the accepted point
    double alpha;
    double dF;
    double dxinf;
};

LsResult line_search(mm_ctx *c, const mm_opts &o, const double h[3], int i0, double dp0, double dmax, double a0) {
    const int nm = c->n_mag();
    int iA = (i0 + 1) % 3, iB = (i0 + 2) % 3;
    State &s0 = c->st[i0];
    auto trial = [&](int idx, double alpha, double *dF, double *dp, double *dx) {
        launch_trial(nm, s0.x, c->d, alpha, c->st[idx].x, c->stream);
        eval(c, c->st[idx], h, o, &s0, alpha, dF, dp, dx);
    };
    LsResult res{false, i0, 0, 0, 0};
    if (!(dmax > 0.0)) return res;
    double amax = o.theta_max / dmax;
    double at = std::min(a0, amax);
    double dFt, dpt, dxt;
    trial(iA, at, &dFt, &dpt, &dxt);
    bool arm_t = dFt <= o.c1 * at * dp0;
    if (arm_t && std::fabs(dpt) <= o.c2 * std::fabs(dp0)) return LsResult{true, iA, at, dFt, dxt};
    bool over = !arm_t || dpt > 0.0;
    if (!over && at >= amax) return LsResult{true, iA, at, dFt, dxt};
    double ac;
    if (!cubic_step(at, dFt, dp0, dpt, &ac)) ac = over ? 0.5 * at : std::min(2.0 * at, amax);
    if (over) {
        ac = std::max(ac, 0.1 * at);
        ac = std::min(ac, 0.9 * at);
    } else {
        double hi = std::min(4.0 * at, amax);
        ac = std::min(ac, hi);
        ac = std::max(ac, 1.1 * at);
        if (ac > hi) return LsResult{true, iA, at, dFt, dxt};
    }
    double dFc, dpc, dxc;
    trial(iB, ac, &dFc, &dpc, &dxc);
    if (dFc <= o.c1 * ac * dp0) return LsResult{true, iB, ac, dFc, dxc};
    if (arm_t) return LsResult{true, iA, at, dFt, dxt};
    double a = std::min(at, ac);
    for (int k = 0; k < o.ls_max_halvings; ++k) {
        a *= 0.5;
        double dFa, dpa, dxa;
        trial(iA, a, &dFa, &dpa, &dxa);
        if (dFa <= o.c1 * a * dp0) return LsResult{true, iA, a, dFa, dxa};
    }
    return res;
}

// ---------------------------------------------------------------------------
// Alg. 4 for one reduced field; the start point is in st[*cur].x; on return
// *cur indexes the final state
// ---------------------------------------------------------------------------
int trace_level() {
    static int lvl = [] {
        const char *e = std::getenv("MMNCG_TRACE");
        return e ? std::atoi(e) : 0;
    }();
    return lvl;
}

int minimize(mm_ctx *c, int *cur, const double h[3], const mm_opts &o, mm_stats *stats) {
    auto t0 = std::chrono::steady_clock::now();
    c->c_evals = c->c_mi = c->c_li = 0;
    c->t_mag = c->t_lin = 0;
    long nli = 0, restarts = 0, fallbacks = 0;
    int i0 = *cur;
    eval(c, c->st[i0], h, o);
    int status = MM_NOT_CONVERGED;
    if (o.stop_mode == MM_STOP_TORQUE && c->st[i0].tmax < o.tol_torque) {
        status = MM_OK;
    } else {
        precondition(c, c->st[i0], o.jmax, nullptr, o);
        double dp0, dmax;
        int mode;
        direction(c, c->st[i0], nullptr, true, &dp0, &dmax, &mode);
        account_precondition(c);
        if (mode != 0) fallbacks++;
        bool first = true;
        double a_prev = 0, dp_prev = 0;
        for (long it = 0; it < o.max_nli; ++it) {
            if (!(dp0 < 0.0)) {
                status = MM_OK;
                break;
            }
            double a0 = first ? (o.jmax > 0 ? 1.0 : o.theta_init / dmax) : a_prev * dp_prev / dp0;
            LsResult ls = line_search(c, o, h, i0, dp0, dmax, a0);
            if (!ls.ok) {
                restarts++;
                // steepest descent restart: d = -g (direction() with y = g, first = true)
                HIPCHK(hipMemcpyAsync(c->y, c->st[i0].g, 3 * (size_t)c->n_mag() * sizeof(double),
                                      hipMemcpyDeviceToDevice, c->stream));
                direction(c, c->st[i0], nullptr, true, &dp0, &dmax, &mode);
                if (!(dp0 < 0.0) || !(dmax > 0.0)) {
                    status = MM_STALLED;
                    break;
                }
                ls = line_search(c, o, h, i0, dp0, dmax, o.theta_init / dmax);
                if (!ls.ok) {
                    status = MM_STALLED;
                    break;
                }
            }
            nli++;
            State &s1 = c->st[ls.idx];
            State &s0 = c->st[i0];
            if (trace_level() > 0 && (nli <= 40 || nli % 100 == 0))
                std::fprintf(stderr,
                             "[mmncg] nli %ld alpha %.4e amax %.4e a0 %.4e dp0 %.4e dF %.4e dE %.4e tmax %.4e "
                             "E %.12e evals %ld\n",
                             nli, ls.alpha, o.theta_max / dmax, a0, dp0, ls.dF, s1.E - s0.E, s1.tmax, s1.E,
                             c->c_evals);
            bool conv;
            if (o.stop_mode == MM_STOP_TORQUE) {
                conv = s1.tmax < o.tol_torque;
            } else {
                double tau = o.tau_F;
                bool t1 = (s0.E - s1.E) < tau * (1.0 + std::fabs(s1.E));
                bool t2 = ls.dxinf < std::sqrt(tau) * (1.0 + s1.minf);
                bool t3 = s1.ginf < std::cbrt(tau) * (1.0 + std::fabs(s1.E));
                conv = t1 && t2 && t3;
            }
            if (conv) {
                i0 = ls.idx;
                status = MM_OK;
                break;
            }
            precondition(c, s1, o.jmax, nullptr, o);
            double dpn, dmx;
            direction(c, s1, &s0, false, &dpn, &dmx, &mode);
            account_precondition(c);
            if (mode != 0) fallbacks++;
            a_prev = ls.alpha;
            dp_prev = dp0;
            first = false;
            i0 = ls.idx;
            dp0 = dpn;
            dmax = dmx;
        }
    }
    *cur = i0;
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->evals = c->c_evals;
        stats->nli = nli;
        stats->li = c->c_li;
        stats->mi = c->c_mi;
        stats->restarts = restarts;
        stats->fallbacks = fallbacks;
        stats->t_nl = std::chrono::duration<double>(t1 - t0).count();
        stats->t_lin = c->t_lin;
        stats->t_mag = c->t_mag;
        stats->F = c->st[i0].E;
        stats->torque_max = c->st[i0].tmax;
        stats->status = status;
    }
    return status;
}

void reduce_field(const mm_ctx *c, const double *BT, double h[3]) {
    for (int k = 0; k < 3; ++k) h[k] = BT[k] / (kMu0 * c->as.Ms_ref);
}

// load m (host or device), check finite and unit length
void load_m(mm_ctx *c, State &st, const double *m) {
    const int nm = c->n_mag();
    copy_in(c, st.x, m, 3 * (size_t)nm);
    launch_mavg(nm, st.x, c->L, partp(c, PS_MISC), c->stream);
    launch_finalize(partp(c, PS_MISC), grid_for_rows(nm), 5, 1u << 4, c->dsc + SC_MISC, c->stream);
    pull(c, SC_MISC, 5);
    double dev = c->hsc[SC_MISC + 4];
    if (!(dev <= 1e-6)) throw ApiError{MM_EINVAL, "m must hold finite unit vectors (max | |m_i| - 1 | = " +
                                                      std::to_string(dev) + ")"};
}

bool opts_valid(const mm_opts &o, std::string &why) {
    if (o.jmax < 0) why = "jmax < 0";
    else if (!(o.tol_torque > 0)) why = "tol_torque <= 0";
    else if (!(o.theta_max > 0) || !(o.theta_init > 0)) why = "theta_max/theta_init <= 0";
    else if (!(o.c1 > 0 && o.c1 < 1) || !(o.c2 > o.c1 && o.c2 < 1)) why = "need 0 < c1 < c2 < 1";
    else if (!(o.poisson_rtol > 0)) why = "poisson_rtol <= 0";
    else if (o.max_nli < 1) why = "max_nli < 1";
    else if (o.precision != MM_FP64 && o.precision != MM_FP32_BULK) why = "unknown precision";
    else if (o.stop_mode != MM_STOP_TORQUE && o.stop_mode != MM_STOP_PAPER) why = "unknown stop_mode";
    else if (o.stop_mode == MM_STOP_PAPER && !(o.tau_F > 0)) why = "tau_F <= 0";
    else if (o.poisson_maxit < 1) why = "poisson_maxit < 1";
    else return true;
    return false;
}

template <class F>
int guarded(mm_ctx *c, F &&f) {
    if (!c) return MM_EINVAL;
    try {
        HIPCHK(hipSetDevice(c->device));
        int rc = f();
        if (rc >= 0) c->err.clear();
        return rc;
    } catch (const ApiError &e) {
        c->err = e.msg;
        return e.code;
    } catch (const HipError &e) {
        c->err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
        (void)hipGetLastError();
        return MM_EDEVICE;
    } catch (const std::bad_alloc &) {
        c->err = "host allocation failed";
        return MM_ENOMEM;
    } catch (const std::exception &e) {
        c->err = e.what();
        return MM_EDEVICE;
    }
}

void require_ready(mm_ctx *c) {
    if (!c->have_mesh || !c->have_mat) throw ApiError{MM_ESTATE, "mesh and material must be set first"};
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int mm_opts_default(mm_opts *o) {
    if (!o) return MM_EINVAL;
    std::memset(o, 0, sizeof *o);
    o->jmax = 4;
    o->tol_torque = 1e-6;
    o->stop_mode = MM_STOP_TORQUE;
    o->tau_F = 1e-10;
    o->theta_max = 0.2;
    o->theta_init = 0.01;
    o->c1 = 1e-4;
    o->c2 = 0.1;
    o->poisson_rtol = 1e-10;
    o->max_nli = 20000;
    o->precision = MM_FP64;
    o->terms = MM_T_ALL;
    o->ls_max_halvings = 20;
    o->poisson_maxit = 100000;
    return MM_OK;
}

int mm_create(mm_ctx **out, int device, void *hip_stream, mm_alloc_fn dev_alloc, mm_free_fn dev_free,
              void *alloc_user) {
    if (!out) return MM_EINVAL;
    *out = nullptr;
    if ((dev_alloc == nullptr) != (dev_free == nullptr)) return MM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return MM_EDEVICE;
    }
    mm_ctx *c = new (std::nothrow) mm_ctx();
    if (!c) return MM_ENOMEM;
    c->device = device;
    c->ualloc = dev_alloc;
    c->ufree = dev_free;
    c->user = alloc_user;
    mm_opts_default(&c->opts);
    int rc = guarded(c, [&] {
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipHostMalloc((void **)&c->hsc, SC_TOTAL * sizeof(double), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&c->hflags, FL_TOTAL * sizeof(int), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&c->hpst, sizeof(PcgState), hipHostMallocDefault));
        std::memset(c->hpst, 0, sizeof(PcgState));
        std::memset(c->hsc, 0, SC_TOTAL * sizeof(double));
        std::memset(c->hflags, 0, FL_TOTAL * sizeof(int));
        return MM_OK;
    });
    if (rc != MM_OK) {
        mm_destroy(c);
        return rc;
    }
    *out = c;
    return MM_OK;
}

int mm_destroy(mm_ctx *c) {
    if (!c) return MM_EINVAL;
    (void)hipSetDevice(c->device);
    free_all(c);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->prof_ev) (void)hipEventDestroy(e);
    if (c->hsc) (void)hipHostFree(c->hsc);
    if (c->hflags) (void)hipHostFree(c->hflags);
    if (c->hpst) (void)hipHostFree(c->hpst);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MM_OK;
}

const char *mm_last_error(const mm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int mm_get_info(const mm_ctx *c, mm_info *info) {
    if (!c || !info) return MM_EINVAL;
    std::memset(info, 0, sizeof *info);
    info->n_nodes = (long)c->xyz.size() / 3;
    info->n_tets = (long)c->tets.size() / 4;
    if (c->have_mat) {
        info->n_mag = c->as.n_mag;
        info->n_pot = c->as.n_pot;
        info->nnz_C_blocks = (long)c->C.nnz;
        info->nnz_K = (long)c->K.nnz;
        info->nnz_B = (long)c->B.nnz;
        info->Ms_ref = c->as.Ms_ref;
        size_t bytes = 0;
        for (const Sell *m : {&c->C, &c->S, &c->K, &c->B, &c->Bt})
            bytes += (size_t)m->padded * (sizeof(int) + m->vw * (sizeof(double) + sizeof(float)));
        bytes += (size_t)c->as.n_mag * (3 * 3 * 8 + 3 * 8 + 6 * 3 * 8 + 3 * 8);
        bytes += (size_t)c->as.n_pot * (8 * 6 + 4 * 5);
        info->device_bytes = bytes;
    }
    return MM_OK;
}

int mm_mesh_upload(mm_ctx *c, const double *xyz, long n_nodes, const int *tets, long n_tets, const int *region) {
    return guarded(c, [&] {
        if (!xyz || !tets || !region || n_nodes < 4 || n_tets < 1) throw ApiError{MM_EINVAL, "bad mesh arguments"};
        if (is_device_ptr(xyz) || is_device_ptr(tets) || is_device_ptr(region))
            throw ApiError{MM_EINVAL, "mesh arrays must be host memory"};
        for (long e = 0; e < 4 * n_tets; ++e)
            if (tets[e] < 0 || tets[e] >= n_nodes) throw ApiError{MM_EMESH, "tet node index out of range"};
        for (long i = 0; i < 3 * n_nodes; ++i)
            if (!std::isfinite(xyz[i])) throw ApiError{MM_EMESH, "non-finite coordinate"};
        c->xyz.assign(xyz, xyz + 3 * n_nodes);
        c->tets.assign(tets, tets + 4 * n_tets);
        c->region.assign(region, region + n_tets);
        c->have_mesh = true;
        c->have_mat = false;
        free_all(c);
        return MM_OK;
    });
}

int mm_material_set(mm_ctx *c, const double *Ms, const double *A, const double *K1, const double *axis) {
    return guarded(c, [&] {
        if (!c->have_mesh) throw ApiError{MM_ESTATE, "upload the mesh first"};
        if (!Ms || !A || !K1) throw ApiError{MM_EINVAL, "Ms, A and K1 are required"};
        Assembly as;
        std::string e = assemble(c->xyz.data(), (long)c->xyz.size() / 3, c->tets.data(), (long)c->tets.size() / 4,
                                 c->region.data(), Ms, A, K1, axis, as);
        if (!e.empty()) throw ApiError{MM_EMESH, e};
        if (as.n_mag == 0) throw ApiError{MM_EMESH, "no magnet nodes"};
        for (int a = 0; a < as.n_mag; ++a)
            if (!(as.Dex[a] > 0.0)) throw ApiError{MM_EMESH, "zero exchange diagonal at a magnet node"};
        c->as = std::move(as);
        setup_device(c);
        c->have_mat = true;
        return MM_OK;
    });
}

int mm_magnet_nodes(const mm_ctx *c, long *n_mag, int *node_ids) {
    if (!c || !n_mag) return MM_EINVAL;
    if (!c->have_mat) return MM_ESTATE;
    *n_mag = c->as.n_mag;
    if (node_ids) std::memcpy(node_ids, c->as.node_of_mag.data(), sizeof(int) * c->as.n_mag);
    return MM_OK;
}

int mm_set_opts(mm_ctx *c, const mm_opts *o) {
    return guarded(c, [&] {
        if (!o) throw ApiError{MM_EINVAL, "null opts"};
        std::string why;
        if (!opts_valid(*o, why)) throw ApiError{MM_EINVAL, why};
        c->opts = *o;
        return MM_OK;
    });
}

int mm_reset_warm_start(mm_ctx *c) {
    return guarded(c, [&] {
        require_ready(c);
        HIPCHK(hipMemsetAsync(c->u, 0, c->n_pot() * sizeof(double), c->stream));
        sync(c);
        c->last_poisson_iters = 16;
        return MM_OK;
    });
}

int mm_energy_grad(mm_ctx *c, const double *m, const double h_ext[3], double E_parts[5], double *grad, double *gproj,
                   double *torque_max) {
    return guarded(c, [&] {
        require_ready(c);
        if (!m || !h_ext) throw ApiError{MM_EINVAL, "m and h_ext are required"};
        State &st = c->st[0];
        load_m(c, st, m);
        double h[3];
        reduce_field(c, h_ext, h);
        eval(c, st, h, c->opts);
        const size_t n3 = 3 * (size_t)c->n_mag();
        if (E_parts) energy_parts(c, st, c->opts, E_parts);
        if (grad) copy_out(c, grad, st.G, n3);
        if (gproj) copy_out(c, gproj, st.g, n3);
        if (torque_max) *torque_max = st.tmax;
        sync(c);
        return MM_OK;
    });
}

int mm_precondition(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax, const double *dscale,
                    double *y, int *inner_iters) {
    return guarded(c, [&] {
        require_ready(c);
        if (!m || !grad || !gproj || !y || jmax < 0) throw ApiError{MM_EINVAL, "bad precondition arguments"};
        const int nm = c->n_mag();
        State &st = c->st[0];
        load_m(c, st, m);
        copy_in(c, st.G, grad, 3 * (size_t)nm);
        copy_in(c, st.g, gproj, 3 * (size_t)nm);
        launch_lambda(nm, st.x, st.G, st.lam, c->stream);
        const double *ds = nullptr;
        if (dscale) {
            copy_in(c, c->dscale, dscale, nm);
            ds = c->dscale;
        }
        c->c_li = 0;
        c->t_lin = 0;
        precondition(c, st, jmax, ds, c->opts);
        copy_out(c, y, c->y, 3 * (size_t)nm);
        sync(c);
        account_precondition(c);
        if (inner_iters) *inner_iters = (int)c->c_li;
        return MM_OK;
    });
}

int mm_ncg_minimize(mm_ctx *c, double *m_inout, const double h_ext[3], const mm_opts *o, mm_stats *st,
                    double E_parts[5]) {
    return guarded(c, [&] {
        require_ready(c);
        if (!m_inout || !h_ext) throw ApiError{MM_EINVAL, "m and h_ext are required"};
        mm_opts op;
        if (o) op = *o;
        else mm_opts_default(&op);
        std::string why;
        if (!opts_valid(op, why)) throw ApiError{MM_EINVAL, why};
        int cur = 0;
        load_m(c, c->st[cur], m_inout);
        double h[3];
        reduce_field(c, h_ext, h);
        mm_stats s;
        int rc = minimize(c, &cur, h, op, &s);
        if (E_parts) energy_parts(c, c->st[cur], op, E_parts);
        copy_out(c, m_inout, c->st[cur].x, 3 * (size_t)c->n_mag());
        sync(c);
        if (st) *st = s;
        return rc;
    });
}

int mm_demag_curve(mm_ctx *c, double *m_inout, const double *h_list, long n, const mm_opts *o, double *m_avg,
                   double *E_tot, mm_stats *st, double *m_hist) {
    return guarded(c, [&] {
        require_ready(c);
        if (!m_inout || !h_list || n < 0) throw ApiError{MM_EINVAL, "bad curve arguments"};
        mm_opts op;
        if (o) op = *o;
        else mm_opts_default(&op);
        std::string why;
        if (!opts_valid(op, why)) throw ApiError{MM_EINVAL, why};
        const int nm = c->n_mag();
        int cur = 0;
        load_m(c, c->st[cur], m_inout);
        int worst = MM_OK;
        for (long k = 0; k < n; ++k) {
            double h[3];
            reduce_field(c, h_list + 3 * k, h);
            mm_stats s;
            int rc = minimize(c, &cur, h, op, &s);
            worst = std::max(worst, rc);
            if (m_avg) {
                launch_mavg(nm, c->st[cur].x, c->L, partp(c, PS_MISC), c->stream);
                launch_finalize(partp(c, PS_MISC), grid_for_rows(nm), 4, 0u, c->dsc + SC_MISC, c->stream);
                pull(c, SC_MISC, 4);
                for (int q = 0; q < 3; ++q) m_avg[3 * k + q] = c->hsc[SC_MISC + q] / c->hsc[SC_MISC + 3];
            }
            if (E_tot) E_tot[k] = c->st[cur].E;
            if (st) st[k] = s;
            if (m_hist) copy_out(c, m_hist + 3 * (size_t)nm * k, c->st[cur].x, 3 * (size_t)nm);
        }
        copy_out(c, m_inout, c->st[cur].x, 3 * (size_t)nm);
        sync(c);
        return worst;
    });
}

int mm_operator_apply(mm_ctx *c, int op, const double *in, double *out) {
    return guarded(c, [&] {
        require_ready(c);
        if (!in || !out) throw ApiError{MM_EINVAL, "null vector"};
        const int nm = c->n_mag(), np = c->n_pot();
        const bool fp32 = c->opts.precision == MM_FP32_BULK;
        hipStream_t s = c->stream;
        switch (op) {
            case MM_OP_C:
                copy_in(c, c->tmp3, in, 3 * (size_t)nm);
                launch_spmv_block6(c->C, c->tmp3, c->pq, fp32, s);
                copy_out(c, out, c->pq, 3 * (size_t)nm);
                break;
            case MM_OP_B:
                copy_in(c, c->tmp3, in, 3 * (size_t)nm);
                HIPCHK(hipMemsetAsync(c->cq, 0, np * sizeof(double), s));
                launch_bmul(c->B, c->tmp3, c->cq, fp32, s);
                copy_out(c, out, c->cq, np);
                break;
            case MM_OP_BT:
                copy_in(c, c->cq, in, np);
                launch_btmul(c->Bt, c->cq, c->pq, fp32, s);
                copy_out(c, out, c->pq, 3 * (size_t)nm);
                break;
            case MM_OP_K:
                copy_in(c, c->cr, in, np);
                launch_spmv_scalar(c->K, c->cr, c->cq, fp32, s);
                copy_out(c, out, c->cq, np);
                break;
            default:
                throw ApiError{MM_EINVAL, "unknown operator"};
        }
        sync(c);
        return MM_OK;
    });
}

int mm_poisson_solve(mm_ctx *c, const double *b, double *u_inout, double rtol, long *iters) {
    return guarded(c, [&] {
        require_ready(c);
        if (!b || !u_inout || !(rtol > 0)) throw ApiError{MM_EINVAL, "bad Poisson arguments"};
        const int np = c->n_pot();
        // the solve runs on the context's b and u: keep the warm start aside
        HIPCHK(hipMemcpyAsync(c->usave, c->u, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        copy_in(c, c->b, b, np);
        copy_in(c, c->u, u_inout, np);
        c->t_mag = 0;
        c->c_mi = 0;
        long it = poisson(c, rtol, c->opts.poisson_maxit, c->opts.precision == MM_FP32_BULK);
        copy_out(c, u_inout, c->u, np);
        // evaluations write only the magnet rows of b: clear it; restore u
        HIPCHK(hipMemsetAsync(c->b, 0, np * sizeof(double), c->stream));
        HIPCHK(hipMemcpyAsync(c->u, c->usave, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        sync(c);
        if (iters) *iters = it;
        return MM_OK;
    });
}

int mm_profile(mm_ctx *c, int enable, double out[4]) {
    return guarded(c, [&] {
        sync(c);
        prof_harvest(c);
        if (enable < 0) {
            c->prof_launches = c->prof_seconds = c->prof_units = 0;
        } else {
            c->prof_on = enable != 0;
        }
        if (out) {
            const bool fp32 = c->opts.precision == MM_FP32_BULK;
            const double vb = fp32 ? 4.0 : 8.0;
            out[0] = c->prof_units;
            out[1] = c->prof_seconds;
            // kernel A: matrix + r, D^-1, p_old read + p_new, q written;
            // kernel B: x, r, p, q, D^-1 read + x, r written (x is FP64 in the FP64 mode only)
            out[2] = c->have_mat ? (double)c->K.nnz * (vb + 4.0) + 12.0 * vb * c->K.nrows : 0.0;
            out[3] = c->have_mat ? (double)c->K.nrows : 0.0;
        }
        return MM_OK;
    });
}

}  // extern "C"
