// Context of the mmncg library shared by its host translation units (the
// solver control in solver.cpp, the learned component in gnn.cpp): device
// buffers and control block of a batch of instances, error handling and the
// helpers both use. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "mmncg.h"
#include "internal.h"

namespace mmncg {


constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr int kPcgChunk = 16;  // CG iterations per captured graph (even: the double buffers return to parity 0)
constexpr int kAmgChunk = 2;   // the same for the multigrid-preconditioned CG (about 10 launches per iteration)
constexpr int kPrecCheck = 16; // inner preconditioner iterations between host looks at its exit flags

struct HipError {
    hipError_t e;
    const char *what;
};
#define HIPCHK(x)                                     \
    do {                                              \
        hipError_t _e = (x);                          \
        if (_e != hipSuccess) throw HipError{_e, #x}; \
    } while (0)

struct ApiError {
    int code;
    std::string msg;
};

// magnet-row partial slots (each M.nblk doubles)
enum MagSlot {
    MS_EVAL = 0,                   // kEvalParts
    MS_PREC = MS_EVAL + kEvalParts,  // 7
    MS_DOTS = MS_PREC + 7,         // kDirParts
    MS_DOUT = MS_DOTS + kDirParts,  // 2
    MS_MISC = MS_DOUT + 2,         // 5
    MS_TOTAL = MS_MISC + 5
};

// field kernels with per-launch timers
enum KernelTimer { KT_EVAL = 0, KT_BMUL = 1, KT_PREC_APPLY = 2, KT_N = 3 };

// per-instance metadata kept on the host
struct InstInfo {
    long n_nodes = 0, n_tets = 0;
    int n_mag = 0, n_pot = 0, n_brow = 0;
    int mag_off = 0, pot_off = 0, brow_off = 0;  // first global (padded) row
    long user_off = 0;                           // first magnet node in caller arrays
    long nnz_C = 0, nnz_K = 0, nnz_B = 0, nnz_S = 0;
    double Ms_ref = 0;
    std::vector<int> node_of_mag;
    std::vector<int> pot_order;  // device row r (local) holds free node pot_order[r]
};

// device tables of one RowMap
struct DevMap {
    RowMap map;
};

// scalars of one evaluation point
struct Sc {
    double E = 0, Eloc = 0, Ez = 0, Ed = 0, tmax = 0, ginf = 0, minf = 0, dF = 0, dphi = 0, dxinf = 0;
};

// running counters of an instance (monotone; per-field stats are differences)
struct Cnt {
    long evals = 0, mi = 0, li = 0;
    double t_mag = 0, t_lin = 0;
};


}  // namespace mmncg

struct mm_gnn;
struct mm_graph;
namespace mmncg {
struct AmgState;
}

using namespace mmncg;  // private header: the context's members are library types

struct mm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mm_alloc_fn ualloc = nullptr;
    mm_free_fn ufree = nullptr;
    void *user = nullptr;
    std::string err;
    std::vector<std::pair<void *, size_t>> allocs;
    size_t dev_bytes = 0;

    // single-instance mesh (host copy until materials arrive)
    std::vector<double> xyz;
    std::vector<int> tets, region;
    bool have_mesh = false, have_mat = false;

    int ninst = 0;
    std::vector<InstInfo> inst;
    long tot_mag = 0;   // sum of n_mag (caller layout)
    int rows_m = 0, rows_p = 0, rows_b = 0;  // padded global row counts

    Sell C, S, K, B, Bt;
    DevMap Mm, Mp, Mb;  // magnet rows, potential rows, divergence rows
    // block shape of the scalar-potential kernels: waves per block (launch
    // wide) and SELL slices per wave of each instance
    int pnw = kPoissonWaves;
    int pbm = 1;  // multiplier of the default cap on blocks per instance (make_map)
    std::vector<int> pspw, poff, pn;
    bool tuned = false;
    double *L = nullptr, *invDex = nullptr, *invDK = nullptr;
    // potential rows: free-node index of each device row and device row of
    // each free node (global, instance offsets included)
    int *pord = nullptr, *ppos = nullptr;
    float *invDK32 = nullptr;

    StateV st[3];  // current state, trial T, trial C
    double *gprev = nullptr, *d = nullptr, *y = nullptr, *pr = nullptr, *pp = nullptr, *pq = nullptr,
           *dscale = nullptr, *tmp3 = nullptr;
    double *gy = nullptr;  // per instance <g, y> of the last direction, and its snapshot (2 x ninst)
    double *u = nullptr, *b = nullptr, *cr = nullptr, *cq = nullptr, *usave = nullptr;
    // the line search's potentials: ux at the accepted state, ut at the last
    // trial of role 1 (the start of a role-2 trial's solve is interpolated
    // between them); per-instance operations staged in pinned memory, two
    // slots (before and after an evaluation round) of ninst doubles and ninst
    // ints each
    double *ux = nullptr, *ut = nullptr;
    double *hpr = nullptr, *dpr = nullptr;
    PcgNode<double> *q64[2] = {};  // CG node records by parity
    PcgNode<float> *q32[2] = {};
    double *p64 = nullptr;         // CG directions
    float *p32 = nullptr;
    float *x32 = nullptr;
    PcgState *pst = nullptr;    // device, ninst
    PcgState *hpst = nullptr;   // pinned host mirror
    double *mpart = nullptr;    // magnet-row partials, MS_TOTAL slots
    double *ppart = nullptr;    // potential-row partials, kPcgSlots slots
    hipGraphExec_t graph64 = nullptr, graph32 = nullptr;
    // multigrid preconditioner: host copies of the scalar-potential matrices,
    // the hierarchies once built, their captured graphs
    std::vector<HostCsr> hostK;  // per instance
    mmncg::AmgState *amg = nullptr;
    hipGraphExec_t agraph64 = nullptr, mgraph = nullptr;

    // control block: ints {act, role, first, from, pact, plive} (host-written)
    // then {info, pflags x4} (device-written); doubles {alpha, h3 x3, pin x4}
    int *dci = nullptr, *hci = nullptr;
    double *dcd = nullptr, *hcd = nullptr;
    // finalize outputs: eval (kEvalParts), dir (2), misc (5) per instance
    double *dsc = nullptr, *hsc = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

    mm_opts opts;
    // iterations of the last scalar-potential solve of each kind, per instance
    // (kPcgKinds slots: the evaluation's role 0..2, first or later pass of the
    // defect correction): the next solve of that kind replays as many before
    // it first asks the device whether it has converged
    std::vector<long> last_pcg;
    int pcg_pass = 0;  // defect-correction pass of the solve being replayed
    std::vector<double> pcg_bytes64, pcg_bytes32;
    std::vector<Cnt> cnt;
    // kernel timing (mm_profile)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
    double prof_seconds = 0, prof_units = 0, prof_bytes = 0;
    // per-launch timing of the field kernels (mm_profile_kernels): event pairs
    // around k_eval_epilogue, k_bmul and the first k_prec_apply of each inner
    // solve, with the algorithmic bytes of each timed launch
    bool kt_on = false;
    std::vector<hipEvent_t> kt_ev[KT_N];
    std::vector<double> kt_pend[KT_N];   // bytes of the pairs not yet harvested
    double kt_sec[KT_N] = {0, 0, 0}, kt_calls[KT_N] = {0, 0, 0}, kt_bytes[KT_N] = {0, 0, 0};

    // control block accessors
    int *act() const { return hci; }
    int *role() const { return hci + ninst; }
    int *first() const { return hci + 2 * ninst; }
    int *from() const { return hci + 3 * ninst; }
    int *pact() const { return hci + 4 * ninst; }
    int *plive() const { return hci + 5 * ninst; }
    int *info() const { return hci + 6 * ninst; }
    int *pflags() const { return hci + 7 * ninst; }
    double *alpha() const { return hcd; }
    double *h3() const { return hcd + ninst; }
    double *pin() const { return hcd + 4 * ninst; }
    template <class T>
    T *dev(T *hostp, T *hbase, T *dbase) const {
        return dbase + (hostp - hbase);
    }
    int *d_(int *hp) const { return dci + (hp - hci); }
    double *d_(double *hp) const { return dcd + (hp - hcd); }
};

namespace mmncg {

// --- helpers (solver.cpp) ---
void *dalloc(mm_ctx *c, size_t bytes);
template <class T>
T *dalloc_n(mm_ctx *c, size_t n) {
    return (T *)dalloc(c, n * sizeof(T));
}
void dfree(mm_ctx *c, void *p);
bool is_device_ptr(const void *p);
void copy_in(mm_ctx *c, double *dst, const double *src, size_t n);
void copy_out(mm_ctx *c, double *dst, const double *src, size_t n);
// instance 0's potential vectors across the ABI (free-node numbering) and the
// device (locality order); tmp: a scratch vector of n_pot doubles
void pot_in(mm_ctx *c, double *dev, const double *abi, double *tmp);
void pot_out(mm_ctx *c, double *abi, const double *dev, double *tmp);
void sync(mm_ctx *c);
void upload_ctl(mm_ctx *c);
void poisson(mm_ctx *c, double rtol, long maxit, bool fp32, bool amg, const std::vector<int> &on);
double now_s();
PcgLaunch pcg_args(mm_ctx *c);

// --- multigrid preconditioner (amg.cpp) ---
AmgState *amg_get(mm_ctx *c);   // builds the hierarchy on first use
void amg_release(mm_ctx *c);
const AmgLaunch<double> &amg_launch64(AmgState *s);
const AmgLaunch<float> &amg_launch32(AmgState *s);
// algorithmic bytes of one CG iteration per instance: form 0 FP64, 1 FP32, 2 mixed
const std::vector<double> &amg_bytes(AmgState *s, int form);
void load_m(mm_ctx *c, const double *m);
void reduce_field(const InstInfo &I, const double *BT, double h[3]);
void eval_all(mm_ctx *c, const mm_opts &o, const std::vector<double> &h);
Sc eval_result(mm_ctx *c, int i);
mm_opts resolve_opts(const mm_opts *o);
void require_ready(mm_ctx *c);
void require_single(mm_ctx *c);

// --- learned component (gnn.cpp) ---
// After the evaluation of instance 0 at (m_k, h_next) has filled the current
// state, writes the network's tangent proposal into c->d and its Jacobi
// factors into c->dscale (both on the magnet rows).
void gnn_propose(mm_ctx *c, mm_gnn *g, mm_graph *gr, const double h_prev[3], const double h_next[3]);

// scratch of the inner solve of Alg. 1 (the residual, direction and product
// vectors, 3 x rows_m doubles each; the 7 partial-sum slots of the magnet-row
// map, 7 x nblk doubles; the exit flags, 4 ints per instance); null members
// mean the context's own buffers
struct PrecScratch {
    double *r = nullptr, *p = nullptr, *q = nullptr, *part = nullptr;
    int *flags = nullptr;
};
// bytes a PrecScratch for this context needs when carved out of one block
// (each piece aligned to 256 bytes), and the carving itself
size_t prec_scratch_bytes(const mm_ctx *c);
PrecScratch prec_scratch_at(const mm_ctx *c, void *base);
// mm_precondition's body; ext = nullptr uses the context's buffers
int precondition_call(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax,
                      const double *dscale, double *y, int *inner_iters, const PrecScratch *ext);

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

}  // namespace mmncg
