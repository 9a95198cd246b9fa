// Internal declarations of the mmncg library (host assembly, device operators,
// kernel launchers). Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mmncg {

constexpr int kSlice = 64;      // rows per SELL slice = one wavefront
constexpr int kBlock = 256;     // threads per block for row kernels (4 slices)
constexpr int kPcgKinds = 6;    // kinds of scalar-potential solve per instance (3 roles x 2 passes)
constexpr int kMaxBlocksPerInst = 2048;  // per instance and row space (256 below 2M rows)
constexpr int kPoissonWaves = 16;       // default waves per block of the scalar-potential kernels

// ---------------------------------------------------------------------------
// host-side CSR produced by the assembly (row-major, sorted columns)
// ---------------------------------------------------------------------------
struct HostCsr {
    int nrows = 0;
    int vw = 1;                    // values per entry (1 scalar, 3 vector, 6 symmetric block)
    std::vector<int64_t> ptr;      // nrows + 1
    std::vector<int> col;
    std::vector<double> val;       // nnz * vw
    std::vector<int> row_out;      // optional output index per row
};

// ---------------------------------------------------------------------------
// device SELL-64 matrix: slice s holds rows [64 s, 64 s + 64); entry (s, k, lane)
// sits at e = sptr[s] + 64 k + lane; its value component c at
// val[(sptr[s] + 64 k) * vw + 64 c + lane]. Padding: col = 0, value 0.
// ---------------------------------------------------------------------------
struct Sell {
    int nrows = 0, nslices = 0, vw = 1;
    int64_t padded = 0, nnz = 0;
    int64_t *sptr = nullptr;   // nslices + 1
    int *col = nullptr;
    double *val = nullptr;
    float *val32 = nullptr;    // FP32 copy for the FP32-bulk mode (may be null)
    int *row_out = nullptr;    // optional output index per row
};

// Host assembly result (everything in reduced units).
struct Assembly {
    double Ms_ref = 0;
    long n_nodes = 0, n_tets = 0;
    int n_mag = 0, n_pot = 0;
    std::vector<int> mag_of_node, node_of_mag, pot_of_node;
    std::vector<double> L;         // Ms-weighted lumped nodal volume (n_mag)
    std::vector<double> Dex;       // exchange diagonal (n_mag)
    std::vector<double> DK;        // Poisson diagonal (n_pot)
    HostCsr C;                     // exchange + anisotropy, symmetric 3x3 blocks (vw 6: xx yy zz xy xz yz)
    HostCsr S;                     // exchange only, scalar (for the energy split)
    HostCsr K;                     // Poisson matrix on free nodes
    HostCsr B;                     // rows: magnet nodes that are free (row_out = free index), cols magnet, vw 3
    HostCsr Bt;                    // rows: magnet nodes, cols free nodes, vw 3
    // device order of the free nodes: device row r holds free node pot_order[r]
    // (locality_order); every matrix above keeps the free-node numbering
    std::vector<int> pot_order;
};

// Order of the free (potential) nodes on the device: the bounding box is cut
// into cubic tiles of about 4096 nodes, the tiles are taken in x-fastest order
// and the nodes keep their numbering order inside a tile. A matrix-vector
// product then gathers its neighbours from rows close by in every direction,
// not from whole grid planes away, so they stay in the L2 cache. Identity
// below 8,192 nodes (one tile). order[r] = the free node on device row r.
std::vector<int> locality_order(const double *xyz, const std::vector<int> &node_of_free);

// Builds every operator from the mesh and per-tet SI materials. Returns an
// error message (empty on success).
std::string assemble(const double *xyz, long n_nodes, const int *tets, long n_tets, const int *region,
                     const double *Ms, const double *A, const double *K1, const double *axis,
                     Assembly &out);

// ---------------------------------------------------------------------------
// Instance batching. Several independent problems ("instances") share every
// launch: their rows are concatenated, each instance padded to whole SELL
// slices. A RowMap partitions one row space (magnet rows, potential rows or
// divergence rows) into logical blocks that never straddle two instances:
// block b covers slices [tab[b].y, tab[b].z) of instance tab[b].x, the blocks
// of instance i are [ipb[i], ipb[i+1]), and its real rows end at rend[i].
// Per-block partial sums are stored at part[q * nblk + b]; the reductions of
// instance i read only its own blocks.
// ---------------------------------------------------------------------------
struct RowMap {
    const int4 *tab = nullptr;
    const int *ipb = nullptr;
    const int *rend = nullptr;
    int nblk = 0;
    int ninst = 0;
};

// state vectors of one evaluation point (magnet rows)
struct StateV {
    double *x = nullptr, *G = nullptr, *g = nullptr, *lam = nullptr;
};

// per-instance scalar-potential CG state (device memory). alpha/gamma hold
// the step and r.z of the last two iterations (slot = iteration parity).
struct PcgState {
    double tol2, bb, rr, scale;
    double alpha[2], gamma[2];
    int done, iters, zero_u, active;
};

constexpr int kEvalParts = 10;  // Eloc, Ezee, Edemag, dF, dphi, |g|^2, max torque, max|g|_inf, max|m-x0|_inf, max|m|_inf
unsigned eval_max_mask();
constexpr int kDirParts = 6;
constexpr int kPcgSlots = 8;    // partial slots of the scalar-potential CG

// --- operators (kernels.hip) ---
void launch_spmv_block6(const Sell &C, const RowMap &M, const double *x, double *y, bool fp32, hipStream_t s);
void launch_spmv_scalar(const Sell &A, const RowMap &M, const double *x, double *y, bool fp32, hipStream_t s);
void launch_bmul(const Sell &B, const RowMap &MB, const int *act, const StateV *sv, const int *role, double *b,
                 bool fp32, hipStream_t s);
void launch_btmul(const Sell &Bt, const RowMap &M, const double *u, double *gout, bool fp32, hipStream_t s);

// --- evaluation (kernels.hip) ---
struct EvalLaunch {
    const Sell *C, *S, *Bt;
    const RowMap *M;
    int cmode, use_demag;
    const int *act, *role;     // per instance: active, which state (0 cur, 1 T, 2 C)
    StateV st[3];              // cur, T, C
    const double *u, *L, *h3, *d, *alpha;
    double *part;
    bool fp32;
};
void launch_trial(const RowMap &M, const int *act, const int *role, const StateV st[3], const double *d,
                  const double *alpha, hipStream_t s);
void launch_eval_epilogue(const EvalLaunch &e, hipStream_t s);
void launch_finalize_inst(const RowMap &M, const double *part, int nslot, unsigned is_max, double *out,
                          hipStream_t s);
void launch_copy_state(const RowMap &M, const int *from, const StateV st[3], double *gprev, hipStream_t s);

// --- preconditioner (kernels.hip) ---
struct PrecLaunch {
    const Sell *C;
    const RowMap *M;
    const int *act;
    const double *m, *lam, *g, *invDex, *dscale;
    double *y, *r, *p, *q;
    double *part;              // 7 slots: INIT(2), PQ(1), RZ0(2), RZ1(2)
    int *flags;                // per instance: {stop phase, iterations, exit reason, -}
    bool fp32;
    int form = 0;              // MM_PFORM_*: terms of eq. (precond)
};
void launch_prec_init(const PrecLaunch &a, hipStream_t s);
void launch_prec_iter(const PrecLaunch &a, int j, bool last, hipStream_t s);
// the two halves of launch_prec_iter: q = P p, then the update kernels
void launch_prec_apply(const PrecLaunch &a, int j, hipStream_t s);
void launch_prec_tail(const PrecLaunch &a, int j, bool last, hipStream_t s);

// --- direction (kernels.hip) ---
// beta_kind: 0 beta*ZA, 1 beta*FR, 2 beta*PRP, 3 beta*HS; gy: 2 x ninst doubles
// (<g, y> of the last direction per instance, and its snapshot)
void launch_dir(const RowMap &M, const int *act, const int *first, const double *g1, const double *g0,
                const double *y1, double *d, double *part_dots, double *part_out, int *info, int beta_kind,
                double *gy, hipStream_t s);

// --- misc (kernels.hip) ---
void launch_energy_split(const Sell &S, const RowMap &M, const double *m, double *part, bool fp32, hipStream_t s);
void launch_mavg(const RowMap &M, const double *m, const double *L, double *part, hipStream_t s);
void launch_lambda(const RowMap &M, const double *m, const double *G, double *lam, hipStream_t s);
void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s);
void launch_fill(int64_t n, double *x, double v, hipStream_t s);
// per-instance operations on the scalar potential over the potential rows M:
// op[i] = 0 none, 1 ux <- u, 2 ut <- u, 3 ux <- ut, 4 u <- ux + rho[i] (ut - ux),
// 5 ux <- u and ut <- u
enum { POT_NONE = 0, POT_UX_U = 1, POT_UT_U = 2, POT_UX_UT = 3, POT_INTERP = 4, POT_BOTH_U = 5 };
void launch_pot_op(const RowMap &M, const int *op, const double *rho, double *u, double *ux, double *ut,
                   hipStream_t s);
void launch_gather(int64_t n, const int *idx, const double *in, double *out, hipStream_t s);

// --- scalar-potential CG (poisson.hip) ---
// per-node record of the single-reduction CG: residual r, w = K D^-1 r,
// s = K p and the Jacobi factor d = D^-1, interleaved so that the neighbour
// values one stored matrix entry needs come in one 16-byte (FP32) or 32-byte
// (FP64) load; double-buffered by iteration parity (d is written to both
// buffers at the start of a solve). The direction p is a plain array.
template <class VT>
struct alignas(4 * sizeof(VT)) PcgNode {
    VT r, w, s, d;
};
template <class VT>
struct PcgVecs {
    PcgNode<VT> *q[2];
    VT *p;
};
struct PcgLaunch {
    const Sell *K;
    const RowMap *M;
    PcgState *st;              // per instance
    double *part;              // kPcgSlots slots of M->nblk
    double *u, *b;             // FP64 solution and right-hand side
    double *r64;               // FP64 residual of the defect-correction mode
    const double *invD;
    PcgVecs<double> v64;
    float *x32;                // FP32 correction of the defect-correction mode
    const float *invD32;
    PcgVecs<float> v32;
    const double *pin;         // per instance 4 doubles: FP32 rhs scale, inner tol^2 (<= 0: inactive), rn, -
    int nw;                    // waves per block of the row map M (4, 8 or 16)
};
void launch_pcg_init64(const PcgLaunch &a, const int *act, double rtol2, hipStream_t s);
void launch_residual64(const PcgLaunch &a, const int *act, hipStream_t s);
void launch_pcg_init32(const PcgLaunch &a, hipStream_t s);
void launch_pcg_iter64(const PcgLaunch &a, int parity, hipStream_t s);
void launch_pcg_iter32(const PcgLaunch &a, int parity, hipStream_t s);
void launch_add_correction(const PcgLaunch &a, hipStream_t s);
// pieces of the CG start shared with the multigrid variant: r = b - K u into
// the r fields of records 0 with the partials (b.b, r.r); the FP32 inner
// start (x = 0, r = r64 * scale); the start partials into the CG state
// (mode 0: CG start, 1: FP32 inner start, 2: residual only)
void launch_pcg_residual_q(const PcgLaunch &a, const int *act, bool fp32_matrix, hipStream_t s);
void launch_pcg_start32_only(const PcgLaunch &a, hipStream_t s);
void launch_pcg_fin(const PcgLaunch &a, const int *act, double rtol2, int mode, hipStream_t s);

// --- algebraic multigrid preconditioner of the scalar-potential CG (amg.hip) ---
// Level l of the smoothed-aggregation hierarchies of all instances (device
// pointers). Every instance has its own hierarchy; level l of the launch is
// the concatenation of the instances' level-l rows, each instance's block
// padded to a multiple of 4 rows (level 0: the potential row space of the
// row map). Level 0 is the scalar-potential matrix itself (the SELL matrix K
// of the CG) with P (prolongation from level 1, CSR over the level-0 rows)
// and R = P^T (rows of level 1). On a level 0 < l < L_i of instance i the
// V(1,1) step is two fused operators: down, b_{l+1} = Dn b_l with Dn = P^T
// (I - omega A D^-1); up, y_l = Up [b_l; y_{l+1}] with Up = [S | Q], S =
// 2 omega D^-1 - omega^2 D^-1 A D^-1, Q = (I - omega D^-1 A) P (the two
// damped-Jacobi sweeps and the coarse correction multiplied out). The b
// part of level l and the y part of level l+1 are one array (b at its start,
// y after the level's rows). Instances whose coarsest level is l solve it
// with their dense inverse (rows ld apart, ld = rows padded to 4; padding
// zero), listed in a table: dense row r belongs to entry dinst[r], whose
// rows start at drow0, number dn, lie at row dboff of the level's b and y,
// and whose inverse starts at daoff.
constexpr int kAmgMaxLevels = 12;
template <class VT>
struct AmgLevel {
    int n = 0;                 // rows of the level (padded blocks)
    const VT *wd = nullptr;    // level 0: omega_i / a_ii per row (0 on padding)
    const int *Pp = nullptr, *Pj = nullptr;  // level 0
    const VT *Pv = nullptr;
    const int *Rp = nullptr, *Rj = nullptr;
    const VT *Rv = nullptr;
    const int *Dp = nullptr, *Dj = nullptr;  // levels 1 .. nlev - 2
    const VT *Dv = nullptr;
    const int *Up = nullptr, *Uj = nullptr;
    const VT *Uv = nullptr;
    const int *iof = nullptr;  // instance of every row of the level (-1: padding)
    int ndense = 0;            // dense rows on this level (0: none)
    const int *dinst = nullptr, *drow0 = nullptr, *dn = nullptr, *dld = nullptr, *dboff = nullptr, *dwho = nullptr;
    const int64_t *daoff = nullptr;
    const VT *Ainv = nullptr;
    VT *b = nullptr, *y = nullptr;  // right-hand side and result of the level
    VT *t = nullptr, *z = nullptr;  // level 0: pre-smoothing residual, prolongated correction
    int gP = 4, gR = 8, gD = 8, gU = 8;  // lanes per row of the CSR kernels (4..64)
};
template <class VT>
struct AmgLaunch {
    int nlev = 0;                  // levels of the deepest hierarchy
    AmgLevel<VT> lv[kAmgMaxLevels];
    VT *u = nullptr;               // level 0: the preconditioned residual M r
    VT *rf = nullptr;              // level 0: the CG residual r as a plain vector (the records hold it
                                   // too, among three other fields the cycle does not read)
    VT *wf = nullptr;              // level 0: w = K u of the CG as a plain vector
    const VT *omega = nullptr;     // per instance: the fine smoothing weight
    bool single = true;            // one instance: the cycle's kernels read its flag without the row tables
};
// CG start: residual, one cycle, w = K u, partials, state (the instances of act)
void launch_amg_init64(const PcgLaunch &a, const AmgLaunch<double> &g, const int *act, double rtol2, hipStream_t s);
// mixed solve (FP32-bulk mode): FP64 CG vectors and residual norms on the
// FP32-stored matrix, the cycle in FP32; the solution goes straight to u
void launch_amg_initmix(const PcgLaunch &a, const AmgLaunch<float> &g, const AmgLaunch<double> &g64, const int *act,
                        double rtol2, hipStream_t s);
// one CG iteration of parity `parity` (a chain of launches)
void launch_amg_iter64(const PcgLaunch &a, const AmgLaunch<double> &g, int parity, hipStream_t s);
void launch_amg_itermix(const PcgLaunch &a, const AmgLaunch<float> &g, const AmgLaunch<double> &g64, int parity,
                        hipStream_t s);
// one cycle applied to the plain vector r (n_pot rows) into g.u
void launch_amg_apply64(const PcgLaunch &a, const AmgLaunch<double> &g, const double *r, hipStream_t s);
void launch_amg_apply32(const PcgLaunch &a, const AmgLaunch<float> &g, const float *r, hipStream_t s);

// --- learned component (gnn.hip); widths fixed: 32 features, 64 channels ---
// f32: FP32 operands on the vector units (debug mode) instead of BF16 MFMA
void gnn_mm(int M, int K, int NC, int epi, const float *A, int lda, const float *W, int ldw, bool transW,
            const float *bias, float *Y, int ldy, float *Ypre, int ldp, const float *R, int ldr, bool f32,
            hipStream_t s);
int gnn_tn_blocks(int M);
void gnn_targets(int n, const double *m, const double *m1, const double *diag3, const double *invD, double *dmt,
                 double *st, hipStream_t s);
int gnn_moment_blocks(int n);
void gnn_moments(int n, const float *X, double *part, double *out, hipStream_t s);
void gnn_mm_tn(int M, int KI, int NC, const float *A, int lda, const float *B, int ldb, float *part, float *out,
               bool accumulate, bool f32, hipStream_t s);
void gnn_tn32(int M, int KI, int NC, const float *A, int lda, const float *B, int ldb, float *part, float *out,
              hipStream_t s);
void gnn_agg(int n, const int *ptr, const int *idx, const float *invdeg, const float *H, int ldh, float *out, int ldo,
             hipStream_t s);
void gnn_agg_t_add(int n, const int *ptr, const int *idx, const float *invdeg, const float *G, int ldg, float *out,
                   int ldo, hipStream_t s);
void gnn_edge_add(int n, const float *ebar, const float *We2, float *q, int ldq, hipStream_t s);
void gnn_silu_bwd(int64_t len, const float *x, const float *pre, float *y, hipStream_t s);
void gnn_add64(int n, const float *in, int ldi, float *out, int ldo, hipStream_t s);
void gnn_copy64(int n, const float *in, int ldi, float *out, int ldo, hipStream_t s);
void gnn_heads(int n, const float *h, const float *Wm, const float *bm, const float *Ws, const float *bs,
               const double *m, float *zm, float *zs, double *dm, double *sv, hipStream_t s);
int gnn_loss_blocks(int n);
void gnn_loss_heads(int n, const float *zm, const float *zs, const double *m, const double *dm_t, const double *s_t,
                    const double *L, double inv_sumL, double inv_dm2, double w_s, float *d_zm, float *d_zs,
                    double *part, double *loss_out, hipStream_t s);
void gnn_heads_dh(int n, const float *d_zm, const float *d_zs, const float *Wm, const float *Ws, float *dh,
                  hipStream_t s);
void gnn_adam(int np, float *th, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps,
              float bc1, float bc2, hipStream_t s);
void gnn_features(int n, const double *m, const double *G, const double *g, const double *Cm, const double *L,
                  const float *stat, const double hn[3], const double hp[3], float *X, hipStream_t s);
void gnn_norm_features(int n, const float *X, const float *mu, const float *sd, float *Xn, hipStream_t s);
void gnn_f64_to_f32(int64_t n, const double *a, float *b, hipStream_t s);
void gnn_f32_to_f64(int64_t n, const float *a, double *b, hipStream_t s);

}  // namespace mmncg
