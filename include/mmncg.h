/*
 * mmncg.h - C ABI of the MI355X (gfx950) library for micromagnetic energy
 * minimization with the preconditioned projected nonlinear conjugate gradient
 * method of Exl, Fischbacher, Kovacs, Oezelt, Gusenbauer and Schrefl
 * ("Preconditioned nonlinear conjugate gradient method for micromagnetic
 * energy minimization").
 *
 * The problem (Sec. 2.2, eq. (opt)): minimize the P1 finite-element energy
 *   F(m) = 1/2 m^T C m - 1/2 h_d^T M m - h_ext^T M m      (eq. (energy))
 * subject to |m_i| = 1 at every magnet node, for a sequence of applied fields
 * (Sec. 3.1: one minimization per field value, each started from the previous
 * minimizer). The minimizer is Alg. 4 with the restarted Hestenes-Stiefel
 * beta*ZA; the preconditioner is the sparse local-field approximation of the
 * Hessian of the Lagrangian, eq. (precond) without its last term, solved with a
 * few steps of Alg. 1 with the exchange diagonal as Jacobi preconditioner.
 * The stray field comes from a scalar potential on the magnet plus an air box
 * with zero Dirichlet values on the outer boundary (Sec. 3.1).
 *
 * Units. Coordinates in nm. Materials in SI (Ms in A/m, A in J/m, K1 in
 * J/m^3). Applied fields in Tesla (mu0 H). Internally the library works in
 * reduced units: length 1 nm, magnetization Ms_ref = max Ms, energy
 * mu0 Ms_ref^2 nm^3, fields in units of Ms_ref. Energies and gradients
 * returned by the ABI are in these reduced units; torques |m x h_eff| are in
 * units of Ms_ref.
 *
 * Vectors. A magnetization or gradient is n_mag x 3 doubles, node-major
 * (x, y, z of node 0, then node 1, ...), ordered by ascending mesh-node index
 * of the magnet nodes (nodes touched by a tet with region > 0).
 *
 * Host or device pointers. Every double* vector argument may point to host
 * memory or to device memory of the context's GPU; the library detects which.
 * Device vectors are read/written on the context's stream.
 *
 * Ownership. The caller owns every pointer it passes; the library copies what
 * it needs during the call and keeps no caller pointer after return. Device
 * buffers belong to the context and come from the allocator callbacks given to
 * mm_create (hipMalloc/hipFree when NULL).
 *
 * Errors. Negative return codes mean failure and that no output was written;
 * mm_last_error() then holds a message. Positive codes mean the outputs were
 * written with a warning (not converged within max_nli, or the line search
 * stalled). The library never aborts the process; HIP failures map to
 * MM_EDEVICE.
 *
 * Concurrency. One context per host thread; contexts share no state. Calls on
 * one context are serialized by the caller. Every call that returns host
 * results synchronizes the context's stream before returning.
 */
#ifndef MMNCG_H
#define MMNCG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_ctx mm_ctx;

enum {
    MM_OK = 0,
    MM_EINVAL = -1,        /* bad argument (NULL, size, NaN, non-unit m) */
    MM_ENOMEM = -2,        /* device or host allocation failed */
    MM_EDEVICE = -3,       /* a HIP call failed */
    MM_EMESH = -4,         /* degenerate tet, no magnet, inconsistent mesh */
    MM_ESTATE = -5,        /* call out of order (e.g. no mesh/material yet) */
    MM_NOT_CONVERGED = 1,  /* max_nli reached; outputs hold the last iterate */
    MM_STALLED = 2,        /* line search failed twice (also along -g) */
    MM_NONFINITE = 3       /* an evaluation gave a NaN or infinite energy (e.g. a breakdown of a
                              linear solve); outputs hold the last finite accepted iterate */
};

enum { MM_FP64 = 0, MM_FP32_BULK = 1 };
enum { MM_PREC_JACOBI = 0, MM_PREC_AMG = 1 };
enum { MM_BETA_ZA = 0, MM_BETA_FR = 1, MM_BETA_PRP = 2, MM_BETA_HS = 3 };
enum { MM_PFORM_PAPER = 0, MM_PFORM_FULL = 1, MM_PFORM_LOCAL = 2 };
enum { MM_STOP_TORQUE = 0, MM_STOP_PAPER = 1 };
enum { MM_T_EXCH = 1, MM_T_ANIS = 2, MM_T_ZEE = 4, MM_T_DEMAG = 8, MM_T_ALL = 15 };

typedef struct {
    int jmax;              /* (li1) inner PCG iteration cap; 0 = unpreconditioned NCG */
    double tol_torque;     /* MM_STOP_TORQUE: stop when max_i |m_i x h_eff,i| < tol */
    int stop_mode;         /* MM_STOP_TORQUE or MM_STOP_PAPER ((t1)-(t3) of Sec. 3.1) */
    double tau_F;          /* function tolerance for (t1)-(t3) */
    double theta_max;      /* line search: largest nodal rotation per step (rad) */
    double theta_init;     /* first trial rotation when jmax = 0 (rad) */
    double c1, c2;         /* sufficient-decrease and curvature constants */
    double poisson_rtol;   /* scalar-potential CG: stop at |r| <= rtol |b| */
    long max_nli;          /* nonlinear iteration cap per field value */
    int precision;         /* MM_FP64 or MM_FP32_BULK: FP32-stored operators; the
                              scalar potential by FP32 CG inside FP64 defect
                              correction (Jacobi), or by FP64 CG vectors on the
                              FP32-stored matrix with an FP32 multigrid cycle
                              (multigrid); FP64 reductions and master m */
    int terms;             /* energy terms, MM_T_* bitmask */
    int ls_max_halvings;   /* line-search backtracking cap */
    long poisson_maxit;    /* scalar-potential CG iteration cap per solve */
    int poisson_prec;      /* scalar-potential CG preconditioner: MM_PREC_JACOBI,
                              or MM_PREC_AMG (algebraic multigrid as in Sec. 3.1;
                              in a batch every instance needs more than 2048
                              free potential nodes, else MM_ESTATE) */
    int beta;              /* beta* of the direction update: MM_BETA_ZA (Alg. 4, the
                              default), or the preconditioned FR*, PRP* or HS*
                              forms of Sec. 2.1 (FR*, PRP*: <g_{j+1}, y_{j+1}> and
                              <g_{j+1} - g_j, y_{j+1}> over <g_j, y_j>; HS*: ZA
                              without its restart); a non-positive denominator
                              gives beta = 0 */
    int prec_form;         /* preconditioner action, a form of eq. (precond) with
                              C = exchange + anisotropy: MM_PFORM_PAPER (the
                              default, without the last term, as Sec. 2.2 chooses),
                              MM_PFORM_FULL (all four terms; not symmetric), or
                              MM_PFORM_LOCAL (the projected local part
                              C v - (m.Cv) m only) */
    int theta_adapt;       /* 1: the rotation cap follows the accepted steps: a
                              step the cap stopped doubles it (up to theta_hi), a
                              step below a quarter of it halves it (down to
                              theta_max); each field starts at theta_max.
                              0 (the default): the cap stays theta_max */
    double theta_hi;       /* upper bound of the adapted cap (rad), >= theta_max */
} mm_opts;

typedef struct {
    long evals;            /* energy+gradient evaluations */
    long nli;              /* nonlinear (outer) iterations */
    long li;               /* inner preconditioner CG iterations */
    long mi;               /* scalar-potential CG iterations */
    long restarts;         /* steepest-descent restarts after a failed line search */
    long fallbacks;        /* descent safeguard activations */
    double t_nl, t_lin, t_mag; /* seconds: total, preconditioner, magnetostatics */
    double F;              /* final total energy (reduced units) */
    double torque_max;     /* final max |m x h_eff| */
    int status;            /* MM_OK, MM_NOT_CONVERGED, MM_STALLED or MM_NONFINITE */
} mm_stats;

typedef struct {
    long n_nodes, n_tets, n_mag, n_pot;   /* mesh nodes, tets, magnet nodes, free potential nodes */
    long nnz_C_blocks, nnz_K, nnz_B;      /* stored nonzeros (padding excluded) */
    double Ms_ref;                        /* A/m */
    size_t device_bytes;                  /* device memory held by the context */
} mm_info;

/* Fill o with the defaults: jmax 4, tol_torque 1e-6, torque stopping,
   tau_F 1e-10, theta_max 0.2, theta_init 0.01, c1 1e-4, c2 0.1,
   poisson_rtol 1e-10, max_nli 20000, FP64, all terms, 20 halvings,
   poisson_maxit 100000, Jacobi-preconditioned scalar-potential CG,
   beta*ZA. */
int mm_opts_default(mm_opts *o);

typedef void *(*mm_alloc_fn)(size_t bytes, void *user);
typedef void (*mm_free_fn)(void *ptr, void *user);

/* Create a context on HIP device `device`. `hip_stream` (a hipStream_t, may be
   NULL) is borrowed: all work is enqueued on it; NULL makes the context create
   its own stream. dev_alloc/dev_free (both NULL or both set) provide device
   memory; `alloc_user` is passed through to them. */
int mm_create(mm_ctx **out, int device, void *hip_stream, mm_alloc_fn dev_alloc, mm_free_fn dev_free,
              void *alloc_user);
int mm_destroy(mm_ctx *c);
const char *mm_last_error(const mm_ctx *c);
int mm_get_info(const mm_ctx *c, mm_info *info);

/* Tetrahedral mesh (Sec. 2.2: P1 finite elements). xyz: n_nodes x 3 (nm);
   tets: n_tets x 4 node indices (0-based); region[t] = 0 for air, > 0 for
   magnetic material. Nodes on faces that belong to exactly one tet form the
   outer boundary, where the scalar potential is zero. Host pointers only. */
int mm_mesh_upload(mm_ctx *c, const double *xyz, long n_nodes, const int *tets, long n_tets,
                   const int *region);

/* Per-tet SI materials (Sec. 2.2: C = C_A + C_K and M carrying local Ms):
   Ms, A, K1 (n_tets each) and the easy axis (n_tets x 3, normalized here; may
   be NULL when every K1 is 0). Air tets are ignored. Assembles the device
   operators (the matrices C, K, B, B^T, the nodal weights of M and the
   exchange diagonal). Host pointers only. */
int mm_material_set(mm_ctx *c, const double *Ms, const double *A, const double *K1, const double *axis);

/* Number of magnet nodes and (when node_ids != NULL) their mesh-node ids. */
int mm_magnet_nodes(const mm_ctx *c, long *n_mag, int *node_ids);

/* Options used by mm_energy_grad / mm_precondition (minimize and curve take
   their own). */
int mm_set_opts(mm_ctx *c, const mm_opts *o);

/* Zero the scalar-potential warm start (the potential of the previous
   evaluation is the starting guess of the next Poisson CG). */
int mm_reset_warm_start(mm_ctx *c);

/* Energy and gradient (eq. (energy)) at unit vectors m for the applied field
   h_ext (Tesla). E_parts = {exchange, anisotropy, Zeeman, demag, total};
   grad = dF/dm (n_mag x 3); gproj = Pi_{m-perp}(grad) (eq. (nablaLF));
   torque_max = max_i |gproj_i| / L_i = max_i |m_i x h_eff,i| (eq. (optcond)).
   Every output may be NULL. */
int mm_energy_grad(mm_ctx *c, const double *m, const double h_ext[3], double E_parts[5], double *grad,
                   double *gproj, double *torque_max);

/* Approximately solve P y = gproj with at most jmax steps of Alg. 1 from
   y = 0, P v = C v - (m.(C v)) m - lambda v (eq. (precond) without its last
   term), lambda_i = m_i . grad_i, Jacobi = exchange diagonal (times dscale_i
   when dscale != NULL), exits (li1)-(li3). jmax = 0 returns y = gproj. */
int mm_precondition(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax,
                    const double *dscale, double *y, int *inner_iters);

/* For callers that cannot allocate device memory during a call (code under
   HIP graph capture, tight serving loops, harnesses that forbid allocation):
   mm_precondition with the same arguments, results and errors, except that
   the scratch of its inner solve (the residual, direction and product vectors
   of Alg. 1, the block partial sums and the exit flags) lives in a static
   device array of MM_NOALLOC_SCRATCH_BYTES per GPU instead of context memory;
   the call allocates nothing. The array is shared by every call on that GPU
   and keeps the last call's contents (the call clears what must start at
   zero); calls that overlap on one GPU race. A context whose inner solve
   needs more than the array holds (about 460,000 magnet nodes) is refused
   with MM_EINVAL. Each GPU the library runs on keeps its array until the
   process ends. */
#define MM_NOALLOC_SCRATCH_BYTES (32u << 20)
int mm_precondition_noalloc(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax,
                            const double *dscale, double *y, int *inner_iters);

/* Alg. 4 for one field (Tesla), m_inout updated in place. Returns MM_OK,
   MM_NOT_CONVERGED or MM_STALLED (outputs written in all three cases). */
int mm_ncg_minimize(mm_ctx *c, double *m_inout, const double h_ext[3], const mm_opts *o, mm_stats *st,
                    double E_parts[5]);

/* Demagnetization curve (Sec. 3.1): for k = 0..n-1 minimize at h_list[k]
   (Tesla, n x 3) from the previous minimizer. m_avg (n x 3) = sum_i L_i m_i /
   sum_i L_i, E_tot (n), st (n), m_hist (n x n_mag x 3) may each be NULL.
   m_inout ends at the last minimizer. Returns the worst per-step status. */
int mm_demag_curve(mm_ctx *c, double *m_inout, const double *h_list, long n, const mm_opts *o,
                   double *m_avg, double *E_tot, mm_stats *st, double *m_hist);

/* Single operators for checking (same kernels as the solver):
   MM_OP_C   : out = C in            (n_mag x 3 -> n_mag x 3; exchange + anisotropy)
   MM_OP_B   : out = b(in)           (n_mag x 3 -> n_pot; divergence right-hand side)
   MM_OP_BT  : out = B^T in          (n_pot -> n_mag x 3; stray-field gradient from a potential)
   MM_OP_K   : out = K in            (n_pot -> n_pot; Poisson matrix, Dirichlet rows removed) */
enum { MM_OP_C = 0, MM_OP_B = 1, MM_OP_BT = 2, MM_OP_K = 3 };
int mm_operator_apply(mm_ctx *c, int op, const double *in, double *out);

/* Scalar-potential solve K u = b by preconditioned CG (the preconditioner
   and precision of the context's options: Jacobi or multigrid, FP64 or
   FP32-bulk), warm-started from u_inout (n_pot), until |r| <= rtol |b|.
   iters may be NULL. Returns MM_NOT_CONVERGED with the last iterate in
   u_inout when poisson_maxit iterations do not reach rtol. The solve uses the
   context's own potential buffers; on every exit, failures included, they are
   reset so that later evaluations see the context as before the call. */
int mm_poisson_solve(mm_ctx *c, const double *b, double *u_inout, double rtol, long *iters);

/* Measurement hook. enable = 1 times the scalar-potential CG iterations (the
   dominant work of an evaluation) with HIP events on the context's stream
   around every batch of iterations (the iterations run as replays of a
   captured graph); enable = 0 stops; enable = -1 resets the counters. out
   (may be NULL) receives {instance-iterations executed, seconds, algorithmic
   bytes of those iterations, potential rows of all instances}. Algorithmic
   bytes of one iteration: Jacobi CG (one kernel): the stored matrix (values +
   column indices, no padding) once plus 11 vector passes (read r, w, s, D^-1,
   p, x; write r, w, s, p, x); multigrid CG: the fine matrix three times, the
   fine prolongator and restriction once each, 17 fine vector passes, each
   coarse level's two fused operators and 3 vector passes, and the coarsest
   dense inverse. Values are 8 bytes in the FP64 mode and 4 bytes in the FP32
   inner solves and FP32-stored operators (the mixed multigrid form keeps its
   fine CG vectors at 8 bytes). */
int mm_profile(mm_ctx *c, int enable, double out[4]);

/* Per-launch timing of the field kernels of the energy evaluation (Sec. 2.2,
   eq. (energy): C m + B^T u with the projection of eqs. (proj), (nablaLF)),
   the divergence right-hand side B m (the scalar potential of Sec. 3.1), and
   the preconditioner product P v of Alg. 1 (eq. (precond)). With enable = 1,
   HIP events on the context's stream bracket every launch of the evaluation
   epilogue and of B m, and the first P v of each inner solve (later ones may
   return at once after an exit of Alg. 1); enable = 0 stops; -1 resets. out
   (9 doubles, may be NULL) receives, for the epilogue, B m and P v in turn:
   timed launches, seconds, algorithmic bytes of those launches. Algorithmic
   bytes: every stored operator entry (values + column index, no padding) once
   and every magnet-node vector the kernel reads or writes once (epilogue: C,
   B^T, m, L, G, g, lambda, and for a line-search trial x, d, g, lambda of the
   current state; B m: B, m, b; P v: C, m, lambda, v, P v, and g with all four
   terms of eq. (precond)). */
int mm_profile_kernels(mm_ctx *c, int enable, double out[9]);

/* Block shape of the scalar-potential kernels (the dominant work). Waves per
   block NW in {4, 8, 16} is one choice for the whole launch; SELL slices per
   wave in {1, 2, 4} is chosen per instance size bucket (bucket =
   floor(log2(n_pot / 4096)) clamped to 0..7). A block of an instance covers NW
   x slices-per-wave slices (up to the block cap below).
   MM_TUNE_DEFAULT: NW = 16, one slice per wave (the state after upload).
   MM_TUNE_MEASURE: times 32 CG iterations (best of 3, HIP events) of a
   synthetic solve of the whole batch (b = 1, u = 0, every instance active):
   for each NW one slices-per-wave value for all buckets, then each bucket's
   value in turn with the others fixed; the fastest NW wins.
   MM_TUNE_CACHE: as MEASURE, but a batch of the same composition (buckets and
   their instance counts) on the same device and precision (options of
   mm_set_opts) reuses the choice stored in the JSON file cache_path without
   timing; otherwise the new choice is appended to the file. Every choice is
   timed at 1, 2 and 4 times the default cap on blocks per instance (256, or
   one per 8192 rows for very large instances; at most 2048).
   The chosen shape stays fixed until the next mm_tune or upload, so a run is
   deterministic; another shape may change the rounding of the potential
   solves (another grouping of the reductions), never their tolerance. The
   warm start and the context's right-hand side are preserved. Outputs (may be
   NULL): waves_per_block, slices_per_wave (n_inst ints), block_mult (the
   multiplier of the block cap). */
enum { MM_TUNE_DEFAULT = 0, MM_TUNE_MEASURE = 1, MM_TUNE_CACHE = 2 };
int mm_tune(mm_ctx *c, int mode, const char *cache_path, int *waves_per_block, int *slices_per_wave,
            int *block_mult);

/* ---------------------------------------------------------------------------
   Batches of independent instances (parameter studies, Sec. 3.1 curves of
   many grains). A context may hold n_inst independent problems, each with
   its own mesh, materials, air box, Dirichlet boundary and reduced units
   (Ms_ref = max Ms of that instance). Every kernel launch serves all
   instances; each instance runs its own minimizer (Alg. 4) and walks its own
   field list. Results per instance equal those of a context holding that
   instance alone, up to the order of floating-point sums.

   Caller layout: per-instance arrays are concatenated in instance order.
   Magnetizations (and gradients) are sum_i n_mag_i x 3 doubles, instance i
   occupying the rows after those of instances 0..i-1, each ordered like
   mm_magnet_nodes. The single-instance calls above (mm_energy_grad,
   mm_precondition, mm_ncg_minimize, mm_demag_curve, mm_operator_apply,
   mm_poisson_solve, mm_magnet_nodes) need a context with one instance and
   return MM_ESTATE otherwise.
   --------------------------------------------------------------------------- */

/* Upload n_inst meshes with their materials (replaces mm_mesh_upload +
   mm_material_set). n_nodes, n_tets: per instance. xyz (sum n_nodes x 3),
   tets (sum n_tets x 4, node indices local to the instance), region, Ms, A,
   K1 (sum n_tets each) and axis (sum n_tets x 3, may be NULL when every K1 is
   0) are concatenated in instance order; meaning and units as in
   mm_mesh_upload / mm_material_set. Host pointers only. On failure the
   context holds no problem (MM_ESTATE until the next successful upload). */
int mm_batch_upload(mm_ctx *c, int n_inst, const long *n_nodes, const long *n_tets, const double *xyz,
                    const int *tets, const int *region, const double *Ms, const double *A, const double *K1,
                    const double *axis);

/* Number of instances of the context (0 before any problem is set). */
int mm_batch_size(const mm_ctx *c, int *n_inst);

/* Sizes and Ms_ref of instance inst (device_bytes: the whole context). */
int mm_batch_info(const mm_ctx *c, int inst, mm_info *info);

/* Magnet nodes of instance inst (local mesh-node ids, ascending). */
int mm_batch_magnet_nodes(const mm_ctx *c, int inst, long *n_mag, int *node_ids);

/* Energy and gradient of every instance at once (eq. (energy)), options of
   mm_set_opts. m: concatenated unit vectors; h_ext: n_inst x 3 (Tesla).
   E_tot, torque_max: n_inst; grad, gproj: concatenated like m. Every output
   may be NULL. */
int mm_batch_energy_grad(mm_ctx *c, const double *m, const double *h_ext, double *E_tot, double *grad,
                         double *gproj, double *torque_max);

/* Demagnetization curves of every instance (Sec. 3.1): instance i minimizes
   at h_list[i][k] (Tesla; h_list is n_inst x n x 3) for k = 0..n-1, each
   from its previous minimizer. m_inout: concatenated start / final states.
   m_avg (n_inst x n x 3), E_tot (n_inst x n) and st (n_inst x n) may be NULL.
   Returns the worst status over all instances and fields. */
int mm_batch_demag_curve(mm_ctx *c, double *m_inout, const double *h_list, long n, const mm_opts *o,
                         double *m_avg, double *E_tot, mm_stats *st);


/* ---------------------------------------------------------------------------
   Learned warm start and preconditioner scaling. Not part of the paper's
   method: an addition on top of it. A small graph network on the magnet nodes
   of a single-instance context proposes, for the step from the minimizer m_k
   at field h_k to the next field h_{k+1}, a tangent update dm (candidate
   start N(m_k + dm)) and a factor s_a in [1/4, 4] per node that multiplies
   the exchange diagonal used as Jacobi preconditioner inside the
   preconditioner's CG (the mm_precondition dscale). Alg. 4 always runs to the
   same stopping rule afterwards, and the candidate start is used only when
   its energy at h_{k+1} is lower than that of m_k (energy-raise fallback).

   Network (widths fixed): inputs X (n x 32 node features, below),
   standardized per column (mm_gnn_set_input_norm); h0 = SiLU(X W_in + b_in); three layers a = mean of h over the mesh neighbours, q
   = a We1 + ebar We2 (ebar: mean edge features (x_j - x_i)/l, |x_j - x_i|/l,
   l the mean edge length), t = SiLU([h | q] W1 + b1), h <- h + t W2 + b2;
   heads dm = P_m(h Wm + bm), s = clip(softplus(h Ws + bs) + 1/4, 1/4, 4).
   Neighbours: magnet nodes sharing a magnetic tet. The products with W_in,
   We1, W1, W2 (and their gradients) run on BF16 operands (inputs rounded to
   nearest even) with FP32 accumulation; everything else in FP32, losses and
   node reductions accumulated in FP64. Parameters: one flat vector of
   mm_gnn_param_count() values, matrices row-major [in][out], in the order
   W_in (32x64), b_in, then per layer We1 (64x64), We2 (4x64), W1 (128x64),
   b1, W2 (64x64), b2, then Wm (64x3), bm (3), Ws (64x1), bs (1).

   Node features (columns): 0-2 m; 3-5 h_{k+1}; 6-8 h_{k+1} - h_k (reduced
   units); 9-11 -(C m)_a / L_a; 12-14 -(B^T u)_a / L_a; 15-17 -g_a / L_a, all
   at (m, h_{k+1}) with the options of mm_set_opts; 18 D_a / mean D (exchange
   diagonal); 19 L_a / mean L; 20 deg_a / max deg; 21-31 zero.

   Objects: a graph belongs to the context it was created on and is invalid
   after that context's next upload or its destruction; destroy it before.
   --------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------
   Algebraic multigrid preconditioner of the scalar-potential CG (Sec. 3.1:
   the paper preconditions its CG with algebraic multigrid without fixing
   the variant). Smoothed aggregation on the assembled matrix K (free
   potential rows):
     strong neighbour j of row i: |a_ij| >= theta_l sqrt(|a_ii a_jj|),
       theta_l = 0.08 / 2^l;
     aggregates: pass 1 over the rows in order starts an aggregate at a free
       row whose strong neighbours are all free (with them); pass 2 adds each
       remaining row to the pass-1 aggregate of its strongest strong
       neighbour (weights within a relative 1e-12 are equal; lowest column);
     P = (I - omega D^-1 A) P0, P0 the aggregate indicator, omega = (4/3) /
       max_i sum_j |a_ij| / a_ii; next level P^T A P; coarsest level (at most
       2048 rows, or coarsening stalled, or 12 levels) solved by its dense
       inverse;
     cycle: V(1,1) with damped Jacobi (weight omega) from zero.
   Every instance has its own hierarchy, built on the host on first use (a
   solve with poisson_prec = MM_PREC_AMG or one of the calls below) and kept
   until the mesh changes; a batch runs all instances' cycles in shared
   launches. The calls below inspect or apply the hierarchy of a
   single-instance context (MM_ESTATE on a batch). */

/* Number of levels and, per level l < 12 (arrays of 12, may be NULL): rows,
   stored entries of the level operator and of the prolongator from level
   l + 1 (0 on the coarsest level); the host seconds of the build. */
int mm_amg_info(mm_ctx *c, int *n_levels, long *rows, long *nnz_A, long *nnz_P, double *setup_seconds);
/* Aggregate (coarse row) of every row of level `level` (not the coarsest):
   host array of rows[level] ints. */
int mm_amg_aggregates(mm_ctx *c, int level, int *agg);
/* Level operator (which = 0) or prolongator (which = 1, not on the coarsest
   level) of level `level` as host CSR: ptr (rows + 1 longs), col and val
   (nnz entries each, sizes from mm_amg_info); any of them may be NULL. */
int mm_amg_level_matrix(mm_ctx *c, int level, int which, long *ptr, int *col, double *val);
/* One cycle z = M r on the free potential rows (n_pot doubles, host or
   device pointers), in FP64 (precision MM_FP64) or in FP32 operators and
   vectors (MM_FP32_BULK; r rounded to FP32, z widened back). */
int mm_amg_apply(mm_ctx *c, const double *r, double *z, int precision);

typedef struct mm_gnn mm_gnn;
typedef struct mm_graph mm_graph;
enum { MM_LEARN_START = 1, MM_LEARN_SCALE = 2 };

long mm_gnn_param_count(void);
/* Network on the context's device; parameters zero until set. */
int mm_gnn_create(mm_ctx *c, mm_gnn **out);
int mm_gnn_destroy(mm_gnn *g);
/* Message of the network's last failed call. The network keeps the device,
   stream and allocator callbacks of its creating context, not that context's
   buffers: it may serve graphs of any context on the same device and outlives
   uploads to the creating context. */
const char *mm_gnn_last_error(const mm_gnn *g);
/* Parameters as doubles (host or device), kept as FP32 masters; setting
   them also resets the optimizer state. */
int mm_gnn_set_params(mm_gnn *g, const double *theta);

/* Arithmetic of the network's dense layers: MM_GNN_BF16 (the default: BF16
   operands on the matrix cores, FP32 accumulation) or MM_GNN_FP32 (a debug
   mode: the same products with FP32 operands on the vector units, for checking
   the forward and backward passes against an FP64 reference). */
enum { MM_GNN_BF16 = 0, MM_GNN_FP32 = 1 };
int mm_gnn_set_precision(mm_gnn *g, int precision);
int mm_gnn_get_params(mm_gnn *g, double *theta);
/* Input standardization applied in FP32 before the first layer: X_c <-
   (X_c - mu_c) / sd_c for the 32 feature columns (host arrays; sd > 0).
   Default mu = 0, sd = 1. */
int mm_gnn_set_input_norm(mm_gnn *g, const double *mu, const double *sd);

/* Graph of the magnet nodes of a single-instance context set with
   mm_mesh_upload + mm_material_set. */
int mm_graph_create(mm_ctx *c, mm_graph **out);
int mm_graph_destroy(mm_graph *gr);
int mm_graph_size(const mm_graph *gr, long *n_nodes, long *n_edges);

/* Node features for (m, h_prev -> h_next) (Tesla): one evaluation at
   (m, h_next). Kept in the graph; copied to X (n x 32 floats, host or device)
   when X != NULL. */
int mm_gnn_features(mm_graph *gr, const double *m, const double h_prev[3], const double h_next[3], float *X);

/* Forward pass: X (n x 32 floats, host or device; NULL = the graph's last
   features), m (n x 3) -> dm (n x 3), s (n); outputs may be NULL. */
int mm_gnn_forward(mm_gnn *g, mm_graph *gr, const float *X, const double *m, double *dm, double *s);

/* Loss inv_dm2 * sum_a L_a |dm_a - dm*_a|^2 / sum_a L_a + w_s * mean_a
   (log s_a - log s*_a)^2 (L: the lumped Ms-weighted volumes) and its gradient
   with respect to the parameters, which is kept for mm_gnn_adam and copied to
   grad (mm_gnn_param_count() doubles, host or device) when grad != NULL. */
int mm_gnn_loss_grad(mm_gnn *g, mm_graph *gr, const float *X, const double *m, const double *dm_target,
                     const double *s_target, double inv_dm2, double w_s, double *loss, double *grad);

/* One Adam step (bias-corrected) with the last gradient. */
int mm_gnn_adam(mm_gnn *g, double lr, double beta1, double beta2, double eps);

/* Training on the solver's own trajectories: `epochs` passes over n_samples
   samples, each pass in an order shuffled by SplitMix64 from `seed` (the same
   seed gives the same order and the same parameters), every sample one
   mm_gnn_loss_grad (graph[k], X[k], m[k], dm_target[k], s_target[k],
   inv_dm2[k], w_s) and one Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8).
   The per-sample arrays are device pointers (n x 32 floats, n x 3 and n
   doubles of that sample's graph); graphs may repeat. epoch_loss (epochs
   doubles, may be NULL) receives the mean loss of each pass. */
int mm_gnn_train(mm_gnn *g, long n_samples, mm_graph *const *graph, const float *const *X, const double *const *m,
                 const double *const *dm_target, const double *const *s_target, const double *inv_dm2, double w_s,
                 int epochs, double lr, unsigned long long seed, double *epoch_loss);

/* The network's parameters (FP32 masters) and input standardization written
   to / read from a file of this library's own format (a 24-byte header: magic,
   parameter count, feature count; then the parameters, the 32 means and the
   32 spreads as little-endian floats). mm_gnn_load checks the header and that
   every value is finite (spreads > 0), and clears the Adam state. */
int mm_gnn_save(mm_gnn *g, const char *path);
int mm_gnn_load(mm_gnn *g, const char *path);

/* Training targets of one field step k -> k+1 at the graph's magnet nodes
   (host or device vectors): dm_target = the step m_next - m projected on the
   tangent plane of m (n x 3), and s_target = 1 + t / D (n) with D the
   exchange diagonal (mm_jacobi_diag) and t the mean over the two directions
   normal to m of the magnetostatic Hessian's diagonal diag3 (n x 3, e.g. from
   mm_demag_diag): t = (sum_c diag3_c - sum_c m_c^2 diag3_c) / 2. */
int mm_gnn_targets(mm_graph *graph, const double *m, const double *m_next, const double *diag3, double *dm_target,
                   double *s_target);

/* Column sums and sums of squares (FP64, 32 each, host) of node features X
   (n x 32 floats, host or device): the input standardization's statistics. */
int mm_gnn_moments(mm_graph *graph, const float *X, double *sum, double *sumsq);

/* Exchange diagonal D (n_mag): the Jacobi preconditioner of Alg. 1 inside
   mm_precondition (before any dscale). */
int mm_jacobi_diag(mm_ctx *c, double *D);

/* Hutchinson estimate of the diagonal of the magnetostatic Hessian block
   B^T K^-1 B of instance 0: mean over the n_probe probe vectors z (n_probe x
   n_mag x 3, host or device) of z * (B^T K^-1 B z), each potential solved to
   |r| <= rtol |b| from zero. diag: n_mag x 3. The warm start is kept. */
int mm_demag_diag(mm_ctx *c, const double *probes, int n_probe, double rtol, double *diag);

/* Demagnetization curve (as mm_demag_curve, single instance) with the
   learned proposal at every field after the first: mode MM_LEARN_START uses
   the candidate start when it lowers the energy, MM_LEARN_SCALE uses the
   Jacobi factors for that field step's preconditioner solves; mode 0 is the
   plain method. accepted (n ints, may be NULL) marks the fields whose
   candidate start was taken. h_prev (3 doubles, Tesla, may be NULL) is the
   field at which m_inout is a minimizer when the call continues a curve: the
   first field then gets the proposal as well, so a curve run in several calls
   takes the same steps as one call. */
int mm_demag_curve_learned(mm_ctx *c, mm_gnn *net, mm_graph *graph, int mode, double *m_inout,
                           const double *h_prev, const double *h_list, long n, const mm_opts *o, double *m_avg,
                           double *E_tot, mm_stats *st, int *accepted);

#ifdef __cplusplus
}
#endif
#endif /* MMNCG_H */
