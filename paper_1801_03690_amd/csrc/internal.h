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
constexpr int kMaxPartials = 1024;  // upper bound on blocks of a reducing kernel

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
};

// Builds every operator from the mesh and per-tet SI materials. Returns an
// error message (empty on success).
std::string assemble(const double *xyz, long n_nodes, const int *tets, long n_tets, const int *region,
                     const double *Ms, const double *A, const double *K1, const double *axis,
                     Assembly &out);

// ---------------------------------------------------------------------------
// kernel launchers (defined in kernels.hip); all enqueue on `s`. Partial
// buffers hold NQ slots of kMaxPartials doubles (slot q at q * kMaxPartials).
// ---------------------------------------------------------------------------
int grid_for_rows(int nrows);   // blocks of a row kernel (multiple of 8 when >= 8, <= kMaxPartials)
unsigned eval_max_mask();
constexpr int kEvalParts = 10;  // Eloc, Ezee, Edemag, dF, dphi, |g|^2, max torque, max|g|_inf, max|m-x0|_inf, max|m|_inf

void launch_spmv_block6(const Sell &C, const double *x, double *y, bool fp32, hipStream_t s);
void launch_spmv_scalar(const Sell &A, const double *x, double *y, bool fp32, hipStream_t s);
void launch_spmv_scalar3(const Sell &A, const double *x, double *y, bool fp32, hipStream_t s);
void launch_bmul(const Sell &B, const double *m, double *b, bool fp32, hipStream_t s);
void launch_btmul(const Sell &Bt, const double *u, double *gout, bool fp32, hipStream_t s);

// Poisson CG state (device memory): start scalars, tolerance, stop flag and
// iteration count
struct PcgState {
    double rz, beta, alpha, tol2, bb, rr;
    int done, iters, zero_u, pad;
};
// partial buffer of the Poisson kernels (8 slots of kMaxPartials doubles)
constexpr int kPcgPartDoubles = 8 * kMaxPartials;

void launch_pcg_init64(const Sell &K, const double *b, const double *u, double *r, const double *invD, double rtol2,
                       PcgState *st, double *part, bool fp32, hipStream_t s);
void launch_residual64(const Sell &K, const double *b, const double *u, double *r, PcgState *st, double *part,
                       hipStream_t s);
void launch_pcg_init32(int n, const double *r64, double scale, float *x, float *r, const float *invD, double inner2,
                       PcgState *st, double *part, hipStream_t s);
void launch_pcg_iter64(const Sell &K, double *u, double *r, double *p_old, double *p_new, double *q,
                       const double *invD, PcgState *st, int phase_a, int odd, double *part, hipStream_t s);
void launch_pcg_iter32(const Sell &K, float *x, float *r, float *p_old, float *p_new, float *q, const float *invD,
                       PcgState *st, int phase_a, int odd, double *part, hipStream_t s);
void launch_add_correction(int n, double *u, const float *x, double scale, hipStream_t s);

void launch_eval_epilogue(const Sell &C, const Sell &S, const Sell &Bt, int cmode, int use_demag, const double *m,
                          const double *u, const double *L, const double h[3], double *G, double *g, double *lam,
                          const double *x0, const double *g0, const double *lam0, const double *d, double alpha,
                          double *part, bool fp32, hipStream_t s);
void launch_trial(int n, const double *x0, const double *d, double alpha, double *xt, hipStream_t s);
void launch_finalize(const double *part, int nblk, int nslot, unsigned is_max, double *out, hipStream_t s);

void launch_prec_init(int n, const double *gv, const double *invDex, const double *dscale, double *y, double *r,
                      double *p, double *part, int *flags, hipStream_t s);
void launch_prec_apply(const Sell &C, const double *m, const double *lam, const double *p, double *q, double *part,
                       const int *flags, int phase, bool fp32, hipStream_t s);
void launch_prec_update(int n, int j, const double *gv, const double *invDex, const double *dscale, double *y,
                        double *r, const double *p, const double *q, const double *part_pq, const double *part_rz_prev,
                        int rz_slot, double *part_out, int *flags, int phase, hipStream_t s);
void launch_prec_pupdate(int n, const double *invDex, const double *dscale, double *p, const double *r,
                         const double *part_init, const double *part_new, const double *part_old, int old_slot,
                         int *flags, int phase, hipStream_t s);

constexpr int kDirParts = 6;
void launch_dir_dots(int n, const double *g1, const double *g0, const double *y1, const double *d, double *part,
                     int *nblk_out, hipStream_t s);
void launch_dir_update(int n, const double *g1, const double *y1, double *d, const double *part_dots, int nblk_dots,
                       int first, double *part_out, int *info, hipStream_t s);

void launch_energy_split(const Sell &S, const double *m, double *part, bool fp32, hipStream_t s);
void launch_mavg(int n, const double *m, const double *L, double *part, hipStream_t s);
void launch_lambda(int n, const double *m, const double *G, double *lam, hipStream_t s);
void launch_to_f32(int64_t n, const double *x, float *y, hipStream_t s);

}  // namespace mmncg
