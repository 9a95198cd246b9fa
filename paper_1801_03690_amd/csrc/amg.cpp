// Host side of the algebraic-multigrid preconditioner of the scalar-potential
// CG (the paper preconditions its CG with algebraic multigrid, Sec. 3.1,
// without fixing the variant): the smoothed-aggregation hierarchy is built
// once per mesh from the assembled matrix (untimed like the assembly), copied
// to the device in FP64 and FP32, and handed to the kernels of amg.hip.
//
// Hierarchy (level l, matrix A with diagonal a_ii):
//   strength     j != i is strong when |a_ij| >= theta_l sqrt(|a_ii a_jj|),
//                theta_l = 0.08 / 2^l;
//   aggregates   pass 1 over the rows in order: a free row whose strong
//                neighbours are all free starts an aggregate with them;
//                pass 2: each row still free joins the pass-1 aggregate of
//                its strongest strong neighbour (weights within a relative
//                1e-12 count as equal; the lowest column wins);
//   prolongator  P = (I - omega D^-1 A) P0 with P0 the aggregate indicator,
//                omega = (4/3) / rho, rho = max_i sum_j |a_ij| / a_ii;
//   next level   A_c = P^T A P; stop at <= 2048 rows (dense inverse), when
//                coarsening stalls (more than 0.9 n aggregates) or at 12
//                levels.
// Entries that sum to exactly zero are dropped from every product.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "context.h"

namespace mmncg {

namespace {

constexpr double kTheta0 = 0.08;
constexpr int kCoarseMax = 2048;
constexpr double kStall = 0.9;
constexpr double kTie = 1e-12;
constexpr int kDenseLimit = 8192;  // largest coarsest level held as a dense inverse

struct Csr {
    int n = 0, ncols = 0;
    std::vector<int64_t> p;
    std::vector<int> j;
    std::vector<double> v;
    int64_t nnz() const { return p.empty() ? 0 : p[n]; }
};

Csr from_host(const HostCsr &h, int n) {
    Csr a;
    a.n = n;
    a.ncols = n;
    a.p.assign(n + 1, 0);
    for (int r = 0; r < n; ++r) {
        for (int64_t e = h.ptr[r]; e < h.ptr[r + 1]; ++e)
            if (h.val[e] != 0.0) {
                a.j.push_back(h.col[e]);
                a.v.push_back(h.val[e]);
            }
        a.p[r + 1] = (int64_t)a.j.size();
    }
    return a;
}

std::vector<double> diag(const Csr &a) {
    std::vector<double> d(a.n, 0.0);
    for (int r = 0; r < a.n; ++r)
        for (int64_t e = a.p[r]; e < a.p[r + 1]; ++e)
            if (a.j[e] == r) d[r] += a.v[e];
    return d;
}

// C = A B with a dense accumulator per row: for row i, every stored a_ik
// (columns ascending) times every stored b_kj; columns of C ascending, exact
// zeros dropped
Csr spmm(const Csr &A, const Csr &B) {
    Csr C;
    C.n = A.n;
    C.ncols = B.ncols;
    C.p.assign(A.n + 1, 0);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int> mark(B.ncols, -1), cols;
    for (int i = 0; i < A.n; ++i) {
        cols.clear();
        for (int64_t e = A.p[i]; e < A.p[i + 1]; ++e) {
            const int k = A.j[e];
            const double a = A.v[e];
            for (int64_t f = B.p[k]; f < B.p[k + 1]; ++f) {
                const int c = B.j[f];
                if (mark[c] != i) {
                    mark[c] = i;
                    acc[c] = 0.0;
                    cols.push_back(c);
                }
                acc[c] += a * B.v[f];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int c : cols)
            if (acc[c] != 0.0) {
                C.j.push_back(c);
                C.v.push_back(acc[c]);
            }
        C.p[i + 1] = (int64_t)C.j.size();
    }
    return C;
}

Csr transpose(const Csr &A) {
    Csr T;
    T.n = A.ncols;
    T.ncols = A.n;
    T.p.assign(T.n + 1, 0);
    for (int64_t e = 0; e < A.nnz(); ++e) T.p[A.j[e] + 1] += 1;
    for (int r = 0; r < T.n; ++r) T.p[r + 1] += T.p[r];
    T.j.resize(A.nnz());
    T.v.resize(A.nnz());
    std::vector<int64_t> pos(T.p.begin(), T.p.end() - 1);
    for (int r = 0; r < A.n; ++r)
        for (int64_t e = A.p[r]; e < A.p[r + 1]; ++e) {
            const int64_t q = pos[A.j[e]]++;
            T.j[q] = r;
            T.v[q] = A.v[e];
        }
    return T;
}

double gershgorin_rho(const Csr &A, const std::vector<double> &d) {
    double rho = 0.0;
    for (int r = 0; r < A.n; ++r) {
        double s = 0.0;
        for (int64_t e = A.p[r]; e < A.p[r + 1]; ++e) s += std::fabs(A.v[e]);
        rho = std::max(rho, s / d[r]);
    }
    return rho;
}

// aggregate of every row; returns the number of aggregates
int aggregate(const Csr &A, const std::vector<double> &d, double theta, std::vector<int> &agg) {
    const int n = A.n;
    auto strong = [&](int i, int64_t e) {
        const int j = A.j[e];
        return j != i && std::fabs(A.v[e]) >= theta * std::sqrt(std::fabs(d[i] * d[j]));
    };
    agg.assign(n, -1);
    int na = 0;
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (int64_t e = A.p[i]; e < A.p[i + 1] && free_nb; ++e)
            if (strong(i, e) && agg[A.j[e]] >= 0) free_nb = false;
        if (!free_nb) continue;
        agg[i] = na;
        for (int64_t e = A.p[i]; e < A.p[i + 1]; ++e)
            if (strong(i, e)) agg[A.j[e]] = na;
        ++na;
    }
    const std::vector<int> first = agg;
    for (int i = 0; i < n; ++i) {
        if (first[i] >= 0) continue;
        int best = -1;
        double bw = -1.0;
        for (int64_t e = A.p[i]; e < A.p[i + 1]; ++e) {
            if (!strong(i, e)) continue;
            const int j = A.j[e];
            const double w = std::fabs(A.v[e]);
            if (first[j] >= 0 && w > bw * (1.0 + kTie)) {
                best = j;
                bw = w;
            }
        }
        if (best < 0) throw ApiError{MM_EMESH, "multigrid: a row has no aggregated strong neighbour"};
        agg[i] = first[best];
    }
    return na;
}

// P = (I - omega D^-1 A) P0: entry (i, I) = [agg_i == I] + (-omega sum_{k in I} a_ik) / a_ii
Csr smoothed_prolongator(const Csr &A, const std::vector<double> &d, const std::vector<int> &agg, int na,
                         double omega) {
    Csr P0;
    P0.n = A.n;
    P0.ncols = na;
    P0.p.resize(A.n + 1);
    P0.j = agg;
    P0.v.assign(A.n, 1.0);
    for (int i = 0; i <= A.n; ++i) P0.p[i] = i;
    const Csr AP = spmm(A, P0);
    Csr P;
    P.n = A.n;
    P.ncols = na;
    P.p.assign(A.n + 1, 0);
    for (int i = 0; i < A.n; ++i) {
        bool own = false;
        for (int64_t e = AP.p[i]; e < AP.p[i + 1]; ++e) {
            const int c = AP.j[e];
            if (!own && c > agg[i]) {
                P.j.push_back(agg[i]);
                P.v.push_back(1.0);
                own = true;
            }
            double v = (-omega * AP.v[e]) / d[i];
            if (c == agg[i]) {
                v = 1.0 + v;
                own = true;
            }
            if (v != 0.0) {
                P.j.push_back(c);
                P.v.push_back(v);
            }
        }
        if (!own) {
            P.j.push_back(agg[i]);
            P.v.push_back(1.0);
        }
        P.p[i + 1] = (int64_t)P.j.size();
    }
    return P;
}

// inverse of a symmetric positive definite matrix through its Cholesky
// factor: A = L L^T, then L^-1 row by row (row i = (e_i - sum_{m<i} l_im
// row m) / l_ii) and A^-1 = L^-T L^-1 as a sum of outer products of the rows
// of L^-1; every inner loop runs over contiguous memory
std::vector<double> spd_inverse(const Csr &A) {
    // the sums may be reassociated (vectorized): this is set-up, and the
    // result is checked against the oracle's inverse to round-off
#pragma clang fp reassociate(on)
    const int n = A.n;
    std::vector<double> L((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r)
        for (int64_t e = A.p[r]; e < A.p[r + 1]; ++e) L[(size_t)r * n + A.j[e]] = A.v[e];
    for (int k = 0; k < n; ++k) {
        double *lk = &L[(size_t)k * n];
        double s = lk[k];
        for (int m = 0; m < k; ++m) s -= lk[m] * lk[m];
        if (!(s > 0.0)) throw ApiError{MM_EMESH, "multigrid: coarsest matrix is not positive definite"};
        const double lkk = std::sqrt(s);
        lk[k] = lkk;
        for (int i = k + 1; i < n; ++i) {
            double *li = &L[(size_t)i * n];
            double t = li[k];
            for (int m = 0; m < k; ++m) t -= li[m] * lk[m];
            li[k] = t / lkk;
        }
        for (int m = k + 1; m < n; ++m) lk[m] = 0.0;
    }
    std::vector<double> Li((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        double *ri = &Li[(size_t)i * n];
        const double *li = &L[(size_t)i * n];
        ri[i] = 1.0;
        for (int m = 0; m < i; ++m) {
            const double c = li[m];
            if (c == 0.0) continue;
            const double *rm = &Li[(size_t)m * n];
            for (int j = 0; j <= m; ++j) ri[j] -= c * rm[j];
        }
        const double d = 1.0 / li[i];
        for (int j = 0; j <= i; ++j) ri[j] *= d;
    }
    std::vector<double> inv((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        const double *rk = &Li[(size_t)k * n];
        for (int i = 0; i <= k; ++i) {
            const double a = rk[i];
            if (a == 0.0) continue;
            double *oi = &inv[(size_t)i * n];
            for (int j = i; j <= k; ++j) oi[j] += a * rk[j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) inv[(size_t)i * n + j] = inv[(size_t)j * n + i];
    return inv;
}

struct HostLevel {
    Csr A, P, R, AP;
    std::vector<double> d;
    double rho = 0, omega = 0, theta = 0;
    std::vector<int> agg;
    std::vector<double> Ainv;
};

// the hierarchy of one matrix, fine to coarse (the rules at the top)
std::vector<HostLevel> build_hierarchy(const HostCsr &K, int n) {
    std::vector<HostLevel> lv;
    Csr A = from_host(K, n);
    double theta = kTheta0;
    for (;;) {
        HostLevel L;
        L.d = diag(A);
        for (double x : L.d)
            if (!(x > 0.0)) throw ApiError{MM_EMESH, "multigrid: non-positive diagonal"};
        L.rho = gershgorin_rho(A, L.d);
        L.omega = (4.0 / 3.0) / L.rho;
        L.theta = theta;
        const bool last = A.n <= kCoarseMax || (int)lv.size() + 1 == kAmgMaxLevels;
        int na = 0;
        if (!last) {
            na = aggregate(A, L.d, theta, L.agg);
            if (na > kStall * A.n || na == 0) L.agg.clear();
        }
        if (L.agg.empty()) {
            if (A.n > kDenseLimit) throw ApiError{MM_EMESH, "multigrid coarsening stalled"};
            L.A = std::move(A);
            L.Ainv = spd_inverse(L.A);
            lv.push_back(std::move(L));
            break;
        }
        L.P = smoothed_prolongator(A, L.d, L.agg, na, L.omega);
        L.R = transpose(L.P);
        L.AP = spmm(A, L.P);
        Csr Ac = spmm(L.R, L.AP);
        L.A = std::move(A);
        lv.push_back(std::move(L));
        A = std::move(Ac);
        theta *= 0.5;
    }
    return lv;
}

int pad4(int n) { return (n + 3) / 4 * 4; }

// global CSR of nrows rows from instance blocks placed at increasing first
// rows; rows outside every block are empty
struct GBlock {
    int row0;
    const Csr *m;
    std::function<int(int)> col;
};
Csr concat(int nrows, int ncols, const std::vector<GBlock> &bl) {
    Csr G;
    G.n = nrows;
    G.ncols = ncols;
    G.p.assign(nrows + 1, 0);
    int r = 0;
    for (const GBlock &b : bl) {
        for (; r < b.row0; ++r) G.p[r + 1] = (int64_t)G.j.size();
        for (int i = 0; i < b.m->n; ++i, ++r) {
            for (int64_t e = b.m->p[i]; e < b.m->p[i + 1]; ++e) {
                G.j.push_back(b.col(b.m->j[e]));
                G.v.push_back(b.m->v[e]);
            }
            G.p[r + 1] = (int64_t)G.j.size();
        }
    }
    for (; r < nrows; ++r) G.p[r + 1] = (int64_t)G.j.size();
    return G;
}

}  // namespace

struct AmgState {
    std::vector<std::vector<HostLevel>> H;  // per instance, fine to coarse
    AmgLaunch<double> g64;
    AmgLaunch<float> g32;
    double setup_seconds = 0;
    std::vector<double> bytes[3];  // per instance: algorithmic bytes of one CG iteration (FP64, FP32, mixed)
};

namespace {

template <class T>
T *upload(mm_ctx *c, const T *h, size_t n) {
    T *d = dalloc_n<T>(c, std::max<size_t>(n, 1));
    if (n) HIPCHK(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return d;
}

template <class T>
T *upload_v(mm_ctx *c, const std::vector<T> &v) {
    return upload(c, v.data(), v.size());
}

std::vector<float> to32(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }

// lanes per row of a CSR product: the power of two (1..64) at or above the
// mean row length over kEntriesPerLane. Several entries per lane beat one: a
// wave then serves more rows, with fewer shuffle steps per row (measured on
// the 23.6M-row polycrystal's hierarchy: one CG iteration took 4,471 us with
// one entry per lane and at least 4 lanes per row, 3,872 with two entries,
// 3,522 with four and 3,605 with eight)
constexpr int kEntriesPerLane = 4;
int lanes_for(const Csr &a) {
    const double mean = a.n > 0 ? (double)a.nnz() / a.n : 1.0;
    int g = 1;
    while (g < 64 && g * kEntriesPerLane < mean) g *= 2;
    return g;
}

std::vector<int> ptr32(const Csr &a) {
    if (a.nnz() > 0x7fffffffLL) throw ApiError{MM_ENOMEM, "multigrid: a level has more than 2^31 entries"};
    return std::vector<int>(a.p.begin(), a.p.end());
}

// device copies of a CSR in both precisions
void up_csr(mm_ctx *c, const Csr &a, const int **p, const int **j, const double **v64, const int **p2,
            const int **j2, const float **v32) {
    const std::vector<int> pp = ptr32(a);
    *p = *p2 = upload_v(c, pp);
    *j = *j2 = upload_v(c, a.j);
    *v64 = upload_v(c, a.v);
    *v32 = upload_v(c, to32(a.v));
}

// Q = P - omega D^-1 (A P) of a level (rows of the level, columns of the next)
Csr smoothed_transfer(const HostLevel &H) {
    Csr Q;
    Q.n = H.P.n;
    Q.ncols = H.P.ncols;
    Q.p.assign(Q.n + 1, 0);
    for (int i = 0; i < Q.n; ++i) {
        int64_t e = H.P.p[i], f = H.AP.p[i];
        const int64_t e1 = H.P.p[i + 1], f1 = H.AP.p[i + 1];
        while (e < e1 || f < f1) {
            const int ce = e < e1 ? H.P.j[e] : 0x7fffffff, cf = f < f1 ? H.AP.j[f] : 0x7fffffff;
            const int col = std::min(ce, cf);
            double v = 0.0;
            if (ce == col) v += H.P.v[e++];
            if (cf == col) v -= H.omega * H.AP.v[f++] / H.d[i];
            if (v != 0.0) {
                Q.j.push_back(col);
                Q.v.push_back(v);
            }
        }
        Q.p[i + 1] = (int64_t)Q.j.size();
    }
    return Q;
}

// S = 2 omega D^-1 - omega^2 D^-1 A D^-1 of a level (the pattern of A)
Csr smoother_pair(const HostLevel &H) {
    const double w = H.omega;
    Csr S;
    S.n = H.A.n;
    S.ncols = H.A.n;
    S.p.assign(S.n + 1, 0);
    for (int i = 0; i < S.n; ++i) {
        for (int64_t e = H.A.p[i]; e < H.A.p[i + 1]; ++e) {
            const int j = H.A.j[e];
            double v = -(w * w) * H.A.v[e] / (H.d[i] * H.d[j]);
            if (j == i) v += 2.0 * w / H.d[i];
            if (v != 0.0) {
                S.j.push_back(j);
                S.v.push_back(v);
            }
        }
        S.p[i + 1] = (int64_t)S.j.size();
    }
    return S;
}

// rows of A in the order ord (row r of the result is row ord[r] of A)
Csr permute_rows(const Csr &A, const std::vector<int> &ord) {
    Csr P;
    P.n = A.n;
    P.ncols = A.ncols;
    P.p.assign(A.n + 1, 0);
    for (int r = 0; r < A.n; ++r) {
        const int a = ord[r];
        for (int64_t e = A.p[a]; e < A.p[a + 1]; ++e) {
            P.j.push_back(A.j[e]);
            P.v.push_back(A.v[e]);
        }
        P.p[r + 1] = (int64_t)P.j.size();
    }
    return P;
}

// [S | Q] as one CSR over the columns [0, ncols_b) + [yoff, ...)
Csr side_by_side(const Csr &S, const Csr &Q, int qoff) {
    Csr U;
    U.n = S.n;
    U.ncols = qoff + Q.ncols;
    U.p.assign(U.n + 1, 0);
    for (int i = 0; i < U.n; ++i) {
        for (int64_t e = S.p[i]; e < S.p[i + 1]; ++e) {
            U.j.push_back(S.j[e]);
            U.v.push_back(S.v[e]);
        }
        for (int64_t e = Q.p[i]; e < Q.p[i + 1]; ++e) {
            U.j.push_back(qoff + Q.j[e]);
            U.v.push_back(Q.v[e]);
        }
        U.p[i + 1] = (int64_t)U.j.size();
    }
    return U;
}

}  // namespace

void amg_release(mm_ctx *c) {
    delete c->amg;
    c->amg = nullptr;
}

// Builds the hierarchy of every instance once per mesh and lays the levels of
// all instances side by side on the device (a batch shares every launch of
// the cycle, as it shares those of the Jacobi CG).
AmgState *amg_get(mm_ctx *c) {
    if (c->amg) return c->amg;
    const int ni = c->ninst;
    if (ni < 1 || (int)c->hostK.size() != ni) throw ApiError{MM_ESTATE, "no host copy of the scalar-potential matrix"};
    const double t0 = now_s();
    std::unique_ptr<AmgState> S(new AmgState());
    int nlev = 1;
    for (int i = 0; i < ni; ++i) {
        S->H.push_back(build_hierarchy(c->hostK[i], c->inst[i].n_pot));
        nlev = std::max(nlev, (int)S->H[i].size());
    }
    if (ni > 1)
        for (int i = 0; i < ni; ++i)
            if (S->H[i].size() < 2)
                throw ApiError{MM_ESTATE, "multigrid batches need every instance above 2048 free potential nodes"};
    // row offsets of every instance's block on every level
    std::vector<std::vector<int>> off(nlev, std::vector<int>(ni, -1));
    std::vector<int> N(nlev, 0);
    N[0] = std::max(c->rows_p, 1);
    for (int i = 0; i < ni; ++i) off[0][i] = c->inst[i].pot_off;
    for (int l = 1; l < nlev; ++l)
        for (int i = 0; i < ni; ++i)
            if ((int)S->H[i].size() > l) {
                off[l][i] = N[l];
                N[l] += pad4(S->H[i][l].A.n);
            }
    auto L_of = [&](int i) { return (int)S->H[i].size() - 1; };
    AmgLaunch<double> &D = S->g64;
    AmgLaunch<float> &F = S->g32;
    D.nlev = F.nlev = nlev;
    D.single = F.single = ni == 1;
    // instance of every row of every level (-1: padding)
    for (int l = 0; l < nlev; ++l) {
        std::vector<int> iof(N[l], -1);
        for (int i = 0; i < ni; ++i) {
            if (off[l][i] < 0) continue;
            const int n = l == 0 ? c->inst[i].n_pot : S->H[i][l].A.n;
            for (int r = 0; r < n; ++r) iof[off[l][i] + r] = i;
        }
        D.lv[l].iof = F.lv[l].iof = upload_v(c, iof);
    }
    auto vec2 = [&](size_t n, double **d, float **f) {
        n = std::max<size_t>(n, 1);
        *d = dalloc_n<double>(c, n);
        *f = dalloc_n<float>(c, n);
        HIPCHK(hipMemsetAsync(*d, 0, n * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(*f, 0, n * sizeof(float), c->stream));
    };
    // per instance fine smoothing weight; level 0 work vectors
    {
        std::vector<double> om(ni), wd(N[0], 0.0);
        for (int i = 0; i < ni; ++i) {
            // level 0 lives on the device rows (the locality order of the
            // potential rows); the hierarchy itself is in free-node numbering
            const HostLevel &H0 = S->H[i][0];
            const std::vector<int> &ord = c->inst[i].pot_order;
            om[i] = H0.omega;
            for (int r = 0; r < H0.A.n; ++r) wd[off[0][i] + r] = H0.omega / H0.d[ord[r]];
        }
        D.omega = upload_v(c, om);
        F.omega = upload_v(c, to32(om));
        D.lv[0].wd = upload_v(c, wd);
        F.lv[0].wd = upload_v(c, to32(wd));
        D.lv[0].n = F.lv[0].n = N[0];
        vec2(N[0], &D.lv[0].t, &F.lv[0].t);
        vec2(N[0], &D.lv[0].z, &F.lv[0].z);
        vec2(N[0], &D.lv[0].b, &F.lv[0].b);  // staging of mm_amg_apply
        vec2(N[0], &D.lv[0].y, &F.lv[0].y);
    }
    // level 0 transfer
    if (nlev > 1) {
        std::vector<GBlock> bl;
        std::vector<Csr> Pd(ni);
        for (int i = 0; i < ni; ++i) {
            const int c0 = off[1][i];
            Pd[i] = permute_rows(S->H[i][0].P, c->inst[i].pot_order);
            bl.push_back(GBlock{off[0][i], &Pd[i], [c0](int j) { return c0 + j; }});
        }
        const Csr P = concat(N[0], N[1], bl);
        const Csr R = transpose(P);
        up_csr(c, P, &D.lv[0].Pp, &D.lv[0].Pj, &D.lv[0].Pv, &F.lv[0].Pp, &F.lv[0].Pj, &F.lv[0].Pv);
        up_csr(c, R, &D.lv[0].Rp, &D.lv[0].Rj, &D.lv[0].Rv, &F.lv[0].Rp, &F.lv[0].Rj, &F.lv[0].Rv);
        D.lv[0].gP = F.lv[0].gP = lanes_for(P);
        D.lv[0].gR = F.lv[0].gR = lanes_for(R);
    }
    // coarse levels: right-hand sides and results, fused operators, dense solves
    for (int l = 1; l < nlev; ++l) {
        AmgLevel<double> &d = D.lv[l];
        AmgLevel<float> &f = F.lv[l];
        d.n = f.n = N[l];
        double *b64;
        float *b32;
        const size_t nb = (size_t)N[l] + (l + 1 < nlev ? N[l + 1] : 0) + 4;
        vec2(nb, &b64, &b32);
        d.b = b64;
        f.b = b32;
        if (l + 1 < nlev) {
            D.lv[l + 1].y = b64 + N[l];
            F.lv[l + 1].y = b32 + N[l];
        }
        if (l == 1) vec2((size_t)N[1], &d.y, &f.y);
        if (l + 1 < nlev) {
            std::vector<Csr> Q(ni), Dn(ni), U(ni);
            std::vector<GBlock> bd, bu;
            for (int i = 0; i < ni; ++i) {
                if (L_of(i) <= l) continue;  // this instance ends on this level or above
                const HostLevel &H = S->H[i][l];
                Q[i] = smoothed_transfer(H);
                Dn[i] = transpose(Q[i]);
                U[i] = side_by_side(smoother_pair(H), Q[i], H.A.n);
                const int cb = off[l][i], cy = N[l] + off[l + 1][i], n_l = H.A.n;
                bd.push_back(GBlock{off[l + 1][i], &Dn[i], [cb](int j) { return cb + j; }});
                bu.push_back(GBlock{off[l][i], &U[i], [cb, cy, n_l](int j) { return j < n_l ? cb + j : cy + (j - n_l); }});
            }
            const Csr Dg = concat(N[l + 1], N[l], bd);
            const Csr Ug = concat(N[l], N[l] + N[l + 1], bu);
            up_csr(c, Dg, &d.Dp, &d.Dj, &d.Dv, &f.Dp, &f.Dj, &f.Dv);
            up_csr(c, Ug, &d.Up, &d.Uj, &d.Uv, &f.Up, &f.Uj, &f.Uv);
            d.gD = f.gD = lanes_for(Dg);
            d.gU = f.gU = lanes_for(Ug);
        }
    }
    // dense tables: the instances whose coarsest level is l
    for (int l = 0; l < nlev; ++l) {
        std::vector<int> dinst, drow0, dn, dld, dboff, dwho;
        std::vector<int64_t> daoff;
        std::vector<double> inv;
        int rows = 0;
        for (int i = 0; i < ni; ++i) {
            if (L_of(i) != l) continue;
            const HostLevel &H = S->H[i][l];
            const int n = H.A.n, ld = pad4(n), k = (int)dn.size();
            drow0.push_back(rows);
            dn.push_back(n);
            dld.push_back(ld);
            daoff.push_back((int64_t)inv.size());
            dboff.push_back(l == 0 ? 0 : off[l][i]);
            dwho.push_back(i);
            // a single-level hierarchy works on the device rows of level 0
            std::vector<int> ord(n);
            for (int r = 0; r < n; ++r) ord[r] = l == 0 ? c->inst[i].pot_order[r] : r;
            for (int r = 0; r < n; ++r) {
                dinst.push_back(k);
                const size_t at = inv.size();
                inv.resize(at + ld, 0.0);
                const double *row = H.Ainv.data() + (size_t)ord[r] * n;
                for (int q = 0; q < n; ++q) inv[at + q] = row[ord[q]];
            }
            rows += n;
        }
        if (rows == 0) continue;
        const int *di = upload_v(c, dinst), *r0 = upload_v(c, drow0), *nn = upload_v(c, dn), *lds = upload_v(c, dld),
                  *bo = upload_v(c, dboff), *wh = upload_v(c, dwho);
        const int64_t *ao = upload_v(c, daoff);
        D.lv[l].ndense = F.lv[l].ndense = rows;
        D.lv[l].dinst = F.lv[l].dinst = di;
        D.lv[l].drow0 = F.lv[l].drow0 = r0;
        D.lv[l].dn = F.lv[l].dn = nn;
        D.lv[l].dld = F.lv[l].dld = lds;
        D.lv[l].dboff = F.lv[l].dboff = bo;
        D.lv[l].dwho = F.lv[l].dwho = wh;
        D.lv[l].daoff = F.lv[l].daoff = ao;
        D.lv[l].Ainv = upload_v(c, inv);
        F.lv[l].Ainv = upload_v(c, to32(inv));
    }
    D.u = dalloc_n<double>(c, N[0]);
    D.rf = dalloc_n<double>(c, N[0]);
    D.wf = dalloc_n<double>(c, N[0]);
    F.u = dalloc_n<float>(c, N[0]);
    HIPCHK(hipMemsetAsync(D.u, 0, (size_t)N[0] * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(D.rf, 0, (size_t)N[0] * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(D.wf, 0, (size_t)N[0] * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(F.u, 0, (size_t)N[0] * sizeof(float), c->stream));
    sync(c);
    // algorithmic bytes of one CG iteration per instance: the fine matrix
    // three times (the iteration, the post-smoothing, w = K u), P and R once
    // each and 18 vector passes on the fine level (one of them the plain copy
    // of r); the two fused operators and
    // 3 vector passes on each further level; the dense inverse of the coarsest
    for (int k = 0; k < 3; ++k) S->bytes[k].assign(ni, 0.0);
    for (int i = 0; i < ni; ++i) {
        const std::vector<HostLevel> &Hi = S->H[i];
        const int L = L_of(i);
        for (int k = 0; k < 2; ++k) {
            const double v = k ? 4.0 : 8.0;
            double by = 0;
            for (int l = 0; l <= L; ++l) {
                const HostLevel &H = Hi[l];
                const double n = (double)H.A.n;
                if (l == L) {
                    by += n * n * v + 2.0 * n * v;
                } else if (l == 0) {
                    by += 3.0 * (double)c->inst[i].nnz_K * (v + 4) + 2.0 * (double)H.P.nnz() * (v + 4) + 18.0 * n * v;
                } else {
                    // the fused operators: Q^T (nnz of AP, P) and [S | Q]
                    const double nq = (double)std::max(H.AP.nnz(), H.P.nnz());
                    by += (2.0 * nq + (double)H.A.nnz()) * (v + 4) + 3.0 * n * v;
                }
            }
            S->bytes[k][i] = by;
        }
        S->bytes[2][i] = S->bytes[1][i] + (L > 0 ? 18.0 * 4.0 * (double)Hi[0].A.n : 0.0);
    }
    for (auto &Hi : S->H)
        for (auto &H : Hi) H.AP = Csr();
    S->setup_seconds = now_s() - t0;
    c->amg = S.release();
    return c->amg;
}

const AmgLaunch<double> &amg_launch64(AmgState *s) { return s->g64; }
const AmgLaunch<float> &amg_launch32(AmgState *s) { return s->g32; }
const std::vector<double> &amg_bytes(AmgState *s, int form) { return s->bytes[form]; }

}  // namespace mmncg

using namespace mmncg;

extern "C" {

int mm_amg_info(mm_ctx *c, int *n_levels, long *rows, long *nnz_A, long *nnz_P, double *setup_seconds) {
    return guarded(c, [&] {
        require_single(c);
        if (!n_levels) throw ApiError{MM_EINVAL, "null n_levels"};
        AmgState *S = amg_get(c);
        const int nl = (int)S->H[0].size();
        *n_levels = nl;
        for (int l = 0; l < kAmgMaxLevels; ++l) {
            const bool in = l < nl;
            if (rows) rows[l] = in ? S->H[0][l].A.n : 0;
            if (nnz_A) nnz_A[l] = in ? (long)S->H[0][l].A.nnz() : 0;
            if (nnz_P) nnz_P[l] = in ? (long)S->H[0][l].P.nnz() : 0;
        }
        if (setup_seconds) *setup_seconds = S->setup_seconds;
        return MM_OK;
    });
}

int mm_amg_aggregates(mm_ctx *c, int level, int *agg) {
    return guarded(c, [&] {
        require_single(c);
        AmgState *S = amg_get(c);
        if (!agg || level < 0 || level + 1 >= (int)S->H[0].size())
            throw ApiError{MM_EINVAL, "level must have a coarser level below it"};
        std::memcpy(agg, S->H[0][level].agg.data(), S->H[0][level].agg.size() * sizeof(int));
        return MM_OK;
    });
}

int mm_amg_level_matrix(mm_ctx *c, int level, int which, long *ptr, int *col, double *val) {
    return guarded(c, [&] {
        require_single(c);
        AmgState *S = amg_get(c);
        if (level < 0 || level >= (int)S->H[0].size()) throw ApiError{MM_EINVAL, "no such level"};
        const HostLevel &H = S->H[0][level];
        const Csr *m = which == 0 ? &H.A : which == 1 ? &H.P : nullptr;
        if (!m || m->p.empty()) throw ApiError{MM_EINVAL, "which: 0 = level operator, 1 = prolongator (not on the coarsest level)"};
        if (ptr)
            for (int r = 0; r <= m->n; ++r) ptr[r] = (long)m->p[r];
        if (col) std::memcpy(col, m->j.data(), m->j.size() * sizeof(int));
        if (val) std::memcpy(val, m->v.data(), m->v.size() * sizeof(double));
        return MM_OK;
    });
}

int mm_amg_apply(mm_ctx *c, const double *r, double *z, int precision) {
    return guarded(c, [&] {
        require_single(c);
        if (!r || !z) throw ApiError{MM_EINVAL, "null vector"};
        if (precision != MM_FP64 && precision != MM_FP32_BULK) throw ApiError{MM_EINVAL, "unknown precision"};
        AmgState *S = amg_get(c);
        const int n = c->inst[0].n_pot;
        const PcgLaunch a = pcg_args(c);
        // the fine level's b and y are not used by the cycle: input and output staging
        double *r64 = S->g64.lv[0].b, *z64 = S->g64.lv[0].y;
        pot_in(c, r64, r, z64);
        if (precision == MM_FP64) {
            launch_amg_apply64(a, S->g64, r64, c->stream);
            pot_out(c, z, S->g64.u, z64);
        } else {
            float *r32 = S->g32.lv[0].b;
            launch_to_f32(n, r64, r32, c->stream);
            launch_amg_apply32(a, S->g32, r32, c->stream);
            gnn_f32_to_f64(n, S->g32.u, z64, c->stream);
            pot_out(c, z, z64, r64);
        }
        sync(c);
        return MM_OK;
    });
}

}  // extern "C"
