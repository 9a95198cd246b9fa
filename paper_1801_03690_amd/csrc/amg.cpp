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

}  // namespace

struct AmgState {
    std::vector<HostLevel> lv;
    AmgLaunch<double> g64;
    AmgLaunch<float> g32;
    double setup_seconds = 0;
    double bytes64 = 0, bytes32 = 0, bytesmix = 0;  // algorithmic bytes of one CG iteration
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

// lanes per row: the power of two at or above the mean row length, 4..64
int lanes_for(const Csr &a) {
    const double mean = a.n > 0 ? (double)a.nnz() / a.n : 1.0;
    int g = 4;
    while (g < 64 && g < mean) g *= 2;
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

}  // namespace

void amg_release(mm_ctx *c) {
    delete c->amg;
    c->amg = nullptr;
}

// builds the hierarchy of instance 0 (single-instance contexts) once per mesh
AmgState *amg_get(mm_ctx *c) {
    if (c->amg) return c->amg;
    if (c->ninst != 1) throw ApiError{MM_ESTATE, "the multigrid preconditioner needs a single-instance context"};
    if (c->hostK.nrows != c->inst[0].n_pot) throw ApiError{MM_ESTATE, "no host copy of the scalar-potential matrix"};
    const double t0 = now_s();
    std::unique_ptr<AmgState> S(new AmgState());
    Csr A = from_host(c->hostK, c->inst[0].n_pot);
    double theta = kTheta0;
    for (;;) {
        HostLevel L;
        L.d = diag(A);
        for (double x : L.d)
            if (!(x > 0.0)) throw ApiError{MM_EMESH, "multigrid: non-positive diagonal"};
        L.rho = gershgorin_rho(A, L.d);
        L.omega = (4.0 / 3.0) / L.rho;
        L.theta = theta;
        const bool last = A.n <= kCoarseMax || (int)S->lv.size() + 1 == kAmgMaxLevels;
        int na = 0;
        if (!last) {
            na = aggregate(A, L.d, theta, L.agg);
            if (na > kStall * A.n || na == 0) L.agg.clear();
        }
        if (L.agg.empty()) {
            if (A.n > kDenseLimit) throw ApiError{MM_EMESH, "multigrid coarsening stalled"};
            L.A = std::move(A);
            L.Ainv = spd_inverse(L.A);
            S->lv.push_back(std::move(L));
            break;
        }
        L.P = smoothed_prolongator(A, L.d, L.agg, na, L.omega);
        L.R = transpose(L.P);
        L.AP = spmm(A, L.P);
        Csr Ac = spmm(L.R, L.AP);
        L.A = std::move(A);
        S->lv.push_back(std::move(L));
        A = std::move(Ac);
        theta *= 0.5;
    }
    // device copies
    const int nl = (int)S->lv.size();
    const int L = nl - 1;
    S->g64.nlev = S->g32.nlev = nl;
    const size_t RP = std::max(c->rows_p, 1);
    double b64 = 0, b32 = 0;
    auto vec2 = [&](size_t n, double **d, float **f) {
        *d = dalloc_n<double>(c, std::max<size_t>(n, 1));
        *f = dalloc_n<float>(c, std::max<size_t>(n, 1));
        HIPCHK(hipMemsetAsync(*d, 0, std::max<size_t>(n, 1) * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(*f, 0, std::max<size_t>(n, 1) * sizeof(float), c->stream));
    };
    for (int l = 0; l < nl; ++l) {
        HostLevel &H = S->lv[l];
        AmgLevel<double> &D = S->g64.lv[l];
        AmgLevel<float> &F = S->g32.lv[l];
        D.n = F.n = H.A.n;
        D.omega = H.omega;
        F.omega = (float)H.omega;
        const double n = (double)H.A.n, nA = (double)(l == 0 ? c->inst[0].nnz_K : H.A.nnz());
        if (l == 0) {
            D.dinv = c->invDK;
            F.dinv = c->invDK32;
            vec2(RP, &D.t, &F.t);
            vec2(RP, &D.z, &F.z);
            vec2(RP, &D.b, &F.b);  // staging of mm_amg_apply
            vec2(RP, &D.y, &F.y);
            if (l < L) {
                up_csr(c, H.P, &D.Pp, &D.Pj, &D.Pv, &F.Pp, &F.Pj, &F.Pv);
                up_csr(c, H.R, &D.Rp, &D.Rj, &D.Rv, &F.Rp, &F.Rj, &F.Rv);
                D.gP = F.gP = lanes_for(H.P);
                D.gR = F.gR = lanes_for(H.R);
            }
        } else if (l < L) {
            // Q = P - omega D^-1 (A P); down = Q^T; up = [S | Q] with S =
            // 2 omega D^-1 - omega^2 D^-1 A D^-1
            const double w = H.omega;
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
                    if (cf == col) v -= w * H.AP.v[f++] / H.d[i];
                    if (v != 0.0) {
                        Q.j.push_back(col);
                        Q.v.push_back(v);
                    }
                }
                Q.p[i + 1] = (int64_t)Q.j.size();
            }
            const Csr Dn = transpose(Q);
            Csr U;
            U.n = H.A.n;
            U.ncols = H.A.n + Q.ncols;
            U.p.assign(U.n + 1, 0);
            for (int i = 0; i < U.n; ++i) {
                for (int64_t e = H.A.p[i]; e < H.A.p[i + 1]; ++e) {
                    const int j = H.A.j[e];
                    double v = -(w * w) * H.A.v[e] / (H.d[i] * H.d[j]);
                    if (j == i) v += 2.0 * w / H.d[i];
                    if (v != 0.0) {
                        U.j.push_back(j);
                        U.v.push_back(v);
                    }
                }
                for (int64_t e = Q.p[i]; e < Q.p[i + 1]; ++e) {
                    U.j.push_back(H.A.n + Q.j[e]);
                    U.v.push_back(Q.v[e]);
                }
                U.p[i + 1] = (int64_t)U.j.size();
            }
            up_csr(c, Dn, &D.Dp, &D.Dj, &D.Dv, &F.Dp, &F.Dj, &F.Dv);
            up_csr(c, U, &D.Up, &D.Uj, &D.Uv, &F.Up, &F.Uj, &F.Uv);
            D.gD = F.gD = lanes_for(Dn);
            D.gU = F.gU = lanes_for(U);
            // [b_l; y_{l+1}] in one array
            const size_t nb = (size_t)H.A.n + S->lv[l + 1].A.n;
            double *d64;
            float *d32;
            vec2(nb, &d64, &d32);
            D.b = d64;
            F.b = d32;
            S->g64.lv[l + 1].y = d64 + H.A.n;
            S->g32.lv[l + 1].y = d32 + H.A.n;
            if (l == 1) vec2((size_t)H.A.n, &D.y, &F.y);
            for (int k = 0; k < 2; ++k) {
                const double v = k ? 4.0 : 8.0;
                (k ? b32 : b64) += (double)(Dn.nnz() + U.nnz()) * (v + 4) + 3.0 * n * v;
            }
        }
        if (l == L) {
            // rows padded to a multiple of 4 values (16 bytes in FP32, 32 in FP64)
            const int ld = (H.A.n + 3) / 4 * 4;
            std::vector<double> pad((size_t)H.A.n * ld, 0.0);
            for (int i = 0; i < H.A.n; ++i)
                std::copy(H.Ainv.begin() + (size_t)i * H.A.n, H.Ainv.begin() + (size_t)(i + 1) * H.A.n,
                          pad.begin() + (size_t)i * ld);
            D.Ainv = upload_v(c, pad);
            F.Ainv = upload_v(c, to32(pad));
            D.ld = F.ld = ld;
            if (l > 0) {
                // the right-hand side is read 16 bytes at a time up to ld (zero padding)
                vec2((size_t)ld, &D.b, &F.b);
                if (l == 1) vec2((size_t)H.A.n, &D.y, &F.y);
            }
            for (int k = 0; k < 2; ++k) {
                const double v = k ? 4.0 : 8.0;
                (k ? b32 : b64) += n * n * v + 2.0 * n * v;
            }
        }
        if (l == 0 && l < L) {
            // fine level: K three times (the iteration, the post-smoothing,
            // w = K u), R and P once each, and 17 vector passes
            const double nP = (double)H.P.nnz();
            for (int k = 0; k < 2; ++k) {
                const double v = k ? 4.0 : 8.0;
                (k ? b32 : b64) += 3.0 * nA * (v + 4) + 2.0 * nP * (v + 4) + 17.0 * n * v;
            }
        }
        H.AP = Csr();
    }
    S->g64.u = dalloc_n<double>(c, RP);
    S->g32.u = dalloc_n<float>(c, RP);
    HIPCHK(hipMemsetAsync(S->g64.u, 0, RP * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(S->g32.u, 0, RP * sizeof(float), c->stream));
    sync(c);
    S->bytes64 = b64;
    S->bytes32 = b32;
    // mixed form: FP32 matrices and cycle, FP64 CG vectors on the fine level
    // (the 17 fine vector passes at 8 instead of 4 bytes)
    S->bytesmix = b32 + (nl > 1 ? 17.0 * 4.0 * (double)S->lv[0].A.n : 0.0);
    S->setup_seconds = now_s() - t0;
    c->amg = S.release();
    return c->amg;
}

const AmgLaunch<double> &amg_launch64(AmgState *s) { return s->g64; }
const AmgLaunch<float> &amg_launch32(AmgState *s) { return s->g32; }
double amg_bytes(AmgState *s, int form) { return form == 2 ? s->bytesmix : form == 1 ? s->bytes32 : s->bytes64; }

}  // namespace mmncg

using namespace mmncg;

extern "C" {

int mm_amg_info(mm_ctx *c, int *n_levels, long *rows, long *nnz_A, long *nnz_P, double *setup_seconds) {
    return guarded(c, [&] {
        require_single(c);
        if (!n_levels) throw ApiError{MM_EINVAL, "null n_levels"};
        AmgState *S = amg_get(c);
        const int nl = (int)S->lv.size();
        *n_levels = nl;
        for (int l = 0; l < kAmgMaxLevels; ++l) {
            const bool in = l < nl;
            if (rows) rows[l] = in ? S->lv[l].A.n : 0;
            if (nnz_A) nnz_A[l] = in ? (long)S->lv[l].A.nnz() : 0;
            if (nnz_P) nnz_P[l] = in ? (long)S->lv[l].P.nnz() : 0;
        }
        if (setup_seconds) *setup_seconds = S->setup_seconds;
        return MM_OK;
    });
}

int mm_amg_aggregates(mm_ctx *c, int level, int *agg) {
    return guarded(c, [&] {
        require_single(c);
        AmgState *S = amg_get(c);
        if (!agg || level < 0 || level + 1 >= (int)S->lv.size())
            throw ApiError{MM_EINVAL, "level must have a coarser level below it"};
        std::memcpy(agg, S->lv[level].agg.data(), S->lv[level].agg.size() * sizeof(int));
        return MM_OK;
    });
}

int mm_amg_level_matrix(mm_ctx *c, int level, int which, long *ptr, int *col, double *val) {
    return guarded(c, [&] {
        require_single(c);
        AmgState *S = amg_get(c);
        if (level < 0 || level >= (int)S->lv.size()) throw ApiError{MM_EINVAL, "no such level"};
        const HostLevel &H = S->lv[level];
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
        copy_in(c, r64, r, n);
        if (precision == MM_FP64) {
            launch_amg_apply64(a, S->g64, r64, c->stream);
            copy_out(c, z, S->g64.u, n);
        } else {
            float *r32 = S->g32.lv[0].b;
            launch_to_f32(n, r64, r32, c->stream);
            launch_amg_apply32(a, S->g32, r32, c->stream);
            gnn_f32_to_f64(n, S->g32.u, z64, c->stream);
            copy_out(c, z, z64, n);
        }
        sync(c);
        return MM_OK;
    });
}

}  // extern "C"
