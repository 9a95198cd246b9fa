// Host-side finite-element assembly: a precomputation, and like the paper's
// timings (Sec. 3.1) every timing here leaves it out.
//
// P1 tetrahedra. In reduced units (length 1 nm, magnetization Ms_ref = max Ms,
// energy mu0 Ms_ref^2 nm^3) the operators of the energy of Sec. 2.2, eq. (energy), are:
//   exchange     C_A = 2 S (x) I3,  S_ab = sum_e a_e V_e grad(phi_a).grad(phi_b),  a_e = A_e/(mu0 Ms_ref^2 nm^2)
//   anisotropy   C_K,ab = -2 sum_e k_e M^e_ab u_e u_e^T,  M^e_ab = V_e (1 + delta_ab) / 20 (consistent P1 mass)
//   Zeeman       M = diag(L) (x) I3,  L_a = sum_{e ni a} ms_e V_e / 4
//   stray field  K_jk = sum_e V_e grad(phi_j).grad(phi_k) over all tets (Dirichlet rows/columns removed),
//                b = B m with B_ja = sum_{e ni j,a; magnet} ms_e (V_e/4) grad(phi_j^e)  (3-vector),
//                dE_d/dm_a = sum_j B_ja u_j  (B^T)
// Rows are built node-centrically (each row gathers over the tets incident to its
// node), in parallel over rows, so every value is a fixed-order sum.
// Entries that cancel exactly in exact arithmetic (the P1 Laplacian on face and
// body diagonals of a Kuhn cell) come out as round-off; they are dropped when
// below 1e-12 of the row's diagonal.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.h"

namespace mmncg {
namespace {

constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kDropRel = 1e-12;

template <class F>
void parallel_rows(long n, F &&f) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 4096) nt = 1;
    std::vector<std::thread> th;
    long chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        long lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([lo, hi, &f] {
            for (long i = lo; i < hi; ++i) f(i);
        });
    }
    for (auto &x : th) x.join();
}

struct Geo {
    std::vector<double> vol;     // V_e
    std::vector<double> grad;    // 12 per tet
};

// grad(lambda_i) = n_i / ((x_i - x_f) . n_i), n_i normal of the face opposite vertex i
bool tet_geometry(const double *xyz, const int *t, double *vol, double *gr) {
    const double *x[4];
    for (int i = 0; i < 4; ++i) x[i] = xyz + 3 * (long)t[i];
    static const int opp[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    double e1[3], e2[3], e3[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[1][d] - x[0][d];
        e2[d] = x[2][d] - x[0][d];
        e3[d] = x[3][d] - x[0][d];
    }
    double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                 e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    *vol = std::fabs(det) / 6.0;
    for (int i = 0; i < 4; ++i) {
        const double *a = x[opp[i][0]], *b = x[opp[i][1]], *c = x[opp[i][2]];
        double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        double h = (x[i][0] - a[0]) * n[0] + (x[i][1] - a[1]) * n[1] + (x[i][2] - a[2]) * n[2];
        for (int d = 0; d < 3; ++d) gr[3 * i + d] = n[d] / h;
    }
    return true;
}

// small row accumulator: columns with vw values each
struct RowAcc {
    std::vector<int> col;
    std::vector<double> val;
    int vw;
    explicit RowAcc(int w) : vw(w) {}
    void clear() { col.clear(); val.clear(); }
    double *at(int c) {
        for (size_t i = 0; i < col.size(); ++i)
            if (col[i] == c) return &val[i * vw];
        col.push_back(c);
        val.resize(val.size() + vw, 0.0);
        return &val[(col.size() - 1) * vw];
    }
    // sort by column and return permutation-applied copies
    void sorted(std::vector<int> &c, std::vector<double> &v) const {
        std::vector<int> idx(col.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        std::sort(idx.begin(), idx.end(), [&](int a, int b) { return col[a] < col[b]; });
        c.resize(idx.size());
        v.resize(idx.size() * vw);
        for (size_t i = 0; i < idx.size(); ++i) {
            c[i] = col[idx[i]];
            for (int k = 0; k < vw; ++k) v[i * vw + k] = val[idx[i] * vw + k];
        }
    }
};

// Two-pass parallel CSR build: fill(row, acc) populates a RowAcc; keep(acc, i) filters entries.
template <class Fill, class Keep>
void build_csr(int nrows, int vw, HostCsr &out, Fill &&fill, Keep &&keep) {
    out.nrows = nrows;
    out.vw = vw;
    out.ptr.assign(nrows + 1, 0);
    std::vector<int> cnt(nrows, 0);
    parallel_rows(nrows, [&](long r) {
        thread_local RowAcc acc(1);
        acc.vw = vw;
        acc.clear();
        fill((int)r, acc);
        int k = 0;
        for (size_t i = 0; i < acc.col.size(); ++i) k += keep((int)r, acc, (int)i) ? 1 : 0;
        cnt[r] = k;
    });
    for (int r = 0; r < nrows; ++r) out.ptr[r + 1] = out.ptr[r] + cnt[r];
    out.col.assign(out.ptr[nrows], 0);
    out.val.assign(out.ptr[nrows] * vw, 0.0);
    parallel_rows(nrows, [&](long r) {
        thread_local RowAcc acc(1);
        acc.vw = vw;
        acc.clear();
        fill((int)r, acc);
        RowAcc kept(vw);
        for (size_t i = 0; i < acc.col.size(); ++i)
            if (keep((int)r, acc, (int)i)) {
                double *d = kept.at(acc.col[i]);
                for (int k = 0; k < vw; ++k) d[k] = acc.val[i * vw + k];
            }
        std::vector<int> c;
        std::vector<double> v;
        kept.sorted(c, v);
        int64_t o = out.ptr[r];
        for (size_t i = 0; i < c.size(); ++i) {
            out.col[o + i] = c[i];
            for (int k = 0; k < vw; ++k) out.val[(o + i) * vw + k] = v[i * vw + k];
        }
    });
}

}  // namespace

std::vector<int> locality_order(const double *xyz, const std::vector<int> &node_of_free) {
    const int n = (int)node_of_free.size();
    std::vector<int> order(n);
    for (int r = 0; r < n; ++r) order[r] = r;
    if (n < 8192) return order;
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int r = 0; r < n; ++r)
        for (int d = 0; d < 3; ++d) {
            const double x = xyz[3 * (long)node_of_free[r] + d];
            lo[d] = std::min(lo[d], x);
            hi[d] = std::max(hi[d], x);
        }
    double ext[3], vol = 1.0, emax = 0.0;
    for (int d = 0; d < 3; ++d) emax = std::max(emax, hi[d] - lo[d]);
    if (!(emax > 0.0)) return order;
    for (int d = 0; d < 3; ++d) {
        ext[d] = std::max(hi[d] - lo[d], 1e-9 * emax);
        vol *= ext[d];
    }
    const double side = std::cbrt(vol * 4096.0 / n);
    long nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = std::max(1L, (long)std::ceil(ext[d] / side));
    std::vector<long> key(n);
    for (int r = 0; r < n; ++r) {
        long t[3];
        for (int d = 0; d < 3; ++d) {
            const double x = xyz[3 * (long)node_of_free[r] + d];
            t[d] = std::min(nt[d] - 1, (long)((x - lo[d]) / side));
        }
        key[r] = t[0] + nt[0] * (t[1] + nt[1] * t[2]);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    return order;
}

std::string assemble(const double *xyz, long nn, const int *tets, long nt, const int *region, const double *Ms,
                     const double *A, const double *K1, const double *axis, Assembly &out) {
    if (nn <= 0 || nt <= 0) return "empty mesh";
    for (long e = 0; e < 4 * nt; ++e)
        if (tets[e] < 0 || tets[e] >= nn) return "tet node index out of range";
    out.n_nodes = nn;
    out.n_tets = nt;
    // reduced units
    double msr = 0.0;
    for (long e = 0; e < nt; ++e)
        if (region[e] > 0) {
            if (!(Ms[e] >= 0.0) || !std::isfinite(Ms[e]) || !(A[e] >= 0.0) || !std::isfinite(K1[e]))
                return "invalid material value";
            msr = std::max(msr, Ms[e]);
        }
    if (!(msr > 0.0)) return "no magnetic tet with Ms > 0";
    out.Ms_ref = msr;
    const double unitE = kMu0 * msr * msr;  // J/m^3
    std::vector<double> ms(nt, 0.0), aa(nt, 0.0), kk(nt, 0.0), uu(3 * nt, 0.0);
    for (long e = 0; e < nt; ++e) {
        if (region[e] <= 0) continue;
        ms[e] = Ms[e] / msr;
        aa[e] = A[e] / (unitE * 1e-18);
        kk[e] = K1[e] / unitE;
        if (kk[e] != 0.0) {
            if (!axis) return "easy axis required where K1 != 0";
            double n = std::sqrt(axis[3 * e] * axis[3 * e] + axis[3 * e + 1] * axis[3 * e + 1] +
                                 axis[3 * e + 2] * axis[3 * e + 2]);
            if (!(n > 0.0)) return "zero easy axis";
            for (int d = 0; d < 3; ++d) uu[3 * e + d] = axis[3 * e + d] / n;
        }
    }
    Geo geo;
    geo.vol.resize(nt);
    geo.grad.resize(12 * nt);
    bool bad = false;
    parallel_rows(nt, [&](long e) {
        if (!tet_geometry(xyz, tets + 4 * e, &geo.vol[e], &geo.grad[12 * e])) bad = true;
    });
    if (bad) return "degenerate tetrahedron";

    // node -> incident tets
    std::vector<int64_t> nptr(nn + 1, 0);
    for (long e = 0; e < 4 * nt; ++e) nptr[tets[e] + 1]++;
    for (long i = 0; i < nn; ++i) nptr[i + 1] += nptr[i];
    std::vector<int64_t> fillp(nptr.begin(), nptr.end() - 1);
    std::vector<int> ntet(4 * nt);
    for (long e = 0; e < nt; ++e)
        for (int j = 0; j < 4; ++j) ntet[fillp[tets[4 * e + j]]++] = (int)e;

    // magnet nodes: touched by a magnetic tet
    out.mag_of_node.assign(nn, -1);
    int nm = 0;
    for (long i = 0; i < nn; ++i) {
        bool mag = false;
        for (int64_t q = nptr[i]; q < nptr[i + 1]; ++q) mag |= region[ntet[q]] > 0;
        if (mag) out.mag_of_node[i] = nm++;
    }
    out.n_mag = nm;
    out.node_of_mag.resize(nm);
    for (long i = 0; i < nn; ++i)
        if (out.mag_of_node[i] >= 0) out.node_of_mag[out.mag_of_node[i]] = (int)i;

    // outer boundary: a face (sorted triple) owned by its smallest node, counted
    // over the tets incident to that node; count 1 => boundary face
    std::vector<char> onb(nn, 0);
    {
        // faces of the tets incident to node i whose smallest vertex is i
        auto owned_faces = [&](long i, std::vector<std::array<int, 3>> &faces) {
            faces.clear();
            for (int64_t q = nptr[i]; q < nptr[i + 1]; ++q) {
                const int *t = tets + 4 * (long)ntet[q];
                for (int f = 0; f < 4; ++f) {
                    std::array<int, 3> tri;
                    int k = 0;
                    for (int j = 0; j < 4; ++j)
                        if (j != f) tri[k++] = t[j];
                    std::sort(tri.begin(), tri.end());
                    if (tri[0] == (int)i) faces.push_back(tri);
                }
            }
            std::sort(faces.begin(), faces.end());
        };
        std::vector<char> owner(nn, 0);
        parallel_rows(nn, [&](long i) {
            std::vector<std::array<int, 3>> faces;
            owned_faces(i, faces);
            for (size_t a = 0; a < faces.size();) {
                size_t b = a + 1;
                while (b < faces.size() && faces[b] == faces[a]) ++b;
                if (b - a == 1) owner[i] = 1;
                a = b;
            }
        });
        std::vector<std::array<int, 3>> faces;
        for (long i = 0; i < nn; ++i) {
            if (!owner[i]) continue;
            owned_faces(i, faces);
            for (size_t a = 0; a < faces.size();) {
                size_t b = a + 1;
                while (b < faces.size() && faces[b] == faces[a]) ++b;
                if (b - a == 1)
                    for (int v : faces[a]) onb[v] = 1;
                a = b;
            }
        }
    }
    out.pot_of_node.assign(nn, -1);
    int np = 0;
    for (long i = 0; i < nn; ++i)
        if (!onb[i]) out.pot_of_node[i] = np++;
    out.n_pot = np;
    std::vector<int> node_of_pot(np);
    for (long i = 0; i < nn; ++i)
        if (out.pot_of_node[i] >= 0) node_of_pot[out.pot_of_node[i]] = (int)i;
    out.pot_order = locality_order(xyz, node_of_pot);

    auto gdot = [&](long e, int i, int j) {
        const double *g = &geo.grad[12 * e];
        return g[3 * i] * g[3 * j] + g[3 * i + 1] * g[3 * j + 1] + g[3 * i + 2] * g[3 * j + 2];
    };
    auto local_index = [&](long e, int node) {
        for (int j = 0; j < 4; ++j)
            if (tets[4 * e + j] == node) return j;
        return -1;
    };

    // L and exchange diagonal
    out.L.assign(nm, 0.0);
    out.Dex.assign(nm, 0.0);
    parallel_rows(nm, [&](long a) {
        int node = out.node_of_mag[a];
        double L = 0.0, D = 0.0;
        for (int64_t q = nptr[node]; q < nptr[node + 1]; ++q) {
            long e = ntet[q];
            if (region[e] <= 0) continue;
            int ia = local_index(e, node);
            L += ms[e] * geo.vol[e] / 4.0;
            D += 2.0 * aa[e] * geo.vol[e] * gdot(e, ia, ia);
        }
        out.L[a] = L;
        out.Dex[a] = D;
    });

    // C: symmetric 3x3 blocks (xx yy zz xy xz yz) on magnet rows
    auto fillC = [&](int a, RowAcc &acc, bool exch_only) {
        int node = out.node_of_mag[a];
        for (int64_t q = nptr[node]; q < nptr[node + 1]; ++q) {
            long e = ntet[q];
            if (region[e] <= 0) continue;
            int ia = local_index(e, node);
            for (int jb = 0; jb < 4; ++jb) {
                int b = out.mag_of_node[tets[4 * e + jb]];
                double *v = acc.at(b);
                double s = 2.0 * aa[e] * geo.vol[e] * gdot(e, ia, jb);
                if (exch_only) {
                    v[0] += s;
                    continue;
                }
                v[0] += s;
                v[1] += s;
                v[2] += s;
                if (kk[e] != 0.0) {
                    double w = -2.0 * kk[e] * geo.vol[e] * (ia == jb ? 2.0 : 1.0) / 20.0;
                    const double *u = &uu[3 * e];
                    v[0] += w * u[0] * u[0];
                    v[1] += w * u[1] * u[1];
                    v[2] += w * u[2] * u[2];
                    v[3] += w * u[0] * u[1];
                    v[4] += w * u[0] * u[2];
                    v[5] += w * u[1] * u[2];
                }
            }
        }
    };
    auto diag_scale = [](const RowAcc &acc, int row, int vw) {
        double d = 0.0;
        for (size_t i = 0; i < acc.col.size(); ++i)
            if (acc.col[i] == row)
                for (int k = 0; k < std::min(vw, 3); ++k) d = std::max(d, std::fabs(acc.val[i * vw + k]));
        return d;
    };
    build_csr(nm, 6, out.C, [&](int a, RowAcc &acc) { fillC(a, acc, false); },
              [&](int a, const RowAcc &acc, int i) {
                  if (acc.col[i] == a) return true;
                  double d = diag_scale(acc, a, 6), mx = 0.0;
                  for (int k = 0; k < 6; ++k) mx = std::max(mx, std::fabs(acc.val[i * 6 + k]));
                  return mx > kDropRel * d;
              });
    build_csr(nm, 1, out.S, [&](int a, RowAcc &acc) { fillC(a, acc, true); },
              [&](int a, const RowAcc &acc, int i) {
                  if (acc.col[i] == a) return true;
                  return std::fabs(acc.val[i]) > kDropRel * diag_scale(acc, a, 1);
              });

    // K on free nodes
    out.DK.assign(np, 0.0);
    build_csr(np, 1, out.K,
              [&](int r, RowAcc &acc) {
                  int node = node_of_pot[r];
                  for (int64_t q = nptr[node]; q < nptr[node + 1]; ++q) {
                      long e = ntet[q];
                      int ir = local_index(e, node);
                      for (int j = 0; j < 4; ++j) {
                          int c = out.pot_of_node[tets[4 * e + j]];
                          if (c < 0) continue;
                          *acc.at(c) += geo.vol[e] * gdot(e, ir, j);
                      }
                  }
              },
              [&](int r, const RowAcc &acc, int i) {
                  if (acc.col[i] == r) return true;
                  return std::fabs(acc.val[i]) > kDropRel * diag_scale(acc, r, 1);
              });
    for (int r = 0; r < np; ++r)
        for (int64_t q = out.K.ptr[r]; q < out.K.ptr[r + 1]; ++q)
            if (out.K.col[q] == r) out.DK[r] = out.K.val[q];
    for (int r = 0; r < np; ++r)
        if (!(out.DK[r] > 0.0)) return "non-positive Poisson diagonal";

    // B rows: magnet nodes that are free; B_ja = sum_e ms_e V_e/4 grad phi_j
    std::vector<int> brow_nodes;
    for (int a = 0; a < nm; ++a)
        if (out.pot_of_node[out.node_of_mag[a]] >= 0) brow_nodes.push_back(a);
    build_csr((int)brow_nodes.size(), 3, out.B,
              [&](int r, RowAcc &acc) {
                  int node = out.node_of_mag[brow_nodes[r]];
                  for (int64_t q = nptr[node]; q < nptr[node + 1]; ++q) {
                      long e = ntet[q];
                      if (region[e] <= 0) continue;
                      int ij = local_index(e, node);
                      const double *g = &geo.grad[12 * e + 3 * ij];
                      double w = ms[e] * geo.vol[e] / 4.0;
                      for (int jb = 0; jb < 4; ++jb) {
                          double *v = acc.at(out.mag_of_node[tets[4 * e + jb]]);
                          for (int d = 0; d < 3; ++d) v[d] += w * g[d];
                      }
                  }
              },
              [&](int, const RowAcc &, int) { return true; });
    out.B.row_out.resize(brow_nodes.size());
    for (size_t r = 0; r < brow_nodes.size(); ++r) out.B.row_out[r] = out.pot_of_node[out.node_of_mag[brow_nodes[r]]];

    // B^T rows: magnet nodes a; entries over free j: sum_e ms_e V_e/4 grad phi_j^e
    build_csr(nm, 3, out.Bt,
              [&](int a, RowAcc &acc) {
                  int node = out.node_of_mag[a];
                  for (int64_t q = nptr[node]; q < nptr[node + 1]; ++q) {
                      long e = ntet[q];
                      if (region[e] <= 0) continue;
                      double w = ms[e] * geo.vol[e] / 4.0;
                      for (int j = 0; j < 4; ++j) {
                          int c = out.pot_of_node[tets[4 * e + j]];
                          if (c < 0) continue;
                          const double *g = &geo.grad[12 * e + 3 * j];
                          double *v = acc.at(c);
                          for (int d = 0; d < 3; ++d) v[d] += w * g[d];
                      }
                  }
              },
              [&](int, const RowAcc &, int) { return true; });
    return std::string();
}

}  // namespace mmncg
