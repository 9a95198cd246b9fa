// Host AddressSanitizer / UBSan run of the library's host-side assembly
// (test infrastructure): the finite-element operators behind mm_mesh_upload /
// mm_material_set and the locality order of the potential rows, on a small
// Kuhn-split grain in an air box and on a box large enough for the order to
// cut it into tiles. Exit status 0 means the calls completed and the order is
// a permutation; the sanitizers abort on any invalid access, leak or
// undefined behaviour.
#include <cstdio>
#include <vector>

#include "internal.h"

namespace {

struct Box {
    std::vector<double> xyz;
    std::vector<int> tets, region;
};

// Kuhn split of an nx x ny x nz box of cubic cells of edge h; cells inside
// [m0, m1) per axis are magnetic (region 1)
Box kuhn_box(int nx, int ny, int nz, double h, const int m0[3], const int m1[3]) {
    Box b;
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                b.xyz.push_back(i * h);
                b.xyz.push_back(j * h);
                b.xyz.push_back(k * h);
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const bool mag = i >= m0[0] && i < m1[0] && j >= m0[1] && j < m1[1] && k >= m0[2] && k < m1[2];
                for (int p = 0; p < 6; ++p) {
                    int c[3] = {i, j, k};
                    for (int q = 0; q < 4; ++q) {
                        if (q > 0) c[perm[p][q - 1]]++;
                        b.tets.push_back(c[0] + (nx + 1) * (c[1] + (ny + 1) * c[2]));
                    }
                    b.region.push_back(mag ? 1 : 0);
                }
            }
    return b;
}

bool is_permutation(const std::vector<int> &o) {
    std::vector<char> seen(o.size(), 0);
    for (int v : o) {
        if (v < 0 || v >= (int)o.size() || seen[v]) return false;
        seen[v] = 1;
    }
    return true;
}

int run(int nx, int ny, int nz, const int m0[3], const int m1[3]) {
    Box b = kuhn_box(nx, ny, nz, 4.0, m0, m1);
    const long nt = (long)b.region.size(), nn = (long)b.xyz.size() / 3;
    std::vector<double> Ms(nt, 1.61 / (4e-7 * 3.14159265358979323846)), A(nt, 7.7e-12), K1(nt, 4.3e6), ax;
    for (long e = 0; e < nt; ++e) {
        ax.push_back(0.1);
        ax.push_back(0.0);
        ax.push_back(0.995);
    }
    mmncg::Assembly as;
    const std::string err = mmncg::assemble(b.xyz.data(), nn, b.tets.data(), nt, b.region.data(), Ms.data(), A.data(),
                                            K1.data(), ax.data(), as);
    if (!err.empty()) {
        std::printf("assembly failed: %s\n", err.c_str());
        return 2;
    }
    if ((int)as.pot_order.size() != as.n_pot || !is_permutation(as.pot_order)) return 3;
    bool identity = true;
    for (int r = 0; r < as.n_pot; ++r) identity = identity && as.pot_order[r] == r;
    std::printf("assembly under sanitizers: n_mag %d n_pot %d nnz(K) %lld order %s\n", as.n_mag, as.n_pot,
                (long long)as.K.ptr[as.K.nrows], identity ? "identity" : "tiled");
    return 0;
}

}  // namespace

int main() {
    const int a0[3] = {3, 2, 2}, a1[3] = {6, 4, 4};
    if (int rc = run(9, 6, 6, a0, a1)) return rc;  // below one tile: identity order
    const int b0[3] = {8, 8, 8}, b1[3] = {16, 16, 16};
    return run(24, 24, 24, b0, b1);                // 23^3 free nodes: several tiles
}
