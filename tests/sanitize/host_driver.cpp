// Host-setup driver for the sanitizer test (built with -fsanitize=address,
// undefined by tests/test_sanitizers.py; no GPU code): runs every path of the
// host build -- classification and ordering, the splitting, incomplete LDL^T
// with its level schedule, the approximate inverse of C_alpha, the Chebyshev
// interval, the import of a stored setup, the graph partitioner and the
// tridiagonal eigensolver -- on small matrices, and the input checks on bad
// input.  Prints "ok" when every call returned.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <vector>

#include "host_setup.hpp"

using namespace ddlr;

namespace {

struct Mat {
    int64_t n = 0;
    std::vector<int64_t> rp{0};
    std::vector<int32_t> ci;
    std::vector<double> v;
};

// Stencil on an nx x ny x nz grid: offsets with |d| <= 1 per axis, `faces`
// keeps only the 2 * dim face neighbours; weights from a fixed hash so the
// matrix is symmetric, diagonally dominant (SPD) and shifted by `shift`.
Mat grid_matrix(int nx, int ny, int nz, bool faces, double shift) {
    Mat M;
    M.n = (int64_t)nx * ny * nz;
    auto id = [&](int x, int y, int z) { return (int32_t)(x + nx * (y + ny * z)); };
    auto w = [](int32_t a, int32_t b) {
        const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
        uint32_t hsh = lo * 2654435761u ^ (hi + 0x9e3779b9u + (lo << 6) + (lo >> 2));
        return 0.5 + (hsh % 1000) / 1000.0;
    };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int32_t i = id(x, y, z);
                double diag = shift;
                std::vector<std::pair<int32_t, double>> row;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int nb = (dx != 0) + (dy != 0) + (dz != 0);
                            if (nb == 0 || (faces && nb != 1)) continue;
                            const int X = x + dx, Y = y + dy, Z = z + dz;
                            if (X < 0 || Y < 0 || Z < 0 || X >= nx || Y >= ny || Z >= nz) {
                                diag += 1.0;
                                continue;
                            }
                            const int32_t j = id(X, Y, Z);
                            const double a = w(i, j);
                            diag += a;
                            row.push_back({j, -a});
                        }
                row.push_back({i, diag});
                std::sort(row.begin(), row.end());
                for (auto& e : row) {
                    M.ci.push_back(e.first);
                    M.v.push_back(e.second);
                }
                M.rp.push_back((int64_t)M.ci.size());
            }
    return M;
}

std::vector<int32_t> boxes(int nx, int ny, int nz, int px, int py, int pz) {
    std::vector<int32_t> part((size_t)nx * ny * nz);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                part[x + nx * (y + ny * z)] = (x * px / nx) + px * ((y * py / ny) + py * (z * pz / nz));
    return part;
}

int failures = 0;

void expect_error(const char* what, void (*fn)()) {
    try {
        fn();
        std::printf("no error: %s\n", what);
        ++failures;
    } catch (const SetupError&) {
    }
}

}  // namespace

int main() {
    struct Case {
        int nx, ny, nz, px, py, pz;
        bool faces;
        double shift;
    };
    const Case cases[] = {{24, 20, 1, 3, 2, 1, true, 0.0}, {10, 9, 8, 2, 2, 2, true, 0.0},
                          {8, 8, 7, 2, 2, 1, false, 0.0}, {12, 12, 1, 2, 2, 1, true, -0.3}};
    for (const Case& c : cases) {
        const Mat M = grid_matrix(c.nx, c.ny, c.nz, c.faces, c.shift);
        const std::vector<int32_t> part = boxes(c.nx, c.ny, c.nz, c.px, c.py, c.pz);
        const int32_t p = c.px * c.py * c.pz;
        validate(M.n, M.rp.data(), M.ci.data(), M.v.data(), part.data(), p);
        for (int factor = 0; factor < 2; ++factor)
            for (int corder = 0; corder < 2; ++corder)
                for (int csolve = 0; csolve < 3; ++csolve) {
                    HostPlan P;
                    try {
                        build_plan(P, M.n, M.rp.data(), M.ci.data(), M.v.data(), part.data(), p, 1.0, factor, corder,
                                   csolve);
                    } catch (const SetupError&) {
                        continue;  // an IC(0) breakdown on the shifted matrix is a reported error
                    }
                    if (csolve != 0) continue;
                    // the stored-setup path on the same data
                    HostPlan Q;
                    build_plan_imported(Q, M.n, M.rp.data(), M.ci.data(), M.v.data(), p, 1.0, P.perm, P.boff,
                                        P.colour, P.L, P.D, 0);
                    if (Q.lvl_ptr != P.lvl_ptr || Q.level != P.level) {
                        std::printf("imported schedule differs\n");
                        ++failures;
                    }
                }
        std::vector<int32_t> gp((size_t)M.n);
        for (int32_t q : {1, 2, 7}) partition_graph(M.n, M.rp.data(), M.ci.data(), q, gp.data());
    }
    // tridiagonal eigensolver: a random-looking tridiagonal and a diagonal one
    for (int m : {1, 2, 9, 40}) {
        std::vector<double> a(m), b(m > 1 ? m - 1 : 1, 0.0), ev, Z;
        for (int i = 0; i < m; ++i) a[i] = std::sin(1.0 + i);
        for (int i = 0; i + 1 < m; ++i) b[i] = 0.5 * std::cos(2.0 + i);
        tridiag_eig(m, a.data(), b.data(), ev, Z);
        if ((int)ev.size() != m || (int)Z.size() != m * m) ++failures;
    }
    // the input checks
    expect_error("unsorted columns", [] {
        const int64_t rp[] = {0, 2, 4};
        const int32_t ci[] = {1, 0, 0, 1};
        const double v[] = {-1, 4, -1, 4};
        const int32_t part[] = {0, 1};
        validate(2, rp, ci, v, part, 2);
    });
    expect_error("part out of range", [] {
        const int64_t rp[] = {0, 2, 4};
        const int32_t ci[] = {0, 1, 0, 1};
        const double v[] = {4, -1, -1, 4};
        const int32_t part[] = {0, 5};
        validate(2, rp, ci, v, part, 2);
    });
    expect_error("unsymmetric values", [] {
        const int64_t rp[] = {0, 2, 4};
        const int32_t ci[] = {0, 1, 0, 1};
        const double v[] = {4, -1, -2, 4};
        const int32_t part[] = {0, 1};
        validate(2, rp, ci, v, part, 2);
    });
    if (failures) {
        std::printf("failures: %d\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
