// Drives every entry point of the CPU oracle on small inputs, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py:
// any out-of-bounds access, use after free, leak or undefined operation
// aborts the run.  Inputs: jittered lattices from a fixed linear
// congruential sequence (no method arithmetic here).
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../../oracle/sph_oracle.cpp"

namespace {

uint64_t g_state = 12345;
double uniform() {  // in [0, 1)
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

struct Case {
    OrcParams P;
    int64_t n;
    std::vector<double> x, u, m;
    std::vector<uint8_t> type;
};

Case lattice_case(int dim, int side, int kernel, int periodic, int cell_div, int brute) {
    Case c{};
    OrcParams& P = c.P;
    P.dim = dim;
    P.kernel = kernel;
    P.cell_div = cell_div;
    P.brute = brute;
    const double L = 1.0, dx = L / side;
    P.h = 1.3 * dx;
    P.rho0 = 1.0;
    P.c0 = 10.0;
    P.nu = 0.01;
    P.eta = 0.01;
    P.dt = 1e-4;
    for (int k = 0; k < 3; ++k) {
        P.periodic[k] = k < dim ? periodic : 0;
        P.lo[k] = periodic ? 0.0 : -0.2;
        P.hi[k] = periodic ? L : L + 0.2;
        P.g[k] = periodic ? 0.0 : (k == dim - 1 ? -1.0 : 0.0);
    }
    int64_t n = 1;
    for (int k = 0; k < dim; ++k) n *= side;
    c.n = n;
    c.x.resize(dim * n);
    c.u.resize(dim * n);
    c.m.assign(n, dx * (dim == 3 ? dx * dx : dx));
    c.type.assign(n, 0);
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = i;
        for (int k = 0; k < dim; ++k) {
            const int64_t q = r % side;
            r /= side;
            c.x[k * n + i] = (q + 0.5 + 0.6 * (uniform() - 0.5)) * dx;
            c.u[k * n + i] = 0.2 * (uniform() - 0.5);
        }
        if (!periodic && i % 7 == 0) {
            c.type[i] = 1;
            for (int k = 0; k < dim; ++k) c.u[k * n + i] = 0.0;
        }
    }
    return c;
}

int run(Case c) {
    const OrcParams* P = &c.P;
    const int64_t n = c.n, dn = (int64_t)c.P.dim * n;
    std::vector<double> rho(n), p(n), a(dn), arho(n), diag(4 * 3);
    for (double r = 0.0; r < 3.5 * c.P.h; r += 0.1 * c.P.h) {
        orc_kernel_w(P, r);
        orc_kernel_dwdr(P, r);
        orc_kernel_d2wdr2(P, r);
    }
    int64_t nc[3];
    double cs[3];
    if (orc_grid(P, nc, cs) != 0) return 1;
    const int64_t ncells = nc[0] * nc[1] * nc[2];
    std::vector<uint32_t> keys(n), ks(n), cst(ncells), cen(ncells);
    std::vector<int64_t> perm(n), off(n + 1);
    if (orc_cell_keys(P, n, c.x.data(), keys.data()) != 0) return 2;
    if (orc_bin_sort(P, n, c.x.data(), ks.data(), perm.data(), cst.data(), cen.data()) != 0) return 3;
    const int64_t total = orc_neighbors(P, n, c.x.data(), off.data(), nullptr, 0);
    std::vector<int64_t> idx(total);
    if (orc_neighbors(P, n, c.x.data(), off.data(), idx.data(), total) != total) return 4;
    if (orc_density(P, n, c.x.data(), c.m.data(), rho.data()) != 0) return 5;
    orc_eos(P, n, rho.data(), p.data());
    if (orc_momentum(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), rho.data(), p.data(),
                     a.data()) != 0)
        return 6;
    if (orc_evaluate(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), rho.data(), p.data(),
                     a.data()) != 0)
        return 7;
    orc_diag(P, n, c.u.data(), c.m.data(), diag.data());
    if (orc_continuity(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), arho.data()) != 0)
        return 8;
    std::vector<int64_t> sub = {0, n / 3, n - 1};
    std::vector<double> rs(3), ps(3), as(3 * c.P.dim);
    if (orc_eval_subset(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), 3, sub.data(),
                        rs.data(), ps.data(), as.data()) != 0)
        return 9;
    std::vector<double> lam(dn, 0.5), lx(dn, 0.0), lv(dn, 0.0);
    double lnu = 0.0;
    if (orc_rhs_adjoint(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), lam.data(),
                        lx.data(), lv.data(), &lnu) != 0)
        return 10;
    std::vector<double> gu(dn);
    double gnu = 0.0, ke = 0.0;
    if (orc_adjoint_ke(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), 2, gu.data(), &gnu,
                       &ke) != 0)
        return 11;
    if (orc_rollout_ke(P, n, c.x.data(), c.u.data(), c.m.data(), c.type.data(), 2, &ke) != 0)
        return 12;
    {
        std::vector<double> x = c.x, u = c.u;
        if (orc_step(P, n, x.data(), u.data(), a.data(), c.m.data(), c.type.data(), rho.data(),
                     p.data(), 3, 1, diag.data()) != 0)
            return 13;
    }
    {
        std::vector<double> x = c.x, u = c.u, r(n, 1.0);
        if (orc_step_continuity(P, n, x.data(), u.data(), r.data(), c.m.data(), c.type.data(), 2,
                                p.data(), a.data(), arho.data()) != 0)
            return 14;
    }
    {
        std::vector<double> x = c.x, u = c.u, r(n, 1.0);
        if (orc_step_continuity_pc(P, n, x.data(), u.data(), r.data(), c.m.data(), c.type.data(), 2,
                                   1, p.data(), a.data(), arho.data()) != 0)
            return 15;
    }
    return 0;
}

}  // namespace

int main() {
    orc_set_threads(2);
    const int cases[][6] = {
        // dim, side, kernel, periodic, cell_div, brute
        {2, 12, 0, 1, 1, 0}, {2, 12, 1, 1, 2, 1}, {2, 12, 2, 0, 1, 0},
        {3, 8, 1, 1, 1, 0},  {3, 7, 0, 0, 2, 0},  {3, 6, 2, 0, 1, 1},
    };
    for (const auto& k : cases) {
        const int rc = run(lattice_case(k[0], k[1], k[2], k[3], k[4], k[5]));
        if (rc != 0) {
            std::printf("case dim=%d side=%d kernel=%d failed at %d\n", k[0], k[1], k[2], rc);
            return rc;
        }
    }
    std::printf("oracle sanitize driver: all cases ok\n");
    return 0;
}
