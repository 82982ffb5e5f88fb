/*
 * Plain FP64 CPU oracle for the weakly-compressible SPH (WCSPH) hot path of
 * PySPH (arXiv:1909.04504, Section "The SPH method").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the bench's
 * CPU-baseline leg load this library.  It shares no code, header, table or
 * constant with the GPU library: every formula below is written out again
 * from the paper (and, where the paper is silent, from the readings listed in
 * the design notes: A-numbers in the comments refer to that list).
 *
 * Conventions
 *   - Arrays are SoA: a d-vector field f of n particles is f[k*n + i].
 *   - Everything is double precision; no fused or reordered arithmetic beyond
 *     what the definitions state (build with -ffp-contract=off).
 *   - Neighbour set (Section "Nearest neighbor particle search", A1, A13):
 *       j in N(i)  <=>  |x_i - x_j|^2 < R^2 (R = 2h; 3h for the quintic
 *       spline), minimum image on periodic axes, i itself included.
 *     Computed by brute force O(n^2) or by the paper's uniform cell grid with
 *     the (2s+1)^d stencil; both give the same set (pinned by the tests).
 *
 * Threads: the per-destination loops (neighbour rows, density, EOS,
 * momentum, continuity) may run on several OpenMP threads (orc_set_threads);
 * each destination's sum is still formed by one thread in the same order, so
 * the results are bitwise those of one thread.  Everything else (the
 * integrator stages, the diagnostics, the scatter-form adjoint) stays
 * sequential.  Default: one thread.
 *
 * Parity status of every function is stated next to it; all are pinned by
 * the CPU tests except where a function says "parity unpinned".
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

extern "C" {

/* Parameters of one run.  Mirrored by a ctypes Structure in oracle/__init__.py */
struct OrcParams {
    int32_t dim;         /* 2 or 3 */
    int32_t kernel;      /* 0 = cubic spline (M4), 1 = Wendland C2, 2 = quintic spline */
    int32_t cell_div;    /* cells per support radius along an axis (>= 1) */
    int32_t brute;       /* 1: brute-force neighbour sets; 0: cell list */
    int32_t periodic[3];
    int32_t cell_order;  /* sort key: 0 = row-major, 1 = Z-order (Morton) of the cell coordinates */
    double h;            /* smoothing length; support radius R = 2h, 3h for the quintic (A1) */
    double rho0;         /* reference density */
    double c0;           /* reference speed of sound */
    double nu;           /* kinematic viscosity */
    double eta;          /* regulariser in |r|^2 + eta h^2 (A4) */
    double dt;           /* time step (A10) */
    double g[3];         /* body acceleration */
    double lo[3], hi[3]; /* domain box */
};

}  // extern "C"

namespace {

const double kPi = 3.14159265358979323846;

/* ---- Smoothing kernels (Section 2: compact W with support k h; k = 2 for
 * the cubic spline and Wendland C2, k = 3 for the quintic spline) ---- */

/* Support radius R = k h. */
double support(const OrcParams& P) { return (P.kernel == 2 ? 3.0 : 2.0) * P.h; }

/* Normalisation sigma so that the integral of W over R^d is one (A2, A3, and
 * for the quintic the exact integrals of its shape: 239 pi/7 in 2D and
 * 120 pi in 3D, in units of h^d). */
double sigma(const OrcParams& P) {
    const double h = P.h;
    if (P.kernel == 0) {  /* cubic spline (Monaghan 1992 M4) */
        return P.dim == 2 ? 10.0 / (7.0 * kPi * h * h) : 1.0 / (kPi * h * h * h);
    }
    if (P.kernel == 2) {  /* quintic spline (Morris 1997), support 3h */
        return P.dim == 2 ? 7.0 / (478.0 * kPi * h * h) : 1.0 / (120.0 * kPi * h * h * h);
    }
    /* Wendland C2 scaled to support 2h */
    return P.dim == 2 ? 7.0 / (4.0 * kPi * h * h) : 21.0 / (16.0 * kPi * h * h * h);
}

/* Quintic spline shape and its q-derivatives, piecewise:
 *   w(q) = (3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5   (q < 1)
 *        = (3-q)^5 - 6 (2-q)^5                (1 <= q < 2)
 *        = (3-q)^5                            (2 <= q < 3) */
double quintic(double q, int deriv) {
    double w = 0.0;
    const double a[3] = {3.0, 2.0, 1.0}, c[3] = {1.0, -6.0, 15.0};
    for (int k = 0; k < 3; ++k) {
        const double t = a[k] - q;
        if (t <= 0.0) continue;
        const double t2 = t * t;
        if (deriv == 0) w += c[k] * t2 * t2 * t;
        if (deriv == 1) w += -5.0 * c[k] * t2 * t2;
        if (deriv == 2) w += 20.0 * c[k] * t2 * t;
    }
    return w;
}

/* W(|r|, h) */
double W(const OrcParams& P, double r) {
    const double q = r / P.h;
    const double s = sigma(P);
    if (P.kernel == 2) return q >= 3.0 ? 0.0 : s * quintic(q, 0);
    if (q >= 2.0) return 0.0;
    if (P.kernel == 0) {
        if (q < 1.0) return s * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
        const double t = 2.0 - q;
        return s * 0.25 * t * t * t;
    }
    const double t = 1.0 - 0.5 * q;
    return s * t * t * t * t * (2.0 * q + 1.0);
}

/* dW/dr (radial derivative, i.e. W'(q)/h) */
double dWdr(const OrcParams& P, double r) {
    const double q = r / P.h;
    const double s = sigma(P);
    if (P.kernel == 2) return q >= 3.0 ? 0.0 : s * quintic(q, 1) / P.h;
    if (q >= 2.0) return 0.0;
    if (P.kernel == 0) {
        if (q < 1.0) return s * (-3.0 * q + 2.25 * q * q) / P.h;
        const double t = 2.0 - q;
        return -0.75 * s * t * t / P.h;
    }
    const double t = 1.0 - 0.5 * q;
    return -5.0 * s * q * t * t * t / P.h;
}

/* d^2W/dr^2, needed by the adjoint only */
double d2Wdr2(const OrcParams& P, double r) {
    const double q = r / P.h;
    const double s = sigma(P);
    if (P.kernel == 2) return q >= 3.0 ? 0.0 : s * quintic(q, 2) / (P.h * P.h);
    if (q >= 2.0) return 0.0;
    if (P.kernel == 0) {
        if (q < 1.0) return s * (-3.0 + 4.5 * q) / (P.h * P.h);
        return 1.5 * s * (2.0 - q) / (P.h * P.h);
    }
    /* d/dq [-5 q (1-q/2)^3] = -5 (1-q/2)^3 + 7.5 q (1-q/2)^2 */
    const double t = 1.0 - 0.5 * q;
    return s * (-5.0 * t * t * t + 7.5 * q * t * t) / (P.h * P.h);
}

/* ---- Geometry: minimum image and the neighbour predicate (A13) ---- */

void separation(const OrcParams& P, int64_t n, const double* x, int64_t i, int64_t j, double* d) {
    for (int k = 0; k < P.dim; ++k) {
        double v = x[k * n + i] - x[k * n + j];
        if (P.periodic[k]) {
            const double L = P.hi[k] - P.lo[k];
            v -= L * std::nearbyint(v / L);
        }
        d[k] = v;
    }
}

double dot(const double* a, const double* b, int dim) {
    double s = 0.0;
    for (int k = 0; k < dim; ++k) s += a[k] * b[k];
    return s;
}

/* ---- Uniform cell grid (Section "Nearest neighbor particle search") ---- */

struct Grid {
    int64_t nc[3];
    double cs[3];
    int64_t ncells;
    int stencil;  /* cells searched on each side of the home cell */
    int64_t nkeys;  /* size of the sort-key space: ncells (row-major) or 2^(dim bits) (Z-order) */
    int bits;       /* Z-order: bits per coordinate, the smallest with 2^bits >= every nc */
};

/* Cells of size >= R / cell_div on every axis; returns false if a periodic
 * axis is too short for the stencil to visit each cell once, or if the grid
 * has more than 2^31 cells. */
bool make_grid(const OrcParams& P, Grid& G) {
    const double R = support(P);
    G.stencil = P.cell_div;
    G.ncells = 1;
    for (int k = 0; k < 3; ++k) {
        G.nc[k] = 1;
        G.cs[k] = 1.0;
    }
    for (int k = 0; k < P.dim; ++k) {
        const double L = P.hi[k] - P.lo[k];
        int64_t nc = (int64_t)std::floor(L * P.cell_div / R);
        if (nc < 1) nc = 1;
        if (P.periodic[k] && nc < 2 * P.cell_div + 1) return false;
        G.nc[k] = nc;
        G.cs[k] = L / (double)nc;
        G.ncells *= nc;
        if (G.ncells > (int64_t)1 << 31) return false; /* keys are 31-bit */
    }
    G.nkeys = G.ncells;
    G.bits = 0;
    if (P.cell_order == 1) {
        int64_t m = 1;
        for (int k = 0; k < P.dim; ++k) m = std::max(m, G.nc[k]);
        while (((int64_t)1 << G.bits) < m) ++G.bits;
        if (G.bits < 1) G.bits = 1;
        if (P.dim * G.bits > 31) return false;
        G.nkeys = (int64_t)1 << (P.dim * G.bits);
    }
    return true;
}

/* cell coordinate: clamp(floor((x - lo)/cs), 0, nc-1)  (A14) */
int64_t cell_coord(const OrcParams& P, const Grid& G, double x, int k) {
    int64_t c = (int64_t)std::floor((x - P.lo[k]) / G.cs[k]);
    if (c < 0) c = 0;
    if (c > G.nc[k] - 1) c = G.nc[k] - 1;
    return c;
}

/* row-major key, x fastest (A15) */
uint32_t cell_key(const OrcParams& P, const Grid& G, int64_t n, const double* x, int64_t i) {
    int64_t c[3] = {0, 0, 0};
    for (int k = 0; k < P.dim; ++k) c[k] = cell_coord(P, G, x[k * n + i], k);
    return (uint32_t)(c[0] + G.nc[0] * (c[1] + G.nc[1] * c[2]));
}

/* Sort key of the cell of particle i (Section 2.2 sorts by a cell key; the
 * paper's GPU search uses Z-order keys): row-major as cell_key, or the
 * Z-order (Morton) key, whose bit 3b + k (3D; dim b + k in general) is bit
 * b of the cell coordinate along axis k. */
uint32_t sort_key(const OrcParams& P, const Grid& G, int64_t n, const double* x, int64_t i) {
    if (P.cell_order != 1) return cell_key(P, G, n, x, i);
    int64_t c[3] = {0, 0, 0};
    for (int k = 0; k < P.dim; ++k) c[k] = cell_coord(P, G, x[k * n + i], k);
    uint64_t key = 0;
    for (int b = 0; b < G.bits; ++b)
        for (int k = 0; k < P.dim; ++k) key |= (uint64_t)((c[k] >> b) & 1) << (P.dim * b + k);
    return (uint32_t)key;
}

/* Neighbour lists as CSR: nbr[off[i] .. off[i+1]) ascending j. */
struct Nbrs {
    std::vector<int64_t> off;
    std::vector<int64_t> idx;
};

bool in_support(const OrcParams& P, const double* d) {
    const double R = support(P);
    return dot(d, d, P.dim) < R * R;
}

/* CSR lists from rows formed independently per particle, row_of(i, row). */
template <typename RowFn>
void build_rows(int64_t n, Nbrs& N, RowFn&& row_of) {
    std::vector<std::vector<int64_t>> rows(n);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) row_of(i, rows[i]);
    N.off.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) N.off[i + 1] = N.off[i] + (int64_t)rows[i].size();
    N.idx.resize(N.off[n]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) std::copy(rows[i].begin(), rows[i].end(), N.idx.begin() + N.off[i]);
}

void neighbours_brute(const OrcParams& P, int64_t n, const double* x, Nbrs& N) {
    build_rows(n, N, [&](int64_t i, std::vector<int64_t>& row) {
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            separation(P, n, x, i, j, d);
            if (in_support(P, d)) row.push_back(j);
        }
    });
}

/* Cell-list search: bucket the particles by cell, then test the particles of
 * the (2s+1)^d cells around each particle's own cell. */
bool neighbours_cells(const OrcParams& P, int64_t n, const double* x, Nbrs& N) {
    Grid G;
    if (!make_grid(P, G)) return false;
    std::vector<int64_t> cnt(G.ncells + 1, 0), bucket(n);
    std::vector<uint32_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
        key[i] = cell_key(P, G, n, x, i);
        cnt[key[i] + 1]++;
    }
    for (int64_t c = 0; c < G.ncells; ++c) cnt[c + 1] += cnt[c];
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t i = 0; i < n; ++i) bucket[fill[key[i]]++] = i;
    }
    const int s = G.stencil;
    build_rows(n, N, [&](int64_t i, std::vector<int64_t>& row) {
        double d[3];
        int64_t ci[3] = {0, 0, 0};
        for (int k = 0; k < P.dim; ++k) ci[k] = cell_coord(P, G, x[k * n + i], k);
        const int oz_lo = P.dim == 3 ? -s : 0, oz_hi = P.dim == 3 ? s : 0;
        for (int oz = oz_lo; oz <= oz_hi; ++oz)
            for (int oy = -s; oy <= s; ++oy)
                for (int ox = -s; ox <= s; ++ox) {
                    const int o[3] = {ox, oy, oz};
                    int64_t cj[3] = {0, 0, 0};
                    bool ok = true;
                    for (int k = 0; k < P.dim; ++k) {
                        int64_t c = ci[k] + o[k];
                        if (P.periodic[k]) {
                            c = ((c % G.nc[k]) + G.nc[k]) % G.nc[k];
                        } else if (c < 0 || c >= G.nc[k]) {
                            ok = false;
                        }
                        cj[k] = c;
                    }
                    if (!ok) continue;
                    const int64_t cell = cj[0] + G.nc[0] * (cj[1] + G.nc[1] * cj[2]);
                    for (int64_t b = cnt[cell]; b < cnt[cell + 1]; ++b) {
                        const int64_t j = bucket[b];
                        separation(P, n, x, i, j, d);
                        if (in_support(P, d)) row.push_back(j);
                    }
                }
        std::sort(row.begin(), row.end());
    });
    return true;
}

bool neighbours(const OrcParams& P, int64_t n, const double* x, Nbrs& N) {
    if (P.brute) {
        neighbours_brute(P, n, x, N);
        return true;
    }
    return neighbours_cells(P, n, x, N);
}

/* ---- Summation density (eq. 2), Tait EOS (eq. eos) ---- */

void density(const OrcParams& P, int64_t n, const double* x, const double* m, const Nbrs& N,
             double* rho) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double d[3];
        double s = 0.0;
        for (int64_t b = N.off[i]; b < N.off[i + 1]; ++b) {
            const int64_t j = N.idx[b];
            separation(P, n, x, i, j, d);
            s += m[j] * W(P, std::sqrt(dot(d, d, P.dim)));
        }
        rho[i] = s;
    }
}

/* p = B[(rho/rho0)^7 - 1], B = rho0 c0^2 / 7; the seventh power as the chain
 * r2 = r r, r4 = r2 r2, r7 = r4 r2 r (A9, A16). */
double eos(const OrcParams& P, double rho) {
    const double B = P.rho0 * P.c0 * P.c0 / 7.0;
    const double r = rho / P.rho0;
    const double r2 = r * r;
    const double r4 = r2 * r2;
    const double r7 = r4 * r2 * r;
    return B * (r7 - 1.0);
}

/* d p / d rho = 7 B r^6 / rho0 */
double deos(const OrcParams& P, double rho) {
    const double B = P.rho0 * P.c0 * P.c0 / 7.0;
    const double r = rho / P.rho0;
    const double r2 = r * r;
    const double r6 = r2 * r2 * r2;
    return 7.0 * B * r6 / P.rho0;
}

/* ---- Momentum (eq. mom:sph, mom:sph:press, mom:sph:visc; A5, A17) ----
 * a_i = g + sum_{j in N(i), j != i} m_j [ -(p_i/rho_i^2 + p_j/rho_j^2) gradW_ij
 *        + 4 nu / (rho_i + rho_j) (r_ij . gradW_ij) / (|r_ij|^2 + eta h^2) v_ij ]
 * for fluid particles (type 0); wall particles (type 1) get a = 0. */
void momentum(const OrcParams& P, int64_t n, const double* x, const double* v, const double* m,
              const uint8_t* type, const double* rho, const double* p, const Nbrs& N, double* a) {
    const int dim = P.dim;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double d[3];
        if (type[i] != 0) {
            for (int k = 0; k < dim; ++k) a[k * n + i] = 0.0;
            continue;
        }
        double acc[3] = {P.g[0], P.g[1], P.g[2]};
        const double Pi = p[i] / (rho[i] * rho[i]);
        for (int64_t b = N.off[i]; b < N.off[i + 1]; ++b) {
            const int64_t j = N.idx[b];
            if (j == i) continue;
            separation(P, n, x, i, j, d);
            const double r = std::sqrt(dot(d, d, dim));
            if (r == 0.0) continue; /* gradW(0) = 0 */
            double gw[3];
            const double f = dWdr(P, r) / r;
            for (int k = 0; k < dim; ++k) gw[k] = f * d[k];
            const double Pj = p[j] / (rho[j] * rho[j]);
            const double rdotgw = dot(d, gw, dim);
            const double visc = 4.0 * P.nu / (rho[i] + rho[j]) * rdotgw /
                                (r * r + P.eta * P.h * P.h);
            for (int k = 0; k < dim; ++k) {
                const double vij = v[k * n + i] - v[k * n + j];
                acc[k] += m[j] * (-(Pi + Pj) * gw[k] + visc * vij);
            }
        }
        for (int k = 0; k < dim; ++k) a[k * n + i] = acc[k];
    }
}

/* Full right-hand side: neighbours, density, EOS, momentum */
bool evaluate(const OrcParams& P, int64_t n, const double* x, const double* v, const double* m,
              const uint8_t* type, double* rho, double* p, double* a, Nbrs* keep = nullptr) {
    Nbrs local;
    Nbrs& N = keep ? *keep : local;
    if (!neighbours(P, n, x, N)) return false;
    density(P, n, x, m, N, rho);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) p[i] = eos(P, rho[i]);
    momentum(P, n, x, v, m, type, rho, p, N, a);
    return true;
}

/* ---- Continuity density: the paper's worked example (Section 3.2; its equation
 * listing and Euler stepper) ----
 * d rho_i / dt = sum_j m_j (v_i - v_j) . gradW_ij (eqn continuity:sph), over
 * every neighbour for fluid destinations and over fluid neighbours only for
 * solid (wall) destinations, as the example's equation groups state. */
void continuity(const OrcParams& P, int64_t n, const double* x, const double* v, const double* m,
                const uint8_t* type, const Nbrs& N, double* arho) {
    const int dim = P.dim;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double d[3];
        double s = 0.0;
        for (int64_t b = N.off[i]; b < N.off[i + 1]; ++b) {
            const int64_t j = N.idx[b];
            if (j == i) continue; /* v_ii = 0 */
            if (type[i] != 0 && type[j] != 0) continue;
            separation(P, n, x, i, j, d);
            const double r = std::sqrt(dot(d, d, dim));
            if (r == 0.0) continue; /* gradW(0) = 0 */
            const double f = dWdr(P, r) / r;
            double vg = 0.0;
            for (int k = 0; k < dim; ++k) vg += (v[k * n + i] - v[k * n + j]) * f * d[k];
            s += m[j] * vg;
        }
        arho[i] = s;
    }
}

/* Periodic wrap into [lo, hi) (A14) */
double wrap(const OrcParams& P, double x, int k) {
    if (!P.periodic[k]) return x;
    const double L = P.hi[k] - P.lo[k];
    double y = x - L * std::floor((x - P.lo[k]) / L);
    if (y >= P.hi[k]) y = P.lo[k];
    return y;
}

/* Neumaier-compensated sum */
struct Sum {
    double s = 0.0, c = 0.0;
    void add(double v) {
        const double t = s + v;
        if (std::fabs(s) >= std::fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};

void diagnostics(const OrcParams& P, int64_t n, const double* u, const double* m, double* out) {
    Sum ke, mom[3];
    for (int64_t i = 0; i < n; ++i) {
        double u2 = 0.0;
        for (int k = 0; k < P.dim; ++k) u2 += u[k * n + i] * u[k * n + i];
        ke.add(0.5 * m[i] * u2);
        for (int k = 0; k < P.dim; ++k) mom[k].add(m[i] * u[k * n + i]);
    }
    out[0] = ke.value();
    for (int k = 0; k < P.dim; ++k) out[1 + k] = mom[k].value();
}

/* ---- Adjoint of the right-hand side, scatter form ----
 * Given lam (d-vector per particle, the adjoint of a), accumulate
 *   lx += (dA/dx)^T lam,  lv += (dA/dv)^T lam,  *lnu += (dA/dnu)^T lam
 * at the state (x, v).  rho and p must be the values at that state and N its
 * neighbour lists.  Written over pairs with both ends updated, the plain
 * transpose of the forward sums. */
void rhs_adjoint(const OrcParams& P, int64_t n, const double* x, const double* v, const double* m,
                 const uint8_t* type, const double* rho, const double* p, const Nbrs& N,
                 const double* lam, double* lx, double* lv, double* lnu) {
    const int dim = P.dim;
    std::vector<double> lrho(n, 0.0), lP(n, 0.0);
    double d[3];
    const double eh2 = P.eta * P.h * P.h;
    double nu_acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != 0) continue; /* a_i = 0 for walls: no dependence */
        const double Pi = p[i] / (rho[i] * rho[i]);
        for (int64_t b = N.off[i]; b < N.off[i + 1]; ++b) {
            const int64_t j = N.idx[b];
            if (j == i) continue;
            separation(P, n, x, i, j, d);
            const double r = std::sqrt(dot(d, d, dim));
            if (r == 0.0) continue;
            const double Pj = p[j] / (rho[j] * rho[j]);
            const double w1 = dWdr(P, r), w2 = d2Wdr2(P, r);
            const double F = w1 / r;              /* gradW = F d */
            const double dF = (w2 - F) / r;       /* dF/dr */
            const double G = F * r * r / (r * r + eh2);
            /* dG/dr = dF r^2/(r^2+e) + F * 2 r e / (r^2+e)^2 */
            const double dG = dF * r * r / (r * r + eh2) + F * 2.0 * r * eh2 / ((r * r + eh2) * (r * r + eh2));
            const double rs = rho[i] + rho[j];
            double vij[3];
            for (int k = 0; k < dim; ++k) vij[k] = v[k * n + i] - v[k * n + j];
            const double* li = lam;  /* lam[k*n+i] */
            double ld = 0.0, lvv = 0.0;
            for (int k = 0; k < dim; ++k) {
                ld += li[k * n + i] * d[k];
                lvv += li[k * n + i] * vij[k];
            }
            const double mj = m[j];
            /* pressure part: -mj (Pi+Pj) F (lam . d) */
            /* viscous part:   mj 4 nu G/(rs) (lam . vij) */
            for (int k = 0; k < dim; ++k) {
                const double rhat = d[k] / r;
                const double gr = mj * (-(Pi + Pj) * (F * li[k * n + i] + dF * ld * rhat) +
                                        4.0 * P.nu / rs * lvv * dG * rhat);
                lx[k * n + i] += gr;
                lx[k * n + j] -= gr;
                const double gv = mj * 4.0 * P.nu * G / rs * li[k * n + i];
                lv[k * n + i] += gv;
                lv[k * n + j] -= gv;
            }
            const double gP = -mj * F * ld;
            lP[i] += gP;
            lP[j] += gP;
            const double grho = -mj * 4.0 * P.nu * G * lvv / (rs * rs);
            lrho[i] += grho;
            lrho[j] += grho;
            nu_acc += mj * 4.0 * G / rs * lvv;
        }
    }
    /* P_k = p(rho_k) / rho_k^2 */
    for (int64_t k = 0; k < n; ++k) {
        const double r = rho[k];
        lrho[k] += lP[k] * (deos(P, r) / (r * r) - 2.0 * p[k] / (r * r * r));
    }
    /* rho_k = sum_l m_l W(|x_k - x_l|) */
    for (int64_t k = 0; k < n; ++k) {
        for (int64_t b = N.off[k]; b < N.off[k + 1]; ++b) {
            const int64_t l = N.idx[b];
            if (l == k) continue;
            separation(P, n, x, k, l, d);
            const double r = std::sqrt(dot(d, d, dim));
            if (r == 0.0) continue;
            const double w1 = dWdr(P, r);
            for (int kk = 0; kk < dim; ++kk) {
                const double gr = lrho[k] * m[l] * w1 * d[kk] / r;
                lx[kk * n + k] += gr;
                lx[kk * n + l] -= gr;
            }
        }
    }
    *lnu += nu_acc;
}

}  // namespace

extern "C" {

int orc_version(void) { return 1; }

/* Number of OpenMP threads of the per-destination loops (>= 1); returns the
 * number in effect. */
int orc_set_threads(int k) {
    if (k >= 1) omp_set_num_threads(k);
    return omp_get_max_threads();
}

double orc_kernel_w(const OrcParams* P, double r) { return W(*P, r); }
double orc_kernel_dwdr(const OrcParams* P, double r) { return dWdr(*P, r); }
double orc_kernel_d2wdr2(const OrcParams* P, double r) { return d2Wdr2(*P, r); }

/* Grid dimensions (cells per axis, cell sizes); returns 0 or -1 if invalid. */
int orc_grid(const OrcParams* P, int64_t* nc, double* cs) {
    Grid G;
    if (!make_grid(*P, G)) return -1;
    for (int k = 0; k < 3; ++k) {
        nc[k] = G.nc[k];
        cs[k] = G.cs[k];
    }
    return 0;
}

/* Size of the sort-key space (cells, or Z-order keys). */
int64_t orc_nkeys(const OrcParams* P) {
    Grid G;
    if (!make_grid(*P, G)) return -1;
    return G.nkeys;
}

/* Cell keys of every particle (A14, A15). */
int orc_cell_keys(const OrcParams* P, int64_t n, const double* x, uint32_t* keys) {
    Grid G;
    if (!make_grid(*P, G)) return -1;
    for (int64_t i = 0; i < n; ++i) keys[i] = sort_key(*P, G, n, x, i);
    return 0;
}

/* Stable sort of particles by sort key (row-major or Z-order cell key):
 * perm[s] = index before sorting of the particle in sorted slot s;
 * keys_sorted[s] its key; cell_start/cell_end per key of the key space
 * (empty cells and unused Z-order keys: start = end = first slot of a larger
 * key). */
int orc_bin_sort(const OrcParams* P, int64_t n, const double* x, uint32_t* keys_sorted,
                 int64_t* perm, uint32_t* cell_start, uint32_t* cell_end) {
    Grid G;
    if (!make_grid(*P, G)) return -1;
    std::vector<uint32_t> key(n);
    for (int64_t i = 0; i < n; ++i) key[i] = sort_key(*P, G, n, x, i);
    std::vector<int64_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    for (int64_t s = 0; s < n; ++s) {
        perm[s] = order[s];
        keys_sorted[s] = key[order[s]];
    }
    for (int64_t c = 0; c < G.nkeys; ++c) {
        cell_start[c] = (uint32_t)(std::lower_bound(keys_sorted, keys_sorted + n, (uint32_t)c) - keys_sorted);
        cell_end[c] = (uint32_t)(std::upper_bound(keys_sorted, keys_sorted + n, (uint32_t)c) - keys_sorted);
    }
    return 0;
}

/* Neighbour lists (CSR, ascending j).  Returns the total count, or -1 on an
 * invalid grid.  idx is written only if total <= cap. */
int64_t orc_neighbors(const OrcParams* P, int64_t n, const double* x, int64_t* offsets,
                      int64_t* idx, int64_t cap) {
    Nbrs N;
    if (!neighbours(*P, n, x, N)) return -1;
    for (int64_t i = 0; i <= n; ++i) offsets[i] = N.off[i];
    const int64_t total = (int64_t)N.idx.size();
    if (idx && total <= cap) std::memcpy(idx, N.idx.data(), sizeof(int64_t) * total);
    return total;
}

int orc_density(const OrcParams* P, int64_t n, const double* x, const double* m, double* rho) {
    Nbrs N;
    if (!neighbours(*P, n, x, N)) return -1;
    density(*P, n, x, m, N, rho);
    return 0;
}

void orc_eos(const OrcParams* P, int64_t n, const double* rho, double* p) {
    for (int64_t i = 0; i < n; ++i) p[i] = eos(*P, rho[i]);
}

int orc_momentum(const OrcParams* P, int64_t n, const double* x, const double* v, const double* m,
                 const uint8_t* type, const double* rho, const double* p, double* a) {
    Nbrs N;
    if (!neighbours(*P, n, x, N)) return -1;
    momentum(*P, n, x, v, m, type, rho, p, N, a);
    return 0;
}

/* rho, p and a at (x, v) */
int orc_evaluate(const OrcParams* P, int64_t n, const double* x, const double* v, const double* m,
                 const uint8_t* type, double* rho, double* p, double* a) {
    return evaluate(*P, n, x, v, m, type, rho, p, a) ? 0 : -1;
}

void orc_diag(const OrcParams* P, int64_t n, const double* u, const double* m, double* out) {
    diagnostics(*P, n, u, m, out);
}

/* Predictor-corrector steps (Section "Time Integration"; A11: the second
 * half kick uses the acceleration evaluated at (x^{n+1}, u^{n+1/2}), which is
 * reused as the first half kick of the next step).
 *   prime = 1: a, rho, p are first evaluated at (x, u).
 *   diag (optional): nsteps*(1+dim) values, KE and momentum after each step. */
int orc_step(const OrcParams* P, int64_t n, double* x, double* u, double* a, const double* m,
             const uint8_t* type, double* rho, double* p, int64_t nsteps, int prime, double* diag) {
    const int dim = P->dim;
    const double dt = P->dt;
    if (prime && !evaluate(*P, n, x, u, m, type, rho, p, a)) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i) {
            for (int k = 0; k < dim; ++k) {
                if (type[i] != 0) {
                    u[k * n + i] = 0.0;
                    continue;
                }
                const double v = u[k * n + i] + 0.5 * dt * a[k * n + i];
                u[k * n + i] = v;
                x[k * n + i] = wrap(*P, x[k * n + i] + dt * v, k);
            }
        }
        /* u now holds v = u^{n+1/2} */
        if (!evaluate(*P, n, x, u, m, type, rho, p, a)) return -1;
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < dim; ++k)
                u[k * n + i] = type[i] != 0 ? 0.0 : u[k * n + i] + 0.5 * dt * a[k * n + i];
        if (diag) diagnostics(*P, n, u, m, diag + s * (1 + dim));
    }
    return 0;
}

/* Steps of the paper's worked example: accelerations at the start of the
 * step from (x, u, rho) -- p = EOS(rho) on every particle, d rho/dt by the
 * continuity equation, a by the momentum equation (fluid; walls a = 0) --
 * then the Euler stage u += dt a; x += dt u (with the new u, then the
 * periodic wrap); rho += dt d rho/dt.  Walls keep u = 0 and their position.
 * p, a and arho (if not NULL) receive the values of the last step's
 * evaluation. */
int orc_step_continuity(const OrcParams* P, int64_t n, double* x, double* u, double* rho,
                        const double* m, const uint8_t* type, int64_t nsteps, double* p_out,
                        double* a_out, double* arho_out) {
    const int dim = P->dim;
    const double dt = P->dt;
    std::vector<double> p(n), a((size_t)dim * n), arho(n);
    for (int64_t s = 0; s < nsteps; ++s) {
        Nbrs N;
        if (!neighbours(*P, n, x, N)) return -1;
        for (int64_t i = 0; i < n; ++i) p[i] = eos(*P, rho[i]);
        continuity(*P, n, x, u, m, type, N, arho.data());
        momentum(*P, n, x, u, m, type, rho, p.data(), N, a.data());
        for (int64_t i = 0; i < n; ++i) {
            for (int k = 0; k < dim; ++k) {
                if (type[i] != 0) {
                    u[k * n + i] = 0.0;
                    continue;
                }
                u[k * n + i] = u[k * n + i] + dt * a[k * n + i];
                x[k * n + i] = wrap(*P, x[k * n + i] + dt * u[k * n + i], k);
            }
            rho[i] = rho[i] + dt * arho[i];
        }
    }
    if (nsteps > 0) {
        if (p_out) std::copy(p.begin(), p.end(), p_out);
        if (a_out) std::copy(a.begin(), a.end(), a_out);
        if (arho_out) std::copy(arho.begin(), arho.end(), arho_out);
    }
    return 0;
}

/* The continuity scheme under the predictor-corrector integration of
 * Section 2.1, with the density advanced like the velocity (dt/2 kicks of its
 * rate around the drift), the rates at the step's end being evaluated at the
 * predicted end state (u* = u' + dt/2 a, rho* = rho' + dt/2 arho) so that
 * the scheme stays second order (A33):
 *   u' = u + dt/2 a,  rho' = rho + dt/2 arho   (fluid u; every particle's rho)
 *   x <- wrap(x + dt u')                        (fluid)
 *   neighbour rebuild; p = EOS(rho*); arho, a at (x, u*, rho*)
 *   u <- u' + dt/2 a,  rho <- rho' + dt/2 arho
 * The rates at a step's end start the next step (first-same-as-last); with
 * prime they are first evaluated at the input state, else a_io and arho_io
 * hold them on entry.  Walls keep x and u = 0.  On return a_io, arho_io hold
 * the last evaluation's rates and p_out its pressure. */
int orc_step_continuity_pc(const OrcParams* P, int64_t n, double* x, double* u, double* rho,
                           const double* m, const uint8_t* type, int64_t nsteps, int prime,
                           double* p_out, double* a_io, double* arho_io) {
    const int dim = P->dim;
    const double hdt = 0.5 * P->dt;
    std::vector<double> p(n), us((size_t)dim * n), rhos(n);
    auto evaluate = [&](const double* xe, const double* ue, const double* rhoe) -> bool {
        Nbrs N;
        if (!neighbours(*P, n, xe, N)) return false;
        for (int64_t i = 0; i < n; ++i) p[i] = eos(*P, rhoe[i]);
        continuity(*P, n, xe, ue, m, type, N, arho_io);
        momentum(*P, n, xe, ue, m, type, rhoe, p.data(), N, a_io);
        return true;
    };
    if (prime && !evaluate(x, u, rho)) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i) {
            rho[i] = rho[i] + hdt * arho_io[i];
            rhos[i] = rho[i] + hdt * arho_io[i];
            for (int k = 0; k < dim; ++k) {
                if (type[i] != 0) {
                    u[k * n + i] = 0.0;
                    us[k * n + i] = 0.0;
                    continue;
                }
                u[k * n + i] = u[k * n + i] + hdt * a_io[k * n + i];
                us[k * n + i] = u[k * n + i] + hdt * a_io[k * n + i];
                x[k * n + i] = wrap(*P, x[k * n + i] + P->dt * u[k * n + i], k);
            }
        }
        if (!evaluate(x, us.data(), rhos.data())) return -1;
        for (int64_t i = 0; i < n; ++i) {
            rho[i] = rho[i] + hdt * arho_io[i];
            for (int k = 0; k < dim; ++k)
                u[k * n + i] = type[i] != 0 ? 0.0 : u[k * n + i] + hdt * a_io[k * n + i];
        }
    }
    if (p_out && (prime || nsteps > 0)) std::copy(p.begin(), p.end(), p_out);
    return 0;
}

/* d rho/dt alone at (x, v) (pins and parity tests). */
int orc_continuity(const OrcParams* P, int64_t n, const double* x, const double* v,
                   const double* m, const uint8_t* type, double* arho) {
    Nbrs N;
    if (!neighbours(*P, n, x, N)) return -1;
    continuity(*P, n, x, v, m, type, N, arho);
    return 0;
}

/* Field values at a subset of destination particles, for checking very large
 * runs: rho, p at sub[], a at sub[] (evaluated with the density of every
 * neighbour of every sub particle). */
int orc_eval_subset(const OrcParams* P, int64_t n, const double* x, const double* v,
                    const double* m, const uint8_t* type, int64_t nsub, const int64_t* sub,
                    double* rho_sub, double* p_sub, double* a_sub) {
    Grid G;
    if (!make_grid(*P, G)) return -1;
    const int dim = P->dim;
    /* bucket particles by cell */
    std::vector<int64_t> cnt(G.ncells + 1, 0), bucket(n);
    std::vector<uint32_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
        key[i] = cell_key(*P, G, n, x, i);
        cnt[key[i] + 1]++;
    }
    for (int64_t c = 0; c < G.ncells; ++c) cnt[c + 1] += cnt[c];
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t i = 0; i < n; ++i) bucket[fill[key[i]]++] = i;
    }
    const int s = G.stencil;
    auto nbrs_of = [&](int64_t i, std::vector<int64_t>& row) {
        row.clear();
        int64_t ci[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) ci[k] = cell_coord(*P, G, x[k * n + i], k);
        double d[3];
        const int oz_lo = dim == 3 ? -s : 0, oz_hi = dim == 3 ? s : 0;
        for (int oz = oz_lo; oz <= oz_hi; ++oz)
            for (int oy = -s; oy <= s; ++oy)
                for (int ox = -s; ox <= s; ++ox) {
                    const int o[3] = {ox, oy, oz};
                    int64_t cj[3] = {0, 0, 0};
                    bool ok = true;
                    for (int k = 0; k < dim; ++k) {
                        int64_t c = ci[k] + o[k];
                        if (P->periodic[k])
                            c = ((c % G.nc[k]) + G.nc[k]) % G.nc[k];
                        else if (c < 0 || c >= G.nc[k])
                            ok = false;
                        cj[k] = c;
                    }
                    if (!ok) continue;
                    const int64_t cell = cj[0] + G.nc[0] * (cj[1] + G.nc[1] * cj[2]);
                    for (int64_t b = cnt[cell]; b < cnt[cell + 1]; ++b) {
                        const int64_t j = bucket[b];
                        separation(*P, n, x, i, j, d);
                        if (in_support(*P, d)) row.push_back(j);
                    }
                }
        std::sort(row.begin(), row.end());
    };
    auto rho_at = [&](int64_t i, const std::vector<int64_t>& row) {
        double d[3], acc = 0.0;
        for (int64_t j : row) {
            separation(*P, n, x, i, j, d);
            acc += m[j] * W(*P, std::sqrt(dot(d, d, dim)));
        }
        return acc;
    };
    std::vector<int64_t> row, row2;
    for (int64_t t = 0; t < nsub; ++t) {
        const int64_t i = sub[t];
        nbrs_of(i, row);
        const double rhoi = rho_at(i, row);
        const double pi = eos(*P, rhoi);
        rho_sub[t] = rhoi;
        p_sub[t] = pi;
        double acc[3] = {P->g[0], P->g[1], P->g[2]};
        if (type[i] != 0) {
            for (int k = 0; k < dim; ++k) a_sub[k * nsub + t] = 0.0;
            continue;
        }
        const double Pi = pi / (rhoi * rhoi);
        double d[3];
        for (int64_t j : row) {
            if (j == i) continue;
            nbrs_of(j, row2);
            const double rhoj = rho_at(j, row2);
            const double Pj = eos(*P, rhoj) / (rhoj * rhoj);
            separation(*P, n, x, i, j, d);
            const double r = std::sqrt(dot(d, d, dim));
            if (r == 0.0) continue;
            double gw[3];
            const double f = dWdr(*P, r) / r;
            for (int k = 0; k < dim; ++k) gw[k] = f * d[k];
            const double visc = 4.0 * P->nu / (rhoi + rhoj) * dot(d, gw, dim) /
                                (r * r + P->eta * P->h * P->h);
            for (int k = 0; k < dim; ++k) {
                const double vij = v[k * n + i] - v[k * n + j];
                acc[k] += m[j] * (-(Pi + Pj) * gw[k] + visc * vij);
            }
        }
        for (int k = 0; k < dim; ++k) a_sub[k * nsub + t] = acc[k];
    }
    return 0;
}

/* Transpose of the right-hand side at (x, v): lx, lv accumulate (dA/dx)^T lam
 * and (dA/dv)^T lam; lnu[0] accumulates (dA/dnu)^T lam. */
int orc_rhs_adjoint(const OrcParams* P, int64_t n, const double* x, const double* v,
                    const double* m, const uint8_t* type, const double* lam, double* lx,
                    double* lv, double* lnu) {
    Nbrs N;
    std::vector<double> rho(n), p(n), a(P->dim * n);
    if (!evaluate(*P, n, x, v, m, type, rho.data(), p.data(), a.data(), &N)) return -1;
    rhs_adjoint(*P, n, x, v, m, type, rho.data(), p.data(), N, lam, lx, lv, lnu);
    return 0;
}

/* Gradient of J = 1/2 sum m |u^N|^2 after nsteps predictor-corrector steps
 * from (x0, u0) (a^0 evaluated at (x0, u0)) with respect to u0 and nu.
 * Forward with a full tape, then the reverse sweep:
 *   lam_v = lam_u';  lamhat = lam_a' + dt/2 lam_u';
 *   (lam_x', lam_v, lam_nu) += (dA/dx', dA/dv, dA/dnu)^T lamhat;
 *   lam_x = lam_x';  lam_v += dt lam_x';  lam_u = lam_v;  lam_a = dt/2 lam_v.
 * Wall particles are fixed and carry no adjoint. */
int orc_adjoint_ke(const OrcParams* P, int64_t n, const double* x0, const double* u0,
                   const double* m, const uint8_t* type, int64_t nsteps, double* grad_u0,
                   double* grad_nu, double* ke_out) {
    const int dim = P->dim;
    const double dt = P->dt;
    const size_t dn = (size_t)dim * n;
    /* tape: positions and half-step velocities at which A was evaluated */
    std::vector<std::vector<double>> tx(nsteps + 1), tv(nsteps + 1);
    std::vector<double> x(x0, x0 + dn), u(u0, u0 + dn), a(dn), rho(n), p(n);
    if (!evaluate(*P, n, x.data(), u.data(), m, type, rho.data(), p.data(), a.data())) return -1;
    tx[0] = x;
    tv[0] = u;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < dim; ++k) {
                if (type[i] != 0) {
                    u[k * n + i] = 0.0;
                    continue;
                }
                const double v = u[k * n + i] + 0.5 * dt * a[k * n + i];
                u[k * n + i] = v;
                x[k * n + i] = wrap(*P, x[k * n + i] + dt * v, k);
            }
        tx[s + 1] = x;
        tv[s + 1] = u;
        if (!evaluate(*P, n, x.data(), u.data(), m, type, rho.data(), p.data(), a.data())) return -1;
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < dim; ++k)
                u[k * n + i] = type[i] != 0 ? 0.0 : u[k * n + i] + 0.5 * dt * a[k * n + i];
    }
    double dg[4];
    diagnostics(*P, n, u.data(), m, dg);
    if (ke_out) *ke_out = dg[0];

    std::vector<double> lx(dn, 0.0), lu(dn, 0.0), la(dn, 0.0), lv(dn), lhat(dn), ax(dn), av(dn);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) lu[k * n + i] = type[i] != 0 ? 0.0 : m[i] * u[k * n + i];
    double lnu = 0.0;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        /* state of this step's evaluation: x' = tx[s+1], v = tv[s+1] */
        for (size_t q = 0; q < dn; ++q) {
            lv[q] = lu[q];
            lhat[q] = la[q] + 0.5 * dt * lu[q];
            ax[q] = 0.0;
            av[q] = 0.0;
        }
        Nbrs N;
        if (!evaluate(*P, n, tx[s + 1].data(), tv[s + 1].data(), m, type, rho.data(), p.data(),
                      a.data(), &N))
            return -1;
        rhs_adjoint(*P, n, tx[s + 1].data(), tv[s + 1].data(), m, type, rho.data(), p.data(), N,
                    lhat.data(), ax.data(), av.data(), &lnu);
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < dim; ++k) {
                const size_t q = (size_t)k * n + i;
                if (type[i] != 0) {
                    lx[q] = lu[q] = la[q] = 0.0;
                    continue;
                }
                const double lxp = lx[q] + ax[q];
                double lvq = lv[q] + av[q];
                lvq += dt * lxp;
                lx[q] = lxp;
                lu[q] = lvq;
                la[q] = 0.5 * dt * lvq;
            }
    }
    /* a^0 = A(x0, u0) */
    {
        Nbrs N;
        for (size_t q = 0; q < dn; ++q) {
            ax[q] = 0.0;
            av[q] = 0.0;
        }
        if (!evaluate(*P, n, tx[0].data(), tv[0].data(), m, type, rho.data(), p.data(), a.data(), &N))
            return -1;
        rhs_adjoint(*P, n, tx[0].data(), tv[0].data(), m, type, rho.data(), p.data(), N, la.data(),
                    ax.data(), av.data(), &lnu);
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < dim; ++k) {
                const size_t q = (size_t)k * n + i;
                lu[q] = type[i] != 0 ? 0.0 : lu[q] + av[q];
            }
    }
    std::memcpy(grad_u0, lu.data(), sizeof(double) * dn);
    *grad_nu = lnu;
    return 0;
}

/* Kinetic energy after nsteps from (x0, u0), used by the finite-difference
 * checks of the adjoint. */
int orc_rollout_ke(const OrcParams* P, int64_t n, const double* x0, const double* u0,
                   const double* m, const uint8_t* type, int64_t nsteps, double* ke_out) {
    const size_t dn = (size_t)P->dim * n;
    std::vector<double> x(x0, x0 + dn), u(u0, u0 + dn), a(dn), rho(n), p(n);
    if (orc_step(P, n, x.data(), u.data(), a.data(), m, type, rho.data(), p.data(), nsteps, 1,
                 nullptr) != 0)
        return -1;
    double dg[4];
    diagnostics(*P, n, u.data(), m, dg);
    *ke_out = dg[0];
    return 0;
}

}  // extern "C"
