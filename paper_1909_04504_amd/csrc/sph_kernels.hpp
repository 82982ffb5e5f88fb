// Device kernels of the gfx950 WCSPH hot path.
//
// Method (arXiv:1909.04504, Section 2): summation density (eq. 2) or the
// continuity equation (eqn continuity:sph), Tait EOS (eq. eos), momentum with
// pressure and viscous terms (eqs. mom:sph, mom:sph:press, mom:sph:visc),
// predictor-corrector integration (Sec. 2.1) or the Euler stage of the
// paper's dam-break example, uniform-cell neighbour search (Sec. 2.2).
//
// Design for CDNA4 (wave64, 256 CUs in 8 XCDs):
//  * Particles are kept sorted by cell key, so the particles of a stencil row
//    of cells are contiguous and every cell walk reads contiguous,
//    cache-resident slot ranges.  The sort is a counting sort on cell keys:
//    integer atomics count particles per cell, a two-kernel scan turns counts
//    into cell offsets, an atomic scatter groups particles by cell and a
//    per-cell rank (number of smaller previous indices in the same cell)
//    makes the result identical to a stable sort, hence deterministic.
//  * Pair records are packed per sorted slot: the position record, the
//    velocity as a 4-vector and (rho, P = p/rho^2) as a 2-vector (in 2D
//    (rho, P) ride in the velocity record and the particle type in the
//    position record, so a pair pass gathers two records).  FP64
//    records hold the absolute position; mixed-precision records hold
//    fixed-point offsets from the centre of the particle's cell, so that a
//    separation is an exact integer difference.  Either way swapping i and j
//    negates the separation bitwise and the neighbour predicate (decided in
//    FP64) is exactly symmetric.
//  * Each step builds neighbour lists once (one cell walk, or waves that
//    take whole cells in 2D) and the pair passes read them densely, in
//    the walk's order; a particle with more neighbours than the list
//    capacity is walked instead, with bitwise the same result.
//  * No floating-point atomics anywhere: every sum is formed by one thread in
//    a fixed order, so results are bitwise reproducible run to run.
//  * Integration (kick, drift, wrap) is FP64 with contraction disabled, so
//    it rounds exactly as the plain definition does.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

constexpr int kBlock = 256;          // threads per workgroup (4 waves of 64)
constexpr int kScanItems = 16;       // items per thread in the scans of long arrays
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int kScanItemsShort = 4;   // and of arrays of at most kScanShortMax
constexpr int64_t kScanShortMax = (int64_t)kBlock * kScanItemsShort * 512;
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, workgroups dealt round-robin

enum : uint32_t { kFlagOutside = 1u, kFlagNonFinite = 2u };

// Cell grid (Sec. 2.2): cs_k >= R / S on every used axis, S = stencil reach.
struct Grid {
    int nc[3];
    int S;
    int periodic[3];
    int dim;
    double lo[3];
    double L[3];
    double cs[3];
    // division of a key by nc[0] and of the quotient by nc[1] by multiply
    // and shift (Granlund and Montgomery, 1994): magic, shift 1, shift 2
    uint32_t dmag[2];
    int dsh1[2], dsh2[2];
    // sort key: 0 = row-major (x fastest), 1 = Z-order (Morton, 3D only):
    // bit 3b + k of the key is bit b of the cell coordinate along axis k,
    // over mbits bits per coordinate (keys in [0, 8^mbits))
    int order;
    int mbits;
};

// Bits 0..9 of v moved to bits 0, 3, 6, ..., 27 (and back): the bit
// interleave of the Z-order key by masked shifts, four steps of halving
// strides (16, 8, 4, 2) instead of a loop over bits.
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}

// Magic numbers of unsigned 32-bit division by d >= 1 (round-up method with
// the add step): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1 (mod
// 2^32), and n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) with
// t = mulhi(m, n), exact for every n < 2^32.
inline void div_magic(uint32_t d, uint32_t* m, int* s1, int* s2) {
    int l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;
    *m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
    *s1 = l < 1 ? l : 1;
    *s2 = l - 1 > 0 ? l - 1 : 0;
}

// Particle state arrays (device pointers); a and p are of the pair type T,
// rho too unless rho64 (continuity scheme: rho is integrated, so it is kept
// in FP64 like x and u, and arho holds its rate, else arho is null).
struct State {
    double* x[3];
    double* u[3];
    void* a[3];
    void* rho;
    void* p;
    double* m;
    uint8_t* type;
    int32_t* id;
    double* arho;
    int rho64;
};

template <typename T>
__device__ __forceinline__ double load_rho(const void* rho, int i, int rho64) {
    return rho64 ? ((const double*)rho)[i] : (double)((const T*)rho)[i];
}
template <typename T>
__device__ __forceinline__ void store_rho(void* rho, int i, double v, int rho64) {
    if (rho64)
        ((double*)rho)[i] = v;
    else
        ((T*)rho)[i] = (T)v;
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Position record of a sorted particle: FP64 keeps the absolute position and
// the mass; mixed precision keeps fixed-point offsets from the centre of the
// particle's cell (2^27 units per cell, int32) and the mass as float bits.
template <typename T> struct Rec;
template <> struct Rec<double> { using type = double4; };
template <> struct Rec<float> { using type = int4; };
constexpr int kFixBits = 27;
constexpr int kFixClamp = (1 << 29) - 1;  // offsets within 4 cells of the centre

__device__ __forceinline__ double rec_mass(const double4& r) { return r.w; }
__device__ __forceinline__ float rec_mass(const int4& r) { return __int_as_float(r.w); }

// Separation of an accepted pair: r_ij and |r_ij|^2 in the pair precision;
// in mixed precision also the exact fixed-point difference, from which
// geom_r2d() forms |r_ij|^2 in FP64 for the density terms.
template <typename T> struct Geom;
template <> struct Geom<double> {
    double d[3];
    double r2;
};
template <> struct Geom<float> {
    float d[3];
    float r2;
    int id[3];
};
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// (rho, P = p / rho^2) records of the pair passes.  In 2D they ride in the
// unused z, w slots of the velocity record, so a pass gathers two records per
// neighbour instead of three; in 3D they have an array of their own.
template <int DIM, typename T>
__device__ __forceinline__ typename Vec2<T>::type load_rp(
    const typename Vec4<T>::type& v, const typename Vec2<T>::type* __restrict__ rp, uint32_t i) {
    typename Vec2<T>::type r;
    if (DIM == 2) {
        r.x = v.z;
        r.y = v.w;
        return r;
    }
    r = rp[i];
    // one load for both: rho alone is read in the viscous term's branch, and
    // the compiler would otherwise load it there, late, as a gather of its own
    asm("" : "+v"(r.x), "+v"(r.y));
    return r;
}
template <int DIM, typename T>
__device__ __forceinline__ void store_rp(typename Vec4<T>::type* __restrict__ vel,
                                         typename Vec2<T>::type* __restrict__ rp, uint32_t i,
                                         const typename Vec2<T>::type& r) {
    if (DIM == 2)
        reinterpret_cast<typename Vec2<T>::type*>(vel + i)[1] = r;  // the z, w slots
    else
        rp[i] = r;
}

// Constants of the pair terms in the pair precision T.
template <typename T>
struct PairConst {
    T R2;          // (2h)^2
    T inv_h;       // 1/h
    T sigma;       // kernel normalisation (includes h^-dim)
    T sigma_h2;    // sigma / h^2: scale of F = (dW/dr)/r
    T eta_h2;      // eta h^2
    T four_nu;     // 4 nu
    T g[3];        // body acceleration
    T cs[3];       // cell sizes
    T rho0, inv_rho0, B;  // Tait: p = B((rho/rho0)^7 - 1)
    double rho0_d, B_d;   // the same in FP64 (per-particle EOS)
    T L[3];        // box lengths (periodic image shifts)
    T h;           // smoothing length
    double R2_d;         // (2h)^2 in FP64: the neighbour predicate
    double inv_h_d, sigma_d;  // FP64 density terms
    double half_inv_h_d, two_inv_h_d;  // 1/(2h), 2/h: Wendland's factors in r
    double fix_scale[3];      // cell size / 2^27: one fixed-point unit
    float fix_scale_f[3];     // the same in FP32
    float R2_lo, R2_hi;       // (2h)^2 (1 -+ 1e-5): FP32 test band, FP64 inside it
    float R2_mid, R2_w;       // (2h)^2 and 2e-5 (2h)^2: |r2 - mid| < w covers the band
    T sigma_h4;    // sigma / h^4 (adjoint only)
    T b7;          // 7 B / rho0 = dp/drho at rho0 (adjoint only)
};

__device__ __forceinline__ double geom_r2d(const Geom<double>& g, const PairConst<double>&) {
    return g.r2;
}
__device__ __forceinline__ double geom_r2d(const Geom<float>& g, const PairConst<float>& C) {
    const double x = (double)g.id[0] * C.fix_scale[0];
    const double y = (double)g.id[1] * C.fix_scale[1];
    const double z = (double)g.id[2] * C.fix_scale[2];
    return x * x + y * y + z * z;
}

// ---------------------------------------------------------------------------
// Precision-generic helpers.  Mixed precision uses the hardware square root
// and reciprocal (1 ulp); FP64 uses the correctly rounded library forms.
__device__ __forceinline__ float p_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double p_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float p_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double p_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float p_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double p_rsqrt(double x) { return 1.0 / sqrt(x); }

// FP64 square root for the mixed-precision density terms: an FP32
// reciprocal square root y as the seed, r = x y, and one Newton step
// r + (x - r^2) y / 2, relative error ~1e-14 (one transcendental instead of
// a square root and a reciprocal).  x is taken at least the smallest normal
// float, so that x = 0 (the self pair) gives r ~ 1e-19 instead of 0 * inf;
// a kernel evaluated at q ~ 1e-19 / h rounds to its value at 0 (every
// kernel here is flat there).  The FP64 path uses the correctly rounded sqrt.
__device__ __forceinline__ double sqrt_newton(double x) {
    const double xc = fmax(x, 1.1754943508222875e-38);
    const double y = (double)__builtin_amdgcn_rsqf((float)xc);
    const double r = xc * y;
    return fma(fma(-r, r, xc), 0.5 * y, r);
}
__device__ __forceinline__ double density_sqrt(double x, float) { return sqrt_newton(x); }
__device__ __forceinline__ double density_sqrt(double x, double) { return sqrt(x); }

// Smoothing kernel W(q) = sigma w(q), q = r/h, support q < 2 (q < 3 for
// the quintic spline).
//   cubic spline (M4):  1 - 1.5 q^2 + 0.75 q^3 (q < 1);  0.25 (2 - q)^3 (q < 2)
//   Wendland C2:        (1 - q/2)^4 (2 q + 1)
//   quintic spline:     (3-q)^5 - 6 (2-q)_+^5 + 15 (1-q)_+^5
// The cubic spline is evaluated as 0.25 (2-q)^3 - (1-q)_+^3, the same
// polynomial as 1 - 1.5 q^2 + 0.75 q^3 on q < 1 without a second branch.
template <typename T>
__device__ __forceinline__ T pow5(T t) {
    const T t2 = t * t;
    return t2 * t2 * t;
}
template <typename T>
__device__ __forceinline__ T pos_part(T t) {
    return t > T(0) ? t : T(0);
}
template <int KERNEL, typename T>
__device__ __forceinline__ T kernel_w(T q, T sigma) {
    if (KERNEL == 0) {
        const T t2 = T(2) - q;
        T t1 = T(1) - q;
        t1 = t1 > T(0) ? t1 : T(0);
        return sigma * (T(0.25) * t2 * t2 * t2 - t1 * t1 * t1);
    } else if (KERNEL == 2) {
        return sigma * (pow5(T(3) - q) - T(6) * pow5(pos_part(T(2) - q)) +
                        T(15) * pow5(pos_part(T(1) - q)));
    } else {
        const T t = T(1) - T(0.5) * q;
        const T t2 = t * t;
        return sigma * (t2 * t2 * (T(2) * q + T(1)));
    }
}

// The density pass's form, in FP64: w(q) without sigma (the sum is scaled
// once per particle), from r = |r_ij| (Wendland's two factors straight from
// r, the splines through q = r/h).
template <int KERNEL, typename T>
__device__ __forceinline__ double kernel_w_r(double r, const PairConst<T>& C) {
    if (KERNEL == 1) {
        const double t = fma(-C.half_inv_h_d, r, 1.0);
        const double u = fma(C.two_inv_h_d, r, 1.0);
        const double t2 = t * t;
        return t2 * t2 * u;
    }
    return kernel_w<KERNEL, double>(r * C.inv_h_d, 1.0);
}

// F(q) = (dW/dr) / r, so that grad_i W_ij = F r_ij.
//   cubic:    sigma/h^2 (-3 + 2.25 q)  (q < 1);  -0.75 sigma/h^2 (2-q)^2 / q  (q < 2)
//   Wendland: -5 sigma/h^2 (1 - q/2)^3
//   quintic:  sigma/h^2 (-120 + q^2 (120 - 50 q))  (q < 1);
//             sigma/h^2 (-5 (3-q)^4 + 30 (2-q)_+^4) / q  (q < 3)
// (the q < 1 form is w'(q)/q expanded, without the division at q -> 0).
template <typename T>
__device__ __forceinline__ T quintic_dw(T q) {  // w'(q) for q >= 1
    const T t3 = T(3) - q, t2 = pos_part(T(2) - q);
    const T a = t3 * t3, b = t2 * t2;
    return T(-5) * a * a + T(30) * b * b;
}
template <int KERNEL, typename T>
__device__ __forceinline__ T kernel_f(T q, T sigma_h2) {
    if (KERNEL == 0) {
        const T t = T(2) - q;
        if (q < T(1)) return sigma_h2 * (T(-3) + T(2.25) * q);
        return T(-0.75) * sigma_h2 * t * t * p_rcp(q);
    } else if (KERNEL == 2) {
        if (q < T(1)) return sigma_h2 * (T(-120) + q * q * (T(120) - T(50) * q));
        return sigma_h2 * quintic_dw(q) * p_rcp(q);
    } else {
        const T t = T(1) - T(0.5) * q;
        return T(-5) * sigma_h2 * t * t * t;
    }
}

// F = (dW/dr)/r from |r|^2 with one reciprocal square root: rinv = 1/|r|,
// q = |r| / h, 1/q = h rinv.  At r = 0 (the self pair), F r = 0 anyway.
// In FP32 the square root is then taken of the smallest normal number
// instead (every nonzero |r|^2 of a pair is far above it), so rinv stays
// finite, q = 0 exactly and F is the inner branch's value at q = 0: no
// select.  In FP64 rinv is set to 0 there by a select, which measured
// faster than the clamp (the FP64 square root is a software sequence).
template <typename T> __device__ __forceinline__ T tiny_normal();
template <> __device__ __forceinline__ float tiny_normal<float>() { return 1.17549435e-38f; }
template <> __device__ __forceinline__ double tiny_normal<double>() { return 2.2250738585072014e-308; }
template <int KERNEL, typename T>
__device__ __forceinline__ T kernel_f_r2(T r2, const PairConst<T>& C) {
    T rinv;
    if constexpr (sizeof(T) == 8)
        rinv = r2 > T(0) ? p_rsqrt(r2) : T(0);
    else
        rinv = p_rsqrt(fmax(r2, tiny_normal<T>()));
    const T q = r2 * rinv * C.inv_h;
    if (KERNEL == 0) {
        const T t = T(2) - q;
        const T inner = C.sigma_h2 * (T(-3) + T(2.25) * q);
        const T outer = T(-0.75) * C.sigma_h2 * t * t * (C.h * rinv);
        return q < T(1) ? inner : outer;
    } else if (KERNEL == 2) {
        const T inner = C.sigma_h2 * (T(-120) + q * q * (T(120) - T(50) * q));
        const T outer = C.sigma_h2 * quintic_dw(q) * (C.h * rinv);
        return q < T(1) ? inner : outer;
    } else {
        const T t = T(1) - T(0.5) * q;
        return T(-5) * C.sigma_h2 * t * t * t;
    }
}

// Tait EOS, evaluated per particle in FP64 in both precisions, with the
// seventh power as r2 = r r, r4 = r2 r2, r7 = r4 r2 r.  In mixed precision
// the pair terms are FP32 but the density sum and this per-particle
// evaluation are FP64: the EOS multiplies density rounding by about
// 7 B / rho0 before it reaches the pressure force.
template <typename T>
__device__ __forceinline__ double tait64(double rho, const PairConst<T>& C) {
    const double r = rho / C.rho0_d;
    const double r2 = r * r;
    const double r4 = r2 * r2;
    return C.B_d * (r4 * r2 * r - 1.0);
}

// Map the hardware workgroup id to a logical block so that each XCD (blocks
// are dealt to XCDs round-robin) works on one contiguous range of sorted
// particles: neighbour data then stays in that XCD's L2.
__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b % kNumXcd, k = b / kNumXcd;
    const int per = nb / kNumXcd, rem = nb % kNumXcd;
    return x * per + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ uint32_t div_by(uint32_t n, const Grid& G, int a) {
    const uint32_t t = __umulhi(G.dmag[a], n);
    return (t + ((n - t) >> G.dsh1[a])) >> G.dsh2[a];
}
// Sort key of cell c (row-major or Z-order).
__device__ __forceinline__ uint32_t cell_key(const int c[3], const Grid& G) {
    if (G.order)
        return spread3((uint32_t)c[0]) | (spread3((uint32_t)c[1]) << 1) |
               (spread3((uint32_t)c[2]) << 2);
    return (uint32_t)c[0] + (uint32_t)G.nc[0] * ((uint32_t)c[1] + (uint32_t)G.nc[1] * (uint32_t)c[2]);
}
__device__ __forceinline__ void decode_key(uint32_t key, const Grid& G, int c[3]) {
    if (G.order) {
        c[0] = (int)compact3(key);
        c[1] = (int)compact3(key >> 1);
        c[2] = (int)compact3(key >> 2);
        return;
    }
    const uint32_t q = div_by(key, G, 0);
    c[0] = (int)(key - q * (uint32_t)G.nc[0]);
    const uint32_t r = div_by(q, G, 1);
    c[1] = (int)(q - r * (uint32_t)G.nc[1]);
    c[2] = (int)r;
}

// cell coordinate clamp(floor((x - lo)/cs), 0, nc-1); NaN goes to 0.  A
// clamp on a non-periodic axis marks the particle as outside the box (its
// neighbours are still found: all of them are clamped into the same edge
// cells or lie in the stencil).  On a periodic axis a clamp only absorbs the
// rounding of a wrapped coordinate just below hi.
__device__ __forceinline__ int cell_coord(double x, const Grid& G, int k, bool* outside) {
    const double f = floor((x - G.lo[k]) / G.cs[k]);
    if (!(f >= 0.0)) {
        *outside |= !G.periodic[k];
        return 0;
    }
    if (f > (double)(G.nc[k] - 1)) {
        *outside |= !G.periodic[k];
        return G.nc[k] - 1;
    }
    return (int)f;
}

// ---------------------------------------------------------------------------
// Frames of the pair records.
//  * FP64: absolute positions; r_ij = fl(x_i - x_j) minus a periodic shift of
//    +-L for a wrapped stencil cell, which rounds exactly as the minimum-image
//    difference of the definition.
//  * Mixed precision: fixed-point offsets k from the centre of the particle's
//    cell; r_ij = (k_i - k_j - o 2^27) units, an exact integer (o the stencil
//    offset of j's cell), converted once.  Positions are quantised to
//    cs/2^27 (~4e-11 for the workloads here), far below float resolution.
// Both are exactly antisymmetric (r_ji = -r_ij bitwise), so the neighbour
// predicate |r|^2 < (2h)^2, evaluated in FP64, is symmetric.

// Neighbour cell along one axis for stencil offset o; returns false outside a
// non-periodic grid.  wrap = -1 / +1 if the periodic stencil wrapped.
__device__ __forceinline__ bool stencil_axis(int c, int o, int nc, int periodic, int* cell,
                                             int* wrap) {
    int cc = c + o;
    *wrap = 0;
    if (cc < 0) {
        if (!periodic) return false;
        cc += nc;
        *wrap = -1;
    } else if (cc >= nc) {
        if (!periodic) return false;
        cc -= nc;
        *wrap = 1;
    }
    *cell = cc;
    return true;
}

// Record coordinates of a particle at x in cell c along axis k.
__device__ __forceinline__ double frame_coord64(double x) { return x; }
__device__ __forceinline__ int frame_coord_fix(double x, int c, const Grid& G, int k) {
    const double centre = G.lo[k] + ((double)c + 0.5) * G.cs[k];
    double u = rint((x - centre) / G.cs[k] * (double)(1 << kFixBits));
    if (!(u == u)) u = 0.0;  // non-finite positions are flagged by the hash
    u = u > (double)kFixClamp ? (double)kFixClamp : (u < -(double)kFixClamp ? -(double)kFixClamp : u);
    return (int)u;
}

template <typename T>
__device__ __forceinline__ typename Rec<T>::type make_rec(const double* x, const int* c, double m,
                                                          int type, const Grid& G, int dim);
// In 2D the z slot carries the particle type (the continuity pass reads it
// with the record instead of gathering it); every reader of a record's z
// coordinate is 3D only.
template <>
__device__ __forceinline__ double4 make_rec<double>(const double* x, const int*, double m,
                                                    int type, const Grid&, int dim) {
    double4 r;
    r.x = x[0];
    r.y = x[1];
    r.z = dim == 3 ? x[2] : (double)type;
    r.w = m;
    return r;
}
template <>
__device__ __forceinline__ int4 make_rec<float>(const double* x, const int* c, double m, int type,
                                                const Grid& G, int dim) {
    int4 r;
    r.x = frame_coord_fix(x[0], c[0], G, 0);
    r.y = frame_coord_fix(x[1], c[1], G, 1);
    r.z = dim == 3 ? frame_coord_fix(x[2], c[2], G, 2) : type;
    r.w = __float_as_int((float)m);
    return r;
}
__device__ __forceinline__ int rec_type2(const double4& r) { return (int)r.z; }
__device__ __forceinline__ int rec_type2(const int4& r) { return r.z; }

// Pair geometry for candidate j of particle i.
//  * FP64: r_ij = fl(x_i - x_j) minus the periodic shift w L of a wrapped
//    stencil cell (w in {-1, 0, 1} per axis).
//  * Mixed precision: r_ij = (k_i - k_j - o 2^27) fixed-point units, o the
//    stencil offset of j's cell (an exact integer), converted to FP32; the
//    integers are kept for the FP64 |r|^2 of the density terms.
template <int DIM>
__device__ __forceinline__ Geom<double> pair_geom(const double4& ri, const double4& rj, int, int,
                                                  int, int wx, int wy, int wz,
                                                  const PairConst<double>& C) {
    auto shift = [&](int w, int k) { return w == 0 ? 0.0 : (w < 0 ? -C.L[k] : C.L[k]); };
    Geom<double> g;
    g.d[0] = (ri.x - rj.x) - shift(wx, 0);
    g.d[1] = (ri.y - rj.y) - shift(wy, 1);
    g.d[2] = DIM == 3 ? (ri.z - rj.z) - shift(wz, 2) : 0.0;
    g.r2 = g.d[0] * g.d[0] + g.d[1] * g.d[1];
    if (DIM == 3) g.r2 += g.d[2] * g.d[2];
    return g;
}
template <int DIM>
__device__ __forceinline__ Geom<float> pair_geom(const int4& ri, const int4& rj, int ox, int oy,
                                                 int oz, int, int, int,
                                                 const PairConst<float>& C) {
    Geom<float> g;
    g.id[0] = (ri.x - rj.x) - ox * (1 << kFixBits);
    g.id[1] = (ri.y - rj.y) - oy * (1 << kFixBits);
    g.id[2] = DIM == 3 ? (ri.z - rj.z) - oz * (1 << kFixBits) : 0;
    g.d[0] = (float)g.id[0] * C.fix_scale_f[0];
    g.d[1] = (float)g.id[1] * C.fix_scale_f[1];
    g.d[2] = DIM == 3 ? (float)g.id[2] * C.fix_scale_f[2] : 0.f;
    g.r2 = g.d[0] * g.d[0] + g.d[1] * g.d[1] + (DIM == 3 ? g.d[2] * g.d[2] : 0.f);
    return g;
}

// Neighbour predicate |r_ij|^2 < (2h)^2, decided in FP64.  FP64: on the
// separation itself.  Mixed precision: the FP32 |r|^2 decides outside a band
// of +-1e-5 around (2h)^2 (well above its rounding error), the exact FP64
// |r|^2 of the integer separation inside it; both are exactly symmetric
// (swapping i and j negates the integers).
__device__ __forceinline__ bool pair_accept(const Geom<double>& g, const PairConst<double>& C) {
    return g.r2 < C.R2_d;
}
__device__ __forceinline__ bool pair_accept(const Geom<float>& g, const PairConst<float>& C) {
    bool acc = g.r2 < C.R2_lo;
    // the band, as one compare: r2 - mid is exact near it (Sterbenz), so
    // |r2 - mid| < w holds on all of [R2_lo, R2_hi] and a little beyond, where
    // the FP64 test decides alike; that test runs only when some lane of the
    // wave is inside the band
    const bool band = fabsf(g.r2 - C.R2_mid) < C.R2_w;
    if (__builtin_amdgcn_ballot_w64(band)) acc = acc || (band && geom_r2d(g, C) < C.R2_d);
    return acc;
}

// ---------------------------------------------------------------------------
// Stencil codes.  An accepted neighbour is stored as one 32-bit word,
// (slot j << bits) | code, where the code gives what pair_geom needs besides
// the two records: the stencil offsets o (mixed precision, base 2S+1 digits)
// or the periodic images w (FP64, base 3 digits).
template <int DIM, int SR, typename T>
struct NbrCode {
    static constexpr int NR = 2 * SR + 1;
    static constexpr bool kFp64 = sizeof(T) == 8;
    static constexpr int kCodes = kFp64 ? (DIM == 3 ? 27 : 9) : (DIM == 3 ? NR * NR * NR : NR * NR);
    static constexpr int kBits = kCodes <= 16 ? 4 : (kCodes <= 32 ? 5 : (kCodes <= 64 ? 6 : 7));
    static constexpr uint32_t kMask = (1u << kBits) - 1u;
    // Largest particle count whose slots fit beside the code.
    static constexpr uint32_t kMaxN = 1u << (32 - kBits);

    // Part of the code fixed for one stencil row piece; the mixed-precision
    // code adds the candidate's own x offset.
    static __device__ __forceinline__ int row_base(int oy, int oz, int wx, int wy, int wz) {
        if (kFp64) return (wx + 1) + 3 * ((wy + 1) + (DIM == 3 ? 3 * (wz + 1) : 0));
        return SR + NR * ((oy + SR) + (DIM == 3 ? NR * (oz + SR) : 0));
    }
    static __device__ __forceinline__ uint32_t code(int base, int ox) {
        return kFp64 ? (uint32_t)base : (uint32_t)(base + ox);
    }
    template <typename R>
    static __device__ __forceinline__ Geom<T> geom(const R& ri, const R& rj, uint32_t c,
                                                   const PairConst<T>& C) {
        const int B = kFp64 ? 3 : NR, off = kFp64 ? 1 : SR;
        const int a = (int)(c % (uint32_t)B) - off;
        const uint32_t t = c / (uint32_t)B;
        const int b = (int)(t % (uint32_t)B) - off;
        const int d = DIM == 3 ? (int)(t / (uint32_t)B) - off : 0;
        return kFp64 ? pair_geom<DIM>(ri, rj, 0, 0, 0, a, b, d, C)
                     : pair_geom<DIM>(ri, rj, a, b, d, 0, 0, 0, C);
    }
};

// Neighbour lists are stored in tiles of 64 particles (one wave): entry k of
// sorted slot i at ((i / 64) cap + k) 64 + i % 64, so that the lanes of a
// wave read entry k of their 64 lists as one contiguous 256-byte row.
constexpr uint32_t kListTile = 64;
__device__ __forceinline__ size_t list_column(uint32_t i, uint32_t cap) {
    return ((size_t)(i / kListTile) * cap) * kListTile + (size_t)(i % kListTile);
}

// Keep a gathered 16-byte 2D record whole: with a use of every component
// the compiler loads it in one 16-byte access instead of narrowing it to the
// components a pass reads (x, y and w of a 2D position record become two
// gathers, and a component read only in a branch a third one, issued late).
// No code.  (Measured on the 512^2 step: momentum 23.5 -> 18.6 us.)  FP64
// records and 3D ones are left to the compiler: there whole loads only add
// bytes.
template <int DIM>
__device__ __forceinline__ void keep_whole(int4& r) {
    if (DIM == 2) asm("" : "+v"(r.x), "+v"(r.y), "+v"(r.z), "+v"(r.w));
}
template <int DIM>
__device__ __forceinline__ void keep_whole(float4& r) {
    if (DIM == 2) asm("" : "+v"(r.x), "+v"(r.y), "+v"(r.z), "+v"(r.w));
}
template <int DIM>
__device__ __forceinline__ void keep_whole(double4&) {}

// No per-candidate payload beyond the position record.
struct NoPayload {
    __device__ __forceinline__ int operator()(uint32_t) const { return 0; }
};

// The slot ranges of one stencil row: the cells cx-S .. cx+S of row `row`,
// split where a periodic x boundary wraps; piece k covers cells
// [first[k], last[k]] with periodic image wrap[k].  Pieces that do not exist
// are empty (first > last).
template <int S>
__device__ __forceinline__ void row_pieces(int cx, const Grid& G, int first[2], int last[2],
                                           int wrap[2]) {
    const int nc = G.nc[0];
    const int lo = cx - S, hi = cx + S;
    first[1] = 1;
    last[1] = 0;
    wrap[1] = 0;
    wrap[0] = 0;
    if (!G.periodic[0]) {
        first[0] = lo < 0 ? 0 : lo;
        last[0] = hi > nc - 1 ? nc - 1 : hi;
    } else if (lo < 0) {
        first[0] = lo + nc;
        last[0] = nc - 1;
        wrap[0] = -1;
        first[1] = 0;
        last[1] = hi;
    } else if (hi > nc - 1) {
        first[0] = lo;
        last[0] = nc - 1;
        first[1] = 0;
        last[1] = hi - nc;
        wrap[1] = 1;
    } else {
        first[0] = lo;
        last[0] = hi;
    }
}

// Cell walk: calls f(j, rec_j, payload_j, geom, code) for every sorted slot
// j with |r_ij|^2 < (2h)^2 in the (2S+1)^dim stencil cells of i's cell (self
// included), payload_j = load(j), code = j's stencil code.
//  * The cells of one stencil row are adjacent in memory (row-major keys), so
//    a row is walked as one slot range (two if it wraps a periodic x
//    boundary).  A candidate's x offset comes from its own sorted key:
//    ox = (cx_j - cx_i) + wrap nc.
//  * The ranges of all rows of a stencil plane are loaded before any
//    candidate; candidates are taken four at a time with their records and
//    payloads loaded ahead of the arithmetic, so each lane keeps several
//    independent loads in flight instead of one dependent chain.
template <int DIM, int S, typename T, typename Load, typename Fn>
__device__ __forceinline__ void walk_pairs(const Grid& G, const PairConst<T>& C, uint32_t key,
                                           const typename Rec<T>::type& ri,
                                           const typename Rec<T>::type* __restrict__ pos,
                                           const uint32_t* __restrict__ skey,
                                           const uint32_t* __restrict__ cstart,
                                           const uint32_t* __restrict__ cend, uint32_t n,
                                           Load&& load, Fn&& f) {
    using R = typename Rec<T>::type;
    using Code = NbrCode<DIM, S, T>;
    constexpr int NR = 2 * S + 1;
    int c[3];
    decode_key(key, G, c);
    if (DIM == 3 && G.order) {
        // Z-order keys: the cells of a stencil row are not adjacent in
        // memory, so each cell is a slot range of its own; same cell order
        // (rows in stencil order, x ascending) and the same codes
#pragma unroll 1
        for (int zi = 0; zi < NR; ++zi) {
            const int oz = zi - S;
            int cz, wz;
            if (!stencil_axis(c[2], oz, G.nc[2], G.periodic[2], &cz, &wz)) continue;
#pragma unroll 1
            for (int yi = 0; yi < NR; ++yi) {
                const int oy = yi - S;
                int cy, wy;
                if (!stencil_axis(c[1], oy, G.nc[1], G.periodic[1], &cy, &wy)) continue;
#pragma unroll 1
                for (int xi = 0; xi < NR; ++xi) {
                    const int ox = xi - S;
                    int cx, wx;
                    if (!stencil_axis(c[0], ox, G.nc[0], G.periodic[0], &cx, &wx)) continue;
                    const int cc[3] = {cx, cy, cz};
                    const uint32_t ck = cell_key(cc, G);
                    uint32_t e = cend[ck];
                    e = e < n ? e : n;
                    const int cb = Code::row_base(oy, oz, wx, wy, wz);
                    for (uint32_t j = cstart[ck]; j < e; ++j) {
                        const R rj = pos[j];
                        const auto pj = load(j);
                        const Geom<T> g = pair_geom<DIM>(ri, rj, ox, oy, oz, wx, wy, wz, C);
                        if (pair_accept(g, C)) f(j, rj, pj, g, Code::code(cb, ox));
                    }
                }
            }
        }
        return;
    }
    int first[2], last[2], wrap[2];
    row_pieces<S>(c[0], G, first, last, wrap);
#pragma unroll
    for (int zi = 0; zi < (DIM == 3 ? NR : 1); ++zi) {
        const int oz = DIM == 3 ? zi - S : 0;
        int cz = 0, wz = 0;
        if (DIM == 3 && !stencil_axis(c[2], oz, G.nc[2], G.periodic[2], &cz, &wz)) continue;
        // phase A: slot ranges of the rows of this plane
        uint32_t pb[NR][2], pe[NR][2], prow[NR];
        int pwy[NR];
#pragma unroll
        for (int yi = 0; yi < NR; ++yi) {
            int cy, wy;
            const bool ok = stencil_axis(c[1], yi - S, G.nc[1], G.periodic[1], &cy, &wy);
            const uint32_t row = (uint32_t)G.nc[0] * ((uint32_t)cy + (uint32_t)G.nc[1] * (uint32_t)cz);
            prow[yi] = row;
            pwy[yi] = wy;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                uint32_t b = 0, e = 0;
                if (ok && first[k] <= last[k]) {
                    b = cstart[row + (uint32_t)first[k]];
                    e = cend[row + (uint32_t)last[k]];
                    e = e < n ? e : n;
                }
                pb[yi][k] = b;
                pe[yi][k] = e;
            }
        }
        // phase B: the candidates, four at a time
#pragma unroll
        for (int yi = 0; yi < NR; ++yi) {
            const int oy = yi - S, wy = pwy[yi];
            const int xbase = (int)prow[yi] + c[0];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int wx = wrap[k];
                const int xoff = wx * G.nc[0] - xbase;
                const int cb = Code::row_base(oy, oz, wx, wy, wz);
                auto visit = [&](uint32_t j, const R& rj, const auto& pj, int ox) {
                    const Geom<T> g = pair_geom<DIM>(ri, rj, ox, oy, oz, wx, wy, wz, C);
                    if (pair_accept(g, C)) f(j, rj, pj, g, Code::code(cb, ox));
                };
                const uint32_t e = pe[yi][k];
                uint32_t j = pb[yi][k];
                // records and keys of the row through pointers, so that
                // consecutive candidates are immediate offsets of one address
                const R* __restrict__ pr = pos + j;
                const uint32_t* __restrict__ pk = skey + j;
                for (; j + 4 <= e; j += 4, pr += 4, pk += 4) {
                    const R r0 = pr[0], r1 = pr[1], r2 = pr[2], r3 = pr[3];
                    const int o0 = (int)pk[0] + xoff, o1 = (int)pk[1] + xoff;
                    const int o2 = (int)pk[2] + xoff, o3 = (int)pk[3] + xoff;
                    const auto p0 = load(j), p1 = load(j + 1), p2 = load(j + 2), p3 = load(j + 3);
                    visit(j, r0, p0, o0);
                    visit(j + 1, r1, p1, o1);
                    visit(j + 2, r2, p2, o2);
                    visit(j + 3, r3, p3, o3);
                }
                for (; j < e; ++j, ++pr, ++pk) {
                    const R rj = pr[0];
                    const int oj = (int)pk[0] + xoff;
                    const auto pj = load(j);
                    visit(j, rj, pj, oj);
                }
            }
        }
    }
}

// The neighbours of sorted slot i, in walk order: from its stored list when
// it holds all of them (cnt <= cap), else by the cell walk.  Calls
// f(j, rec_j, payload_j, geom) with the same geometry either way.
template <int DIM, int S, typename T, typename Load, typename Fn>
__device__ __forceinline__ void for_each_neighbor_p(
    int i, const Grid& G, const PairConst<T>& C, const typename Rec<T>::type& ri,
    const typename Rec<T>::type* __restrict__ pos, const uint32_t* __restrict__ skey,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, uint32_t n,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap,
    Load&& load, Fn&& f) {
    using R = typename Rec<T>::type;
    using Code = NbrCode<DIM, S, T>;
    const uint32_t cnt = list ? ncnt[i] : 0xffffffffu;
    if (cnt <= cap) {
        const uint32_t* __restrict__ col = list + list_column((uint32_t)i, cap);
        // slot of entry e (clamped into [0, n), which a current list never needs)
        auto slot = [&](uint32_t e) { return min(e >> Code::kBits, n - 1u); };
        // entry k, read within the particle's cap entries (values past cnt
        // are loaded ahead but never used)
        auto entry = [&](uint32_t k) { return col[min(k, cap - 1u) * kListTile]; };
        // groups of kGroup neighbours: their records are gathered together,
        // and the entries of the next group are loaded meanwhile
        constexpr uint32_t kGroup = 4;
        using P = decltype(load(0u));
        uint32_t q[kGroup];
#pragma unroll
        for (uint32_t u = 0; u < kGroup; ++u) q[u] = entry(u);
        uint32_t k = 0;
        for (; k + kGroup <= cnt; k += kGroup) {
            uint32_t jj[kGroup], cc[kGroup];
            R rr[kGroup];
            P pp[kGroup];
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) {
                jj[u] = slot(q[u]);
                cc[u] = q[u] & Code::kMask;
            }
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) {
                rr[u] = pos[jj[u]];
                keep_whole<DIM>(rr[u]);
            }
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) pp[u] = load(jj[u]);
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) q[u] = entry(k + kGroup + u);
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) f(jj[u], rr[u], pp[u], Code::geom(ri, rr[u], cc[u], C));
        }
        // fewer than kGroup entries left, already loaded: gathered together
        // too (unused ones read slot i's own, cached, records)
        {
            uint32_t jj[kGroup - 1];
            R rr[kGroup - 1];
            P pp[kGroup - 1];
#pragma unroll
            for (uint32_t u = 0; u + 1 < kGroup; ++u) jj[u] = k + u < cnt ? slot(q[u]) : (uint32_t)i;
#pragma unroll
            for (uint32_t u = 0; u + 1 < kGroup; ++u) {
                rr[u] = pos[jj[u]];
                keep_whole<DIM>(rr[u]);
            }
#pragma unroll
            for (uint32_t u = 0; u + 1 < kGroup; ++u) pp[u] = load(jj[u]);
#pragma unroll
            for (uint32_t u = 0; u + 1 < kGroup; ++u)
                if (k + u < cnt) f(jj[u], rr[u], pp[u], Code::geom(ri, rr[u], q[u] & Code::kMask, C));
        }
        return;
    }
    walk_pairs<DIM, S, T>(G, C, skey[i], ri, pos, skey, cstart, cend, n, load,
                          [&](uint32_t j, const R& rj, const auto& pj, const Geom<T>& g,
                              uint32_t) { f(j, rj, pj, g); });
}

// Neighbour loop without payload: f(j, rec_j, geom).
template <int DIM, int S, typename T, typename Fn>
__device__ __forceinline__ void for_each_neighbor(
    int i, const Grid& G, const PairConst<T>& C, const typename Rec<T>::type& ri,
    const typename Rec<T>::type* __restrict__ pos, const uint32_t* __restrict__ skey,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, uint32_t n,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap, Fn&& f) {
    for_each_neighbor_p<DIM, S, T>(i, G, C, ri, pos, skey, cstart, cend, n, list, ncnt, cap,
                                   NoPayload(),
                                   [&](uint32_t j, const typename Rec<T>::type& rj, int,
                                       const Geom<T>& g) { f(j, rj, g); });
}

// ---------------------------------------------------------------------------
// Lanes of the wave holding the same key (active lanes only): the group's
// leader lane, this lane's rank in the group (lane order) and the group size.
// The particles of a wave are consecutive in the previous sorted order, so a
// wave holds ~dim-dependent few distinct cells and the loop runs once per
// distinct key; one atomic per group replaces one per particle.
__device__ __forceinline__ void wave_group(uint32_t key, int* leader, int* rank, int* size) {
    const int lane = __lane_id();
    unsigned long long rem = __ballot(1);
    while (rem) {
        const int l = __ffsll((long long)rem) - 1;
        const uint32_t lk = __builtin_amdgcn_readlane(key, l);
        const unsigned long long m = __ballot(key == lk);
        if (key == lk) {
            *leader = l;
            *rank = __popcll(m & ((1ull << lane) - 1ull));
            *size = __popcll(m);
        }
        rem &= ~m;
    }
}

// ---------------------------------------------------------------------------
// Opening half kick + drift + periodic wrap of one particle (fluid only;
// walls keep x and get v = 0), then its cell key and one count for the sort:
//   v = u + dt/2 a;  x <- wrap(x + dt v);  key = cell(x);  counts[key] += 1.
// With drift = false only the key and count of the current x; with
// hash = false only the motion and the domain checks.
template <int DIM>
__device__ __forceinline__ void drift_and_hash(int i, const State& S, const Grid& G, bool fluid,
                                               const double* u, const double* a, double hdt,
                                               double dt, bool drift, uint32_t* __restrict__ key,
                                               uint32_t* __restrict__ counts,
                                               uint32_t* __restrict__ flags, bool hash = true,
                                               const double* x_in = nullptr) {
#pragma clang fp contract(off)
    bool outside = false, nonfinite = false;
    int c[3] = {0, 0, 0};
    for (int k = 0; k < DIM; ++k) {
        double x = x_in ? x_in[k] : S.x[k][i];
        if (drift) {
            double v = 0.0;
            if (fluid) {
                v = u[k] + hdt * a[k];
                x = x + dt * v;
                if (G.periodic[k]) {
                    const double hi = G.lo[k] + G.L[k];
                    double y = x - G.L[k] * floor((x - G.lo[k]) / G.L[k]);
                    if (y >= hi) y = G.lo[k];
                    x = y;
                }
                S.x[k][i] = x;
            }
            S.u[k][i] = v;
            nonfinite |= !isfinite(v);
        }
        nonfinite |= !isfinite(x);
        c[k] = cell_coord(x, G, k, &outside);
    }
    if (outside) atomicOr(flags, kFlagOutside);
    if (nonfinite) atomicOr(flags, kFlagNonFinite);
    if (!hash) return;
    const uint32_t kk = cell_key(c, G);
    key[i] = kk;
    int leader = 0, rank = 0, size = 1;
    wave_group(kk, &leader, &rank, &size);
    if (rank == 0) atomicAdd(&counts[kk], (uint32_t)size);
}

// Standalone hash (first step of a call, or a plain sort).
// kick_rho: the opening half kick of the continuity scheme's density,
// rho <- rho + dt/2 arho, for every particle.
template <int DIM, typename TA>
__global__ __launch_bounds__(kBlock) void k_drift_hash(int n, State S, Grid G, double hdt,
                                                       double dt, int drift, int kick_rho,
                                                       uint32_t* __restrict__ key,
                                                       uint32_t* __restrict__ counts,
                                                       uint32_t* __restrict__ flags) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double u[3] = {0.0, 0.0, 0.0}, a[3] = {0.0, 0.0, 0.0};
    if (drift)
        for (int k = 0; k < DIM; ++k) {
            u[k] = S.u[k][i];
            a[k] = (double)((const TA*)S.a[k])[i];
        }
    if (drift && kick_rho)
        store_rho<TA>(S.rho, i, load_rho<TA>(S.rho, i, S.rho64) + hdt * S.arho[i], S.rho64);
    drift_and_hash<DIM>(i, S, G, S.type[i] == 0, u, a, hdt, dt, drift != 0, key, counts, flags);
}

// Block sum of up to four FP64 values per thread into part[q * nparts + b]
// (fixed tree order).
template <int NV>
__device__ __forceinline__ void block_sum4(const double* v, double* __restrict__ part, int b,
                                           int nparts) {
    __shared__ double sh[NV][kBlock];
    for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) part[(int64_t)q * nparts + b] = sh[q][0];
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one value per thread (256 threads, wave64).
template <typename V>
__device__ __forceinline__ V block_exclusive_scan(V v, V* total) {
    __shared__ V wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    V incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const V o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    V before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) {
        before += k < w ? wsum[k] : V(0);
        all += wsum[k];
    }
    __syncthreads();
    if (total) *total = all;
    return before + incl - v;
}

// Sum of each chunk of kBlock * ITEMS input counts.
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_chunk_sum(const uint32_t* __restrict__ in, int64_t n,
                                                      uint64_t* __restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * (kBlock * ITEMS) + (int64_t)threadIdx.x * ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    uint64_t tot;
    block_exclusive_scan<uint64_t>(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of the input counts: out[i] = sum_{k<i} in[k], out[n] = total.
template <typename OUT, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_chunk_scan(const uint32_t* __restrict__ in, int64_t n,
                                                       const uint64_t* __restrict__ sums,
                                                       OUT* __restrict__ out) {
    // offset of this chunk: sum of the chunk sums before it
    uint64_t off = 0;
    for (int c = threadIdx.x; c < (int)blockIdx.x; c += kBlock) off += sums[c];
    uint64_t offtot;
    block_exclusive_scan<uint64_t>(off, &offtot);
    const int64_t base = (int64_t)blockIdx.x * (kBlock * ITEMS) + (int64_t)threadIdx.x * ITEMS;
    uint32_t v[ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint64_t chunk_total;
    uint64_t run = offtot + block_exclusive_scan<uint64_t>(s, &chunk_total);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (base + k < n) out[base + k] = (OUT)run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (OUT)(offtot + chunk_total);
}

// Scatter particles into their cell's slot range; counts return to zero.
static __global__ __launch_bounds__(kBlock) void k_scatter(int n, const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ counts,
                                                    uint32_t* __restrict__ tmp) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    int leader = 0, rank = 0, size = 1;
    wave_group(k, &leader, &rank, &size);
    uint32_t old = 0;
    if (rank == 0) old = atomicSub(&counts[k], (uint32_t)size);
    old = (uint32_t)__shfl((int)old, leader, 64);
    // the group takes slots [start + old - size, start + old)
    tmp[start[k] + old - (uint32_t)size + (uint32_t)rank] = (uint32_t)i;
}

// Stable order inside each cell: slot s holds particle i = tmp[s]; its final
// slot is start[key] + (number of particles of the same cell with a smaller
// index).  Gathers the state into that slot and packs the pair records
// (with eos, also rho and the EOS records of the continuity scheme).
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_rank_gather(int n, const uint32_t* __restrict__ tmp,
                                                        const uint32_t* __restrict__ key,
                                                        const uint32_t* __restrict__ start,
                                                        State src, State dst, Grid G,
                                                        uint32_t* __restrict__ perm,
                                                        uint32_t* __restrict__ skey,
                                                        typename Rec<T>::type* __restrict__ pos,
                                                        typename Vec4<T>::type* __restrict__ vel,
                                                        int copy_derived,
                                                        uint8_t* __restrict__ type_tape,
                                                        PairConst<T> C,
                                                        typename Vec2<T>::type* __restrict__ rp,
                                                        int eos, double predict) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const uint32_t i = tmp[s];
    const uint32_t k = key[i];
    const uint32_t b = start[k], e = start[k + 1];
    uint32_t rank = 0;
    for (uint32_t t = b; t < e; ++t) rank += tmp[t] < i ? 1u : 0u;
    const uint32_t d = b + rank;
    perm[d] = i;
    skey[d] = k;
    int c[3];
    decode_key(k, G, c);
    double xs[3] = {0.0, 0.0, 0.0};
    T vv[3] = {T(0), T(0), T(0)};
    for (int q = 0; q < DIM; ++q) {
        const double x = src.x[q][i];
        const double u = src.u[q][i];
        dst.x[q][d] = x;
        dst.u[q][d] = u;
        if (copy_derived) ((T*)dst.a[q])[d] = ((const T*)src.a[q])[i];
        xs[q] = x;
        // with predict, the pair records carry u + predict a (the predicted
        // end-of-step velocity of the continuity scheme's corrector)
        vv[q] = predict != 0.0 ? (T)(u + predict * (double)((const T*)src.a[q])[i]) : (T)u;
    }
    const double m = src.m[i];
    dst.m[d] = m;
    const uint8_t ty = src.type[i];
    dst.type[d] = ty;
    if (type_tape) type_tape[d] = ty;
    dst.id[d] = src.id[i];
    if (copy_derived) {
        store_rho<T>(dst.rho, d, load_rho<T>(src.rho, i, src.rho64), dst.rho64);
        ((T*)dst.p)[d] = ((const T*)src.p)[i];
        if (src.arho && dst.arho) dst.arho[d] = src.arho[i];
    }
    typename Vec2<T>::type v2;
    v2.x = T(0);
    v2.y = T(0);
    if (eos) {
        // density is a state (continuity scheme): gather it, and the EOS
        // (eq. eos) gives p and P = p / rho^2, in FP64 as in the density pass,
        // at rho + predict arho (the predicted end-of-step density)
        const double rho = load_rho<T>(src.rho, i, src.rho64);
        const double rs = predict != 0.0 ? rho + predict * src.arho[i] : rho;
        const double p = tait64<T>(rs, C);
        store_rho<T>(dst.rho, d, rho, dst.rho64);
        ((T*)dst.p)[d] = (T)p;
        v2.x = (T)rs;
        v2.y = (T)(p / (rs * rs));
        if (DIM == 3) rp[d] = v2;
    }
    // in 2D the (rho, P) record rides in z, w: zero here unless the EOS
    // above formed it (the density pass fills it otherwise)
    typename Vec4<T>::type vr;
    vr.x = vv[0]; vr.y = vv[1];
    vr.z = DIM == 2 ? v2.x : vv[2];
    vr.w = DIM == 2 ? v2.y : T(0);
    pos[d] = make_rec<T>(xs, c, m, (int)ty, G, DIM);
    vel[d] = vr;
}

// Pack pair records of an already sorted state (standalone evaluations):
// key = cell of x, the position record, (u), and (rho, p/rho^2) if with_rp.
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_pack(int n, State S, Grid G,
                                                 uint32_t* __restrict__ skey,
                                                 typename Rec<T>::type* __restrict__ pos,
                                                 typename Vec4<T>::type* __restrict__ vel,
                                                 typename Vec2<T>::type* __restrict__ rp,
                                                 int with_rp) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    bool outside = false;
    int c[3] = {0, 0, 0};
    double xs[3] = {0.0, 0.0, 0.0};
    T vv[3] = {T(0), T(0), T(0)};
    for (int q = 0; q < DIM; ++q) {
        const double x = S.x[q][i];
        c[q] = cell_coord(x, G, q, &outside);
        xs[q] = x;
        vv[q] = (T)S.u[q][i];
    }
    skey[i] = cell_key(c, G);
    typename Vec4<T>::type vr;
    vr.x = vv[0]; vr.y = vv[1]; vr.z = vv[2]; vr.w = T(0);
    pos[i] = make_rec<T>(xs, c, S.m[i], (int)S.type[i], G, DIM);
    vel[i] = vr;
    if (with_rp) {
        const T rho = (T)load_rho<T>(S.rho, i, S.rho64);
        const T p = ((const T*)S.p)[i];
        typename Vec2<T>::type v2;
        v2.x = rho;
        v2.y = p / (rho * rho);
        store_rp<DIM, T>(vel, rp, (uint32_t)i, v2);
    }
}

// ---------------------------------------------------------------------------
// Density epilogue: rho from the sum of density_add (in mixed precision
// the sum of m_j w_ij, scaled here by sigma; in FP64 the sum of m_j W_ij
// itself), stored with, if with_eos, p and (rho, P = p / rho^2), computed
// in FP64 and rounded to the pair type.
template <int DIM, typename T>
__device__ __forceinline__ void finish_density(int i, double wsum, const PairConst<T>& C,
                                               void* __restrict__ rho_out, int rho64,
                                               T* __restrict__ p_out,
                                               typename Vec4<T>::type* __restrict__ vel,
                                               typename Vec2<T>::type* __restrict__ rp,
                                               int with_eos) {
    const double rho = sizeof(T) == 8 ? wsum : C.sigma_d * wsum;  // see density_add
    store_rho<T>(rho_out, i, rho, rho64);
    if (with_eos) {
        const double p = tait64<T>(rho, C);
        p_out[i] = (T)p;
        typename Vec2<T>::type v2;
        v2.x = (T)rho;
        v2.y = (T)(p / (rho * rho));
        store_rp<DIM, T>(vel, rp, (uint32_t)i, v2);
    }
}

// Uniform copies of lane t's values (t the same on every lane).
__device__ __forceinline__ int lane_bcast(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ __forceinline__ double lane_bcast(double v, int t) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), t);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), t);
    return __hiloint2double(hi, lo);
}
template <int DIM>
__device__ __forceinline__ int4 rec_bcast(const int4& r, int t) {
    int4 o;
    o.x = lane_bcast(r.x, t);
    o.y = lane_bcast(r.y, t);
    o.z = DIM == 3 ? lane_bcast(r.z, t) : 0;
    o.w = 0;
    return o;
}
template <int DIM>
__device__ __forceinline__ double4 rec_bcast(const double4& r, int t) {
    double4 o;
    o.x = lane_bcast(r.x, t);
    o.y = lane_bcast(r.y, t);
    o.z = DIM == 3 ? lane_bcast(r.z, t) : 0.0;
    o.w = 0.0;
    return o;
}

// Adds a block's interaction count to its own counter pairs[blk] (plain
// read-modify-write: each block owns its slot and launches are stream
// ordered); block 0 raises pairs[-1], the number of counters the reader sums,
// to at least the grid size.
__device__ __forceinline__ void add_pairs(unsigned long long* __restrict__ pairs, int blk,
                                          unsigned long long t) {
    pairs[blk] += t;
    if (blk == 0 && pairs[-1] < (unsigned long long)gridDim.x)
        pairs[-1] = (unsigned long long)gridDim.x;
}

// Block-wide sum of a per-thread count into the block's counter (kBlock
// threads).
__device__ __forceinline__ void block_count(uint32_t cnt, unsigned long long* __restrict__ pairs,
                                            int blk) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    __shared__ uint32_t wcnt[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wcnt[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += wcnt[w];
        add_pairs(pairs, blk, t);
    }
}

// Coordinates of the list builder's filter test, in FP32, relative to the
// centre of the target cell c: the target's position, and the position of
// candidate j's image for stencil offset o / periodic image w.  Their
// difference is r_ij to within ~1e-6 of a cell (conversion and subtraction
// roundings), well inside the +-1e-5 band of (2h)^2 around which the exact
// FP64 predicate decides.
__device__ __forceinline__ float filt_target(const int4& r, int k, const PairConst<float>& C,
                                             double) {
    return (float)(k == 0 ? r.x : (k == 1 ? r.y : r.z)) * C.fix_scale_f[k];
}
__device__ __forceinline__ float filt_cand(const int4& r, int k, int o, int,
                                           const PairConst<float>& C, double) {
    const int v = (k == 0 ? r.x : (k == 1 ? r.y : r.z)) + o * (1 << kFixBits);
    return (float)v * C.fix_scale_f[k];
}
__device__ __forceinline__ float filt_target(const double4& r, int k, const PairConst<double>&,
                                             double centre) {
    return (float)((k == 0 ? r.x : (k == 1 ? r.y : r.z)) - centre);
}
__device__ __forceinline__ float filt_cand(const double4& r, int k, int, int w,
                                           const PairConst<double>& C, double centre) {
    const double v = k == 0 ? r.x : (k == 1 ? r.y : r.z);
    return (float)((v + (w == 0 ? 0.0 : (w < 0 ? -C.L[k] : C.L[k]))) - centre);
}

// v_writelane: value into lane `lane` of old (the other lanes keep theirs).
__device__ int amdgcn_writelane_i32(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t lane_write(uint32_t value, int lane, uint32_t old) {
    return (uint32_t)amdgcn_writelane_i32((int)value, lane, (int)old);
}

// Neighbour lists of all particles (Sec. 2.2), built cell by cell.  Wave w
// takes per_wave (<= 64) consecutive cells from w per_wave on (dense grids),
// or, with by_slots, the cells whose first sorted slot lies in
// [w per_wave, (w + 1) per_wave): one load of the slots' keys and a ballot of
// the cell starts name them, so the work follows the particles and empty
// cells cost nothing however sparse the grid.  Per cell:
//  * Lane s < number of stencil segments (z row, y row, x piece) loads the
//    slot range of segment s, and lane t the record of the cell's target t,
//    all in one round of loads; the loops below read them with readlane.
//  * The lanes take the candidates of the non-empty segments 64 at a time,
//    in walk order (segments in order, ascending slots), with coalesced loads
//    of their records, and test each candidate against every target in
//    turn: an FP32 filter on cell-relative coordinates decides outside a
//    band of +-1e-5 around (2h)^2, the exact FP64 predicate of walk_pairs
//    inside it (and for coordinates too far from the cell for the filter's
//    error bound), so the accepted set is exactly the walk's.  A ballot over
//    the lanes hands each target its accepted candidates in walk order,
//    appended to its list with one store.
// So every candidate record is loaded once per cell instead of once per
// target, and the lists are those of walk_pairs, entry for entry.  Entries
// beyond cap are not stored; ncnt[i] holds the full count, and a count above
// cap tells the pair kernels to walk the cells for that particle.  With
// count_pairs, the number of interactions |N(i)| is added to the block's own
// 64-bit counter pairs[block]: each block owns its slot (plain
// read-modify-write, no atomics; launches are stream-ordered), and block 0
// records the number of counters in pairs[-1] so that the reader can sum
// them.
template <int DIM, int SR, typename T>
__global__ __launch_bounds__(kBlock) void k_nlist(int n, uint32_t ncells, uint32_t per_wave,
                                                  int by_slots, Grid G, PairConst<T> C,
                                                  const uint32_t* __restrict__ skey,
                                                  const typename Rec<T>::type* __restrict__ pos,
                                                  const uint32_t* __restrict__ cstart,
                                                  const uint32_t* __restrict__ cend, uint32_t cap,
                                                  uint32_t* __restrict__ list,
                                                  uint32_t* __restrict__ ncnt, int count_pairs,
                                                  unsigned long long* __restrict__ pairs) {
    using R = typename Rec<T>::type;
    using Code = NbrCode<DIM, SR, T>;
    constexpr bool kFp64 = sizeof(T) == 8;
    constexpr int NR = 2 * SR + 1;
    constexpr int kSegs = (DIM == 3 ? NR : 1) * NR * 2;
    static_assert(kSegs <= 64, "one lane per stencil segment");
    const int lane = (int)(threadIdx.x & 63);
    const int blk = xcd_block();
    const uint64_t wave = (uint64_t)blk * (kBlock / 64) + (threadIdx.x >> 6);
    // this wave's cells, one per lane: lane l takes cell w per_wave + l, or
    // the cell that starts at slot w per_wave + l, if any
    const uint64_t idx = wave * per_wave + (uint64_t)lane;
    uint32_t lkey = 0;
    bool has = false;
    if ((uint32_t)lane < per_wave) {
        if (by_slots) {
            if (idx < (uint64_t)n) {
                lkey = skey[idx];
                has = idx == 0 || skey[idx - 1] != lkey;
            }
        } else if (idx < (uint64_t)ncells) {
            lkey = (uint32_t)idx;
            has = true;
        }
    }
    unsigned long long rest = __ballot(has);
    // stencil position of lane s's segment
    const int sk = lane & 1, syi = (lane >> 1) % NR, szi = (lane >> 1) / NR;
    const int soy = syi - SR, soz = DIM == 3 ? szi - SR : 0;
    // FP64 records far from the cell (outside the box) take the exact test;
    // "far" is four cell sizes summed over the used axes (the unused z axis
    // of a 2D grid has a placeholder size)
    const float far = (float)(4.0 * (G.cs[0] + G.cs[1] + (DIM == 3 ? G.cs[2] : 0.0)));
    // Slot ranges of cell c (tb, te: the targets; lane s: segment s) and the
    // segments' packed stencil data (oy, oz, wx, wy, wz as 3-bit fields, the
    // code base above them) and x offset terms.  The loads of the next cell
    // are issued before the current one is processed.
    struct Ranges {
        uint32_t tb, te, sb, se;
        int meta, xoff;
    };
    auto load_ranges = [&](uint32_t c, Ranges& Rg) {
        int cc[3];
        decode_key(c, G, cc);
        int first[2], last[2], wrap[2];
        row_pieces<SR>(cc[0], G, first, last, wrap);
        int cz = 0, wz = 0, cy = 0, wy = 0;
        bool ok = lane < kSegs;
        if (DIM == 3) ok = ok && stencil_axis(cc[2], soz, G.nc[2], G.periodic[2], &cz, &wz);
        ok = ok && stencil_axis(cc[1], soy, G.nc[1], G.periodic[1], &cy, &wy);
        const int fk = sk ? first[1] : first[0], lk = sk ? last[1] : last[0];
        ok = ok && fk <= lk;
        const int wx = sk ? wrap[1] : wrap[0];
        const uint32_t row = (uint32_t)G.nc[0] * ((uint32_t)cy + (uint32_t)G.nc[1] * (uint32_t)cz);
        Rg.sb = 0;
        Rg.se = 0;
        if (ok) {
            Rg.sb = cstart[row + (uint32_t)fk];
            Rg.se = cend[row + (uint32_t)lk];
        }
        Rg.tb = cstart[c];
        Rg.te = cend[c];
        Rg.xoff = wx * G.nc[0] - (int)row - cc[0];
        Rg.meta = (soy + 2) | ((soz + 2) << 3) | ((wx + 2) << 6) | ((wy + 2) << 9) |
                  ((wz + 2) << 12) | (Code::row_base(soy, soz, wx, wy, wz) << 15);
    };
    uint32_t total = 0;
    Ranges cur{}, nxt{};
    // each pass consumes one bit of rest, so the loop ends within 64 passes
    int bit = -1;
    if (rest) {
        bit = __ffsll((long long)rest) - 1;
        rest &= rest - 1ull;
        load_ranges(__builtin_amdgcn_readlane(lkey, bit), cur);
    }
    while (bit >= 0) {
        const uint32_t c = __builtin_amdgcn_readlane(lkey, bit);
        int nbit = -1;
        if (rest) {
            nbit = __ffsll((long long)rest) - 1;
            rest &= rest - 1ull;
            load_ranges(__builtin_amdgcn_readlane(lkey, nbit), nxt);
        }
        bit = nbit;
        const uint32_t tb = __builtin_amdgcn_readfirstlane(cur.tb);
        uint32_t te = __builtin_amdgcn_readfirstlane(cur.te);
        te = te < (uint32_t)n ? te : (uint32_t)n;
        const uint32_t sb = cur.sb, se = cur.se < (uint32_t)n ? cur.se : (uint32_t)n;
        const int smeta = cur.meta, sxoff = cur.xoff;
        cur = nxt;
        if (tb >= te) continue;
        int cc[3];
        decode_key(c, G, cc);
        double centre[3];
        for (int k = 0; k < 3; ++k) centre[k] = G.lo[k] + ((double)cc[k] + 0.5) * G.cs[k];
        const unsigned long long segs = __ballot(sb < se);  // non-empty segments
        for (uint32_t g0 = tb; g0 < te; g0 += 64) {  // targets, 64 at a time
            const uint32_t nt = te - g0 < 64u ? te - g0 : 64u;
            const R tr = pos[g0 + ((uint32_t)lane < nt ? (uint32_t)lane : 0u)];
            float tf[3];
            bool tfar = false;
            for (int k = 0; k < DIM; ++k) {
                tf[k] = filt_target(tr, k, C, centre[k]);
                tfar |= kFp64 && !(fabsf(tf[k]) < far);
            }
            // with a far target in the group, every pair takes the exact test
            const bool gfar = kFp64 && __ballot(tfar && (uint32_t)lane < nt) != 0ull;
            uint32_t cntv = 0;  // lane t: count of target g0 + t
            // lane t: byte offset of target g0 + t's column in the list (entry
            // k of slot u at u + 64 (k + (u / 64)(cap - 1)) words; the host
            // keeps the list below 4 GiB for this kernel)
            const uint32_t ul = g0 + (uint32_t)lane;
            const uint32_t colv = 4u * ((ul / kListTile) * cap * kListTile + ul % kListTile);
            // this lane's candidate in the current chunk and its stencil data
            uint32_t cj = 0;
            int valid = 0, cmeta = 0, cxoff = 0;
            uint32_t fill = 0;
            auto process = [&]() {
                const R rj = pos[cj];
                const int ox = kFp64 ? 0 : (int)skey[cj] + cxoff;
                const int oy = (cmeta & 7) - 2, oz = ((cmeta >> 3) & 7) - 2;
                const int wx = ((cmeta >> 6) & 7) - 2, wy = ((cmeta >> 9) & 7) - 2;
                const int wz = ((cmeta >> 12) & 7) - 2;
                const uint32_t word = (cj << Code::kBits) | Code::code(cmeta >> 15, ox);
                const int o[3] = {ox, oy, oz}, w[3] = {wx, wy, wz};
                float cf[3];
                bool cfar = false;
                for (int k = 0; k < DIM; ++k) {
                    cf[k] = filt_cand(rj, k, o[k], w[k], C, centre[k]);
                    cfar |= kFp64 && !(fabsf(cf[k]) < far);
                }
                const bool exact_all = valid && (cfar || gfar);
                // a lane without a candidate is infinitely far from every
                // target, so neither test below accepts it
                if (!valid) cf[0] = __builtin_huge_valf();
                for (uint32_t t = 0; t < nt; ++t) {
                    // target t's coordinates, read from its lane
                    auto tcoord = [&](int k) {
                        return __int_as_float(
                            __builtin_amdgcn_readlane(__float_as_int(tf[k]), (int)t));
                    };
                    const float dx = tcoord(0) - cf[0], dy = tcoord(1) - cf[1];
                    float r2 = dx * dx + dy * dy;
                    if (DIM == 3) {
                        const float dz = tcoord(2) - cf[2];
                        r2 += dz * dz;
                    }
                    // accepted lanes: below the band, or inside it (or far) and
                    // accepted by the exact predicate.  r2 - mid is exact near
                    // the band (Sterbenz), so |r2 - mid| < w holds on all of
                    // [R2_lo, R2_hi] and a little beyond, where the exact test
                    // decides alike.  The mask is taken from the compare itself
                    // (no per-lane flag to convert) unless the band needs the
                    // exact test.
                    bool acc = r2 < C.R2_lo;
                    unsigned long long m = __builtin_amdgcn_ballot_w64(r2 < C.R2_lo);
                    const bool band = exact_all || fabsf(r2 - C.R2_mid) < C.R2_w;
                    if (__builtin_amdgcn_ballot_w64(band)) {
                        const R ri = rec_bcast<DIM>(tr, (int)t);
                        const Geom<T> gm = pair_geom<DIM>(ri, rj, ox, oy, oz, wx, wy, wz, C);
                        acc = acc || (band && geom_r2d(gm, C) < C.R2_d);
                        m = __builtin_amdgcn_ballot_w64(acc);
                    }
                    // entry k of target t, written by the accepted lane of rank
                    // k - base; the count kept in lane t
                    const uint32_t base = __builtin_amdgcn_readlane(cntv, t);
                    const uint32_t colb = __builtin_amdgcn_readlane(colv, t);
                    const uint32_t k = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base));
                    if (acc && k < cap)
                        *(uint32_t*)((char*)list + (colb + k * (uint32_t)(4 * kListTile))) = word;
                    cntv = lane_write(base + (uint32_t)__popcll(m), (int)t, cntv);
                }
                valid = 0;
                fill = 0;
            };
            for (unsigned long long rest = segs; rest; rest &= rest - 1ull) {
                const int seg = __ffsll((long long)rest) - 1;
                uint32_t b = __builtin_amdgcn_readlane(sb, seg);
                const uint32_t e = __builtin_amdgcn_readlane(se, seg);
                const int meta = __builtin_amdgcn_readlane(smeta, seg);
                const int xoff = __builtin_amdgcn_readlane(sxoff, seg);
                while (b < e) {
                    const uint32_t take = e - b < 64u - fill ? e - b : 64u - fill;
                    if ((uint32_t)lane >= fill && (uint32_t)lane < fill + take) {
                        cj = b + ((uint32_t)lane - fill);
                        valid = 1;
                        cmeta = meta;
                        cxoff = xoff;
                    }
                    fill += take;
                    b += take;
                    if (fill == 64u) process();
                }
            }
            if (fill) process();
            if ((uint32_t)lane < nt) {
                ncnt[g0 + (uint32_t)lane] = cntv;
                total += cntv;
            }
        }
    }
    if (count_pairs) block_count(total, pairs, blk);
}

// Neighbour lists of all particles (Sec. 2.2), one particle per lane: the
// cell walk of walk_pairs, each accepted neighbour (self included) stored as
// (j << bits) | code while the list has room; ncnt[i] = the full count.
// Interaction counters as in k_nlist.
template <int DIM, int SR, typename T>
__global__ __launch_bounds__(kBlock) void k_nlist_walk(int n, Grid G, PairConst<T> C,
                                                       const uint32_t* __restrict__ skey,
                                                       const typename Rec<T>::type* __restrict__ pos,
                                                       const uint32_t* __restrict__ cstart,
                                                       const uint32_t* __restrict__ cend,
                                                       uint32_t cap, uint32_t* __restrict__ list,
                                                       uint32_t* __restrict__ ncnt, int count_pairs,
                                                       unsigned long long* __restrict__ pairs) {
    using R = typename Rec<T>::type;
    const int blk = xcd_block();
    const int i = blk * kBlock + threadIdx.x;
    uint32_t cnt = 0;
    if (i < n) {
        const R ri = pos[i];
        uint32_t* __restrict__ col = list + list_column((uint32_t)i, cap);
        walk_pairs<DIM, SR, T>(G, C, skey[i], ri, pos, skey, cstart, cend, (uint32_t)n,
                               NoPayload(),
                               [&](uint32_t j, const R&, int, const Geom<T>&, uint32_t code) {
                                   if (cnt < cap)
                                       col[cnt * kListTile] =
                                           (j << NbrCode<DIM, SR, T>::kBits) | code;
                                   ++cnt;
                               });
        ncnt[i] = cnt;
    }
    if (count_pairs) block_count(cnt, pairs, blk);
}

// Pair terms shared by the list, walk and tile passes (one definition, so the
// paths round alike; multiply-adds are fused within each statement only).
//
// Summation density (eq. 2), FP64 terms in both precisions.  Mixed
// precision: acc += m_j w(|r_ij|), the kernel without its normalisation
// sigma (finish_density scales the sum), Wendland's factors straight from
// r.  FP64: acc += m_j W(q) with q = |r_ij|/h, the normalised kernel; in
// the FP64 list pass this form keeps the kernel at 96 registers (five
// waves per SIMD), the other measured 10% slower there.
template <int KERNEL, typename T>
__device__ __forceinline__ void density_add(double& acc, const Geom<T>& g, double mj,
                                            const PairConst<T>& C) {
    const double r = density_sqrt(geom_r2d(g, C), T(0));
    if constexpr (sizeof(T) == 8)
        acc += mj * kernel_w<KERNEL, double>(r * C.inv_h_d, C.sigma_d);
    else
        acc += mj * kernel_w_r<KERNEL, T>(r, C);
}

// Momentum terms of pair (i, j) (eqs. mom:sph:press, mom:sph:visc):
//   a_i += m_j [ -(P_i + P_j) F r_ij + 4 nu/(rho_i+rho_j) F |r|^2/(|r|^2 + eta h^2) v_ij ]
// with F = (dW/dr)/r.  The self pair (j = i) is not skipped: r = 0 and
// v_i - v_i = 0 multiply finite factors (F is finite at r = 0, and the
// viscous factor holds |r|^2 = 0 over a positive denominator in FP32 and
// is set to 0 by a select in FP64, the faster form in each), so it adds
// exactly zero.
template <int DIM, int KERNEL, typename T>
__device__ __forceinline__ void momentum_add(T& ax, T& ay, T& az, const Geom<T>& g, T mj,
                                             const typename Vec4<T>::type& vi,
                                             const typename Vec2<T>::type& rpi,
                                             const typename Vec4<T>::type& vj,
                                             const typename Vec2<T>::type& rpj,
                                             const PairConst<T>& C) {
    const T r2 = g.r2;
    const T F = kernel_f_r2<KERNEL, T>(r2, C);
    const T pres = -(rpi.y + rpj.y) * F;
    T visc = C.four_nu * F * r2 * p_rcp((rpi.x + rpj.x) * (r2 + C.eta_h2));
    if constexpr (sizeof(T) == 8) visc = r2 > T(0) ? visc : T(0);
    // m_j folded into the two factors once per pair; each component takes
    // two multiply-adds, the pressure term first
    const T mp = mj * pres, mv = mj * visc;
    ax += mp * g.d[0];
    ax += mv * (vi.x - vj.x);
    ay += mp * g.d[1];
    ay += mv * (vi.y - vj.y);
    if (DIM == 3) {
        az += mp * g.d[2];
        az += mv * (vi.z - vj.z);
    }
}

// Summation density (eq. 2) of sorted slot i and, if with_eos, the Tait EOS
// (eq. eos) with P = p / rho^2 packed for the momentum pass, over its
// neighbour list (or the cell walk).  Returns |N(i)|.
template <int DIM, int SR, int KERNEL, typename T>
__device__ __forceinline__ uint32_t density_one(
    int i, const Grid& G, const PairConst<T>& C, const uint32_t* __restrict__ skey,
    const typename Rec<T>::type* __restrict__ pos, const uint32_t* __restrict__ cstart,
    const uint32_t* __restrict__ cend, int n, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ ncnt, uint32_t cap, void* __restrict__ rho_out, int rho64,
    T* __restrict__ p_out, typename Vec4<T>::type* __restrict__ vel,
    typename Vec2<T>::type* __restrict__ rp, int with_eos) {
    const typename Rec<T>::type ri = pos[i];
    // The density terms are FP64 in both precisions: the EOS multiplies
    // density rounding by ~7 B / rho0 before it reaches the forces.
    double acc = 0.0;
    uint32_t cnt = 0;
    for_each_neighbor<DIM, SR, T>(i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, list, ncnt,
                                  cap,
                                  [&](uint32_t, const typename Rec<T>::type& rj, const Geom<T>& g) {
                                      density_add<KERNEL, T>(acc, g, (double)rec_mass(rj), C);
                                      ++cnt;
                                  });
    finish_density<DIM, T>(i, acc, C, rho_out, rho64, p_out, vel, rp, with_eos);
    return cnt;
}

// Summation density over the neighbour lists (or the cell walk).  Without
// lists (list == nullptr) and with count_pairs, the number of interactions
// |N(i)| is added to the block's own counter pairs[block] as the list build
// does otherwise.
template <int DIM, int SR, int KERNEL, typename T>
__global__ __launch_bounds__(kBlock) void k_density(int n, Grid G, PairConst<T> C,
                                                    const uint32_t* __restrict__ skey,
                                                    const typename Rec<T>::type* __restrict__ pos,
                                                    const uint32_t* __restrict__ cstart,
                                                    const uint32_t* __restrict__ cend,
                                                    const uint32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ ncnt,
                                                    uint32_t cap, void* __restrict__ rho_out,
                                                    int rho64, T* __restrict__ p_out,
                                                    typename Vec4<T>::type* __restrict__ vel,
                                                    typename Vec2<T>::type* __restrict__ rp,
                                                    int with_eos, int count_pairs,
                                                    unsigned long long* __restrict__ pairs) {
    const int blk = xcd_block();
    const int i = blk * kBlock + threadIdx.x;
    uint32_t cnt = 0;
    if (i < n)
        cnt = density_one<DIM, SR, KERNEL, T>(i, G, C, skey, pos, cstart, cend, n, list, ncnt, cap,
                                              rho_out, rho64, p_out, vel, rp, with_eos);
    if (count_pairs) block_count(cnt, pairs, blk);
}

// Per-particle state that momentum_close reads (u; x when it drifts; m for
// the diagnostics), loaded by close_load: the tile pass loads it before its
// pair loop so that the loads' latency hides behind the loop (the list and
// walk passes let momentum_close load it, which keeps their registers as
// they were).
struct CloseIn {
    double u[3], x[3], m;
};
template <int DIM>
__device__ __forceinline__ CloseIn close_load(int i, const State& S, int drift, bool diag) {
    CloseIn c;
    for (int k = 0; k < 3; ++k) c.u[k] = c.x[k] = 0.0;
    for (int k = 0; k < DIM; ++k) {
        c.u[k] = S.u[k][i];
        if (drift) c.x[k] = S.x[k][i];
    }
    c.m = diag ? S.m[i] : 0.0;
    return c;
}

// Closing epilogue of the momentum pass for slot i with acceleration acc
// (FP64, per particle, in registers; its loads from close_load, if ci):
//   kick  = 1: close the step, u = v + dt/2 a (walls: u = 0);
//   dv: m|u|^2/2 and m u after it (for the diagnostics' block sums);
//   drift = 1: open the next step (half kick, drift, wrap, hash and count),
//              leaving v of the next step in u.
template <int DIM, typename T>
__device__ __forceinline__ void momentum_close(int i, const T acc[3], bool fluid, const State& S,
                                               const Grid& G, int kick, int drift, double hdt,
                                               double dt, uint32_t* __restrict__ key,
                                               uint32_t* __restrict__ counts,
                                               uint32_t* __restrict__ flags, bool diag,
                                               double dv[1 + DIM], const CloseIn* ci = nullptr) {
    for (int k = 0; k < DIM; ++k) ((T*)S.a[k])[i] = acc[k];
    double u[3] = {0.0, 0.0, 0.0}, a[3] = {0.0, 0.0, 0.0};
    {
#pragma clang fp contract(off)
        for (int k = 0; k < DIM; ++k) {
            a[k] = (double)acc[k];
            const double uk = ci ? ci->u[k] : S.u[k][i];
            u[k] = kick ? (fluid ? uk + hdt * a[k] : 0.0) : uk;
        }
        if (diag) {
            const double m = ci ? ci->m : S.m[i];
            double u2 = 0.0;
            for (int k = 0; k < DIM; ++k) {
                u2 += u[k] * u[k];
                dv[1 + k] = m * u[k];
            }
            dv[0] = 0.5 * m * u2;
        }
    }
    if (drift) {
        drift_and_hash<DIM>(i, S, G, fluid, u, a, hdt, dt, true, key, counts, flags, true,
                            ci ? ci->x : nullptr);
    } else if (kick) {
        for (int k = 0; k < DIM; ++k) S.u[k][i] = u[k];
    }
}

// Momentum equation of sorted slot i (fluid; walls get a = 0) over its
// neighbour list (or the cell walk), then momentum_close.
template <int DIM, int SR, int KERNEL, typename T>
__device__ __forceinline__ void momentum_one(
    int i, const Grid& G, const PairConst<T>& C, const uint32_t* __restrict__ skey,
    const typename Rec<T>::type* __restrict__ pos, const typename Vec4<T>::type* __restrict__ vel,
    const typename Vec2<T>::type* __restrict__ rp, const uint8_t* __restrict__ type,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, int n,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap,
    const State& S, int kick, int drift, double hdt, double dt, uint32_t* __restrict__ key,
    uint32_t* __restrict__ counts, uint32_t* __restrict__ flags, bool diag,
    double dv[1 + DIM]) {
    const bool fluid = type[i] == 0;
    T acc[3] = {T(0), T(0), T(0)};
    if (fluid) {
        const typename Rec<T>::type ri = pos[i];
        const typename Vec4<T>::type vi = vel[i];
        const typename Vec2<T>::type rpi = load_rp<DIM, T>(vi, rp, (uint32_t)i);
        T ax = C.g[0], ay = C.g[1], az = C.g[2];
        struct Pay {
            typename Vec4<T>::type v;
            typename Vec2<T>::type rp;
        };
        for_each_neighbor_p<DIM, SR, T>(
            i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, list, ncnt, cap,
            [&](uint32_t j) {
                typename Vec4<T>::type v = vel[j];
                keep_whole<DIM>(v);
                return Pay{v, load_rp<DIM, T>(v, rp, j)};
            },
            [&](uint32_t, const typename Rec<T>::type& rj, const Pay& pj, const Geom<T>& g) {
                momentum_add<DIM, KERNEL, T>(ax, ay, az, g, rec_mass(rj), vi, rpi, pj.v, pj.rp,
                                             C);
            });
        acc[0] = ax;
        acc[1] = ay;
        acc[2] = az;
    }
    momentum_close<DIM, T>(i, acc, fluid, S, G, kick, drift, hdt, dt, key, counts, flags, diag,
                           dv);
}

// Momentum equation for fluid particles (walls: a = 0), over the lists (or
// the cell walk), with momentum_close as the epilogue; diag_part != 0: per
// block partial sums of m|u|^2/2 and m u into diag_part.
template <int DIM, int SR, int KERNEL, typename T>
__global__ __launch_bounds__(kBlock) void k_momentum(
    int n, Grid G, PairConst<T> C, const uint32_t* __restrict__ skey,
    const typename Rec<T>::type* __restrict__ pos, const typename Vec4<T>::type* __restrict__ vel,
    const typename Vec2<T>::type* __restrict__ rp, const uint8_t* __restrict__ type,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap, State S,
    int kick,
    int drift, double hdt, double dt, uint32_t* __restrict__ key, uint32_t* __restrict__ counts,
    uint32_t* __restrict__ flags, double* __restrict__ diag_part) {
    const int blk = xcd_block();
    const int i = blk * kBlock + threadIdx.x;
    double dv[1 + DIM];
    for (int q = 0; q <= DIM; ++q) dv[q] = 0.0;
    if (i < n)
        momentum_one<DIM, SR, KERNEL, T>(i, G, C, skey, pos, vel, rp, type, cstart, cend, n, list,
                                         ncnt, cap, S, kick, drift, hdt, dt, key, counts, flags,
                                         diag_part != nullptr, dv);
    if (diag_part) block_sum4<1 + DIM>(dv, diag_part, blk, gridDim.x);
}

// The continuity scheme in one pass over the neighbour lists: the density
// rate (eqn continuity:sph) drho_i/dt = sum_j m_j v_ij . grad_i W_ij of every
// particle -- over all neighbours of a fluid particle, over the fluid
// neighbours of a solid one -- and the momentum equation (pressure, the nu
// term, g) of the fluid ones (walls: a = 0); both are stored (a, arho).  The
// FP64 epilogue then takes one of two integrators:
//  * euler (the paper's dam-break example): u += dt a; x += dt u with the new
//    u (and the periodic wrap); rho += dt arho; with drift, the new position
//    is hashed and counted for the next sort;
//  * predictor-corrector (Section 2.1): kick closes the step, u = v + dt/2 a
//    and rho = rho' + dt/2 arho; drift opens the next, v = u + dt/2 a,
//    rho' = rho + dt/2 arho, x += dt v, and hashes.
// Walls keep u = 0 and x.  diag_part (after the step) and count_pairs as in
// k_momentum and k_density.
template <int DIM, int SR, int KERNEL, typename T>
__global__ __launch_bounds__(kBlock) void k_cont_momentum(
    int n, Grid G, PairConst<T> C, const uint32_t* __restrict__ skey,
    const typename Rec<T>::type* __restrict__ pos, const typename Vec4<T>::type* __restrict__ vel,
    const typename Vec2<T>::type* __restrict__ rp, const uint8_t* __restrict__ type,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap, State S,
    int euler, int kick, int drift, double dt, uint32_t* __restrict__ key,
    uint32_t* __restrict__ counts, uint32_t* __restrict__ flags, double* __restrict__ diag_part,
    int count_pairs,
    unsigned long long* __restrict__ pairs) {
    const int blk = xcd_block();
    const int i = blk * kBlock + threadIdx.x;
    double dv[1 + DIM];
    for (int q = 0; q <= DIM; ++q) dv[q] = 0.0;
    uint32_t cnt = 0;
    if (i < n) {
        const bool fluid = type[i] == 0;
        const typename Rec<T>::type ri = pos[i];
        const typename Vec4<T>::type vi = vel[i];
        const typename Vec2<T>::type rpi = load_rp<DIM, T>(vi, rp, (uint32_t)i);
        T ax = C.g[0], ay = C.g[1], az = C.g[2], ar = T(0);
        struct Pay {
            typename Vec4<T>::type v;
            typename Vec2<T>::type rp;
            uint8_t t;
        };
        for_each_neighbor_p<DIM, SR, T>(
            i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, list, ncnt, cap,
            [&](uint32_t j) {
                typename Vec4<T>::type v = vel[j];
                keep_whole<DIM>(v);
                // 2D: the type rides in the position record
                return Pay{v, load_rp<DIM, T>(v, rp, j), DIM == 3 ? type[j] : (uint8_t)0};
            },
            [&](uint32_t, const typename Rec<T>::type& rj, const Pay& pj, const Geom<T>& g) {
                const int tj = DIM == 3 ? (int)pj.t : rec_type2(rj);
                // the self pair adds exact zeros (r = 0, v_ii = 0), as in
                // k_momentum; a wall's terms are formed and not used
                ++cnt;
                const T r2 = g.r2;
                const T F = kernel_f_r2<KERNEL, T>(r2, C);
                const T mj = rec_mass(rj);
                const T vx = vi.x - pj.v.x, vy = vi.y - pj.v.y;
                const T vz = DIM == 3 ? vi.z - pj.v.z : T(0);
                const T rv = g.d[0] * vx + g.d[1] * vy + (DIM == 3 ? g.d[2] * vz : T(0));
                if (fluid || tj == 0) ar += mj * (F * rv);
                const T pres = -(rpi.y + pj.rp.y) * F;
                const T visc = C.four_nu * F * r2 * p_rcp((rpi.x + pj.rp.x) * (r2 + C.eta_h2));
                const T mp = mj * pres, mv = mj * visc;
                ax += mp * g.d[0];
                ax += mv * vx;
                ay += mp * g.d[1];
                ay += mv * vy;
                if (DIM == 3) {
                    az += mp * g.d[2];
                    az += mv * vz;
                }
            });
        const T acc[3] = {ax, ay, az};
        double u[3] = {0.0, 0.0, 0.0}, a[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < DIM; ++k) {
            a[k] = fluid ? (double)acc[k] : 0.0;
            ((T*)S.a[k])[i] = (T)a[k];
        }
        const double arho = (double)ar;
        S.arho[i] = arho;
        {
#pragma clang fp contract(off)
            const double hdt = 0.5 * dt;
            double rho = load_rho<T>(S.rho, i, S.rho64);
            if (euler) {
                rho = rho + dt * arho;
                for (int k = 0; k < DIM; ++k) u[k] = fluid ? S.u[k][i] + dt * a[k] : 0.0;
            } else {
                for (int k = 0; k < DIM; ++k) u[k] = S.u[k][i];
                if (kick) {
                    rho = rho + hdt * arho;
                    for (int k = 0; k < DIM; ++k) u[k] = fluid ? u[k] + hdt * a[k] : 0.0;
                }
            }
            if (diag_part) {
                const double m = S.m[i];
                double u2 = 0.0;
                for (int k = 0; k < DIM; ++k) {
                    u2 += u[k] * u[k];
                    dv[1 + k] = m * u[k];
                }
                dv[0] = 0.5 * m * u2;
            }
            if (euler) {
                // x += dt u with the new u: the drift of drift_and_hash with a
                // zero half kick
                const double zero[3] = {0.0, 0.0, 0.0};
                drift_and_hash<DIM>(i, S, G, fluid, u, zero, 0.0, dt, true, key, counts, flags,
                                    drift != 0);
                store_rho<T>(S.rho, i, rho, S.rho64);
            } else {
                if (drift) {
                    rho = rho + hdt * arho;
                    drift_and_hash<DIM>(i, S, G, fluid, u, a, hdt, dt, true, key, counts, flags);
                } else if (kick) {
                    for (int k = 0; k < DIM; ++k) S.u[k][i] = u[k];
                }
                if (kick || drift) store_rho<T>(S.rho, i, rho, S.rho64);
            }
        }
    }
    if (diag_part) block_sum4<1 + DIM>(dv, diag_part, blk, gridDim.x);
    if (count_pairs) block_count(cnt, pairs, blk);
}

// Neighbour counts (phase 1) and lists (phase 2) of sph_neighbors.
template <int DIM, int SR, typename T>
__global__ __launch_bounds__(kBlock) void k_nbr_count(int n, Grid G, PairConst<T> C,
                                                      const uint32_t* __restrict__ skey,
                                                      const typename Rec<T>::type* __restrict__ pos,
                                                      const uint32_t* __restrict__ cstart,
                                                      const uint32_t* __restrict__ cend,
                                                      uint32_t* __restrict__ cnt) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const typename Rec<T>::type ri = pos[i];
    uint32_t c = 0;
    for_each_neighbor<DIM, SR, T>(i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, nullptr,
                                  nullptr, 0u,
                                  [&](uint32_t, const typename Rec<T>::type&, const Geom<T>&) { ++c; });
    cnt[i] = c;
}

template <int DIM, int SR, typename T>
__global__ __launch_bounds__(kBlock) void k_nbr_fill(int n, Grid G, PairConst<T> C,
                                                     const uint32_t* __restrict__ skey,
                                                     const typename Rec<T>::type* __restrict__ pos,
                                                     const uint32_t* __restrict__ cstart,
                                                     const uint32_t* __restrict__ cend,
                                                     const int64_t* __restrict__ off,
                                                     int32_t* __restrict__ nbr) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const typename Rec<T>::type ri = pos[i];
    int64_t w = off[i];
    const int64_t wend = off[i + 1];
    for_each_neighbor<DIM, SR, T>(i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, nullptr,
                                  nullptr, 0u,
                                  [&](uint32_t j, const typename Rec<T>::type&, const Geom<T>&) {
                                      if (w < wend) nbr[w++] = (int32_t)j;
                                  });
}

// Tait EOS alone (sph_eos).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_eos(int n, PairConst<T> C, const void* __restrict__ rho,
                                                int rho64, T* __restrict__ p) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    p[i] = (T)tait64<T>(load_rho<T>(rho, i, rho64), C);
}

// Fill with a constant (used instead of a memset so the sequence can be
// captured into a graph).
static __global__ __launch_bounds__(kBlock) void k_fill_u32(int64_t len, uint32_t v,
                                                     uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) out[i] = v;
}

// cell_start / cell_end from the scanned offsets.
static __global__ __launch_bounds__(kBlock) void k_cell_ranges(int64_t ncells,
                                                        const uint32_t* __restrict__ start,
                                                        uint32_t* __restrict__ cs,
                                                        uint32_t* __restrict__ ce) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncells) return;
    cs[c] = start[c];
    ce[c] = start[c + 1];
}

// Copy a state (all fields) slot by slot.
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_copy_state(int n, State src, State dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < DIM; ++q) {
        dst.x[q][i] = src.x[q][i];
        dst.u[q][i] = src.u[q][i];
        ((T*)dst.a[q])[i] = ((const T*)src.a[q])[i];
    }
    dst.m[i] = src.m[i];
    dst.type[i] = src.type[i];
    dst.id[i] = src.id[i];
    store_rho<T>(dst.rho, i, load_rho<T>(src.rho, i, src.rho64), dst.rho64);
    ((T*)dst.p)[i] = ((const T*)src.p)[i];
    if (src.arho && dst.arho) dst.arho[i] = src.arho[i];
}

// ---------------------------------------------------------------------------
// FP64 diagnostics: KE = sum m |u|^2 / 2 and momentum sum m u, as fixed-order
// tree sums: per-block partials (momentum epilogue), then one block over them.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_diag_final(int nparts, const double* __restrict__ part,
                                                       double* __restrict__ out) {
    __shared__ double sh[4][kBlock];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += kBlock)
        for (int q = 0; q < 1 + DIM; ++q) v[q] += part[(int64_t)q * nparts + b];
    for (int q = 0; q < 1 + DIM; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 1 + DIM; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 1 + DIM; ++q) out[q] = sh[q][0];
}

}  // namespace sph
