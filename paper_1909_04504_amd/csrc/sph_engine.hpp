// Host engine of the C ABI declared in include/sph.h: argument validation,
// workspace layout and the launch sequences of every entry point.  Included
// by the C ABI (sph.hip) and by the per-combination translation units
// (sph_part.hip) that instantiate the launch sequences.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "sph.h"
#include "sph_kernels.hpp"
#include "sph_adjoint.hpp"
#include "sph_tiles.hpp"

namespace sph_host {


inline thread_local std::string g_err;

inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define SPH_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(SPH_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define SPH_TRY(expr)                \
    do {                             \
        int rc_ = (expr);            \
        if (rc_ != SPH_OK) return rc_; \
    } while (0)

inline int launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SPH_EDEVICE, "launch of %s: %s", what, hipGetErrorString(e));
    return SPH_OK;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + sph::kBlock - 1) / sph::kBlock); }

// ---------------------------------------------------------------------------
// Opt-in per-kernel event timing (benchmark instrumentation)

enum KernelId {
    K_FILL, K_HASH, K_CHUNK_SUM, K_CHUNK_SCAN, K_SCATTER, K_RANK_GATHER, K_PACK, K_DENSITY,
    K_MOMENTUM, K_EOS, K_NBR_COUNT, K_NBR_FILL, K_CELL_RANGES, K_COPY, K_DIAG, K_ADJ_SEED,
    K_ADJ_PAIR1, K_ADJ_PAIR2, K_ADJ_REDUCE, K_ADJ_KICK, K_NLIST, K_CONT, K_TILE_BUILD,
    K_TILE_DENSITY, K_TILE_MOMENTUM, K_TILE_FALLBACK, K_COUNT
};
inline const char* const kKernelNames[K_COUNT] = {
    "fill", "drift_hash", "chunk_sum", "chunk_scan", "scatter", "rank_gather", "pack",
    "density", "momentum", "eos", "nbr_count", "nbr_fill", "cell_ranges", "copy_state", "diag",
    "adj_seed", "adj_pair1", "adj_pair2", "adj_reduce", "adj_kick", "nlist", "cont_momentum",
    "tile_build", "tile_density", "tile_momentum", "tile_fallback"};

struct Timer {
    bool on = false;
    struct Pending { int id; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    double ms[K_COUNT] = {};
    int64_t launches[K_COUNT] = {};

    hipEvent_t get() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        // timing-only events: no system-scope fence (cache writeback and
        // invalidation) around the bracketed launch
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
    void fold() {
        for (const Pending& q : pending) {
            float t = 0.f;
            if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&t, q.a, q.b) == hipSuccess) {
                ms[q.id] += t;
                launches[q.id] += 1;
            }
            spare.push_back(q.a);
            spare.push_back(q.b);
        }
        pending.clear();
    }
};
inline Timer g_timer;

// Compute units of the current device, looked up once per device (256 if
// the runtime cannot say).
inline unsigned device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return (unsigned)v;
}

// Launches kernel k on stream st with grid blocks of kBlock threads.  While
// timing is on, the launch carries start and stop events recorded by the
// dispatch itself (hipExtLaunchKernel), so the elapsed time is the kernel's
// own duration.
template <typename... KArgs, typename... Args>
void launch_b(int id, void (*k)(KArgs...), unsigned grid, unsigned block, hipStream_t st,
              Args... args) {
    if (g_timer.on) {
        hipEvent_t a = g_timer.get(), b = g_timer.get();
        if (a && b) {
            hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), 0, st, a, b, 0,
                                  static_cast<KArgs>(args)...);
            g_timer.pending.push_back({id, a, b});
            if (g_timer.pending.size() > 200000) g_timer.fold();
            return;
        }
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), 0, st, static_cast<KArgs>(args)...);
}
template <typename... KArgs, typename... Args>
void launch(int id, void (*k)(KArgs...), unsigned grid, hipStream_t st, Args... args) {
    launch_b(id, k, grid, sph::kBlock, st, args...);
}

// ---------------------------------------------------------------------------
// Validation

constexpr int kMaxNbrCap = 4096;

inline int check_params(const sph_params* p, bool need_dt) {
    if (!p) return fail(SPH_EINVAL, "params is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(SPH_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->kernel != SPH_CUBIC_SPLINE && p->kernel != SPH_WENDLAND_C2 &&
        p->kernel != SPH_QUINTIC_SPLINE)
        return fail(SPH_EINVAL, "unknown kernel %d", p->kernel);
    if (p->precision != SPH_FP64 && p->precision != SPH_FP32_MIXED)
        return fail(SPH_EINVAL, "unknown precision %d", p->precision);
    if (p->cell_div != 1 && p->cell_div != 2) return fail(SPH_EINVAL, "cell_div must be 1 or 2");
    if (p->scheme != SPH_SCHEME_SUMMATION && p->scheme != SPH_SCHEME_CONTINUITY)
        return fail(SPH_EINVAL, "unknown scheme %d", p->scheme);
    if (p->integrator != SPH_INTEGRATOR_PREDICTOR_CORRECTOR &&
        p->integrator != SPH_INTEGRATOR_EULER)
        return fail(SPH_EINVAL, "unknown integrator %d", p->integrator);
    if (p->integrator == SPH_INTEGRATOR_EULER && p->scheme != SPH_SCHEME_CONTINUITY)
        return fail(SPH_EINVAL, "the Euler stage is defined for the continuity scheme only");
    if (p->cell_order != 0 && p->cell_order != 1)
        return fail(SPH_EINVAL, "cell_order must be 0 (row-major) or 1 (Z-order)");
    if (p->cell_order == 1 && p->dim != 3)
        return fail(SPH_EINVAL, "Z-order cell keys are available in 3D only");
    if (p->nbr_cap > kMaxNbrCap)
        return fail(SPH_EINVAL, "nbr_cap must be at most %d (got %d)", kMaxNbrCap, p->nbr_cap);
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(SPH_EINVAL, "h must be > 0");
    if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return fail(SPH_EINVAL, "rho0 must be > 0");
    if (!(p->c0 > 0) || !std::isfinite(p->c0)) return fail(SPH_EINVAL, "c0 must be > 0");
    if (!(p->nu >= 0) || !std::isfinite(p->nu)) return fail(SPH_EINVAL, "nu must be >= 0");
    if (!(p->eta >= 0) || !std::isfinite(p->eta)) return fail(SPH_EINVAL, "eta must be >= 0");
    if (need_dt && (!(p->dt > 0) || !std::isfinite(p->dt))) return fail(SPH_EINVAL, "dt must be > 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->g[k])) return fail(SPH_EINVAL, "g must be finite");
    for (int k = 0; k < p->dim; ++k) {
        if (p->periodic[k] != 0 && p->periodic[k] != 1)
            return fail(SPH_EINVAL, "periodic[%d] must be 0 or 1", k);
        if (!std::isfinite(p->lo[k]) || !std::isfinite(p->hi[k]) || !(p->hi[k] > p->lo[k]))
            return fail(SPH_EINVAL, "axis %d: need lo < hi (finite)", k);
    }
    return SPH_OK;
}

// Support radius R = k h of the smoothing kernel: k = 3 for the quintic
// spline, 2 otherwise.
inline double support_radius(const sph_params* p) {
    return (p->kernel == SPH_QUINTIC_SPLINE ? 3.0 : 2.0) * p->h;
}

inline int make_grid(const sph_params* p, sph::Grid* G, int64_t* ncells) {
    const double R = support_radius(p);
    *ncells = 1;
    std::memset(G, 0, sizeof *G);
    G->dim = p->dim;
    G->S = p->cell_div;
    for (int k = 0; k < 3; ++k) {
        G->nc[k] = 1;
        G->cs[k] = 1.0;
        G->L[k] = 1.0;
        G->lo[k] = 0.0;
    }
    for (int k = 0; k < p->dim; ++k) {
        const double L = p->hi[k] - p->lo[k];
        double f = std::floor(L * p->cell_div / R);
        if (f < 1) f = 1;
        if (f > 2147483647.0) return fail(SPH_EINVAL, "axis %d: too many cells", k);
        const int64_t nc = (int64_t)f;
        if (p->periodic[k] && nc < 2 * p->cell_div + 1)
            return fail(SPH_EINVAL,
                        "periodic axis %d has %lld cells; the %d-cell stencil needs at least %d",
                        k, (long long)nc, 2 * p->cell_div + 1, 2 * p->cell_div + 1);
        *ncells *= nc;
        if (*ncells > ((int64_t)1 << 31)) return fail(SPH_EINVAL, "grid exceeds 2^31 cells");
        G->nc[k] = (int)nc;
        G->cs[k] = L / (double)nc;
        G->L[k] = L;
        G->lo[k] = p->lo[k];
        G->periodic[k] = p->periodic[k];
    }
    for (int a = 0; a < 2; ++a) sph::div_magic((uint32_t)G->nc[a], &G->dmag[a], &G->dsh1[a], &G->dsh2[a]);
    G->order = p->cell_order == 1 ? 1 : 0;
    G->mbits = 0;
    if (G->order) {
        // Z-order keys over the smallest power-of-two grid holding every
        // axis: 8^mbits keys, one slot range each (unused keys are empty)
        int64_t m = 1;
        for (int k = 0; k < 3; ++k) m = std::max<int64_t>(m, G->nc[k]);
        while (((int64_t)1 << G->mbits) < m) ++G->mbits;
        if (G->mbits < 1) G->mbits = 1;
        if (G->mbits > 10) return fail(SPH_EINVAL, "Z-order keys need at most 1024 cells per axis");
        *ncells = (int64_t)1 << (3 * G->mbits);
    }
    return SPH_OK;
}

// Largest particle count whose slot indices fit beside the stencil code of
// a list entry.
template <int DIM, int SR, typename T>
uint32_t list_max_n() {
    return sph::NbrCode<DIM, SR, T>::kMaxN;
}
inline uint32_t list_max_n(const sph_params* p) {
    const bool f64 = p->precision == SPH_FP64, s2 = p->cell_div == 2;
    if (p->dim == 2)
        return f64 ? (s2 ? list_max_n<2, 2, double>() : list_max_n<2, 1, double>())
                   : (s2 ? list_max_n<2, 2, float>() : list_max_n<2, 1, float>());
    return f64 ? (s2 ? list_max_n<3, 2, double>() : list_max_n<3, 1, double>())
               : (s2 ? list_max_n<3, 2, float>() : list_max_n<3, 1, float>());
}

// Neighbour-list capacity per particle (0: no lists).
inline uint32_t list_cap(const sph_params* p, int64_t n) {
    if (p->nbr_cap < 0 || n > (int64_t)list_max_n(p)) return 0;
    if (p->nbr_cap > 0) return (uint32_t)((p->nbr_cap + 3) & ~3);
    return p->dim == 2 ? 64u : 192u;
}

// Tiles of the 3D mixed-precision summation passes (ntiles = 0: not used).
// Boxes of 6 x 6 x 4 cells with half-size cells (about 490 targets for the
// 512 threads; a union of 10 x 10 x 8 cells, about 2,700 particles on the
// 256^3 lattice at h = 1.5 dx; measured against 8 x 4 x 4, 4 x 6 x 6,
// 6 x 4 x 6, 7 x 5 x 4 and 8 x 6 x 3 boxes: 13.6 against 14.5, 13.8, 13.7,
// 14.3 and 15.3 ms per cube step), and of 4 x 4 x 2 or 2 x 2 x 2 whole
// cells (by the mean occupancy).  By default
// (pair_tiles = 0) only on dense grids, at least one particle per cell on
// average: on a sparse grid most boxes hold few particles, and the lists in
// global memory stay cache-resident (3D dam break, 2.18M particles on 5.4M
// cells: 1.72 ms per step with global lists, 4.44 ms tiled); pair_tiles > 0
// uses them wherever they apply.
inline sph::Tiles make_tiles(const sph_params* p, const sph::Grid& G, int64_t n, int64_t ncells) {
    sph::Tiles T;
    std::memset(&T, 0, sizeof T);
    if (p->dim != 3 || p->precision != SPH_FP32_MIXED || p->scheme != SPH_SCHEME_SUMMATION ||
        p->pair_tiles < 0 || list_cap(p, n) < 8)
        return T;
    if (p->pair_tiles == 0 && n < ncells) return T;
    T.S = G.S;
    if (T.S == 2) {
        T.tw = 6; T.th = 6; T.td = 4;
    } else if ((double)n / (double)ncells <= 19.0) {
        T.tw = 4; T.th = 4; T.td = 2;
    } else {
        T.tw = 2; T.th = 2; T.td = 2;
    }
    T.uw = T.tw + 2 * T.S;
    T.uh = T.th + 2 * T.S;
    T.ud = T.td + 2 * T.S;
    int64_t nt = 1;
    for (int k = 0; k < 3; ++k) {
        const int t = k == 0 ? T.tw : (k == 1 ? T.th : T.td);
        T.nt[k] = (G.nc[k] + t - 1) / t;
        nt *= T.nt[k];
        T.csf[k] = (float)G.cs[k];
        T.inv_csf[k] = (float)(1.0 / G.cs[k]);
    }
    T.inv_uw = 1.0f / (float)T.uw;
    T.inv_uwh = 1.0f / (float)(T.uw * T.uh);
    T.cen[0] = T.uw / 2;
    T.cen[1] = T.uh / 2;
    T.cen[2] = T.ud / 2;
    const double R = support_radius(p);
    T.rclip2 = (float)(R * R * (1.0 + 1e-4));
    T.clip_pad = (float)(1e-4 * std::min(G.cs[0], std::min(G.cs[1], G.cs[2])));
    T.cap = p->pair_tiles > 0 ? std::min(p->pair_tiles, sph::kTileCap) : sph::kTileCap;
    if (nt > (int64_t)1 << 30 || T.uw > sph::kTileUnionAxisMax || T.uh > sph::kTileUnionAxisMax ||
        T.ud > sph::kTileUnionAxisMax || T.uw * T.uh * T.ud > sph::kTileCellsMax ||
        T.tw * T.th * T.td > sph::kTileTargetCellsMax) {
        std::memset(&T, 0, sizeof T);
        return T;
    }
    T.ntiles = (int)nt;
    return T;
}
inline unsigned fallback_blocks(int64_t n) {
    return std::min<unsigned>((unsigned)sph::kFallbackBlocks, blocks_for(n));
}
inline uint32_t next_tile_epoch() {
    static std::atomic<uint32_t> e{0};
    uint32_t v = ++e;
    if (v == 0) v = ++e;
    return v;
}

inline int check_particles(const sph_params* p, const sph_particles* pa) {
    if (!pa) return fail(SPH_EINVAL, "particles is NULL");
    if (pa->n < 1 || pa->n >= ((int64_t)1 << 31) - sph::kScanChunk)
        return fail(SPH_EINVAL, "n must be in [1, 2^31 - %d)", sph::kScanChunk);
    for (int k = 0; k < p->dim; ++k) {
        if (!pa->x[k] || !pa->u[k] || !pa->a[k])
            return fail(SPH_EINVAL, "x/u/a component %d is NULL", k);
    }
    if (!pa->rho || !pa->p || !pa->m || !pa->type || !pa->id)
        return fail(SPH_EINVAL, "rho, p, m, type or id is NULL");
    if (p->scheme == SPH_SCHEME_CONTINUITY && !pa->arho)
        return fail(SPH_EINVAL, "arho is NULL (needed by the continuity scheme)");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Workspace layout (all offsets 256-byte aligned)

struct StateOff {
    size_t x, u, a, m, type, id, rho, p, arho;
};

// One recompute-tape slot: the pair records and sort results of one step.
struct SlotOff {
    size_t pos, vel, rp, skey, perm, type, start;
};

struct Layout {
    size_t flags, counts, start, chunks, key, tmp, perm, skey, ncnt, lcnt, list;
    uint32_t cap;
    sph::Tiles tiles;
    StateOff s1, s2;
    size_t pos, vel, rp, diag;
    // adjoint (present when adj_k > 0; the tape is the last region)
    int64_t adj_k;
    size_t lamB, lamC, lhat, lxd, lvd, lrho, nupart;
    SlotOff slot;
    size_t slot_bytes, tape;
    size_t bytes;
};

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Launch shape of the cell-cooperative list build.  Dense grids (no more
// cells than particles): one cell per wave up to 65,536 cells, above that
// kNlistCells consecutive cells per wave, each wave
// overlapping the range loads of its next cell with the current one; short
// waves also finish the list rows they share before those leave L2
// (measured, 512^2 / 1024^2 / 2048^2 lattices: 1 cell 36.4 / 117 / 489 us,
// 2 cells 37.5 / 109 / 454, 3 cells 37.5 / 110 / 462, waves capped at 16,384
// (38 cells each at 2048^2) 39.1 / 135 / 738).  Sparse grids (a tank mostly
// empty): one wave per kNlistSlots sorted slots, taking the cells that start
// there, so that empty cells cost nothing (measured on the 2D dam break at
// dx = 0.1/32, 351k cells for 216k particles: 103 -> 34 us per build; 8, 16,
// 32, 64 slots: 34.0, 34.3, 35.7, 50.0 us, and 39.6, 38.9, 44.7, 50.1 us on
// the dense 512^2 lattice).
constexpr uint32_t kNlistCells = 2;
constexpr uint32_t kNlistSlots = 16;
static_assert(kNlistSlots >= 1 && kNlistSlots <= 64, "one lane per slot");
struct NlistShape {
    unsigned blocks;
    uint32_t per_wave;
    int by_slots;
};
inline NlistShape nlist_shape(int64_t n, int64_t ncells) {
    const int64_t per_block = sph::kBlock / 64;
    if (ncells <= n) {
        // one cell per wave on small grids: more waves (512^2: build 33.2 ->
        // 32.7 us with the current per-target loop)
        const uint32_t per = ncells <= 65536 ? 1u : kNlistCells;
        const int64_t waves = (ncells + per - 1) / per;
        return {(unsigned)((waves + per_block - 1) / per_block), per, 0};
    }
    const int64_t waves = (n + kNlistSlots - 1) / kNlistSlots;
    return {(unsigned)((waves + per_block - 1) / per_block), kNlistSlots, 1};
}

inline Layout make_layout(const sph_params* p, const sph::Grid& G, int64_t n, int64_t ncells,
                          int64_t adj_k) {
    Layout L;
    std::memset(&L, 0, sizeof L);
    L.tiles = make_tiles(p, G, n, ncells);
    const size_t ntiles = (size_t)L.tiles.ntiles;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t T = p->precision == SPH_FP64 ? 8 : 4;
    const size_t d = (size_t)p->dim, N = (size_t)n;
    auto take_state = [&]() {
        StateOff so;
        so.x = take(8 * d * N);
        so.u = take(8 * d * N);
        so.a = take(T * d * N);
        so.m = take(8 * N);
        so.type = take(N);
        so.id = take(4 * N);
        so.rho = take(8 * N);
        so.p = take(T * N);
        so.arho = p->scheme == SPH_SCHEME_CONTINUITY ? take(8 * N) : 0;
        return so;
    };
    const int64_t longest = (ncells + 1 > n + 1) ? ncells + 1 : n + 1;
    // chunk sums of the scans: long arrays in chunks of kScanChunk, short
    // ones in chunks of kBlock * kScanItemsShort (at most 512 of them)
    const size_t nchunks =
        std::max<size_t>(512, (size_t)((longest + sph::kScanChunk - 1) / sph::kScanChunk));
    // header (flag word at 0, number of interaction counters at 8), then one
    // 64-bit interaction counter per block of the counting kernel (k_nlist,
    // or k_density without lists) from offset 16
    // (and the tile passes' fallback epoch at offset 4)
    L.flags = take(16 + 8 * std::max<size_t>(std::max(nlist_shape(n, ncells).blocks, blocks_for(n)),
                                             ntiles));
    L.counts = take(4 * (size_t)ncells);
    L.start = take(4 * ((size_t)ncells + 1));
    L.chunks = take(8 * nchunks);
    L.key = take(4 * N);
    L.tmp = take(4 * N);
    L.perm = take(4 * N);
    L.skey = take(4 * N);
    L.ncnt = take(4 * N);
    L.cap = list_cap(p, n);
    L.lcnt = take(4 * N);
    L.list = take(4 * (size_t)L.cap * (size_t)sph::kListTile *
                  ((N + sph::kListTile - 1) / sph::kListTile));
    L.s1 = take_state();
    L.pos = take(4 * T * N);
    L.vel = take(4 * T * N);
    L.rp = take(2 * T * N);
    // diagnostics partials: per block, or per tile and fallback block
    L.diag = take(8 * 4 * std::max<size_t>(blocks_for(n), ntiles + fallback_blocks(n)));
    L.adj_k = adj_k;
    if (adj_k > 0) {
        L.s2 = take_state();
        L.lamB = take(8 * 3 * d * N);
        L.lamC = take(8 * 3 * d * N);
        L.lhat = take(4 * T * N);
        L.lxd = take(8 * d * N);
        L.lvd = take(8 * d * N);
        L.lrho = take(T * N);
        L.nupart = take(8 * N);
        size_t so = 0;
        auto slot_take = [&](size_t bytes) {
            const size_t o = so;
            so = align256(so + bytes);
            return o;
        };
        L.slot.pos = slot_take(4 * T * N);
        L.slot.vel = slot_take(4 * T * N);
        L.slot.rp = slot_take(2 * T * N);
        L.slot.skey = slot_take(4 * N);
        L.slot.perm = slot_take(4 * N);
        L.slot.type = slot_take(N);
        L.slot.start = slot_take(4 * ((size_t)ncells + 1));
        L.slot_bytes = so;
        L.tape = take(L.slot_bytes * (size_t)adj_k);
    }
    L.bytes = off;
    return L;
}

// rho is FP64 under the continuity scheme (an integrated state), else of the
// pair type.
inline int rho_is_f64(const sph_params* p) { return p->scheme == SPH_SCHEME_CONTINUITY; }

inline sph::State user_state(const sph_particles* pa, const sph_params* p) {
    sph::State s;
    for (int k = 0; k < 3; ++k) {
        s.x[k] = pa->x[k];
        s.u[k] = pa->u[k];
        s.a[k] = pa->a[k];
    }
    s.rho = pa->rho;
    s.p = pa->p;
    s.m = pa->m;
    s.type = pa->type;
    s.id = pa->id;
    s.rho64 = rho_is_f64(p);
    s.arho = rho_is_f64(p) ? pa->arho : nullptr;
    return s;
}

inline sph::State ws_state(char* ws, const StateOff& L, const sph_params* p, int64_t n) {
    const size_t T = p->precision == SPH_FP64 ? 8 : 4;
    sph::State s;
    for (int k = 0; k < 3; ++k) {
        const bool used = k < p->dim;
        s.x[k] = used ? (double*)(ws + L.x) + k * n : nullptr;
        s.u[k] = used ? (double*)(ws + L.u) + k * n : nullptr;
        s.a[k] = used ? (void*)(ws + L.a + T * k * n) : nullptr;
    }
    s.rho = ws + L.rho;
    s.p = ws + L.p;
    s.m = (double*)(ws + L.m);
    s.type = (uint8_t*)(ws + L.type);
    s.id = (int32_t*)(ws + L.id);
    s.rho64 = rho_is_f64(p);
    s.arho = rho_is_f64(p) ? (double*)(ws + L.arho) : nullptr;
    return s;
}

template <typename T>
sph::PairConst<T> pair_const(const sph_params* p, const sph::Grid& G) {
    const double pi = 3.14159265358979323846;
    const double h = p->h;
    double sigma;
    if (p->kernel == SPH_CUBIC_SPLINE)
        sigma = p->dim == 2 ? 10.0 / (7.0 * pi * h * h) : 1.0 / (pi * h * h * h);
    else if (p->kernel == SPH_QUINTIC_SPLINE)
        sigma = p->dim == 2 ? 7.0 / (478.0 * pi * h * h) : 1.0 / (120.0 * pi * h * h * h);
    else
        sigma = p->dim == 2 ? 7.0 / (4.0 * pi * h * h) : 21.0 / (16.0 * pi * h * h * h);
    const double R = support_radius(p), R2 = R * R;
    sph::PairConst<T> C;
    C.R2 = (T)R2;
    C.R2_d = R2;
    C.inv_h_d = 1.0 / h;
    C.half_inv_h_d = 0.5 / h;
    C.two_inv_h_d = 2.0 / h;
    C.sigma_d = sigma;
    for (int k = 0; k < 3; ++k) {
        C.fix_scale[k] = G.cs[k] / (double)(1 << sph::kFixBits);
        C.fix_scale_f[k] = (float)C.fix_scale[k];
    }
    C.R2_lo = (float)(R2 * (1.0 - 1e-5));
    C.R2_hi = (float)(R2 * (1.0 + 1e-5));
    C.R2_mid = (float)R2;
    C.R2_w = (float)(2e-5 * R2);
    C.h = (T)h;
    C.inv_h = (T)(1.0 / h);
    C.sigma = (T)sigma;
    C.sigma_h2 = (T)(sigma / (h * h));
    C.eta_h2 = (T)(p->eta * h * h);
    C.four_nu = (T)(4.0 * p->nu);
    for (int k = 0; k < 3; ++k) {
        C.g[k] = (T)p->g[k];
        C.cs[k] = (T)G.cs[k];
        C.L[k] = (T)G.L[k];
    }
    C.rho0 = (T)p->rho0;
    C.rho0_d = p->rho0;
    C.B_d = p->rho0 * p->c0 * p->c0 / 7.0;
    C.inv_rho0 = (T)(1.0 / p->rho0);
    C.B = (T)(p->rho0 * p->c0 * p->c0 / 7.0);
    C.sigma_h4 = (T)(sigma / (h * h * h * h));
    C.b7 = (T)(p->c0 * p->c0);  // 7 B / rho0 = c0^2
    return C;
}

// ---------------------------------------------------------------------------
// Launch sequences for one (dimension, kernel, pair precision)

template <int DIM, int KERNEL, typename T>
struct Engine {
    using V4 = typename sph::Vec4<T>::type;
    using V2 = typename sph::Vec2<T>::type;
    using R4 = typename sph::Rec<T>::type;
    const sph_params* prm;
    sph::Grid G;
    int64_t ncells;
    int n;
    char* ws;
    Layout L;
    hipStream_t st;
    sph::PairConst<T> C;

    uint32_t* flags() const { return (uint32_t*)(ws + L.flags); }
    unsigned long long* pairs() const { return (unsigned long long*)(ws + L.flags + 16); }
    uint32_t* counts() const { return (uint32_t*)(ws + L.counts); }
    uint64_t* chunks() const { return (uint64_t*)(ws + L.chunks); }
    uint32_t* key() const { return (uint32_t*)(ws + L.key); }
    uint32_t* tmp() const { return (uint32_t*)(ws + L.tmp); }
    uint32_t* ncnt() const { return (uint32_t*)(ws + L.ncnt); }
    uint32_t* lcnt() const { return (uint32_t*)(ws + L.lcnt); }
    uint32_t* list() const { return (uint32_t*)(ws + L.list); }

    // Pair records and sort results of the current evaluation: the default
    // buffers, or one slot of the adjoint's recompute tape.
    R4* posp = nullptr;
    V4* velp = nullptr;
    V2* rpp = nullptr;
    uint32_t* skeyp = nullptr;
    uint32_t* permp = nullptr;
    uint32_t* startp = nullptr;
    uint8_t* typetape = nullptr;
    uint32_t* perm() const { return permp; }
    uint32_t* skey() const { return skeyp; }
    uint32_t* start() const { return startp; }
    R4* pos() const { return posp; }
    V4* vel() const { return velp; }
    V2* rp() const { return rpp; }

    void default_records() {
        posp = (R4*)(ws + L.pos);
        velp = (V4*)(ws + L.vel);
        rpp = (V2*)(ws + L.rp);
        skeyp = (uint32_t*)(ws + L.skey);
        permp = (uint32_t*)(ws + L.perm);
        startp = (uint32_t*)(ws + L.start);
        typetape = nullptr;
    }
    void tape_records(int64_t slot) {
        char* b = ws + L.tape + (size_t)slot * L.slot_bytes;
        posp = (R4*)(b + L.slot.pos);
        velp = (V4*)(b + L.slot.vel);
        rpp = (V2*)(b + L.slot.rp);
        skeyp = (uint32_t*)(b + L.slot.skey);
        permp = (uint32_t*)(b + L.slot.perm);
        typetape = (uint8_t*)(b + L.slot.type);
        startp = (uint32_t*)(b + L.slot.start);
    }

    // Calls fn(std::integral_constant<int, S>) for the grid's stencil reach.
    template <typename Fn>
    void with_reach(Fn&& fn) const {
        if (G.S == 2)
            fn(std::integral_constant<int, 2>());
        else
            fn(std::integral_constant<int, 1>());
    }

    int zero_counts() {
        launch(K_FILL, sph::k_fill_u32, blocks_for(ncells), st, ncells, 0u, counts());
        return launch_check("k_fill_u32");
    }

    // exclusive scan of `len` u32 counts into out[0..len] (short arrays, e.g.
    // the cells of a 512^2 lattice, in chunks of 1,024 so that both launches
    // have several times more blocks)
    template <typename OUT>
    int scan(const uint32_t* in, int64_t len, OUT* out) {
        if (len <= sph::kScanShortMax) return scan_items<OUT, sph::kScanItemsShort>(in, len, out);
        return scan_items<OUT, sph::kScanItems>(in, len, out);
    }
    template <typename OUT, int ITEMS>
    int scan_items(const uint32_t* in, int64_t len, OUT* out) {
        constexpr int64_t chunk = (int64_t)sph::kBlock * ITEMS;
        const unsigned nch = (unsigned)((len + chunk - 1) / chunk);
        {
        launch(K_CHUNK_SUM, sph::k_chunk_sum<ITEMS>, nch, st, in, len, chunks());
        SPH_TRY(launch_check("k_chunk_sum"));
        }
        launch(K_CHUNK_SCAN, sph::k_chunk_scan<OUT, ITEMS>, nch, st, in, len, chunks(), out);
        return launch_check("k_chunk_scan");
    }

    // hash (with the opening half kick + drift if drift), counting sort, and
    // gather of src into dst in sorted order with pair records packed.
    // hashed: src already holds the drifted positions with keys and counts
    // (from the epilogue of the previous momentum launch).
    // eos: gather rho, and form p and the (rho, p/rho^2) records from it
    // (continuity scheme); predict: records of u + predict a and the EOS at
    // rho + predict arho (the predictor-corrector's predicted end state);
    // kick_rho: the opening drift also kicks rho by dt/2 arho.
    int sort_into(const sph::State& src, const sph::State& dst, bool drift, bool copy_derived,
                  bool hashed = false, bool eos = false, double predict = 0.0,
                  bool kick_rho = false) {
        const unsigned nb = blocks_for(n);
        using TA = T;
        if (!hashed) {
            launch(K_HASH, sph::k_drift_hash<DIM, TA>, nb, st,
                n, src, G, 0.5 * prm->dt, prm->dt, drift ? 1 : 0, kick_rho ? 1 : 0, key(),
                counts(), flags());
            SPH_TRY(launch_check("k_drift_hash"));
        }
        SPH_TRY(scan<uint32_t>(counts(), ncells, start()));
        {
        launch(K_SCATTER, sph::k_scatter, nb, st, n, key(), start(), counts(), tmp());
        SPH_TRY(launch_check("k_scatter"));
        }
        launch(K_RANK_GATHER, sph::k_rank_gather<DIM, T>, nb, st, n, tmp(), key(), start(), src, dst, G,
                                                             perm(), skey(), pos(), vel(),
                                                             copy_derived ? 1 : 0, typetape, C,
                                                             rp(), eos ? 1 : 0, predict);
        return launch_check("k_rank_gather");
    }

    // Neighbour lists of the current records (count_pairs: add the number
    // of interactions to the counters).  Every pair pass reads the lists
    // built last, so each change of records is followed by this launch.
    int nlist(const uint32_t* cs, const uint32_t* ce, bool count_pairs) {
        with_reach([&](auto R) {
            // cell-cooperative build in 2D with cells of 2h (about 7 targets
            // and 61 candidates per cell); the walk build elsewhere, where a
            // cell's candidates are many times a wave (measured: 3D dam break
            // 0.88 ms walk at cell_div 2 against 2.6 ms cooperative at 1).
            // The cooperative build addresses the list with 32-bit byte
            // offsets: lists of 4 GiB or more take the walk build.
            const bool small_list = (uint64_t)4 * L.cap * sph::kListTile *
                                        (((uint64_t)n + sph::kListTile - 1) / sph::kListTile) <
                                    ((uint64_t)1 << 32);
            if (DIM == 2 && decltype(R)::value == 1 && small_list) {
                const NlistShape sh = nlist_shape(n, ncells);
                launch(K_NLIST, sph::k_nlist<DIM, decltype(R)::value, T>, sh.blocks, st, n,
                       (uint32_t)ncells, sh.per_wave, sh.by_slots, G, C, skey(), pos(), cs, ce,
                       L.cap, list(), lcnt(), count_pairs ? 1 : 0, pairs());
            } else {
                launch(K_NLIST, sph::k_nlist_walk<DIM, decltype(R)::value, T>, blocks_for(n), st,
                       n, G, C, skey(), pos(), cs, ce, L.cap, list(), lcnt(), count_pairs ? 1 : 0,
                       pairs());
            }
        });
        return launch_check("k_nlist");
    }
    const uint32_t* list_or_null() const { return L.cap ? list() : nullptr; }

    // --- LDS-tiled passes (3D mixed precision, summation scheme) -----------
    static constexpr bool kTileable = DIM == 3 && std::is_same<T, float>::value;
    bool tiled() const { return kTileable && L.tiles.ntiles > 0; }
    uint32_t tcap() const { return L.cap & ~7u; }
    uint32_t* fbword() const { return (uint32_t*)(ws + L.flags + 4); }
    uint32_t tile_epoch = 0;

    // Tile lists of the current records and, with_density, the density (and
    // EOS) over them; then the fallback density of the targets the tiles left.
    int tile_lists(const sph::State& s, const uint32_t* cs, const uint32_t* ce, bool with_density,
                   bool with_eos, bool count_pairs) {
        if constexpr (kTileable) {
            tile_epoch = next_tile_epoch();
            const sph::Tiles TL = L.tiles;
            with_reach([&](auto R) {
                launch_b(K_TILE_BUILD, sph::k_tile_build<decltype(R)::value>, (unsigned)TL.ntiles,
                         sph::kTileThreads, st, n, G, C, TL, TL.cap, pos(), cs, ce, tcap(),
                         (uint4*)list(), lcnt(), count_pairs ? 1 : 0, pairs(), tile_epoch,
                         fbword());
            });
            SPH_TRY(launch_check("k_tile_build"));
            if (!with_density) return SPH_OK;
            with_reach([&](auto R) {
                launch_b(K_TILE_DENSITY, sph::k_tile_density<decltype(R)::value, KERNEL>,
                         (unsigned)TL.ntiles, sph::kTileThreads, st, n, G, C, TL, TL.cap, pos(), cs,
                         ce, tcap(), (const uint4*)list(), lcnt(), (float*)s.rho, (float*)s.p,
                         vel(), rp(), with_eos ? 1 : 0);
            });
            SPH_TRY(launch_check("k_tile_density"));
            with_reach([&](auto R) {
                launch(K_TILE_FALLBACK, sph::k_tile_fallback_density<decltype(R)::value, KERNEL>,
                       fallback_blocks(n), st, n, G, C, skey(), pos(), cs, ce, lcnt(), tcap(),
                       (float*)s.rho, (float*)s.p, vel(), rp(), with_eos ? 1 : 0,
                       count_pairs ? 1 : 0, pairs(), tile_epoch, fbword());
            });
            return launch_check("k_tile_fallback_density");
        }
        return fail(SPH_EINVAL, "tiled passes need 3D mixed precision");
    }

    // Tiled momentum of the targets with complete tile lists, then the
    // fallback momentum; diagnostics over both kernels' partial sums.
    int tile_momentum(const sph::State& s, const uint32_t* cs, const uint32_t* ce, bool kick,
                      bool drift, double* diag_out) {
        if constexpr (kTileable) {
            const sph::Tiles TL = L.tiles;
            const unsigned fb = fallback_blocks(n);
            const int stride = TL.ntiles + (int)fb;
            double* part = diag_out ? (double*)(ws + L.diag) : nullptr;
            // one workgroup per CU (the staging's LDS), each over every
            // wgs-th tile
            const unsigned wgs = std::min<unsigned>((unsigned)TL.ntiles, device_cus());
            with_reach([&](auto R) {
                launch_b(K_TILE_MOMENTUM, sph::k_tile_momentum<decltype(R)::value, KERNEL>, wgs,
                         sph::kTileThreads, st, n, G, C, TL, TL.cap, pos(), vel(), rp(), s.type,
                         cs, ce, tcap(), (const uint4*)list(), lcnt(), s, kick ? 1 : 0,
                         drift ? 1 : 0, 0.5 * prm->dt, prm->dt, key(), counts(), flags(), part,
                         stride);
            });
            SPH_TRY(launch_check("k_tile_momentum"));
            with_reach([&](auto R) {
                launch(K_TILE_FALLBACK, sph::k_tile_fallback_momentum<decltype(R)::value, KERNEL>,
                       fb, st, n, G, C, skey(), pos(), vel(), rp(), s.type, cs, ce, lcnt(), tcap(),
                       s, kick ? 1 : 0, drift ? 1 : 0, 0.5 * prm->dt, prm->dt, key(), counts(),
                       flags(), part ? part + TL.ntiles : nullptr, stride, tile_epoch, fbword());
            });
            SPH_TRY(launch_check("k_tile_fallback_momentum"));
            if (!diag_out) return SPH_OK;
            launch(K_DIAG, sph::k_diag_final<DIM>, 1, st, stride, part, diag_out);
            return launch_check("k_diag_final");
        }
        return fail(SPH_EINVAL, "tiled passes need 3D mixed precision");
    }

    // Lists of the current records, then the density over them; without
    // lists the density walk counts the interactions.
    int density(const sph::State& s, const uint32_t* cs, const uint32_t* ce, bool with_eos) {
        if (tiled()) return tile_lists(s, cs, ce, true, with_eos, true);
        if (L.cap) SPH_TRY(nlist(cs, ce, true));
        with_reach([&](auto R) {
            launch(K_DENSITY, sph::k_density<DIM, decltype(R)::value, KERNEL, T>, blocks_for(n), st,
                n, G, C, skey(), pos(), cs, ce, list_or_null(), lcnt(), L.cap, s.rho, s.rho64,
                (T*)s.p, vel(), rp(), with_eos ? 1 : 0, L.cap ? 0 : 1, pairs());
        });
        return launch_check("k_density");
    }

    // kick: close the step; drift: open the next one (hash + count);
    // diag_out: KE and momentum after the kick, 1 + DIM doubles.
    int momentum(const sph::State& s, const uint32_t* cs, const uint32_t* ce, bool kick,
                 bool drift = false, double* diag_out = nullptr) {
        if (tiled()) return tile_momentum(s, cs, ce, kick, drift, diag_out);
        double* part = diag_out ? (double*)(ws + L.diag) : nullptr;
        const unsigned nb = blocks_for(n);
        {
            with_reach([&](auto R) {
                launch(K_MOMENTUM, sph::k_momentum<DIM, decltype(R)::value, KERNEL, T>, nb, st,
                    n, G, C, skey(), pos(), vel(), rp(), s.type, cs, ce, list_or_null(), lcnt(),
                    L.cap, s, kick ? 1 : 0,
                    drift ? 1 : 0, 0.5 * prm->dt, prm->dt, key(), counts(), flags(), part);
            });
            SPH_TRY(launch_check("k_momentum"));
        }
        if (!diag_out) return SPH_OK;
        launch(K_DIAG, sph::k_diag_final<DIM>, 1, st, (int)nb, part, diag_out);
        return launch_check("k_diag_final");
    }

    int pack(const sph::State& s, bool with_rp) {
        launch(K_PACK, sph::k_pack<DIM, T>, blocks_for(n), st, n, s, G, skey(), pos(), vel(),
                                                                  rp(), with_rp ? 1 : 0);
        return launch_check("k_pack");
    }

    int copy(const sph::State& src, const sph::State& dst) {
        launch(K_COPY, sph::k_copy_state<DIM, T>, blocks_for(n), st, n, src, dst);
        return launch_check("k_copy_state");
    }

    // --- entry points ---------------------------------------------------

    int bin_sort(sph_particles* pa, uint32_t* cs_out, uint32_t* ce_out) {
        const sph::State user = user_state(pa, prm);
        const sph::State tmp_state = ws_state(ws, L.s1, prm, n);
        SPH_TRY(zero_counts());
        SPH_TRY(sort_into(user, tmp_state, false, true));
        SPH_TRY(copy(tmp_state, user));
        launch(K_CELL_RANGES, sph::k_cell_ranges, blocks_for(ncells), st, ncells, start(), cs_out, ce_out);
        return launch_check("k_cell_ranges");
    }

    int density_only(sph_particles* pa, const uint32_t* cs, const uint32_t* ce) {
        const sph::State user = user_state(pa, prm);
        SPH_TRY(pack(user, false));
        return density(user, cs, ce, false);
    }

    int momentum_only(sph_particles* pa, const uint32_t* cs, const uint32_t* ce) {
        const sph::State user = user_state(pa, prm);
        SPH_TRY(pack(user, true));
        if (tiled())
            SPH_TRY(tile_lists(user, cs, ce, false, false, false));
        else if (L.cap)
            SPH_TRY(nlist(cs, ce, false));
        return momentum(user, cs, ce, false);
    }

    int eos_only(sph_particles* pa) {
        launch(K_EOS, sph::k_eos<T>, blocks_for(n), st, n, C, (const void*)pa->rho,
               rho_is_f64(prm), (T*)pa->p);
        return launch_check("k_eos");
    }

    int neighbors(const sph_particles* pa, const uint32_t* cs, const uint32_t* ce, int64_t capacity,
                  int64_t* offsets, int32_t* nbr, int64_t* total) {
        const sph::State user = user_state(pa, prm);
        SPH_TRY(pack(user, false));
        {
        with_reach([&](auto R) {
            launch(K_NBR_COUNT, sph::k_nbr_count<DIM, decltype(R)::value, T>, blocks_for(n), st,
                n, G, C, skey(), pos(), cs, ce, ncnt());
        });
        SPH_TRY(launch_check("k_nbr_count"));
        }
        SPH_TRY(scan<int64_t>(ncnt(), n, offsets));
        int64_t tot = 0;
        SPH_HIP(hipMemcpyAsync(&tot, offsets + n, sizeof tot, hipMemcpyDeviceToHost, st));
        SPH_HIP(hipStreamSynchronize(st));
        *total = tot;
        if (tot > capacity)
            return fail(SPH_ECAPACITY, "neighbour list needs %lld entries, capacity %lld",
                        (long long)tot, (long long)capacity);
        if (tot > 0 && !nbr) return fail(SPH_EINVAL, "nbr is NULL");
        with_reach([&](auto R) {
            launch(K_NBR_FILL, sph::k_nbr_fill<DIM, decltype(R)::value, T>, blocks_for(n), st,
                n, G, C, skey(), pos(), cs, ce, offsets, nbr);
        });
        return launch_check("k_nbr_fill");
    }

    int step(sph_particles* pa, int64_t nsteps, int prime, double* diag_out) {
        const sph::State user = user_state(pa, prm);
        const sph::State wst = ws_state(ws, L.s1, prm, n);
        sph::State cur = user, nxt = wst;
        const uint32_t* cs = start();
        const uint32_t* ce = start() + 1;
        SPH_TRY(zero_counts());
        bool hashed = false;  // cur already drifted and hashed by a fused epilogue
        if (prime) {
            SPH_TRY(sort_into(cur, nxt, false, false));
            SPH_TRY(density(nxt, cs, ce, true));
            SPH_TRY(momentum(nxt, cs, ce, false, nsteps > 0));
            std::swap(cur, nxt);
            hashed = nsteps > 0;
        }
        for (int64_t s = 0; s < nsteps; ++s) {
            const bool last = s == nsteps - 1;
            SPH_TRY(sort_into(cur, nxt, true, false, hashed));
            SPH_TRY(density(nxt, cs, ce, true));
            SPH_TRY(momentum(nxt, cs, ce, true, !last, diag_out ? diag_out + s * (1 + DIM) : nullptr));
            std::swap(cur, nxt);
            hashed = !last;
        }
        if (cur.m != user.m) SPH_TRY(copy(cur, user));
        return SPH_OK;
    }

    // Continuity scheme: lists, then one pass for drho/dt and a with the
    // integrator's stage and the next step's hash in its epilogue.
    int cont_pass(const sph::State& s, bool euler, bool kick, bool drift, double* diag_out) {
        const unsigned nb = blocks_for(n);
        double* part = diag_out ? (double*)(ws + L.diag) : nullptr;
        if (L.cap) SPH_TRY(nlist(start(), start() + 1, true));
        with_reach([&](auto R) {
            launch(K_CONT, sph::k_cont_momentum<DIM, decltype(R)::value, KERNEL, T>, nb, st, n, G,
                   C, skey(), pos(), vel(), rp(), (const uint8_t*)s.type, start(), start() + 1,
                   list_or_null(), lcnt(), L.cap, s, euler ? 1 : 0, kick ? 1 : 0, drift ? 1 : 0,
                   prm->dt, key(), counts(), flags(), part, L.cap ? 0 : 1, pairs());
        });
        SPH_TRY(launch_check("k_cont_momentum"));
        if (!diag_out) return SPH_OK;
        launch(K_DIAG, sph::k_diag_final<DIM>, 1, st, (int)nb, part, diag_out);
        return launch_check("k_diag_final");
    }

    // Euler stage (the paper's dam-break example): per step, sort with rho
    // gathered and p = EOS(rho), then the pass.  Predictor-corrector
    // (Section 2.1): as sph_step's summation scheme with rho kicked like u and
    // the rates at a step's end evaluated at the predicted end state.
    int step_continuity(sph_particles* pa, int64_t nsteps, int prime, double* diag_out) {
        const sph::State user = user_state(pa, prm);
        const sph::State wst = ws_state(ws, L.s1, prm, n);
        sph::State cur = user, nxt = wst;
        const bool euler = prm->integrator == SPH_INTEGRATOR_EULER;
        const double hdt = 0.5 * prm->dt;
        SPH_TRY(zero_counts());
        bool hashed = false;  // cur already opened and hashed by a fused epilogue
        if (!euler && prime) {
            SPH_TRY(sort_into(cur, nxt, false, false, false, true));
            SPH_TRY(cont_pass(nxt, false, false, nsteps > 0, nullptr));
            std::swap(cur, nxt);
            hashed = nsteps > 0;
        }
        for (int64_t s = 0; s < nsteps; ++s) {
            const bool last = s == nsteps - 1;
            double* dg = diag_out ? diag_out + s * (1 + DIM) : nullptr;
            if (euler) {
                SPH_TRY(sort_into(cur, nxt, false, false, s > 0, true));
                SPH_TRY(cont_pass(nxt, true, false, !last, dg));
            } else {
                SPH_TRY(sort_into(cur, nxt, true, false, hashed, true, hdt, true));
                SPH_TRY(cont_pass(nxt, false, true, !last, dg));
            }
            std::swap(cur, nxt);
            hashed = !last;
        }
        if (cur.m != user.m) SPH_TRY(copy(cur, user));
        return SPH_OK;
    }

    // (dA/dx)^T lhat -> lxd, (dA/dv)^T lhat -> lvd, (dA/dnu)^T lhat added to
    // *dJ, at the evaluation whose records are current; lhat = lam_a +
    // hdt lam_u (fluid), read through `gather` (identity if null).
    int adjoint_rhs(const double* lam_u, const double* lam_a, int64_t ld, double hdt,
                    const uint8_t* type, const uint32_t* gather, double* dJ, bool build_list) {
        const unsigned nb = blocks_for(n);
        if (build_list && L.cap) SPH_TRY(nlist(start(), start() + 1, false));
        V4* lhat = (V4*)(ws + L.lhat);
        double* lxd = (double*)(ws + L.lxd);
        double* lvd = (double*)(ws + L.lvd);
        T* lrho = (T*)(ws + L.lrho);
        double* nup = (double*)(ws + L.nupart);
        double* part = (double*)(ws + L.diag);
        {
            launch(K_ADJ_SEED, sph::k_adj_seed<DIM, T>, nb, st, n, lam_u, lam_a, ld, hdt, type,
                                                               gather, lhat);
            SPH_TRY(launch_check("k_adj_seed"));
        }
        {
            with_reach([&](auto R) {
                launch(K_ADJ_PAIR1, sph::k_adj_pair1<DIM, decltype(R)::value, KERNEL, T>, nb, st,
                    n, G, C, skey(), pos(), vel(), rp(), lhat, start(), start() + 1,
                    list_or_null(), lcnt(), L.cap, lxd, lvd, lrho, nup);
            });
            SPH_TRY(launch_check("k_adj_pair1"));
        }
        {
            with_reach([&](auto R) {
                launch(K_ADJ_PAIR2, sph::k_adj_pair2<DIM, decltype(R)::value, KERNEL, T>, nb, st,
                    n, G, C, skey(), pos(), lrho, start(), start() + 1, list_or_null(), lcnt(),
                    L.cap, lxd);
            });
            SPH_TRY(launch_check("k_adj_pair2"));
        }
        launch(K_ADJ_REDUCE, sph::k_sum_partial, nb, st, n, nup, part);
        SPH_TRY(launch_check("k_sum_partial"));
        launch(K_ADJ_REDUCE, sph::k_sum_accum, 1, st, (int)nb, part, dJ);
        return launch_check("k_sum_accum");
    }

    // k recomputed steps from the checkpoint, then their reverse.
    int step_backward(const sph_particles* ck, int64_t k, const double* lam_in, double* lam_out,
                      double* dJ) {
        const sph::State user = user_state(ck, prm);
        const sph::State s1 = ws_state(ws, L.s1, prm, n);
        const sph::State s2 = ws_state(ws, L.s2, prm, n);
        SPH_TRY(copy(user, s2));
        sph::State cur = s2, nxt = s1;
        SPH_TRY(zero_counts());
        for (int64_t s = 0; s < k; ++s) {
            tape_records(s);
            SPH_TRY(sort_into(cur, nxt, true, false, s > 0));
            SPH_TRY(density(nxt, start(), start() + 1, true));
            SPH_TRY(momentum(nxt, start(), start() + 1, true, s < k - 1));
            std::swap(cur, nxt);
        }
        const int64_t N = n;
        const double hdt = 0.5 * prm->dt;
        double* bufs[2] = {(double*)(ws + L.lamB), (double*)(ws + L.lamC)};
        const double* in = lam_in;
        for (int64_t s = k - 1; s >= 0; --s) {
            tape_records(s);
            double* out = s == 0 ? lam_out : bufs[s & 1];
            SPH_TRY(adjoint_rhs(in + DIM * N, in + 2 * DIM * N, N, hdt, typetape, nullptr, dJ,
                                true));
            launch(K_ADJ_KICK, sph::k_adj_kick<DIM>, blocks_for(n), st,
                n, in, (const double*)(ws + L.lxd), (const double*)(ws + L.lvd), typetape, perm(),
                prm->dt, hdt, out);
            SPH_TRY(launch_check("k_adj_kick"));
            in = out;
        }
        default_records();
        return SPH_OK;
    }

    // Adjoint of one acceleration evaluation at the (unsorted) state st.
    int accel_backward(const sph_particles* stp, const double* lam_a, double* lam_x,
                       double* lam_u, double* dJ) {
        const sph::State user = user_state(stp, prm);
        const sph::State s1 = ws_state(ws, L.s1, prm, n);
        default_records();
        SPH_TRY(zero_counts());
        SPH_TRY(sort_into(user, s1, false, false));
        SPH_TRY(density(s1, start(), start() + 1, true));
        // the adjoint passes read global-format lists: rebuilt if the density
        // went through the tiles
        SPH_TRY(adjoint_rhs(nullptr, lam_a, n, 0.0, s1.type, perm(), dJ, tiled()));
        launch(K_ADJ_KICK, sph::k_adj_accum<DIM>, blocks_for(n), st,
            n, (const double*)(ws + L.lxd), (const double*)(ws + L.lvd), s1.type, perm(), lam_x,
            lam_u);
        return launch_check("k_adj_accum");
    }
};


// Common preparation: grid, layout, workspace check, engine.
template <int DIM, int KERNEL, typename T>
int make_engine(const sph_params* p, const sph_particles* pa, void* ws, size_t ws_bytes,
                void* stream, Engine<DIM, KERNEL, T>* E, int64_t adj_k = 0) {
    int64_t ncells;
    SPH_TRY(make_grid(p, &E->G, &ncells));
    E->prm = p;
    E->ncells = ncells;
    E->n = (int)pa->n;
    E->L = make_layout(p, E->G, pa->n, ncells, adj_k);
    if (!ws) return fail(SPH_EINVAL, "workspace is NULL");
    if ((uintptr_t)ws % 256 != 0) return fail(SPH_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < E->L.bytes)
        return fail(SPH_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, E->L.bytes);
    E->ws = (char*)ws;
    E->st = (hipStream_t)stream;
    E->C = pair_const<T>(p, E->G);
    E->default_records();
    return SPH_OK;
}

// The entry points for one (dimension, kernel, pair precision).  Declared
// here, defined out of class below and instantiated explicitly, one
// combination per translation unit (sph_part.hip), so that the library
// builds in parallel; the C ABI (sph.hip) only calls them.
template <int DIM, int KERNEL, typename T>
struct Api {
    static int bin_sort(const sph_params* p, sph_particles* pa, void* ws, size_t wb, uint32_t* cs,
                        uint32_t* ce, void* st);
    static int density(const sph_params* p, sph_particles* pa, const uint32_t* cs,
                       const uint32_t* ce, void* ws, size_t wb, void* st);
    static int momentum(const sph_params* p, sph_particles* pa, const uint32_t* cs,
                        const uint32_t* ce, void* ws, size_t wb, void* st);
    static int eos(const sph_params* p, sph_particles* pa, void* st);
    static int neighbors(const sph_params* p, const sph_particles* pa, const uint32_t* cs,
                         const uint32_t* ce, int64_t cap, int64_t* off, int32_t* nbr,
                         int64_t* total, void* ws, size_t wb, void* st);
    static int step(const sph_params* p, sph_particles* pa, int64_t nsteps, int prime, void* ws,
                    size_t wb, double* diag, void* st);
    static int step_backward(const sph_params* p, const sph_particles* ck, int64_t k,
                             const double* lin, double* lout, double* dJ, void* ws, size_t wb,
                             void* st);
    static int accel_backward(const sph_params* p, const sph_particles* stp, const double* la,
                              double* lx, double* lu, double* dJ, void* ws, size_t wb, void* st);
};

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::bin_sort(const sph_params* p, sph_particles* pa, void* ws, size_t wb,
                                  uint32_t* cs, uint32_t* ce, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, pa, ws, wb, st, &E));
    return E.bin_sort(pa, cs, ce);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::density(const sph_params* p, sph_particles* pa, const uint32_t* cs,
                                 const uint32_t* ce, void* ws, size_t wb, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, pa, ws, wb, st, &E));
    return E.density_only(pa, cs, ce);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::momentum(const sph_params* p, sph_particles* pa, const uint32_t* cs,
                                  const uint32_t* ce, void* ws, size_t wb, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, pa, ws, wb, st, &E));
    return E.momentum_only(pa, cs, ce);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::eos(const sph_params* p, sph_particles* pa, void* st) {
    Engine<DIM, KERNEL, T> E;
    E.prm = p;
    E.n = (int)pa->n;
    E.st = (hipStream_t)st;
    int64_t ncells;
    SPH_TRY(make_grid(p, &E.G, &ncells));
    E.C = pair_const<T>(p, E.G);
    return E.eos_only(pa);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::neighbors(const sph_params* p, const sph_particles* pa,
                                   const uint32_t* cs, const uint32_t* ce, int64_t cap,
                                   int64_t* off, int32_t* nbr, int64_t* total, void* ws,
                                   size_t wb, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, pa, ws, wb, st, &E));
    return E.neighbors(pa, cs, ce, cap, off, nbr, total);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::step(const sph_params* p, sph_particles* pa, int64_t nsteps, int prime,
                              void* ws, size_t wb, double* diag, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, pa, ws, wb, st, &E));
    if (p->scheme == SPH_SCHEME_CONTINUITY) return E.step_continuity(pa, nsteps, prime, diag);
    return E.step(pa, nsteps, prime, diag);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::step_backward(const sph_params* p, const sph_particles* ck, int64_t k,
                                       const double* lin, double* lout, double* dJ, void* ws,
                                       size_t wb, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, ck, ws, wb, st, &E, k));
    return E.step_backward(ck, k, lin, lout, dJ);
}

template <int DIM, int KERNEL, typename T>
int Api<DIM, KERNEL, T>::accel_backward(const sph_params* p, const sph_particles* stp,
                                        const double* la, double* lx, double* lu, double* dJ,
                                        void* ws, size_t wb, void* st) {
    Engine<DIM, KERNEL, T> E;
    SPH_TRY(make_engine(p, stp, ws, wb, st, &E, 1));
    return E.accel_backward(stp, la, lx, lu, dJ);
}

// Every (dimension, kernel, pair precision) the library is built for.
#define SPH_FOR_EACH_COMBO(X) \
    X(2, 0, float) X(2, 1, float) X(2, 2, float) X(2, 0, double) X(2, 1, double) X(2, 2, double) \
    X(3, 0, float) X(3, 1, float) X(3, 2, float) X(3, 0, double) X(3, 1, double) X(3, 2, double)

// Calls fn(Api<DIM, KERNEL, T>()) for the combination the parameters name.
template <typename Fn>
int dispatch(const sph_params* p, Fn&& fn) {
    const bool f64 = p->precision == SPH_FP64;
    const int k = p->kernel == SPH_CUBIC_SPLINE ? 0 : (p->kernel == SPH_QUINTIC_SPLINE ? 2 : 1);
#define SPH_DISPATCH_CASE(D, K, TT) \
    if (p->dim == D && k == K && f64 == (sizeof(TT) == 8)) return fn(Api<D, K, TT>());
    SPH_FOR_EACH_COMBO(SPH_DISPATCH_CASE)
#undef SPH_DISPATCH_CASE
    return fail(SPH_EINVAL, "no build for dim %d, kernel %d", p->dim, p->kernel);
}

}  // namespace sph_host
