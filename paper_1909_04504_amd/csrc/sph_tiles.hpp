// LDS-staged cell tiles for the 3D mixed-precision pair passes.
//
// The cell grid (Sec. 2.2) is cut into boxes of tw x th x td cells.  A
// workgroup takes one box: its targets are the particles of the box's cells,
// its candidates those of the union box (the box grown by the stencil reach S
// on every side), which holds every neighbour of every target.  The union is
// staged in LDS once per workgroup; the targets then find their neighbours,
// and later gather their neighbours' records, from LDS instead of from
// cache-resident global memory.
//
//  * Frame: a staged position is the fixed-point offset of the particle from
//    its cell centre plus its union cell's index times 2^27, so the
//    separation of two staged particles is the same exact integer as the
//    cell-relative one of pair_geom; the pair terms are bitwise those of the
//    global passes.  A float copy, relative to the union centre, filters
//    candidates outside a band around (2h)^2 (its error is below a tenth of
//    the band); the exact predicate decides inside the band.
//  * Walk order: rows (z, y) in stencil order, x cells ascending, slots
//    ascending -- the order of walk_pairs -- so the lists, their counts and
//    every sum are those of the global passes.  Rows whose y/z distance from
//    the target leaves no room for a neighbour are skipped and the others are
//    clipped in x to the cells the support can reach (with a margin of 1e-4 of
//    R^2 and of a cell), which drops only candidates the predicate rejects.
//  * Lists: entries are 16-bit union indices, written by each lane in
//    octets (16 bytes, one store per eight entries) into tiles of 64 sorted
//    slots: entry k of slot i at ((i/64) cap/8 + k/8) 64 + i%64 octets.  They
//    are only meaningful to the tile passes of the same grid.
//  * Targets the tile passes cannot take -- more neighbours than the list
//    capacity, or a tile whose union does not fit in LDS (then every target's
//    count is set to kTileOverflow) -- are left to the fallback kernels, which
//    walk the cells in global memory with the same arithmetic.  A build that
//    leaves any such target stores its epoch in the workspace's fallback
//    word; the fallback kernels exit at once when the word holds another
//    epoch.
#pragma once

#include "sph_kernels.hpp"

namespace sph {

constexpr int kTileThreads = 512;                // 8 waves per workgroup
constexpr int kTileCellsMax = 1024;              // union cells per tile (two per thread)
constexpr int kTileTargetCellsMax = 160;         // target cells per tile
constexpr int kTileCap = 3072;                   // union particles staged in LDS
constexpr int kTileUnionAxisMax = 12;            // union cells per axis: 12 * 2^27 + 2^29 < 2^31
constexpr uint32_t kTileOverflow = 0xffffffffu;  // count of a target left to the fallback
constexpr int kFallbackBlocks = 1024;            // grid of the fallback kernels (grid-stride)

// Tile geometry of one grid (host-computed).
struct Tiles {
    int S;                 // stencil reach
    int tw, th, td;        // tile box, cells
    int uw, uh, ud;        // union box: tile box + S cells on each side
    int nt[3];             // tiles per axis
    int ntiles;
    int cap;               // staged particles per tile (<= kTileCap)
    float csf[3];          // cell sizes
    float inv_csf[3];
    int cen[3];            // union centre in cells (uw/2, uh/2, ud/2): origin of the float copy
    float rclip2;          // R^2 (1 + 1e-4): rows farther than this hold no neighbour
    float clip_pad;        // 1e-4 of a cell: padding of a row's clipped x range
    float inv_uw, inv_uwh; // 1 / uw, 1 / (uw uh): union cell coordinates (union_coords)
};

// q = floor(c / d) for 0 <= c < 2^10 and 1 <= d <= 144, inv_d = fl(1 / d):
// (c + 1/2) / d is at least 1/(2d) >= 1/288 away from an integer, and the
// FP32 product (c + 1/2) inv_d is within 2^-12 of it, so its truncation is
// exact (a few VALU instructions instead of an integer division).
static_assert(kTileCellsMax <= 1024 && kTileUnionAxisMax * kTileUnionAxisMax <= 144,
              "small_quot's range");
__device__ __forceinline__ int small_quot(int c, float inv_d) {
    return (int)(((float)c + 0.5f) * inv_d);
}
// Coordinates (ux, uy, uz) of union cell c of a tile.
__device__ __forceinline__ void union_coords(const Tiles& TL, int c, int uc[3]) {
    const int z = small_quot(c, TL.inv_uwh);
    const int r = c - z * (TL.uw * TL.uh);
    const int y = small_quot(r, TL.inv_uw);
    uc[0] = r - y * TL.uw;
    uc[1] = y;
    uc[2] = z;
}

// Per-workgroup bookkeeping in LDS.
struct TileMeta {
    uint32_t off[kTileCellsMax + 1];  // union index of each cell's first particle; off[ncu] = total
    uint32_t gs[kTileCellsMax];       // global slot of each cell's first particle
    uint32_t tpre[kTileTargetCellsMax + 1];  // targets before each target cell
    int tc[kTileTargetCellsMax];             // union index of each target cell
    int ntcells;
    uint32_t total, ntargets;
    uint32_t wsum[kTileThreads / 64];
};

// Exclusive scan of two counts per thread (cells 2t, 2t+1) over the
// workgroup; returns the offset of cell 2t, total in *total.
__device__ __forceinline__ uint32_t tile_scan2(uint32_t a, uint32_t b, TileMeta& M,
                                               uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t v = a + b;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) M.wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kTileThreads / 64; ++k) {
        before += k < w ? M.wsum[k] : 0u;
        all += M.wsum[k];
    }
    __syncthreads();  // wsum is reused by the next scan
    *total = all;
    return before + incl - v;
}

// Global cell coordinate of union coordinate u along axis k of a tile whose
// box starts at cell c0; -1 outside a non-periodic grid.
__device__ __forceinline__ int tile_axis(const Grid& G, int k, int c0, int u, int S) {
    int c = c0 - S + u;
    const int nc = G.nc[k];
    if (c >= 0 && c < nc) return c;
    if (!G.periodic[k]) return -1;
    // c lies within a few grid lengths: wrap by steps, not by a division
    while (c < 0) c += nc;
    while (c >= nc) c -= nc;
    return c;
}

// Tile origin (first cell) of tile t.
__device__ __forceinline__ void tile_origin(const Tiles& TL, int t, int c0[3]) {
    c0[0] = (t % TL.nt[0]) * TL.tw;
    c0[1] = ((t / TL.nt[0]) % TL.nt[1]) * TL.th;
    c0[2] = (t / (TL.nt[0] * TL.nt[1])) * TL.td;
}

// Whether the tile's box holds no particle: the keys of its cells lie
// between those of its first and last corner cells (row-major and Z-order
// keys both grow with each coordinate), so an empty slot range between them
// means empty cells.  Two loads per workgroup, before any other work.
__device__ __forceinline__ bool tile_empty(const Grid& G, const Tiles& TL, const int c0[3],
                                           const uint32_t* __restrict__ cstart,
                                           const uint32_t* __restrict__ cend) {
    __shared__ uint32_t se[2];
    if (threadIdx.x == 0) {
        const int a[3] = {c0[0], c0[1], c0[2]};
        const int b[3] = {min(c0[0] + TL.tw, G.nc[0]) - 1, min(c0[1] + TL.th, G.nc[1]) - 1,
                          min(c0[2] + TL.td, G.nc[2]) - 1};
        se[0] = cstart[cell_key(a, G)];
        se[1] = cend[cell_key(b, G)];
    }
    __syncthreads();
    return se[1] <= se[0];
}

// Cell ranges of the union, their scan, and the target cells, in two
// halves: tile_setup_loads issues each thread's loads (union cells 2t and
// 2t + 1), tile_setup_finish forms the counts, the scans and the target
// cells from them (so that a pass can have the loads in flight while it
// works on another tile).
struct SetupLoads {
    uint32_t s[2], e[2];
    bool in[2];
};
// Marks a loaded value as used here and not before: the compiler otherwise
// moves its first use (and the wait for the load) up to where the load was
// issued, ahead of loads that were meant to overlap it.
template <typename V>
__device__ __forceinline__ void keep_in_flight(V& v) {
    static_assert(sizeof(V) % 4 == 0, "whole registers");
    uint32_t* w = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(V) / 4); ++k) asm volatile("" : "+v"(w[k]));
}
__device__ __forceinline__ SetupLoads tile_setup_loads(const Grid& G, const Tiles& TL,
                                                       const int c0[3],
                                                       const uint32_t* __restrict__ cstart,
                                                       const uint32_t* __restrict__ cend) {
    const int ncu = TL.uw * TL.uh * TL.ud;
    SetupLoads r;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int c = 2 * (int)threadIdx.x + q;
        r.s[q] = r.e[q] = 0;
        r.in[q] = false;
        if (c < ncu) {
            int uc[3];
            union_coords(TL, c, uc);
            const int gx = tile_axis(G, 0, c0[0], uc[0], TL.S);
            const int gy = tile_axis(G, 1, c0[1], uc[1], TL.S);
            const int gz = tile_axis(G, 2, c0[2], uc[2], TL.S);
            if (gx >= 0 && gy >= 0 && gz >= 0) {
                const int gc[3] = {gx, gy, gz};
                const uint32_t key = cell_key(gc, G);
                r.s[q] = cstart[key];
                r.e[q] = cend[key];
                r.in[q] = true;
            }
        }
    }
    return r;
}
// Returns the number of union particles (every thread).
__device__ __forceinline__ uint32_t tile_setup_finish(const Grid& G, const Tiles& TL,
                                                      const int c0[3], int n,
                                                      const SetupLoads& r, TileMeta& M) {
    const int ncu = TL.uw * TL.uh * TL.ud;
    uint32_t cnt[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int c = 2 * (int)threadIdx.x + q;
        cnt[q] = 0;
        if (c < ncu) {
            uint32_t s = 0;
            if (r.in[q]) {
                s = r.s[q];
                const uint32_t e = r.e[q] < (uint32_t)n ? r.e[q] : (uint32_t)n;
                cnt[q] = e > s ? e - s : 0u;
            }
            M.gs[c] = s;
        }
    }
    uint32_t total;
    const uint32_t o = tile_scan2(cnt[0], cnt[1], M, &total);
    {
        const int c = 2 * (int)threadIdx.x;
        if (c < ncu) M.off[c] = o;
        if (c + 1 < ncu) M.off[c + 1] = o + cnt[0];
    }
    if (threadIdx.x == 0) {
        M.off[ncu] = total;
        M.total = total;
    }
    __syncthreads();
    // target cells: the box's cells inside the grid, each its own slot range
    // (with Z-order keys the cells of a row are not adjacent); thread r
    // takes target cell r, and a workgroup scan gives their offsets
    const int twc = min(TL.tw, G.nc[0] - c0[0]);
    const int thc = min(TL.th, G.nc[1] - c0[1]);
    const int tdc = min(TL.td, G.nc[2] - c0[2]);
    const int ntc = twc * thc * tdc;
    const int rr = (int)threadIdx.x;
    uint32_t tcnt = 0;
    int tcell = 0;
    if (rr < ntc) {
        // rr < kTileTargetCellsMax, twc thc <= 144: exact FP32 quotients
        const int z = small_quot(rr, __builtin_amdgcn_rcpf((float)(twc * thc)));
        const int rem = rr - z * (twc * thc);
        const int y = small_quot(rem, __builtin_amdgcn_rcpf((float)twc));
        const int x = rem - y * twc;
        tcell = (TL.S + x) + TL.uw * ((TL.S + y) + TL.uh * (TL.S + z));
        tcnt = M.off[tcell + 1] - M.off[tcell];
    }
    uint32_t ntargets;
    const uint32_t tpre = tile_scan2(tcnt, 0u, M, &ntargets);
    if (rr < ntc) {
        M.tc[rr] = tcell;
        M.tpre[rr] = tpre;
    }
    if (threadIdx.x == 0) {
        M.tpre[ntc] = ntargets;
        M.ntcells = ntc;
        M.ntargets = ntargets;
    }
    __syncthreads();
    return total;
}
__device__ __forceinline__ uint32_t tile_setup(const Grid& G, const Tiles& TL, const int c0[3],
                                               const uint32_t* __restrict__ cstart,
                                               const uint32_t* __restrict__ cend, int n,
                                               TileMeta& M) {
    return tile_setup_finish(G, TL, c0, n, tile_setup_loads(G, TL, c0, cstart, cend), M);
}

// Target t of the tile: its union index, global slot and union cell coords.
__device__ __forceinline__ void tile_target(const Tiles& TL, const TileMeta& M, uint32_t t,
                                            uint32_t* ui, uint32_t* gi, int uc[3]) {
    // the target cell: the last r with tpre[r] <= t (binary search)
    int lo = 0, hi = M.ntcells;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (M.tpre[mid] <= t) lo = mid; else hi = mid;
    }
    const int c = M.tc[lo];
    const uint32_t k = t - M.tpre[lo];
    *ui = M.off[c] + k;
    *gi = M.gs[c] + k;
    union_coords(TL, c, uc);
}

// Marks every target of the tile for the fallback (its union does not fit).
__device__ __forceinline__ void tile_mark_overflow(const TileMeta& M, uint32_t* __restrict__ ncnt) {
    for (int r = 0; r < M.ntcells; ++r) {
        const uint32_t len = M.tpre[r + 1] - M.tpre[r];
        for (uint32_t k = threadIdx.x; k < len; k += kTileThreads)
            ncnt[M.gs[M.tc[r]] + k] = kTileOverflow;
    }
}

// Stages the union's records: store(u, load(j), ux, uy, uz) for union
// particle u held in global slot j of union cell (ux, uy, uz).  The cell of
// every union index is noted first (tile_cellof), so that each thread then
// loads its particles at indices t, t + 512, ... with all loads in flight
// (tile_stage_loads; kTileCap <= 8 * kTileThreads: a single round) and
// stores them (tile_stage_store).  cellof: kTileCap entries of LDS, the
// union cell of each staged particle.
__device__ __forceinline__ void tile_cellof(const Tiles& TL, const TileMeta& M,
                                            uint16_t* cellof) {
    const int ncu = TL.uw * TL.uh * TL.ud;
    for (int c = threadIdx.x; c < ncu; c += kTileThreads)
        for (uint32_t u = M.off[c]; u < M.off[c + 1]; ++u) cellof[u] = (uint16_t)c;
    __syncthreads();
}
constexpr int kStageQ = (kTileCap + kTileThreads - 1) / kTileThreads;
static_assert(kStageQ <= 8, "staging registers");
template <typename P>
struct StageRegs {
    P v[kStageQ];
};
template <typename P, typename Load>
__device__ __forceinline__ void tile_stage_loads(const TileMeta& M, const uint16_t* cellof,
                                                 Load&& load, StageRegs<P>& R) {
    const uint32_t total = M.total;
#pragma unroll
    for (int q = 0; q < kStageQ; ++q) {
        const uint32_t u = threadIdx.x + (uint32_t)q * kTileThreads;
        if (u < total) {
            const int c = cellof[u];
            R.v[q] = load(M.gs[c] + (u - M.off[c]));
        }
    }
}
template <typename P, typename Store>
__device__ __forceinline__ void tile_stage_store(const Tiles& TL, const TileMeta& M,
                                                 const uint16_t* cellof, const StageRegs<P>& R,
                                                 Store&& store) {
    const uint32_t total = M.total;
#pragma unroll
    for (int q = 0; q < kStageQ; ++q) {
        const uint32_t u = threadIdx.x + (uint32_t)q * kTileThreads;
        if (u < total) {
            int uc[3];
            union_coords(TL, cellof[u], uc);
            store(u, R.v[q], uc[0], uc[1], uc[2]);
        }
    }
}
template <typename Load, typename Store>
__device__ __forceinline__ void tile_stage(const Tiles& TL, TileMeta& M, uint16_t* cellof,
                                           Load&& load, Store&& store) {
    tile_cellof(TL, M, cellof);
    using P = decltype(load(0u));
    StageRegs<P> R;
    tile_stage_loads(M, cellof, load, R);
    tile_stage_store(TL, M, cellof, R, store);
}

// Union-frame record: cell-relative fixed point plus the union cell times 2^27.
__device__ __forceinline__ int4 tile_rec(const int4& r, int ux, int uy, int uz) {
    int4 p;
    p.x = ux * (1 << kFixBits) + r.x;
    p.y = uy * (1 << kFixBits) + r.y;
    p.z = uz * (1 << kFixBits) + r.z;
    p.w = r.w;
    return p;
}

// Octet k8 (entries 8 k8 .. 8 k8 + 7) of slot i's list.
__device__ __forceinline__ size_t tile_octet(uint32_t i, uint32_t cap, uint32_t k8) {
    return ((size_t)(i >> 6) * (cap >> 3) + k8) * 64 + (i & 63);
}
__device__ __forceinline__ uint32_t half_of(const uint4& v, int e) {
    const uint32_t w = e < 2 ? v.x : (e < 4 ? v.y : (e < 6 ? v.z : v.w));
    return (e & 1) ? (w >> 16) : (w & 0xffffu);
}

// The first two octets of slot i's list, fetched before its count is known
// (both within the slot's cap / 8 octets, so always in bounds), for
// tile_list_loop.
struct ListHead {
    uint4 o0, o1;
};
__device__ __forceinline__ ListHead tile_list_head(const uint4* __restrict__ list, uint32_t i,
                                                  uint32_t cap) {
    const uint4* __restrict__ base = list + tile_octet(i, cap, 0);
    return ListHead{base[0], base[cap >= 16 ? 64 : 0]};
}

// Calls body(load(u)) for the cnt entries u of slot i's list, in order
// (head: tile_list_head of the slot).  The loads of a full octet's eight
// entries are issued together and the next octet is fetched meanwhile; the
// last, partial octet goes entry by entry.  Octet fetches are unconditional,
// their index clamped to the list's last octet, so that the rotating octets
// stay in registers (a conditional fetch makes the compiler keep them in
// scratch memory and wait on every fetch at the top of the loop).  Two
// octets per iteration, for a longer fetch distance, measured slower (the
// larger code and register count cost more than the latency they hide).
template <int kGroup = 8, typename Load, typename Body>
__device__ __forceinline__ void tile_list_loop(const uint4* __restrict__ list, uint32_t i,
                                               uint32_t cap, uint32_t cnt, const ListHead& head,
                                               Load&& load, Body&& body) {
    static_assert(kGroup == 8 || kGroup == 4, "whole or half octets");
    using P = decltype(load(0u));
    const uint32_t nfull = cnt >> 3, rest = cnt & 7u;
    const uint32_t noct = nfull + (rest ? 1u : 0u);
    if (noct == 0) return;
    const uint32_t last = noct - 1;
    // octet k8 of the slot is 64 k8 uint4 after its first
    const uint4* __restrict__ base = list + tile_octet(i, cap, 0);
    uint4 nxt = head.o0;
    uint4 nxt2 = head.o1;
    for (uint32_t k8 = 0; k8 < nfull; ++k8) {
        const uint4 cur = nxt;
        nxt = nxt2;
        nxt2 = base[(size_t)min(k8 + 2, last) * 64];
#pragma unroll
        for (int h = 0; h < 8; h += kGroup) {
            P p[kGroup];
#pragma unroll
            for (int e = 0; e < kGroup; ++e) p[e] = load(half_of(cur, h + e));
#pragma unroll
            for (int e = 0; e < kGroup; ++e) body(p[e]);
        }
    }
    if (rest) {
#pragma unroll
        for (int e = 0; e < 7; ++e)
            if ((uint32_t)e < rest) body(load(half_of(nxt, e)));
    }
}

// Per-thread FP64 values summed over the workgroup (wave butterflies, then
// the waves in order) into part[q * stride + b].
template <int NV>
__device__ __forceinline__ void tile_block_sum(double v[NV], double* __restrict__ part, int b,
                                               int stride) {
    __shared__ double sh[NV][kTileThreads / 64];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
        v[q] = x;
    }
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < NV; ++q) sh[q][threadIdx.x >> 6] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < kTileThreads / 64; ++w) s += sh[q][w];
            part[(int64_t)q * stride + b] = s;
        }
}

// Workgroup sum of a per-thread count into the tile's interaction counter.
__device__ __forceinline__ void tile_count(uint32_t cnt, unsigned long long* __restrict__ pairs,
                                           int blk) {
    __shared__ uint32_t wc[kTileThreads / 64];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kTileThreads / 64; ++w) t += wc[w];
        add_pairs(pairs, blk, t);
    }
}

// Neighbour lists of the tile's targets: ncnt[i] = |N(i)|, entries while the
// count is within cap; targets with more are left to the fallback, as are all
// targets of a tile whose union exceeds cap_union.  count_pairs: the
// interactions of the counted targets go to the tile's counter.  Only the
// float copy of the union is staged (so that two workgroups share a CU); the
// exact predicate inside the band reads the candidate's record from global
// memory.  Entries are appended without branches: every candidate is written
// at the next free place of a 16-entry ring and the count advances only for
// accepted ones; a completed octet is stored at once.
template <int S>
__global__ __launch_bounds__(kTileThreads) void k_tile_build(
    int n, Grid G, PairConst<float> C, Tiles TL, int cap_union, const int4* __restrict__ pos,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, uint32_t cap,
    uint4* __restrict__ list, uint32_t* __restrict__ ncnt, int count_pairs,
    unsigned long long* __restrict__ pairs, uint32_t epoch, uint32_t* __restrict__ fallback) {
    __shared__ TileMeta M;
    // float copy of the union (w: the particle's union cell), + the
    // candidates read past a row's end
    __shared__ float4 Pf[kTileCap + 8];
    // each thread's ring of 16 list entries (two octets), 40 bytes apart so
    // that the lanes' appends spread over the LDS banks; the staging's cell
    // table before that
    constexpr int kRingStride = 5;  // uint2 per thread
    __shared__ uint2 ringbuf[kTileThreads * kRingStride];
    static_assert(sizeof(ringbuf) >= kTileCap * sizeof(uint16_t), "cell table");
    const int blk = xcd_block();
    int c0[3];
    tile_origin(TL, blk, c0);
    // the cell-range loads go out before the empty-box probe, so that the
    // two round trips overlap
    const SetupLoads sl = tile_setup_loads(G, TL, c0, cstart, cend);
    if (tile_empty(G, TL, c0, cstart, cend)) {
        if (count_pairs) tile_count(0u, pairs, blk);
        return;
    }
    const uint32_t total = tile_setup_finish(G, TL, c0, n, sl, M);
    if (total > (uint32_t)cap_union) {
        tile_mark_overflow(M, ncnt);
        if (threadIdx.x == 0 && M.ntargets) *fallback = epoch;
        // the counter is still touched: tile 0 raises the number of counters
        // the reader sums
        if (count_pairs) tile_count(0u, pairs, blk);
        return;
    }
    tile_stage(TL, M, (uint16_t*)ringbuf, [&](uint32_t j) { return pos[j]; },
               [&](uint32_t u, const int4& r, int ux, int uy, int uz) {
                   const int4 p = tile_rec(r, ux, uy, uz);
                   float4 f;
                   f.x = (float)(p.x - TL.cen[0] * (1 << kFixBits)) * C.fix_scale_f[0];
                   f.y = (float)(p.y - TL.cen[1] * (1 << kFixBits)) * C.fix_scale_f[1];
                   f.z = (float)(p.z - TL.cen[2] * (1 << kFixBits)) * C.fix_scale_f[2];
                   f.w = __int_as_float(ux + TL.uw * (uy + TL.uh * uz));
                   Pf[u] = f;
               });
    __syncthreads();
    uint2* const myring = &ringbuf[threadIdx.x * kRingStride];
    uint16_t* my = (uint16_t*)myring;
    auto ring_octet = [&](uint32_t k8) {
        const uint2 lo = myring[2 * (k8 & 1)], hi = myring[2 * (k8 & 1) + 1];
        return make_uint4(lo.x, lo.y, hi.x, hi.y);
    };
    uint32_t counted = 0;
    bool need_fb = false;
    const float cxf = (float)TL.cen[0], cyf = (float)TL.cen[1], czf = (float)TL.cen[2];
    for (uint32_t t = threadIdx.x; t < M.ntargets; t += kTileThreads) {
        uint32_t ui, i;
        int uc[3];
        tile_target(TL, M, t, &ui, &i, uc);
        const float4 pf = Pf[ui];
        const int4 pi = tile_rec(pos[i], uc[0], uc[1], uc[2]);
        // rows are clipped only for a target inside its cell (a particle
        // clamped into an edge cell from outside a non-periodic box walks
        // whole rows, as walk_pairs does)
        const int half = 1 << (kFixBits - 1);
        const bool clip = abs(pi.x - uc[0] * (1 << kFixBits)) <= half &&
                          abs(pi.y - uc[1] * (1 << kFixBits)) <= half &&
                          abs(pi.z - uc[2] * (1 << kFixBits)) <= half;
        // exact predicate on the integer separation (candidate's record from
        // global memory, in the union frame)
        auto exact = [&](uint32_t u) {
            const int c = __float_as_int(Pf[u].w);
            int cu[3];
            union_coords(TL, c, cu);
            const int4 pj = tile_rec(pos[M.gs[c] + (u - M.off[c])], cu[0], cu[1], cu[2]);
            const Geom<float> g = pair_geom<3>(pi, pj, 0, 0, 0, 0, 0, 0, C);
            return geom_r2d(g, C) < C.R2_d;
        };
        uint32_t cnt = 0;
        // the (2S+1)^2 stencil rows in walk order (z planes, then y rows);
        // loops, not unrolled, so the kernel's code stays small enough for the
        // instruction cache.  A plane's distance is taken once for its rows,
        // and the x range in cell units from px_c, the target's x in cells
        // shifted by the union centre and 1/2 (the clip keeps its margins:
        // roundings of these forms move it by far less than clip_pad)
        constexpr int NR = 2 * S + 1;
        const float px_c = pf.x * TL.inv_csf[0] + (cxf + 0.5f);
#pragma unroll 1
        for (int iz = 0; iz < NR; ++iz) {
            const int uz = uc[2] + iz - S;
            const float dz =
                fmaxf(fabsf(pf.z - ((float)uz - czf) * TL.csf[2]) - 0.5f * TL.csf[2], 0.f);
            const float w2z = TL.rclip2 - dz * dz;
            if (clip && !(w2z > 0.f)) continue;
            const int planec = TL.uw * TL.uh * uz;
#pragma unroll 1
            for (int iy = 0; iy < NR; ++iy) {
                const int uy = uc[1] + iy - S;
                const float dy =
                    fmaxf(fabsf(pf.y - ((float)uy - cyf) * TL.csf[1]) - 0.5f * TL.csf[1], 0.f);
                const float w2 = w2z - dy * dy;
                if (clip && !(w2 > 0.f)) continue;
                int xa = uc[0] - S, xb = uc[0] + S;
                if (clip) {
                    const float wc = (__builtin_amdgcn_sqrtf(w2) + TL.clip_pad) * TL.inv_csf[0];
                    xa = max(xa, (int)floorf(px_c - wc));
                    xb = min(xb, (int)floorf(px_c + wc));
                    if (xa > xb) continue;
                }
                const int rowc = planec + TL.uw * uy;
                const uint32_t ua = M.off[rowc + xa], ue = M.off[rowc + xb + 1];
                // candidates four at a time, the next four loaded while these
                // are tested; those past the row's end (read from the padding or
                // the next row) are infinitely far
                uint32_t u = ua;
                float4 c[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) c[q] = Pf[u + q];
#pragma unroll 1
                for (; u < ue; u += 4) {
                    const uint32_t lim = ue - u;  // candidates left in the row
                    float r2[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float dx = pf.x - c[q].x, ddy = pf.y - c[q].y, ddz = pf.z - c[q].z;
                        r2[q] = dx * dx + ddy * ddy + ddz * ddz;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) c[q] = Pf[u + 4 + q];
                    uint32_t acc[4];
                    bool band[4];
                    bool anyband = false;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float x = (uint32_t)q < lim ? r2[q] : __builtin_huge_valf();
                        acc[q] = x < C.R2_lo ? 1u : 0u;
                        band[q] = fabsf(x - C.R2_mid) < C.R2_w;
                        anyband |= band[q];
                    }
                    if (__builtin_amdgcn_ballot_w64(anyband)) {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (band[q]) acc[q] = exact(u + q) ? 1u : 0u;
                    }
                    const uint32_t c_in = cnt;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        my[cnt & 15] = (uint16_t)(u + q);
                        cnt += acc[q];
                    }
                    // an octet completed (at most one per group of four)
                    if ((cnt ^ c_in) & ~7u) {
                        const uint32_t k8 = c_in >> 3;
                        if (k8 < (cap >> 3)) list[tile_octet(i, cap, k8)] = ring_octet(k8);
                    }
                }
            }
        }
        if (cnt <= cap && (cnt & 7)) list[tile_octet(i, cap, cnt >> 3)] = ring_octet(cnt >> 3);
        ncnt[i] = cnt;
        counted += cnt;
        need_fb |= cnt > cap;
    }
    if (__syncthreads_or(need_fb) && threadIdx.x == 0) *fallback = epoch;
    if (count_pairs) tile_count(counted, pairs, blk);
}

// Summation density (eq. 2), and with_eos the Tait EOS (eq. eos), of the
// tile's targets with complete lists (as k_density), over the union's
// position records staged in LDS.
template <int S, int KERNEL>
__global__ __launch_bounds__(kTileThreads) void k_tile_density(
    int n, Grid G, PairConst<float> C, Tiles TL, int cap_union, const int4* __restrict__ pos,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend, uint32_t cap,
    const uint4* __restrict__ list, const uint32_t* __restrict__ ncnt,
    float* __restrict__ rho_out, float* __restrict__ p_out, float4* __restrict__ vel,
    float2* __restrict__ rp, int with_eos) {
    __shared__ TileMeta M;
    __shared__ int4 Pi[kTileCap];
    __shared__ uint16_t cellof[kTileCap];
    const int blk = xcd_block();
    int c0[3];
    tile_origin(TL, blk, c0);
    const SetupLoads sl = tile_setup_loads(G, TL, c0, cstart, cend);
    if (tile_empty(G, TL, c0, cstart, cend)) return;
    const uint32_t total = tile_setup_finish(G, TL, c0, n, sl, M);
    if (total > (uint32_t)cap_union) return;  // every target is the fallback's
    tile_stage(TL, M, cellof, [&](uint32_t j) { return pos[j]; },
               [&](uint32_t u, const int4& r, int ux, int uy, int uz) {
                   Pi[u] = tile_rec(r, ux, uy, uz);
               });
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < M.ntargets; t += kTileThreads) {
        uint32_t ui, i;
        int uc[3];
        tile_target(TL, M, t, &ui, &i, uc);
        const uint32_t cnt = ncnt[i];
        const ListHead head = tile_list_head(list, i, cap);
        if (cnt > cap) continue;  // the fallback's
        const int4 pi = Pi[ui];
        double acc = 0.0;
        tile_list_loop(list, i, cap, cnt, head, [&](uint32_t u) { return Pi[u]; },
                       [&](const int4& pj) {
                           const Geom<float> g = pair_geom<3>(pi, pj, 0, 0, 0, 0, 0, 0, C);
                           density_add<KERNEL, float>(acc, g, (double)rec_mass(pj), C);
                       });
        finish_density<3, float>((int)i, acc, C, rho_out, 0, p_out, vel, rp, with_eos);
    }
}

// Momentum equation (as k_momentum) of the tile's targets whose lists are
// complete, over the union's position, velocity and (rho, P) records staged
// in LDS, with momentum_close as the epilogue; per-tile partial sums of the
// diagnostics into diag_part[q * stride + tile].
//
// The staging takes most of the LDS, so one workgroup runs per CU and
// nothing else covers its global round trips (a tile's cell ranges, then
// its records, then its targets' counts and list heads: about 45% of the
// pass measured without the pair loops).  Each workgroup therefore takes
// every P-th tile (P workgroups, one per CU, so that the tiles in flight
// are P consecutive ones) and issues, with the loads of its tile t's
// targets, the staging loads of its next tile (whose cell ranges were set
// up before) and the cell-range loads of the one after: the three round
// trips overlap.  (They cannot reach past the first wait of the pair loops:
// the vector memory counter is in order.)  After the pair loops the loaded
// records and ranges go to the LDS that tile t no longer needs; two tile
// metas and two cell tables alternate.  The pair loops take half octets at
// a time, which keeps the staging registers clear of spills.
template <int S, int KERNEL>
__global__ __launch_bounds__(kTileThreads) void k_tile_momentum(
    int n, Grid G, PairConst<float> C, Tiles TL, int cap_union, const int4* __restrict__ pos,
    const float4* __restrict__ vel, const float2* __restrict__ rp,
    const uint8_t* __restrict__ type, const uint32_t* __restrict__ cstart,
    const uint32_t* __restrict__ cend, uint32_t cap, const uint4* __restrict__ list,
    const uint32_t* __restrict__ ncnt, State St, int kick, int drift, double hdt, double dt,
    uint32_t* __restrict__ key, uint32_t* __restrict__ counts, uint32_t* __restrict__ flags,
    double* __restrict__ diag_part, int stride) {
    __shared__ TileMeta MM[2];
    __shared__ uint16_t cellofs[2][kTileCap];
    __shared__ int4 Pi[kTileCap];
    __shared__ float4 V[kTileCap];
    __shared__ float2 RP[kTileCap];
    // tiles w, w + P, w + 2P, ... (P workgroups): the tiles in flight at
    // any time are P consecutive ones, each XCD's a contiguous run of them
    const int P = (int)gridDim.x;
    const int t0 = xcd_block();
    const int t1 = TL.ntiles;
    if (t0 >= t1) return;  // the whole workgroup
    struct Rc {
        int4 p;
        float4 v;
        float2 rp;
    };
    auto load_rc = [&](uint32_t j) { return Rc{pos[j], vel[j], rp[j]}; };
    auto store_rc = [&](uint32_t u, const Rc& r, int ux, int uy, int uz) {
        Pi[u] = tile_rec(r.p, ux, uy, uz);
        V[u] = r.v;
        RP[u] = r.rp;
    };
    auto fits = [&](const TileMeta& M) { return M.total <= (uint32_t)cap_union; };
    int c0[3];
    // prologue: tile t0 set up and staged, tile t0 + 1 set up
    tile_origin(TL, t0, c0);
    tile_setup(G, TL, c0, cstart, cend, n, MM[0]);
    tile_cellof(TL, MM[0], cellofs[0]);
    if (fits(MM[0])) {
        StageRegs<Rc> R0;
        tile_stage_loads(MM[0], cellofs[0], load_rc, R0);
        tile_stage_store(TL, MM[0], cellofs[0], R0, store_rc);
    }
    if (t0 + P < t1) {
        tile_origin(TL, t0 + P, c0);
        tile_setup(G, TL, c0, cstart, cend, n, MM[1]);  // its barriers also publish the staging
        tile_cellof(TL, MM[1], cellofs[1]);
    } else {
        __syncthreads();
    }
    int cur = 0;
    for (int t = t0; t < t1; t += P) {
        const TileMeta& M = MM[cur];
        const TileMeta& MN = MM[cur ^ 1];
        // issued with the targets' loads: the next tile's staging loads and
        // the cell-range loads of the one after
        const bool stage_next = t + P < t1 && fits(MN);
        StageRegs<Rc> R;
        if (stage_next) tile_stage_loads(MN, cellofs[cur ^ 1], load_rc, R);
        const bool setup_next2 = t + 2 * P < t1;
        int c2[3] = {0, 0, 0};
        SetupLoads sl{};
        if (setup_next2) {
            tile_origin(TL, t + 2 * P, c2);
            sl = tile_setup_loads(G, TL, c2, cstart, cend);
        }
        double dsum[4] = {0.0, 0.0, 0.0, 0.0};
        const uint32_t nt = M.ntargets;
        if (fits(M) && nt > 0) {
            // every global load of a target up front (count, type, the list's
            // first octets, the epilogue's state); those of a thread's next
            // target while it works on the current one
            struct Tgt {
                uint32_t ui, i, cnt;
                bool fluid;
                ListHead head;
                CloseIn ci;
            };
            auto target_loads = [&](uint32_t tt) {
                Tgt g;
                int uc[3];
                tile_target(TL, M, tt, &g.ui, &g.i, uc);
                g.cnt = ncnt[g.i];
                g.fluid = type[g.i] == 0;
                g.head = tile_list_head(list, g.i, cap);
                g.ci = close_load<3>((int)g.i, St, drift, diag_part != nullptr);
                return g;
            };
            for (uint32_t tt = threadIdx.x; tt < nt; tt += kTileThreads) {
                const Tgt cur_t = target_loads(tt);
                const uint32_t ui = cur_t.ui, i = cur_t.i, cnt = cur_t.cnt;
                if (cnt > cap) continue;  // the fallback's
                float acc[3] = {0.f, 0.f, 0.f};
                if (cur_t.fluid) {
                    const int4 pi = Pi[ui];
                    const float4 vi = V[ui];
                    const float2 rpi = RP[ui];
                    float ax = C.g[0], ay = C.g[1], az = C.g[2];
                    struct Nb {
                        int4 p;
                        float4 v;
                        float2 rp;
                    };
                    tile_list_loop<4>(list, i, cap, cnt, cur_t.head,
                                   [&](uint32_t u) { return Nb{Pi[u], V[u], RP[u]}; },
                                   [&](const Nb& b) {
                                       const Geom<float> g =
                                           pair_geom<3>(pi, b.p, 0, 0, 0, 0, 0, 0, C);
                                       momentum_add<3, KERNEL, float>(ax, ay, az, g,
                                                                      rec_mass(b.p), vi, rpi,
                                                                      b.v, b.rp, C);
                                   });
                    acc[0] = ax;
                    acc[1] = ay;
                    acc[2] = az;
                }
                double dv[4] = {0.0, 0.0, 0.0, 0.0};
                momentum_close<3, float>((int)i, acc, cur_t.fluid, St, G, kick, drift, hdt, dt,
                                         key, counts, flags, diag_part != nullptr, dv,
                                         &cur_t.ci);
                for (int q = 0; q < 4; ++q) dsum[q] += dv[q];
            }
        }
        if (diag_part) tile_block_sum<4>(dsum, diag_part, t, stride);
        __syncthreads();  // tile t's records, meta and cell table are free
        if (stage_next) {
#pragma unroll
            for (int q = 0; q < kStageQ; ++q) keep_in_flight(R.v[q]);
            tile_stage_store(TL, MN, cellofs[cur ^ 1], R, store_rc);
        }
        if (setup_next2) {
            keep_in_flight(sl.s);
            keep_in_flight(sl.e);
            tile_setup_finish(G, TL, c2, n, sl, MM[cur]);
            tile_cellof(TL, MM[cur], cellofs[cur]);  // its barrier publishes the staging
        } else {
            __syncthreads();
        }
        cur ^= 1;
    }
}

// Fallback density: the targets the tile build left (count above cap, or
// kTileOverflow), by the cell walk in global memory (density_one); only the
// kTileOverflow ones are counted (the build counted the others).
template <int S, int KERNEL>
__global__ __launch_bounds__(kBlock) void k_tile_fallback_density(
    int n, Grid G, PairConst<float> C, const uint32_t* __restrict__ skey,
    const int4* __restrict__ pos, const uint32_t* __restrict__ cstart,
    const uint32_t* __restrict__ cend, const uint32_t* __restrict__ ncnt, uint32_t cap,
    float* __restrict__ rho_out, float* __restrict__ p_out, float4* __restrict__ vel,
    float2* __restrict__ rp, int with_eos, int count_pairs, unsigned long long* __restrict__ pairs,
    uint32_t epoch, const uint32_t* __restrict__ fallback) {
    if (*fallback != epoch) return;
    uint32_t counted = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint32_t c = ncnt[i];
        if (c <= cap) continue;
        // a null list makes density_one walk the cells
        const uint32_t k = density_one<3, S, KERNEL, float>(i, G, C, skey, pos, cstart, cend, n,
                                                            nullptr, ncnt, cap, rho_out, 0, p_out,
                                                            vel, rp, with_eos);
        if (c == kTileOverflow) counted += k;
    }
    if (count_pairs) block_count(counted, pairs, blockIdx.x);
}

// Fallback momentum, as k_tile_fallback_density; diagnostics partials of its
// blocks at diag_part[q * stride + b] (zeros when there is nothing to do).
template <int S, int KERNEL>
__global__ __launch_bounds__(kBlock) void k_tile_fallback_momentum(
    int n, Grid G, PairConst<float> C, const uint32_t* __restrict__ skey,
    const int4* __restrict__ pos, const float4* __restrict__ vel, const float2* __restrict__ rp,
    const uint8_t* __restrict__ type, const uint32_t* __restrict__ cstart,
    const uint32_t* __restrict__ cend, const uint32_t* __restrict__ ncnt, uint32_t cap, State St,
    int kick, int drift, double hdt, double dt, uint32_t* __restrict__ key,
    uint32_t* __restrict__ counts, uint32_t* __restrict__ flags, double* __restrict__ diag_part,
    int stride, uint32_t epoch, const uint32_t* __restrict__ fallback) {
    double dsum[4] = {0.0, 0.0, 0.0, 0.0};
    if (*fallback == epoch) {
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
            if (ncnt[i] <= cap) continue;
            double dv[4] = {0.0, 0.0, 0.0, 0.0};
            momentum_one<3, S, KERNEL, float>(i, G, C, skey, pos, vel, rp, type, cstart, cend, n,
                                              nullptr, ncnt, cap, St, kick, drift, hdt, dt, key,
                                              counts, flags, diag_part != nullptr, dv);
            for (int q = 0; q < 4; ++q) dsum[q] += dv[q];
        }
    }
    if (diag_part) block_sum4<4>(dsum, diag_part, blockIdx.x, stride);
}

}  // namespace sph
