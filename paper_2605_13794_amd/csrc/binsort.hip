// Tile binning: scan of per-entry tile counts, pair emission, LSD radix
// passes (reduce-then-scan form) over the tile bits, the depth order inside
// each tile (a per-tile sort, or for long lists a depth sort of the visible
// entries before the emission), and tile-range detection.  All counts stay on
// the device (no host synchronisation).
#include "common.h"

namespace gsmi {

// ---------------------------------------------------------------------------
// Emission
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;

constexpr int kScanItems = kScanThreads;  // entries per block (per round of a larger block)
constexpr int kScanItLong = 8;            // rounds per block of a long depth-first input

struct EmitIn {
    const float* rec[GS_MAX_CAMS];
    const float* m2d[GS_MAX_CAMS];  // [2][n_in] screen centres, if use_m2d
    const float* depth[GS_MAX_CAMS];
    const int32_t* radius[GS_MAX_CAMS];
    const uint32_t* tiles[GS_MAX_CAMS];
    uint32_t tile_off[GS_MAX_CAMS];
    int32_t TX[GS_MAX_CAMS];
    int32_t TY[GS_MAX_CAMS];
    int n_cams;
    int use_m2d;   // every camera has its component-major centres
    int64_t n_in;  // entries per camera
};

// Per-camera input pointers staged in LDS.  Indexing the kernel-argument
// arrays with a per-lane camera index loads the pointer from memory, and that
// load shares the in-order counter of the data loads behind it, so a kernel
// that issues several rounds of loads would wait after each pointer.
// The pointers keep the global address space: read back from LDS, plain
// pointers would be generic, and generic loads make every wait a full one.
#define GS_GLOBAL __attribute__((address_space(1)))
struct CamPtrs {
    const float GS_GLOBAL* rec[GS_MAX_CAMS];
    const float GS_GLOBAL* m2d[GS_MAX_CAMS];
    const float GS_GLOBAL* depth[GS_MAX_CAMS];
    const int32_t GS_GLOBAL* radius[GS_MAX_CAMS];
    const uint32_t GS_GLOBAL* tiles[GS_MAX_CAMS];
    uint32_t tile_off[GS_MAX_CAMS];
    int32_t TX[GS_MAX_CAMS];
    int32_t TY[GS_MAX_CAMS];
};

__device__ __forceinline__ void stage_cam_ptrs(const EmitIn& E, CamPtrs& P) {
    const int t = threadIdx.x;
    if (t < GS_MAX_CAMS) {
        P.rec[t] = (const float GS_GLOBAL*)E.rec[t];
        P.m2d[t] = (const float GS_GLOBAL*)E.m2d[t];
        P.depth[t] = (const float GS_GLOBAL*)E.depth[t];
        P.radius[t] = (const int32_t GS_GLOBAL*)E.radius[t];
        P.tiles[t] = (const uint32_t GS_GLOBAL*)E.tiles[t];
        P.tile_off[t] = E.tile_off[t];
        P.TX[t] = E.TX[t];
        P.TY[t] = E.TY[t];
    }
    __syncthreads();
}

// Inclusive prefix sum over the wavefront (Hillis-Steele with DPP-free
// cross-lane reads via __shfl_up; 6 steps).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane_id() >= uint32_t(o)) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (256 threads), returns
// the exclusive prefix and writes the block total to *total.
template <int W = 4>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds4, uint32_t* total) {
    const uint32_t inc = wave_incl_scan(v);
    const int w = threadIdx.x / 64;
    if (lane_id() == 63) lds4[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t s = lds4[k];
        if (k < w) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// Adds v to sums[b] for every lane of the wavefront, with one atomic per
// maximal run of lanes (in lane order) that share b; b = ~0u adds nothing.
// Called by the whole wavefront.
__device__ __forceinline__ void wave_run_add(uint32_t* sums, uint32_t b, uint32_t v) {
    const uint32_t lane = lane_id();
    const uint32_t prev = __shfl_up(b, 1, 64);
    const uint64_t heads = ballot(lane == 0 || b != prev);
    const uint32_t inc = wave_incl_scan(v);
    const int start = 63 - __clzll(heads & ((2ull << lane) - 1ull));  // lane 0 is always a head
    const uint32_t before = __shfl(inc - v, start, 64);
    const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    if (tail && b != ~0u) atomicAdd(&sums[b], inc - before);
}

// Per block of 256 * ITERS entries: the number of pairs and, if vis_sums is
// set, the number of visible entries (tile count > 0).  All tile counts are
// loaded before the first is used (index clamped to the last entry).
template <int ITERS>
__global__ __launch_bounds__(256) void k_scan_reduce(EmitIn E, int64_t n_total, uint32_t* __restrict__ block_sums,
                                                     uint32_t* __restrict__ vis_sums) {
    __shared__ uint32_t lds4[4];
    __shared__ CamPtrs P;
    stage_cam_ptrs(E, P);
    const int64_t base = int64_t(blockIdx.x) * (kScanThreads * ITERS) + threadIdx.x;
    uint32_t c_[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int64_t e = min<int64_t>(base + it * kScanThreads, n_total - 1);
        const int c = int(e / E.n_in);
        c_[it] = P.tiles[c][e - int64_t(c) * E.n_in];
    }
    uint32_t acc = 0, vis = 0;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const uint32_t c = base + it * kScanThreads < n_total ? c_[it] : 0u;
        acc += c;
        vis += c > 0u;
    }
    uint32_t tot;
    block_excl_scan(acc, lds4, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
    if (vis_sums) {
        uint32_t tv;
        block_excl_scan(vis, lds4, &tv);
        if (threadIdx.x == 0) vis_sums[blockIdx.x] = tv;
    }
}

// Exclusive scan in place of nb per-block sums by one workgroup of
// kScanWgThreads threads, kScanPer consecutive sums per thread per round: the
// sums are staged through LDS (coalesced loads and stores; one pad word per
// 32 keeps the per-thread runs free of bank conflicts); returns the total.
constexpr int kScanWgThreads = 1024;
constexpr int kScanPer = 8;
constexpr int kScanRound = kScanWgThreads * kScanPer;
constexpr int kScanStage = kScanRound + kScanRound / 32;

__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

__device__ uint64_t scan_sums_1wg(uint32_t* __restrict__ sums, int64_t nb, uint32_t* lds_w, uint64_t* carry_s,
                                  uint32_t* stage) {
    const int tid = threadIdx.x;
    if (tid == 0) *carry_s = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kScanRound) {
        // unconditional loads (index clamped to the last sum), all issued
        // before the first store to LDS
        uint32_t ld[kScanPer];
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) ld[q] = sums[min<int64_t>(b0 + q * kScanWgThreads + tid, nb - 1)];
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const int idx = q * kScanWgThreads + tid;
            stage[scan_pad(idx)] = (b0 + idx < nb) ? ld[q] : 0u;
        }
        __syncthreads();
        uint32_t v[kScanPer], sum = 0;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            v[q] = stage[scan_pad(tid * kScanPer + q)];
            sum += v[q];
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kScanWgThreads / 64>(sum, lds_w, &tot);
        const uint64_t carry = *carry_s;
        uint64_t run = carry + ex;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            stage[scan_pad(tid * kScanPer + q)] = uint32_t(run);  // totals below 2^32 are checked by the caller
            run += v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const int idx = q * kScanWgThreads + tid;
            if (b0 + idx < nb) sums[b0 + idx] = stage[scan_pad(idx)];
        }
        if (tid == 0) *carry_s = carry + tot;
        __syncthreads();
    }
    return *carry_s;
}

// Counters of the sort (counters[7]: the long tile segments).
constexpr int kCounters = 8;

// One workgroup: exclusive scan of the block sums, total pair count; also
// clears the digit totals of the radix passes and the counters.  With
// vis_sums (depth-first path) it also scans the visible-entry counts and
// writes their total to n_sorted[1] (0 if the pairs do not fit).
__global__ __launch_bounds__(kScanWgThreads) void k_scan_blocks(uint32_t* __restrict__ block_sums, int64_t n_blocks,
                                                     int64_t* __restrict__ n_pairs, int64_t capacity,
                                                     uint32_t* __restrict__ n_sorted, uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ counters,
                                                     uint32_t* __restrict__ vis_sums) {
    __shared__ uint32_t lds4[kScanWgThreads / 64];
    __shared__ uint64_t carry_s;
    __shared__ uint32_t stage[kScanStage];
    for (int k = threadIdx.x; k < 8 * 256; k += kScanWgThreads) hist[k] = 0;
    if (threadIdx.x < kCounters) counters[threadIdx.x] = 0;
    const uint64_t K = scan_sums_1wg(block_sums, n_blocks, lds4, &carry_s, stage);
    const bool fits = int64_t(K) <= capacity;
    uint64_t nv = 0;
    if (vis_sums) nv = scan_sums_1wg(vis_sums, n_blocks, lds4, &carry_s, stage);
    if (threadIdx.x == 0) {
        *n_pairs = int64_t(K);
        n_sorted[0] = fits ? uint32_t(K) : 0u;
        n_sorted[1] = fits ? uint32_t(nv) : 0u;
    }
}

__device__ __forceinline__ int64_t fdiv16(int64_t a) { return a >= 0 ? a / 16 : -((-a + 15) / 16); }

// Integer tile rectangle of a visible entry: first global tile, width in
// tiles, and the camera's tiles per row.
__device__ __forceinline__ void vis_rect_of(uint32_t tile_off, int64_t TX, int64_t TY, float2 q0, int64_t r,
                                            uint32_t* bt, uint32_t* wd, uint32_t* tx) {
    const int64_t xi = int64_t(floorf(fminf(fmaxf(q0.x, -1073741824.f), 1073741824.f)));
    const int64_t yi = int64_t(floorf(fminf(fmaxf(q0.y, -1073741824.f), 1073741824.f)));
    const int64_t x0 = min<int64_t>(max<int64_t>(fdiv16(xi - r), 0), TX);
    const int64_t x1 = min<int64_t>(max<int64_t>(fdiv16(xi + r) + 1, 0), TX);
    const int64_t y0 = min<int64_t>(max<int64_t>(fdiv16(yi - r), 0), TY);
    *bt = tile_off + uint32_t(y0 * TX + x0);
    *wd = uint32_t(max<int64_t>(x1 - x0, 1));
    *tx = uint32_t(TX);
}

// Emission: per 256 entries a block-wide scan of the tile counts gives the
// block a contiguous run of output pairs; all 256 threads then write
// consecutive pairs of that run (each finds its entry by binary search over the
// 256 entry starts in LDS), so the stores are coalesced and the work of large
// Gaussians, or of runs of visible entries, is spread over the whole block.
struct EmitLds {
    uint32_t start[kScanThreads + 1];
    uint32_t base_tile[kScanThreads];
    uint32_t w[kScanThreads];
    uint32_t tx[kScanThreads];
    uint32_t dbits[kScanThreads];
    uint32_t j[kScanThreads];
};

// Writes a block's `tot` pairs from position run on: output o belongs to the
// last entry l with start[l] <= o (zero-count entries share the next start);
// its tile is the (o - start[l])-th of the entry's rectangle in row-major
// order.  Each thread takes kEmitIlp outputs at a time and interleaves their
// binary searches (always 8 steps over the 256 starts): a block whose entries
// cover thousands of tiles (6,150 pairs in one block of the 1M view, against
// 121 on average) runs its rounds a quarter as long.  COMPACT: the layout of
// the tile passes (at most 65,536 tiles), tile id as 16 bits in out16 and
// depth bits << 32 | entry in out64; else keys out64 = tile << 32 | depth
// bits and values out32 = entry.
constexpr int kEmitIlp = 4;

template <bool COMPACT>
__device__ __forceinline__ void emit_block_pairs(const EmitLds& L, uint32_t tot, uint32_t run,
                                                 uint64_t* __restrict__ out64, uint32_t* __restrict__ out32,
                                                 uint16_t* __restrict__ out16) {
    for (uint32_t o0 = threadIdx.x; o0 < tot; o0 += kEmitIlp * kScanThreads) {
        uint32_t lo[kEmitIlp], hi[kEmitIlp];
#pragma unroll
        for (int u = 0; u < kEmitIlp; ++u) {
            lo[u] = 0;
            hi[u] = kScanThreads;
        }
#pragma unroll
        for (int step = 0; step < 8; ++step) {
#pragma unroll
            for (int u = 0; u < kEmitIlp; ++u) {
                const uint32_t mid = (lo[u] + hi[u]) >> 1;
                if (L.start[mid] <= o0 + u * kScanThreads) lo[u] = mid;
                else hi[u] = mid;
            }
        }
#pragma unroll
        for (int u = 0; u < kEmitIlp; ++u) {
            const uint32_t o = o0 + u * kScanThreads;
            if (o >= tot) break;
            const uint32_t l = lo[u];
            const uint32_t local = o - L.start[l];
            const uint32_t ww = L.w[l];
            const uint32_t dy = local / ww, dx = local - dy * ww;
            const uint32_t tile = L.base_tile[l] + dy * L.tx[l] + dx;
            if (COMPACT) {
                out16[run + o] = uint16_t(tile);
                out64[run + o] = (uint64_t(L.dbits[l]) << 32) | uint64_t(L.j[l]);
            } else {
                out64[run + o] = (uint64_t(tile) << 32) | uint64_t(L.dbits[l]);
                out32[run + o] = L.j[l];
            }
        }
    }
}

// Emission in entry order (the per-tile path): per block of 256 entries,
// the block's pairs as one contiguous run; with tile16 set in the compact
// layout of the tile passes (tile16, dv) instead of keys/vals.
__global__ __launch_bounds__(256) void k_emit(EmitIn E, int64_t n_total, const uint32_t* __restrict__ block_offs,
                                              const uint32_t* __restrict__ n_sorted,
                                              uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                              uint16_t* __restrict__ tile16, uint64_t* __restrict__ dv) {
    __shared__ uint32_t lds4[4];
    __shared__ EmitLds L;
    __shared__ CamPtrs P;
    const uint32_t n_s = *n_sorted;
    if (n_s == 0) return;  // nothing fits (or nothing to emit)
    stage_cam_ptrs(E, P);
    const int64_t base = int64_t(blockIdx.x) * kScanItems;
    const uint32_t tid = threadIdx.x;
    const uint32_t run = block_offs[blockIdx.x];
    // every input of the entry loaded at once (index clamped to the last
    // entry), whether it is visible or not
    const int64_t e = min<int64_t>(base + tid, n_total - 1);
    const int c = int(e / E.n_in);
    const int64_t j = e - int64_t(c) * E.n_in;
    uint32_t cnt = P.tiles[c][j];
    float2 q;
    if (E.use_m2d) {
        q = make_float2(P.m2d[c][j], P.m2d[c][E.n_in + j]);
    } else {
        const float GS_GLOBAL* qp = P.rec[c] + j * kRec;
        q = make_float2(qp[0], qp[1]);
    }
    const int32_t rad = P.radius[c][j];
    const uint32_t dbits = __float_as_uint(P.depth[c][j]);
    if (base + tid >= n_total) cnt = 0;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(cnt, lds4, &tot);
    uint32_t bt = 0, wd = 1, tx = 0, db = 0;
    if (cnt > 0) {
        vis_rect_of(P.tile_off[c], P.TX[c], P.TY[c], q, rad, &bt, &wd, &tx);
        db = dbits;
    }
    L.start[tid] = ex;
    L.base_tile[tid] = bt;
    L.w[tid] = wd;
    L.tx[tid] = tx;
    L.dbits[tid] = db;
    L.j[tid] = uint32_t(j);
    if (tid == 0) L.start[kScanThreads] = tot;
    __syncthreads();
    if (tile16) emit_block_pairs<true>(L, tot, run, dv, nullptr, tile16);
    else emit_block_pairs<false>(L, tot, run, keys, vals, nullptr);
}

// ---------------------------------------------------------------------------
// Depth-first binning (long tile lists): the visible entries are compacted
// and sorted by depth once (four 8-bit passes over 32-bit keys), the pairs are
// then emitted in that order, so that stable passes over the tile bits alone
// leave every tile's list in (depth, entry) order - the order of the stable
// sort by the full (tile | depth) key.  Per pair this moves the 12-byte pairs
// through the tile passes only; the depth passes move 8 bytes per visible
// entry.
// ---------------------------------------------------------------------------
// Visible-entry record: entry index within its camera, first global tile of
// the rectangle, rectangle width | camera tiles-per-row << 16, tile count.
// Compaction of the visible entries (ascending entry order): depth bits (the
// depth sort's keys; its first pass takes the rank from the position) and
// the entry's record.  Per block of 256 * ITERS entries: the visible ones are
// listed in LDS in entry order, then read back in list order, so that every
// load of a round is issued before the first is used and the stores are
// consecutive.
template <int ITERS>
__global__ __launch_bounds__(256) void k_vis_compact(EmitIn E, int64_t n_total, const uint32_t* __restrict__ vis_offs,
                                                     const uint32_t* __restrict__ n_sorted,
                                                     uint32_t* __restrict__ dkey, uint4* __restrict__ vrec,
                                                     uint32_t* __restrict__ emit_sums) {
    __shared__ uint32_t lds4[4];
    __shared__ uint32_t list[kScanThreads * ITERS];
    __shared__ uint32_t lcnt[kScanThreads * ITERS];
    __shared__ CamPtrs P;
    const uint32_t n_v = n_sorted[1];
    if (n_v == 0) return;  // nothing visible, or the pairs do not fit
    // the pair counts per 256 depth-sorted entries, which the last depth pass
    // accumulates
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < (n_v + 255) / 256; k += gridDim.x * 256) emit_sums[k] = 0;
    stage_cam_ptrs(E, P);
    const uint32_t tid = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * (kScanThreads * ITERS);
    uint32_t c_[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int64_t e = min<int64_t>(base + it * kScanThreads + tid, n_total - 1);
        const int c = int(e / E.n_in);
        c_[it] = P.tiles[c][e - int64_t(c) * E.n_in];
    }
    uint32_t nv = 0;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const uint32_t off = uint32_t(it * kScanThreads) + tid;
        const bool v = base + off < n_total && c_[it] > 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v ? 1u : 0u, lds4, &tot);
        if (v) {
            list[nv + ex] = off;
            lcnt[nv + ex] = c_[it];
        }
        nv += tot;
    }
    __syncthreads();
    if (nv == 0) return;  // uniform
    const uint32_t o0 = vis_offs[blockIdx.x];
    float2 q_[ITERS];
    int32_t r_[ITERS];
    uint32_t d_[ITERS];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int64_t e = base + list[min(uint32_t(it * kScanThreads) + tid, nv - 1u)];
        const int c = int(e / E.n_in);
        const int64_t j = e - int64_t(c) * E.n_in;
        if (E.use_m2d) {
            q_[it] = make_float2(P.m2d[c][j], P.m2d[c][E.n_in + j]);
        } else {
            const float GS_GLOBAL* q = P.rec[c] + j * kRec;
            q_[it] = make_float2(q[0], q[1]);
        }
        r_[it] = P.radius[c][j];
        d_[it] = __float_as_uint(P.depth[c][j]);
    }
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const uint32_t k = uint32_t(it * kScanThreads) + tid;
        if (k < nv) {
            const int64_t e = base + list[k];
            const int c = int(e / E.n_in);
            const int64_t j = e - int64_t(c) * E.n_in;
            uint32_t bt, wd, tx;
            vis_rect_of(P.tile_off[c], P.TX[c], P.TY[c], q_[it], r_[it], &bt, &wd, &tx);
            dkey[o0 + k] = d_[it];
            vrec[o0 + k] = make_uint4(uint32_t(j), bt, wd | (tx << 16), lcnt[k]);
        }
    }
}

__global__ __launch_bounds__(kScanWgThreads) void k_scan_sums(uint32_t* __restrict__ sums,
                                                              const uint32_t* __restrict__ n_sorted) {
    __shared__ uint32_t lds_w[kScanWgThreads / 64];
    __shared__ uint64_t carry_s;
    __shared__ uint32_t stage[kScanStage];
    const int64_t nb = (int64_t(n_sorted[1]) + 255) / 256;
    scan_sums_1wg(sums, nb, lds_w, &carry_s, stage);
}

// Emission in depth order: per block of 256 depth-sorted visible entries, the
// block's pairs are written as one contiguous run, spread over all threads;
// with tile16 set, in the compact layout (tile16, dv) instead of keys/vals.
__global__ __launch_bounds__(256) void k_emit_sorted(const uint4* __restrict__ srec, const uint32_t* __restrict__ dkey,
                                                     const uint32_t* __restrict__ n_sorted,
                                                     const uint32_t* __restrict__ offs, uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals, uint16_t* __restrict__ tile16,
                                                     uint64_t* __restrict__ dv) {
    __shared__ uint32_t lds4[4];
    __shared__ EmitLds L;
    const uint32_t n_v = n_sorted[1];
    if (n_v == 0) return;
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x * 256u >= n_v) return;  // uniform per block
    const uint32_t i = blockIdx.x * 256 + tid;
    uint4 r = make_uint4(0u, 0u, 1u, 0u);
    uint32_t db = 0;
    if (i < n_v) {
        r = srec[i];
        db = dkey[i];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(r.w, lds4, &tot);
    L.start[tid] = ex;
    L.base_tile[tid] = r.y;
    L.w[tid] = r.z & 0xffffu;
    L.tx[tid] = r.z >> 16;
    L.dbits[tid] = db;
    L.j[tid] = r.x;
    if (tid == 0) L.start[kScanThreads] = tot;
    __syncthreads();
    if (tile16) emit_block_pairs<true>(L, tot, offs[blockIdx.x], dv, nullptr, tile16);
    else emit_block_pairs<false>(L, tot, offs[blockIdx.x], keys, vals, nullptr);
}

// ---------------------------------------------------------------------------
// LSD radix passes, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kWaves = kSortThreads / 64;
// Keys per thread: 15 (3,840-key partitions) for large pair counts, 5 (1,280)
// when the pair buffer is small, so that enough workgroups fill the chip.
constexpr int kIptLarge = 15;
constexpr int kIptSmall = 5;
constexpr int64_t kSmallSortCapacity = 2 << 20;
constexpr int kPartMin = kSortThreads * kIptSmall;

template <int IPT, typename KeyT, typename ValT>
struct SortLds {
    ValT vals[kSortThreads * IPT];
    KeyT keys[kSortThreads * IPT];
    uint32_t wcnt[kWaves][256];
    uint32_t bin_start[256];
    uint32_t gbase[256];
    uint32_t dig_off[256];
    uint32_t scan4[4];
};

// The scatter of a reduce-then-scan pass: ranks every partition stably
// (eight ballots per key), stages it in LDS in (digit, input order) and writes
// it at the scanned offsets.  At least three wavefronts per SIMD, which the
// LDS of the 3,840-key instance allows (three workgroups per compute unit).
// KeyT: uint64_t (full pairs), uint16_t (tile ids of the compact layout, with
// 64-bit values) or uint32_t (depth keys of the depth-first path).
// With gather_src set, the pass writes gather_dst[g] = gather_src[value]
// instead of the value (the last depth pass: the records in depth order).
// Without vals_in the value of the key at position i is i.  With final_keys
// set (the last tile pass of the compact layout: 16-bit tile keys, values
// depth bits << 32 | entry) the pass writes the full pairs instead,
// final_keys[g] = tile << 32 | depth bits and final_vals[g] = entry.  With
// gsums (gather mode) it also adds the gathered records' pair counts (.w) per
// 256 output positions into gsums (cleared beforehand).
template <int IPT, typename KeyT, typename ValT = uint32_t>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_sort_pass(const KeyT* __restrict__ keys_in,
                                                   const ValT* __restrict__ vals_in,
                                                   KeyT* __restrict__ keys_out, ValT* __restrict__ vals_out,
                                                   const uint32_t* __restrict__ n_sorted,
                                                   const uint32_t* __restrict__ hist_pass,
                                                   const uint32_t* __restrict__ offs, uint32_t offs_stride,
                                                   int shift, const uint4* __restrict__ gather_src,
                                                   uint4* __restrict__ gather_dst,
                                                   uint64_t* __restrict__ final_keys,
                                                   uint32_t* __restrict__ final_vals, uint32_t* __restrict__ gsums) {
    constexpr int kSortPerThread = IPT;
    constexpr int kPart = kSortThreads * IPT;
    __shared__ SortLds<IPT, KeyT, ValT> L;
    const uint32_t n = *n_sorted;
    const uint32_t n_parts = (n + kPart - 1) / kPart;
    const int tid = threadIdx.x;
    const int w = tid / 64;
    const uint32_t lane = lane_id();

    // Global exclusive offsets of each digit (scan of this pass's histogram).
    bool trivial;
    {
        const uint32_t v = hist_pass[tid];
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, L.scan4, &tot);
        L.dig_off[tid] = ex;
        trivial = __syncthreads_or(v == n) != 0;
    }
    if (trivial) {
        // every key has the same digit: the stable pass is the identity, so
        // the pass is a copy
        const uint32_t stride = gridDim.x * kSortThreads;
        if (gsums) {
            // a wavefront's 64 positions lie in one block of 256
            for (uint32_t i0 = blockIdx.x * kSortThreads + (uint32_t(tid) & ~63u); i0 < n; i0 += stride) {
                const uint32_t i = i0 + lane;
                uint32_t wv = 0;
                if (i < n) {
                    keys_out[i] = keys_in[i];
                    const uint4 r = gather_src[vals_in ? uint32_t(vals_in[i]) : i];
                    gather_dst[i] = r;
                    wv = r.w;
                }
                wave_run_add(gsums, i < n ? i >> 8 : ~0u, wv);
            }
        }
        for (uint32_t i = blockIdx.x * kSortThreads + tid; i < n && !gsums; i += stride) {
            const KeyT key = keys_in[i];
            const ValT v = vals_in ? vals_in[i] : ValT(i);
            if (final_keys) {
                final_keys[i] = (uint64_t(key) << 32) | (uint64_t(v) >> 32);
                final_vals[i] = uint32_t(v);
                continue;
            }
            keys_out[i] = key;
            if (gather_src) gather_dst[i] = gather_src[v];
            else vals_out[i] = v;
        }
        return;
    }
    // Partitions are independent (their offsets come scanned): taken in
    // grid-stride order.
    for (uint32_t part = blockIdx.x; part < n_parts; part += gridDim.x) {
        for (int k = tid; k < kWaves * 256; k += 256) (&L.wcnt[0][0])[k] = 0;
        __syncthreads();

        // 1. load (wave-striped) and rank within the wavefront, stably
        const uint32_t wbase = part * kPart + uint32_t(w) * (kSortPerThread * 64);
        KeyT k_[kSortPerThread];
        ValT v_[kSortPerThread];
        uint32_t rank_[kSortPerThread];
        // unconditional loads (index clamped to the last key), all issued
        // before the ranking; a guarded load would wait on its own
#pragma unroll
        for (int it = 0; it < kSortPerThread; ++it) {
            const uint32_t idx = min(wbase + uint32_t(it) * 64 + lane, n - 1u);
            k_[it] = keys_in[idx];
            v_[it] = vals_in ? vals_in[idx] : ValT(idx);
        }
#pragma unroll
        for (int it = 0; it < kSortPerThread; ++it) {
            const uint32_t idx = wbase + uint32_t(it) * 64 + lane;
            const bool valid = idx < n;
            if (!valid) k_[it] = ~KeyT(0);
            const uint32_t d = uint32_t(k_[it] >> shift) & 255u;
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t before = popc64(peers & lanemask_lt());
            const uint32_t base = L.wcnt[w][d];
            rank_[it] = base + before;
            // the lowest lane of each group bumps the wavefront's bin count
            if (valid && before == 0) L.wcnt[w][d] = base + popc64(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        // 2. per-bin totals, wavefront offsets, and the partition's bin starts
        uint32_t total = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            const uint32_t c = L.wcnt[ww][tid];
            L.wcnt[ww][tid] = total;
            total += c;
        }
        {
            uint32_t tot;
            const uint32_t ex = block_excl_scan(total, L.scan4, &tot);
            L.bin_start[tid] = ex;
        }

        // 3. this partition's first output position per bin: the digit's
        // global offset plus the scanned counts of the earlier partitions
        L.gbase[tid] = L.dig_off[tid] + offs[size_t(tid) * offs_stride + part] - L.bin_start[tid];
        __syncthreads();

        // 4. stage in LDS in (digit, input order) order
#pragma unroll
        for (int it = 0; it < kSortPerThread; ++it) {
            const uint32_t idx = wbase + uint32_t(it) * 64 + lane;
            if (idx < n) {
                const uint32_t d = uint32_t(k_[it] >> shift) & 255u;
                const uint32_t lp = L.bin_start[d] + L.wcnt[w][d] + rank_[it];
                L.keys[lp] = k_[it];
                L.vals[lp] = v_[it];
            }
        }
        __syncthreads();

        // 5. coalesced write-out
        const uint32_t cnt = min<uint32_t>(kPart, n - part * kPart);
        if (gsums) {
            // the records in depth order and the pair count of every block of
            // 256 output positions (every wavefront runs all rounds)
            for (uint32_t i0 = 0; i0 < uint32_t(kPart); i0 += 256) {
                const uint32_t i = i0 + tid;
                uint32_t b = ~0u, wv = 0;
                if (i < cnt) {
                    const KeyT key = L.keys[i];
                    const uint32_t g = L.gbase[uint32_t(key >> shift) & 255u] + i;
                    keys_out[g] = key;
                    const uint4 r = gather_src[uint32_t(L.vals[i])];
                    gather_dst[g] = r;
                    b = g >> 8;
                    wv = r.w;
                }
                wave_run_add(gsums, b, wv);
            }
        }
        for (uint32_t i = tid; i < cnt && !gsums; i += 256) {
            const KeyT key = L.keys[i];
            const uint32_t d = uint32_t(key >> shift) & 255u;
            const uint32_t g = L.gbase[d] + i;
            if (final_keys) {
                final_keys[g] = (uint64_t(key) << 32) | (uint64_t(L.vals[i]) >> 32);
                final_vals[g] = uint32_t(L.vals[i]);
                continue;
            }
            keys_out[g] = key;
            if (gather_src) gather_dst[g] = gather_src[L.vals[i]];
            else vals_out[g] = L.vals[i];
        }
        __syncthreads();
    }
}

// A radix pass in reduce-then-scan form: the digit counts of every partition,
// then one scan per digit over the partitions, then k_sort_pass ranks and
// scatters each partition independently.  No partition waits for another: a
// decoupled look-back serialises on a chain of round trips between the
// partitions resident at the same time, up to a thousand on this chip.
// counts is digit-major: counts[d * stride + partition] (the scan reads a
// digit's counts contiguously; a partition-major table made it 2.4x slower).
template <int IPT, typename KeyT>
__global__ __launch_bounds__(256) void k_part_count(const KeyT* __restrict__ keys,
                                                    const uint32_t* __restrict__ n_sorted, int shift,
                                                    uint32_t* __restrict__ counts, uint32_t stride, int wave_agg) {
    constexpr int kPart = kSortThreads * IPT;
    __shared__ uint32_t h[256];
    const uint32_t n = *n_sorted;
    const uint32_t n_parts = (n + kPart - 1) / kPart;
    const int tid = threadIdx.x;
    for (uint32_t part = blockIdx.x; part < n_parts; part += gridDim.x) {
        h[tid] = 0;
        __syncthreads();
        const uint32_t wbase = part * kPart + uint32_t(tid / 64) * (IPT * 64);
        // unconditional loads (index clamped to the last key), all issued
        // before the first use; a guarded load would wait on its own
        KeyT k_[IPT];
#pragma unroll
        for (int it = 0; it < IPT; ++it)
            k_[it] = keys[min(wbase + uint32_t(it) * 64 + lane_id(), n - 1u)];
        uint32_t d_[IPT];
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const uint32_t idx = wbase + uint32_t(it) * 64 + lane_id();
            d_[it] = idx < n ? uint32_t(k_[it] >> shift) & 255u : 256u;
        }
        if (!wave_agg) {
            // spread digits: one LDS atomic per key
#pragma unroll
            for (int it = 0; it < IPT; ++it)
                if (d_[it] < 256u) atomicAdd(&h[d_[it]], 1u);
        } else {
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            // few distinct digits (a key's top digit), where lanes would
            // collide on the same counters: lanes with equal digits found by
            // eight ballots, the lowest adds for all of them
            const uint32_t d = d_[it];
            const bool valid = d < 256u;
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = ballot(bit);
                peers &= bit ? m : ~m;
            }
            if (valid && (peers & lanemask_lt()) == 0ull) atomicAdd(&h[d], popc64(peers));
        }
        }
        __syncthreads();
        counts[size_t(tid) * stride + part] = h[tid];
        __syncthreads();
    }
}

// One workgroup per digit: exclusive scan in place of the digit's partition
// counts (a row of the table); total[d] = the digit's count over the pass.
__global__ __launch_bounds__(kScanWgThreads) void k_part_scan(uint32_t* __restrict__ counts, uint32_t stride,
                                                             const uint32_t* __restrict__ n_sorted, int part,
                                                             uint32_t* __restrict__ total) {
    __shared__ uint32_t lds_w[kScanWgThreads / 64];
    __shared__ uint64_t carry_s;
    __shared__ uint32_t stage[kScanStage];
    const int64_t np = (int64_t(*n_sorted) + part - 1) / part;
    const uint64_t t = scan_sums_1wg(counts + size_t(blockIdx.x) * stride, np, lds_w, &carry_s, stage);
    if (threadIdx.x == 0) total[blockIdx.x] = uint32_t(t);
}

// Tile ranges from the sorted keys: boundary b (0 <= b <= n_tiles) is the
// first position whose tile id is >= b, found by binary search; tile t spans
// [boundary t, boundary t+1).  Empty tiles get start == end, and when nothing
// was sorted every range is empty.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_sorted, uint32_t n_tiles,
                                                     uint32_t* __restrict__ ranges) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b > n_tiles) return;
    const uint32_t n = *n_sorted;
    uint32_t lo = 0, hi = n;  // first index with tile >= b
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (uint32_t(keys[mid] >> 32) < b) lo = mid + 1;
        else hi = mid;
    }
    if (b < n_tiles) ranges[b] = lo;
    if (b > 0) ranges[n_tiles + b - 1] = lo;
}

// ---------------------------------------------------------------------------
// Depth order inside each tile
// ---------------------------------------------------------------------------
// After the radix passes over the tile bits, every tile's pairs are contiguous
// and in emission order (ascending entry index).  One wavefront per tile then
// orders its segment by depth, ties by position (= by index): a bitonic
// network over the composite keys (depth bits << 32 | position) in LDS for
// segments of up to kSegMax pairs, else a stable 8-bit LSD radix sort of the
// depth bits through global memory (ping-pong between the two pair buffers).
constexpr int kSegWaves = 2;
constexpr int64_t kSegAvgMax = 256;  // pair capacity per tile up to which the per-tile sort is used
constexpr int kSegMax = 2048;

__device__ __forceinline__ void seg_bitonic(uint64_t* S, uint32_t n, uint32_t lane) {
    uint32_t N = 2;
    while (N < n) N <<= 1;
    for (uint32_t i = n + lane; i < N; i += 64) S[i] = ~0ull;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = lane; t < N / 2; t += 64) {
                const uint32_t i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));
                const uint32_t j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = S[i], b = S[j];
                if ((a > b) == asc) {
                    S[i] = b;
                    S[j] = a;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Stable LSD radix sort of a long segment by its 32 depth bits, one wavefront:
// per 8-bit digit a histogram, a scan, and a scatter of 64-pair chunks in
// order with ranks from eight ballots.  Four passes (a->b->a->b->a), then a
// copy a -> b, so the result ends in b.
__device__ void seg_lsd_global(uint64_t* ka, uint32_t* va, uint64_t* kb, uint32_t* vb, uint32_t n, uint32_t* hist,
                               uint32_t lane) {
    for (int pass = 0; pass < 4; ++pass) {
        uint64_t* ks = (pass & 1) ? kb : ka;
        uint32_t* vs = (pass & 1) ? vb : va;
        uint64_t* kd = (pass & 1) ? ka : kb;
        uint32_t* vd = (pass & 1) ? va : vb;
        const int shift = 8 * pass;
        for (int b = lane; b < 256; b += 64) hist[b] = 0;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < n; i += 64) atomicAdd(&hist[uint32_t(ks[i] >> shift) & 255u], 1u);
        __builtin_amdgcn_wave_barrier();
        {   // exclusive scan of the 256 bins, four per lane
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) { c[q] = hist[lane * 4 + q]; sum += c[q]; }
            uint32_t inc = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o, 64);
                if (lane >= uint32_t(o)) inc += t;
            }
            uint32_t run = inc - sum;
#pragma unroll
            for (int q = 0; q < 4; ++q) { hist[lane * 4 + q] = run; run += c[q]; }
        }
        __builtin_amdgcn_wave_barrier();
        for (uint32_t c0 = 0; c0 < n; c0 += 64) {
            const uint32_t i = c0 + lane;
            const bool valid = i < n;
            const uint64_t key = valid ? ks[i] : 0ull;
            const uint32_t val = valid ? vs[i] : 0u;
            const uint32_t d = uint32_t(key >> shift) & 255u;
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool on = (d >> bit) & 1u;
                const uint64_t m = ballot(on);
                peers &= on ? m : ~m;
            }
            const uint32_t before = popc64(peers & lanemask_lt());
            const uint32_t base = hist[d];
            if (valid) {
                kd[base + before] = key;
                vd[base + before] = val;
            }
            __builtin_amdgcn_wave_barrier();
            if (valid && before == 0) hist[d] = base + popc64(peers);
            __builtin_amdgcn_wave_barrier();
        }
    }
    for (uint32_t i = lane; i < n; i += 64) {
        kb[i] = ka[i];
        vb[i] = va[i];
    }
}

// keys_in / vals_in are not const: a long segment uses its input range as
// scratch (nothing else reads it afterwards).
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    const uint32_t lo = uint32_t(__shfl_xor(int(uint32_t(v)), mask, 64));
    const uint32_t hi = uint32_t(__shfl_xor(int(uint32_t(v >> 32)), mask, 64));
    return (uint64_t(hi) << 32) | lo;
}

// Bitonic network over 64*E keys held in registers, element r*64 + lane in
// k[r]: strides below 64 exchange across lanes, larger ones between registers.
template <int E>
__device__ __forceinline__ void reg_bitonic(uint64_t (&k)[E], uint32_t lane) {
    constexpr uint32_t N = 64u * E;
#pragma unroll
    for (uint32_t size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= 64) {
                const uint32_t rs = stride >> 6;
#pragma unroll
                for (uint32_t r = 0; r < uint32_t(E); ++r) {
                    if (r & rs) continue;
                    const uint32_t r2 = r | rs;
                    const bool asc = ((r << 6) & size) == 0;
                    const uint64_t a = k[r], b = k[r2];
                    const bool sw = (a > b) == asc;
                    k[r] = sw ? b : a;
                    k[r2] = sw ? a : b;
                }
            } else {
#pragma unroll
                for (uint32_t r = 0; r < uint32_t(E); ++r) {
                    const uint64_t o = shfl_xor_u64(k[r], int(stride));
                    const bool asc = (((r << 6) | lane) & size) == 0;
                    const bool lower = (lane & stride) == 0;
                    const bool less = k[r] < o;
                    // the lower element keeps the minimum when ascending
                    k[r] = ((lower == asc) == less) ? k[r] : o;
                }
            }
        }
    }
}

template <int E>
__device__ __forceinline__ void seg_sort_regs(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* keys_out,
                                              uint32_t* vals_out, uint32_t start, uint32_t n, uint32_t lane) {
    // loads unconditional (index clamped to the segment's last pair), all
    // issued before the first use; stores guarded
    uint32_t lo[E];
#pragma unroll
    for (int r = 0; r < E; ++r) lo[r] = uint32_t(keys_in[start + min(uint32_t(r) * 64 + lane, n - 1)]);
    uint64_t k[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = uint32_t(r) * 64 + lane;
        k[r] = i < n ? (uint64_t(lo[r]) << 32) | i : ~0ull;
    }
    reg_bitonic<E>(k, lane);
    uint64_t ko[E];
    uint32_t vo[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t p = min(uint32_t(k[r]), n - 1);
        ko[r] = keys_in[start + p];
        vo[r] = vals_in[start + p];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = uint32_t(r) * 64 + lane;
        if (i < n) {
            keys_out[start + i] = ko[r];
            vals_out[start + i] = vo[r];
        }
    }
}

// Pass A: one wavefront per tile; segments of up to kSegRegs pairs are sorted
// in registers, longer ones are listed for pass B.
constexpr uint32_t kSegRegs = 512;

__global__ __launch_bounds__(256) void k_seg_sort(const uint64_t* __restrict__ keys_in,
                                                  const uint32_t* __restrict__ vals_in,
                                                  uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                  const uint32_t* __restrict__ ranges, uint32_t n_tiles,
                                                  const uint32_t* __restrict__ n_sorted, uint32_t* __restrict__ long_list,
                                                  uint32_t* __restrict__ long_count) {
    const uint32_t n_s = *n_sorted;
    if (n_s == 0) return;
    const uint32_t lane = lane_id();
    const uint32_t tile = blockIdx.x * 4 + threadIdx.x / 64;
    if (tile >= n_tiles) return;
    const uint32_t start = ranges[tile], end = ranges[n_tiles + tile];
    if (end <= start || end > n_s) return;  // empty (or ranges of a failed sort)
    const uint32_t n = end - start;
    if (n <= 64) seg_sort_regs<1>(keys_in, vals_in, keys_out, vals_out, start, n, lane);
    else if (n <= 128) seg_sort_regs<2>(keys_in, vals_in, keys_out, vals_out, start, n, lane);
    else if (n <= 256) seg_sort_regs<4>(keys_in, vals_in, keys_out, vals_out, start, n, lane);
    else if (n <= kSegRegs) seg_sort_regs<8>(keys_in, vals_in, keys_out, vals_out, start, n, lane);
    else if (lane == 0) long_list[atomicAdd(long_count, 1u)] = tile;
}

// Pass B: the listed long segments, one wavefront each (LDS bitonic up to
// kSegMax pairs, else the global radix sort).  keys_in / vals_in are not
// const: a segment beyond kSegMax uses its input range as scratch.
__global__ __launch_bounds__(64 * kSegWaves) void k_seg_sort_long(uint64_t* keys_in, uint32_t* vals_in,
                                                                  uint64_t* keys_out, uint32_t* vals_out,
                                                                  const uint32_t* __restrict__ ranges,
                                                                  uint32_t n_tiles,
                                                                  const uint32_t* __restrict__ long_list,
                                                                  const uint32_t* __restrict__ long_count) {
    __shared__ uint64_t S[kSegWaves][kSegMax];
    __shared__ uint32_t H[kSegWaves][256];
    const uint32_t w = threadIdx.x / 64, lane = lane_id();
    const uint32_t cnt = *long_count;
    for (uint32_t q = blockIdx.x * kSegWaves + w; q < cnt; q += gridDim.x * kSegWaves) {
        const uint32_t tile = long_list[q];
        const uint32_t start = ranges[tile], n = ranges[n_tiles + tile] - start;
        if (n > uint32_t(kSegMax)) {
            seg_lsd_global(keys_in + start, vals_in + start, keys_out + start, vals_out + start, n, H[w], lane);
            continue;
        }
        uint64_t* Sw = S[w];
        for (uint32_t i = lane; i < n; i += 64) Sw[i] = (uint64_t(uint32_t(keys_in[start + i])) << 32) | i;
        seg_bitonic(Sw, n, lane);
        for (uint32_t i = lane; i < n; i += 64) {
            const uint32_t p = uint32_t(Sw[i]);
            keys_out[start + i] = keys_in[start + p];
            vals_out[start + i] = vals_in[start + p];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

struct SortWs {
    uint32_t* block_sums;
    uint32_t* vis_sums;   // depth-first path only
    uint32_t* emit_sums;  // depth-first path only
    uint4* vrec;          // depth-first path only: records in entry order
    uint4* srec;          // depth-first path only: records in depth order
    uint32_t* n_sorted;
    uint32_t* hist;      // digit totals of the radix passes (256 per pass)
    uint32_t* counters;
    uint32_t* counts;    // partition counts of a radix pass, 256 rows of np
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* long_list;
    size_t bytes;
};

// Short tile lists (pair capacity per tile up to kSegAvgMax): radix passes
// over the tile bits, then a per-tile depth sort.  Longer lists: the
// depth-first path.
static bool per_tile_path(int64_t capacity, int64_t n_tiles) {
    return capacity <= kSegAvgMax * std::max<int64_t>(n_tiles, 1);
}

static SortWs carve_sort(void* ws, int64_t n_total, int64_t capacity, int64_t n_tiles) {
    Carve cv(ws);
    SortWs s;
    const int64_t nb = (n_total + kScanItems - 1) / kScanItems + 1;
    const int64_t np = (capacity + kPartMin - 1) / kPartMin + 1;
    const bool depth_first = !per_tile_path(capacity, n_tiles);
    s.block_sums = cv.take<uint32_t>(size_t(nb));
    s.vis_sums = depth_first ? cv.take<uint32_t>(size_t(nb)) : nullptr;
    s.emit_sums = depth_first ? cv.take<uint32_t>(size_t(nb)) : nullptr;
    s.vrec = depth_first ? cv.take<uint4>(size_t(n_total > 0 ? n_total : 1)) : nullptr;
    s.srec = depth_first ? cv.take<uint4>(size_t(n_total > 0 ? n_total : 1)) : nullptr;
    s.n_sorted = cv.take<uint32_t>(4);
    s.hist = cv.take<uint32_t>(8 * 256);
    s.counters = cv.take<uint32_t>(kCounters);
    s.counts = cv.take<uint32_t>(size_t(np) * 256);
    s.keys_alt = cv.take<uint64_t>(size_t(capacity > 0 ? capacity : 1));
    s.vals_alt = cv.take<uint32_t>(size_t(capacity > 0 ? capacity : 1));
    s.long_list = cv.take<uint32_t>(size_t(n_tiles > 0 ? n_tiles : 1));
    s.bytes = cv.used();
    return s;
}

// ---------------------------------------------------------------------------
// LOD labels by multi-resolution voxelisation (Sec. 3.3): cubes of edge
// delta0 / 2^l, one representative per occupied cube - its first point in
// (Z-order code of the finest cell, index).  One stable radix sort of the
// 63-bit Z-order codes puts every cube's points in one run at every level
// (the level-l cube of a point is its code shifted right by 3 (K-1-l)), so
// a point's label follows from its predecessor alone: the highest bit in
// which the two codes differ names the coarsest level at which a new cube
// starts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Finest cell coordinate of one axis: floor((m - o) * s) in float32 (a
// subtraction and a product, each rounded once), NaN -> 0, clamped to
// [0, 2^21 - 1].
__device__ __forceinline__ uint32_t fine_cell(float m, float o, float sc) {
    const float d = __fsub_rn(m, o);
    const float q = floorf(__fmul_rn(d, sc));
    if (q != q) return 0u;
    return uint32_t(fminf(fmaxf(q, 0.f), 2097151.f));
}

__global__ void k_voxel_init(uint32_t* __restrict__ n_sorted, uint32_t n) {
    if (threadIdx.x == 0) {
        n_sorted[0] = n;
        n_sorted[1] = 0;
    }
}

__global__ __launch_bounds__(256) void k_voxel_codes(const float* __restrict__ mean, int64_t n, float o0, float o1,
                                                     float o2, float sc, uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t cx = fine_cell(mean[i], o0, sc);
    const uint32_t cy = fine_cell(mean[n + i], o1, sc);
    const uint32_t cz = fine_cell(mean[2 * n + i], o2, sc);
    keys[i] = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
    vals[i] = uint32_t(i);
}

// Label of the point at sorted position p from its predecessor's code.
__global__ __launch_bounds__(256) void k_voxel_label(const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ vals, int64_t n, int n_levels,
                                                     uint8_t* __restrict__ lod) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= n) return;
    int label = 0;
    if (p > 0) {
        const uint64_t x = keys[p] ^ keys[p - 1];
        if (x == 0) {
            label = n_levels - 1;
        } else {
            const int h = 63 - __clzll((long long)x);
            label = max(0, n_levels - 1 - h / 3);
        }
    }
    lod[vals[p]] = uint8_t(label);
}

struct VoxWs {
    uint64_t* keys[2];
    uint32_t* vals[2];
    uint32_t* counts;  // partition counts of a radix pass, 256 rows of np
    uint32_t* hist;    // digit totals of the eight passes
    uint32_t* n_sorted;
    uint32_t np;
    size_t bytes;
};

static VoxWs carve_vox(void* ws, int64_t n) {
    Carve cv(ws);
    VoxWs s;
    const size_t m = size_t(n > 0 ? n : 1);
    const int64_t np = (n + kPartMin - 1) / kPartMin + 1;
    for (int b = 0; b < 2; ++b) {
        s.keys[b] = cv.take<uint64_t>(m);
        s.vals[b] = cv.take<uint32_t>(m);
    }
    s.counts = cv.take<uint32_t>(size_t(np) * 256);
    s.hist = cv.take<uint32_t>(8 * 256);
    s.n_sorted = cv.take<uint32_t>(4);
    s.np = uint32_t(np);
    s.bytes = cv.used();
    return s;
}

// Workgroups of a reduce-then-scan pass (larger inputs loop over partitions).
constexpr int64_t kRtsGrid = 2048;

// One reduce-then-scan radix pass over the n = *n_sorted keys in kin/vin
// (few: a digit with few distinct values, counted with wave aggregation):
// partition counts into counts (digit-major, rows of `stride` >= max_parts
// partitions), their scan (digit totals into total), then the ranking scatter.
template <int IPT, typename KeyT, typename ValT = uint32_t>
static void rts_pass(const KeyT* kin, const ValT* vin, KeyT* kout, ValT* vout, const uint32_t* n_sorted, int shift,
                     bool few, uint32_t* counts, uint32_t stride, uint32_t* total, int64_t max_parts,
                     const uint4* gsrc, uint4* gdst, uint64_t* final_keys, uint32_t* final_vals,
                     uint32_t* gsums, hipStream_t stream) {
    const int grid = int(std::max<int64_t>(1, std::min<int64_t>(max_parts, kRtsGrid)));
    launch("part_count", k_part_count<IPT, KeyT>, dim3(grid), dim3(256), 0, stream, kin, n_sorted, shift, counts,
           stride, int(few));
    hipLaunchKernelGGL(k_part_scan, dim3(256), dim3(kScanWgThreads), 0, stream, counts, stride, n_sorted,
                       int(kSortThreads * IPT), total);
    launch("sort_pass", k_sort_pass<IPT, KeyT, ValT>, dim3(grid), dim3(kSortThreads), 0, stream, kin, vin, kout, vout,
           n_sorted, static_cast<const uint32_t*>(total), static_cast<const uint32_t*>(counts), stride, shift, gsrc,
           gdst, final_keys, final_vals, gsums);
}

}  // namespace gsmi

using namespace gsmi;

size_t ws_bin_sort(int64_t n_total, int64_t capacity, int64_t n_tiles) {
    return carve_sort(nullptr, n_total, capacity, n_tiles).bytes;
}

size_t ws_voxel_levels(int64_t n) { return carve_vox(nullptr, n).bytes; }

extern "C" int gs_voxel_levels(const float* mean, int64_t n, const float* origin, float delta0, int32_t n_levels,
                               uint8_t* lod, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_voxel_levels: need 0 <= n < 2^31");
    if (n_levels < 1 || n_levels > 22) return fail(GS_ERR_INVALID_ARG, "gs_voxel_levels: n_levels in [1, 22]");
    if (!origin || !std::isfinite(origin[0]) || !std::isfinite(origin[1]) || !std::isfinite(origin[2]))
        return fail(GS_ERR_INVALID_ARG, "gs_voxel_levels: origin must be three finite floats");
    if (!(delta0 > 0.f) || !std::isfinite(delta0))
        return fail(GS_ERR_INVALID_ARG, "gs_voxel_levels: delta0 must be positive and finite");
    if (n > 0 && (!mean || !lod)) return fail(GS_ERR_INVALID_ARG, "gs_voxel_levels: null mean or lod");
    VoxWs V = carve_vox(ws, n);
    if (!ws || ws_bytes < V.bytes || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_voxel_levels: workspace needs %zu bytes (256-aligned)", V.bytes);
    if (n == 0) return GS_OK;
    // cell scale 2^(K-1) / delta0, one float32 division (correctly rounded)
    const float sc = float(1u << (n_levels - 1)) / delta0;
    const bool small = n <= kSmallSortCapacity;
    const int part = kSortThreads * (small ? kIptSmall : kIptLarge);
    const int64_t parts = (n + part - 1) / part;
    hipLaunchKernelGGL(k_voxel_init, dim3(1), dim3(64), 0, stream, V.n_sorted, uint32_t(n));
    launch("voxel_codes", k_voxel_codes, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, mean, n, origin[0],
           origin[1], origin[2], sc, V.keys[0], V.vals[0]);
    // eight passes over the 64-bit codes (their digits may take few values:
    // wave-aggregated counting), ending in buffer 0
    for (int p = 0; p < 8; ++p) {
        const int a = p & 1, b = a ^ 1;
        if (small)
            rts_pass<kIptSmall, uint64_t>(V.keys[a], V.vals[a], V.keys[b], V.vals[b], V.n_sorted, 8 * p, true,
                                          V.counts, V.np, V.hist + p * 256, parts, nullptr, nullptr, nullptr, nullptr,
                                          nullptr, stream);
        else
            rts_pass<kIptLarge, uint64_t>(V.keys[a], V.vals[a], V.keys[b], V.vals[b], V.n_sorted, 8 * p, true,
                                          V.counts, V.np, V.hist + p * 256, parts, nullptr, nullptr, nullptr, nullptr,
                                          nullptr, stream);
    }
    launch("voxel_label", k_voxel_label, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream,
           static_cast<const uint64_t*>(V.keys[0]), static_cast<const uint32_t*>(V.vals[0]), n, int(n_levels), lod);
    return check_launch("gs_voxel_levels");
}

extern "C" int gs_bin_sort(const gs_projected* proj, const gs_camera* cams, int n_cams, int64_t n_in,
                           uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* tile_ranges,
                           int64_t* n_pairs_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
    int64_t total_tiles = 0;
    int rc = validate_cams(cams, n_cams, GS_MAX_CAMS, &total_tiles);
    if (rc) return rc;
    if (!proj || n_in < 0 || n_in >= (int64_t(1) << 31))
        return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: bad projection or n_in");
    if (capacity < 0 || capacity >= GS_MAX_PAIRS)
        return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: capacity must be in [0, 2^30)");
    if (!tile_ranges || !n_pairs_dev || (capacity > 0 && (!keys || !vals)))
        return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: null output");
    const int64_t n_total = n_in * n_cams;
    if (n_total >= (int64_t(1) << 32)) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: too many entries");
    SortWs S = carve_sort(ws, n_total, capacity, total_tiles);
    if (!ws || ws_bytes < S.bytes || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_bin_sort: workspace needs %zu bytes (256-aligned)", S.bytes);
    EmitIn E;
    memset(&E, 0, sizeof(E));
    uint32_t off = 0;
    for (int c = 0; c < n_cams; ++c) {
        const gs_projected& p = proj[c];
        if (n_in > 0 && (!p.rec || !p.depth || !p.radius || !p.tiles_touched))
            return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: camera %d: null projection array", c);
        E.rec[c] = p.rec; E.depth[c] = p.depth; E.radius[c] = p.radius; E.tiles[c] = p.tiles_touched;
        E.m2d[c] = p.mean2d;
        E.tile_off[c] = off;
        E.TX[c] = int32_t(tiles_x(cams[c].width));
        E.TY[c] = int32_t(tiles_y(cams[c].height));
        off += uint32_t(gs_num_tiles(cams[c].width, cams[c].height));
    }
    E.n_cams = n_cams;
    E.n_in = n_in > 0 ? n_in : 1;
    // the rectangles read the screen centre from the component-major copy
    // when every camera has one (8 bytes per entry instead of a line of the
    // 48-byte records)
    E.use_m2d = 1;
    for (int c = 0; c < n_cams; ++c) E.use_m2d &= proj[c].mean2d != nullptr;

    // Two orderings with the same result (the stable sort by the full key).
    // Short tile lists: radix passes over the global tile id only (bits 32
    // and up), the depth order inside each tile from the per-tile sort.  Long
    // lists: the depth-first path (visible entries sorted by depth, pairs
    // emitted in that order, then the tile passes).
    int tile_bits = 0;
    while ((int64_t(1) << tile_bits) < total_tiles) ++tile_bits;
    const bool per_tile = per_tile_path(capacity, total_tiles);
    const int tile_passes = (tile_bits + 7) / 8;
    if (tile_passes > 4) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: too many tiles");

    // Entry blocks of 256 * scan_it entries: larger blocks for long inputs
    // (fewer, fuller workgroups and a one-round scan of the block sums).
    const int scan_it = (!per_tile && n_total >= (int64_t(1) << 21)) ? kScanItLong : 1;
    const int64_t nb = (n_total + kScanItems * scan_it - 1) / (kScanItems * scan_it);
    const int64_t nb256 = (n_total + kScanItems - 1) / kScanItems;
    if (nb > 0) {
        if (scan_it == 1)
            launch("scan_reduce", k_scan_reduce<1>, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, E, n_total,
                   S.block_sums, per_tile ? nullptr : S.vis_sums);
        else
            launch("scan_reduce", k_scan_reduce<kScanItLong>, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, E,
                   n_total, S.block_sums, S.vis_sums);
    }
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanWgThreads), 0, stream, S.block_sums, nb, n_pairs_dev, capacity,
                       S.n_sorted, S.hist, S.counters, per_tile ? nullptr : S.vis_sums);
    if ((rc = check_launch("gs_bin_sort scan"))) return rc;
    if (capacity == 0) {
        rc = fill_u32(tile_ranges, 0u, size_t(2 * total_tiles), stream);
        return rc;
    }
    uint64_t* kb[2] = {keys, S.keys_alt};
    uint32_t* vb[2] = {vals, S.vals_alt};
    const bool small = capacity <= kSmallSortCapacity;
    const int part = kSortThreads * (small ? kIptSmall : kIptLarge);
    const int64_t max_parts = (capacity + part - 1) / part;
    // Reduce-then-scan passes over the tile bits, from buffer `cur`; returns
    // the buffer that holds the result.  The partition counts live in the
    // counts array (rows of `stride` partitions, enough for any pass:
    // visible entries and pairs are both at most the capacity).  Compact
    // layout (tile ids fit 16 bits): 16-bit tile keys in the value arrays,
    // depth << 32 | entry in the key arrays; the last pass writes the full
    // pairs.
    const uint32_t stride = uint32_t((capacity + kPartMin - 1) / kPartMin + 1);
    uint32_t* counts = S.counts;
    const bool compact = tile_passes >= 1 && tile_bits <= 16;
    auto tile_passes_rts = [&](int cur) {
        for (int q = 0; q < tile_passes; ++q) {
            const bool last = q + 1 == tile_passes;
            // wave-aggregated counting for the top digit, whose few values
            // make lanes collide on the same counters (per-lane atomics: 33
            // -> 38 us for the 32 values of the 8M orbit view)
            const bool few = last;
            uint32_t* hist = S.hist + (4 + q) * 256;
            if (compact) {
                // 16-bit tile keys in the value arrays, depth << 32 | entry
                // in the key arrays; the last pass writes the full pairs
                const uint16_t* tin = reinterpret_cast<const uint16_t*>(vb[cur]);
                uint16_t* tout = last ? nullptr : reinterpret_cast<uint16_t*>(vb[cur ^ 1]);
                uint64_t* dvout = last ? nullptr : kb[cur ^ 1];
                uint64_t* fk = last ? kb[cur ^ 1] : nullptr;
                uint32_t* fv = last ? vb[cur ^ 1] : nullptr;
                if (small)
                    rts_pass<kIptSmall, uint16_t, uint64_t>(tin, kb[cur], tout, dvout, S.n_sorted, 8 * q, few,
                                                            counts, stride, hist, max_parts, nullptr, nullptr,
                                                            fk, fv, nullptr, stream);
                else
                    rts_pass<kIptLarge, uint16_t, uint64_t>(tin, kb[cur], tout, dvout, S.n_sorted, 8 * q, few,
                                                            counts, stride, hist, max_parts, nullptr, nullptr,
                                                            fk, fv, nullptr, stream);
            } else if (small) {
                rts_pass<kIptSmall, uint64_t>(kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], S.n_sorted, 32 + 8 * q,
                                              few, counts, stride, hist, max_parts, nullptr, nullptr,
                                              nullptr, nullptr, nullptr, stream);
            } else {
                rts_pass<kIptLarge, uint64_t>(kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], S.n_sorted, 32 + 8 * q,
                                              few, counts, stride, hist, max_parts, nullptr, nullptr,
                                              nullptr, nullptr, nullptr, stream);
            }
            cur ^= 1;
        }
        return cur;
    };

    if (!per_tile) {
        // Depth-first path.  The emission writes into buffer z and the tile
        // passes ping-pong from there, ending in the caller's keys/vals; the
        // depth sort runs in the other buffer x (its 32-bit keys in the
        // first half of the key array), ending where it started.  Every pass
        // takes the reduce-then-scan form.
        const int z = tile_passes & 1, x = z ^ 1;
        uint32_t* dk[2] = {reinterpret_cast<uint32_t*>(kb[x]), reinterpret_cast<uint32_t*>(kb[z])};
        uint32_t* dv[2] = {vb[x], vb[z]};
        const bool small_d = n_total <= kSmallSortCapacity;
        const int part_d = kSortThreads * (small_d ? kIptSmall : kIptLarge);
        const int64_t parts_d = (std::min(n_total, capacity) + part_d - 1) / part_d;
        if (nb > 0) {
            if (scan_it == 1)
                launch("vis_compact", k_vis_compact<1>, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, E,
                       n_total, static_cast<const uint32_t*>(S.vis_sums), static_cast<const uint32_t*>(S.n_sorted),
                       dk[0], S.vrec, S.emit_sums);
            else
                launch("vis_compact", k_vis_compact<kScanItLong>, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream,
                       E, n_total, static_cast<const uint32_t*>(S.vis_sums),
                       static_cast<const uint32_t*>(S.n_sorted), dk[0], S.vrec, S.emit_sums);
        }
        for (int p = 0; p < 4; ++p) {
            const int a = p & 1, b = a ^ 1;
            // the last pass writes the records in depth order instead of the ranks
            const uint4* gsrc = p == 3 ? static_cast<const uint4*>(S.vrec) : nullptr;
            uint4* gdst = p == 3 ? S.srec : nullptr;
            // the first pass ranks by position (the compaction stores no values)
            const uint32_t* vin = p == 0 ? nullptr : dv[a];
            if (small_d)
                rts_pass<kIptSmall, uint32_t>(dk[a], vin, dk[b], dv[b], S.n_sorted + 1, 8 * p, p == 3, counts,
                                              stride, S.hist + p * 256, parts_d, gsrc, gdst, nullptr, nullptr,
                                              p == 3 ? S.emit_sums : nullptr, stream);
            else
                rts_pass<kIptLarge, uint32_t>(dk[a], vin, dk[b], dv[b], S.n_sorted + 1, 8 * p, p == 3, counts,
                                              stride, S.hist + p * 256, parts_d, gsrc, gdst, nullptr, nullptr,
                                              p == 3 ? S.emit_sums : nullptr, stream);
        }
        if (nb256 > 0) {
            hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanWgThreads), 0, stream, S.emit_sums,
                               static_cast<const uint32_t*>(S.n_sorted));
            launch("emit", k_emit_sorted, dim3(unsigned(nb256)), dim3(256), 0, stream, static_cast<const uint4*>(S.srec),
                   static_cast<const uint32_t*>(dk[0]), static_cast<const uint32_t*>(S.n_sorted),
                   static_cast<const uint32_t*>(S.emit_sums), kb[z], vb[z],
                   compact ? reinterpret_cast<uint16_t*>(vb[z]) : nullptr, compact ? kb[z] : nullptr);
        }
        tile_passes_rts(z);
        if ((rc = check_launch("gs_bin_sort sort"))) return rc;
        launch("tile_ranges", k_tile_ranges, dim3(unsigned((total_tiles + 1 + 255) / 256)), dim3(256), 0, stream,
               static_cast<const uint64_t*>(kb[0]), S.n_sorted, uint32_t(total_tiles), tile_ranges);
        return check_launch("gs_bin_sort ranges");
    }

    // Per-tile path: each tile pass moves the pairs to the other buffer and
    // the per-tile sort writes the caller's keys/vals from the workspace copy.
    int cur = (tile_passes + 1) & 1;
    if (nb > 0)
        launch("emit", k_emit, dim3(unsigned(nb)), dim3(kScanThreads), 0, stream, E, n_total, S.block_sums,
               S.n_sorted, kb[cur], vb[cur], compact ? reinterpret_cast<uint16_t*>(vb[cur]) : nullptr,
               compact ? kb[cur] : nullptr);
    cur = tile_passes_rts(cur);
    if ((rc = check_launch("gs_bin_sort sort"))) return rc;
    // cur == 1: the tile-ordered pairs are in the workspace copy
    launch("tile_ranges", k_tile_ranges, dim3(unsigned((total_tiles + 1 + 255) / 256)), dim3(256), 0, stream,
           static_cast<const uint64_t*>(kb[cur]), S.n_sorted, uint32_t(total_tiles), tile_ranges);
    if ((rc = check_launch("gs_bin_sort ranges"))) return rc;
    // counters[7] (cleared by the scan) counts the long segments
    uint32_t* long_count = S.counters + 7;
    launch("seg_sort", k_seg_sort, dim3(unsigned((total_tiles + 3) / 4)), dim3(256), 0, stream,
           static_cast<const uint64_t*>(kb[cur]), static_cast<const uint32_t*>(vb[cur]), kb[0], vb[0],
           static_cast<const uint32_t*>(tile_ranges), uint32_t(total_tiles),
           static_cast<const uint32_t*>(S.n_sorted), S.long_list, long_count);
    const int64_t long_grid = std::min<int64_t>((total_tiles + kSegWaves - 1) / kSegWaves, 1024);
    launch("seg_sort_long", k_seg_sort_long, dim3(unsigned(long_grid)), dim3(64 * kSegWaves), 0, stream, kb[cur],
           vb[cur], kb[0], vb[0], static_cast<const uint32_t*>(tile_ranges), uint32_t(total_tiles),
           static_cast<const uint32_t*>(S.long_list), static_cast<const uint32_t*>(long_count));
    return check_launch("gs_bin_sort tile sort");
}
