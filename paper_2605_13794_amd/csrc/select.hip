// View-level gate + active-set compaction, importance aggregation with the
// per-view top-mass cut, and the score mask.  Order statistics use an
// MSD radix select over float bits (4 passes of 8 bits, histograms in LDS);
// ties at the threshold are resolved by index with a block-count scan.
#include <mutex>

#include "common.h"

namespace gsmi {

constexpr int kBlk = 256;  // elements per block, one per thread

// Exclusive scan of per-block counts in place (one workgroup); writes the
// total to *total if non-null.  Each thread takes kScanPer consecutive counts
// per round (4,096 counts a round), all loaded before the first use.
struct SelState;
__device__ bool ties_need_ranks(const SelState* s);

constexpr int kScanPer = 16;

__global__ __launch_bounds__(256) void k_scan_counts(uint32_t* __restrict__ cnt, int64_t nb,
                                                     uint64_t* __restrict__ total, const SelState* __restrict__ gate) {
    __shared__ uint32_t w4[4];
    __shared__ uint64_t carry_s;
    if (gate && !ties_need_ranks(gate)) return;  // no tie ranks needed: offsets unused
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256 * kScanPer) {
        const int64_t s0 = b0 + int64_t(threadIdx.x) * kScanPer;
        uint32_t v[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) v[k] = cnt[min<int64_t>(s0 + k, nb - 1)];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = s0 + k < nb ? v[k] : 0u;
            sum += v[k];
        }
        // wave inclusive scan of the per-thread sums
        uint32_t inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane_id() >= uint32_t(o)) inc += t;
        }
        const int w = threadIdx.x / 64;
        if (lane_id() == 63) w4[w] = inc;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int k = 0; k < 4; ++k) {
            if (k < w) before += w4[k];
            tot += w4[k];
        }
        uint64_t run = carry_s + before + inc - sum;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (s0 + k < nb) cnt[s0 + k] = uint32_t(run);
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry_s;
}

// Block-local exclusive rank of `pred` over the block's 256 elements, plus the
// block's count.
__device__ __forceinline__ uint32_t block_rank(bool pred, uint32_t* w4, uint32_t* count) {
    const uint64_t m = ballot(pred);
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) w4[w] = popc64(m);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int k = 0; k < 4; ++k) {
        if (k < w) before += w4[k];
        tot += w4[k];
    }
    __syncthreads();
    *count = tot;
    return before + popc64(m & lanemask_lt());
}

// Writes the wavefront's 64 predicate bits as two 32-bit words.
__device__ __forceinline__ void store_bits(uint32_t* words, int64_t n, int64_t elem0_of_wave, uint64_t m) {
    const int64_t w0 = elem0_of_wave / 32;
    const int64_t nw = (n + 31) / 32;
    if (lane_id() == 0 && w0 < nw) words[w0] = uint32_t(m);
    if (lane_id() == 1 && w0 + 1 < nw) words[w0 + 1] = uint32_t(m >> 32);
}

__device__ __forceinline__ bool bit_of(const uint32_t* words, int64_t i) {
    return (words[i >> 5] >> (i & 31)) & 1u;
}

// ---------------------------------------------------------------------------
// LOD gate and active set
// ---------------------------------------------------------------------------
struct GateArgs {
    const float* mean;
    const float* log_scale;
    const uint8_t* lod;
    const uint32_t* keep;
    int64_t n;
    int mode;
    float campos[3];
    float d0, inv_log2f, fx_k, rmin, fallback;
    int l_max;
};

// Most gate workgroups of a call (the chunk grows with n to stay within it).
constexpr int kGateMaxGroups = 2048;

// Pass 1: each workgroup takes `chunk` consecutive Gaussians (a multiple of
// 512), stores the gate bits and counts gated, gated-and-kept and kept ones.
// Two rounds of 256 Gaussians per trip, every load of both rounds (index
// clamped) issued before the first use; MODE is the call's G.mode.
template <int MODE>
__global__ __launch_bounds__(256) void k_gate(GateArgs G, int64_t chunk, uint32_t* __restrict__ gate_words,
                                              uint32_t* __restrict__ c_gate, uint32_t* __restrict__ c_act,
                                              uint32_t* __restrict__ c_keep) {
    __shared__ uint32_t w4[3][4];
    uint32_t ng = 0, na = 0, nk = 0;  // per wavefront; summed over the workgroup at the end
    const int64_t end = min<int64_t>(G.n, int64_t(blockIdx.x + 1) * chunk);
    for (int64_t base = int64_t(blockIdx.x) * chunk; base < end; base += 2 * kBlk) {
        float mx[2], my[2], mz[2], s0[2], s1[2], s2[2];
        uint32_t lod_[2], kw[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t ic = min<int64_t>(base + u * kBlk + threadIdx.x, G.n - 1);
            mx[u] = my[u] = mz[u] = s0[u] = s1[u] = s2[u] = 0.f;
            lod_[u] = 0u;
            if (MODE != GS_LOD_NONE) {
                mx[u] = G.mean[ic];
                my[u] = G.mean[G.n + ic];
                mz[u] = G.mean[2 * G.n + ic];
                if (MODE == GS_LOD_LEVEL) {
                    lod_[u] = G.lod[ic];
                } else {
                    s0[u] = G.log_scale[ic];
                    s1[u] = G.log_scale[G.n + ic];
                    s2[u] = G.log_scale[2 * G.n + ic];
                }
            }
            kw[u] = G.keep ? G.keep[ic >> 5] : ~0u;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t i = base + u * kBlk + threadIdx.x;
            const bool in = i < G.n;
            bool gate = in;
            if (MODE != GS_LOD_NONE) {
                const float dx = mx[u] - G.campos[0];
                const float dy = my[u] - G.campos[1];
                const float dz = mz[u] - G.campos[2];
                const float d = sqrtf(dx * dx + dy * dy + dz * dz);
                if (MODE == GS_LOD_LEVEL) {
                    int lv;
                    if (d < 1e-6f) {
                        lv = G.l_max;
                    } else {
                        const float x = floorf(log2f(G.d0 / d) * G.inv_log2f + 0.5f);
                        lv = int(fminf(fmaxf(x, 0.f), float(G.l_max)));
                    }
                    gate = in && int(lod_[u]) <= lv;
                } else {
                    const float smax = fmaxf(fmaxf(s0[u], s1[u]), s2[u]);
                    gate = in && G.fx_k * __expf(smax) >= G.rmin * d;
                }
            }
            const bool keep = in && ((kw[u] >> (i & 31)) & 1u);
            const uint64_t mg = ballot(gate);
            store_bits(gate_words, G.n, base + u * kBlk + (threadIdx.x / 64) * 64, mg);
            ng += popc64(mg);
            na += popc64(ballot(gate && keep));
            nk += popc64(ballot(keep));
        }
    }
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) {
        w4[0][w] = ng;
        w4[1][w] = na;
        w4[2][w] = nk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c_gate[blockIdx.x] = w4[0][0] + w4[0][1] + w4[0][2] + w4[0][3];
        c_act[blockIdx.x] = w4[1][0] + w4[1][1] + w4[1][2] + w4[1][3];
        c_keep[blockIdx.x] = w4[2][0] + w4[2][1] + w4[2][2] + w4[2][3];
    }
}

// Pass 2 (same grid): every workgroup sums the nb <= 2048 block counts itself
// (wavefront sums, one barrier) — the total gated count decides the fallback,
// and the counts of the workgroups before it give its output offset.  It then
// takes its Gaussians 32 at a time as words (gate bits and keep bits), ranks
// the words by a block scan of their popcounts, expands the indices of the set
// bits in LDS and writes them out coalesced, in ascending order.  Workgroup 0
// stores the active count.  A round takes `rw` <= 256 words (one per thread);
// the LDS stage holds 32 indices per word, sized at launch (2 KB for 512
// Gaussians per workgroup), since the gate runs beside the blends of another
// stream and a larger stage would hold LDS they could use.
constexpr int kGateWords = 256;  // most words per round of the compaction

__global__ __launch_bounds__(256) void k_gate_compact(GateArgs G, int64_t chunk, int64_t nb,
                                                      const uint32_t* __restrict__ gate_words,
                                                      const uint32_t* __restrict__ c_gate,
                                                      const uint32_t* __restrict__ c_act,
                                                      const uint32_t* __restrict__ c_keep,
                                                      int32_t* __restrict__ out, int64_t* __restrict__ n_active) {
    __shared__ uint32_t part[5][4];
    __shared__ uint32_t wsum[4];
    extern __shared__ int32_t stage[];  // rw * 32 indices
    const int64_t rw = min<int64_t>(kGateWords, chunk / 32);
    const int w = threadIdx.x / 64;
    // gated, active and kept in all workgroups; active and kept before this
    // one.  nb <= 2048: every count load of a thread (index clamped) is issued
    // before the first use.
    uint32_t s[5] = {0u, 0u, 0u, 0u, 0u};
    {
        constexpr int kIt = kGateMaxGroups / 256;
        uint32_t g_[kIt], a_[kIt], k_[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int64_t b = min<int64_t>(int64_t(threadIdx.x) + it * 256, nb - 1);
            g_[it] = c_gate[b];
            a_[it] = c_act[b];
            k_[it] = c_keep[b];
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int64_t b = int64_t(threadIdx.x) + it * 256;
            const bool in = b < nb, before = b < int64_t(blockIdx.x);
            s[0] += in ? g_[it] : 0u;
            s[1] += in ? a_[it] : 0u;
            s[2] += in ? k_[it] : 0u;
            s[3] += before ? a_[it] : 0u;
            s[4] += before ? k_[it] : 0u;
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q] = wave_sum_to_last_u32(s[q]);
    if (lane_id() == 63)
        for (int q = 0; q < 5; ++q) part[q][w] = s[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q] = part[q][0] + part[q][1] + part[q][2] + part[q][3];
    const bool fb = G.n > 0 && double(s[0]) >= double(G.fallback) * double(G.n);
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_active = int64_t(fb ? s[2] : s[1]);
    uint32_t off = fb ? s[4] : s[3];
    const int64_t nw = (G.n + 31) / 32;
    const int64_t w_end = min<int64_t>(nw, (int64_t(blockIdx.x) + 1) * (chunk / 32));
    for (int64_t w0 = int64_t(blockIdx.x) * (chunk / 32); w0 < w_end; w0 += rw) {
        const int64_t wi = w0 + threadIdx.x;
        uint32_t m = 0u;
        if (int64_t(threadIdx.x) < rw && wi < w_end) {
            m = fb ? ~0u : gate_words[wi];
            if (G.keep) m &= G.keep[wi];
            const int64_t rem = G.n - wi * 32;  // >= 1 for wi < nw
            if (rem < 32) m &= (1u << rem) - 1u;
        }
        const uint32_t c = __popc(m);
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane_id() >= uint32_t(o)) inc += t;
        }
        if (lane_id() == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int k = 0; k < 4; ++k) {
            before += k < w ? wsum[k] : 0u;
            tot += wsum[k];
        }
        uint32_t pos = before + inc - c;
        const int32_t i0 = int32_t(wi * 32);
        while (m) {
            stage[pos++] = i0 + (__ffs(m) - 1);
            m &= m - 1u;
        }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < tot; t += 256) out[off + t] = stage[t];
        off += tot;
        __syncthreads();  // stage and wsum are reused by the next round
    }
}

// Gaussians per gate workgroup: 512 (many workgroups in flight; on the 1M view
// the step runs 5 % faster than with 2,048), doubled until there are at most
// 2,048 workgroups, since every compaction workgroup reduces all their counts.
static int64_t gate_chunk(int64_t n) {
    int64_t c = 512;
    while ((n + c - 1) / c > kGateMaxGroups) c *= 2;
    return c;
}

// ---------------------------------------------------------------------------
// Radix select
// ---------------------------------------------------------------------------
struct SelState {
    uint32_t prefix;       // selected high bits so far
    uint32_t done_bits;    // number of bits fixed
    uint32_t need_eq;      // ties at the threshold to take (by ascending index)
    uint32_t cnt_eq;       // elements equal to the threshold
    uint32_t active;       // 0: nothing selected, 1: threshold valid
    uint32_t take_all_eq;  // 1 if every tie is taken
    uint32_t pad[2];
    double target;         // mass mode: frac * W
    double mass_above;     // mass mode: sum of values above the prefix range
    uint64_t k_rem;        // count mode: rank still to place inside the prefix range
};

__device__ bool ties_need_ranks(const SelState* s) { return s->active && !s->take_all_eq; }

// Histograms of the 4 digit passes (8 bits each, most significant first).
struct SelHist {
    uint32_t cnt[4][256];
    double mass[4][256];
};

// One digit pick, computed by all 256 threads of a block from that pass's
// histogram; updates the shared state `s` (mode 0: top mass, mode 1: k-th
// smallest).  Every block computes the same result.
__device__ void block_pick(const uint32_t* __restrict__ hc, const double* __restrict__ hm, SelState& s, int shift,
                          int mode, double* sd, unsigned long long* su, int* si) {
    const int b = threadIdx.x;
    const uint32_t c = hc[b];
    if (mode == 0) {
        // suffix sums of the bin masses: sd[b] = sum over bins >= b
        sd[b] = hm[b];
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const double v = (b + o < 256) ? sd[b + o] : 0.0;
            __syncthreads();
            sd[b] += v;
            __syncthreads();
        }
        if (b == 0) { si[0] = -1; si[1] = 256; }
        __syncthreads();
        const bool ok = s.active && c > 0 && (s.mass_above + sd[b] >= s.target);
        if (ok) atomicMax(&si[0], b);
        if (s.active && c > 0) atomicMin(&si[1], b);
        __syncthreads();
        if (b == 0 && s.active) {
            int chosen = si[0] >= 0 ? si[0] : (si[1] < 256 ? si[1] : -1);  // rounding left the total short
            if (chosen < 0) {
                s.active = 0;
            } else {
                s.mass_above += (chosen < 255) ? sd[chosen + 1] : 0.0;
                s.prefix |= uint32_t(chosen) << shift;
                s.done_bits += 8;
                if (shift == 0) {
                    s.cnt_eq = hc[chosen];
                    const double tau = double(__uint_as_float(s.prefix));
                    double need = ceil((s.target - s.mass_above) / tau);
                    if (need < 1.0) need = 1.0;
                    if (need > double(s.cnt_eq)) need = double(s.cnt_eq);
                    s.need_eq = uint32_t(need);
                    s.take_all_eq = s.need_eq >= s.cnt_eq ? 1u : 0u;
                }
            }
        }
    } else {
        // exclusive prefix counts: su[b] = sum over bins < b
        su[b] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const unsigned long long v = (b >= o) ? su[b - o] : 0ull;
            __syncthreads();
            su[b] += v;
            __syncthreads();
        }
        const unsigned long long excl = su[b] - c;
        if (b == 0) si[0] = 256;
        __syncthreads();
        if (s.active && excl + c >= s.k_rem) atomicMin(&si[0], b);
        __syncthreads();
        if (b == 0 && s.active) {
            const int chosen = si[0];
            if (chosen >= 256) {
                s.active = 0;
            } else {
                s.k_rem -= (su[chosen] - hc[chosen]);
                s.prefix |= uint32_t(chosen) << shift;
                s.done_bits += 8;
                if (shift == 0) {
                    s.cnt_eq = hc[chosen];
                    s.need_eq = uint32_t(s.k_rem);
                    s.take_all_eq = s.need_eq >= s.cnt_eq ? 1u : 0u;
                }
            }
        }
    }
    __syncthreads();
}

__device__ void init_state(SelState& s, int mode, double total, float frac, uint64_t k) {
    memset(&s, 0, sizeof(s));
    if (mode == 0) {
        s.target = double(frac) * total;
        s.active = total > 0.0 ? 1u : 0u;
    } else {
        s.k_rem = k;
        s.active = k > 0 ? 1u : 0u;
    }
}

constexpr int kSelIlp = 8;

// Histogram of digit pass `pass` (shift 24 - 8 pass) over the elements whose
// higher digits match the picks of the earlier passes (replayed per block).
// mode 0 also sums the total mass in pass 0.
__global__ __launch_bounds__(256) void k_sel_hist(const float* __restrict__ v, int64_t n, int pass,
                                                  SelHist* __restrict__ H, double* __restrict__ total, int mode,
                                                  float frac, uint64_t k) {
    __shared__ uint32_t lc[256];
    __shared__ double lm[256];
    __shared__ double sd[256];
    __shared__ unsigned long long su[256];
    __shared__ int si[2];
    __shared__ SelState st;
    const int shift = 24 - 8 * pass;
    if (pass > 0) {
        if (threadIdx.x == 0) init_state(st, mode, *total, frac, k);
        __syncthreads();
        for (int p = 0; p < pass; ++p) block_pick(H->cnt[p], H->mass[p], st, 24 - 8 * p, mode, sd, su, si);
    } else if (threadIdx.x == 0) {
        memset(&st, 0, sizeof(st));
        st.active = 1;
    }
    lc[threadIdx.x] = 0;
    lm[threadIdx.x] = 0.0;
    __syncthreads();
    if (!st.active) return;
    const uint32_t pre = st.prefix;
    const uint32_t hi_mask = shift >= 24 ? 0u : (0xffffffffu << (shift + 8));
    double tsum = 0.0;
    // kSelIlp values per thread per round, loaded before the first is used
    // (index clamped to the last value)
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i0 = int64_t(blockIdx.x) * 256 + threadIdx.x; i0 < n; i0 += stride * kSelIlp) {
        float xs[kSelIlp];
#pragma unroll
        for (int u = 0; u < kSelIlp; ++u) xs[u] = v[min(i0 + u * stride, n - 1)];
#pragma unroll
        for (int u = 0; u < kSelIlp; ++u) {
            const float x = xs[u];
            if (i0 + u * stride >= n) continue;
            if (mode == 0 && !(x > 0.f)) continue;
            if (mode == 0 && pass == 0) tsum += double(x);
            const uint32_t b = __float_as_uint(x);
            if ((b & hi_mask) != (pre & hi_mask)) continue;
            const uint32_t d = (b >> shift) & 255u;
            atomicAdd(&lc[d], 1u);
            if (mode == 0) atomicAdd(&lm[d], double(x));
        }
    }
    __syncthreads();
    if (lc[threadIdx.x]) {
        atomicAdd(&H->cnt[pass][threadIdx.x], lc[threadIdx.x]);
        if (mode == 0) atomicAdd(&H->mass[pass][threadIdx.x], lm[threadIdx.x]);
    }
    if (mode == 0 && pass == 0) {
        sd[threadIdx.x] = tsum;
        __syncthreads();
        for (uint32_t o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) sd[threadIdx.x] += sd[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0 && sd[0] != 0.0) atomicAdd(total, sd[0]);
    }
}

// Final state from the four histograms (one block).
__global__ __launch_bounds__(256) void k_sel_final(const SelHist* __restrict__ H, const double* __restrict__ total,
                                                   SelState* __restrict__ out, int mode, float frac, uint64_t k) {
    __shared__ double sd[256];
    __shared__ unsigned long long su[256];
    __shared__ int si[2];
    __shared__ SelState st;
    if (threadIdx.x == 0) init_state(st, mode, *total, frac, k);
    __syncthreads();
    for (int p = 0; p < 4; ++p) block_pick(H->cnt[p], H->mass[p], st, 24 - 8 * p, mode, sd, su, si);
    if (threadIdx.x == 0) *out = st;
}

__global__ void k_sel_init(SelHist* __restrict__ H, double* __restrict__ total) {
    for (int k = threadIdx.x; k < 4 * 256; k += blockDim.x) {
        (&H->cnt[0][0])[k] = 0;
        (&H->mass[0][0])[k] = 0.0;
    }
    if (threadIdx.x == 0) *total = 0.0;
}

// Per-block count of elements equal to the threshold (only when ranks matter).
__global__ __launch_bounds__(256) void k_eq_count(const float* __restrict__ v, int64_t n,
                                                  const SelState* __restrict__ st, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t w4[4];
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    const bool need = st->active && !st->take_all_eq;
    const bool eq = need && i < n && __float_as_uint(v[i]) == st->prefix;
    uint32_t tot;
    block_rank(eq, w4, &tot);
    if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

__device__ __forceinline__ bool selected(float x, uint32_t rank_eq, const SelState& s, int mode) {
    if (!s.active) return false;
    const uint32_t b = __float_as_uint(x);
    if (mode == 0) {
        if (!(x > 0.f)) return false;
        if (b > s.prefix) return true;  // positive floats order as their bits
    } else {
        if (b < s.prefix) return true;
    }
    if (b != s.prefix) return false;
    return s.take_all_eq || rank_eq < s.need_eq;
}

// ---------------------------------------------------------------------------
// Importance fold
// ---------------------------------------------------------------------------
// The blend's (w, count) records to the w and a arrays.
__global__ __launch_bounds__(256) void k_importance_split(const float2* __restrict__ wa, int64_t n,
                                                          float* __restrict__ w, uint32_t* __restrict__ a) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= n) return;
    const float2 r = wa[i];
    w[i] = r.x;
    a[i] = uint32_t(r.y);
}

__global__ __launch_bounds__(256) void k_importance_fold(const float* __restrict__ w, const uint32_t* __restrict__ a,
                                                         const int32_t* __restrict__ radius, int64_t n,
                                                         const SelState* __restrict__ stp,
                                                         const uint32_t* __restrict__ eq_off, float eps,
                                                         float* __restrict__ score, uint32_t* __restrict__ c_rad,
                                                         uint32_t* __restrict__ c_vis, uint32_t* __restrict__ cull) {
    __shared__ uint32_t w4[4];
    const SelState s = *stp;
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    const bool in = i < n;
    const float wi = in ? w[i] : 0.f;
    const bool eq = in && s.active && !s.take_all_eq && __float_as_uint(wi) == s.prefix;
    uint32_t tot;
    const uint32_t r = block_rank(eq, w4, &tot);
    const uint32_t rank_eq = eq ? eq_off[blockIdx.x] + r : 0u;
    const bool vis = in && selected(wi, rank_eq, s, 0);
    const uint64_t m = ballot(in && !vis);
    store_bits(cull, n, int64_t(blockIdx.x) * kBlk + (threadIdx.x / 64) * 64, m);
    if (!in) return;
    const uint32_t ai = a[i];
    if (ai > 0) score[i] += wi / (float(ai) + eps);
    if (radius[i] > 0) c_rad[i] += 1u;
    if (vis) c_vis[i] += 1u;
}

// Keep bitmap from a selection: mode 1 selects the k smallest values (keep =
// not selected for the score mask, keep = selected for race sampling); mode 0
// selects the top-mass prefix (keep = selected).  Also counts the kept bits.
__global__ __launch_bounds__(256) void k_keep_bits(const float* __restrict__ score, int64_t n,
                                                   const SelState* __restrict__ stp, const uint32_t* __restrict__ eq_off,
                                                   uint32_t* __restrict__ keep, int mode, int keep_selected,
                                                   unsigned long long* __restrict__ n_keep) {
    __shared__ uint32_t w4[4];
    const SelState s = *stp;
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    const bool in = i < n;
    const float x = in ? score[i] : 0.f;
    const bool eq = in && s.active && !s.take_all_eq && __float_as_uint(x) == s.prefix;
    uint32_t tot;
    const uint32_t r = block_rank(eq, w4, &tot);
    const uint32_t rank_eq = eq ? eq_off[blockIdx.x] + r : 0u;
    const bool sel = in && selected(x, rank_eq, s, mode);
    const bool k = in && (keep_selected ? sel : !sel);
    const uint64_t m = ballot(k);
    store_bits(keep, n, int64_t(blockIdx.x) * kBlk + (threadIdx.x / 64) * 64, m);
    if (n_keep) {
        uint32_t cnt;
        block_rank(k, w4, &cnt);
        if (threadIdx.x == 0 && cnt) atomicAdd(n_keep, (unsigned long long)cnt);
    }
}

// Race times of weighted sampling without replacement: -ln(u) / s, +inf for s = 0.
__global__ __launch_bounds__(256) void k_race_times(const float* __restrict__ score, const float* __restrict__ u,
                                                    int64_t n, float* __restrict__ e) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const float s = score[i];
    e[i] = s > 0.f ? -logf(u[i]) / s : __uint_as_float(0x7f800000u);
}

// Compaction of component-major arrays by a keep bitmap.
struct CompactArgs {
    const void* src[16];
    void* dst[16];
    int32_t rows[16];
    int32_t bytes[16];
    int n_arrays;
};

#define GS_GLOBAL __attribute__((address_space(1)))

// Columns per thread in the compaction (kBlk apart, so that every load of a
// row is one coalesced dword per lane) and rows whose loads are issued
// together before the first store.
constexpr int kCompJ = 4;
constexpr int kCompCols = kBlk * kCompJ;
constexpr int kCompRows = 8;

// Kept elements per block of kBlk * J elements.
template <int J>
__global__ __launch_bounds__(256) void k_keep_count(const uint32_t* __restrict__ keep, int64_t n,
                                                    uint32_t* __restrict__ cnt) {
    __shared__ uint32_t w4[4];
    const int64_t i0 = int64_t(blockIdx.x) * (kBlk * J) + threadIdx.x;
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int64_t i = i0 + int64_t(j) * kBlk;
        uint32_t tot;
        block_rank(i < n && bit_of(keep, i), w4, &tot);
        sum += tot;
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = sum;
}

// One array's rows for this thread's kCompJ columns: kCompRows x kCompJ
// loads (row index clamped, column clamped in range) issued before the
// stores of the kept columns. The row base is wave-uniform and the column
// and destination offsets fit 32 bits (n < 2^31).
template <typename T>
__device__ __forceinline__ void compact_rows(const T GS_GLOBAL* s, T GS_GLOBAL* d, int rows, int64_t n,
                                             int64_t n_keep, const uint32_t (&col)[kCompJ],
                                             const uint32_t (&r)[kCompJ], const bool (&k)[kCompJ]) {
    for (int c = 0; c < rows; c += kCompRows) {
        T v[kCompRows][kCompJ];
#pragma unroll
        for (int u = 0; u < kCompRows; ++u) {
            const T GS_GLOBAL* sr = s + int64_t(min(c + u, rows - 1)) * n;
#pragma unroll
            for (int j = 0; j < kCompJ; ++j) v[u][j] = sr[col[j]];
        }
#pragma unroll
        for (int u = 0; u < kCompRows; ++u) {
            T GS_GLOBAL* dr = d + int64_t(c + u) * n_keep;
#pragma unroll
            for (int j = 0; j < kCompJ; ++j)
                if (k[j] && c + u < rows) dr[r[j]] = v[u][j];
        }
    }
}

__global__ __launch_bounds__(256) void k_compact_arrays(CompactArgs A, const uint32_t* __restrict__ keep, int64_t n,
                                                        int64_t n_keep, const uint32_t* __restrict__ offs) {
    __shared__ uint32_t w4[4];
    const int64_t i0 = int64_t(blockIdx.x) * kCompCols + threadIdx.x;
    uint32_t word[kCompJ], col[kCompJ], r[kCompJ];
    bool k[kCompJ];
#pragma unroll
    for (int j = 0; j < kCompJ; ++j) {
        col[j] = uint32_t(min(i0 + int64_t(j) * kBlk, n - 1));
        word[j] = keep[col[j] >> 5];
    }
    int64_t run = offs[blockIdx.x];
    bool any = false;
#pragma unroll
    for (int j = 0; j < kCompJ; ++j) {
        const bool kj = i0 + int64_t(j) * kBlk < n && ((word[j] >> (col[j] & 31)) & 1u);
        uint32_t tot;
        const int64_t rj = run + block_rank(kj, w4, &tot);
        run += tot;
        k[j] = kj && rj < n_keep;
        r[j] = uint32_t(rj);
        any |= k[j];
    }
    if (!any) return;
    for (int a = 0; a < A.n_arrays; ++a) {
        if (A.bytes[a] == 4)
            compact_rows<float>((const float GS_GLOBAL*)A.src[a], (float GS_GLOBAL*)A.dst[a], A.rows[a], n, n_keep,
                                col, r, k);
        else
            compact_rows<uint8_t>((const uint8_t GS_GLOBAL*)A.src[a], (uint8_t GS_GLOBAL*)A.dst[a], A.rows[a], n,
                                  n_keep, col, r, k);
    }
}

struct SelWs {
    SelState* st;
    SelHist* hist;
    double* total;
    uint32_t* eq_cnt;
    uint64_t* tot64;
    size_t bytes;
};

static SelWs carve_sel(Carve& cv, int64_t n) {
    SelWs s;
    const int64_t nb = (n + kBlk - 1) / kBlk + 1;
    s.st = cv.take<SelState>(1);
    s.hist = cv.take<SelHist>(1);
    s.total = cv.take<double>(1);
    s.eq_cnt = cv.take<uint32_t>(size_t(nb));
    s.tot64 = cv.take<uint64_t>(1);
    s.bytes = 0;
    return s;
}

static int run_select(const float* v, int64_t n, int mode, float frac, uint64_t k, const SelWs& W, hipStream_t s) {
    const int64_t nb = (n + kBlk - 1) / kBlk;
    const int hb = int(std::min<int64_t>(1024, std::max<int64_t>(1, (n + 4095) / 4096)));
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, W.hist, W.total);
    for (int pass = 0; pass < 4; ++pass)
        launch("sel_hist", k_sel_hist, dim3(hb), dim3(256), 0, s, v, n, pass, W.hist, W.total, mode, frac, k);
    hipLaunchKernelGGL(k_sel_final, dim3(1), dim3(256), 0, s, W.hist, W.total, W.st, mode, frac, k);
    if (nb > 0) {
        hipLaunchKernelGGL(k_eq_count, dim3(unsigned(nb)), dim3(256), 0, s, v, n, W.st, W.eq_cnt);
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, s, W.eq_cnt, nb, W.tot64,
                           static_cast<const SelState*>(W.st));
    }
    return check_launch("radix select");
}

}  // namespace gsmi

using namespace gsmi;

size_t ws_lod_mask(int64_t n) {
    Carve cv(nullptr);
    const int64_t nb = (n + gate_chunk(n) - 1) / gate_chunk(n) + 1;
    cv.take<uint32_t>(size_t((n + 31) / 32 + 2));
    cv.take<uint32_t>(size_t(nb));
    cv.take<uint32_t>(size_t(nb));
    cv.take<uint32_t>(size_t(nb));
    return cv.used();
}

size_t ws_importance(int64_t n) {
    Carve cv(nullptr);
    cv.take<float>(size_t(2 * (n > 0 ? n : 1)));
    carve_sel(cv, n);
    return cv.used();
}

size_t ws_score_keep(int64_t n) {
    Carve cv(nullptr);
    carve_sel(cv, n);
    return cv.used();
}

namespace gsmi {
int launch_importance_blend(const gs_projected* proj, const gs_camera* cam, const uint32_t* vals,
                            const uint32_t* ranges, float* wa, int footprint, hipStream_t stream);
}

static int lod_mask_checks(const gs_scene* scene, const gs_camera* cam, const gs_lod_params* params,
                           const int32_t* active_idx, const int64_t* n_active_dev) {
    if (!scene || !cam || !params || !active_idx || !n_active_dev)
        return fail(GS_ERR_INVALID_ARG, "gs_lod_mask: null argument");
    if (scene->n < 0 || scene->n >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_lod_mask: bad n");
    const int64_t n = scene->n;
    if (params->mode != GS_LOD_NONE && params->mode != GS_LOD_LEVEL && params->mode != GS_LOD_RADIUS)
        return fail(GS_ERR_INVALID_ARG, "gs_lod_mask: unknown mode %d", params->mode);
    if (n > 0 && params->mode != GS_LOD_NONE && !scene->mean)
        return fail(GS_ERR_INVALID_ARG, "gs_lod_mask: null means");
    if (n > 0 && params->mode == GS_LOD_LEVEL && (!scene->lod || !(params->d0 > 0.f) || !(params->f > 1.f)))
        return fail(GS_ERR_INVALID_ARG, "gs_lod_mask: level mode needs lod labels, d0 > 0 and f > 1");
    if (n > 0 && params->mode == GS_LOD_RADIUS && !scene->log_scale)
        return fail(GS_ERR_INVALID_ARG, "gs_lod_mask: radius mode needs log-scales");
    return GS_OK;
}

// Gate and compaction with the scratch at `ws` (checked by the caller).
static int lod_mask_launch(const gs_scene* scene, const gs_camera* cam, const gs_lod_params* params,
                           const uint32_t* keep_bits, int32_t* active_idx, int64_t* n_active_dev, void* ws,
                           hipStream_t stream) {
    const int64_t n = scene->n;
    DevCam dc = make_devcam(*cam, 0);
    GateArgs G;
    memset(&G, 0, sizeof(G));
    G.mean = scene->mean; G.log_scale = scene->log_scale; G.lod = scene->lod; G.keep = keep_bits; G.n = n;
    G.mode = params->mode;
    for (int k = 0; k < 3; ++k) G.campos[k] = dc.campos[k];
    G.d0 = params->d0;
    G.inv_log2f = params->mode == GS_LOD_LEVEL ? float(1.0 / std::log2(double(params->f))) : 1.f;
    G.fx_k = cam->fx * params->radius_sigma_k;
    G.rmin = params->radius_min_px;
    G.fallback = params->fallback_ratio;
    G.l_max = params->l_max;
    Carve cv(ws);
    const int64_t chunk = gate_chunk(n);
    const int64_t nb = (n + chunk - 1) / chunk;
    uint32_t* words = cv.take<uint32_t>(size_t((n + 31) / 32 + 2));
    uint32_t* c_gate = cv.take<uint32_t>(size_t(nb + 1));
    uint32_t* c_act = cv.take<uint32_t>(size_t(nb + 1));
    uint32_t* c_keep = cv.take<uint32_t>(size_t(nb + 1));
    if (n == 0) {
        int rc = fill_u32(n_active_dev, 0u, 2, stream);
        if (rc) return rc;
        return check_launch("gs_lod_mask");
    }
    if (G.mode == GS_LOD_LEVEL)
        launch("gate", k_gate<GS_LOD_LEVEL>, dim3(unsigned(nb)), dim3(256), 0, stream, G, chunk, words, c_gate, c_act,
               c_keep);
    else if (G.mode == GS_LOD_RADIUS)
        launch("gate", k_gate<GS_LOD_RADIUS>, dim3(unsigned(nb)), dim3(256), 0, stream, G, chunk, words, c_gate,
               c_act, c_keep);
    else
        launch("gate", k_gate<GS_LOD_NONE>, dim3(unsigned(nb)), dim3(256), 0, stream, G, chunk, words, c_gate, c_act,
               c_keep);
    const size_t stage_bytes = size_t(std::min<int64_t>(kGateWords, chunk / 32)) * 32 * sizeof(int32_t);
    launch("compact", k_gate_compact, dim3(unsigned(nb)), dim3(256), stage_bytes, stream, G, chunk, nb,
           static_cast<const uint32_t*>(words), static_cast<const uint32_t*>(c_gate),
           static_cast<const uint32_t*>(c_act), static_cast<const uint32_t*>(c_keep), active_idx, n_active_dev);
    return check_launch("gs_lod_mask");
}

extern "C" int gs_lod_mask(const gs_scene* scene, const gs_camera* cam, const gs_lod_params* params,
                           const uint32_t* keep_bits, int32_t* active_idx, int64_t* n_active_dev, void* ws,
                           size_t ws_bytes, hipStream_t stream) {
    int rc = lod_mask_checks(scene, cam, params, active_idx, n_active_dev);
    if (rc) return rc;
    const size_t need = ws_lod_mask(scene->n);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_lod_mask: workspace needs %zu bytes (256-aligned)", need);
    return lod_mask_launch(scene, cam, params, keep_bits, active_idx, n_active_dev, ws, stream);
}

// ---------------------------------------------------------------------------
// Allocation-free gate: the scratch of gs_lod_mask (gate bitmap and
// per-workgroup counts, fully rewritten by every call, so nothing needs
// clearing) lives in a fixed device array.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is looked up once
// per device with hipGetSymbolAddress and only that address is handed to
// kernels.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxN = int64_t(1) << 24;
constexpr size_t kNoAllocScratchBytes = (size_t(2) << 20) + (size_t(64) << 10);
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_on_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GS_ERR_HIP, "gs_lod_mask_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_HIP, "gs_lod_mask_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GS_ERR_HIP, "gs_lod_mask_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GS_OK;
}

extern "C" int gs_lod_mask_noalloc(const gs_scene* scene, const gs_camera* cam, const gs_lod_params* params,
                                   const uint32_t* keep_bits, int32_t* active_idx, int64_t* n_active_dev,
                                   hipStream_t stream) {
    int rc = lod_mask_checks(scene, cam, params, active_idx, n_active_dev);
    if (rc) return rc;
    if (scene->n > kNoAllocMaxN || ws_lod_mask(scene->n) > kNoAllocScratchBytes)
        return fail(GS_ERR_INVALID_ARG, "gs_lod_mask_noalloc: n = %lld exceeds the fixed scratch (at most %lld)",
                    (long long)scene->n, (long long)kNoAllocMaxN);
    void* ws = nullptr;
    if ((rc = scratch_on_current_device(&ws))) return rc;
    return lod_mask_launch(scene, cam, params, keep_bits, active_idx, n_active_dev, ws, stream);
}

extern "C" int gs_importance(const gs_projected* proj, const gs_camera* cam, int64_t n, const uint32_t* vals,
                             const uint32_t* tile_ranges, float mass_frac, float eps, int32_t count_mode, float* w,
                             uint32_t* a, float* score, uint32_t* c_rad, uint32_t* c_vis, uint32_t* cull_row,
                             void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!proj || !cam || !tile_ranges || !w || !a || !score || !c_rad || !c_vis || !cull_row)
        return fail(GS_ERR_INVALID_ARG, "gs_importance: null argument");
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_importance: bad n");
    if (!(mass_frac > 0.f) || mass_frac > 1.f) return fail(GS_ERR_INVALID_ARG, "gs_importance: mass_frac in (0, 1]");
    if (!proj->radius) return fail(GS_ERR_INVALID_ARG, "gs_importance: null radius");
    if (count_mode != GS_COUNT_COMPOSITED && count_mode != GS_COUNT_FOOTPRINT)
        return fail(GS_ERR_INVALID_ARG, "gs_importance: unknown count mode %d", count_mode);
    const size_t need = ws_importance(n);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_importance: workspace needs %zu bytes (256-aligned)", need);
    if (n == 0) return GS_OK;
    int rc;
    Carve cv(ws);
    float* wa = cv.take<float>(size_t(2 * n));
    if ((rc = fill_u32(wa, 0u, size_t(2 * n), stream))) return rc;
    if ((rc = launch_importance_blend(proj, cam, vals, tile_ranges, wa, count_mode == GS_COUNT_FOOTPRINT, stream)))
        return rc;
    const int64_t nbs = (n + kBlk - 1) / kBlk;
    launch("importance_split", k_importance_split, dim3(unsigned(nbs)), dim3(256), 0, stream,
           static_cast<const float2*>(static_cast<void*>(wa)), n, w, a);
    SelWs S = carve_sel(cv, n);
    if ((rc = run_select(w, n, 0, mass_frac, 0, S, stream))) return rc;
    const int64_t nb = (n + kBlk - 1) / kBlk;
    launch("importance_fold", k_importance_fold, dim3(unsigned(nb)), dim3(256), 0, stream, w, a, proj->radius, n, S.st,
                       S.eq_cnt, eps, score, c_rad, c_vis, cull_row);
    return check_launch("gs_importance");
}

extern "C" int gs_score_keep_bits(const float* score, int64_t n, int64_t n_drop, uint32_t* keep_bits, void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
    if (!score || !keep_bits) return fail(GS_ERR_INVALID_ARG, "gs_score_keep_bits: null argument");
    if (n < 0 || n >= (int64_t(1) << 31) || n_drop < 0 || n_drop > n)
        return fail(GS_ERR_INVALID_ARG, "gs_score_keep_bits: need 0 <= n_drop <= n < 2^31");
    const size_t need = ws_score_keep(n);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_score_keep_bits: workspace needs %zu bytes (256-aligned)", need);
    if (n == 0) return GS_OK;
    Carve cv(ws);
    SelWs S = carve_sel(cv, n);
    int rc;
    if ((rc = run_select(score, n, 1, 0.f, uint64_t(n_drop), S, stream))) return rc;
    const int64_t nb = (n + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(k_keep_bits, dim3(unsigned(nb)), dim3(256), 0, stream, score, n, S.st, S.eq_cnt, keep_bits, 1,
                       0, static_cast<unsigned long long*>(nullptr));
    return check_launch("gs_score_keep_bits");
}

size_t ws_simplify(int64_t n) {
    Carve cv(nullptr);
    carve_sel(cv, n);
    cv.take<float>(size_t(n > 0 ? n : 1));
    cv.take<uint32_t>(size_t((n + kBlk - 1) / kBlk + 1));
    return cv.used();
}

extern "C" int gs_mass_keep_bits(const float* score, int64_t n, float mass_frac, uint32_t* keep_bits,
                                 int64_t* n_keep_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!score || !keep_bits || !n_keep_dev) return fail(GS_ERR_INVALID_ARG, "gs_mass_keep_bits: null argument");
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_mass_keep_bits: bad n");
    if (!(mass_frac > 0.f) || mass_frac > 1.f) return fail(GS_ERR_INVALID_ARG, "gs_mass_keep_bits: mass_frac in (0, 1]");
    const size_t need = ws_simplify(n);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_mass_keep_bits: workspace needs %zu bytes (256-aligned)", need);
    int rc;
    if ((rc = fill_u32(n_keep_dev, 0u, 2, stream))) return rc;
    if (n == 0) return GS_OK;
    Carve cv(ws);
    SelWs S = carve_sel(cv, n);
    if ((rc = run_select(score, n, 0, mass_frac, 0, S, stream))) return rc;
    const int64_t nb = (n + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(k_keep_bits, dim3(unsigned(nb)), dim3(256), 0, stream, score, n, S.st, S.eq_cnt, keep_bits, 0,
                       1, reinterpret_cast<unsigned long long*>(n_keep_dev));
    return check_launch("gs_mass_keep_bits");
}

extern "C" int gs_sample_keep_bits(const float* score, const float* uniforms, int64_t n, int64_t n_keep,
                                   uint32_t* keep_bits, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!score || !uniforms || !keep_bits) return fail(GS_ERR_INVALID_ARG, "gs_sample_keep_bits: null argument");
    if (n < 0 || n >= (int64_t(1) << 31) || n_keep < 0 || n_keep > n)
        return fail(GS_ERR_INVALID_ARG, "gs_sample_keep_bits: need 0 <= n_keep <= n < 2^31");
    const size_t need = ws_simplify(n);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_sample_keep_bits: workspace needs %zu bytes (256-aligned)", need);
    if (n == 0) return GS_OK;
    Carve cv(ws);
    SelWs S = carve_sel(cv, n);
    float* e = cv.take<float>(size_t(n));
    hipLaunchKernelGGL(k_race_times, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, score, uniforms, n, e);
    int rc;
    if ((rc = run_select(e, n, 1, 0.f, uint64_t(n_keep), S, stream))) return rc;
    const int64_t nb = (n + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(k_keep_bits, dim3(unsigned(nb)), dim3(256), 0, stream, e, n, S.st, S.eq_cnt, keep_bits, 1, 1,
                       static_cast<unsigned long long*>(nullptr));
    return check_launch("gs_sample_keep_bits");
}

extern "C" int gs_compact(const void* const* src, void* const* dst, const int32_t* rows, const int32_t* elem_bytes,
                          int n_arrays, int64_t n, int64_t n_keep, const uint32_t* keep_bits, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
    if (n_arrays < 1 || n_arrays > 16 || !src || !dst || !rows || !elem_bytes || (n > 0 && !keep_bits))
        return fail(GS_ERR_INVALID_ARG, "gs_compact: bad arguments");
    if (n < 0 || n >= (int64_t(1) << 31) || n_keep < 0 || n_keep > n)
        return fail(GS_ERR_INVALID_ARG, "gs_compact: need 0 <= n_keep <= n < 2^31");
    CompactArgs A;
    memset(&A, 0, sizeof(A));
    A.n_arrays = n_arrays;
    for (int a = 0; a < n_arrays; ++a) {
        if ((elem_bytes[a] != 4 && elem_bytes[a] != 1) || rows[a] < 1 || (n > 0 && (!src[a] || !dst[a])))
            return fail(GS_ERR_INVALID_ARG, "gs_compact: array %d", a);
        A.src[a] = src[a]; A.dst[a] = dst[a]; A.rows[a] = rows[a]; A.bytes[a] = elem_bytes[a];
    }
    const size_t need = ws_simplify(n);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_compact: workspace needs %zu bytes (256-aligned)", need);
    if (n == 0 || n_keep == 0) return GS_OK;
    Carve cv(ws);
    SelWs S = carve_sel(cv, n);
    (void)S;
    cv.take<float>(size_t(n));
    const int64_t nb = (n + kCompCols - 1) / kCompCols;
    uint32_t* cnt = cv.take<uint32_t>(size_t(nb + 1));
    hipLaunchKernelGGL(k_keep_count<kCompJ>, dim3(unsigned(nb)), dim3(256), 0, stream, keep_bits, n, cnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, stream, cnt, nb, static_cast<uint64_t*>(nullptr),
                       static_cast<const SelState*>(nullptr));
    hipLaunchKernelGGL(k_compact_arrays, dim3(unsigned(nb)), dim3(256), 0, stream, A, keep_bits, n, n_keep, cnt);
    return check_launch("gs_compact");
}

// ---------------------------------------------------------------------------
// Spawn gate (Sec. 3.2 "Spawn gate"; veto equation of Appendix E): within
// each candidate set the ceil(rho |C|) candidates of lowest predicted
// survival are vetoed (ties by index, the lower vetoed first), the survivors
// are instantiated with the inherited level (clone: the parent's, split: one
// finer, clamped at K-1).
// ---------------------------------------------------------------------------
namespace gsmi {

__global__ __launch_bounds__(256) void k_spawn_emit(const int32_t* __restrict__ parent, const uint32_t* __restrict__ keep,
                                                    int64_t n, const uint8_t* __restrict__ lod, int split, int n_levels,
                                                    const uint32_t* __restrict__ offs, int64_t out_base,
                                                    int32_t* __restrict__ child_parent, uint8_t* __restrict__ child_lod,
                                                    uint8_t* __restrict__ child_split) {
    __shared__ uint32_t w4[4];
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    const bool k = i < n && bit_of(keep, i);
    uint32_t tot;
    const uint32_t r = block_rank(k, w4, &tot);
    if (!k) return;
    const int64_t o = out_base + offs[blockIdx.x] + r;
    const int32_t pj = parent[i];
    child_parent[o] = pj;
    child_lod[o] = uint8_t(min(int(lod[pj]) + split, n_levels - 1));
    child_split[o] = uint8_t(split);
}

// Stand-in survival score: the parent's opacity.
__global__ __launch_bounds__(256) void k_spawn_stub(const float* __restrict__ opacity_logit,
                                                    const int32_t* __restrict__ parent, int64_t n,
                                                    float* __restrict__ p) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= n) return;
    p[i] = 1.f / (1.f + expf(-opacity_logit[parent[i]]));
}

}  // namespace gsmi

static int64_t veto_count(int64_t n, double rho) {
    const double v = std::ceil(rho * double(n));
    return std::min<int64_t>(n, std::max<int64_t>(0, int64_t(v)));
}

size_t ws_spawn_gate(int64_t n) {
    Carve cv(nullptr);
    carve_sel(cv, n);
    cv.take<uint32_t>(size_t((n + 31) / 32 + 1));
    cv.take<uint32_t>(size_t((n + kBlk - 1) / kBlk + 1));
    return cv.used();
}

extern "C" int gs_spawn_gate(const uint8_t* lod, const int32_t* clone_parent, const float* p_clone, int64_t n_clone,
                             const int32_t* split_parent, const float* p_split, int64_t n_split, double rho,
                             int32_t n_levels, int32_t* child_parent, uint8_t* child_lod, uint8_t* child_split,
                             int64_t* n_children, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_clone < 0 || n_split < 0 || n_clone >= (int64_t(1) << 31) || n_split >= (int64_t(1) << 31))
        return fail(GS_ERR_INVALID_ARG, "gs_spawn_gate: candidate counts must be in [0, 2^31)");
    if (!(rho >= 0.0 && rho <= 1.0)) return fail(GS_ERR_INVALID_ARG, "gs_spawn_gate: rho must be in [0, 1]");
    if (n_levels < 1 || n_levels > 255) return fail(GS_ERR_INVALID_ARG, "gs_spawn_gate: n_levels in [1, 255]");
    if (!n_children) return fail(GS_ERR_INVALID_ARG, "gs_spawn_gate: null n_children");
    if ((n_clone > 0 && (!clone_parent || !p_clone)) || (n_split > 0 && (!split_parent || !p_split)))
        return fail(GS_ERR_INVALID_ARG, "gs_spawn_gate: null candidate array");
    const int64_t v_c = veto_count(n_clone, rho), v_s = veto_count(n_split, rho);
    const int64_t total = (n_clone - v_c) + (n_split - v_s);
    if (total > 0 && (!lod || !child_parent || !child_lod || !child_split))
        return fail(GS_ERR_INVALID_ARG, "gs_spawn_gate: null level or output array");
    const int64_t nmax = std::max(n_clone, n_split);
    const size_t need = ws_spawn_gate(nmax);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_spawn_gate: workspace needs %zu bytes (256-aligned)", need);
    *n_children = total;
    Carve cv(ws);
    SelWs S = carve_sel(cv, nmax);
    uint32_t* keep = cv.take<uint32_t>(size_t((nmax + 31) / 32 + 1));
    uint32_t* cnt = cv.take<uint32_t>(size_t((nmax + kBlk - 1) / kBlk + 1));
    int rc;
    int64_t base = 0;
    const int32_t* parents[2] = {clone_parent, split_parent};
    const float* scores[2] = {p_clone, p_split};
    const int64_t counts[2] = {n_clone, n_split}, vetoes[2] = {v_c, v_s};
    for (int set = 0; set < 2; ++set) {
        const int64_t n = counts[set];
        if (n == 0) continue;
        if ((rc = run_select(scores[set], n, 1, 0.f, uint64_t(vetoes[set]), S, stream))) return rc;
        const int64_t nb = (n + kBlk - 1) / kBlk;
        hipLaunchKernelGGL(k_keep_bits, dim3(unsigned(nb)), dim3(256), 0, stream, scores[set], n,
                           static_cast<const SelState*>(S.st), static_cast<const uint32_t*>(S.eq_cnt), keep, 1, 0,
                           static_cast<unsigned long long*>(nullptr));
        hipLaunchKernelGGL(k_keep_count<1>, dim3(unsigned(nb)), dim3(256), 0, stream, static_cast<const uint32_t*>(keep),
                           n, cnt);
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, stream, cnt, nb, static_cast<uint64_t*>(nullptr),
                           static_cast<const SelState*>(nullptr));
        launch("spawn_emit", k_spawn_emit, dim3(unsigned(nb)), dim3(256), 0, stream, parents[set],
               static_cast<const uint32_t*>(keep), n, lod, set, int(n_levels), static_cast<const uint32_t*>(cnt), base,
               child_parent, child_lod, child_split);
        base += n - vetoes[set];
    }
    return check_launch("gs_spawn_gate");
}

extern "C" int gs_spawn_stub_score(const gs_scene* scene, const int32_t* parent, int64_t n, float* p,
                                   hipStream_t stream) {
    if (!scene || n < 0 || n >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_spawn_stub_score: bad arguments");
    if (n > 0 && (!scene->opacity_logit || !parent || !p))
        return fail(GS_ERR_INVALID_ARG, "gs_spawn_stub_score: null argument");
    if (n == 0) return GS_OK;
    launch("spawn_stub", k_spawn_stub, dim3(unsigned((n + kBlk - 1) / kBlk)), dim3(256), 0, stream,
           scene->opacity_logit, parent, n, p);
    return check_launch("gs_spawn_stub_score");
}

// Coarse-to-fine ceiling L_max(t) of the level gate (host arithmetic).
extern "C" int32_t gs_lod_level_ceiling(int64_t t, int64_t t0, int64_t t1, int32_t n_levels) {
    if (n_levels <= 1 || t <= t0) return 0;
    if (t >= t1) return n_levels - 1;
    int32_t best = 0;
    for (int32_t k = 0; k < n_levels; ++k) {
        const double u = double(t0) * std::pow(double(t1) / double(t0), double(k) / double(n_levels - 1));
        if (u <= double(t)) best = k;
    }
    return best;
}
