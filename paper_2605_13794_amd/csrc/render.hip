// Front-to-back compositing of 16x16 tiles, its backward, and the
// colour-less instrumented blend of the importance sweep.
//
// One wavefront (64 lanes) owns one tile; lane l covers column l % 16 and
// rows l / 16 + {0, 4, 8, 12}, so each record staged in LDS is read once per
// lane and evaluated for four pixels that share dx.  Records are gathered
// from the packed per-Gaussian render record in batches of 64.
#include "common.h"

namespace gsmi {

struct RenderCams {
    const float* rec[GS_MAX_CAMS];
    uint32_t tile_off[GS_MAX_CAMS + 1];
    int32_t TX[GS_MAX_CAMS];
    int32_t W[GS_MAX_CAMS];
    int32_t H[GS_MAX_CAMS];
    int n_cams;
};

struct TileCtx {
    int c;
    int px, py0;
    float fxp;
    float fyp[4];
    float ymid0;  // centre row of the strip of rows 0..3 (strip r: + 4r)
    bool valid[4];
    uint32_t start, end;
};

__device__ __forceinline__ TileCtx tile_ctx(const RenderCams& A, const uint32_t* ranges, uint32_t n_tiles) {
    TileCtx t;
    const uint32_t tile = blockIdx.x;
    int c = 0;
    while (c + 1 < A.n_cams && tile >= A.tile_off[c + 1]) ++c;
    t.c = c;
    const uint32_t lt = tile - A.tile_off[c];
    const int TX = A.TX[c];
    const int tx = int(lt % uint32_t(TX)), ty = int(lt / uint32_t(TX));
    const int lane = threadIdx.x;
    t.px = tx * GS_TILE + (lane & 15);
    t.py0 = ty * GS_TILE + (lane >> 4);
    t.fxp = float(t.px) + 0.5f;
    t.ymid0 = float(ty * GS_TILE) + 2.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        t.fyp[r] = float(t.py0 + 4 * r) + 0.5f;
        t.valid[r] = t.px < A.W[c] && (t.py0 + 4 * r) < A.H[c];
    }
    t.start = ranges[tile];
    t.end = ranges[n_tiles + tile];
    return t;
}

// Staged record: (mx, my, na, nb), (nc, o, r, g), (b), with the conic scaled
// so that the log2-domain exponent is na dx^2 + nb dx dy + nc dy^2.
// A raw render record held in registers while the previous batch is blended.
struct RawRec {
    float4 q0, q1;
    float q2;
    uint32_t j;
};

__device__ __forceinline__ void fetch_record(const float* rec, const uint32_t* vals, uint32_t base, uint32_t end,
                                             int lane, RawRec& R) {
    if (base + uint32_t(lane) < end) {
        R.j = vals[base + lane];
        const float4* p = reinterpret_cast<const float4*>(rec) + size_t(R.j) * 3;
        R.q0 = p[0];
        R.q1 = p[1];
        R.q2 = p[2].x;
    }
}

__device__ __forceinline__ float4 scaled_a(const RawRec& R) {
    return make_float4(R.q0.x, R.q0.y, -0.5f * kLog2e * R.q0.z, -kLog2e * R.q0.w);
}
__device__ __forceinline__ float4 scaled_b(const RawRec& R) {
    return make_float4(-0.5f * kLog2e * R.q1.x, R.q1.y, R.q1.z, R.q1.w);
}

// Reach of a record in y, plus half a strip: 1.5 + the largest |dy| at which
// o * exp(-Q/2) can still reach 1/255 (Q = a dx^2 + 2b dx dy + c dy^2, so
// |dy| <= sqrt(2 ln(255 o) a / (ac - b^2))), widened by 0.1% + 0.5 px against
// rounding.  A strip of four rows whose centre row is farther than this from
// the record's centre has no pixel with alpha >= 1/255, so it is skipped (the
// skip changes no result).  Degenerate conics are never skipped.
__device__ __forceinline__ float strip_reach(const RawRec& R) {
    const float a = R.q0.z, b = R.q0.w, c = R.q1.x, o = R.q1.y;
    const float det = a * c - b * b;
    if (!(det > 0.f) || !(a > 0.f)) return __builtin_inff();
    if (!(o * 255.f >= 0.999f)) return -1.f;  // o G < 1/255 everywhere (G <= 1)
    const float t = fmaxf(logf(255.f * o), 0.f);
    return sqrtf(2.f * t * a / det) * 1.001f + 0.5f + 1.5f;
}

// Strips of this tile (bit r: rows 4r..4r+3) that a record can reach,
// computed once per record when it is staged, so the blend loop tests a bit
// of a wavefront-uniform mask instead of comparing per strip.
__device__ __forceinline__ uint32_t strip_mask(const RawRec& R, float ymid0) {
    const float reach = strip_reach(R);
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) m |= (fabsf(R.q0.y - (ymid0 + 4.f * float(r))) > reach) ? 0u : (1u << r);
    return m;
}

// alpha of a staged record at one pixel; identical in forward and backward.
__device__ __forceinline__ float eval_alpha(float ebase, float eb, float nc, float o, float dy, float& G,
                                            bool& pass) {
    const float e2 = gauss_e2(ebase, eb, nc, dy);
    G = fast_exp2(e2);
    const float alpha = fminf(kAlphaMax, o * G);
    pass = (e2 <= 0.f) && (alpha >= kAlphaMin);
    return alpha;
}

struct FwdOut {
    float* rgb[GS_MAX_CAMS];
    float* T[GS_MAX_CAMS];
    uint32_t* last[GS_MAX_CAMS];
    float* chain;   // optional: [pairs][256] transmittance before each composited position
    uint8_t* live;  // optional: [pairs], 1 if some pixel of the tile composites the pair
    float bg[3];
};

// Slot of pixel (lane, row r) inside a tile's 256-float block of the chain.
__device__ __forceinline__ uint32_t chain_slot(int lane, int r) { return uint32_t(lane + 64 * r); }

// Eight wavefronts per SIMD (at most 64 VGPRs, no spills): 101.6 -> 94.6 us
// on the 1M city view against the seven the compiler picks by itself.
template <bool kChain>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_render_fwd(RenderCams A, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges, uint32_t n_tiles, FwdOut O) {
    __shared__ float4 sA[64];
    __shared__ float4 sB[64];
    __shared__ float2 sC[64];  // (b channel, strip mask bits)
    const TileCtx t = tile_ctx(A, ranges, n_tiles);
    const float* rec = A.rec[t.c];
    // thr: the smallest alpha a pixel still composites, 1/255 while it blends
    // and 2 (unreachable) once it has stopped or lies outside the image
    float T[4], thr[4], C0[4], C1[4], C2[4];
    uint32_t last[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        T[r] = 1.f; thr[r] = t.valid[r] ? kAlphaMin : 2.f; C0[r] = C1[r] = C2[r] = 0.f; last[r] = 0;
    }
    const int lane = threadIdx.x;
    RawRec R = {};
    fetch_record(rec, vals, t.start, t.end, lane, R);
    for (uint32_t b0 = t.start; b0 < t.end; b0 += 64) {
        if (__all(thr[0] > 1.f && thr[1] > 1.f && thr[2] > 1.f && thr[3] > 1.f)) break;
        const uint32_t nb = min(64u, t.end - b0);
        __syncthreads();
        if (uint32_t(lane) < nb) {
            sA[lane] = scaled_a(R); sB[lane] = scaled_b(R);
            sC[lane] = make_float2(R.q2, __uint_as_float(strip_mask(R, t.ymid0)));
        }
        __syncthreads();
        fetch_record(rec, vals, b0 + 64, t.end, lane, R);  // next batch in flight during the blend
        uint64_t lmask = 0;  // bit i: some pixel composites record b0 + i
        for (uint32_t i = 0; i < nb; ++i) {
            const float4 a = sA[i];
            const float4 b = sB[i];
            const float2 ce = sC[i];
            const float cb = ce.x;
            const uint32_t smask = __builtin_amdgcn_readfirstlane(__float_as_uint(ce.y));
            const float dx = a.x - t.fxp;
            const float ebase = a.z * dx * dx;
            const float eb = a.w * dx;
            const uint32_t pos = b0 - t.start + i + 1;
            bool any_comp = false;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!((smask >> r) & 1u)) continue;
                const float e2 = gauss_e2(ebase, eb, b.x, a.y - t.fyp[r]);
                const float alpha = fminf(kAlphaMax, b.y * fast_exp2(e2));
                // the same decisions as eval_alpha's, with a stopped pixel's
                // threshold out of reach
                const bool ok = (e2 <= 0.f) && (alpha >= thr[r]);
                const float Tn = T[r] * (1.f - alpha);
                const bool stop = ok && (Tn < kTMin);
                const bool comp = ok && !stop;
                const float wgt = comp ? alpha * T[r] : 0.f;
                if (kChain && comp) O.chain[size_t(b0 + i) * 256 + chain_slot(lane, r)] = T[r];
                C0[r] = fmaf(wgt, b.z, C0[r]);
                C1[r] = fmaf(wgt, b.w, C1[r]);
                C2[r] = fmaf(wgt, cb, C2[r]);
                T[r] = comp ? Tn : T[r];
                thr[r] = stop ? 2.f : thr[r];
                last[r] = comp ? pos : last[r];
                any_comp |= comp;
            }
            if (__any(any_comp)) lmask |= 1ull << i;
            if (__all(thr[0] > 1.f && thr[1] > 1.f && thr[2] > 1.f && thr[3] > 1.f)) break;
        }
        // records after an early stop stay 0: they lie beyond every pixel's last
        if (O.live && uint32_t(lane) < nb) O.live[b0 + lane] = uint8_t((lmask >> lane) & 1u);
    }
    const int W = A.W[t.c], H = A.H[t.c];
    const size_t plane = size_t(W) * H;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (!t.valid[r]) continue;
        const size_t p = size_t(t.py0 + 4 * r) * W + t.px;
        const float Tf = T[r];
        O.rgb[t.c][p] = fmaf(Tf, O.bg[0], C0[r]);
        O.rgb[t.c][plane + p] = fmaf(Tf, O.bg[1], C1[r]);
        O.rgb[t.c][2 * plane + p] = fmaf(Tf, O.bg[2], C2[r]);
        O.T[t.c][p] = Tf;
        O.last[t.c][p] = last[r];
    }
}

// ---------------------------------------------------------------------------
// Backward of the compositing
// ---------------------------------------------------------------------------
struct BwdImg {
    const float* T[GS_MAX_CAMS];
    const uint32_t* last[GS_MAX_CAMS];
    const float* grad[GS_MAX_CAMS];
    float* d2[GS_MAX_CAMS];  // [n_in][kD2Stride]
    const float* chain;      // optional stored transmittance chain
    const uint8_t* live;     // optional: the forward's per-pair "composited in the tile" flags
    int64_t n_in;
    float bg[3];
};

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, uint32_t(__shfl_xor(int(v), o, 64)));
    return v;
}

template <bool kChain>
__global__ __launch_bounds__(64) void k_render_bwd(RenderCams A, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges, uint32_t n_tiles, BwdImg I) {
    __shared__ float4 sA[64];
    __shared__ float4 sB[64];
    __shared__ float4 sR[64];  // (raw conic a, b, c, b channel)
    __shared__ uint32_t sJ[64];
    __shared__ float4 sRed[64][3];  // per lane: the nine partial sums of its group of 8
    const TileCtx t = tile_ctx(A, ranges, n_tiles);
    const float* rec = A.rec[t.c];
    const int W = A.W[t.c];
    const size_t plane = size_t(W) * A.H[t.c];
    // S = g . (colour behind the current position, divided by the
    // transmittance after it): the three running colour sums enter the
    // backward only through their dot product with the pixel's dL/dC
    float T[4], S[4], g0[4], g1[4], g2[4], gbg[4];
    uint32_t lst[4];
    uint32_t lmax = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const size_t p = size_t(t.py0 + 4 * r) * W + t.px;
        const bool v = t.valid[r];
        T[r] = v ? I.T[t.c][p] : 1.f;
        lst[r] = v ? I.last[t.c][p] : 0u;
        g0[r] = v ? I.grad[t.c][p] : 0.f;
        g1[r] = v ? I.grad[t.c][plane + p] : 0.f;
        g2[r] = v ? I.grad[t.c][2 * plane + p] : 0.f;
        gbg[r] = T[r] * (g0[r] * I.bg[0] + g1[r] * I.bg[1] + g2[r] * I.bg[2]);
        S[r] = 0.f;
        lmax = max(lmax, lst[r]);
    }
    lmax = wave_max_u32(lmax);
    const int lane = threadIdx.x;
    float* d2 = I.d2[t.c];
    const uint32_t stop_at = t.start + min(lmax, t.end - t.start);
    RawRec R = {};
    uint32_t lv = 1;  // live flag of this lane's prefetched record
    if (stop_at > t.start) {
        const uint32_t nb0 = min(64u, stop_at - t.start);
        fetch_record(rec, vals, stop_at - nb0, stop_at, lane, R);
        if (I.live && stop_at - nb0 + uint32_t(lane) < stop_at) lv = I.live[stop_at - nb0 + lane];
    }
    for (uint32_t b_end = stop_at; b_end > t.start;) {
        const uint32_t nb = min(64u, b_end - t.start);
        const uint32_t b0 = b_end - nb;
        __syncthreads();
        if (uint32_t(lane) < nb) {
            sA[lane] = scaled_a(R); sB[lane] = scaled_b(R);
            sR[lane] = make_float4(R.q0.z, R.q0.w, R.q1.x, R.q2);
            sJ[lane] = R.j;
        }
        // records that no pixel of the tile composites contribute nothing
        uint64_t todo = ballot(uint32_t(lane) < nb && lv != 0);
        __syncthreads();
        if (b0 > t.start) {  // the preceding batch, fetched during this one
            const uint32_t nbn = min(64u, b0 - t.start);
            fetch_record(rec, vals, b0 - nbn, b0, lane, R);
            if (I.live && b0 - nbn + uint32_t(lane) < b0) lv = I.live[b0 - nbn + lane];
        }
        while (todo) {  // back to front over the live records
            const int i = 63 - __builtin_clzll(todo);
            todo &= ~(1ull << i);
            const float4 a = sA[i];
            const float4 b = sB[i];
            const float4 rw = sR[i];
            const uint32_t pos = b0 - t.start + uint32_t(i);  // 0-based list position
            const float dx = a.x - t.fxp;
            const float ebase = a.z * dx * dx;
            const float eb = a.w * dx;
            const float o = b.y;
            // the four rows' alphas first (four independent exponentials in
            // flight); a record that no pixel of the tile composites is done
            float alv[4], Gv[4];
            bool okv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                bool pass;
                alv[r] = eval_alpha(ebase, eb, b.x, o, a.y - t.fyp[r], Gv[r], pass);
                okv[r] = pass && (pos < lst[r]);
            }
            if (__any(okv[0] || okv[1] || okv[2] || okv[3])) {
                // per lane, over its composited rows: u = dL/dalpha * G (the
                // opacity partial), and the moments sum(u dy), sum(u dy^2); the
                // mean and conic partials are linear in them and are formed
                // once per record
                float s_op = 0.f, q1 = 0.f, q2 = 0.f, s_r = 0.f, s_g = 0.f, s_b = 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (!okv[r]) continue;
                    const float dy = a.y - t.fyp[r];
                    const float alpha = alv[r];
                    const float G = Gv[r];
                    const float om = 1.f - alpha;
                    const float rom = fast_rcp(om);
                    float Tk = T[r] * rom;
                    if (kChain) Tk = I.chain[size_t(b0 + uint32_t(i)) * 256 + chain_slot(lane, r)];
                    const float gc = fmaf(g2[r], rw.w, fmaf(g1[r], b.w, g0[r] * b.z));
                    const float dLda = fmaf(Tk, gc - S[r], -gbg[r] * rom);
                    S[r] = fmaf(alpha, gc, om * S[r]);
                    T[r] = Tk;
                    const float aT = alpha * Tk;
                    s_r = fmaf(g0[r], aT, s_r);
                    s_g = fmaf(g1[r], aT, s_g);
                    s_b = fmaf(g2[r], aT, s_b);
                    // a clamped alpha (o G > 0.99) passes no gradient to o or G;
                    // a select instead of a branch (the clamp is rare)
                    const float u = (o * G <= kAlphaMax) ? dLda * G : 0.f;
                    s_op += u;
                    const float uy = u * dy;
                    q1 += uy;
                    q2 = fmaf(uy, dy, q2);
                }
                // dL/dG = o dL/dalpha; dG/dmean = -G (a dx + b dy, b dx + c dy),
                // dG/d(a, b, c) = -G (dx^2 / 2, dx dy, dy^2 / 2)
                const float k = o * s_op;
                const float kx = k * dx;
                const float qy = o * q1;
                float s_mx = -fmaf(rw.x, kx, rw.y * qy);
                float s_my = -fmaf(rw.y, kx, rw.z * qy);
                float s_ca = -0.5f * kx * dx;
                float s_cb = -dx * qy;
                float s_cc = -0.5f * o * q2;
                // groups of 8 lanes reduce with three DPP steps; the eight group
                // sums of each partial meet in LDS, and lanes 0..8 each add one
                // partial (a single atomic instruction for the nine)
                float red[9] = {s_mx, s_my, s_ca, s_cb, s_cc, s_op, s_r, s_g, s_b};
                oct_sum8_n<9>(red);
                // every lane stores (keeps the DPP adds fused); lanes 7, 15, ..
                // hold the group sums
                sRed[lane][0] = make_float4(red[0], red[1], red[2], red[3]);
                sRed[lane][1] = make_float4(red[4], red[5], red[6], red[7]);
                sRed[lane][2].x = red[8];
                __builtin_amdgcn_wave_barrier();
                if (lane < 9) {
                    const float* rr = reinterpret_cast<const float*>(&sRed[7][0]) + lane;  // lane 8g+7: rr[96 g]
                    const float v = ((rr[0] + rr[96]) + (rr[192] + rr[288])) +
                                    ((rr[384] + rr[480]) + (rr[576] + rr[672]));
                    atomicAdd(d2 + int64_t(sJ[i]) * kD2Stride + lane, v);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        b_end = b0;
    }
}

// ---------------------------------------------------------------------------
// Importance: colour-less blend, w_j += alpha T and a_j += 1 per composited
// (pixel, Gaussian), reduced per (Gaussian, tile) across the wavefront.
// ---------------------------------------------------------------------------
// w and the composited count of Gaussian j accumulate in one 8-byte record
// wa[2j], wa[2j+1] (the count as a float, exact below 2^24), so that one
// atomic instruction of two lanes updates both.
// FOOTPRINT: the count is every pixel (inside the image) whose kernel value
// passes the 1/255 test, composited or not, so the loop runs over the whole
// list instead of ending when every pixel has stopped.
template <bool FOOTPRINT>
__global__ __launch_bounds__(64) void k_importance_blend(RenderCams A, const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ ranges, uint32_t n_tiles,
                                                         float* __restrict__ wa) {
    __shared__ float4 sA[64];
    __shared__ float4 sB[64];  // (nc, o, strip mask bits, -)
    __shared__ uint32_t sJ[64];
    __shared__ float2 sRed[64];
    const TileCtx t = tile_ctx(A, ranges, n_tiles);
    const float* rec = A.rec[t.c];
    float T[4], thr[4];  // thr as in the forward: 2 once the pixel has stopped (or lies outside)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        T[r] = 1.f;
        thr[r] = t.valid[r] ? kAlphaMin : 2.f;
    }
    const int lane = threadIdx.x;
    RawRec R = {};
    fetch_record(rec, vals, t.start, t.end, lane, R);
    float cthr[4];  // footprint count: 1/255 inside the image
#pragma unroll
    for (int r = 0; r < 4; ++r) cthr[r] = t.valid[r] ? kAlphaMin : 2.f;
    for (uint32_t b0 = t.start; b0 < t.end; b0 += 64) {
        if (!FOOTPRINT && __all(thr[0] > 1.f && thr[1] > 1.f && thr[2] > 1.f && thr[3] > 1.f)) break;
        const uint32_t nb = min(64u, t.end - b0);
        __syncthreads();
        if (uint32_t(lane) < nb) {
            const float4 b = scaled_b(R);
            sA[lane] = scaled_a(R);
            sB[lane] = make_float4(b.x, b.y, __uint_as_float(strip_mask(R, t.ymid0)), 0.f);
            sJ[lane] = R.j;
        }
        __syncthreads();
        fetch_record(rec, vals, b0 + 64, t.end, lane, R);
        for (uint32_t i = 0; i < nb; ++i) {
            const float4 a = sA[i];
            const float4 b = sB[i];
            const uint32_t smask = __builtin_amdgcn_readfirstlane(__float_as_uint(b.z));
            const float dx = a.x - t.fxp;
            const float ebase = a.z * dx * dx;
            const float eb = a.w * dx;
            float sw = 0.f, sn = 0.f;  // the count as a float (exact, at most 4)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!((smask >> r) & 1u)) continue;
                const float e2 = gauss_e2(ebase, eb, b.x, a.y - t.fyp[r]);
                const float alpha = fminf(kAlphaMax, b.y * fast_exp2(e2));
                const bool ok = (e2 <= 0.f) && (alpha >= thr[r]);
                const float Tn = T[r] * (1.f - alpha);
                const bool stop = ok && (Tn < kTMin);
                const bool comp = ok && !stop;
                sw += comp ? alpha * T[r] : 0.f;
                if (FOOTPRINT)
                    sn += ((e2 <= 0.f) && (alpha >= cthr[r])) ? 1.f : 0.f;
                else
                    sn += comp ? 1.f : 0.f;
                T[r] = comp ? Tn : T[r];
                thr[r] = stop ? 2.f : thr[r];
            }
            if (__any(sn > 0.f)) {
                // groups of 8 lanes reduce with DPP; lanes 0 and 1 add the
                // eight group sums of w and of the count and issue one atomic
                float red[2] = {sw, sn};
                oct_sum8_n<2>(red);
                sRed[lane] = make_float2(red[0], red[1]);
                __builtin_amdgcn_wave_barrier();
                if (lane < 2) {
                    const float* rr = reinterpret_cast<const float*>(&sRed[7]) + lane;  // lane 8g+7: rr[16 g]
                    const float v = ((rr[0] + rr[16]) + (rr[32] + rr[48])) + ((rr[64] + rr[80]) + (rr[96] + rr[112]));
                    atomicAdd(wa + 2 * int64_t(sJ[i]) + lane, v);
                }
                __builtin_amdgcn_wave_barrier();
            }
            if (!FOOTPRINT && __all(thr[0] > 1.f && thr[1] > 1.f && thr[2] > 1.f && thr[3] > 1.f)) break;
        }
    }
}

int fill_render_cams(const gs_projected* proj, const gs_camera* cams, int n_cams, RenderCams& A,
                     int64_t* total_tiles) {
    int rc = validate_cams(cams, n_cams, GS_MAX_CAMS, total_tiles);
    if (rc) return rc;
    memset(&A, 0, sizeof(A));
    A.n_cams = n_cams;
    uint32_t off = 0;
    for (int c = 0; c < n_cams; ++c) {
        if (!proj[c].rec || !aligned(proj[c].rec, 16))
            return fail(GS_ERR_INVALID_ARG, "camera %d: null or misaligned render record", c);
        A.rec[c] = proj[c].rec;
        A.tile_off[c] = off;
        A.TX[c] = int32_t(tiles_x(cams[c].width));
        A.W[c] = cams[c].width;
        A.H[c] = cams[c].height;
        off += uint32_t(gs_num_tiles(cams[c].width, cams[c].height));
    }
    A.tile_off[n_cams] = off;
    return GS_OK;
}

int launch_importance_blend(const gs_projected* proj, const gs_camera* cam, const uint32_t* vals,
                            const uint32_t* ranges, float* wa, int footprint, hipStream_t stream) {
    RenderCams A;
    int64_t tt = 0;
    int rc = fill_render_cams(proj, cam, 1, A, &tt);
    if (rc) return rc;
    if (tt == 0) return GS_OK;
    if (footprint)
        launch("importance_blend", k_importance_blend<true>, dim3(unsigned(tt)), dim3(64), 0, stream, A, vals,
               ranges, uint32_t(tt), wa);
    else
        launch("importance_blend", k_importance_blend<false>, dim3(unsigned(tt)), dim3(64), 0, stream, A, vals,
               ranges, uint32_t(tt), wa);
    return check_launch("importance blend");
}

int launch_visible_list(int64_t n_in, const int64_t* n_in_dev, int n_cams, float* const* d2, const gs_projected* proj,
                        uint32_t* list, uint32_t* count, hipStream_t stream);
int launch_export_d2(const float* d2, int64_t n_in, const uint32_t* list, const uint32_t* count,
                     const int32_t* radius, float* out, hipStream_t stream);
int launch_project_bwd(const gs_scene* scene, const int32_t* active_idx, int64_t n_in, const gs_camera* cams,
                       int n_cams, float* const* d2, const gs_projected* proj, const gs_grads* grads,
                       const uint32_t* list, const uint32_t* count, hipStream_t stream);
int check_scene(const gs_scene* s);

}  // namespace gsmi

using namespace gsmi;

size_t ws_render_bwd(int64_t n, int n_cams) {
    Carve cv(nullptr);
    cv.take<float>(size_t(kD2Stride) * size_t(n > 0 ? n : 1) * size_t(n_cams));
    cv.take<uint32_t>(size_t(n > 0 ? n : 1));
    cv.take<uint32_t>(4);
    return cv.used();
}

extern "C" int gs_render_fwd(const gs_projected* proj, const gs_camera* cams, int n_cams, const uint32_t* vals,
                             const uint32_t* tile_ranges, const float* bg, float* const* out_rgb,
                             float* const* out_T, uint32_t* const* out_last, float* chain, uint8_t* pair_live,
                             hipStream_t stream) {
    if (!proj || !tile_ranges || !bg || !out_rgb || !out_T || !out_last)
        return fail(GS_ERR_INVALID_ARG, "gs_render_fwd: null argument");
    RenderCams A;
    int64_t tt = 0;
    int rc = fill_render_cams(proj, cams, n_cams, A, &tt);
    if (rc) return rc;
    FwdOut O;
    memset(&O, 0, sizeof(O));
    for (int c = 0; c < n_cams; ++c) {
        if (!out_rgb[c] || !out_T[c] || !out_last[c]) return fail(GS_ERR_INVALID_ARG, "gs_render_fwd: null image");
        O.rgb[c] = out_rgb[c]; O.T[c] = out_T[c]; O.last[c] = out_last[c];
    }
    O.bg[0] = bg[0]; O.bg[1] = bg[1]; O.bg[2] = bg[2];
    O.chain = chain;
    O.live = pair_live;
    if (tt == 0) return GS_OK;
    if (O.chain)
        launch("render_fwd", k_render_fwd<true>, dim3(unsigned(tt)), dim3(64), 0, stream, A, vals, tile_ranges,
               uint32_t(tt), O);
    else
        launch("render_fwd", k_render_fwd<false>, dim3(unsigned(tt)), dim3(64), 0, stream, A, vals, tile_ranges,
               uint32_t(tt), O);
    return check_launch("gs_render_fwd");
}

extern "C" int gs_render_bwd(const gs_scene* scene, const int32_t* active_idx, int64_t n_in, const int64_t* n_in_dev,
                             const gs_projected* proj, const gs_camera* cams, int n_cams, const uint32_t* vals,
                             const uint32_t* tile_ranges, const float* bg, float* const* out_T,
                             uint32_t* const* out_last, float* const* grad_rgb, const float* chain,
                             const uint8_t* pair_live, gs_grads* grads,
                             float* grads2d, void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc = check_scene(scene);
    if (rc) return rc;
    if (!proj || !tile_ranges || !bg || !out_T || !out_last || !grad_rgb || !grads)
        return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: null argument");
    if (!grads->mean || !grads->log_scale || !grads->quat || !grads->opacity_logit || !grads->sh)
        return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: null gradient array");
    if (n_in < 0 || n_in >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: n_in out of range");
    if (!active_idx && n_in > scene->n) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: n_in > n without active_idx");
    RenderCams A;
    int64_t tt = 0;
    rc = fill_render_cams(proj, cams, n_cams, A, &tt);
    if (rc) return rc;
    const size_t need = ws_render_bwd(n_in, n_cams);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_render_bwd: workspace needs %zu bytes (256-aligned)", need);
    BwdImg I;
    memset(&I, 0, sizeof(I));
    Carve cv(ws);
    float* base = cv.take<float>(size_t(kD2Stride) * size_t(n_in > 0 ? n_in : 1) * size_t(n_cams));
    uint32_t* vis_list = cv.take<uint32_t>(size_t(n_in > 0 ? n_in : 1));
    uint32_t* vis_count = cv.take<uint32_t>(4);
    for (int c = 0; c < n_cams; ++c) {
        if (!out_T[c] || !out_last[c] || !grad_rgb[c]) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: null image");
        I.T[c] = out_T[c]; I.last[c] = out_last[c]; I.grad[c] = grad_rgb[c];
        I.d2[c] = base + size_t(kD2Stride) * size_t(n_in) * c;
    }
    // visible entries first: the list clears their partial records
    if ((rc = launch_visible_list(n_in, n_in_dev, n_cams, I.d2, proj, vis_list, vis_count, stream))) return rc;
    I.n_in = n_in;
    I.chain = chain;
    I.live = pair_live;
    I.bg[0] = bg[0]; I.bg[1] = bg[1]; I.bg[2] = bg[2];
    if (tt > 0 && n_in > 0)
    {
        if (chain)
            launch("render_bwd", k_render_bwd<true>, dim3(unsigned(tt)), dim3(64), 0, stream, A, vals, tile_ranges,
                   uint32_t(tt), I);
        else
            launch("render_bwd", k_render_bwd<false>, dim3(unsigned(tt)), dim3(64), 0, stream, A, vals, tile_ranges,
                   uint32_t(tt), I);
    }
    if ((rc = check_launch("gs_render_bwd blend"))) return rc;
    if (grads2d && (rc = launch_export_d2(I.d2[0], n_in, vis_list, vis_count, proj[0].radius, grads2d, stream)))
        return rc;
    return launch_project_bwd(scene, active_idx, n_in, cams, n_cams, I.d2, proj, grads, vis_list, vis_count, stream);
}
