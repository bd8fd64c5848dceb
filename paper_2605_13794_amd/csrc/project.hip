// Per-Gaussian projection (EWA splatting + SH degree-3 colour) and its
// backward.  One thread per input entry; parameters are read as coalesced
// component-major (SoA) loads, the scene once for all cameras of a batch.
#include "common.h"

namespace gsmi {

struct SceneP {
    const float* mean;
    const float* log_scale;
    const float* quat;
    const float* opacity_logit;
    const float* sh;
    int64_t n;
};

struct CamSet {
    DevCam cam[GS_MAX_CAMS];
    int n;
};

struct ProjOut {
    float* rec[GS_MAX_CAMS];
    float* depth[GS_MAX_CAMS];
    int32_t* radius[GS_MAX_CAMS];
    uint32_t* tiles[GS_MAX_CAMS];
    uint8_t* clamp[GS_MAX_CAMS];
    float* mean2d[GS_MAX_CAMS];
    float* conic[GS_MAX_CAMS];
    float* opacity[GS_MAX_CAMS];
    float* rgb[GS_MAX_CAMS];
};

// Real SH of degree 3 (Condon-Shortley phase, index l*l + l + m) at a unit
// direction, as the closed-form polynomials of x, y, z.
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC20 = 1.0925484305920792f, kC21 = -1.0925484305920792f, kC22 = 0.31539156525252005f,
                kC23 = -1.0925484305920792f, kC24 = 0.5462742152960396f;
constexpr float kC30 = -0.5900435899266435f, kC31 = 2.890611442640554f, kC32 = -0.4570457994644658f,
                kC33 = 0.3731763325901154f, kC34 = -0.4570457994644658f, kC35 = 1.445305721320277f,
                kC36 = -0.5900435899266435f;

__device__ __forceinline__ void sh_basis(float x, float y, float z, float Y[16]) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = kC0;
    Y[1] = -kC1 * y;
    Y[2] = kC1 * z;
    Y[3] = -kC1 * x;
    Y[4] = kC20 * x * y;
    Y[5] = kC21 * y * z;
    Y[6] = kC22 * (2.f * zz - xx - yy);
    Y[7] = kC23 * x * z;
    Y[8] = kC24 * (xx - yy);
    Y[9] = kC30 * y * (3.f * xx - yy);
    Y[10] = kC31 * x * y * z;
    Y[11] = kC32 * y * (4.f * zz - xx - yy);
    Y[12] = kC33 * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = kC34 * x * (4.f * zz - xx - yy);
    Y[14] = kC35 * z * (xx - yy);
    Y[15] = kC36 * x * (xx - 3.f * yy);
}

// Gradient of sum_k w[k] Y_k(x, y, z) with respect to (x, y, z), treating the
// polynomials above as functions of three free variables.
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float w[16], float g[3]) {
    const float xx = x * x, yy = y * y, zz = z * z;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    gy += w[1] * -kC1;
    gz += w[2] * kC1;
    gx += w[3] * -kC1;
    gx += w[4] * kC20 * y;                gy += w[4] * kC20 * x;
    gy += w[5] * kC21 * z;                gz += w[5] * kC21 * y;
    gx += w[6] * kC22 * -2.f * x;         gy += w[6] * kC22 * -2.f * y;   gz += w[6] * kC22 * 4.f * z;
    gx += w[7] * kC23 * z;                gz += w[7] * kC23 * x;
    gx += w[8] * kC24 * 2.f * x;          gy += w[8] * kC24 * -2.f * y;
    gx += w[9] * kC30 * 6.f * x * y;      gy += w[9] * kC30 * (3.f * xx - 3.f * yy);
    gx += w[10] * kC31 * y * z;           gy += w[10] * kC31 * x * z;     gz += w[10] * kC31 * x * y;
    gx += w[11] * kC32 * -2.f * x * y;    gy += w[11] * kC32 * (4.f * zz - xx - 3.f * yy);
    gz += w[11] * kC32 * 8.f * y * z;
    gx += w[12] * kC33 * -6.f * x * z;    gy += w[12] * kC33 * -6.f * y * z;
    gz += w[12] * kC33 * (6.f * zz - 3.f * xx - 3.f * yy);
    gx += w[13] * kC34 * (4.f * zz - 3.f * xx - yy);
    gy += w[13] * kC34 * -2.f * x * y;    gz += w[13] * kC34 * 8.f * x * z;
    gx += w[14] * kC35 * 2.f * x * z;     gy += w[14] * kC35 * -2.f * y * z; gz += w[14] * kC35 * (xx - yy);
    gx += w[15] * kC36 * (3.f * xx - 3.f * yy);
    gy += w[15] * kC36 * -6.f * x * y;
    g[0] = gx; g[1] = gy; g[2] = gz;
}

__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float R[9]) {
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

// Shared forward geometry of one Gaussian in one camera.
struct Geo {
    float tx, ty, tz, rz, txtz, tytz, ux, uy;
    float T0[3], T1[3];  // T = J W
    float U0[3], U1[3];  // U = T Sigma
    float a, b, c, det;
};

__device__ __forceinline__ void geo_camera(const DevCam& C, const float mu[3], Geo& g) {
    g.tx = fmaf(C.R[0], mu[0], fmaf(C.R[1], mu[1], fmaf(C.R[2], mu[2], C.t[0])));
    g.ty = fmaf(C.R[3], mu[0], fmaf(C.R[4], mu[1], fmaf(C.R[5], mu[2], C.t[1])));
    g.tz = fmaf(C.R[6], mu[0], fmaf(C.R[7], mu[1], fmaf(C.R[8], mu[2], C.t[2])));
}

__device__ __forceinline__ void geo_cov(const DevCam& C, const float S[6], Geo& g) {
    // S = (s00, s01, s02, s11, s12, s22)
    g.rz = 1.f / g.tz;
    g.txtz = g.tx * g.rz;
    g.tytz = g.ty * g.rz;
    g.ux = fminf(fmaxf(g.txtz, -C.limx), C.limx);
    g.uy = fminf(fmaxf(g.tytz, -C.limy), C.limy);
    const float J00 = C.fx * g.rz, J02 = -C.fx * g.ux * g.rz;
    const float J11 = C.fy * g.rz, J12 = -C.fy * g.uy * g.rz;
    for (int k = 0; k < 3; ++k) {
        g.T0[k] = fmaf(J00, C.R[k], J02 * C.R[6 + k]);
        g.T1[k] = fmaf(J11, C.R[3 + k], J12 * C.R[6 + k]);
    }
    const float s00 = S[0], s01 = S[1], s02 = S[2], s11 = S[3], s12 = S[4], s22 = S[5];
    g.U0[0] = g.T0[0] * s00 + g.T0[1] * s01 + g.T0[2] * s02;
    g.U0[1] = g.T0[0] * s01 + g.T0[1] * s11 + g.T0[2] * s12;
    g.U0[2] = g.T0[0] * s02 + g.T0[1] * s12 + g.T0[2] * s22;
    g.U1[0] = g.T1[0] * s00 + g.T1[1] * s01 + g.T1[2] * s02;
    g.U1[1] = g.T1[0] * s01 + g.T1[1] * s11 + g.T1[2] * s12;
    g.U1[2] = g.T1[0] * s02 + g.T1[1] * s12 + g.T1[2] * s22;
    g.a = g.U0[0] * g.T0[0] + g.U0[1] * g.T0[1] + g.U0[2] * g.T0[2] + kDilation;
    g.b = g.U0[0] * g.T1[0] + g.U0[1] * g.T1[1] + g.U0[2] * g.T1[2];
    g.c = g.U1[0] * g.T1[0] + g.U1[1] * g.T1[1] + g.U1[2] * g.T1[2] + kDilation;
    g.det = g.a * g.c - g.b * g.b;
}

__device__ __forceinline__ void covariance(const float ls[3], const float q[4], float s[3], float qn[4],
                                           float R[9], float M[9], float S[6], float& qlen) {
    s[0] = __expf(ls[0]); s[1] = __expf(ls[1]); s[2] = __expf(ls[2]);
    qlen = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float inv = 1.f / qlen;
    for (int k = 0; k < 4; ++k) qn[k] = q[k] * inv;
    quat_rot(qn[0], qn[1], qn[2], qn[3], R);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[r * 3 + c] = R[r * 3 + c] * s[c];
    S[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    S[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    S[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    S[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    S[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    S[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
}

__device__ __forceinline__ int64_t floordiv16(int64_t a) { return a >= 0 ? a / 16 : -((-a + 15) / 16); }

__device__ __forceinline__ void culled_out(const ProjOut& O, int c, int64_t j, int64_t n) {
    O.depth[c][j] = 0.f;
    O.radius[c][j] = 0;
    O.tiles[c][j] = 0u;
    O.clamp[c][j] = 0;
    if (O.mean2d[c]) { O.mean2d[c][j] = 0.f; O.mean2d[c][n + j] = 0.f; }
    if (O.conic[c]) { O.conic[c][j] = 0.f; O.conic[c][n + j] = 0.f; O.conic[c][2 * n + j] = 0.f; }
    if (O.opacity[c]) O.opacity[c][j] = 0.f;
    if (O.rgb[c]) { O.rgb[c][j] = 0.f; O.rgb[c][n + j] = 0.f; O.rgb[c][2 * n + j] = 0.f; }
}

// Conservative pre-cull per camera: the largest eigenvalue of the screen
// covariance is at most s_max^2 |J|_F^2 + 0.3 (the camera rotation is
// orthonormal), so a centre farther off-screen than that 3-sigma bound
// (+1 px for the ceiling and rounding) has an empty tile rectangle.
// Returns the cameras in which the Gaussian may be visible.
__device__ __forceinline__ uint32_t maybe_visible(const CamSet& C, const float mu[3], const float ls[3]) {
    const float smax2 = __expf(2.f * fmaxf(fmaxf(ls[0], ls[1]), ls[2]));
    uint32_t maybe = 0;
    for (int c = 0; c < C.n; ++c) {
        const DevCam& K = C.cam[c];
        Geo G0;
        geo_camera(K, mu, G0);
        if (!(G0.tz > K.znear)) continue;
        const float rz = 1.f / G0.tz;
        const float ux = fminf(fmaxf(G0.tx * rz, -K.limx), K.limx);
        const float uy = fminf(fmaxf(G0.ty * rz, -K.limy), K.limy);
        const float F = (K.fx * rz) * (K.fx * rz) * (1.f + ux * ux) + (K.fy * rz) * (K.fy * rz) * (1.f + uy * uy);
        const float rb = 3.f * sqrtf(smax2 * F + kDilation) * 1.001f + 2.f;
        const float mx = fmaf(K.fx, G0.tx * rz, K.cx), my = fmaf(K.fy, G0.ty * rz, K.cy);
        const bool off = (mx + rb < -1.f) || (mx - rb > float(K.TX * GS_TILE) + 1.f) || (my + rb < -1.f) ||
                         (my - rb > float(K.TY * GS_TILE) + 1.f);
        if (!off) maybe |= 1u << c;
    }
    return maybe;
}

// Pass 1 (low register count): entries that cannot be visible in any camera
// get their culled outputs; the others are appended to `list` (one atomic per
// workgroup of kChunk entries).
//
// Chunk sizes of the list-building kernels: small inputs use 512 entries per
// workgroup (more workgroups in flight: 15 -> 10 us for the cull and 17 -> 7 us
// for the visible list on a 0.6M-entry view); the visible list of a large
// input uses 4,096 so that the single counter sees at most a few thousand
// atomics (a large projection takes the single pass and builds no list).
constexpr int64_t kSmallListInput = 2 << 20;
constexpr int kChunkSmall = 512;
constexpr int kVisChunkLarge = 4096;

template <int kChunk>
__global__ __launch_bounds__(256) void k_project_cull(SceneP P, const int32_t* __restrict__ active, int64_t n_in,
                                                      const int64_t* __restrict__ n_in_dev, CamSet C, ProjOut O,
                                                      uint32_t* __restrict__ list, uint32_t* __restrict__ count) {
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t base_s;
    int64_t cnt = n_in;
    if (n_in_dev) cnt = min(cnt, *n_in_dev);
    const int64_t j0 = int64_t(blockIdx.x) * kChunk;
    const int w = threadIdx.x / 64;
    const int64_t N = P.n;
    constexpr int kIt = kChunk / 256;
    uint32_t keep_bits = 0;  // per iteration: this thread's entry is a candidate
    uint32_t mine = 0;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t j = j0 + it * 256 + threadIdx.x;
        bool cand = false;
        if (j < n_in) {
            int64_t i = j;
            if (active) i = j < cnt ? int64_t(active[j]) : -1;
            if (j < cnt && i >= 0 && i < N) {
                const float mu[3] = {P.mean[i], P.mean[N + i], P.mean[2 * N + i]};
                const float ls[3] = {P.log_scale[i], P.log_scale[N + i], P.log_scale[2 * N + i]};
                cand = maybe_visible(C, mu, ls) != 0;
            }
            if (!cand)
                for (int c = 0; c < C.n; ++c) culled_out(O, c, j, n_in);
        }
        keep_bits |= uint32_t(cand) << it;
        mine += popc64(ballot(cand));
    }
    if (lane_id() == 0) wsum[w] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base_s = tot ? atomicAdd(count, tot) : 0u;
    }
    __syncthreads();
    uint32_t off = base_s;
    for (int k = 0; k < w; ++k) off += wsum[k];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const bool cand = (keep_bits >> it) & 1u;
        const uint64_t m = ballot(cand);
        if (cand) list[off + popc64(m & lanemask_lt())] = uint32_t(j0 + it * 256 + threadIdx.x);
        off += popc64(m);
    }
}

// Full projection of entry j (Gaussian i) into every camera in which the
// conservative test left it possibly visible.
__device__ __forceinline__ void project_entry(const SceneP& P, int64_t i, int64_t j, int64_t n_in, const CamSet& C,
                                              const ProjOut& O, const float mu[3], const float ls[3],
                                              uint32_t maybe) {
    const int64_t N = P.n;
    const float q[4] = {P.quat[i], P.quat[N + i], P.quat[2 * N + i], P.quat[3 * N + i]};
    float s[3], qn[4], R[9], M[9], S[6], qlen;
    covariance(ls, q, s, qn, R, M, S, qlen);
    const float opa = 1.f / (1.f + __expf(-P.opacity_logit[i]));
    for (int c = 0; c < C.n; ++c) {
        const DevCam& K = C.cam[c];
        Geo G;
        geo_camera(K, mu, G);
        if (!((maybe >> c) & 1u) || !(G.tz > K.znear)) { culled_out(O, c, j, n_in); continue; }
        geo_cov(K, S, G);
        if (!(G.det > 0.f)) { culled_out(O, c, j, n_in); continue; }
        const float idet = 1.f / G.det;
        const float ca = G.c * idet, cb = -G.b * idet, cc = G.a * idet;
        const float mx = fmaf(K.fx, G.txtz, K.cx), my = fmaf(K.fy, G.tytz, K.cy);
        const float mid = 0.5f * (G.a + G.c);
        const float lam = mid + sqrtf(fmaxf(0.f, mid * mid - G.det));
        const float rf = fminf(ceilf(3.f * sqrtf(lam)), 1073741824.f);
        const int64_t r = int64_t(rf);
        const int64_t xi = int64_t(floorf(fminf(fmaxf(mx, -1073741824.f), 1073741824.f)));
        const int64_t yi = int64_t(floorf(fminf(fmaxf(my, -1073741824.f), 1073741824.f)));
        const int64_t x0 = min<int64_t>(max<int64_t>(floordiv16(xi - r), 0), K.TX);
        const int64_t x1 = min<int64_t>(max<int64_t>(floordiv16(xi + r) + 1, 0), K.TX);
        const int64_t y0 = min<int64_t>(max<int64_t>(floordiv16(yi - r), 0), K.TY);
        const int64_t y1 = min<int64_t>(max<int64_t>(floordiv16(yi + r) + 1, 0), K.TY);
        const int64_t touched = (x1 - x0) * (y1 - y0);
        if (touched <= 0 || !(rf > 0.f)) { culled_out(O, c, j, n_in); continue; }
        float vx = mu[0] - K.campos[0], vy = mu[1] - K.campos[1], vz = mu[2] - K.campos[2];
        const float il = 1.f / sqrtf(vx * vx + vy * vy + vz * vz);
        float Y[16];
        sh_basis(vx * il, vy * il, vz * il, Y);
        // the 48 coefficients are read four SH functions (12 loads) at a time
        // rather than all at once: fewer registers, more wavefronts
        float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) acc[ch] = fmaf(P.sh[int64_t(k * 3 + ch) * N + i], Y[k], acc[ch]);
            if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        float rgb[3];
        uint8_t cbits = 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float a = acc[ch] + 0.5f;
            if (a < 0.f) { cbits |= uint8_t(1u << ch); a = 0.f; }
            rgb[ch] = a;
        }
        float4* rp = reinterpret_cast<float4*>(O.rec[c] + j * kRec);
        rp[0] = make_float4(mx, my, ca, cb);
        rp[1] = make_float4(cc, opa, rgb[0], rgb[1]);
        rp[2] = make_float4(rgb[2], G.tz, 0.f, 0.f);
        O.depth[c][j] = G.tz;
        O.radius[c][j] = int32_t(r);
        O.tiles[c][j] = uint32_t(touched);
        O.clamp[c][j] = cbits;
        if (O.mean2d[c]) { O.mean2d[c][j] = mx; O.mean2d[c][n_in + j] = my; }
        if (O.conic[c]) { O.conic[c][j] = ca; O.conic[c][n_in + j] = cb; O.conic[c][2 * n_in + j] = cc; }
        if (O.opacity[c]) O.opacity[c][j] = opa;
        if (O.rgb[c]) { O.rgb[c][j] = rgb[0]; O.rgb[c][n_in + j] = rgb[1]; O.rgb[c][2 * n_in + j] = rgb[2]; }
    }
}

// Pass 2: full projection of the candidates.
__global__ __launch_bounds__(256) void k_project(SceneP P, const int32_t* __restrict__ active, int64_t n_in,
                                                 const uint32_t* __restrict__ list,
                                                 const uint32_t* __restrict__ count, CamSet C, ProjOut O) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= *count) return;
    const int64_t j = list[t];
    const int64_t i = active ? int64_t(active[j]) : j;
    const int64_t N = P.n;
    const float mu[3] = {P.mean[i], P.mean[N + i], P.mean[2 * N + i]};
    const float ls[3] = {P.log_scale[i], P.log_scale[N + i], P.log_scale[2 * N + i]};
    project_entry(P, i, j, n_in, C, O, mu, ls, maybe_visible(C, mu, ls));
}

// Single pass for large inputs: one thread per input entry, culled entries
// leave at once.  With the Gaussians in spatial (Morton) order, visibility is
// coherent along the entries, so wavefronts are mostly all-culled or
// all-visible; the candidate list and the second read of the means and
// scales of the two-pass form are saved.
__global__ __launch_bounds__(256) void k_project_all(SceneP P, const int32_t* __restrict__ active, int64_t n_in,
                                                     const int64_t* __restrict__ n_in_dev, CamSet C, ProjOut O) {
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (j >= n_in) return;
    int64_t cnt = n_in;
    if (n_in_dev) cnt = min(cnt, *n_in_dev);
    int64_t i = j;
    if (active) i = j < cnt ? int64_t(active[j]) : -1;
    const int64_t N = P.n;
    if (j >= cnt || i < 0 || i >= N) {
        for (int c = 0; c < C.n; ++c) culled_out(O, c, j, n_in);
        return;
    }
    const float mu[3] = {P.mean[i], P.mean[N + i], P.mean[2 * N + i]};
    const float ls[3] = {P.log_scale[i], P.log_scale[N + i], P.log_scale[2 * N + i]};
    const uint32_t maybe = maybe_visible(C, mu, ls);
    if (!maybe) {
        for (int c = 0; c < C.n; ++c) culled_out(O, c, j, n_in);
        return;
    }
    project_entry(P, i, j, n_in, C, O, mu, ls, maybe);
}

// ---------------------------------------------------------------------------
// Backward: screen-space partials d2 = (d mean2d x, y, d conic a, b, c,
// d opacity, d rgb r, g, b) of every camera -> parameter gradients.
// ---------------------------------------------------------------------------
struct BwdIn {
    float* d2[GS_MAX_CAMS];             // [n_in][kD2Stride]
    const int32_t* radius[GS_MAX_CAMS];
    const uint8_t* clamp[GS_MAX_CAMS];
};

struct GradOut {
    float* mean;
    float* log_scale;
    float* quat;
    float* opacity_logit;
    float* sh;
    int overwrite;  // 1: store the reached Gaussians' gradients instead of adding them
};

// Entries visible in at least one camera, appended to `list` (order is
// irrelevant: entries are distinct Gaussians, so their gradients are disjoint).
// One workgroup handles kChunk entries: it reads their radii once (every load
// of a camera issued before the first use), counts the visible ones, reserves
// its slice with a single atomic, then writes them.
template <int kChunk>
__global__ __launch_bounds__(256) void k_visible_list(int64_t n_in, const int64_t* __restrict__ n_in_dev, BwdIn B,
                                                      int n_cams, uint32_t* __restrict__ list,
                                                      uint32_t* __restrict__ count) {
    constexpr int kIt = kChunk / 256;
    static_assert(kIt <= 32, "visibility bits per camera fit 32 bits");
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t base_s;
    int64_t cnt = n_in;
    if (n_in_dev) cnt = min(cnt, *n_in_dev);
    const int64_t j0 = int64_t(blockIdx.x) * kChunk;
    if (j0 >= cnt) return;  // uniform
    const int w = threadIdx.x / 64;
    // bit it of cam_vis[c]: entry j0 + it * 256 + tid has radius > 0 in camera c
    // (camera loops unrolled to GS_MAX_CAMS so that cam_vis stays in registers)
    uint32_t cam_vis[GS_MAX_CAMS];
    uint32_t any = 0;
#pragma unroll
    for (int c = 0; c < GS_MAX_CAMS; ++c) {
        cam_vis[c] = 0;
        if (c >= n_cams) continue;
        int32_t r[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) r[it] = B.radius[c][min<int64_t>(j0 + it * 256 + threadIdx.x, cnt - 1)];
        uint32_t bits = 0;
#pragma unroll
        for (int it = 0; it < kIt; ++it)
            if (j0 + it * 256 + threadIdx.x < cnt && r[it] > 0) bits |= 1u << it;
        cam_vis[c] = bits;
        any |= bits;
    }
    uint32_t mine = 0;
#pragma unroll
    for (int it = 0; it < kIt; ++it) mine += popc64(ballot((any >> it) & 1u));
    if (lane_id() == 0) wsum[w] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base_s = tot ? atomicAdd(count, tot) : 0u;
    }
    __syncthreads();
    uint32_t off = base_s;
    for (int k = 0; k < w; ++k) off += wsum[k];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t j = j0 + it * 256 + threadIdx.x;
        const bool vis = (any >> it) & 1u;
        const uint64_t m = ballot(vis);
        if (vis) {
            list[off + popc64(m & lanemask_lt())] = uint32_t(j);
            // the blend accumulates into these records with atomics; only
            // visible entries are ever written or read, so only they are cleared
#pragma unroll
            for (int c = 0; c < GS_MAX_CAMS; ++c) {
                if (!((cam_vis[c] >> it) & 1u)) continue;
                float4* r = reinterpret_cast<float4*>(B.d2[c] + j * kD2Stride);
                r[0] = make_float4(0.f, 0.f, 0.f, 0.f);
                r[1] = make_float4(0.f, 0.f, 0.f, 0.f);
                r[2] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        off += popc64(m);
    }
}

// Copies the partials of camera 0 to the caller's [9][n_in] array (visible
// entries; the others were set to zero beforehand).
__global__ __launch_bounds__(256) void k_export_d2(const float* __restrict__ d2, int64_t n_in,
                                                   const uint32_t* __restrict__ list, const uint32_t* __restrict__ count,
                                                   const int32_t* __restrict__ radius, float* __restrict__ out) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= *count) return;
    const int64_t j = list[t];
    if (radius[j] <= 0) return;
#pragma unroll
    for (int k = 0; k < 9; ++k) out[int64_t(k) * n_in + j] = d2[j * kD2Stride + k];
}

__global__ __launch_bounds__(256) void k_project_bwd(SceneP P, const int32_t* __restrict__ active, int64_t /*n_in*/,
                                                     const uint32_t* __restrict__ list,
                                                     const uint32_t* __restrict__ count, CamSet C, BwdIn B,
                                                     GradOut GO) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= *count) return;
    const int64_t j = list[t];
    const int64_t i = active ? int64_t(active[j]) : j;
    if (i < 0 || i >= P.n) return;
    const int64_t N = P.n;
    const float mu[3] = {P.mean[i], P.mean[N + i], P.mean[2 * N + i]};
    const float ls[3] = {P.log_scale[i], P.log_scale[N + i], P.log_scale[2 * N + i]};
    const float q[4] = {P.quat[i], P.quat[N + i], P.quat[2 * N + i], P.quat[3 * N + i]};
    float s[3], qn[4], R[9], M[9], S[6], qlen;
    covariance(ls, q, s, qn, R, M, S, qlen);
    const float opa = 1.f / (1.f + __expf(-P.opacity_logit[i]));

    float dmu[3] = {0.f, 0.f, 0.f};
    float dS[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // symmetric: 00 01 02 11 12 22
    float dlogit = 0.f;

    for (int c = 0; c < C.n; ++c) {
        if (B.radius[c][j] <= 0) continue;
        const DevCam& K = C.cam[c];
        const float4* d2 = reinterpret_cast<const float4*>(B.d2[c] + j * kD2Stride);
        const float4 q0 = d2[0], q1 = d2[1];
        const float dmx = q0.x, dmy = q0.y;
        const float dca = q0.z, dcb = q0.w, dcc = q1.x;
        const float dop = q1.y;
        float drgb[3] = {q1.z, q1.w, d2[2].x};
        const uint8_t cb = B.clamp[c][j];
        Geo G;
        geo_camera(K, mu, G);
        geo_cov(K, S, G);
        // opacity
        dlogit += dop * opa * (1.f - opa);
        // conic = (c, -b, a) / det  ->  d(a, b, c) of the screen covariance
        const float A = G.a, Bv = G.b, Cv = G.c;
        const float id2 = 1.f / (G.det * G.det);
        const float dA = (-Cv * Cv * dca + Bv * Cv * dcb - Bv * Bv * dcc) * id2;
        const float dB = (2.f * Bv * Cv * dca - (A * Cv + Bv * Bv) * dcb + 2.f * A * Bv * dcc) * id2;
        const float dC = (-Bv * Bv * dca + A * Bv * dcb - A * A * dcc) * id2;
        // Sigma2D = T Sigma T^T with symmetric upstream Gs = [[dA, dB/2], [dB/2, dC]]
        float dT0[3], dT1[3];
        for (int k = 0; k < 3; ++k) {
            dT0[k] = 2.f * dA * G.U0[k] + dB * G.U1[k];
            dT1[k] = dB * G.U0[k] + 2.f * dC * G.U1[k];
        }
        const float hB = 0.5f * dB;
        // dSigma = T^T Gs T
        {
            const float* t0 = G.T0;
            const float* t1 = G.T1;
            auto ent = [&](int k, int l) {
                return dA * t0[k] * t0[l] + hB * (t0[k] * t1[l] + t1[k] * t0[l]) + dC * t1[k] * t1[l];
            };
            dS[0] += ent(0, 0); dS[1] += ent(0, 1); dS[2] += ent(0, 2);
            dS[3] += ent(1, 1); dS[4] += ent(1, 2); dS[5] += ent(2, 2);
        }
        // T = J W: dJ = dT W^T on the non-zero entries of J
        const float dJ00 = dT0[0] * K.R[0] + dT0[1] * K.R[1] + dT0[2] * K.R[2];
        const float dJ02 = dT0[0] * K.R[6] + dT0[1] * K.R[7] + dT0[2] * K.R[8];
        const float dJ11 = dT1[0] * K.R[3] + dT1[1] * K.R[4] + dT1[2] * K.R[5];
        const float dJ12 = dT1[0] * K.R[6] + dT1[1] * K.R[7] + dT1[2] * K.R[8];
        const float rz = G.rz, rz2 = rz * rz, rz3 = rz2 * rz;
        const float txc = G.ux * G.tz, tyc = G.uy * G.tz;
        float dtx = 0.f, dty = 0.f;
        float dtz = -K.fx * rz2 * dJ00 - K.fy * rz2 * dJ11 + 2.f * K.fx * txc * rz3 * dJ02 +
                    2.f * K.fy * tyc * rz3 * dJ12;
        const float gtxc = -K.fx * rz2 * dJ02, gtyc = -K.fy * rz2 * dJ12;
        if (G.txtz >= -K.limx && G.txtz <= K.limx) dtx += gtxc; else dtz += G.ux * gtxc;
        if (G.tytz >= -K.limy && G.tytz <= K.limy) dty += gtyc; else dtz += G.uy * gtyc;
        // mean2d = (fx tx / tz + cx, fy ty / tz + cy)
        dtx += dmx * K.fx * rz;
        dty += dmy * K.fy * rz;
        dtz -= (dmx * K.fx * G.tx + dmy * K.fy * G.ty) * rz2;
        // t = W mu + t_cw
        dmu[0] += K.R[0] * dtx + K.R[3] * dty + K.R[6] * dtz;
        dmu[1] += K.R[1] * dtx + K.R[4] * dty + K.R[7] * dtz;
        dmu[2] += K.R[2] * dtx + K.R[5] * dty + K.R[8] * dtz;
        (void)drgb;
        (void)cb;
    }
    // Sigma = M M^T: dM = 2 dSigma_sym M
    const float D[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
    float dM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            dM[r * 3 + c] = 2.f * (D[r * 3 + 0] * M[0 * 3 + c] + D[r * 3 + 1] * M[1 * 3 + c] + D[r * 3 + 2] * M[2 * 3 + c]);
    // M = R diag(s)
    float dls[3], dR[9];
    for (int c = 0; c < 3; ++c) {
        const float ds = dM[c] * R[c] + dM[3 + c] * R[3 + c] + dM[6 + c] * R[6 + c];
        dls[c] = ds * s[c];
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) dR[r * 3 + c] = dM[r * 3 + c] * s[c];
    const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    float dq[4];
    dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.f * x * dR[8]);
    dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.f * y * dR[8]);
    dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const float qd = dq[0] * qn[0] + dq[1] * qn[1] + dq[2] * qn[2] + dq[3] * qn[3];
    const float iq = 1.f / qlen;
    // (the SH kernel runs after this one and adds its part of the mean
    // gradient to what is stored here)
    if (GO.overwrite) {
        for (int k = 0; k < 4; ++k) GO.quat[int64_t(k) * N + i] = (dq[k] - qd * qn[k]) * iq;
        for (int k = 0; k < 3; ++k) {
            GO.mean[int64_t(k) * N + i] = dmu[k];
            GO.log_scale[int64_t(k) * N + i] = dls[k];
        }
        GO.opacity_logit[i] = dlogit;
        return;
    }
    for (int k = 0; k < 4; ++k) GO.quat[int64_t(k) * N + i] += (dq[k] - qd * qn[k]) * iq;
    for (int k = 0; k < 3; ++k) {
        GO.mean[int64_t(k) * N + i] += dmu[k];
        GO.log_scale[int64_t(k) * N + i] += dls[k];
    }
    GO.opacity_logit[i] += dlogit;
}

// Colour part of the backward: d sh = d rgb * Y (zero on clamped channels),
// and the view-direction term of the mean gradient through the SH basis.  The
// 48 coefficients are loaded once, the SH gradient is summed over the cameras
// in registers, and the accumulation into the caller's gradient loads all 48
// old values before storing any, so the loads of a thread are all in flight
// together.
__global__ __launch_bounds__(256) void k_project_bwd_sh(SceneP P, const int32_t* __restrict__ active,
                                                        int64_t /*n_in*/, const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ count, CamSet C, BwdIn B,
                                                        GradOut GO) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= *count) return;
    const int64_t j = list[t];
    const int64_t i = active ? int64_t(active[j]) : j;
    if (i < 0 || i >= P.n) return;
    const int64_t N = P.n;
    const float mu[3] = {P.mean[i], P.mean[N + i], P.mean[2 * N + i]};
    float shv[48], gacc[48];
#pragma unroll
    for (int o = 0; o < 48; ++o) {
        shv[o] = P.sh[int64_t(o) * N + i];
        gacc[o] = 0.f;
    }
    float dmu[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < C.n; ++c) {
        if (B.radius[c][j] <= 0) continue;
        const DevCam& K = C.cam[c];
        const float* d2 = B.d2[c] + j * kD2Stride;
        const uint8_t cb = B.clamp[c][j];
        float drgb[3] = {d2[6], d2[7], d2[8]};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
            if (cb & (1u << ch)) drgb[ch] = 0.f;
        const float vx = mu[0] - K.campos[0], vy = mu[1] - K.campos[1], vz = mu[2] - K.campos[2];
        const float il = 1.f / sqrtf(vx * vx + vy * vy + vz * vz);
        const float x = vx * il, y = vy * il, z = vz * il;
        float Y[16];
        sh_basis(x, y, z, Y);
        float wsum[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                acc = fmaf(drgb[ch], shv[k * 3 + ch], acc);
                gacc[k * 3 + ch] = fmaf(drgb[ch], Y[k], gacc[k * 3 + ch]);
            }
            wsum[k] = acc;
        }
        float gd[3];
        sh_basis_grad(x, y, z, wsum, gd);
        const float dot = gd[0] * x + gd[1] * y + gd[2] * z;
        dmu[0] += (gd[0] - dot * x) * il;
        dmu[1] += (gd[1] - dot * y) * il;
        dmu[2] += (gd[2] - dot * z) * il;
    }
    if (GO.overwrite) {
#pragma unroll
        for (int o = 0; o < 48; ++o) GO.sh[int64_t(o) * N + i] = gacc[o];
    } else {
        float old[48];
#pragma unroll
        for (int o = 0; o < 48; ++o) old[o] = GO.sh[int64_t(o) * N + i];
#pragma unroll
        for (int o = 0; o < 48; ++o) GO.sh[int64_t(o) * N + i] = old[o] + gacc[o];
    }
    for (int k = 0; k < 3; ++k) GO.mean[int64_t(k) * N + i] += dmu[k];
}

int fill_camset(const gs_camera* cams, int n_cams, CamSet& C) {
    int64_t tt = 0;
    int rc = validate_cams(cams, n_cams, GS_MAX_CAMS, &tt);
    if (rc) return rc;
    memset(&C, 0, sizeof(C));
    C.n = n_cams;
    uint32_t off = 0;
    for (int c = 0; c < n_cams; ++c) {
        C.cam[c] = make_devcam(cams[c], off);
        off += uint32_t(gs_num_tiles(cams[c].width, cams[c].height));
    }
    return GS_OK;
}

static int scene_ok(const gs_scene* s) {
    if (!s || s->n < 0 || s->n >= (int64_t(1) << 31))
        return fail(GS_ERR_INVALID_ARG, "scene: null or n out of range");
    if (s->n > 0 && (!s->mean || !s->log_scale || !s->quat || !s->opacity_logit || !s->sh))
        return fail(GS_ERR_INVALID_ARG, "scene: null parameter array");
    return GS_OK;
}

static void fill_bwdin(BwdIn& B, float* const* d2, const gs_projected* proj, int n_cams) {
    memset(&B, 0, sizeof(B));
    for (int c = 0; c < n_cams; ++c) {
        B.d2[c] = d2[c];
        B.radius[c] = proj[c].radius;
        B.clamp[c] = proj[c].clamp_bits;
    }
}

// Entries visible in some camera, listed once; their partial records are
// cleared for the blend's atomics.
int launch_visible_list(int64_t n_in, const int64_t* n_in_dev, int n_cams, float* const* d2, const gs_projected* proj,
                        uint32_t* list, uint32_t* count, hipStream_t stream) {
    BwdIn B;
    fill_bwdin(B, d2, proj, n_cams);
    int rc = fill_u32(count, 0u, 1, stream);
    if (rc) return rc;
    if (n_in == 0) return GS_OK;
    if (n_in <= kSmallListInput)
        launch("visible_list", k_visible_list<kChunkSmall>, dim3(unsigned((n_in + kChunkSmall - 1) / kChunkSmall)),
               dim3(256), 0, stream, n_in, n_in_dev, B, n_cams, list, count);
    else
        launch("visible_list", k_visible_list<kVisChunkLarge>,
               dim3(unsigned((n_in + kVisChunkLarge - 1) / kVisChunkLarge)), dim3(256), 0, stream, n_in, n_in_dev, B,
               n_cams, list, count);
    return check_launch("visible list");
}

int launch_export_d2(const float* d2, int64_t n_in, const uint32_t* list, const uint32_t* count,
                     const int32_t* radius, float* out, hipStream_t stream) {
    int rc = fill_u32(out, 0u, size_t(9) * size_t(n_in), stream);
    if (rc) return rc;
    if (n_in == 0) return GS_OK;
    launch("export_d2", k_export_d2, dim3(unsigned((n_in + 255) / 256)), dim3(256), 0, stream, d2, n_in, list, count,
           radius, out);
    return check_launch("export partials");
}

int launch_project_bwd(const gs_scene* scene, const int32_t* active_idx, int64_t n_in, const gs_camera* cams,
                       int n_cams, float* const* d2, const gs_projected* proj, const gs_grads* grads,
                       const uint32_t* list, const uint32_t* count, hipStream_t stream) {
    CamSet C;
    int rc = fill_camset(cams, n_cams, C);
    if (rc) return rc;
    SceneP P{scene->mean, scene->log_scale, scene->quat, scene->opacity_logit, scene->sh, scene->n};
    BwdIn B;
    fill_bwdin(B, d2, proj, n_cams);
    GradOut G{grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->sh, grads->overwrite ? 1 : 0};
    if (n_in == 0) return GS_OK;
    launch("project_bwd", k_project_bwd, dim3(unsigned((n_in + 255) / 256)), dim3(256), 0, stream, P, active_idx,
           n_in, list, count, C, B, G);
    launch("project_bwd_sh", k_project_bwd_sh, dim3(unsigned((n_in + 255) / 256)), dim3(256), 0, stream, P,
           active_idx, n_in, list, count, C, B, G);
    return check_launch("project backward");
}

int check_scene(const gs_scene* s) { return scene_ok(s); }

}  // namespace gsmi

using namespace gsmi;

size_t ws_project(int64_t n_in) {
    Carve cv(nullptr);
    cv.take<uint32_t>(size_t(n_in > 0 ? n_in : 1));
    cv.take<uint32_t>(4);
    return cv.used();
}

extern "C" int gs_project(const gs_scene* scene, const int32_t* active_idx, int64_t n_in, const int64_t* n_in_dev,
                          const gs_camera* cams, int n_cams, const gs_projected* out, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
    int rc = scene_ok(scene);
    if (rc) return rc;
    if (n_in < 0 || n_in >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "gs_project: n_in out of range");
    if (!active_idx && n_in > scene->n) return fail(GS_ERR_INVALID_ARG, "gs_project: n_in > n without active_idx");
    if (!out) return fail(GS_ERR_INVALID_ARG, "gs_project: null output");
    CamSet C;
    rc = fill_camset(cams, n_cams, C);
    if (rc) return rc;
    ProjOut O;
    memset(&O, 0, sizeof(O));
    for (int c = 0; c < n_cams; ++c) {
        const gs_projected& p = out[c];
        if (n_in > 0 && (!p.rec || !p.depth || !p.radius || !p.tiles_touched || !p.clamp_bits))
            return fail(GS_ERR_INVALID_ARG, "gs_project: camera %d: null required output", c);
        if (!aligned(p.rec, 16)) return fail(GS_ERR_INVALID_ARG, "gs_project: rec must be 16-byte aligned");
        O.rec[c] = p.rec; O.depth[c] = p.depth; O.radius[c] = p.radius; O.tiles[c] = p.tiles_touched;
        O.clamp[c] = p.clamp_bits; O.mean2d[c] = p.mean2d; O.conic[c] = p.conic; O.opacity[c] = p.opacity;
        O.rgb[c] = p.rgb;
    }
    const size_t need = ws_project(n_in);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_project: workspace needs %zu bytes (256-aligned)", need);
    if (n_in == 0) return GS_OK;
    SceneP P{scene->mean, scene->log_scale, scene->quat, scene->opacity_logit, scene->sh, scene->n};
    Carve cv(ws);
    uint32_t* list = cv.take<uint32_t>(size_t(n_in));
    uint32_t* count = cv.take<uint32_t>(4);
    if ((rc = fill_u32(count, 0u, 1, stream))) return rc;
    if (n_in > kSmallListInput) {
        launch("project", k_project_all, dim3(unsigned((n_in + 255) / 256)), dim3(256), 0, stream, P, active_idx,
               n_in, n_in_dev, C, O);
        return check_launch("gs_project");
    }
    launch("project_cull", k_project_cull<kChunkSmall>, dim3(unsigned((n_in + kChunkSmall - 1) / kChunkSmall)),
           dim3(256), 0, stream, P, active_idx, n_in, n_in_dev, C, O, list, count);
    launch("project", k_project, dim3(unsigned((n_in + 255) / 256)), dim3(256), 0, stream, P, active_idx, n_in,
           static_cast<const uint32_t*>(list), static_cast<const uint32_t*>(count), C, O);
    return check_launch("gs_project");
}
