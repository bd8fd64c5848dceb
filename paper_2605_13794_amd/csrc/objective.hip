// The paper's objective (Sec. 3.4): photometric L1 + SSIM (Eq. 4) and the
// scale regulariser over the visible set (Eq. 5).
//
// SSIM uses an 11x11 Gaussian window (sigma 1.5) applied separably on
// 32x32 output tiles staged in LDS with a 5-pixel halo (zero outside the
// image).  The forward writes, per pixel, the derivatives of the SSIM map
// with respect to the local moments (mean of x, of x^2 and of xy); because
// the window is symmetric, the backward is the same separable blur of those
// three maps, combined with x and y.
#include "common.h"

namespace gsmi {

constexpr int kSsimT = 32;              // output tile edge
constexpr int kHalo = 5;
constexpr int kSsimE = kSsimT + 2 * kHalo;  // 42
constexpr float kC1 = 0.0001f;          // (0.01)^2
constexpr float kC2 = 0.0009f;          // (0.03)^2

struct SsimWin {
    float w[11];
};

// Loads a channel tile (with halo, zero outside the image) into LDS.
__device__ __forceinline__ void load_tile(const float* __restrict__ img, int W, int H, int x0, int y0,
                                          float* __restrict__ dst) {
    for (int k = threadIdx.x; k < kSsimE * kSsimE; k += 256) {
        const int r = k / kSsimE, c = k % kSsimE;
        const int y = y0 - kHalo + r, x = x0 - kHalo + c;
        dst[k] = (x >= 0 && x < W && y >= 0 && y < H) ? img[size_t(y) * W + x] : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ X, const float* __restrict__ Y, int W,
                                                  int H, SsimWin win, float* __restrict__ dmu,
                                                  float* __restrict__ dxx, float* __restrict__ dxy,
                                                  double* __restrict__ part) {
    __shared__ float sx[kSsimE * kSsimE];
    __shared__ float sy[kSsimE * kSsimE];
    __shared__ float hsum[5][kSsimE * kSsimT];
    __shared__ double red[256];
    const int c = blockIdx.z;
    const size_t plane = size_t(W) * H;
    const float* x = X + c * plane;
    const float* y = Y + c * plane;
    const int x0 = blockIdx.x * kSsimT, y0 = blockIdx.y * kSsimT;
    load_tile(x, W, H, x0, y0, sx);
    load_tile(y, W, H, x0, y0, sy);
    __syncthreads();
    // horizontal pass over every row of the halo'd tile
    for (int k = threadIdx.x; k < kSsimE * kSsimT; k += 256) {
        const int r = k / kSsimT, cc = k % kSsimT;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float xv = sx[r * kSsimE + cc + d], yv = sy[r * kSsimE + cc + d];
            const float wd = win.w[d];
            a0 = fmaf(wd, xv, a0);
            a1 = fmaf(wd, yv, a1);
            a2 = fmaf(wd, xv * xv, a2);
            a3 = fmaf(wd, yv * yv, a3);
            a4 = fmaf(wd, xv * yv, a4);
        }
        hsum[0][k] = a0; hsum[1][k] = a1; hsum[2][k] = a2; hsum[3][k] = a3; hsum[4][k] = a4;
    }
    __syncthreads();
    double acc = 0.0;
    for (int k = threadIdx.x; k < kSsimT * kSsimT; k += 256) {
        const int r = k / kSsimT, cc = k % kSsimT;
        const int px = x0 + cc, py = y0 + r;
        if (px >= W || py >= H) continue;
        float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float wd = win.w[d];
#pragma unroll
            for (int q = 0; q < 5; ++q) m[q] = fmaf(wd, hsum[q][(r + d) * kSsimT + cc], m[q]);
        }
        const float mx = m[0], my = m[1];
        const float A1 = 2.f * mx * my + kC1;
        const float B1 = mx * mx + my * my + kC1;
        const float A2 = 2.f * (m[4] - mx * my) + kC2;
        const float B2 = (m[2] - mx * mx) + (m[3] - my * my) + kC2;
        const float S = (A1 * A2) / (B1 * B2);
        acc += double(S);
        const size_t p = c * plane + size_t(py) * W + px;
        dmu[p] = S * (2.f * my / A1 - 2.f * mx / B1 - 2.f * my / A2 + 2.f * mx / B2);
        dxx[p] = -S / B2;
        dxy[p] = 2.f * S / A2;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

// grad = scale * [ (1 - lambda) sign(x - y) / N
//                  - lambda / N (G*Dmu + 2 x G*Dxx + y G*Dxy) ]
__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ X, const float* __restrict__ Y, int W,
                                                  int H, SsimWin win, const float* __restrict__ dmu,
                                                  const float* __restrict__ dxx, const float* __restrict__ dxy,
                                                  float lam, float inv_n, float scale, float* __restrict__ grad,
                                                  double* __restrict__ part_l1) {
    __shared__ float s0[kSsimE * kSsimE];
    __shared__ float s1[kSsimE * kSsimE];
    __shared__ float s2[kSsimE * kSsimE];
    __shared__ float hsum[3][kSsimE * kSsimT];
    __shared__ double red[256];
    const int c = blockIdx.z;
    const size_t plane = size_t(W) * H;
    const int x0 = blockIdx.x * kSsimT, y0 = blockIdx.y * kSsimT;
    load_tile(dmu + c * plane, W, H, x0, y0, s0);
    load_tile(dxx + c * plane, W, H, x0, y0, s1);
    load_tile(dxy + c * plane, W, H, x0, y0, s2);
    __syncthreads();
    for (int k = threadIdx.x; k < kSsimE * kSsimT; k += 256) {
        const int r = k / kSsimT, cc = k % kSsimT;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float wd = win.w[d];
            const int idx = r * kSsimE + cc + d;
            a0 = fmaf(wd, s0[idx], a0);
            a1 = fmaf(wd, s1[idx], a1);
            a2 = fmaf(wd, s2[idx], a2);
        }
        hsum[0][k] = a0; hsum[1][k] = a1; hsum[2][k] = a2;
    }
    __syncthreads();
    double acc = 0.0;
    for (int k = threadIdx.x; k < kSsimT * kSsimT; k += 256) {
        const int r = k / kSsimT, cc = k % kSsimT;
        const int px = x0 + cc, py = y0 + r;
        if (px >= W || py >= H) continue;
        float b0 = 0.f, b1 = 0.f, b2 = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float wd = win.w[d];
            const int idx = (r + d) * kSsimT + cc;
            b0 = fmaf(wd, hsum[0][idx], b0);
            b1 = fmaf(wd, hsum[1][idx], b1);
            b2 = fmaf(wd, hsum[2][idx], b2);
        }
        const size_t p = c * plane + size_t(py) * W + px;
        const float xv = X[p], yv = Y[p];
        const float dlt = xv - yv;
        acc += double(fabsf(dlt));
        const float sg = dlt > 0.f ? 1.f : (dlt < 0.f ? -1.f : 0.f);
        const float gs = -(b0 + 2.f * xv * b1 + yv * b2);
        grad[p] = scale * inv_n * ((1.f - lam) * sg + lam * gs);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part_l1[(size_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_photo_final(const double* __restrict__ ps, const double* __restrict__ pl,
                                                     int nparts, double inv_n, float lam, float scale,
                                                     float* __restrict__ loss) {
    __shared__ double r0[256], r1[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) { a += ps[i]; b += pl[i]; }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) { r0[threadIdx.x] += r0[threadIdx.x + o]; r1[threadIdx.x] += r1[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *loss = float(double(scale) * ((1.0 - lam) * r1[0] * inv_n + lam * (1.0 - r0[0] * inv_n)));
}

// ---------------------------------------------------------------------------
// Scale regulariser
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scale_reg_sum(const float* __restrict__ log_scale, int64_t n,
                                                       const int32_t* __restrict__ active, int64_t n_in,
                                                       const int64_t* __restrict__ n_in_dev,
                                                       const int32_t* __restrict__ radius, double* __restrict__ part_s,
                                                       uint32_t* __restrict__ part_c) {
    __shared__ double rs[256];
    __shared__ uint32_t rc[256];
    int64_t cnt_in = n_in;
    if (n_in_dev) cnt_in = min(cnt_in, *n_in_dev);
    double s = 0.0;
    uint32_t cnt = 0;
    for (int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x; j < cnt_in; j += int64_t(gridDim.x) * 256) {
        if (radius[j] <= 0) continue;
        const int64_t i = active ? int64_t(active[j]) : j;
        if (i < 0 || i >= n) continue;
        const float m = fminf(fminf(log_scale[i], log_scale[n + i]), log_scale[2 * n + i]);
        s += double(__expf(m));
        ++cnt;
    }
    rs[threadIdx.x] = s;
    rc[threadIdx.x] = cnt;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) { rs[threadIdx.x] += rs[threadIdx.x + o]; rc[threadIdx.x] += rc[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { part_s[blockIdx.x] = rs[0]; part_c[blockIdx.x] = rc[0]; }
}

__global__ __launch_bounds__(256) void k_scale_reg_final(const double* __restrict__ part_s,
                                                         const uint32_t* __restrict__ part_c, int nparts, float beta,
                                                         float* __restrict__ loss, float* __restrict__ coef) {
    __shared__ double rs[256];
    __shared__ unsigned long long rc[256];
    double s = 0.0;
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) { s += part_s[i]; c += part_c[i]; }
    rs[threadIdx.x] = s;
    rc[threadIdx.x] = c;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) { rs[threadIdx.x] += rs[threadIdx.x + o]; rc[threadIdx.x] += rc[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nv = double(rc[0]);
        *loss = nv > 0 ? float(double(beta) * rs[0] / nv) : 0.f;
        *coef = nv > 0 ? float(double(beta) / nv) : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_scale_reg_grad(const float* __restrict__ log_scale, int64_t n,
                                                        const int32_t* __restrict__ active, int64_t n_in,
                                                        const int64_t* __restrict__ n_in_dev,
                                                        const int32_t* __restrict__ radius,
                                                        const float* __restrict__ coef, float* __restrict__ grad) {
    int64_t cnt_in = n_in;
    if (n_in_dev) cnt_in = min(cnt_in, *n_in_dev);
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (j >= cnt_in || radius[j] <= 0) return;
    const int64_t i = active ? int64_t(active[j]) : j;
    if (i < 0 || i >= n) return;
    const float l0 = log_scale[i], l1 = log_scale[n + i], l2 = log_scale[2 * n + i];
    int a = 0;
    float m = l0;
    if (l1 < m) { m = l1; a = 1; }
    if (l2 < m) { m = l2; a = 2; }
    grad[int64_t(a) * n + i] += *coef * __expf(m);
}

}  // namespace gsmi

using namespace gsmi;

static SsimWin make_window() {
    SsimWin w;
    double g[11], s = 0.0;
    for (int k = 0; k < 11; ++k) {
        const double x = k - 5.0;
        g[k] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < 11; ++k) w.w[k] = float(g[k] / s);
    return w;
}

static size_t photo_parts(int32_t W, int32_t H) {
    return size_t((W + kSsimT - 1) / kSsimT) * size_t((H + kSsimT - 1) / kSsimT) * 3;
}

size_t ws_photo(int32_t W, int32_t H) {
    Carve cv(nullptr);
    cv.take<float>(size_t(3) * 3 * size_t(W) * H);
    cv.take<double>(photo_parts(W, H));
    cv.take<double>(photo_parts(W, H));
    return cv.used();
}

extern "C" int gs_photo_loss(const float* rgb, const float* target, int32_t width, int32_t height, float lambda,
                             float scale, float* loss_dev, float* grad, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
    if (!rgb || !target || !loss_dev || !grad || width <= 0 || height <= 0 || width > 16384 || height > 16384)
        return fail(GS_ERR_INVALID_ARG, "gs_photo_loss: bad arguments");
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(GS_ERR_INVALID_ARG, "gs_photo_loss: lambda in [0, 1]");
    const size_t need = ws_photo(width, height);
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_photo_loss: workspace needs %zu bytes (256-aligned)", need);
    const size_t plane3 = size_t(3) * width * height;
    Carve cv(ws);
    float* dmu = cv.take<float>(plane3);
    float* dxx = dmu + plane3;
    float* dxy = dxx + plane3;
    cv.take<float>(2 * plane3);
    double* ps = cv.take<double>(photo_parts(width, height));
    double* pl = cv.take<double>(photo_parts(width, height));
    const SsimWin win = make_window();
    dim3 grid((width + kSsimT - 1) / kSsimT, (height + kSsimT - 1) / kSsimT, 3);
    launch("ssim_fwd", k_ssim_fwd, grid, dim3(256), 0, stream, rgb, target, width, height, win, dmu, dxx, dxy, ps);
    launch("ssim_bwd", k_ssim_bwd, grid, dim3(256), 0, stream, rgb, target, width, height, win, dmu, dxx, dxy, lambda,
           float(1.0 / double(plane3)), scale, grad, pl);
    hipLaunchKernelGGL(k_photo_final, dim3(1), dim3(256), 0, stream, ps, pl, int(photo_parts(width, height)),
                       1.0 / double(plane3), lambda, scale, loss_dev);
    return check_launch("gs_photo_loss");
}

constexpr int kRegBlocks = 512;

size_t ws_scale_reg() {
    Carve cv(nullptr);
    cv.take<double>(kRegBlocks);
    cv.take<uint32_t>(kRegBlocks);
    cv.take<float>(4);
    return cv.used();
}

extern "C" int gs_scale_reg(const gs_scene* scene, const int32_t* active_idx, int64_t n_in, const int64_t* n_in_dev,
                            const int32_t* radius, float beta, float* loss_dev, float* grad_log_scale, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
    if (!scene || !scene->log_scale || !radius || !loss_dev || !grad_log_scale || n_in < 0 ||
        n_in >= (int64_t(1) << 31) || (!active_idx && n_in > scene->n))
        return fail(GS_ERR_INVALID_ARG, "gs_scale_reg: bad arguments");
    const size_t need = ws_scale_reg();
    if (!ws || ws_bytes < need || !aligned(ws, 256))
        return fail(GS_ERR_WORKSPACE, "gs_scale_reg: workspace needs %zu bytes (256-aligned)", need);
    Carve cv(ws);
    double* ps = cv.take<double>(kRegBlocks);
    uint32_t* pc = cv.take<uint32_t>(kRegBlocks);
    float* coef = cv.take<float>(4);
    int blocks = int(std::min<int64_t>(kRegBlocks, std::max<int64_t>(1, (n_in + 255) / 256)));
    hipLaunchKernelGGL(k_scale_reg_sum, dim3(blocks), dim3(256), 0, stream, scene->log_scale, scene->n, active_idx,
                       n_in, n_in_dev, radius, ps, pc);
    hipLaunchKernelGGL(k_scale_reg_final, dim3(1), dim3(256), 0, stream, ps, pc, blocks, beta, loss_dev, coef);
    if (n_in > 0)
        hipLaunchKernelGGL(k_scale_reg_grad, dim3(unsigned((n_in + 255) / 256)), dim3(256), 0, stream,
                           scene->log_scale, scene->n, active_idx, n_in, n_in_dev, radius, coef, grad_log_scale);
    return check_launch("gs_scale_reg");
}
