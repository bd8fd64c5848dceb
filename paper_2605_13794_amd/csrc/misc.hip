// Error reporting, workspace sizing, fill kernel, L1 loss and fused Adam.
#include <cmath>
#include <algorithm>
#include <cstdarg>

#include "common.h"

namespace gsmi {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

static thread_local char g_prof_name[64] = "";
static thread_local hipEvent_t g_prof_start = nullptr, g_prof_stop = nullptr;

bool profile_match(const char* name, hipEvent_t* start, hipEvent_t* stop) {
    if (!g_prof_name[0] || strcmp(name, g_prof_name) != 0) return false;
    *start = g_prof_start;
    *stop = g_prof_stop;
    return true;
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return GS_OK;
}

int validate_cams(const gs_camera* cams, int n_cams, int max_cams, int64_t* total_tiles) {
    if (!cams || n_cams < 1 || n_cams > max_cams)
        return fail(GS_ERR_INVALID_ARG, "n_cams must be in [1, %d]", max_cams);
    int64_t tot = 0;
    for (int c = 0; c < n_cams; ++c) {
        const gs_camera& k = cams[c];
        if (k.width <= 0 || k.height <= 0 || k.width > 16384 || k.height > 16384)
            return fail(GS_ERR_INVALID_ARG, "camera %d: bad image size %dx%d", c, k.width, k.height);
        if (!(k.fx > 0.f) || !(k.fy > 0.f))
            return fail(GS_ERR_INVALID_ARG, "camera %d: focal lengths must be positive", c);
        if (!(k.znear > 0.f)) return fail(GS_ERR_INVALID_ARG, "camera %d: znear must be positive", c);
        tot += tiles_x(k.width) * tiles_y(k.height);
    }
    if (tot >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "too many tiles");
    if (total_tiles) *total_tiles = tot;
    return GS_OK;
}

__global__ void k_fill_u32(uint32_t* __restrict__ dst, uint32_t value, size_t count) {
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) dst[i] = value;
}

int fill_u32(void* dst, uint32_t value, size_t count, hipStream_t s) {
    if (count == 0) return GS_OK;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(blocks)), dim3(256), 0, s,
                       static_cast<uint32_t*>(dst), value, count);
    return check_launch("fill");
}

// ---------------------------------------------------------------------------
// L1 loss: per-block partial sums in double, then one block sums them in a
// fixed order (deterministic).  Either output may be skipped: `part` NULL
// (no loss) or `grad` NULL (no gradient); the gradient is multiplied by
// *scale when `scale` is non-NULL (the upstream derivative of an autograd
// graph, read on the device).
// ---------------------------------------------------------------------------
constexpr int kL1Blocks = 1024;

__device__ __forceinline__ float l1_sign(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// Sum of one double per thread over a 256-thread workgroup, in a fixed order
// (butterfly within each wavefront, then the four wavefront sums); valid in
// thread 0.
__device__ __forceinline__ double block_sum_f64(double v, double* w4) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) w4[threadIdx.x / 64] = v;
    __syncthreads();
    return (w4[0] + w4[1]) + (w4[2] + w4[3]);
}

__global__ __launch_bounds__(256) void k_l1_partial(const float* __restrict__ rgb,
                                                    const float* __restrict__ target, int64_t n,
                                                    float* __restrict__ grad, const float* __restrict__ scale,
                                                    double* __restrict__ part) {
    __shared__ double red[4];
    const float inv = (scale ? *scale : 1.0f) / float(n);
    double acc = 0.0;
    const int64_t stride = int64_t(gridDim.x) * 256;
    int64_t done = 0;
    if (((reinterpret_cast<uintptr_t>(rgb) | reinterpret_cast<uintptr_t>(target) |
          reinterpret_cast<uintptr_t>(grad)) & 15) == 0) {
        // four values per thread and load
        const int64_t n4 = n / 4;
        for (int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x; q < n4; q += stride) {
            const float4 a = reinterpret_cast<const float4*>(rgb)[q];
            const float4 b = reinterpret_cast<const float4*>(target)[q];
            const float d[4] = {a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w};
            acc += double(fabsf(d[0]) + fabsf(d[1]) + fabsf(d[2]) + fabsf(d[3]));
            if (grad)
                reinterpret_cast<float4*>(grad)[q] =
                    make_float4(l1_sign(d[0]) * inv, l1_sign(d[1]) * inv, l1_sign(d[2]) * inv, l1_sign(d[3]) * inv);
        }
        done = n4 * 4;
    }
    for (int64_t i = done + int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        const float d = rgb[i] - target[i];
        acc += double(fabsf(d));
        if (grad) grad[i] = l1_sign(d) * inv;
    }
    if (!part) return;
    const double tot = block_sum_f64(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// nparts <= kL1Blocks: every load of a thread (index clamped) is issued
// before the first use.
__global__ __launch_bounds__(256) void k_l1_final(const double* __restrict__ part, int nparts, int64_t n,
                                                  float* __restrict__ loss) {
    __shared__ double red[4];
    constexpr int kIt = kL1Blocks / 256;
    double v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) v[it] = part[min(int(threadIdx.x) + it * 256, nparts - 1)];
    double acc = 0.0;
#pragma unroll
    for (int it = 0; it < kIt; ++it) acc += int(threadIdx.x) + it * 256 < nparts ? v[it] : 0.0;
    const double tot = block_sum_f64(acc, red);
    if (threadIdx.x == 0) *loss = float(tot / double(n));
}

// ---------------------------------------------------------------------------
// Fused Adam over up to 8 groups
// ---------------------------------------------------------------------------
struct AdamGroups {
    float* p[8];
    float* g[8];
    float* m[8];
    float* v[8];
    int64_t start[9];  // prefix of counts (flattened element space)
    float lr[8];
    int n;
};

// Bias corrections come from the host step, or from a device step counter
// (t = *step_dev + 1) so that a captured graph replays correct steps.  One
// grid row per group; float4 accesses when the group's arrays allow it.
__device__ __forceinline__ void adam_one(float& p, float& g, float& m, float& v, bool& gz, float b1, float b2,
                                         float eps, float lr_bc1, float inv_sqrt_bc2) {
    gz = (g == 0.f);
    m = fmaf(b1, m, (1.f - b1) * g);
    v = fmaf(b2, v, (1.f - b2) * g * g);
    p -= lr_bc1 * m / (sqrtf(v) * inv_sqrt_bc2 + eps);
}

__global__ __launch_bounds__(256) void k_adam(AdamGroups G, float b1, float b2, float eps, float inv_bc1,
                                              float inv_sqrt_bc2, int64_t total, int clear,
                                              const int32_t* __restrict__ step_dev) {
    (void)total;
    if (step_dev) {
        const float t = float(*step_dev + 1);
        inv_bc1 = 1.f / (1.f - powf(b1, t));
        inv_sqrt_bc2 = rsqrtf(1.f - powf(b2, t));
    }
    const int k = blockIdx.y;
    const int64_t cnt = G.start[k + 1] - G.start[k];
    const float lr_bc1 = G.lr[k] * inv_bc1;
    float* __restrict__ P = G.p[k];
    float* __restrict__ Gd = G.g[k];
    float* __restrict__ M = G.m[k];
    float* __restrict__ V = G.v[k];
    const bool vec = ((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(Gd) |
                       reinterpret_cast<uintptr_t>(M) | reinterpret_cast<uintptr_t>(V)) & 15) == 0;
    const int64_t stride = int64_t(gridDim.x) * 256;
    int64_t done = 0;
    if (vec) {
        // each workgroup streams one contiguous chunk of whole 256-float4 rows
        const int64_t n4 = cnt / 4;
        const int64_t chunk = ((n4 + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
        const int64_t q0 = int64_t(blockIdx.x) * chunk;
        const int64_t q1 = min(q0 + chunk, n4);
        for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) {
            // streamed once per step: non-temporal loads and stores keep the
            // 2 GB pass from evicting the caches the other kernels use
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 p4 = __builtin_nontemporal_load(reinterpret_cast<f4*>(P) + q);
            const f4 g4 = __builtin_nontemporal_load(reinterpret_cast<const f4*>(Gd) + q);
            const f4 m4 = __builtin_nontemporal_load(reinterpret_cast<f4*>(M) + q);
            const f4 v4 = __builtin_nontemporal_load(reinterpret_cast<f4*>(V) + q);
            float p[4] = {p4.x, p4.y, p4.z, p4.w}, g[4] = {g4.x, g4.y, g4.z, g4.w};
            float m[4] = {m4.x, m4.y, m4.z, m4.w}, v[4] = {v4.x, v4.y, v4.z, v4.w};
            bool all_zero = true;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bool z;
                adam_one(p[e], g[e], m[e], v[e], z, b1, b2, eps, lr_bc1, inv_sqrt_bc2);
                all_zero = all_zero && z;
            }
            __builtin_nontemporal_store(f4{p[0], p[1], p[2], p[3]}, reinterpret_cast<f4*>(P) + q);
            __builtin_nontemporal_store(f4{m[0], m[1], m[2], m[3]}, reinterpret_cast<f4*>(M) + q);
            __builtin_nontemporal_store(f4{v[0], v[1], v[2], v[3]}, reinterpret_cast<f4*>(V) + q);
            if (clear && !all_zero)
                __builtin_nontemporal_store(f4{0.f, 0.f, 0.f, 0.f}, reinterpret_cast<f4*>(Gd) + q);
        }
        done = n4 * 4;
    }
    for (int64_t i = done + int64_t(blockIdx.x) * 256 + threadIdx.x; i < cnt; i += stride) {
        float p = P[i], g = Gd[i], m = M[i], v = V[i];
        bool z;
        adam_one(p, g, m, v, z, b1, b2, eps, lr_bc1, inv_sqrt_bc2);
        P[i] = p;
        M[i] = m;
        V[i] = v;
        if (clear && !z) Gd[i] = 0.f;
    }
}

__global__ void k_adam_tick(int32_t* __restrict__ step_dev) {
    if (threadIdx.x == 0) *step_dev += 1;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" const char* gs_last_error(void) { return g_err; }

extern "C" int gs_profile_kernel(const char* name, hipEvent_t start, hipEvent_t stop) {
    if (!name || !name[0]) {
        g_prof_name[0] = 0;
        return GS_OK;
    }
    if (!start || !stop || strlen(name) >= sizeof(g_prof_name))
        return fail(GS_ERR_INVALID_ARG, "gs_profile_kernel: bad name or events");
    strcpy(g_prof_name, name);
    g_prof_start = start;
    g_prof_stop = stop;
    return GS_OK;
}

extern "C" int64_t gs_num_tiles(int32_t width, int32_t height) {
    if (width <= 0 || height <= 0) return 0;
    return tiles_x(width) * tiles_y(height);
}

size_t ws_lod_mask(int64_t n);
size_t ws_bin_sort(int64_t n_total, int64_t capacity, int64_t n_tiles);
size_t ws_render_bwd(int64_t n, int n_cams);
size_t ws_importance(int64_t n);
size_t ws_score_keep(int64_t n);
size_t ws_simplify(int64_t n);
size_t ws_photo(int32_t W, int32_t H);
size_t ws_scale_reg();
size_t ws_project(int64_t n_in);
size_t ws_voxel_levels(int64_t n);
size_t ws_spawn_gate(int64_t n);

extern "C" size_t gs_workspace_size(int op, int64_t n, int64_t n_pairs, int64_t n_tiles, int n_cams) {
    if (n < 0) n = 0;
    if (n_cams < 1) n_cams = 1;
    switch (op) {
        case GS_OP_LOD_MASK: return ws_lod_mask(n);
        case GS_OP_BIN_SORT: return ws_bin_sort(n * n_cams, n_pairs, n_tiles);
        case GS_OP_RENDER_BWD: return ws_render_bwd(n, n_cams);
        case GS_OP_IMPORTANCE: return ws_importance(n);
        case GS_OP_SCORE_KEEP: return ws_score_keep(n);
        case GS_OP_L1_LOSS: return size_t(kL1Blocks) * sizeof(double);
        case GS_OP_SIMPLIFY: return ws_simplify(n);
        case GS_OP_PHOTO_LOSS: return ws_photo(int32_t(n / 65536), int32_t(n % 65536));
        case GS_OP_SCALE_REG: return ws_scale_reg();
        case GS_OP_PROJECT: return ws_project(n);
        case GS_OP_VOXEL_LEVELS: return ws_voxel_levels(n);
        case GS_OP_SPAWN_GATE: return ws_spawn_gate(n);
        default: return 0;
    }
}

extern "C" int gs_l1_loss(const float* rgb, const float* target, int64_t n_vals, float* loss_dev,
                          float* grad, const float* grad_scale, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_vals <= 0 || !rgb || !target || (!loss_dev && !grad))
        return fail(GS_ERR_INVALID_ARG, "gs_l1_loss: null pointer or empty input");
    if (loss_dev && (!ws || ws_bytes < size_t(kL1Blocks) * sizeof(double) || !aligned(ws, 8)))
        return fail(GS_ERR_WORKSPACE, "gs_l1_loss: workspace too small");
    int blocks = int((n_vals + 255) / 256);
    if (blocks > kL1Blocks) blocks = kL1Blocks;
    double* part = loss_dev ? static_cast<double*>(ws) : nullptr;
    launch("l1_partial", k_l1_partial, dim3(blocks), dim3(256), 0, stream, rgb, target, n_vals, grad, grad_scale,
           part);
    if (loss_dev)
        launch("l1_final", k_l1_final, dim3(1), dim3(256), 0, stream, static_cast<const double*>(part), blocks,
               n_vals, loss_dev);
    return check_launch("gs_l1_loss");
}

extern "C" int gs_adam_step(float* const* params, float* const* grads, float* const* m,
                            float* const* v, const int64_t* counts, int n_groups, const float* lr,
                            float b1, float b2, float eps, int step, int32_t* step_dev, int clear_grads,
                            hipStream_t stream) {
    if (n_groups < 1 || n_groups > 8 || !params || !grads || !m || !v || !counts || !lr || (step < 1 && !step_dev))
        return fail(GS_ERR_INVALID_ARG, "gs_adam_step: bad arguments");
    if (step < 1) step = 1;
    AdamGroups G;
    memset(&G, 0, sizeof(G));
    G.n = n_groups;
    G.start[0] = 0;
    const double bc1 = 1.0 - std::pow(double(b1), step);
    const double bc2 = 1.0 - std::pow(double(b2), step);
    for (int k = 0; k < n_groups; ++k) {
        if (counts[k] < 0 || (counts[k] > 0 && (!params[k] || !grads[k] || !m[k] || !v[k])))
            return fail(GS_ERR_INVALID_ARG, "gs_adam_step: group %d", k);
        G.p[k] = params[k]; G.g[k] = grads[k]; G.m[k] = m[k]; G.v[k] = v[k];
        G.start[k + 1] = G.start[k] + counts[k];
        G.lr[k] = lr[k];
    }
    const int64_t total = G.start[n_groups];
    if (total == 0) return GS_OK;
    int64_t maxc = 0;
    for (int k = 0; k < n_groups; ++k) maxc = std::max<int64_t>(maxc, counts[k]);
    // contiguous float4 chunks per workgroup; caps measured on the 1M-Gaussian
    // step (62M floats): 1,024 -> 380 us, 2,048 -> 324, 4,096 -> 318,
    // 6,144 -> 312, 8,192 -> 329 (a grid-stride loop was best at 2,048: 330)
    int64_t blocks = (maxc / 4 + 255) / 256;
    if (blocks > 6144) blocks = 6144;
    if (blocks < 1) blocks = 1;
    launch("adam", k_adam, dim3(unsigned(blocks), unsigned(n_groups)), dim3(256), 0, stream, G, b1, b2, eps,
           float(1.0 / bc1),
           float(1.0 / std::sqrt(bc2)), total, clear_grads ? 1 : 0, static_cast<const int32_t*>(step_dev));
    if (step_dev) hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, stream, step_dev);
    return check_launch("gs_adam_step");
}
