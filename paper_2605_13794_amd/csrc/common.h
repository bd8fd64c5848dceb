// Internal helpers shared by the gsmi kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/gsmi.h"

namespace gsmi {

constexpr int kWave = 64;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kDilation = 0.3f;
constexpr float kJacClamp = 1.3f;
// Render record stride in floats (three float4).
constexpr int kRec = 12;
// Screen-space partials of one (entry, camera) in the backward: d mean2d (2),
// d conic (3), d opacity (1), d rgb (3), padded to 12 floats (48 B) so that one
// atomic instruction of nine lanes updates one record.
constexpr int kD2Stride = 12;

// ---------------------------------------------------------------------------
// Host-side error reporting
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
int check_launch(const char* what);

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace (256-byte aligned slices).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t used() const { return align_up(off, 256); }
};

// ---------------------------------------------------------------------------
// Camera as the kernels see it
// ---------------------------------------------------------------------------
struct DevCam {
    float R[9];
    float t[3];
    float campos[3];
    float fx, fy, cx, cy, znear;
    float limx, limy;  // off-axis clamp of x/z and y/z
    int32_t W, H, TX, TY;
    uint32_t tile_off;  // first global tile of this camera
};

inline int64_t tiles_x(int32_t w) { return (w + GS_TILE - 1) / GS_TILE; }
inline int64_t tiles_y(int32_t h) { return (h + GS_TILE - 1) / GS_TILE; }

inline DevCam make_devcam(const gs_camera& c, uint32_t tile_off) {
    DevCam d;
    for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
    // camera centre = -R^T t (computed in double on the host)
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s -= double(c.R[k * 3 + i]) * double(c.t[k]);
        d.campos[i] = float(s);
    }
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy; d.znear = c.znear;
    d.limx = kJacClamp * (0.5f * float(c.width)) / c.fx;
    d.limy = kJacClamp * (0.5f * float(c.height)) / c.fy;
    d.W = c.width; d.H = c.height;
    d.TX = int32_t(tiles_x(c.width)); d.TY = int32_t(tiles_y(c.height));
    d.tile_off = tile_off;
    return d;
}

int validate_cams(const gs_camera* cams, int n_cams, int max_cams, int64_t* total_tiles);

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
// Exponent (log2 domain) of a Gaussian at offset (dx, dy) from its mean,
// with the conic pre-scaled by -0.5 log2(e) (na, nc) and -log2(e) (nb):
//   e2 = log2(e) * (-0.5 (a dx^2 + c dy^2) - b dx dy).
// ebase = na dx^2 and eb = nb dx are shared by the pixels of one column.
__device__ __forceinline__ float gauss_e2(float ebase, float eb, float nc, float dy) {
    return fmaf(dy, fmaf(nc, dy, eb), ebase);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// DPP-based sum over the 64 lanes of a wavefront; the total lands in lane 63.
__device__ __forceinline__ float wave_sum_to_last(float v) {
    // xor 1, xor 2 inside quads
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    // rotate within rows of 16 by 4 and 8: every lane holds its row's sum
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xF, 0xF, false));
    // row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false));
    return v;
}

// Sum over 8 lanes: each lane gets its quad's sum plus that of the quad 4 lanes
// away in its row of 16.  Lanes 7 and 15 of a row (quads 1 and 3) then hold
// complementary halves of the row whichever way the rotation runs.
__device__ __forceinline__ float oct_sum8(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124, 0xF, 0xF, false));
    return v;
}

// oct_sum8 of several values, step by step, so that the DPP adds of
// different values interleave (no wait states between dependent DPP reads).
template <int N>
__device__ __forceinline__ void oct_sum8_n(float (&v)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[k]), 0xB1, 0xF, 0xF, false));
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[k]), 0x4E, 0xF, 0xF, false));
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[k]), 0x124, 0xF, 0xF, false));
}

// Sum over each row of 16 lanes (every lane of the row gets the row's sum).
__device__ __forceinline__ float row_sum16(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xF, 0xF, false));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_to_last_u32(uint32_t v) {
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x124, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x128, 0xF, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xA, 0xF, false));
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xC, 0xF, false));
    return v;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return __popcll(m); }

// lanes strictly below this one
__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Small fill kernel launcher (graph-capture friendly, unlike memset nodes).
int fill_u32(void* dst, uint32_t value, size_t count, hipStream_t s);

// Optional timing of one named kernel with caller events (gs_profile_kernel).
bool profile_match(const char* name, hipEvent_t* start, hipEvent_t* stop);

template <typename Kernel, typename... Args>
inline void launch(const char* name, Kernel kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t s,
                   Args... args) {
    hipEvent_t e0, e1;
    if (profile_match(name, &e0, &e1))
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

}  // namespace gsmi
