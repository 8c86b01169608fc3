// Library-level entry points: status names, version, device check, frame
// selection and the vertex-buffer update (Sec. 3.3 MaGS paragraph, Sec. 3.4
// per-frame steps 1-2 of the paper).
#include "mgu_internal.hpp"

#include <cstring>

namespace mgu {
namespace {

// Plain streaming copy, 16 B per lane per iteration when both ends are
// 16 B aligned, grid-stride.  The O(N_v) vertex-buffer write of a frame.
__global__ __launch_bounds__(256) void copy4_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                    int64_t n4) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void copy1_kernel(const float *__restrict__ src, float *__restrict__ dst,
                                                    int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void fill_kernel(float *__restrict__ x, int64_t n, float value) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = value;
}

// out = wa a + wb b, element by element (out may be a or b).
__global__ __launch_bounds__(256) void blend_kernel(const float *a, const float *b, float wa, float wb, float *out,
                                                    int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = wa * a[i] + wb * b[i];
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" const char *mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "MG_OK";
        case MG_ERR_INVALID_ARGUMENT: return "MG_ERR_INVALID_ARGUMENT";
        case MG_ERR_WORKSPACE_TOO_SMALL: return "MG_ERR_WORKSPACE_TOO_SMALL";
        case MG_ERR_INDEX_OUT_OF_RANGE: return "MG_ERR_INDEX_OUT_OF_RANGE";
        case MG_ERR_NONFINITE_INPUT: return "MG_ERR_NONFINITE_INPUT";
        case MG_ERR_TOPOLOGY_MISMATCH: return "MG_ERR_TOPOLOGY_MISMATCH";
        case MG_ERR_HIP: return "MG_ERR_HIP";
        case MG_ERR_UNSUPPORTED_DEVICE: return "MG_ERR_UNSUPPORTED_DEVICE";
        default: return "MG_ERR_UNKNOWN";
    }
}

extern "C" int32_t mg_version(void) { return 100; }

extern "C" mg_status mg_check_device(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MG_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MG_ERR_HIP;
    return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? MG_OK : MG_ERR_UNSUPPORTED_DEVICE;
}

extern "C" mg_status mg_frame_index(int64_t step, int64_t f_recon_num, int64_t f_recon_den, int64_t f_sim,
                                    int32_t n_frames, int32_t *k_out) {
    if (!k_out || step < 0 || f_recon_num < 0 || f_recon_den <= 0 || f_sim <= 0 || n_frames <= 0)
        return MG_ERR_INVALID_ARGUMENT;
    // floor(step * num / (f_sim * den)) in 128-bit integers (no overflow, no rounding)
    const __int128 num = static_cast<__int128>(step) * f_recon_num;
    const __int128 den = static_cast<__int128>(f_sim) * f_recon_den;
    const __int128 k = num / den;
    *k_out = k >= n_frames ? n_frames - 1 : static_cast<int32_t>(k);
    return MG_OK;
}

extern "C" mg_status mg_vertex_buffer_update(const float *frames, int32_t n_frames, int32_t n_verts, int32_t k,
                                             float *live, void *stream) {
    if (bad_count(n_verts) || n_frames <= 0 || k < 0 || k >= n_frames) return MG_ERR_INVALID_ARGUMENT;
    if (n_verts == 0) return MG_OK;
    if (!frames || !live) return MG_ERR_INVALID_ARGUMENT;
    const int64_t n = 3 * static_cast<int64_t>(n_verts);
    const float *src = frames + static_cast<int64_t>(k) * n;
    if (src < live + n && live < src + n) return MG_ERR_INVALID_ARGUMENT;   // overlap
    hipStream_t s = as_stream(stream);
    const bool vec = (reinterpret_cast<uintptr_t>(src) % 16 == 0) && (reinterpret_cast<uintptr_t>(live) % 16 == 0) &&
                     (n % 4 == 0);
    if (vec) {
        const int64_t n4 = n / 4;
        const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n4, 256), 2048));
        hipLaunchKernelGGL(copy4_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<const float4 *>(src),
                           reinterpret_cast<float4 *>(live), n4);
    } else {
        const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 2048));
        hipLaunchKernelGGL(copy1_kernel, dim3(grid), dim3(256), 0, s, src, live, n);
    }
    return launch_status();
}

extern "C" mg_status mg_fill(float *x, int64_t n, float value, void *stream) {
    if (n < 0 || (n > 0 && !x)) return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 2048));
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, as_stream(stream), x, n, value);
    return launch_status();
}

extern "C" mg_status mg_blend(const float *a, const float *b, float wa, float wb, float *out, int64_t n,
                              void *stream) {
    if (n < 0 || (n > 0 && (!a || !b || !out))) return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 2048));
    hipLaunchKernelGGL(blend_kernel, dim3(grid), dim3(256), 0, as_stream(stream), a, b, wa, wb, out, n);
    return launch_status();
}
